/*
 * Systematic GF(2) encoder for arbitrary sparse parity-check matrices H
 * (input generation for tests and benchmarks; not part of the decoder).
 *
 * Finds a set of parity columns and, for given information bits, the parity
 * bits with H x = 0:
 *   1. Columns of degree 2 are edges between their two checks.  A spanning
 *      forest of that check graph is grown with union-find; forest columns
 *      are parity columns solved last by peeling each tree from its leaves.
 *   2. A tree can satisfy all of its checks iff the sum of those checks over
 *      the remaining (non-forest) columns is zero: one equation per tree.
 *      That small dense system over the non-forest columns is reduced to row
 *      echelon form (bit-packed Gaussian elimination); its pivot columns are
 *      the other parity columns, the rest are information columns.
 *   3. Encoding sets the information bits, back-substitutes the pivot
 *      columns, forms each check's partial syndrome, and peels every tree.
 * rank(H) = (m - #trees) + rank of the tree system; k = n - rank(H).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int m, n, k;
    /* graph */
    int *row_start, *row_cols;          /* columns of each check */
    /* forest */
    int *tree_col_of_check;             /* column joining a check to its parent, -1 for roots */
    int *parent_of_check;               /* parent check, -1 for roots */
    int *order;                         /* checks in BFS order (parents before children) */
    int *is_tree_col;                   /* [n] 1 if the column is a forest edge */
    /* tree system over non-forest columns */
    int nt;                             /* number of non-forest columns */
    int *nt_col;                        /* [nt] column index */
    int *nt_index;                      /* [n] index in nt_col or -1 */
    int rank, words;
    uint64_t *sys;                      /* [rank][words] echelon rows */
    int *pivot;                         /* [rank] nt index of each row's pivot */
    int *info_cols;                     /* [k] */
} encoder_t;

static int uf_find(int *p, int x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
}

void gf2enc_free(encoder_t *e) {
    if (!e) return;
    free(e->row_start); free(e->row_cols); free(e->tree_col_of_check); free(e->parent_of_check);
    free(e->order); free(e->is_tree_col); free(e->nt_col); free(e->nt_index); free(e->sys);
    free(e->pivot); free(e->info_cols);
    free(e);
}

int gf2enc_create(int m, int n, long nnz, const int *rows, const int *cols, encoder_t **out, int *k_out) {
    encoder_t *e = calloc(1, sizeof *e);
    if (!e) return 4;
    e->m = m; e->n = n;
    int *col_deg = calloc((size_t)n, sizeof(int));
    int *col_chk = malloc(sizeof(int) * 2 * (size_t)n);       /* the two checks of degree-2 columns */
    e->row_start = calloc((size_t)m + 1, sizeof(int));
    e->row_cols = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    if (!col_deg || !col_chk || !e->row_start || !e->row_cols) goto nomem;
    for (long q = 0; q < nnz; q++) {
        if (rows[q] < 0 || rows[q] >= m || cols[q] < 0 || cols[q] >= n) { free(col_deg); free(col_chk); gf2enc_free(e); return 2; }
        int j = cols[q];
        if (col_deg[j] < 2) col_chk[2 * j + col_deg[j]] = rows[q];
        col_deg[j]++;
        e->row_start[rows[q] + 1]++;
    }
    for (int i = 0; i < m; i++) e->row_start[i + 1] += e->row_start[i];
    {
        int *fill = calloc((size_t)m, sizeof(int));
        if (!fill) goto nomem;
        for (long q = 0; q < nnz; q++) e->row_cols[e->row_start[rows[q]] + fill[rows[q]]++] = cols[q];
        free(fill);
    }

    /* 1. spanning forest of degree-2 columns */
    int *uf = malloc(sizeof(int) * (size_t)m);
    e->is_tree_col = calloc((size_t)n, sizeof(int));
    if (!uf || !e->is_tree_col) { free(uf); goto nomem; }
    for (int i = 0; i < m; i++) uf[i] = i;
    for (int j = 0; j < n; j++) {
        if (col_deg[j] != 2) continue;
        int a = uf_find(uf, col_chk[2 * j]), b = uf_find(uf, col_chk[2 * j + 1]);
        if (a != b) { uf[a] = b; e->is_tree_col[j] = 1; }
    }
    /* tree adjacency and BFS order from each root */
    int *adj_start = calloc((size_t)m + 1, sizeof(int));
    int *adj = NULL;
    e->tree_col_of_check = malloc(sizeof(int) * (size_t)m);
    e->parent_of_check = malloc(sizeof(int) * (size_t)m);
    e->order = malloc(sizeof(int) * (size_t)m);
    int *comp = malloc(sizeof(int) * (size_t)m);
    if (!adj_start || !e->tree_col_of_check || !e->parent_of_check || !e->order || !comp) {
        free(uf); free(adj_start); free(comp); goto nomem;
    }
    for (int j = 0; j < n; j++)
        if (e->is_tree_col[j]) { adj_start[col_chk[2 * j] + 1]++; adj_start[col_chk[2 * j + 1] + 1]++; }
    for (int i = 0; i < m; i++) adj_start[i + 1] += adj_start[i];
    adj = malloc(sizeof(int) * 2 * (size_t)(adj_start[m] > 0 ? adj_start[m] : 1));
    int *afill = calloc((size_t)m, sizeof(int));
    if (!adj || !afill) { free(uf); free(adj_start); free(adj); free(afill); free(comp); goto nomem; }
    for (int j = 0; j < n; j++) {
        if (!e->is_tree_col[j]) continue;
        int a = col_chk[2 * j], b = col_chk[2 * j + 1];
        int pa = adj_start[a] + afill[a]++, pb = adj_start[b] + afill[b]++;
        adj[2 * pa] = b; adj[2 * pa + 1] = j;
        adj[2 * pb] = a; adj[2 * pb + 1] = j;
    }
    free(afill);
    for (int i = 0; i < m; i++) { e->parent_of_check[i] = -2; comp[i] = -1; }
    int head = 0, tailq = 0, ntrees = 0;
    for (int r = 0; r < m; r++) {
        if (e->parent_of_check[r] != -2) continue;
        e->parent_of_check[r] = -1; e->tree_col_of_check[r] = -1; comp[r] = ntrees;
        e->order[tailq++] = r;
        while (head < tailq) {
            int x = e->order[head++];
            for (int p = adj_start[x]; p < adj_start[x + 1]; p++) {
                int y = adj[2 * p], j = adj[2 * p + 1];
                if (e->parent_of_check[y] != -2) continue;
                e->parent_of_check[y] = x; e->tree_col_of_check[y] = j; comp[y] = ntrees;
                e->order[tailq++] = y;
            }
        }
        ntrees++;
    }
    free(uf); free(adj_start); free(adj);

    /* 2. tree system: one row per tree over the non-forest columns */
    e->nt_index = malloc(sizeof(int) * (size_t)n);
    e->nt_col = malloc(sizeof(int) * (size_t)n);
    if (!e->nt_index || !e->nt_col) { free(comp); goto nomem; }
    e->nt = 0;
    for (int j = 0; j < n; j++) {
        if (e->is_tree_col[j]) e->nt_index[j] = -1;
        else { e->nt_index[j] = e->nt; e->nt_col[e->nt++] = j; }
    }
    e->words = (e->nt + 63) / 64;
    const size_t W = (size_t)(e->words > 0 ? e->words : 1);
    uint64_t *A = calloc((size_t)(ntrees > 0 ? ntrees : 1) * W, sizeof(uint64_t));
    if (!A) { free(comp); goto nomem; }
    for (int i = 0; i < m; i++)
        for (int p = e->row_start[i]; p < e->row_start[i + 1]; p++) {
            int t = e->nt_index[e->row_cols[p]];
            if (t >= 0) A[(size_t)comp[i] * W + (size_t)(t >> 6)] ^= (uint64_t)1 << (t & 63);
        }
    free(comp);
    e->pivot = malloc(sizeof(int) * (size_t)(ntrees > 0 ? ntrees : 1));
    char *is_pivot = calloc((size_t)(e->nt > 0 ? e->nt : 1), 1);
    if (!e->pivot || !is_pivot) { free(A); free(is_pivot); goto nomem; }
    int r = 0;
    for (int c = 0; c < e->nt && r < ntrees; c++) {
        const size_t w = (size_t)(c >> 6);
        const uint64_t bit = (uint64_t)1 << (c & 63);
        int pr = -1;
        for (int q = r; q < ntrees; q++) if (A[(size_t)q * W + w] & bit) { pr = q; break; }
        if (pr < 0) continue;
        if (pr != r)
            for (size_t x = w; x < W; x++) {
                uint64_t tmp = A[(size_t)r * W + x]; A[(size_t)r * W + x] = A[(size_t)pr * W + x]; A[(size_t)pr * W + x] = tmp;
            }
        const uint64_t *prow = A + (size_t)r * W;
#pragma omp parallel for schedule(static)
        for (int q = r + 1; q < ntrees; q++) {
            uint64_t *row = A + (size_t)q * W;
            if (row[w] & bit)
                for (size_t x = w; x < W; x++) row[x] ^= prow[x];
        }
        e->pivot[r] = c;
        is_pivot[c] = 1;
        r++;
    }
    e->rank = r;
    e->sys = A;   /* rows r..ntrees-1 are zero and unused */
    e->k = e->nt - e->rank;
    e->info_cols = malloc(sizeof(int) * (size_t)(e->k > 0 ? e->k : 1));
    if (!e->info_cols) { free(is_pivot); goto nomem; }
    for (int c = 0, q = 0; c < e->nt; c++) if (!is_pivot[c]) e->info_cols[q++] = e->nt_col[c];
    free(is_pivot);
    free(col_deg); free(col_chk);
    *out = e;
    *k_out = e->k;
    return 0;
nomem:
    free(col_deg); free(col_chk);
    gf2enc_free(e);
    return 4;
}

int gf2enc_info_columns(const encoder_t *e, int *cols) {
    memcpy(cols, e->info_cols, sizeof(int) * (size_t)e->k);
    return e->k;
}

/* info [frames][k] (0/1) -> codewords [frames][n] (0/1).  Returns 0, or 5 if a
 * tree root is left unsatisfied (cannot happen for a consistent system). */
int gf2enc_encode(const encoder_t *e, int frames, const uint8_t *info, uint8_t *cw) {
    int status = 0;
#pragma omp parallel
    {
        const size_t W = (size_t)(e->words > 0 ? e->words : 1);
        uint64_t *x = malloc(W * sizeof(uint64_t));
        uint8_t *s = malloc((size_t)(e->m > 0 ? e->m : 1));
#pragma omp for schedule(dynamic, 4)
        for (int f = 0; f < frames; f++) {
            uint8_t *c = cw + (size_t)f * e->n;
            memset(c, 0, (size_t)e->n);
            memset(x, 0, W * sizeof(uint64_t));
            for (int q = 0; q < e->k; q++) {
                if (info[(size_t)f * e->k + q] & 1) {
                    int j = e->info_cols[q];
                    c[j] = 1;
                    int t = e->nt_index[j];
                    x[t >> 6] |= (uint64_t)1 << (t & 63);
                }
            }
            for (int r = e->rank - 1; r >= 0; r--) {       /* pivot of row r = parity of the rest */
                const uint64_t *row = e->sys + (size_t)r * W;
                uint64_t acc = 0;
                for (size_t w = 0; w < W; w++) acc ^= row[w] & x[w];
                int bit = __builtin_parityll(acc);
                int t = e->pivot[r];
                if (bit) { x[t >> 6] |= (uint64_t)1 << (t & 63); c[e->nt_col[t]] = 1; }
            }
            for (int i = 0; i < e->m; i++) {               /* partial syndromes over non-forest columns */
                uint8_t z = 0;
                for (int p = e->row_start[i]; p < e->row_start[i + 1]; p++) {
                    int j = e->row_cols[p];
                    if (!e->is_tree_col[j]) z ^= c[j];
                }
                s[i] = z;
            }
            for (int q = e->m - 1; q >= 0; q--) {          /* peel trees from the leaves */
                int i = e->order[q];
                int par = e->parent_of_check[i];
                if (par < 0) {
                    if (s[i]) {
#pragma omp atomic write
                        status = 5;
                    }
                    continue;
                }
                int j = e->tree_col_of_check[i];
                c[j] = s[i];
                s[par] ^= s[i];
            }
        }
        free(x); free(s);
    }
    return status;
}
