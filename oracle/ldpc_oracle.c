/*
 * FP64 CPU oracle for sum-product (SP) decoding of irregular LDPC codes.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU decoder is checked against.  It shares no code with the GPU library and
 * is used only by the tests, by the smoke check and by the benchmark's CPU
 * baseline leg; the product path never calls it.
 *
 * Source: J. Broulim, A. Ayriyan, V. Georgiev, H. Grigorian, "OpenCL/CUDA
 * algorithms for parallel decoding of any irregular LDPC code using GPU".
 *
 *   adjacency sets M_j (checks of bit j), N_i (bits of check i) .. Eqs. (1)-(2)
 *   bit -> check messages q, check -> bit messages r ............. Algorithm 1
 *   iteration order, stop when the estimate is a codeword ......... Algorithm 2
 *   channel probabilities p_j (taken here as LLRs) ................ Algorithm 3
 *   estimate from p and all incoming r ............................ Algorithm 4
 *   tie rule of the hard decision (1 only if Q1 > Q0) ............. Algorithm 6
 *   syndrome z = c H^T ............................................ Algorithm 7
 *
 * The paper's rules are written on probability pairs.  The oracle carries the
 * same messages as log-likelihood ratios L = ln(P(c=0)/P(c=1)), for which
 * Algorithm 1 reads (exact identities, no approximation):
 *
 *   q: Q[j->i] = L_j + sum_{i' in M_j \ i} R[i'->j]
 *   r: R[i->j] = (prod_{j' in N_i \ j} sgn Q[j'->i]) * phi( sum_{j' in N_i \ j} phi(|Q[j'->i]|) )
 *      with phi(x) = ln((e^x + 1)/(e^x - 1)) = -ln tanh(x/2), phi(0) = inf, phi(inf) = 0,
 *      which is r0 = 1/2 + 1/2 prod(1 - 2 q1) rewritten with 1 - 2 q1 = tanh(L_q/2);
 *   estimate: Lpost_j = L_j + sum_{i in M_j} R[i->j]; c_j = 1 iff Lpost_j < 0.
 *
 * Readings where the paper is silent (each stated in the design notes):
 *   - max_iter counts check-node updates; the pass before Algorithm 2's loop is
 *     iteration 1, and there is no syndrome test before it;
 *   - Q and R are clamped to +-lmax (64 by default); Lpost is not clamped;
 *   - a check of degree 1 sends +lmax (the empty product is 1: the bit must be 0);
 *   - sgn(0) = +1.
 *
 * Every extrinsic sum skips the destination edge explicitly (the "continue" of
 * Algorithm 5), so no quantity is ever formed as "total minus own".
 *
 * Min-Sum family.  Section 3.1 names Min-Sum and adaptive normalized / offset
 * Min-Sum (Wu, Song, Jiang, Zhao, IEEE Commun. Lett. 14(7), 2010) as derived
 * decoders that suit the edge-level approach.  They keep Algorithm 1's bit rule
 * and replace the check rule's magnitude phi(sum phi(|Q|)) by the smallest
 * |Q| among the other bits of the check, m = min_{j' in N_i \ j} |Q[j'->i]|:
 *   normalized: |R| = alpha * m          (alpha in (0, 1]; alpha = 1 is plain Min-Sum)
 *   offset:     |R| = max(m - beta, 0)   (beta >= 0)
 * with the same sign product and the same clamp; an empty set gives m = inf,
 * so a degree-1 check sends +lmax under every rule.
 */
#include <stdint.h>
#include <tgmath.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* The arithmetic type.  The oracle is FP64; ORACLE_REAL=float builds the same
 * steps in FP32 (tgmath.h picks the float forms of log1p, expm1 and fabs).
 * That build is a diagnostic for the tests only: it shows how far two
 * precisions of this very algorithm drift apart on frames that never
 * converge, and it is never a reference. */
#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL real;

#define ORACLE_OK 0
#define RULE_SUM_PRODUCT 0
#define RULE_MIN_SUM_NORMALIZED 1
#define RULE_MIN_SUM_OFFSET 2
#define ORACLE_E_INVAL 1
#define ORACLE_E_RANGE 2
#define ORACLE_E_NOMEM 4

typedef struct {
    int m, n;
    long E;
    const int *row, *col;      /* edge e joins check row[e] and bit col[e] */
    int *chk_start, *chk_edge; /* N_i: edges of check i, in input order     */
    int *bit_start, *bit_edge; /* M_j: edges of bit j, in input order       */
} graph_t;

static void graph_free(graph_t *g) {
    free(g->chk_start); free(g->chk_edge); free(g->bit_start); free(g->bit_edge);
}

/* Adjacency lists N_i and M_j of Eqs. (1)-(2), keeping the input edge order. */
static int graph_build(graph_t *g, int m, int n, long E, const int *row, const int *col) {
    memset(g, 0, sizeof *g);
    if (m < 0 || n < 0 || E < 0) return ORACLE_E_INVAL;
    g->m = m; g->n = n; g->E = E; g->row = row; g->col = col;
    g->chk_start = calloc((size_t)m + 1, sizeof(int));
    g->bit_start = calloc((size_t)n + 1, sizeof(int));
    g->chk_edge = malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    g->bit_edge = malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    if (!g->chk_start || !g->bit_start || !g->chk_edge || !g->bit_edge) { graph_free(g); return ORACLE_E_NOMEM; }
    for (long e = 0; e < E; e++) {
        if (row[e] < 0 || row[e] >= m || col[e] < 0 || col[e] >= n) { graph_free(g); return ORACLE_E_RANGE; }
        g->chk_start[row[e] + 1]++;
        g->bit_start[col[e] + 1]++;
    }
    for (int i = 0; i < m; i++) g->chk_start[i + 1] += g->chk_start[i];
    for (int j = 0; j < n; j++) g->bit_start[j + 1] += g->bit_start[j];
    int *fill_c = calloc((size_t)m + 1, sizeof(int));
    int *fill_b = calloc((size_t)n + 1, sizeof(int));
    if (!fill_c || !fill_b) { free(fill_c); free(fill_b); graph_free(g); return ORACLE_E_NOMEM; }
    for (long e = 0; e < E; e++) {
        g->chk_edge[g->chk_start[row[e]] + fill_c[row[e]]++] = (int)e;
        g->bit_edge[g->bit_start[col[e]] + fill_b[col[e]]++] = (int)e;
    }
    free(fill_c); free(fill_b);
    return ORACLE_OK;
}

/* phi(x) = ln((e^x+1)/(e^x-1)) = log1p(2/expm1(x)) for x >= 0; phi(0) = +inf, phi(+inf) = 0. */
static real phi(real x) {
    if (x == (real)0) return (real)INFINITY;
    return log1p((real)2 / expm1(x));
}

static real clamp(real x, real lim) {
    return x > lim ? lim : (x < -lim ? -lim : x);
}

/* Decode one frame.  Work buffers: R, Q, P (per edge), lpost (per bit), chat (per bit). */
static void decode_frame(const graph_t *g, const float *llr, int max_iter, int early_stop, real lmax,
                         double tie_margin, int rule, real rule_param, real *R, real *Q, real *P,
                         real *lpost, uint8_t *chat, uint8_t *ok_out, int *iters_out, double *min_abs_out,
                         uint8_t *tie_risk_out) {
    const int m = g->m, n = g->n;
    const long E = g->E;
    double min_abs = INFINITY;
    int ok = 0, t, tie_risk = 0;

    /* Algorithm 3: before any check update the bit->check messages are the
       channel values, which is the bit rule with every r at its neutral value
       (R = 0 in LLR form). */
    for (long e = 0; e < E; e++) R[e] = (real)0;

    for (t = 1; t <= max_iter; t++) {
        /* Algorithm 1, "Values to Check Nodes": Q[j->i] = L_j + sum over the
           other checks i' of bit j of R[i'->j]. */
        for (int j = 0; j < n; j++) {
            for (int a = g->bit_start[j]; a < g->bit_start[j + 1]; a++) {
                const int e = g->bit_edge[a];
                real s = (real)llr[j];
                for (int b = g->bit_start[j]; b < g->bit_start[j + 1]; b++) {
                    if (b == a) continue;              /* skip the destination check */
                    s += R[g->bit_edge[b]];
                }
                Q[e] = clamp(s, lmax);
            }
        }
        if (rule != RULE_SUM_PRODUCT) {
            /* Min-Sum family: sign product and smallest magnitude over the other
               bits of check i, then the normalization or the offset. */
            for (int i = 0; i < m; i++) {
                for (int a = g->chk_start[i]; a < g->chk_start[i + 1]; a++) {
                    const int e = g->chk_edge[a];
                    real mn = (real)INFINITY;
                    int negative = 0;
                    for (int b = g->chk_start[i]; b < g->chk_start[i + 1]; b++) {
                        if (b == a) continue;          /* skip the destination bit */
                        const int e2 = g->chk_edge[b];
                        if (fabs(Q[e2]) < mn) mn = fabs(Q[e2]);
                        negative ^= (Q[e2] < (real)0);
                    }
                    real mag;
                    if (rule == RULE_MIN_SUM_NORMALIZED) {
                        mag = rule_param * mn;
                    } else {
                        mag = mn - rule_param;
                        if (mag < (real)0) mag = (real)0;
                    }
                    R[e] = clamp(negative ? -mag : mag, lmax);
                }
            }
        } else {
        /* Each incoming message enters the check rule through phi(|Q|). */
        for (long e = 0; e < E; e++) P[e] = phi(fabs(Q[e]));

        /* Algorithm 1, "Values to Variable Nodes": product of tanh(|Q|/2) over the
           other bits of check i, written as phi of the sum of phi. */
        for (int i = 0; i < m; i++) {
            for (int a = g->chk_start[i]; a < g->chk_start[i + 1]; a++) {
                const int e = g->chk_edge[a];
                real s = (real)0;
                int negative = 0;
                for (int b = g->chk_start[i]; b < g->chk_start[i + 1]; b++) {
                    if (b == a) continue;              /* skip the destination bit */
                    const int e2 = g->chk_edge[b];
                    s += P[e2];
                    negative ^= (Q[e2] < (real)0);
                }
                const real mag = phi(s);             /* phi(0) = inf for an empty product */
                R[e] = clamp(negative ? -mag : mag, lmax);
            }
        }
        }

        /* Algorithm 4: the estimate uses the channel value and every incoming r. */
        long near_degree = 0;                          /* diagnostics only, see below */
        int near = 0;
        for (int j = 0; j < n; j++) {
            real s = (real)llr[j];
            for (int a = g->bit_start[j]; a < g->bit_start[j + 1]; a++) s += R[g->bit_edge[a]];
            lpost[j] = s;
            chat[j] = (uint8_t)(s < (real)0);              /* Algorithm 6: 1 only if Q1 > Q0 */
            if (fabs((double)s) < min_abs) min_abs = fabs((double)s);
            if (fabs((double)s) < tie_margin) { near = 1; near_degree += g->bit_start[j + 1] - g->bit_start[j]; }
        }

        /* Algorithm 7: z = c H^T; the estimate is a codeword iff z = 0. */
        long weight = 0;
        for (int i = 0; i < m; i++) {
            int z = 0;
            for (int a = g->chk_start[i]; a < g->chk_start[i + 1]; a++) z ^= chat[g->col[g->chk_edge[a]]];
            weight += z;
        }
        ok = (weight == 0);

        /* Diagnostics for comparisons with lower-precision decoders (no effect on
           the decode): the hard decisions only reach the outputs through the
           syndrome test and the returned estimate.  Flipping bits with
           |Lpost| < tie_margin can change an output only if it can zero a
           non-zero syndrome before the stop (weight <= sum of their degrees,
           early stop on) or if such a bit exists at the returned iteration. */
        const int stop = (ok && early_stop) || t == max_iter;
        if (stop ? near : (early_stop && weight > 0 && weight <= near_degree)) tie_risk = 1;
        if (ok && early_stop) break;                   /* Algorithm 2: return the codeword */
    }
    *ok_out = (uint8_t)ok;
    *iters_out = (t > max_iter) ? max_iter : t;
    *min_abs_out = min_abs;
    *tie_risk_out = (uint8_t)tie_risk;
}

/* Public entry.  llr: [frames][n] float32 LLRs.  rule: RULE_* above with its
 * parameter (alpha for the normalized rule, beta for the offset rule; ignored
 * for sum-product).  Outputs per frame: lpost [frames][n] (may be NULL),
 * bits [frames][n], ok [frames], iters [frames], min_abs [frames] (smallest
 * |Lpost| over all bits and all iterations run; may be NULL) and tie_risk
 * [frames] (1 if a sign flip of some bit with |Lpost| < tie_margin could change
 * bits, ok or iters; may be NULL). */
int ldpc_oracle_decode_rule(int m, int n, long nnz, const int *rows, const int *cols,
                            const float *llr, int frames, int max_iter, int early_stop, double lmax,
                            double tie_margin, int rule, double rule_param, double *lpost_out, uint8_t *bits_out,
                            uint8_t *ok_out, int *iters_out, double *min_abs_out, uint8_t *tie_risk_out,
                            int nthreads) {
    if (max_iter < 1 || frames < 0 || !(lmax > 0.0)) return ORACLE_E_INVAL;
    if (rule == RULE_MIN_SUM_NORMALIZED && !(rule_param > 0.0 && rule_param <= 1.0)) return ORACLE_E_INVAL;
    if (rule == RULE_MIN_SUM_OFFSET && !(rule_param >= 0.0 && rule_param < lmax)) return ORACLE_E_INVAL;
    if (rule < RULE_SUM_PRODUCT || rule > RULE_MIN_SUM_OFFSET) return ORACLE_E_INVAL;
    graph_t g;
    int st = graph_build(&g, m, n, nnz, rows, cols);
    if (st) return st;
    int status = ORACLE_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        const size_t Eb = (size_t)(nnz > 0 ? nnz : 1);
        real *R = malloc(sizeof(real) * Eb), *Q = malloc(sizeof(real) * Eb), *P = malloc(sizeof(real) * Eb);
        real *lp = malloc(sizeof(real) * (size_t)(n > 0 ? n : 1));
        uint8_t *ch = malloc((size_t)(n > 0 ? n : 1));
        if (!R || !Q || !P || !lp || !ch) {
#pragma omp atomic write
            status = ORACLE_E_NOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int f = 0; f < frames; f++) {
                double mn;
                uint8_t risk;
                decode_frame(&g, llr + (size_t)f * n, max_iter, early_stop, (real)lmax, tie_margin, rule,
                             (real)rule_param, R, Q, P, lp, ch, &ok_out[f], &iters_out[f], &mn, &risk);
                if (min_abs_out) min_abs_out[f] = mn;
                if (tie_risk_out) tie_risk_out[f] = risk;
                if (lpost_out)
                    for (int j = 0; j < n; j++) lpost_out[(size_t)f * n + j] = (double)lp[j];
                memcpy(bits_out + (size_t)f * n, ch, (size_t)n);
            }
        }
        free(R); free(Q); free(P); free(lp); free(ch);
    }
    graph_free(&g);
    return status;
}

/* Sum-product decode (the paper's rule): ldpc_oracle_decode_rule with RULE_SUM_PRODUCT. */
int ldpc_oracle_decode(int m, int n, long nnz, const int *rows, const int *cols,
                       const float *llr, int frames, int max_iter, int early_stop, double lmax,
                       double tie_margin, double *lpost_out, uint8_t *bits_out, uint8_t *ok_out,
                       int *iters_out, double *min_abs_out, uint8_t *tie_risk_out, int nthreads) {
    return ldpc_oracle_decode_rule(m, n, nnz, rows, cols, llr, frames, max_iter, early_stop, lmax, tie_margin,
                                   RULE_SUM_PRODUCT, 0.0, lpost_out, bits_out, ok_out, iters_out, min_abs_out,
                                   tie_risk_out, nthreads);
}

/* The oracle's adjacency lists (bit_start[n+1], bit_edge[nnz], chk_start[m+1], chk_edge[nnz]). */
int ldpc_oracle_adjacency(int m, int n, long nnz, const int *rows, const int *cols,
                          int *bit_start, int *bit_edge, int *chk_start, int *chk_edge) {
    graph_t g;
    int st = graph_build(&g, m, n, nnz, rows, cols);
    if (st) return st;
    memcpy(bit_start, g.bit_start, sizeof(int) * ((size_t)n + 1));
    memcpy(chk_start, g.chk_start, sizeof(int) * ((size_t)m + 1));
    memcpy(bit_edge, g.bit_edge, sizeof(int) * (size_t)nnz);
    memcpy(chk_edge, g.chk_edge, sizeof(int) * (size_t)nnz);
    graph_free(&g);
    return ORACLE_OK;
}
