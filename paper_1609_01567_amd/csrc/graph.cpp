// Tanner-graph construction: from the COO list of ones in H to the two edge
// orders of the paper's address arrays (Sec. III-B, Tables I and II):
// edges sorted by bit (Table I) and edges sorted by check (Table II), both
// stable in the input order, plus the map between the two orders.
//
// Check->bit messages live in check-sorted (CSR) order, so the check-node
// update reads and writes each row contiguously; the bit-node update walks
// the bit-sorted (CSC) order and gathers through csc_to_csr.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace ldpc {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace ldpc

using ldpc::set_error;

extern "C" const char *ldpc_last_error(void) { return ldpc::g_last_error.c_str(); }

extern "C" const char *ldpc_status_str(ldpc_status s) {
    switch (s) {
        case LDPC_OK: return "LDPC_OK";
        case LDPC_E_INVAL: return "LDPC_E_INVAL";
        case LDPC_E_RANGE: return "LDPC_E_RANGE";
        case LDPC_E_DUP_EDGE: return "LDPC_E_DUP_EDGE";
        case LDPC_E_NOMEM: return "LDPC_E_NOMEM";
        case LDPC_E_DEVICE: return "LDPC_E_DEVICE";
        case LDPC_E_UNSUPPORTED: return "LDPC_E_UNSUPPORTED";
    }
    return "LDPC_E_UNKNOWN";
}

static void free_device(ldpc_graph *g) {
    int32_t **ptrs[] = {&g->d_row_ptr, &g->d_col_idx, &g->d_col_ptr, &g->d_csc_to_csr,
                        &g->d_class_rows, &g->d_hub_chunk_base, &g->d_class_rd,
                        &g->d_qc_row_ptr, &g->d_qc_ent};
    for (int32_t **p : ptrs) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
}

static ldpc_status upload(ldpc_graph *g) {
    struct Item { int32_t **dst; const std::vector<int32_t> *src; };
    Item items[] = {{&g->d_row_ptr, &g->row_ptr}, {&g->d_col_idx, &g->col_idx},
                    {&g->d_col_ptr, &g->col_ptr}, {&g->d_csc_to_csr, &g->csc_to_csr},
                    {&g->d_class_rows, &g->class_rows}, {&g->d_hub_chunk_base, &g->hub_chunk_base},
                    {&g->d_class_rd, &g->class_rd}, {&g->d_qc_row_ptr, &g->qc_row_ptr},
                    {&g->d_qc_ent, &g->qc_ent}};
    if (hipGetDevice(&g->device) != hipSuccess) {
        set_error("ldpc_graph_create: no HIP device is available");
        (void)hipGetLastError();
        return LDPC_E_DEVICE;
    }
    g->device_bytes = 0;
    for (const Item &it : items) {
        size_t bytes = std::max<size_t>(it.src->size(), 1) * sizeof(int32_t);
        hipError_t e = hipMalloc(reinterpret_cast<void **>(it.dst), bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_device(g);
            set_error(std::string("ldpc_graph_create: hipMalloc failed: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? LDPC_E_NOMEM : LDPC_E_DEVICE;
        }
        g->device_bytes += static_cast<int64_t>(bytes);
        if (!it.src->empty()) {
            e = hipMemcpy(*it.dst, it.src->data(), it.src->size() * sizeof(int32_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                free_device(g);
                set_error(std::string("ldpc_graph_create: hipMemcpy failed: ") + hipGetErrorString(e));
                return LDPC_E_DEVICE;
            }
        }
    }
    return LDPC_OK;
}

// The graph of (m, n, COO); `qc` (may be null) is moved into it before its
// tables go to the device.
struct QcBase {
    int32_t Z = 0;
    std::vector<int32_t> row_ptr, ent;
};
static ldpc_status build_graph(int32_t m, int32_t n, int64_t nnz, const int32_t *rows, const int32_t *cols,
                               uint32_t flags, QcBase *qc, ldpc_graph **out);

extern "C" ldpc_status ldpc_graph_create(int32_t m, int32_t n, int64_t nnz, const int32_t *rows,
                                         const int32_t *cols, uint32_t flags, ldpc_graph **out) {
    return build_graph(m, n, nnz, rows, cols, flags, nullptr, out);
}

extern "C" ldpc_status ldpc_graph_create_qc(int32_t mb, int32_t nb, int32_t Z, const int32_t *shifts,
                                            uint32_t flags, ldpc_graph **out) {
    if (!out || !shifts) { set_error("ldpc_graph_create_qc: null pointer"); return LDPC_E_INVAL; }
    if (mb < 1 || nb < 1 || Z < 1) { set_error("ldpc_graph_create_qc: mb, nb and Z must be >= 1"); return LDPC_E_INVAL; }
    if (int64_t(mb) * Z > INT32_MAX || int64_t(nb) * Z > INT32_MAX) {
        set_error("ldpc_graph_create_qc: mb * Z and nb * Z must be below 2^31");
        return LDPC_E_INVAL;
    }
    if (flags & ~uint32_t(LDPC_GRAPH_HOST_ONLY)) { set_error("ldpc_graph_create_qc: unknown flags"); return LDPC_E_INVAL; }
    try {
        QcBase qc;
        qc.Z = Z;
        qc.row_ptr.assign(size_t(mb) + 1, 0);
        for (int32_t i = 0; i < mb; i++) {
            for (int32_t j = 0; j < nb; j++) {
                const int32_t s = shifts[size_t(i) * nb + j];
                if (s < -1 || s >= Z) {
                    set_error("ldpc_graph_create_qc: shift (" + std::to_string(i) + ", " + std::to_string(j) +
                              ") = " + std::to_string(s) + " is outside [-1, Z)");
                    return LDPC_E_RANGE;
                }
                if (s >= 0) {
                    qc.ent.push_back(j * Z);
                    qc.ent.push_back(s);
                }
            }
            qc.row_ptr[i + 1] = int32_t(qc.ent.size() / 2);
        }
        const int64_t E = int64_t(qc.row_ptr[mb]) * Z;
        if (E > INT32_MAX) { set_error("ldpc_graph_create_qc: more than 2^31 - 1 edges"); return LDPC_E_INVAL; }
        // the lifted H, check by check, each check's edges in base-column order
        std::vector<int32_t> rows(static_cast<size_t>(E)), cols(static_cast<size_t>(E));
        size_t k = 0;
        for (int32_t i = 0; i < mb; i++) {
            for (int32_t t = 0; t < Z; t++) {
                for (int32_t q = qc.row_ptr[i]; q < qc.row_ptr[i + 1]; q++) {
                    const int32_t u = t + qc.ent[2 * size_t(q) + 1];
                    rows[k] = i * Z + t;
                    cols[k] = qc.ent[2 * size_t(q)] + (u >= Z ? u - Z : u);
                    k++;
                }
            }
        }
        return build_graph(mb * Z, nb * Z, E, rows.data(), cols.data(), flags, &qc, out);
    } catch (const std::bad_alloc &) {
        set_error("ldpc_graph_create_qc: out of host memory");
        return LDPC_E_NOMEM;
    }
}

static ldpc_status build_graph(int32_t m, int32_t n, int64_t nnz, const int32_t *rows, const int32_t *cols,
                               uint32_t flags, QcBase *qc, ldpc_graph **out) {
    if (!out) { set_error("ldpc_graph_create: out is NULL"); return LDPC_E_INVAL; }
    if (m < 1 || n < 1) { set_error("ldpc_graph_create: m and n must be >= 1"); return LDPC_E_INVAL; }
    if (nnz < 0 || nnz > INT32_MAX) { set_error("ldpc_graph_create: nnz must be in [0, 2^31)"); return LDPC_E_INVAL; }
    if (nnz > 0 && (!rows || !cols)) { set_error("ldpc_graph_create: rows/cols are NULL"); return LDPC_E_INVAL; }
    if (flags & ~uint32_t(LDPC_GRAPH_HOST_ONLY)) { set_error("ldpc_graph_create: unknown flags"); return LDPC_E_INVAL; }

    ldpc_graph *g = new (std::nothrow) ldpc_graph;
    if (!g) { set_error("ldpc_graph_create: out of host memory"); return LDPC_E_NOMEM; }
    try {
        const int64_t E = nnz;
        g->m = m; g->n = n; g->E = E;
        g->host_only = (flags & LDPC_GRAPH_HOST_ONLY) != 0;
        for (int64_t k = 0; k < E; k++) {
            if (rows[k] < 0 || rows[k] >= m || cols[k] < 0 || cols[k] >= n) {
                delete g;
                set_error("ldpc_graph_create: edge " + std::to_string(k) + " = (" + std::to_string(rows[k]) +
                          ", " + std::to_string(cols[k]) + ") is outside H");
                return LDPC_E_RANGE;
            }
        }
        // Counting sorts (stable): by check -> CSR, by bit -> CSC.
        g->row_ptr.assign(size_t(m) + 1, 0);
        g->col_ptr.assign(size_t(n) + 1, 0);
        for (int64_t k = 0; k < E; k++) { g->row_ptr[rows[k] + 1]++; g->col_ptr[cols[k] + 1]++; }
        for (int32_t i = 0; i < m; i++) g->row_ptr[i + 1] += g->row_ptr[i];
        for (int32_t j = 0; j < n; j++) g->col_ptr[j + 1] += g->col_ptr[j];
        std::vector<int32_t> csr_of_input(E), csc_of_input(E);
        {
            std::vector<int32_t> fr(g->row_ptr.begin(), g->row_ptr.end() - 1);
            std::vector<int32_t> fc(g->col_ptr.begin(), g->col_ptr.end() - 1);
            for (int64_t k = 0; k < E; k++) {
                csr_of_input[k] = fr[rows[k]]++;
                csc_of_input[k] = fc[cols[k]]++;
            }
        }
        g->col_idx.resize(E); g->row_idx.resize(E); g->csr_to_csc.resize(E); g->csc_to_csr.resize(E);
        for (int64_t k = 0; k < E; k++) {
            g->col_idx[csr_of_input[k]] = cols[k];
            g->row_idx[csc_of_input[k]] = rows[k];
            g->csr_to_csc[csr_of_input[k]] = csc_of_input[k];
            g->csc_to_csr[csc_of_input[k]] = csr_of_input[k];
        }
        // H is binary: a repeated (check, bit) pair is an error.  Rows are
        // short lists, so sort a copy of each row's bits.
        std::vector<int32_t> tmp;
        for (int32_t i = 0; i < m; i++) {
            const int32_t a = g->row_ptr[i], b = g->row_ptr[i + 1];
            g->max_cdeg = std::max(g->max_cdeg, b - a);
            tmp.assign(g->col_idx.begin() + a, g->col_idx.begin() + b);
            std::sort(tmp.begin(), tmp.end());
            for (size_t q = 1; q < tmp.size(); q++) {
                if (tmp[q] == tmp[q - 1]) {
                    delete g;
                    set_error("ldpc_graph_create: (" + std::to_string(i) + ", " + std::to_string(tmp[q]) +
                              ") appears more than once");
                    return LDPC_E_DUP_EDGE;
                }
            }
        }
        for (int32_t j = 0; j < n; j++) g->max_bdeg = std::max(g->max_bdeg, g->col_ptr[j + 1] - g->col_ptr[j]);

        // Degree classes.  Within the segmented class, longest rows first so the
        // longest-running workgroups start first.
        std::vector<int32_t> per_class[ldpc::kNumClasses];
        for (int32_t i = 0; i < m; i++) {
            const int32_t d = g->row_ptr[i + 1] - g->row_ptr[i];
            if (d > 0) per_class[ldpc::check_class_of(d)].push_back(i);
        }
        std::stable_sort(per_class[ldpc::kClassHub].begin(), per_class[ldpc::kClassHub].end(),
                         [&](int32_t a, int32_t b) {
                             return (g->row_ptr[a + 1] - g->row_ptr[a]) > (g->row_ptr[b + 1] - g->row_ptr[b]);
                         });
        g->class_begin[0] = 0;
        for (int c = 0; c < ldpc::kNumClasses; c++) {
            g->class_rows.insert(g->class_rows.end(), per_class[c].begin(), per_class[c].end());
            g->class_begin[c + 1] = static_cast<int32_t>(g->class_rows.size());
        }
        // row descriptors in class order: one load gives a row's first edge and degree
        g->class_rd.reserve(2 * g->class_rows.size());
        for (int32_t r : g->class_rows) {
            g->class_rd.push_back(g->row_ptr[r]);
            g->class_rd.push_back(g->row_ptr[r + 1] - g->row_ptr[r]);
        }
        g->hub_chunk_base.assign(1, 0);
        for (int32_t r : per_class[ldpc::kClassHub]) {
            const int32_t d = g->row_ptr[r + 1] - g->row_ptr[r];
            g->hub_chunk_base.push_back(g->hub_chunk_base.back() + (d + ldpc::kHubChunk - 1) / ldpc::kHubChunk);
            if (d > ldpc::kWideRowMax) g->hub_seg_rows++;   // longest first: these lead the class
        }
        g->hub_chunks = g->hub_chunk_base.back();
        if (qc) {
            g->qc_Z = qc->Z;
            g->qc_row_ptr = std::move(qc->row_ptr);
            g->qc_ent = std::move(qc->ent);
        }
    } catch (const std::bad_alloc &) {
        delete g;
        set_error("ldpc_graph_create: out of host memory");
        return LDPC_E_NOMEM;
    }
    if (!g->host_only) {
        ldpc_status st = upload(g);
        if (st != LDPC_OK) { delete g; return st; }
    }
    *out = g;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_graph_destroy(ldpc_graph *g) {
    if (!g) return LDPC_OK;
    if (!g->host_only && g->device >= 0) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != g->device) (void)hipSetDevice(g->device);
        free_device(g);
        if (cur >= 0 && cur != g->device) (void)hipSetDevice(cur);
    }
    delete g;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_graph_info(const ldpc_graph *g, int64_t *m, int64_t *n, int64_t *nnz,
                                       int32_t *max_check_deg, int32_t *max_bit_deg, int64_t *device_bytes) {
    if (!g) { set_error("ldpc_graph_info: graph is NULL"); return LDPC_E_INVAL; }
    if (m) *m = g->m;
    if (n) *n = g->n;
    if (nnz) *nnz = g->E;
    if (max_check_deg) *max_check_deg = g->max_cdeg;
    if (max_bit_deg) *max_bit_deg = g->max_bdeg;
    if (device_bytes) *device_bytes = g->device_bytes;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_graph_arrays(const ldpc_graph *g, int32_t *row_ptr, int32_t *col_idx,
                                         int32_t *col_ptr, int32_t *row_idx, int32_t *csr_to_csc) {
    if (!g) { set_error("ldpc_graph_arrays: graph is NULL"); return LDPC_E_INVAL; }
    auto put = [](int32_t *dst, const std::vector<int32_t> &src) {
        if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(int32_t));
    };
    put(row_ptr, g->row_ptr);
    put(col_idx, g->col_idx);
    put(col_ptr, g->col_ptr);
    put(row_idx, g->row_idx);
    put(csr_to_csc, g->csr_to_csc);
    return LDPC_OK;
}
