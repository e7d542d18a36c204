// Internal declarations shared by the graph builder and the decode driver.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldpc.h"

namespace ldpc {

// Check rows are grouped by degree into classes, one kernel shape per class:
// rows of up to 8 and of 9..16 edges in one wavefront's registers (the latter
// at most 2 frame slots per lane, which bounds register use); rows of 17..128
// edges cut into 8-edge chunks over 4 wavefronts that exchange chunk
// aggregates through LDS; longer rows on a segmented path that splits them
// into 32-edge chunks with aggregates in global scratch (no degree bound).
enum CheckClass : int { kClassD8 = 0, kClassD16 = 1, kClassD128 = 2, kClassHub = 3, kNumClasses = 4 };
constexpr int kHubChunk = 32;   // edges per chunk on the segmented path
// Rows of the long class up to this degree take the LDS path instead (one
// workgroup of 16 wavefronts per row and slot group, one 32-edge chunk each);
// longer rows the segmented path.
constexpr int kWideRowMax = 512;

inline int check_class_of(int d) {
    return d <= 8 ? kClassD8 : d <= 16 ? kClassD16 : d <= 128 ? kClassD128 : kClassHub;
}

// Wavefronts per row of the chunked class (rows per 256-thread block = 4 / this).
constexpr int class_waves_per_row(int cls) { return cls == kClassD128 ? 4 : 1; }

// Frame slots per wavefront lane for a class when the decode uses V slots per
// lane elsewhere (the segmented path always uses 1).
constexpr int class_lane_slots(int cls, int V) { return cls == kClassHub ? 1 : cls == kClassD16 && V > 2 ? 2 : V; }

void set_error(const std::string &msg);

// Host-side check of a check rule (ldpc_rule_kind and its parameter): false
// with a reason for an unknown kind or a parameter out of range.
inline bool rule_ok(int32_t kind, float param, std::string &why) {
    switch (kind) {
        case LDPC_RULE_SUM_PRODUCT: return true;
        case LDPC_RULE_MIN_SUM_NORMALIZED:
            if (param > 0.f && param <= 1.f) return true;
            why = "alpha must be in (0, 1]";
            return false;
        case LDPC_RULE_MIN_SUM_OFFSET:
            if (param >= 0.f && param < 64.f) return true;
            why = "beta must be in [0, 64)";
            return false;
        default: why = "unknown rule kind"; return false;
    }
}

}  // namespace ldpc

struct ldpc_graph {
    int32_t m = 0, n = 0;
    int64_t E = 0;
    int32_t max_cdeg = 0, max_bdeg = 0;
    bool host_only = false;
    int device = -1;

    // Host tables (Tables I/II in compressed form, see ldpc.h).
    std::vector<int32_t> row_ptr, col_idx;           // check-sorted (CSR)
    std::vector<int32_t> col_ptr, row_idx;           // bit-sorted (CSC)
    std::vector<int32_t> csr_to_csc, csc_to_csr;     // position maps between the two orders

    // Check rows listed by class (rows of degree 0 are in no class).
    std::vector<int32_t> class_rows;                 // concatenated, class by class
    std::vector<int32_t> class_rd;                   // per class row: first edge, degree (pairs, class order)
    int32_t class_begin[ldpc::kNumClasses + 1] = {0};
    // Segmented path: first chunk index of each hub row (in class order) and total chunks.
    std::vector<int32_t> hub_chunk_base;             // [#hub rows + 1]
    int64_t hub_chunks = 0;
    int32_t hub_seg_rows = 0;                        // hub rows (the first, longest ones) above kWideRowMax

    // Quasi-cyclic codes (ldpc_graph_create_qc): lifting size (0: not quasi-cyclic),
    // and per base row its entries in edge order as (j * Z, shift) pairs.
    int32_t qc_Z = 0;
    std::vector<int32_t> qc_row_ptr;                 // [mb + 1] base-entry offsets
    std::vector<int32_t> qc_ent;                     // [2 * base entries]

    // Device copies.
    int32_t *d_row_ptr = nullptr, *d_col_idx = nullptr;
    int32_t *d_col_ptr = nullptr, *d_csc_to_csr = nullptr;
    int32_t *d_class_rows = nullptr, *d_hub_chunk_base = nullptr, *d_class_rd = nullptr;
    int32_t *d_qc_row_ptr = nullptr, *d_qc_ent = nullptr;
    int64_t device_bytes = 0;
};
