// Batched decoding with continuous refill: the ldpc_engine_* entry points.
//
// Every graph owns a pool of S frame slots with the same layout as the plain
// decoder ([n][S] channel/posterior LLRs, [E][S] messages in check-sorted
// order).  Each slot carries its own iteration count, so frames of one graph
// sit at different iterations in the same wavefront.  One decode step is
//
//   I times (I = iterations per step, 1 by default):
//     check pass  (all graphs)  iteration t_s+1 of every running slot s, and the
//                               syndrome of its estimate t_s (Algorithm 7)
//     bit pass    (all graphs)  stop test: estimate t_s passed (early stop) or
//                               t_s = max_iter, and the frame stops; else the
//                               Lpost / hard decision of iteration t_s+1
//                               (Algorithm 4) and t_s += 1
//   advance     (all slots)   write ok/iters of the stopped frames and list them
//   turnover    (listed slots) write the estimate of stopped frames, admit the
//                             next queued frame of the graph into the slot
//   repack      (per graph)   once the queue is empty and the running frames are
//                             scattered, move them into the lowest slots
//
// The check and bit arithmetic (device_common.h) and its order per frame are
// those of decode.hip, so a frame's outputs do not depend on its neighbours.
// K steps are captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "device_common.h"

namespace {

using namespace ldpc_dev;

constexpr int kMaxGraphs = 32;
constexpr int kTurnoverBlocks = 1024;
constexpr int kCounterInts = 7;    // per graph: head, tail, retired, list count, taken, moves, extent
constexpr int kRepackMinExtent = 32;   // below this many slots a repack saves no cache line
constexpr int kMoveBlocks = 512;
constexpr int kMoveRows = 64;      // rows of one graph's state arrays per move work unit

struct EngFrame {   // device mirror of ldpc_frame
    const float *llr;
    uint8_t *bits;
    uint8_t *ok;
    int32_t *iters;
    float *llr_out;
    int32_t *done;
};
static_assert(sizeof(EngFrame) == sizeof(ldpc_frame), "ldpc_frame layout");

struct EngGraph {
    const int32_t *col_idx, *col_ptr, *csc_to_csr, *hub_chunk_base;
    const int32_t *class_rd;   // per class row (class order): first edge, degree
    int32_t n, S, E;
    int32_t post16;       // the posterior storage is fp16 (16-bit message formats)
    int32_t hub_seg;      // rows of the long class on the segmented path (the first ones); the rest are wide rows
    int32_t class_begin[ldpc::kNumClasses + 1];
    float *lch, *lpost;
    void *post;           // posterior in the check pass's storage (Post<M>); lpost for 32/8-bit messages
    int32_t *want32;      // [S] 16-bit formats: 1 if the slot's frame asks for its posterior (lpost kept)
    void *r;
    int32_t *slot_t;      // [2][S] iterations completed by the frame in the slot (-1: empty;
                          // + kStopped: stopped), ping-pong between the passes of a step
    int32_t *fail;        // t of the last estimate whose syndrome failed
    EngFrame *slot_desc;  // descriptor of the frame in the slot
    float *aggd, *aggpre;
    int32_t *aggbits;
    EngFrame *queue;      // ring of cap entries
    int32_t cap;
    int32_t *head, *tail, *retired;   // monotonic counters
    int32_t *list;        // turnover list of this step: slot | (stopped << 31)
    int32_t *list_count;
    int32_t *taken;       // frames admitted by this step's turnover (applied to head next step)
    int32_t *moves;       // frames repacked by this step (slot pairs in move_src / move_dst)
    int32_t *extent;      // one past the highest occupied slot (0: pool empty)
    int32_t *move_src, *move_dst;
};

// Frame descriptors move as three 16-byte words through global loads/stores
// (descriptor arrays are 256-byte aligned and 48 bytes per entry).
static_assert(sizeof(EngFrame) == 48, "EngFrame layout");

__device__ __forceinline__ EngFrame load_frame(const EngFrame *p) {
    const auto q = gmem(reinterpret_cast<const u32x4 *>(p));
    const u32x4 w[3] = {q[0], q[1], q[2]};
    EngFrame f;
    __builtin_memcpy(&f, w, sizeof(f));
    return f;
}

__device__ __forceinline__ void store_frame(EngFrame *p, const EngFrame &f) {
    u32x4 w[3];
    __builtin_memcpy(w, &f, sizeof(f));
    const auto q = gmem(reinterpret_cast<u32x4 *>(p));
    q[0] = w[0];
    q[1] = w[1];
    q[2] = w[2];
}

// Queue and step counters of every graph, in one array of kCounterInts per
// graph: [4c] head, [4c+1] tail, [4c+2] retired, [4c+3] list count, then
// [4G+c] taken, [5G+c] moves, [6G+c] extent (G graphs).  Kernels that size
// their work from them read them here directly, one lane per graph.
__device__ __forceinline__ int ctr_list_count(int c) { return 4 * c + 3; }
__device__ __forceinline__ int ctr_taken(int ng, int c) { return 4 * ng + c; }
__device__ __forceinline__ int ctr_moves(int ng, int c) { return 5 * ng + c; }
__device__ __forceinline__ int ctr_extent(int ng, int c) { return 6 * ng + c; }

// Wavefront 0, lane c < ngraphs holding graph c's item count: p[0..ngraphs]
// receives the exclusive offsets (p[ngraphs] is the total).  At most 32 graphs,
// so a scan over the low 32 lanes covers them.  The caller synchronises.
template <typename I>
__device__ __forceinline__ void scan_items(I items, int32_t ngraphs, I *p) {
    const int c = threadIdx.x;
    for (int off = 1; off < 32; off <<= 1) {
        const I y = __shfl_up(items, off);
        if (c >= off) items += y;
    }
    if (c == 0) p[0] = 0;
    if (c < ngraphs) p[c + 1] = items;
}

struct Prefix {           // offsets of each graph's work items in one launch
    int32_t count;
    int32_t p[kMaxGraphs + 1];
};

__device__ __forceinline__ int find_graph(const Prefix &pre, int x) {
    int c = 0;
    while (c + 1 < pre.count && x >= pre.p[c + 1]) c++;
    return c;
}

// Slot state values: -1 empty; t in [0, kStopped) running with t iterations
// done; kStopped + t stopped after estimate t, waiting for the turnover.
// Within a step, pass j reads row j % 2 of slot_t and the bit pass writes the
// state for pass j + 1 into the other row; the step starts from row 0, which
// holds every slot's state, and for slots at or above the graph's extent
// (empty) only row 0 is kept.
constexpr int32_t kStopped = 1 << 30;

// Frame in slot stops after its estimate t: passed the syndrome (early stop) or t = max_iter.
__device__ __forceinline__ bool slot_stops(int32_t t, int32_t fail, int32_t T, int32_t early) {
    return t >= 1 && ((early && fail != t) || t == T);
}

// ------------------------------------------------------------- check pass

// Per-slot state of a lane's V slots: occupied, first iteration (L from the
// channel array, no previous message), and whether the syndrome of the slot's
// current estimate is checked in this pass.
template <int V>
struct EngLane {
    int32_t t[V];
    bool syn_on[V];
    bool active;
    SlotSrc<V> src;
};

template <int V>
__device__ __forceinline__ void eng_lane(const EngGraph &G, int s0, int32_t T, int32_t early, int32_t par,
                                         EngLane<V> &ln) {
    load_i32<V>(G.slot_t + par * G.S + s0, ln.t);
    ln.active = false;
    ln.src.any = false;
#pragma unroll
    for (int k = 0; k < V; k++) {
        const bool act = ln.t[k] >= 0 && ln.t[k] < kStopped;
        ln.src.alt[k] = ln.t[k] == 0;
        ln.syn_on[k] = act && ln.t[k] >= 1 && (early || ln.t[k] == T);
        ln.active |= act;
        ln.src.any |= ln.src.alt[k];
    }
}

template <int V>
__device__ __forceinline__ void eng_syndrome(const EngGraph &G, const EngLane<V> &ln, const int (&syn)[V], int s0) {
#pragma unroll
    for (int k = 0; k < V; k++)
        if (ln.syn_on[k] && syn[k] && gmem(G.fail)[s0 + k] != ln.t[k]) gmem(G.fail)[s0 + k] = ln.t[k];
}

// Work of one pass over the occupied slot groups of every graph.  Graph c owns
// items [p[c], p[c+1]); an item is one (row or bit, slot group) pair, or for
// the chunked classes a workgroup of `per` such pairs.  Only the groups below
// each graph's extent (one past its highest occupied slot) count, so passes
// over empty pools cost nothing but the launch.  Built by every workgroup.
//
// Packed items (PACK): once a graph's extent fits in 64 / rpw lanes (times V
// slots), a wavefront takes rpw rows or bits at once, 64 / rpw lanes each
// (rpw = 2, 4, 8 or 16), so a nearly drained pool costs few wavefronts.
struct Work {
    int32_t p[kMaxGraphs + 1];
    int32_t groups[kMaxGraphs];
    int32_t rpw[kMaxGraphs];
};
constexpr int kMaxPack = 16;
constexpr int kBitItems = -1;    // `cls` value for the bit pass: items are bits
constexpr int kWideItems = -2;   // `cls` value for the wide rows of the long class (after its segmented rows)

// PM (packing mode): kPackNone counts every graph unpacked; kPackAll packs the
// graphs whose extent allows it; kPackOnlyFlat / kPackOnlyPacked keep only the
// graphs that kPackAll leaves unpacked / packs (two launches, one lean kernel
// body each).
enum PackMode { kPackNone = 0, kPackAll = 1, kPackOnlyFlat = 2, kPackOnlyPacked = 3 };

// Lane-width split, for the chunked class (which has no packed form): the
// launch at the engine's lane width (kSplitWide) takes the graphs whose extent
// exceeds half of `wide_unit` slots (64 lanes at that width); a second launch
// at one slot per lane (kSplitNarrow) takes the others, so a drained pool pays
// for 64-slot groups instead of 64 V-slot ones.
enum LaneSplit { kSplitNone = 0, kSplitWide = 1, kSplitNarrow = 2 };

template <int PM = kPackNone, int SPLIT = kSplitNone>
__device__ __forceinline__ void build_work(const EngGraph *__restrict__ graphs, int32_t ngraphs,
                                           const int32_t *__restrict__ counters, int cls, int unit, int per, Work &w,
                                           int wide_unit = 0) {
    // wavefront 0, one lane per graph (at most 32): the graphs' extents load in
    // parallel and an inclusive scan over the lanes gives the item offsets
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        int32_t items = 0;
        if (c < ngraphs) {
            const EngGraph &G = graphs[c];
            const int32_t x = gmem(counters)[ctr_extent(ngraphs, c)];
            const int32_t gr = (x + unit - 1) / unit;
            const int32_t hubs = G.class_begin[ldpc::kClassHub + 1] - G.class_begin[ldpc::kClassHub];
            const int32_t units = cls == kBitItems ? G.n
                                  : cls == kWideItems ? hubs - G.hub_seg
                                  : cls == ldpc::kClassHub ? G.hub_seg
                                  : G.class_begin[cls + 1] - G.class_begin[cls];
            int32_t rpw = 1;
            if (PM != kPackNone && x > 0)
                while (rpw < kMaxPack && (unit / (2 * rpw)) >= x) rpw *= 2;   // unit = 64 V slots per wavefront
            bool take = PM == kPackNone || PM == kPackAll || (PM == kPackOnlyFlat) == (rpw == 1);
            if (SPLIT != kSplitNone) take = (SPLIT == kSplitNarrow) == (x > 0 && 2 * x <= wide_unit);
            w.groups[c] = gr;
            w.rpw[c] = rpw;
            items = !take ? 0 : rpw > 1 ? (units + rpw - 1) / rpw : (units * gr + per - 1) / per;
        }
        scan_items<int32_t>(items, ngraphs, w.p);
    }
    __syncthreads();
}

// Values read from the work table are the same in every lane; callers pass them
// through wave_uniform so that the compiler keeps the item's indices in scalar
// registers (LDS reads are otherwise treated as per-lane, which turns every
// index load of the item into a vector load).
// The search starts at graph c0, at or before x's graph: a pass's loop visits
// its items in increasing order, so it passes the previous item's graph.
__device__ __forceinline__ int work_graph(const Work &w, int32_t ngraphs, int x, int c0) {
    int c = c0;
    while (c + 1 < ngraphs && x >= w.p[c + 1]) c++;
    return c;
}

// Rows of up to DMAX edges: one wavefront per (row, slot group), looping over
// the items of the pass.
// One (row, slots) item of the register-row classes.  UNIFORM: every lane works
// on row rk (a scalar), so the row descriptor and the column indices come in
// through scalar loads issued before the slot state is examined; otherwise
// each lane has its own row (packed items).
// ln: the slot state of the lane's slots (eng_lane), the same for every row of
// one slot group in one pass.
template <int M, int V, int DMAX, bool UNIFORM, int RULE>
__device__ __forceinline__ void rows_item(const EngGraph &G, int cls, int nrows, int rk, int s0,
                                          const EngLane<V> &ln, float rp) {
    using MT = typename Codec<M>::T;
    if (!UNIFORM && rk >= nrows) return;
    const u32x2 rdv = cload(reinterpret_cast<const u32x2 *>(G.class_rd) + G.class_begin[cls] + rk);
    if (!ln.active) return;
    const int e0 = UNIFORM ? wave_uniform(int(rdv.x)) : int(rdv.x);
    const int d = UNIFORM ? wave_uniform(int(rdv.y)) : int(rdv.y);
    int syn[V];
#pragma unroll
    for (int k = 0; k < V; k++) syn[k] = 0;
    MT *R = static_cast<MT *>(G.r);
    row_rule<M, V, DMAX, UNIFORM, kInMixed, RULE>(G.col_idx, e0, d, static_cast<const typename Post<M>::T *>(G.post),
                                                  R, G.S, s0, ln.src, syn, rp);
    eng_syndrome<V>(G, ln, syn, s0);
}

template <int M, int V, int DMAX, int PM, int RULE>
__global__ __launch_bounds__(256, 4) void eng_check_rows(const EngGraph *__restrict__ graphs, int32_t ngraphs,
                                                      const int32_t *__restrict__ counters, int32_t cls, int32_t T,
                                                      int32_t early, int32_t par, float rp) {
    __shared__ Work w;
    build_work<PM>(graphs, ngraphs, counters, cls, 64 * V, 1, w);
    const int lane = threadIdx.x & 63;
    const int total = wave_uniform(w.p[ngraphs]);
    const int stride = int(gridDim.x * (blockDim.x >> 6));
    int prev_c = -1, prev_g = -1;
    EngLane<V> ln;
    int last_c = 0;
    for (int item = wave_uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6); item < total; item += stride) {
        const int c = wave_uniform(work_graph(w, ngraphs, item, last_c));
        last_c = c;
        const EngGraph &G = graphs[c];
        const int local = item - wave_uniform(w.p[c]);
        const int rpw = wave_uniform(w.rpw[c]);
        const int nrows = G.class_begin[cls + 1] - G.class_begin[cls];
        if (PM == kPackNone || PM == kPackOnlyFlat || (PM == kPackAll && rpw == 1)) {
            const int groups = wave_uniform(w.groups[c]);
            const int rk = local / groups;
            const int g = local - rk * groups;
            const int s0 = (g * 64 + lane) * V;
            // consecutive items of a wavefront often share their graph and slot
            // group: keep its slot state
            if (c != prev_c || g != prev_g) {
                eng_lane<V>(G, s0, T, early, par, ln);
                prev_c = c;
                prev_g = g;
            }
            rows_item<M, V, DMAX, true, RULE>(G, cls, nrows, rk, s0, ln, rp);
        } else {
            const int lpr = 64 / rpw;
            const int rk = local * rpw + lane / lpr;
            if (rk < nrows) {
                const int s0 = (lane % lpr) * V;
                EngLane<V> pl;
                eng_lane<V>(G, s0, T, early, par, pl);
                rows_item<M, V, DMAX, false, RULE>(G, cls, nrows, rk, s0, pl, rp);
            }
        }
    }
}

// Rows of 9..128 edges over WPR wavefronts (see check_chunk_kernel in decode.hip);
// one workgroup item = 4 / WPR (row, slot group) pairs.  SPLIT selects the
// graphs by extent (LaneSplit); wide_unit is 64 times the engine's lane width.
template <int M, int V, int WPR, int RULE, int SPLIT>
__global__ __launch_bounds__(256) void eng_check_chunk(const EngGraph *__restrict__ graphs, int32_t ngraphs,
                                                       const int32_t *__restrict__ counters, int32_t cls, int32_t T,
                                                       int32_t early, int32_t par, float rp, int32_t wide_unit) {
    using MT = typename Codec<M>::T;
    constexpr int C = kRowChunk;
    constexpr int RPB = 4 / WPR;
    constexpr int MAXCH = WPR == 2 ? 2 : 16;
    __shared__ ChunkShare<V, RPB * MAXCH> sh;
    __shared__ Work w;
    build_work<kPackNone, SPLIT>(graphs, ngraphs, counters, cls, 64 * V, RPB, w, wide_unit);
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int lr = wave / WPR;
    const int wr = wave % WPR;
    const int total = wave_uniform(w.p[ngraphs]);
    int last_c = 0;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {     // uniform over the workgroup
        const int c = wave_uniform(work_graph(w, ngraphs, u, last_c));
        last_c = c;
        const EngGraph &G = graphs[c];
        const int groups = wave_uniform(w.groups[c]);
        const int nrows = G.class_begin[cls + 1] - G.class_begin[cls];
        const int item = (u - wave_uniform(w.p[c])) * RPB + lr;
        const bool valid = item < nrows * groups;                // uniform over the wavefront
        const int rk = valid ? item / groups : 0;
        const int g = valid ? item % groups : 0;
        const int s0 = (g * 64 + lane) * V;
        EngLane<V> ln;
        ln.active = false;
        if (valid) eng_lane<V>(G, s0, T, early, par, ln);
        const bool work = valid && __ballot(ln.active) != 0;
        int e0 = 0, d = 0, nch = 0;
        if (work) {
            const u32x2 rdv = cload(reinterpret_cast<const u32x2 *>(G.class_rd) + G.class_begin[cls] + rk);
            e0 = wave_uniform(int(rdv.x));
            d = wave_uniform(int(rdv.y));
            nch = (d + C - 1) / C;
        }
        MT *R = static_cast<MT *>(G.r);
        const auto *PL = static_cast<const typename Post<M>::T *>(G.post);
        const int32_t S = G.S;
        const bool mine = work && ln.active;
        float u_[C][V], suf[C][V], agg[V];
        uint32_t par[V];
        int syn[V];
        for (int ch = wr; ch < nch; ch += WPR) {
            if (mine) {
                chunk_load<M, V, C, kInMixed, RULE>(G.col_idx, e0 + ch * C, min(C, d - ch * C), PL, R, S, s0,
                                                    ln.src, u_, suf, agg, par, syn);
            } else {
#pragma unroll
                for (int k = 0; k < V; k++) { agg[k] = CheckRule<RULE>::identity(); par[k] = 0u; syn[k] = 0; }
            }
#pragma unroll
            for (int k = 0; k < V; k++) sh.agg[lr * MAXCH + ch][lane][k] = agg[k];
            sh.bits[lr * MAXCH + ch][lane] = pack_bits<V>(par, syn);
        }
        __syncthreads();
        if (mine) {
            for (int ch = wr; ch < nch; ch += WPR) {
                if (nch > WPR)
                    chunk_load<M, V, C, kInMixed, RULE>(G.col_idx, e0 + ch * C, min(C, d - ch * C), PL, R, S,
                                                        s0, ln.src, u_, suf, agg, par, syn);
                float pre_a[V], post_a[V];
                uint32_t parity[V];
                int syn_row[V];
                chunk_context<V, RPB * MAXCH, RULE>(sh, lr * MAXCH, nch, ch, lane, pre_a, post_a, parity, syn_row);
                chunk_store<M, V, C, RULE>(e0 + ch * C, min(C, d - ch * C), u_, suf, pre_a, post_a, parity, R, S,
                                           s0, rp);
                if (ch == 0) eng_syndrome<V>(G, ln, syn_row, s0);
            }
        }
        __syncthreads();   // the shared aggregates are reused by the next item
    }
}

// Rows longer than 128 edges: one workgroup of four wavefronts per (row, 64 slots),
// 32-edge chunks combined through an exclusive prefix/suffix scan in scratch.
template <int M, int RULE>
__global__ __launch_bounds__(256) void eng_check_hub(const EngGraph *__restrict__ graphs, int32_t ngraphs,
                                                     const int32_t *__restrict__ counters, int32_t T, int32_t early,
                                                     int32_t par, float rp) {
    using MT = typename Codec<M>::T;
    using Rule = CheckRule<RULE>;
    constexpr int C = ldpc::kHubChunk;
    __shared__ int32_t total_bits[64];
    __shared__ Work w;
    build_work(graphs, ngraphs, counters, ldpc::kClassHub, 64, 1, w);
    const int lane = threadIdx.x & 63;
    const int wv = wave_uniform(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int total = wave_uniform(w.p[ngraphs]);
    int last_c = 0;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {     // uniform over the workgroup
        const int c = wave_uniform(work_graph(w, ngraphs, u, last_c));
        last_c = c;
        const EngGraph &G = graphs[c];
        const int32_t S = G.S;
        const int groups = wave_uniform(w.groups[c]);
        const int local = u - wave_uniform(w.p[c]);
        const int g = local % groups;
        const int rk = local / groups;
        const int s = g * 64 + lane;
        const int32_t ts = gmem(G.slot_t)[par * S + s];
        const bool active = ts >= 0 && ts < kStopped;
        const bool first = active && ts == 0;
        const bool syn_on = active && ts >= 1 && (early || ts == T);
        if (__ballot(active) == 0) continue;   // same slots in every wavefront: uniform over the workgroup

        const u32x2 rdv = cload(reinterpret_cast<const u32x2 *>(G.class_rd) + G.class_begin[ldpc::kClassHub] + rk);
        const int e0 = wave_uniform(int(rdv.x));
        const int d = wave_uniform(int(rdv.y));
        const int nch = (d + C - 1) / C;
        const int cb = wave_uniform(cload(G.hub_chunk_base + (rk)));
        auto R = gmem(static_cast<MT *>(G.r));
        auto L = gmem(static_cast<const typename Post<M>::T *>(G.post));   // channel LLRs in a first pass

        for (int ch = wv; ch < nch; ch += nw) {
            const int j0 = e0 + ch * C;
            const int dc = min(C, d - ch * C);
            float agg = Rule::identity();
            int32_t bits = 0;
#pragma unroll
            for (int jj = 0; jj < C; jj++) {
                if (jj < dc) {
                    const int v = wave_uniform(cload(G.col_idx + (j0 + jj)));
                    const float lv = Codec<Post<M>::kMsg>::dec(L[size_t(v) * S + s]);
                    const float r = first ? 0.f : Codec<M>::dec(R[size_t(j0 + jj) * S + s]);
                    const float qv = rule_q<M, RULE>(lv, r);
                    bits ^= int32_t(qv < 0.f) | (int32_t(lv < 0.f) << 1);
                    agg = Rule::combine(agg, rule_in<M, RULE>(fabsf(qv)));
                }
            }
            gmem(G.aggd)[size_t(cb + ch) * S + s] = agg;
            gmem(G.aggbits)[size_t(cb + ch) * S + s] = bits;
        }
        __syncthreads();
        if (wv == 0) {
            float pre_d = Rule::identity();
            int32_t tot = 0;
            for (int ch = 0; ch < nch; ch++) {
                gmem(G.aggpre)[size_t(cb + ch) * S + s] = pre_d;
                pre_d = Rule::combine(pre_d, gmem(G.aggd)[size_t(cb + ch) * S + s]);
                tot ^= gmem(G.aggbits)[size_t(cb + ch) * S + s];
            }
            float sf = Rule::identity();
            for (int ch = nch - 1; ch >= 0; ch--) {
                const float dcur = gmem(G.aggd)[size_t(cb + ch) * S + s];
                gmem(G.aggd)[size_t(cb + ch) * S + s] = Rule::combine(gmem(G.aggpre)[size_t(cb + ch) * S + s], sf);
                sf = Rule::combine(sf, dcur);
            }
            total_bits[lane] = tot;
            if (syn_on && (tot & 2) && gmem(G.fail)[s] != ts) gmem(G.fail)[s] = ts;
        }
        __syncthreads();
        const uint32_t parity = uint32_t(total_bits[lane]) & 1u;
        for (int ch = wv; ch < nch; ch += nw) {
            const int j0 = e0 + ch * C;
            const int dc = min(C, d - ch * C);
            float uu[C], sf[C];
            uint32_t neg = 0u;
#pragma unroll
            for (int jj = 0; jj < C; jj++) {
                if (jj < dc) {
                    const int v = wave_uniform(cload(G.col_idx + (j0 + jj)));
                    const float lv = Codec<Post<M>::kMsg>::dec(L[size_t(v) * S + s]);
                    const float r = first ? 0.f : Codec<M>::dec(R[size_t(j0 + jj) * S + s]);
                    const float qv = rule_q<M, RULE>(lv, r);
                    neg |= uint32_t(qv < 0.f) << jj;
                    uu[jj] = rule_in<M, RULE>(fabsf(qv));
                }
            }
            float run = Rule::identity();
#pragma unroll
            for (int jj = C - 1; jj >= 0; jj--) {
                if (jj < dc) {
                    sf[jj] = run;
                    run = Rule::combine(uu[jj], run);
                }
            }
            run = gmem(G.aggd)[size_t(cb + ch) * S + s];
#pragma unroll
            for (int jj = 0; jj < C; jj++) {
                if (jj < dc) {
                    const float mag = rule_mag<M, RULE>(Rule::combine(run, sf[jj]), rp);
                    const uint32_t sgn = parity ^ ((neg >> jj) & 1u);
                    R[size_t(j0 + jj) * S + s] = Codec<M>::enc(sgn ? -mag : mag);
                    run = Rule::combine(run, uu[jj]);
                }
            }
        }
        // the next item's wavefront 0 rewrites total_bits only after the first
        // barrier of that item, which every wavefront reaches after reading it here
    }
}

// Rows of the long class up to kWideRowMax edges (after its segmented rows):
// one workgroup of 16 wavefronts per (row, 64 slots), one 32-edge chunk per
// wavefront, chunk aggregates through LDS (wide_row).
template <int M, int RULE>
__global__ __launch_bounds__(1024) void eng_check_wide(const EngGraph *__restrict__ graphs, int32_t ngraphs,
                                                       const int32_t *__restrict__ counters, int32_t T,
                                                       int32_t early, int32_t par, float rp) {
    using MT = typename Codec<M>::T;
    __shared__ ChunkShare<1, kWideWaves> sh;
    __shared__ Work w;
    build_work(graphs, ngraphs, counters, kWideItems, 64, 1, w);
    const int lane = threadIdx.x & 63;
    const int wv = wave_uniform(threadIdx.x >> 6);
    const int total = wave_uniform(w.p[ngraphs]);
    int last_c = 0;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {     // uniform over the workgroup
        const int c = wave_uniform(work_graph(w, ngraphs, u, last_c));
        last_c = c;
        const EngGraph &G = graphs[c];
        const int32_t S = G.S;
        const int groups = wave_uniform(w.groups[c]);
        const int local = u - wave_uniform(w.p[c]);
        const int g = local % groups;
        const int rk = G.hub_seg + local / groups;
        const int s = g * 64 + lane;
        const int32_t ts = gmem(G.slot_t)[par * S + s];
        const bool active = ts >= 0 && ts < kStopped;
        if (__ballot(active) == 0) continue;   // same slots in every wavefront: uniform over the workgroup
        const bool syn_on = active && ts >= 1 && (early || ts == T);
        SlotSrc<1> src;
        src.alt[0] = active && ts == 0;
        src.any = src.alt[0];
        const u32x2 rdv = cload(reinterpret_cast<const u32x2 *>(G.class_rd) + G.class_begin[ldpc::kClassHub] + rk);
        const int e0 = wave_uniform(int(rdv.x));
        const int d = wave_uniform(int(rdv.y));
        const bool syn = wide_row<M, kWideChunk, kInMixed, RULE>(
            G.col_idx, e0, d, static_cast<const typename Post<M>::T *>(G.post), static_cast<MT *>(G.r), S, s, src,
            active, sh, wv, lane, rp);
        if (wv == 0 && syn_on && syn && gmem(G.fail)[s] != ts) gmem(G.fail)[s] = ts;
        __syncthreads();   // the shared aggregates are reused by the next item
    }
}

// --------------------------------------------------------------- bit pass

// Posterior of bit v for the lane's V slots (iteration t_s + 1 of every slot
// whose frame continues).  UNIFORM: one bit per wavefront.  The items of bit 0
// cover every slot below the extent once, and write the slots' next state.
// Slot state of a lane's V slots for the bit pass: the slot's iteration
// counter, whether the slot advances (its frame is still running after this
// pass's stop test) and, with 16-bit messages, whether its frame wants the fp32
// posterior.  The same for every bit of one slot group in one pass.
template <int V>
struct BitSlots {
    int32_t t[V];
    int32_t want[V];
    bool adv[V];
    bool any, all;
};

template <int M, int V>
__device__ __forceinline__ void bit_slots(const EngGraph &G, int s0, int32_t T, int32_t early, int32_t par,
                                          BitSlots<V> &b) {
    int32_t f[V];
    load_i32<V>(G.slot_t + par * G.S + s0, b.t);
    load_i32<V>(G.fail + s0, f);
    if constexpr (kPost16<M>) load_i32<V>(G.want32 + s0, b.want);
    b.any = false;
    b.all = true;
#pragma unroll
    for (int k = 0; k < V; k++) {
        b.adv[k] = b.t[k] >= 0 && b.t[k] < kStopped && !slot_stops(b.t[k], f[k], T, early);
        b.any |= b.adv[k];
        b.all &= b.adv[k];
    }
}

// One (bit, slot group) item of the bit pass, given the group's slot state.
template <int M, int V, bool UNIFORM>
__device__ __forceinline__ void bit_item(const EngGraph &G, int v, int s0, const BitSlots<V> &b, int32_t par,
                                         float bscale) {
    using MT = typename Codec<M>::T;
    const int32_t S = G.S;
    if (v == 0) {
        int32_t nx[V];
#pragma unroll
        for (int k = 0; k < V; k++)
            nx[k] = b.adv[k] ? b.t[k] + 1 : (b.t[k] >= 0 && b.t[k] < kStopped) ? b.t[k] + kStopped : b.t[k];
        store_i32<V>(G.slot_t + (par ^ 1) * S + s0, nx);
    }
    if (!b.any) return;
    const MT *R = static_cast<const MT *>(G.r);
    float sum[V];
    const int a = UNIFORM ? wave_uniform(cload(G.col_ptr + (v))) : cload(G.col_ptr + (v));
    const int e = UNIFORM ? wave_uniform(cload(G.col_ptr + (v + 1))) : cload(G.col_ptr + (v + 1));
    bit_posterior<M, V, UNIFORM>(G.csc_to_csr, a, e, R, S, s0, G.lch + size_t(v) * S, bscale, sum);
    using PT = typename Post<M>::T;
    PT *post = static_cast<PT *>(G.post);
    if (b.all) {
        store_post<V>(post + size_t(v) * S + s0, sum);
    } else {
#pragma unroll
        for (int k = 0; k < V; k++)
            if (b.adv[k]) store_post1(post + size_t(v) * S + s0 + k, sum[k]);
    }
    if constexpr (kPost16<M>) {
#pragma unroll
        for (int k = 0; k < V; k++)
            if (b.adv[k] && b.want[k]) gmem(G.lpost)[size_t(v) * S + s0 + k] = sum[k];
    }
}

template <int M, int V>
__global__ __launch_bounds__(256) void eng_bit(const EngGraph *__restrict__ graphs, int32_t ngraphs,
                                               const int32_t *__restrict__ counters, int32_t T, int32_t early,
                                               int32_t par, float bscale) {
    // The previous step's turnover and admission are complete: move each
    // graph's queue head past the frames it admitted and empty its list
    // (a no-op in the later passes of a step).
    if (blockIdx.x == 0 && int(threadIdx.x) < ngraphs) {
        const EngGraph &H = graphs[threadIdx.x];
        *gmem(H.head) += *gmem(H.taken);
        *gmem(H.taken) = 0;
        *gmem(H.list_count) = 0;
    }
    __shared__ Work w;
    build_work<kPackAll>(graphs, ngraphs, counters, kBitItems, 64 * V, 1, w);
    const int lane = threadIdx.x & 63;
    const int total = wave_uniform(w.p[ngraphs]);
    const int stride = int(gridDim.x * (blockDim.x >> 6));
    int prev_c = -1, prev_g = -1;
    BitSlots<V> bs;
    int last_c = 0;
    for (int item = wave_uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6); item < total; item += stride) {
        const int c = wave_uniform(work_graph(w, ngraphs, item, last_c));
        last_c = c;
        const EngGraph &G = graphs[c];
        const int local = item - wave_uniform(w.p[c]);
        const int rpw = wave_uniform(w.rpw[c]);
        if (rpw == 1) {
            const int groups = wave_uniform(w.groups[c]);
            const int v = local / groups;
            const int g = local - v * groups;
            const int s0 = (g * 64 + lane) * V;
            // consecutive items of a wavefront often share their graph and slot
            // group (one group per pool of up to 64 V slots): keep its state
            if (c != prev_c || g != prev_g) {
                bit_slots<M, V>(G, s0, T, early, par, bs);
                prev_c = c;
                prev_g = g;
            }
            bit_item<M, V, true>(G, v, s0, bs, par, bscale);
        } else {
            const int lpr = 64 / rpw;
            const int v = local * rpw + lane / lpr;
            if (v < G.n) {
                const int s0 = (lane % lpr) * V;
                BitSlots<V> pb;
                bit_slots<M, V>(G, s0, T, early, par, pb);
                bit_item<M, V, false>(G, v, s0, pb, par, bscale);
            }
        }
    }
}

// ------------------------------------------------------ advance / turnover

// One thread per slot, after the step's last bit pass (which wrote row `par`
// of the slot states): per-frame results of the stopped frames, the graph's
// turnover list (stopped frames, and empty slots while the graph has queued
// frames), and row 0 brought up to date for the next step.
// Pool sizes are multiples of 64, so a wavefront never spans two graphs; each
// wavefront appends its entries in slot order with one atomic.
__global__ __launch_bounds__(256) void eng_advance(const EngGraph *__restrict__ graphs, Prefix pre, int32_t T,
                                                   const int32_t *__restrict__ counters, int32_t par) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int c = 0;
    bool listme = false, stopped = false;
    int32_t ent = 0;
    if (x < pre.p[pre.count]) {
        c = find_graph(pre, x);
        const EngGraph &G = graphs[c];
        const int s = x - pre.p[c];
        const bool fresh = par && s < gmem(counters)[ctr_extent(pre.count, c)];   // row 1 holds this slot's state
        const int32_t t = gmem(G.slot_t)[fresh ? G.S + s : s];
        if (fresh) gmem(G.slot_t)[s] = t;
        if (t < 0) {
            listme = *gmem(G.head) < *gmem(G.tail);
            ent = s;
        } else if (t >= kStopped) {
            const int32_t ts = t - kStopped;
            const int32_t f = gmem(G.fail)[s];
            const EngFrame fr = load_frame(G.slot_desc + s);
            *gmem(fr.ok) = (ts < T) ? uint8_t(1) : uint8_t(f != T);
            *gmem(fr.iters) = ts;
            listme = stopped = true;
            ent = s | int32_t(0x80000000u);
        }
    }
    const uint64_t m = __ballot(listme);
    if (m == 0) return;
    const uint64_t ms = __ballot(stopped);
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    const EngGraph &G = graphs[__shfl(c, leader)];
    int base = 0;
    if (lane == leader) {
        base = atomicAdd(G.list_count, __popcll(m));
        if (ms) atomicAdd(G.retired, __popcll(ms));
    }
    base = __shfl(base, leader);
    if (listme) gmem(G.list)[base + __popcll(m & ((uint64_t(1) << lane) - 1u))] = ent;
}

// Workgroup item = (graph, 64 consecutive list entries, 64 bits).  Stopped
// entries write their estimate (bit = 1 iff Lpost < 0, Algorithm 6) and the
// optional posterior to the frame's outputs; entry i receives the channel LLRs
// of queue entry head + i while there is one.  Each 64 x 64 tile goes through
// LDS, so the slot-major state rows and the frame-major user rows are both
// accessed in contiguous runs (the list is in slot order within each run).
constexpr int kTile = 64;

// Posterior of bit v in slot s from the check pass's storage.
__device__ __forceinline__ float post_value(const EngGraph &G, int v, int s) {
    const size_t at = size_t(v) * G.S + s;
    return G.post16 ? float(gmem(static_cast<const _Float16 *>(G.post))[at])
                    : gmem(static_cast<const float *>(G.post))[at];
}

__global__ __launch_bounds__(256) void eng_turnover(const EngGraph *__restrict__ graphs, int32_t ngraphs,
                                                    int32_t *__restrict__ counters) {
    __shared__ int32_t base[kMaxGraphs + 1];
    __shared__ float tile[kTile][kTile + 1];
    __shared__ int32_t slot_of[kTile];
    __shared__ uint8_t *bits_of[kTile];
    __shared__ float *lout_of[kTile];
    __shared__ const float *src_of[kTile];
    __shared__ int32_t any_out, any_in;
    const int tid = threadIdx.x;
    if (tid < 64) {   // one lane per graph
        int32_t items = 0;
        if (tid < ngraphs) {
            const auto ctr = gmem(counters);
            const int32_t cnt = ctr[ctr_list_count(tid)];
            items = (cnt + kTile - 1) / kTile * ((graphs[tid].n + kTile - 1) / kTile);
            // the tail is constant within a step: this is the number admitted now
            if (blockIdx.x == 0) ctr[ctr_taken(ngraphs, tid)] = min(cnt, ctr[4 * tid + 1] - ctr[4 * tid]);
        }
        scan_items<int32_t>(items, ngraphs, base);
    }
    __syncthreads();
    const int total = base[ngraphs];
    const int r = tid >> 6, l = tid & 63;
    int last_c = 0;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {     // uniform over the workgroup
        int c = last_c;   // items in increasing order: start from the previous item's graph
        while (c + 1 < ngraphs && u >= base[c + 1]) c++;
        last_c = c;
        const EngGraph &G = graphs[c];
        const int32_t S = G.S, n = G.n;
        const int nvt = (n + kTile - 1) / kTile;
        const int local = u - base[c];
        const int i0 = (local / nvt) * kTile;
        const int v0 = (local % nvt) * kTile;
        if (tid < kTile) {
            const int i = i0 + tid;
            const int32_t cnt = *gmem(G.list_count);
            int32_t s = 0;
            uint8_t *bo = nullptr;
            float *lo = nullptr;
            const float *src = nullptr;
            if (i < cnt) {
                const int32_t ent = gmem(G.list)[i];
                s = ent & 0x7fffffff;
                if (ent < 0) {
                    const EngFrame fr = load_frame(G.slot_desc + s);
                    bo = fr.bits;
                    lo = fr.llr_out;
                }
                const int32_t qi = *gmem(G.head) + i;
                if (qi < *gmem(G.tail)) src = load_frame(G.queue + qi % G.cap).llr;
            }
            slot_of[tid] = s;
            bits_of[tid] = bo;
            lout_of[tid] = lo;
            src_of[tid] = src;
            const uint64_t mo = __ballot(bo != nullptr), mi = __ballot(src != nullptr);
            if (tid == 0) {
                any_out = mo != 0;
                any_in = mi != 0;
            }
        }
        __syncthreads();
        if (any_out) {
            // posterior rows of the listed slots -> tile[v][entry]
            for (int k = r; k < kTile; k += 4) {
                const int v = v0 + k;
                if (v < n && bits_of[l])
                    tile[k][l] = lout_of[l] ? gmem(G.lpost)[size_t(v) * S + slot_of[l]] : post_value(G, v, slot_of[l]);
            }
            __syncthreads();
            // tile -> each stopped frame's output row
            for (int k = r; k < kTile; k += 4) {
                const int v = v0 + l;
                uint8_t *bo = bits_of[k];
                if (v < n && bo) {
                    const float x = tile[l][k];
                    gmem(bo)[v] = x < 0.f;
                    if (lout_of[k]) gmem(lout_of[k])[v] = x;
                }
            }
            __syncthreads();
        }
        if (any_in) {
            // each admitted frame's channel row -> tile[v][entry]
            for (int k = r; k < kTile; k += 4) {
                const int v = v0 + l;
                const float *src = src_of[k];
                if (v < n && src) tile[l][k] = canon_llr(gmem(src)[v]);
            }
            __syncthreads();
            // tile -> channel rows of the slots; the posterior entries start as
            // the channel LLRs, which the slot's first check pass reads
            for (int k = r; k < kTile; k += 4) {
                const int v = v0 + k;
                if (v < n && src_of[l]) {
                    const size_t at = size_t(v) * S + slot_of[l];
                    gmem(G.lch)[at] = tile[k][l];
                    if (G.post16) *gmem(static_cast<_Float16 *>(G.post) + at) = post16_enc(tile[k][l]);
                    else *gmem(static_cast<float *>(G.post) + at) = tile[k][l];
                }
            }
        }
        __syncthreads();   // the tile and entry tables are reused by the next item
    }
}

// Exclusive prefix count of `flag` over a 1024-thread workgroup (16 wavefronts);
// `total` receives the workgroup's count.  `sh` holds 16 ints.
__device__ __forceinline__ int block_rank(bool flag, int32_t *sh, int &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t m = __ballot(flag);
    const int in_wave = __popcll(m & ((uint64_t(1) << lane) - 1u));
    if (lane == 0) sh[w] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
    for (int i = 0; i < nw; i++) {
        const int c = sh[i];
        before += i < w ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return before + in_wave;
}

// One workgroup per graph, after the turnover.  Slot states are row 0.
// Admission: every listed slot counts its stopped frame as done (its outputs
// are complete) and takes the next queued frame, or stays empty when the
// graph's queue ran dry.
// Repack (REPACK): when nothing is queued any more, A slots hold frames and
// X - 1 is the highest such slot, and 2 A <= X, the frames in slots >= A move
// into the empty slots below A (k-th one up to the k-th hole).  This kernel
// moves the per-slot bookkeeping; eng_repack_move copies the state columns.
template <bool REPACK>
__global__ __launch_bounds__(1024) void eng_admit(const EngGraph *__restrict__ graphs) {
    __shared__ int32_t sh[16];
    __shared__ int32_t red[2][16];
    const EngGraph &G = graphs[blockIdx.x];
    const int tid = threadIdx.x;
    const int32_t count = *gmem(G.list_count);
    const int32_t taken = *gmem(G.taken);
    const int32_t head = *gmem(G.head);
    for (int i = tid; i < count; i += blockDim.x) {
        const int32_t ent = gmem(G.list)[i];
        const int s = ent & 0x7fffffff;
        if (ent < 0) {
            const EngFrame old = load_frame(G.slot_desc + s);
            if (old.done) atomicAdd(old.done, 1);
        }
        if (i < taken) {
            const int32_t qi = head + i;
            const EngFrame fr = load_frame(G.queue + qi % G.cap);
            store_frame(G.slot_desc + s, fr);
            gmem(G.slot_t)[s] = 0;
            gmem(G.fail)[s] = 0;
            gmem(G.want32)[s] = fr.llr_out != nullptr;
        } else {
            gmem(G.slot_t)[s] = -1;
        }
    }
    if (tid == 0) *gmem(G.moves) = 0;
    __syncthreads();
    const int S = G.S;
    int a = 0, x = 0;
    for (int s = tid; s < S; s += blockDim.x)
        if (gmem(G.slot_t)[s] >= 0) { a++; x = s + 1; }
    // workgroup sum of a, max of x
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off);
        x = max(x, __shfl_down(x, off));
    }
    if ((tid & 63) == 0) { red[0][tid >> 6] = a; red[1][tid >> 6] = x; }
    __syncthreads();
    int A = 0, X = 0;
    for (int i = 0; i < int(blockDim.x >> 6); i++) { A += red[0][i]; X = max(X, red[1][i]); }
    // queued frames fill the holes at the next turnovers; repack only a drained pool
    if (!REPACK || head + taken < *gmem(G.tail) || X < kRepackMinExtent || 2 * A > X) {
        if (tid == 0) *gmem(G.extent) = X;
        return;
    }
    int holes = 0, srcs = 0;
    for (int s0 = 0; s0 < X; s0 += blockDim.x) {
        const int s = s0 + tid;
        const bool occ = s < X && gmem(G.slot_t)[s] >= 0;
        int th = 0, ts = 0;
        const int rh = block_rank(s < A && !occ, sh, th);
        const int rs = block_rank(s >= A && occ, sh, ts);
        if (s < A && !occ) gmem(G.move_dst)[holes + rh] = s;
        if (s >= A && occ) gmem(G.move_src)[srcs + rs] = s;
        holes += th;
        srcs += ts;
    }
    __syncthreads();   // the move lists are complete (holes == srcs)
    for (int k = tid; k < holes; k += blockDim.x) {
        const int src = gmem(G.move_src)[k], dst = gmem(G.move_dst)[k];
        store_frame(G.slot_desc + dst, load_frame(G.slot_desc + src));
        gmem(G.slot_t)[dst] = gmem(G.slot_t)[src];
        gmem(G.fail)[dst] = gmem(G.fail)[src];
        gmem(G.want32)[dst] = gmem(G.want32)[src];
        gmem(G.slot_t)[src] = -1;
    }
    if (tid == 0) {
        *gmem(G.moves) = holes;
        *gmem(G.extent) = A;
    }
}

// Copy the state columns of the repacked frames: every message row (edge),
// channel-LLR row and posterior row of the graph (both posterior copies for
// 16-bit messages), slot move_src[k] to slot move_dst[k].  Sources lie above every destination, so the copies are
// independent.  MSG_BYTES is the stored message size.
template <int MSG_BYTES>
__global__ __launch_bounds__(256) void eng_repack_move(const EngGraph *__restrict__ graphs, int32_t ngraphs,
                                                       const int32_t *__restrict__ counters) {
    using MsgWord = typename std::conditional<MSG_BYTES == 1, uint8_t,
                                              typename std::conditional<MSG_BYTES == 2, uint16_t, uint32_t>::type>::type;
    __shared__ long long base[kMaxGraphs + 1];
    __shared__ int32_t nm[kMaxGraphs];
    if (threadIdx.x < 64) {   // one lane per graph
        long long items = 0;
        if (int(threadIdx.x) < ngraphs) {
            const int c = threadIdx.x;
            const int32_t moves = gmem(counters)[ctr_moves(ngraphs, c)];
            nm[c] = moves;
            const long long rows = (long long)graphs[c].E + (graphs[c].post16 ? 3 : 2) * (long long)graphs[c].n;
            items = moves > 0 ? (rows + kMoveRows - 1) / kMoveRows : 0;
        }
        scan_items<long long>(items, ngraphs, base);
    }
    __syncthreads();
    const int64_t total = base[ngraphs];
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        int c = 0;
        while (c + 1 < ngraphs && u >= base[c + 1]) c++;
        const EngGraph &G = graphs[c];
        const int moves = nm[c];
        const int64_t E = G.E, n = G.n, S = G.S;
        const int64_t r0 = (u - base[c]) * kMoveRows;
        const int rcount = int(min(int64_t(kMoveRows), E + (G.post16 ? 3 : 2) * n - r0));
        for (int idx = threadIdx.x; idx < rcount * moves; idx += blockDim.x) {
            const int rr = idx / moves;
            const int k = idx - rr * moves;
            const int64_t row = r0 + rr;
            const int64_t src = gmem(G.move_src)[k], dst = gmem(G.move_dst)[k];
            if (row < E) {
                auto R = gmem(static_cast<MsgWord *>(G.r));
                R[row * S + dst] = R[row * S + src];
            } else if (row >= E + n && row < E + 2 * n && G.post16) {
                auto P = gmem(static_cast<uint16_t *>(G.post));
                const int64_t v = row - E - n;
                P[v * S + dst] = P[v * S + src];
            } else {
                // channel rows, then the fp32 posterior (after the fp16 rows when there are some)
                auto L = gmem(row < E + n ? G.lch : G.lpost);
                const int64_t v = row < E + n ? row - E : row - E - (G.post16 ? 2 : 1) * n;
                L[v * S + dst] = L[v * S + src];
            }
        }
    }
}

__global__ void eng_publish(int32_t *tail, int32_t value) { *tail = value; }

// Between steps: apply the last admissions to the queue heads and empty the
// turnover lists, as the first bit pass of a step does (used before an
// admission outside the step sequence).
__global__ void eng_open_lists(const EngGraph *__restrict__ graphs, int32_t ngraphs) {
    if (int(threadIdx.x) < ngraphs) {
        const EngGraph &H = graphs[threadIdx.x];
        *gmem(H.head) += *gmem(H.taken);
        *gmem(H.taken) = 0;
        *gmem(H.list_count) = 0;
    }
}

}  // namespace

// ===================================================================== host

struct ldpc_engine {
    int device = -1;
    hipStream_t stream = nullptr;
    int32_t ngraphs = 0, T = 0, V = 4, K = 8, I = 1, msg = kF32;   // I: decoder iterations per step
    int rule = kRuleSP;      // check rule (RuleKind) and its parameter
    float rule_param = 0.f;
    uint32_t flags = 0;
    bool early = true;
    bool repack = true;
    bool pack = true;        // packed row items for nearly drained pools
    bool direct = false;     // enqueue each step's kernels instead of replaying the captured graph
    std::vector<const ldpc_graph *> graphs;
    std::vector<int32_t> S, cap;
    std::vector<EngGraph> hg;
    void *dmem = nullptr;
    size_t dbytes = 0;
    EngGraph *d_graphs = nullptr;
    int32_t *d_counters = nullptr;   // [ngraphs][4]: head, tail, retired, list count; then [ngraphs] taken, moves, extent
    ldpc_frame *h_stage = nullptr;   // pinned mirror of every queue ring
    std::vector<size_t> stage_off;
    int32_t *h_counters = nullptr;   // pinned copy of d_counters
    int32_t *h_async[2] = {nullptr, nullptr};   // counters copied after replays, by replay parity
    hipEvent_t ev_async[2] = {nullptr, nullptr};
    bool async_pending[2] = {false, false};
    int parity = 0;
    std::vector<int64_t> submitted, head_seen, retired_seen;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Prefix pre_slots;
    bool has_rows[3] = {false, false, false}, has_hub = false, has_wide = false;
    int64_t bit_waves = 0, hub_blocks = 0, wide_blocks = 0, total_slots = 0, row_waves[3] = {0, 0, 0};   // with every slot occupied
    unsigned grid_rows[3] = {1, 1, 1}, grid_hub = 1, grid_wide = 1, grid_bit = 1;   // workgroups per launch (grid-stride)
    unsigned grid_packed = 256;      // packed row items: few rows per graph once drained
    unsigned grid_chunk_narrow = 1;  // chunked rows of drained pools at one slot per lane
    int64_t chunk_rows = 0;          // rows of the chunked class over all graphs
};

namespace {

using ldpc::set_error;

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Register-row class `cls`: unpacked items in one launch and, when packing is
// on, packed items in a second one, so neither kernel carries the other's body.
template <int M, int V, int DMAX, int RULE>
void launch_rows(ldpc_engine *e, int cls, unsigned grid, int32_t par) {
    const int32_t early = e->early ? 1 : 0;
    const float rp = e->rule_param;
    if (e->pack) {
        hipLaunchKernelGGL((eng_check_rows<M, V, DMAX, kPackOnlyFlat, RULE>), dim3(grid), dim3(256), 0, e->stream,
                           e->d_graphs, e->ngraphs, e->d_counters, int32_t(cls), e->T, early, par, rp);
        hipLaunchKernelGGL((eng_check_rows<M, V, DMAX, kPackOnlyPacked, RULE>), dim3(e->grid_packed), dim3(256), 0,
                           e->stream, e->d_graphs, e->ngraphs, e->d_counters, int32_t(cls), e->T, early, par, rp);
    } else {
        hipLaunchKernelGGL((eng_check_rows<M, V, DMAX, kPackNone, RULE>), dim3(grid), dim3(256), 0, e->stream,
                           e->d_graphs, e->ngraphs, e->d_counters, int32_t(cls), e->T, early, par, rp);
    }
}

template <int M, int V, int RULE>
void enqueue_step_rule(ldpc_engine *e) {
    hipStream_t st = e->stream;
    const int32_t early = e->early ? 1 : 0;
    const int32_t ng = e->ngraphs;
    const float rp = e->rule_param;
    for (int32_t j = 0; j < e->I; j++) {
        const int32_t par = j & 1;
        if (e->has_rows[0])
            launch_rows<M, V, 8, RULE>(e, ldpc::kClassD8, e->grid_rows[0], par);
        if (e->has_rows[1])
            launch_rows<M, ldpc::class_lane_slots(ldpc::kClassD16, V), 16, RULE>(e, ldpc::kClassD16, e->grid_rows[1],
                                                                                 par);
        if (e->has_rows[2]) {
            constexpr int W = ldpc::class_waves_per_row(ldpc::kClassD128);
            const int32_t wide_unit = 64 * V;
            bool split = false;
            if constexpr (V > 1) {
                split = e->pack;
                if (split) {
                    hipLaunchKernelGGL((eng_check_chunk<M, V, W, RULE, kSplitWide>), dim3(e->grid_rows[2]), dim3(256),
                                       0, st, e->d_graphs, ng, e->d_counters, int32_t(ldpc::kClassD128), e->T, early,
                                       par, rp, wide_unit);
                    hipLaunchKernelGGL((eng_check_chunk<M, 1, W, RULE, kSplitNarrow>), dim3(e->grid_chunk_narrow),
                                       dim3(256), 0, st, e->d_graphs, ng, e->d_counters, int32_t(ldpc::kClassD128),
                                       e->T, early, par, rp, wide_unit);
                }
            }
            if (!split)
                hipLaunchKernelGGL((eng_check_chunk<M, V, W, RULE, kSplitNone>), dim3(e->grid_rows[2]), dim3(256), 0,
                                   st, e->d_graphs, ng, e->d_counters, int32_t(ldpc::kClassD128), e->T, early, par,
                                   rp, wide_unit);
        }
        if (e->has_wide)
            hipLaunchKernelGGL((eng_check_wide<M, RULE>), dim3(e->grid_wide), dim3(64 * kWideWaves), 0, st,
                               e->d_graphs, ng, e->d_counters, e->T, early, par, rp);
        if (e->has_hub)
            hipLaunchKernelGGL((eng_check_hub<M, RULE>), dim3(e->grid_hub), dim3(256), 0, st, e->d_graphs, ng,
                               e->d_counters, e->T, early, par, rp);
        hipLaunchKernelGGL((eng_bit<M, V>), dim3(e->grid_bit), dim3(256), 0, st, e->d_graphs, ng, e->d_counters,
                           e->T, early, par, MsgUnits<M, RULE>::kBitScale);
    }
    const unsigned slot_blocks = unsigned((e->total_slots + 255) / 256);
    hipLaunchKernelGGL(eng_advance, dim3(slot_blocks), dim3(256), 0, st, e->d_graphs, e->pre_slots, e->T,
                       e->d_counters, int32_t(e->I & 1));
    hipLaunchKernelGGL(eng_turnover, dim3(unsigned(kTurnoverBlocks)), dim3(256), 0, st, e->d_graphs, e->ngraphs,
                       e->d_counters);
    if (e->repack) {
        hipLaunchKernelGGL(eng_admit<true>, dim3(unsigned(e->ngraphs)), dim3(1024), 0, st, e->d_graphs);
        hipLaunchKernelGGL((eng_repack_move<sizeof(typename Codec<M>::T)>), dim3(unsigned(kMoveBlocks)), dim3(256), 0,
                           st, e->d_graphs, e->ngraphs, e->d_counters);
    } else {
        hipLaunchKernelGGL(eng_admit<false>, dim3(unsigned(e->ngraphs)), dim3(1024), 0, st, e->d_graphs);
    }
}

template <int M, int V>
void enqueue_step(ldpc_engine *e) {
    switch (e->rule) {
        case kRuleNMS: enqueue_step_rule<M, V, kRuleNMS>(e); break;
        case kRuleOMS: enqueue_step_rule<M, V, kRuleOMS>(e); break;
        default: enqueue_step_rule<M, V, kRuleSP>(e); break;
    }
}

template <int M>
void enqueue_step_v(ldpc_engine *e) {
    switch (e->V) {
        case 1: enqueue_step<M, 1>(e); break;
        case 2: enqueue_step<M, 2>(e); break;
        default: enqueue_step<M, 4>(e); break;
    }
}

void enqueue_steps(ldpc_engine *e, int steps) {
    for (int i = 0; i < steps; i++) {
        switch (e->msg) {
            case kF16: enqueue_step_v<kF16>(e); break;
            case kBF16: enqueue_step_v<kBF16>(e); break;
            case kQ8: enqueue_step_v<kQ8>(e); break;
            default: enqueue_step_v<kF32>(e); break;
        }
    }
}

// Workgroups per launch: as many as the device keeps resident at once (the
// kernels loop over their items), never more than a full pool needs.  The
// residency figure is multiplied by LDPC_ENGINE_GRID_FACTOR (1..16, default 1).
int grid_factor() {
    const char *v = std::getenv("LDPC_ENGINE_GRID_FACTOR");
    const int f = v ? std::atoi(v) : 1;
    return f >= 1 && f <= 16 ? f : 1;
}

template <int M, int V>
void size_grids(ldpc_engine *e, int cus) {
    auto fit = [cus](const void *k, int64_t need, int block = 256) -> unsigned {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, 0) != hipSuccess || per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 1;
        }
        if (const char *v = std::getenv("LDPC_ENGINE_BLOCKS_PER_CU")) {
            const int b = std::atoi(v);
            if (b >= 1 && b <= 1024) per_cu = b;
        }
        return unsigned(std::max<int64_t>(1, std::min<int64_t>(need, int64_t(per_cu) * cus * grid_factor())));
    };
    e->grid_rows[0] = fit(reinterpret_cast<const void *>(&eng_check_rows<M, V, 8, kPackOnlyFlat, kRuleSP>),
                          (e->row_waves[0] + 3) / 4);
    e->grid_rows[1] = fit(reinterpret_cast<const void *>(&eng_check_rows<M, ldpc::class_lane_slots(ldpc::kClassD16, V), 16,
                                                                         kPackOnlyFlat, kRuleSP>),
                          (e->row_waves[1] + 3) / 4);
    e->grid_packed = fit(reinterpret_cast<const void *>(&eng_check_rows<M, V, 8, kPackOnlyPacked, kRuleSP>),
                         std::max<int64_t>(1, (e->row_waves[0] + e->row_waves[1] + 3) / 4));
    e->grid_rows[2] = fit(reinterpret_cast<const void *>(&eng_check_chunk<M, V, ldpc::class_waves_per_row(ldpc::kClassD128),
                                                                          kRuleSP, kSplitWide>),
                          e->row_waves[2]);
    // the narrow launch covers at most 32 V slots per row of each graph: V / 2 groups of 64
    if constexpr (V > 1)
        e->grid_chunk_narrow = fit(reinterpret_cast<const void *>(
                                       &eng_check_chunk<M, 1, ldpc::class_waves_per_row(ldpc::kClassD128), kRuleSP,
                                                        kSplitNarrow>),
                                   std::max<int64_t>(1, e->chunk_rows * (V / 2)));
    e->grid_hub = fit(reinterpret_cast<const void *>(&eng_check_hub<M, kRuleSP>), e->hub_blocks);
    e->grid_wide = fit(reinterpret_cast<const void *>(&eng_check_wide<M, kRuleSP>), e->wide_blocks, 64 * kWideWaves);
    e->grid_bit = fit(reinterpret_cast<const void *>(&eng_bit<M, V>), (e->bit_waves + 3) / 4);
}

template <int M>
void size_grids_v(ldpc_engine *e, int cus) {
    switch (e->V) {
        case 1: size_grids<M, 1>(e, cus); break;
        case 2: size_grids<M, 2>(e, cus); break;
        default: size_grids<M, 4>(e, cus); break;
    }
}

void destroy_engine(ldpc_engine *e) {
    if (!e) return;
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    if (e->dmem) (void)hipFree(e->dmem);
    if (e->h_stage) (void)hipHostFree(e->h_stage);
    if (e->h_counters) (void)hipHostFree(e->h_counters);
    for (int p = 0; p < 2; p++) {
        if (e->h_async[p]) (void)hipHostFree(e->h_async[p]);
        if (e->ev_async[p]) (void)hipEventDestroy(e->ev_async[p]);
    }
    if (e->stream) (void)hipStreamDestroy(e->stream);
    (void)hipGetLastError();
    delete e;
}

ldpc_status hip_fail(ldpc_engine *e, const char *what, hipError_t err) {
    set_error(std::string(what) + ": " + hipGetErrorString(err));
    (void)hipGetLastError();
    destroy_engine(e);
    return err == hipErrorOutOfMemory ? LDPC_E_NOMEM : LDPC_E_DEVICE;
}

}  // namespace

extern "C" ldpc_status ldpc_engine_create(const ldpc_graph *const *graphs, int32_t ngraphs, const int32_t *slots,
                                          const int32_t *queue_cap, int32_t max_iter, uint32_t flags,
                                          const ldpc_engine_opts *opts, ldpc_engine **out) {
    if (!out || !graphs || !slots || !queue_cap) { set_error("ldpc_engine_create: NULL argument"); return LDPC_E_INVAL; }
    if (ngraphs < 1 || ngraphs > kMaxGraphs) { set_error("ldpc_engine_create: ngraphs must be in 1..32"); return LDPC_E_INVAL; }
    if (max_iter < 1 || max_iter >= kStopped) {
        set_error("ldpc_engine_create: max_iter must be in 1..2^30-1");
        return LDPC_E_INVAL;
    }
    const uint32_t known = LDPC_NO_EARLY_STOP | LDPC_MSG_FP16 | LDPC_MSG_BF16 | LDPC_MSG_Q8;
    if ((flags & ~known) || __builtin_popcount(flags & (LDPC_MSG_FP16 | LDPC_MSG_BF16 | LDPC_MSG_Q8)) > 1) {
        set_error("ldpc_engine_create: bad flags");
        return LDPC_E_INVAL;
    }
    int V = 4, K = 8, I = 1;
    bool repack = true;
    if (opts) {
        for (int32_t r : opts->reserved)
            if (r != 0) { set_error("ldpc_engine_create: reserved options must be 0"); return LDPC_E_INVAL; }
        if (opts->lane_slots) {
            if (opts->lane_slots != 1 && opts->lane_slots != 2 && opts->lane_slots != 4) {
                set_error("ldpc_engine_create: lane_slots must be 1, 2 or 4");
                return LDPC_E_INVAL;
            }
            V = opts->lane_slots;
        }
        if (opts->graph_steps < 0 || opts->graph_steps > 1024) {
            set_error("ldpc_engine_create: graph_steps must be in 0..1024");
            return LDPC_E_INVAL;
        }
        if (opts->graph_steps) K = opts->graph_steps;
        if (opts->no_compaction != 0 && opts->no_compaction != 1) {
            set_error("ldpc_engine_create: no_compaction must be 0 or 1");
            return LDPC_E_INVAL;
        }
        repack = opts->no_compaction == 0;
        if (opts->iters_per_step < 0 || opts->iters_per_step > 16) {
            set_error("ldpc_engine_create: iters_per_step must be in 0..16");
            return LDPC_E_INVAL;
        }
        if (opts->iters_per_step) I = opts->iters_per_step;
        std::string why;
        if (!ldpc::rule_ok(opts->rule, opts->rule_param, why)) {
            set_error("ldpc_engine_create: " + why);
            return LDPC_E_INVAL;
        }
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); set_error("ldpc_engine_create: no device"); return LDPC_E_DEVICE; }
    for (int32_t c = 0; c < ngraphs; c++) {
        if (!graphs[c] || graphs[c]->host_only || graphs[c]->device != dev) {
            set_error("ldpc_engine_create: graph " + std::to_string(c) + " is NULL, host-only or on another device");
            return LDPC_E_INVAL;
        }
        if (slots[c] < 1 || queue_cap[c] < 1) {
            set_error("ldpc_engine_create: slots and queue_cap must be >= 1");
            return LDPC_E_INVAL;
        }
    }
    ldpc_engine *e = new (std::nothrow) ldpc_engine;
    if (!e) { set_error("ldpc_engine_create: out of host memory"); return LDPC_E_NOMEM; }
    e->device = dev;
    e->ngraphs = ngraphs;
    e->T = max_iter;
    e->flags = flags;
    e->early = !(flags & LDPC_NO_EARLY_STOP);
    e->msg = (flags & LDPC_MSG_FP16) ? kF16 : (flags & LDPC_MSG_BF16) ? kBF16 : (flags & LDPC_MSG_Q8) ? kQ8 : kF32;
    e->V = V;
    e->K = K;
    e->I = I;
    if (opts && opts->rule != LDPC_RULE_SUM_PRODUCT) {
        e->rule = opts->rule == LDPC_RULE_MIN_SUM_NORMALIZED ? kRuleNMS : kRuleOMS;
        e->rule_param = opts->rule_param;
    }
    e->repack = repack;
    if (const char *v = std::getenv("LDPC_ENGINE_NO_PACK")) e->pack = v[0] != '1';
    if (const char *v = std::getenv("LDPC_ENGINE_DIRECT")) e->direct = v[0] == '1';
    e->graphs.assign(graphs, graphs + ngraphs);
    const int32_t unit = 64 * V;
    const size_t msg_bytes = e->msg == kF32 ? 4 : e->msg == kQ8 ? 1 : 2;

    // device layout: per graph state, then counters, turnover list, graph table
    size_t off = 0;
    struct Offs { size_t lch, lpost, post, r, t, fail, want, desc, aggd, aggpre, aggbits, queue, list, msrc, mdst; };
    const bool post16 = e->msg == kF16 || e->msg == kBF16;
    std::vector<Offs> go(static_cast<size_t>(ngraphs));
    for (int32_t c = 0; c < ngraphs; c++) {
        const ldpc_graph *g = graphs[c];
        const int32_t S = int32_t((int64_t(slots[c]) + unit - 1) / unit * unit);
        e->S.push_back(S);
        e->cap.push_back(queue_cap[c]);
        Offs &o = go[size_t(c)];
        o.lch = off;     off = al256(off + size_t(g->n) * S * 4);
        o.lpost = off;   off = al256(off + size_t(g->n) * S * 4);
        o.post = o.lpost;
        if (post16) { o.post = off; off = al256(off + size_t(g->n) * S * 2); }
        o.r = off;       off = al256(off + size_t(g->E) * S * msg_bytes);
        o.t = off;       off = al256(off + size_t(2) * S * 4);
        o.fail = off;    off = al256(off + size_t(S) * 4);
        o.want = off;    off = al256(off + size_t(S) * 4);
        o.desc = off;    off = al256(off + size_t(S) * sizeof(EngFrame));
        o.aggd = off;    off = al256(off + size_t(g->hub_chunks) * S * 4);
        o.aggpre = off;  off = al256(off + size_t(g->hub_chunks) * S * 4);
        o.aggbits = off; off = al256(off + size_t(g->hub_chunks) * S * 4);
        o.queue = off;   off = al256(off + size_t(queue_cap[c]) * sizeof(EngFrame));
        o.list = off;    off = al256(off + size_t(S) * 4);
        o.msrc = off;    off = al256(off + size_t(S) * 4);
        o.mdst = off;    off = al256(off + size_t(S) * 4);
        e->total_slots += S;
    }
    const size_t off_counters = off; off = al256(off + size_t(ngraphs) * kCounterInts * 4);
    const size_t off_graphs = off;   off = al256(off + size_t(ngraphs) * sizeof(EngGraph));
    e->dbytes = off;

    hipError_t err = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking);
    if (err != hipSuccess) return hip_fail(e, "ldpc_engine_create: hipStreamCreate", err);
    err = hipMalloc(&e->dmem, e->dbytes);
    if (err != hipSuccess) return hip_fail(e, "ldpc_engine_create: hipMalloc", err);
    char *base = static_cast<char *>(e->dmem);
    e->d_counters = reinterpret_cast<int32_t *>(base + off_counters);
    e->d_graphs = reinterpret_cast<EngGraph *>(base + off_graphs);

    for (int32_t c = 0; c < ngraphs; c++) {
        const ldpc_graph *g = graphs[c];
        const Offs &o = go[size_t(c)];
        EngGraph G{};
        G.col_idx = g->d_col_idx; G.col_ptr = g->d_col_ptr; G.csc_to_csr = g->d_csc_to_csr;
        G.class_rd = g->d_class_rd; G.hub_chunk_base = g->d_hub_chunk_base;
        G.n = g->n;
        G.E = int32_t(g->E);
        G.S = e->S[size_t(c)];
        for (int k = 0; k <= ldpc::kNumClasses; k++) G.class_begin[k] = g->class_begin[k];
        G.lch = reinterpret_cast<float *>(base + o.lch);
        G.lpost = reinterpret_cast<float *>(base + o.lpost);
        G.post = base + o.post;
        G.post16 = post16 ? 1 : 0;
        G.hub_seg = g->hub_seg_rows;
        G.want32 = reinterpret_cast<int32_t *>(base + o.want);
        G.r = base + o.r;
        G.slot_t = reinterpret_cast<int32_t *>(base + o.t);
        G.fail = reinterpret_cast<int32_t *>(base + o.fail);
        G.slot_desc = reinterpret_cast<EngFrame *>(base + o.desc);
        G.aggd = reinterpret_cast<float *>(base + o.aggd);
        G.aggpre = reinterpret_cast<float *>(base + o.aggpre);
        G.aggbits = reinterpret_cast<int32_t *>(base + o.aggbits);
        G.queue = reinterpret_cast<EngFrame *>(base + o.queue);
        G.cap = e->cap[size_t(c)];
        G.head = e->d_counters + 4 * c;
        G.tail = e->d_counters + 4 * c + 1;
        G.retired = e->d_counters + 4 * c + 2;
        G.list_count = e->d_counters + 4 * c + 3;
        G.taken = e->d_counters + 4 * ngraphs + c;
        G.moves = e->d_counters + 5 * ngraphs + c;
        G.extent = e->d_counters + 6 * ngraphs + c;
        G.list = reinterpret_cast<int32_t *>(base + o.list);
        G.move_src = reinterpret_cast<int32_t *>(base + o.msrc);
        G.move_dst = reinterpret_cast<int32_t *>(base + o.mdst);
        e->hg.push_back(G);
        // every slot starts empty, with defined message state
        if ((err = hipMemsetAsync(base + o.lch, 0, o.t - o.lch, e->stream)) != hipSuccess ||
            (err = hipMemsetAsync(G.slot_t, 0xff, size_t(2) * G.S * 4, e->stream)) != hipSuccess ||
            (err = hipMemsetAsync(G.fail, 0, size_t(G.S) * 4, e->stream)) != hipSuccess ||
            (err = hipMemsetAsync(G.want32, 0, size_t(G.S) * 4, e->stream)) != hipSuccess)
            return hip_fail(e, "ldpc_engine_create: hipMemsetAsync", err);
    }
    if ((err = hipMemsetAsync(e->d_counters, 0, size_t(ngraphs) * kCounterInts * 4, e->stream)) != hipSuccess ||
        (err = hipMemcpyAsync(e->d_graphs, e->hg.data(), e->hg.size() * sizeof(EngGraph), hipMemcpyHostToDevice,
                              e->stream)) != hipSuccess)
        return hip_fail(e, "ldpc_engine_create: initialisation", err);

    // work sizes with every slot occupied: waves (D8 rows, bits) or workgroups (chunked and long rows)
    for (int k = 0; k < 3; k++) {
        const int rpb = k < 2 ? 1 : 4 / ldpc::class_waves_per_row(k);
        const int vk = ldpc::class_lane_slots(k, V);
        int64_t tot = 0;
        for (int32_t c = 0; c < ngraphs; c++) {
            const ldpc_graph *g = graphs[c];
            const int64_t items = int64_t(g->class_begin[k + 1] - g->class_begin[k]) * (e->S[size_t(c)] / (64 * vk));
            tot += (items + rpb - 1) / rpb;
        }
        e->row_waves[k] = tot;
        e->has_rows[k] = tot > 0;
    }
    for (int32_t c = 0; c < ngraphs; c++)
        e->chunk_rows += graphs[c]->class_begin[ldpc::kClassD128 + 1] - graphs[c]->class_begin[ldpc::kClassD128];
    e->pre_slots.count = ngraphs;
    e->pre_slots.p[0] = 0;
    for (int32_t c = 0; c < ngraphs; c++) {
        const ldpc_graph *g = graphs[c];
        const int64_t hubs = g->class_begin[ldpc::kClassHub + 1] - g->class_begin[ldpc::kClassHub];
        e->hub_blocks += int64_t(g->hub_seg_rows) * (e->S[size_t(c)] / 64);
        e->wide_blocks += (hubs - g->hub_seg_rows) * (e->S[size_t(c)] / 64);
        e->bit_waves += int64_t(g->n) * (e->S[size_t(c)] / (64 * V));
        e->pre_slots.p[c + 1] = e->pre_slots.p[c] + e->S[size_t(c)];
    }
    e->has_hub = e->hub_blocks > 0;
    e->has_wide = e->wide_blocks > 0;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
            (void)hipGetLastError();
            cus = 1;
        }
        switch (e->msg) {
            case kF16: size_grids_v<kF16>(e, cus); break;
            case kBF16: size_grids_v<kBF16>(e, cus); break;
            case kQ8: size_grids_v<kQ8>(e, cus); break;
            default: size_grids_v<kF32>(e, cus); break;
        }
    }

    // pinned staging for queue entries and counters
    size_t stage = 0;
    for (int32_t c = 0; c < ngraphs; c++) { e->stage_off.push_back(stage); stage += size_t(e->cap[size_t(c)]); }
    if ((err = hipHostMalloc(reinterpret_cast<void **>(&e->h_stage), stage * sizeof(ldpc_frame), 0)) != hipSuccess ||
        (err = hipHostMalloc(reinterpret_cast<void **>(&e->h_counters), size_t(ngraphs) * kCounterInts * 4, 0)) != hipSuccess ||
        (err = hipHostMalloc(reinterpret_cast<void **>(&e->h_async[0]), size_t(ngraphs) * kCounterInts * 4, 0)) != hipSuccess ||
        (err = hipHostMalloc(reinterpret_cast<void **>(&e->h_async[1]), size_t(ngraphs) * kCounterInts * 4, 0)) != hipSuccess ||
        (err = hipEventCreateWithFlags(&e->ev_async[0], hipEventDisableTiming)) != hipSuccess ||
        (err = hipEventCreateWithFlags(&e->ev_async[1], hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "ldpc_engine_create: hipHostMalloc", err);
    e->submitted.assign(size_t(ngraphs), 0);
    e->head_seen.assign(size_t(ngraphs), 0);
    e->retired_seen.assign(size_t(ngraphs), 0);

    // capture K steps once
    if ((err = hipStreamSynchronize(e->stream)) != hipSuccess) return hip_fail(e, "ldpc_engine_create: sync", err);
    if ((err = hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "ldpc_engine_create: hipStreamBeginCapture", err);
    enqueue_steps(e, e->K);
    err = hipStreamEndCapture(e->stream, &e->graph);
    if (err != hipSuccess) return hip_fail(e, "ldpc_engine_create: hipStreamEndCapture", err);
    if ((err = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(e, "ldpc_engine_create: hipGraphInstantiate", err);
    *out = e;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_engine_destroy(ldpc_engine *e) {
    destroy_engine(e);
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_engine_info(const ldpc_engine *e, int64_t *device_bytes, int32_t *slots) {
    if (!e) { set_error("ldpc_engine_info: NULL engine"); return LDPC_E_INVAL; }
    if (device_bytes) *device_bytes = int64_t(e->dbytes);
    if (slots) for (int32_t c = 0; c < e->ngraphs; c++) slots[c] = e->S[size_t(c)];
    return LDPC_OK;
}

namespace {

// Take queue counters from replays that have already finished, without waiting.
void absorb_counters(ldpc_engine *e, const int32_t *h) {
    for (int32_t c = 0; c < e->ngraphs; c++) {
        const int64_t head = int64_t(h[4 * c]) + h[4 * e->ngraphs + c];
        e->head_seen[size_t(c)] = std::max(e->head_seen[size_t(c)], head);
        e->retired_seen[size_t(c)] = std::max<int64_t>(e->retired_seen[size_t(c)], h[4 * c + 2]);
    }
}

void refresh_counters(ldpc_engine *e) {
    for (int p = 0; p < 2; p++) {
        if (e->async_pending[p] && hipEventQuery(e->ev_async[p]) == hipSuccess) {
            absorb_counters(e, e->h_async[p]);
            e->async_pending[p] = false;
        }
    }
    (void)hipGetLastError();
}

}  // namespace

extern "C" ldpc_status ldpc_engine_stream(const ldpc_engine *e, void **hip_stream) {
    if (!e || !hip_stream) { set_error("ldpc_engine_stream: bad argument"); return LDPC_E_INVAL; }
    *hip_stream = e->stream;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_engine_capacity(const ldpc_engine *e_const, int32_t graph, int32_t *free_entries) {
    ldpc_engine *e = const_cast<ldpc_engine *>(e_const);
    if (!e || !free_entries || graph < 0 || graph >= e->ngraphs) { set_error("ldpc_engine_capacity: bad argument"); return LDPC_E_INVAL; }
    refresh_counters(e);
    const size_t c = size_t(graph);
    *free_entries = int32_t(e->cap[c] - (e->submitted[c] - e->head_seen[c]));
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_engine_submit(ldpc_engine *e, int32_t graph, const ldpc_frame *frames, int32_t count,
                                          void *hip_stream) {
    if (!e || graph < 0 || graph >= e->ngraphs || count < 0 || (count > 0 && !frames)) {
        set_error("ldpc_engine_submit: bad argument");
        return LDPC_E_INVAL;
    }
    if (count == 0) return LDPC_OK;
    const size_t c = size_t(graph);
    refresh_counters(e);
    const int64_t in_queue = e->submitted[c] - e->head_seen[c];
    if (in_queue + count > e->cap[c]) {
        set_error("ldpc_engine_submit: queue of graph " + std::to_string(graph) + " is full (" +
                  std::to_string(e->cap[c] - in_queue) + " free)");
        return LDPC_E_INVAL;
    }
    if (e->submitted[c] + count > INT32_MAX) { set_error("ldpc_engine_submit: frame counter overflow"); return LDPC_E_UNSUPPORTED; }
    hipError_t err;
    if (hip_stream) {
        hipEvent_t ev;
        if ((err = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) goto fail;
        err = hipEventRecord(ev, static_cast<hipStream_t>(hip_stream));
        if (err == hipSuccess) err = hipStreamWaitEvent(e->stream, ev, 0);
        (void)hipEventDestroy(ev);
        if (err != hipSuccess) goto fail;
    }
    {
        const int32_t cap = e->cap[c];
        ldpc_frame *ring = e->h_stage + e->stage_off[c];
        EngFrame *dq = e->hg[c].queue;
        int32_t pos = int32_t(e->submitted[c] % cap);
        int32_t left = count;
        const ldpc_frame *src = frames;
        while (left > 0) {
            const int32_t chunk = std::min(left, cap - pos);
            std::memcpy(ring + pos, src, size_t(chunk) * sizeof(ldpc_frame));
            if ((err = hipMemcpyAsync(dq + pos, ring + pos, size_t(chunk) * sizeof(ldpc_frame), hipMemcpyHostToDevice,
                                      e->stream)) != hipSuccess)
                goto fail;
            src += chunk;
            left -= chunk;
            pos = (pos + chunk) % cap;
        }
        e->submitted[c] += count;
        hipLaunchKernelGGL(eng_publish, dim3(1), dim3(1), 0, e->stream, e->hg[c].tail, int32_t(e->submitted[c]));
        if ((err = hipGetLastError()) != hipSuccess) goto fail;
    }
    return LDPC_OK;
fail:
    set_error(std::string("ldpc_engine_submit: ") + hipGetErrorString(err));
    (void)hipGetLastError();
    return LDPC_E_DEVICE;
}

extern "C" ldpc_status ldpc_engine_step(ldpc_engine *e, int32_t replays) {
    if (!e || replays < 0) { set_error("ldpc_engine_step: bad argument"); return LDPC_E_INVAL; }
    for (int32_t i = 0; i < replays; i++) {
        hipError_t err;
        if (e->direct) {
            enqueue_steps(e, e->K);
            err = hipGetLastError();
        } else {
            err = hipGraphLaunch(e->exec, e->stream);
        }
        if (err == hipSuccess) {
            // counters of this replay, for capacity checks that must not wait
            const int p = e->parity;
            e->parity ^= 1;
            err = hipMemcpyAsync(e->h_async[p], e->d_counters, size_t(e->ngraphs) * kCounterInts * 4, hipMemcpyDeviceToHost,
                                 e->stream);
            if (err == hipSuccess) err = hipEventRecord(e->ev_async[p], e->stream);
            e->async_pending[p] = err == hipSuccess;
        }
        if (err != hipSuccess) {
            set_error(std::string("ldpc_engine_step: ") + hipGetErrorString(err));
            (void)hipGetLastError();
            return LDPC_E_DEVICE;
        }
    }
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_engine_poll(ldpc_engine *e, int64_t *retired, int64_t *pending) {
    if (!e) { set_error("ldpc_engine_poll: NULL engine"); return LDPC_E_INVAL; }
    hipError_t err = hipMemcpyAsync(e->h_counters, e->d_counters, size_t(e->ngraphs) * kCounterInts * 4, hipMemcpyDeviceToHost,
                                    e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
    if (err != hipSuccess) {
        set_error(std::string("ldpc_engine_poll: ") + hipGetErrorString(err));
        (void)hipGetLastError();
        return LDPC_E_DEVICE;
    }
    // admissions of the last step are applied to head at the start of the next step
    absorb_counters(e, e->h_counters);
    for (int32_t c = 0; c < e->ngraphs; c++) {
        if (retired) retired[c] = e->retired_seen[size_t(c)];
        if (pending) pending[c] = e->submitted[size_t(c)] - e->retired_seen[size_t(c)];
    }
    return LDPC_OK;
}

namespace {

// Admit queued frames into empty slots now, outside the step sequence: the
// bookkeeping that ends a step (list the empty slots, load the queued frames'
// channel LLRs, install them), so that a run starting on empty pools does not
// spend its first step's iterations on them.  Call at a step boundary only.
hipError_t admit_now(ldpc_engine *e) {
    hipStream_t st = e->stream;
    hipLaunchKernelGGL(eng_open_lists, dim3(1), dim3(64), 0, st, e->d_graphs, e->ngraphs);
    hipLaunchKernelGGL(eng_advance, dim3(unsigned((e->total_slots + 255) / 256)), dim3(256), 0, st, e->d_graphs,
                       e->pre_slots, e->T, e->d_counters, int32_t(0));
    hipLaunchKernelGGL(eng_turnover, dim3(unsigned(kTurnoverBlocks)), dim3(256), 0, st, e->d_graphs, e->ngraphs,
                       e->d_counters);
    hipLaunchKernelGGL(eng_admit<false>, dim3(unsigned(e->ngraphs)), dim3(1024), 0, st, e->d_graphs);
    return hipGetLastError();
}

}  // namespace

extern "C" ldpc_status ldpc_engine_run(ldpc_engine *e, int32_t max_replays, int64_t *replays_out) {
    if (!e || max_replays < 0) { set_error("ldpc_engine_run: bad argument"); return LDPC_E_INVAL; }
    int64_t done = 0;
    for (;;) {
        ldpc_status st = ldpc_engine_poll(e, nullptr, nullptr);
        if (st != LDPC_OK) return st;
        if (done == 0) {
            // every submitted frame still queued (none in a slot): admit before the first step
            bool empty = true, queued = false;
            for (int32_t c = 0; c < e->ngraphs; c++) {
                empty &= e->head_seen[size_t(c)] == e->retired_seen[size_t(c)];
                queued |= e->submitted[size_t(c)] > e->head_seen[size_t(c)];
            }
            if (empty && queued) {
                const hipError_t err = admit_now(e);
                if (err != hipSuccess) {
                    set_error(std::string("ldpc_engine_run: ") + hipGetErrorString(err));
                    return LDPC_E_DEVICE;
                }
            }
        }
        bool finished = true;
        for (int32_t c = 0; c < e->ngraphs; c++)
            if (e->retired_seen[size_t(c)] < e->submitted[size_t(c)]) finished = false;
        if (finished || (max_replays && done >= max_replays)) break;
        // two replays in flight keep the device busy while the host reads the counters
        st = ldpc_engine_step(e, done == 0 ? 2 : 1);
        if (st != LDPC_OK) return st;
        done += done == 0 ? 2 : 1;
    }
    if (replays_out) *replays_out = done;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_engine_autotune(const ldpc_graph *const *graphs, int32_t ngraphs,
                                            const ldpc_frame *const *frames, const int32_t *frame_counts,
                                            int32_t max_iter, uint32_t flags, int32_t *slots_out,
                                            ldpc_engine_opts *opts_out, float *best_ms) {
    if (!graphs || !frames || !frame_counts || !slots_out || !opts_out || ngraphs < 1 || ngraphs > kMaxGraphs) {
        set_error("ldpc_engine_autotune: bad argument");
        return LDPC_E_INVAL;
    }
    std::vector<int32_t> caps(static_cast<size_t>(ngraphs));
    for (int32_t c = 0; c < ngraphs; c++) {
        if (frame_counts[c] < 0 || (frame_counts[c] > 0 && !frames[c])) {
            set_error("ldpc_engine_autotune: bad frame list");
            return LDPC_E_INVAL;
        }
        caps[size_t(c)] = std::max(1, frame_counts[c]);
    }
    const int lane_options[2] = {2, 4};
    const float scale_options[3] = {0.25f, 0.5f, 1.0f};
    // (steps per replay, iterations per step): at most 16 iterations per replay,
    // since the host looks at the counters once per replay
    const int step_options[6][2] = {{4, 1}, {8, 1}, {2, 2}, {4, 2}, {1, 4}, {2, 4}};
    float best = -1.f;
    for (int ls : lane_options) {
        for (float sc : scale_options) {
            for (const auto &gi : step_options) {
                std::vector<int32_t> slots(static_cast<size_t>(ngraphs));
                for (int32_t c = 0; c < ngraphs; c++)
                    slots[size_t(c)] = std::max(64 * ls, int32_t(std::ceil(sc * float(frame_counts[c]))));
                ldpc_engine_opts o{};
                o.lane_slots = ls;
                o.graph_steps = gi[0];
                o.iters_per_step = gi[1];
                ldpc_engine *e = nullptr;
                ldpc_status st = ldpc_engine_create(graphs, ngraphs, slots.data(), caps.data(), max_iter, flags, &o, &e);
                if (st != LDPC_OK) return st;
                float ms = 0.f;
                for (int rep = 0; rep < 2 && st == LDPC_OK; rep++) {
                    const auto t0 = std::chrono::steady_clock::now();
                    for (int32_t c = 0; c < ngraphs && st == LDPC_OK; c++)
                        if (frame_counts[c] > 0) st = ldpc_engine_submit(e, c, frames[c], frame_counts[c], nullptr);
                    if (st == LDPC_OK) st = ldpc_engine_run(e, 0, nullptr);
                    const auto t1 = std::chrono::steady_clock::now();
                    ms = std::chrono::duration<float, std::milli>(t1 - t0).count();
                }
                ldpc_engine_destroy(e);
                if (st != LDPC_OK) return st;
                if (best < 0.f || ms < best) {
                    best = ms;
                    for (int32_t c = 0; c < ngraphs; c++) slots_out[c] = slots[size_t(c)];
                    *opts_out = o;
                }
            }
        }
    }
    if (best_ms) *best_ms = best;
    return LDPC_OK;
}
