// Sum-product decoding on gfx950: kernels and the ldpc_decode driver.
//
// Data layout (all in the caller's workspace, frames padded to S slots):
//   Lch  [n][S]  f32   channel LLRs (transposed from the caller's [F][n])
//   Lpost[n][S]  f32   posterior LLRs of the latest iteration
//   R    [E][S]  f32/f16/bf16  check->bit messages, edges in check-sorted order
//   iters[S], fail[S]  i32   per-frame stop state
// One wavefront lane owns V consecutive frame slots, so every lane of a wave
// walks the same row or column of the Tanner graph: graph indices are
// wave-uniform (scalar loads) and every message access is a contiguous
// 64*V*sizeof(elem) span.
//
// One iteration (Algorithm 2's loop body) is two passes:
//   check pass  (Algorithm 1 second half): for each check, the bit->check
//               messages are formed as Q = clamp(Lpost - R_old) (Algorithm 1
//               first half, the extrinsic sum written as total minus own
//               message, which is exact up to rounding), the extrinsic check
//               rule produces R_new in place, and the syndrome bit of the
//               previous estimate (Algorithm 7) is folded in from the signs
//               of the same Lpost values;
//   bit pass    (Algorithms 4 and 6): Lpost = Lch + sum of R_new over the
//               bit's checks; the hard decision is the sign of Lpost.
//
// Check rule.  With u = 1 - tanh(|Q|/2) = 2w/(1+w), w = exp(-|Q|), the
// extrinsic product of tanh's is 1 - D where D is the u's combined with
// a (+) b = a + b(1 - a) (the complement of a product of complements), and
// the message magnitude is 2 atanh(1 - D) = ln((2 - D)/D).  Every extrinsic
// D is an exclusive prefix combined with an exclusive suffix, so no quantity
// is ever formed by removing a term; strong messages keep full relative
// precision (D small) and weak ones full absolute precision.
#include <hip/hip_runtime.h>

#include <cmath>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"

#include "device_common.h"

namespace {

using namespace ldpc_dev;

// ------------------------------------------------------------------ kernels

__global__ __launch_bounds__(256) void init_state_kernel(int32_t *__restrict__ iters, int32_t *__restrict__ fail,
                                                         int32_t F, int32_t S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) {
        iters[s] = s < F ? 0 : kPadSlot;
        fail[s] = 0;
    }
}

// llr_in [F][n] -> Lch [n][S] (zeros in padding slots, -0 stored as +0), 64x64
// tiles through LDS; with post16, also their 16-bit copy for the first check pass.
__global__ __launch_bounds__(256) void ingest_kernel(const float *__restrict__ llr, int32_t F, int32_t n,
                                                     float *__restrict__ Lch, int32_t S, _Float16 *__restrict__ post16) {
    __shared__ float tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int v0 = blockIdx.x * 64, s0 = blockIdx.y * 64;
    for (int i = ty; i < 64; i += 4) {
        const int f = s0 + i, v = v0 + tx;
        tile[i][tx] = (f < F && v < n) ? canon_llr(llr[size_t(f) * n + v]) : 0.f;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int v = v0 + i;
        if (v < n) {
            Lch[size_t(v) * S + s0 + tx] = tile[tx][i];
            if (post16) post16[size_t(v) * S + s0 + tx] = post16_enc(tile[tx][i]);
        }
    }
}

// Element type of the array a check pass takes L from: the channel LLRs in
// iteration 1, the posterior afterwards, both in the check pass's storage
// (Post): with 16-bit messages the ingest stores a 16-bit copy of the channel
// LLRs there, otherwise iteration 1 reads the fp32 channel array.
template <int M, int MODE>
using CheckL = typename Post<M>::T;

// Plain-path slot state: kFirst is iteration 1 (L = Lch, no previous
// messages); kIter reads Lpost and R_old.  When syn_iter > 0 the syndrome of
// the previous estimate is checked and failing frames get fail[s] = syn_iter.
template <int V>
__device__ __forceinline__ void plain_syndrome(const int32_t (&st)[V], const int (&syn)[V], int32_t *fail, int s0,
                                               int32_t syn_iter) {
    if (syn_iter > 0) {
#pragma unroll
        for (int k = 0; k < V; k++)
            if (st[k] == 0 && syn[k] && fail[s0 + k] != syn_iter) fail[s0 + k] = syn_iter;
    }
}

// Rows of degree <= DMAX in registers: one wavefront per (row, slot group).
// RULE: the check rule (CheckRule); rp its parameter.  At least four
// wavefronts per SIMD (at most 128 registers): a row keeps all of its loads in
// flight, so the number of resident wavefronts bounds the memory parallelism.
// QC: a quasi-cyclic graph; each edge's bit comes from the row's base entry
// (QcCols) instead of col_idx, with the class's row ids in `rows`.
template <int M, int V, int DMAX, int MODE, int RULE, bool QC>
__device__ __forceinline__ void check_rows_body(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx,
    int32_t nrows, const CheckL<M, MODE> *__restrict__ L, typename Codec<M>::T *__restrict__ R,
    const int32_t *__restrict__ iters, int32_t *__restrict__ fail, int32_t S, int32_t groups, int32_t syn_iter,
    float rp, const int32_t *__restrict__ rows, const int32_t *__restrict__ qc_row_ptr,
    const int32_t *__restrict__ qc_ent, int32_t Z) {
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int g = wave % groups;
    const int rk = wave / groups;
    if (rk >= nrows) return;
    const int s0 = (g * 64 + lane) * V;

    int32_t st[V];
    load_i32<V>(iters + s0, st);
    bool lane_active = false;
#pragma unroll
    for (int k = 0; k < V; k++) lane_active |= (st[k] == 0);
    if (__ballot(lane_active) == 0) return;
    // Lanes whose frames have all stopped issue no loads or stores.
    if (!lane_active) return;

    const int e0 = wave_uniform(rd[2 * rk]);
    const int d = wave_uniform(rd[2 * rk + 1]);
    SlotSrc<V> src;
#pragma unroll
    for (int k = 0; k < V; k++) src.alt[k] = false;
    src.any = false;
    int syn[V];
#pragma unroll
    for (int k = 0; k < V; k++) syn[k] = 0;
    constexpr int IN = MODE == kIter ? kInSteady : kInFirst;
    if constexpr (QC) {
        const int r = wave_uniform(cload(rows + rk));
        const int i = r / Z;
        const QcCols q{qc_ent + 2 * wave_uniform(cload(qc_row_ptr + i)), e0, r - i * Z, Z};
        row_rule<M, V, DMAX, true, IN, RULE>(q, e0, d, L, R, S, s0, src, syn, rp);
    } else {
        row_rule<M, V, DMAX, true, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, syn, rp);
    }
    if (MODE == kIter) plain_syndrome<V>(st, syn, fail, s0, syn_iter);
}

template <int M, int V, int DMAX, int MODE, int RULE, bool QC>
__global__ __launch_bounds__(256, 4) void check_rows_kernel(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx,
    int32_t nrows, const CheckL<M, MODE> *__restrict__ L, typename Codec<M>::T *__restrict__ R,
    const int32_t *__restrict__ iters, int32_t *__restrict__ fail, int32_t S, int32_t groups, int32_t syn_iter,
    float rp, const int32_t *__restrict__ rows, const int32_t *__restrict__ qc_row_ptr,
    const int32_t *__restrict__ qc_ent, int32_t Z) {
    check_rows_body<M, V, DMAX, MODE, RULE, QC>(rd, col_idx, nrows, L, R, iters, fail, S, groups, syn_iter, rp, rows,
                                                qc_row_ptr, qc_ent, Z);
}

// Rows of 9..128 edges: WPR wavefronts per (row, slot group), 8-edge chunks,
// chunk aggregates exchanged through LDS.  A wavefront with more than one
// chunk recomputes its chunks' inputs in the second phase.
// Chunk aggregates of one workgroup of check_chunk_body: 4 / WPR rows.
template <int WPR>
constexpr int chunk_share_entries() { return (4 / WPR) * (WPR == 2 ? 2 : 16); }

template <int M, int V, int WPR, int MODE, int RULE>
__device__ __forceinline__ void check_chunk_body(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx,
    int32_t nrows, const CheckL<M, MODE> *__restrict__ L, typename Codec<M>::T *__restrict__ R,
    const int32_t *__restrict__ iters, int32_t *__restrict__ fail, int32_t S, int32_t groups, int32_t syn_iter,
    float rp, ChunkShare<V, chunk_share_entries<WPR>()> &sh) {
    constexpr int C = kRowChunk;
    constexpr int RPB = 4 / WPR;
    constexpr int MAXCH = WPR == 2 ? 2 : 16;
    constexpr int kChunkIn = MODE == kIter ? kInSteady : kInFirst;
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int lr = wave / WPR;
    const int wr = wave % WPR;
    const int item = blockIdx.x * RPB + lr;
    const int rk = item / groups;
    const int g = item % groups;
    const int s0 = (g * 64 + lane) * V;

    int32_t st[V];
    bool lane_active = false;
    if (rk < nrows) {
        load_i32<V>(iters + s0, st);
#pragma unroll
        for (int k = 0; k < V; k++) lane_active |= (st[k] == 0);
    }
    // same slots for every wavefront of a row: uniform over the row's wavefronts
    const bool work = rk < nrows && __ballot(lane_active) != 0;
    int e0 = 0, d = 0, nch = 0;
    if (work) {
        e0 = wave_uniform(rd[2 * rk]);
        d = wave_uniform(rd[2 * rk + 1]);
        nch = (d + C - 1) / C;
    }
    SlotSrc<V> src;
#pragma unroll
    for (int k = 0; k < V; k++) src.alt[k] = false;
    src.any = false;
    const bool mine = work && lane_active;
    float u[C][V], suf[C][V], agg[V];
    uint32_t par[V];
    int syn[V];
    for (int ch = wr; ch < nch; ch += WPR) {
        if (mine) {
            chunk_load<M, V, C, kChunkIn, RULE>(col_idx, e0 + ch * C, min(C, d - ch * C), L, R, S, s0, src, u,
                                                suf, agg, par, syn);
        } else {
#pragma unroll
            for (int k = 0; k < V; k++) { agg[k] = CheckRule<RULE>::identity(); par[k] = 0u; syn[k] = 0; }
        }
#pragma unroll
        for (int k = 0; k < V; k++) sh.agg[lr * MAXCH + ch][lane][k] = agg[k];
        sh.bits[lr * MAXCH + ch][lane] = pack_bits<V>(par, syn);
    }
    __syncthreads();
    if (!mine) return;
    for (int ch = wr; ch < nch; ch += WPR) {
        if (nch > WPR)
            chunk_load<M, V, C, kChunkIn, RULE>(col_idx, e0 + ch * C, min(C, d - ch * C), L, R, S, s0, src, u,
                                                suf, agg, par, syn);
        float pre[V], post[V];
        uint32_t parity[V];
        int syn_row[V];
        chunk_context<V, RPB * MAXCH, RULE>(sh, lr * MAXCH, nch, ch, lane, pre, post, parity, syn_row);
        chunk_store<M, V, C, RULE>(e0 + ch * C, min(C, d - ch * C), u, suf, pre, post, parity, R, S, s0, rp);
        if (MODE == kIter && ch == 0) plain_syndrome<V>(st, syn_row, fail, s0, syn_iter);
    }
}

template <int M, int V, int WPR, int MODE, int RULE>
__global__ __launch_bounds__(256) void check_chunk_kernel(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx,
    int32_t nrows, const CheckL<M, MODE> *__restrict__ L, typename Codec<M>::T *__restrict__ R,
    const int32_t *__restrict__ iters, int32_t *__restrict__ fail, int32_t S, int32_t groups, int32_t syn_iter,
    float rp) {
    __shared__ ChunkShare<V, chunk_share_entries<WPR>()> sh;
    check_chunk_body<M, V, WPR, MODE, RULE>(rd, col_idx, nrows, L, R, iters, fail, S, groups, syn_iter, rp, sh);
}

// Check pass for rows of 129..512 edges: one workgroup of sixteen wavefronts
// per (row, 64-slot group), one 32-edge chunk per wavefront, chunk aggregates
// exchanged through LDS (wide_row); every input is read once.
template <int M, int MODE, int RULE>
__device__ __forceinline__ void check_wide_body(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx, int32_t nrows,
    const CheckL<M, MODE> *__restrict__ L, typename Codec<M>::T *__restrict__ R, const int32_t *__restrict__ iters,
    int32_t *__restrict__ fail, int32_t S, int32_t groups, int32_t syn_iter, float rp, ChunkShare<1, kWideWaves> &sh) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_uniform(threadIdx.x >> 6);
    const int g = blockIdx.x % groups;
    const int rk = blockIdx.x / groups;
    if (rk >= nrows) return;
    const int s = g * 64 + lane;
    const bool active = iters[s] == 0;
    if (__ballot(active) == 0) return;   // same slots in every wave: uniform over the block
    const int e0 = wave_uniform(rd[2 * rk]);
    const int d = wave_uniform(rd[2 * rk + 1]);
    SlotSrc<1> src;
    src.alt[0] = false;
    src.any = false;
    constexpr int IN = MODE == kIter ? kInSteady : kInFirst;
    const bool syn = wide_row<M, kWideChunk, IN, RULE>(col_idx, e0, d, L, R, S, s, src, active, sh, wv, lane, rp);
    if (MODE == kIter && wv == 0 && syn_iter > 0 && active && syn && fail[s] != syn_iter) fail[s] = syn_iter;
}

template <int M, int MODE, int RULE>
__global__ __launch_bounds__(1024) void check_wide_kernel(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx, int32_t nrows,
    const CheckL<M, MODE> *__restrict__ L, typename Codec<M>::T *__restrict__ R, const int32_t *__restrict__ iters,
    int32_t *__restrict__ fail, int32_t S, int32_t groups, int32_t syn_iter, float rp) {
    __shared__ ChunkShare<1, kWideWaves> sh;
    check_wide_body<M, MODE, RULE>(rd, col_idx, nrows, L, R, iters, fail, S, groups, syn_iter, rp, sh);
}

// Check pass for rows longer than 512 edges: one workgroup of four wavefronts
// per (row, 64-slot group).  The row is cut into 32-edge chunks; each chunk's
// combined u (its D aggregate), sign parity and syndrome parity go to scratch,
// one wavefront scans the chunk aggregates into per-chunk exclusive values,
// and each chunk is then finished with a local prefix/suffix pass.
template <int M, int MODE, int RULE>
__device__ __forceinline__ void check_hub_body(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx,
    int32_t nrows, const int32_t *__restrict__ chunk_base, const CheckL<M, MODE> *__restrict__ L,
    typename Codec<M>::T *__restrict__ R, const int32_t *__restrict__ iters, int32_t *__restrict__ fail,
    int32_t S, int32_t groups, int32_t syn_iter, float *__restrict__ aggD, float *__restrict__ aggPre,
    int32_t *__restrict__ aggBits, float rp, int32_t (&total_bits)[64]) {
    using Rule = CheckRule<RULE>;
    constexpr int C = ldpc::kHubChunk;
    const int lane = threadIdx.x & 63;
    const int wv = wave_uniform(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int g = blockIdx.x % groups;
    const int rk = blockIdx.x / groups;
    if (rk >= nrows) return;
    const int s = g * 64 + lane;
    const bool active = iters[s] == 0;
    if (__ballot(active) == 0) return;   // same slots in every wave: uniform over the block

    const int e0 = wave_uniform(rd[2 * rk]);
    const int d = wave_uniform(rd[2 * rk + 1]);
    const int nch = (d + C - 1) / C;
    const int cb = wave_uniform(chunk_base[rk]);

    // Phase A: per-chunk aggregates.
    for (int c = wv; c < nch; c += nw) {
        const int j0 = e0 + c * C;
        const int dc = min(C, d - c * C);
        float agg = Rule::identity();
        int32_t bits = 0;
#pragma unroll
        for (int jj = 0; jj < C; jj++) {
            if (jj < dc) {
                const int v = wave_uniform(col_idx[j0 + jj]);
                const float lv = Codec<CodecOf<CheckL<M, MODE>>::kMsg>::dec(L[size_t(v) * S + s]);
                const float r = (MODE == kIter) ? Codec<M>::dec(R[size_t(j0 + jj) * S + s]) : 0.f;
                const float q = rule_q<M, RULE>(lv, r);
                bits ^= int32_t(q < 0.f) | (int32_t(lv < 0.f) << 1);
                agg = Rule::combine(agg, rule_in<M, RULE>(fabsf(q)));
            }
        }
        aggD[size_t(cb + c) * S + s] = agg;
        aggBits[size_t(cb + c) * S + s] = bits;
    }
    __syncthreads();

    // Phase B: exclusive prefix and suffix over chunks, serial in wave 0.
    if (wv == 0) {
        float pre = Rule::identity();
        int32_t tot = 0;
        for (int c = 0; c < nch; c++) {
            aggPre[size_t(cb + c) * S + s] = pre;
            pre = Rule::combine(pre, aggD[size_t(cb + c) * S + s]);
            tot ^= aggBits[size_t(cb + c) * S + s];
        }
        float suf = Rule::identity();
        for (int c = nch - 1; c >= 0; c--) {
            const float dcur = aggD[size_t(cb + c) * S + s];
            aggD[size_t(cb + c) * S + s] = Rule::combine(aggPre[size_t(cb + c) * S + s], suf);
            suf = Rule::combine(suf, dcur);
        }
        total_bits[lane] = tot;
        if (MODE == kIter && syn_iter > 0 && active && (tot & 2) && fail[s] != syn_iter) fail[s] = syn_iter;
    }
    __syncthreads();

    // Phase C: finish each chunk with its exclusive outside value.
    const uint32_t parity = uint32_t(total_bits[lane]) & 1u;
    for (int c = wv; c < nch; c += nw) {
        const int j0 = e0 + c * C;
        const int dc = min(C, d - c * C);
        float u[C], sf[C];
        uint32_t neg = 0u;
#pragma unroll
        for (int jj = 0; jj < C; jj++) {
            if (jj < dc) {
                const int v = wave_uniform(col_idx[j0 + jj]);
                const float lv = Codec<CodecOf<CheckL<M, MODE>>::kMsg>::dec(L[size_t(v) * S + s]);
                const float r = (MODE == kIter) ? Codec<M>::dec(R[size_t(j0 + jj) * S + s]) : 0.f;
                const float q = rule_q<M, RULE>(lv, r);
                neg |= uint32_t(q < 0.f) << jj;
                u[jj] = rule_in<M, RULE>(fabsf(q));
            }
        }
        float run = Rule::identity();
#pragma unroll
        for (int jj = C - 1; jj >= 0; jj--) {
            if (jj < dc) {
                sf[jj] = run;
                run = Rule::combine(u[jj], run);
            }
        }
        run = aggD[size_t(cb + c) * S + s];
#pragma unroll
        for (int jj = 0; jj < C; jj++) {
            if (jj < dc) {
                const float mag = rule_mag<M, RULE>(Rule::combine(run, sf[jj]), rp);
                const uint32_t sgn = parity ^ ((neg >> jj) & 1u);
                R[size_t(j0 + jj) * S + s] = Codec<M>::enc(sgn ? -mag : mag);
                run = Rule::combine(run, u[jj]);
            }
        }
    }
}

template <int M, int MODE, int RULE>
__global__ __launch_bounds__(256) void check_hub_kernel(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx,
    int32_t nrows, const int32_t *__restrict__ chunk_base, const CheckL<M, MODE> *__restrict__ L,
    typename Codec<M>::T *__restrict__ R, const int32_t *__restrict__ iters, int32_t *__restrict__ fail,
    int32_t S, int32_t groups, int32_t syn_iter, float *__restrict__ aggD, float *__restrict__ aggPre,
    int32_t *__restrict__ aggBits, float rp) {
    __shared__ int32_t total_bits[64];
    check_hub_body<M, MODE, RULE>(rd, col_idx, nrows, chunk_base, L, R, iters, fail, S, groups, syn_iter, aggD, aggPre,
                                  aggBits, rp, total_bits);
}

// Bit pass: Lpost = Lch + sum of R over the bit's checks (Algorithm 4); one
// wavefront per (bit, slot group).  The posterior goes to the check pass's
// storage `post` (Post<M>) and, when Lpost is not NULL, also to the fp32 array
// Lpost (16-bit message formats only; otherwise `post` is the fp32 array).  A
// frame whose previous estimate passed the syndrome (no fail mark for
// iteration t-1) is finished: its posterior is left as is and the wavefront
// of bit 0 records iters = t-1.
template <int M, int V>
__device__ __forceinline__ void bit_body(const int32_t *__restrict__ col_ptr, const int32_t *__restrict__ csc_to_csr,
                                         int32_t n, const float *__restrict__ Lch,
                                         const typename Codec<M>::T *__restrict__ R,
                                         typename Post<M>::T *__restrict__ post, float *__restrict__ Lpost,
                                         int32_t *__restrict__ iters, const int32_t *__restrict__ fail, int32_t S,
                                         int32_t groups, int32_t t, int32_t early_stop, float bscale) {
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int g = wave % groups;
    const int v = wave / groups;
    if (v >= n) return;
    const int s0 = (g * 64 + lane) * V;

    int32_t st[V];
    load_i32<V>(iters + s0, st);
    bool act[V];
    bool any_active = false;
#pragma unroll
    for (int k = 0; k < V; k++) {
        bool go = st[k] == 0;
        if (go && early_stop && t > 1) {
            const bool failed_prev = fail[s0 + k] == t - 1;
            if (!failed_prev) {
                go = false;
                if (v == 0) iters[s0 + k] = t - 1;
            }
        }
        act[k] = go;
        any_active |= go;
    }
    if (__ballot(any_active) == 0) return;
    if (!any_active) return;   // lanes with no running frame issue no loads or stores

    float sum[V];
    const int a = wave_uniform(col_ptr[v]);
    const int b = wave_uniform(col_ptr[v + 1]);
    bit_posterior<M, V, true>(csc_to_csr, a, b, R, S, s0, Lch + size_t(v) * S, bscale, sum);
    bool all = true;
#pragma unroll
    for (int k = 0; k < V; k++) all &= act[k];
    if (all) {
        store_post<V>(post + size_t(v) * S + s0, sum);
        if (Lpost) store_vec<kF32, V>(Lpost + size_t(v) * S + s0, sum);
    } else {
#pragma unroll
        for (int k = 0; k < V; k++) {
            if (act[k]) {
                store_post1(post + size_t(v) * S + s0 + k, sum[k]);
                if (Lpost) Lpost[size_t(v) * S + s0 + k] = sum[k];
            }
        }
    }
}

template <int M, int V>
__global__ __launch_bounds__(256) void bit_kernel(const int32_t *__restrict__ col_ptr,
                                                  const int32_t *__restrict__ csc_to_csr, int32_t n,
                                                  const float *__restrict__ Lch, const typename Codec<M>::T *__restrict__ R,
                                                  typename Post<M>::T *__restrict__ post,
                                                  float *__restrict__ Lpost, int32_t *__restrict__ iters,
                                                  const int32_t *__restrict__ fail, int32_t S, int32_t groups,
                                                  int32_t t, int32_t early_stop, float bscale) {
    bit_body<M, V>(col_ptr, csc_to_csr, n, Lch, R, post, Lpost, iters, fail, S, groups, t, early_stop, bscale);
}

// Syndrome of the current estimate for every non-empty check (any degree):
// frames still running whose estimate fails get fail[s] = syn_iter.
template <int V, typename PT>
__global__ __launch_bounds__(256) void syndrome_kernel(const int32_t *__restrict__ rd,
                                                       const int32_t *__restrict__ col_idx, int32_t nrows,
                                                       const PT *__restrict__ Lpost,
                                                       const int32_t *__restrict__ iters, int32_t *__restrict__ fail,
                                                       int32_t S, int32_t groups, int32_t syn_iter) {
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int g = wave % groups;
    const int rk = wave / groups;
    if (rk >= nrows) return;
    const int s0 = (g * 64 + lane) * V;
    int32_t st[V];
    load_i32<V>(iters + s0, st);
    bool any_active = false;
#pragma unroll
    for (int k = 0; k < V; k++) any_active |= (st[k] == 0);
    if (__ballot(any_active) == 0) return;
    if (!any_active) return;
    const int a = wave_uniform(rd[2 * rk]);
    const int b = a + wave_uniform(rd[2 * rk + 1]);
    int syn[V];
#pragma unroll
    for (int k = 0; k < V; k++) syn[k] = 0;
    for (int e = a; e < b; e++) {
        const int v = wave_uniform(col_idx[e]);
        float lv[V];
        load_vec<CodecOf<PT>::kMsg, V>(Lpost + size_t(v) * S + s0, lv);
#pragma unroll
        for (int k = 0; k < V; k++) syn[k] ^= (lv[k] < 0.f);
    }
#pragma unroll
    for (int k = 0; k < V; k++)
        if (st[k] == 0 && syn[k] && fail[s0 + k] != syn_iter) fail[s0 + k] = syn_iter;
}

// Per-frame results: a frame still running after max_iter iterations reports
// iters = max_iter and ok = (its final syndrome passed).
__global__ __launch_bounds__(256) void finalize_kernel(const int32_t *__restrict__ iters,
                                                       const int32_t *__restrict__ fail, int32_t F, int32_t max_iter,
                                                       int32_t *__restrict__ iters_out, uint8_t *__restrict__ ok_out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= F) return;
    const int32_t st = iters[s];
    if (st == 0) {
        iters_out[s] = max_iter;
        ok_out[s] = fail[s] != max_iter;
    } else {
        iters_out[s] = st;
        ok_out[s] = 1;
    }
}

// Posterior [n][S] -> bits [F][n] (1 iff Lpost < 0, Algorithm 6) and optional
// llr_out [F][n].  With llr_out the fp32 posterior Lpost is read (its signs
// are those of the check-pass storage); without it, the storage `post`.
template <typename PT>
__global__ __launch_bounds__(256) void egress_kernel(const PT *__restrict__ post, const float *__restrict__ Lpost,
                                                     int32_t S, int32_t F, int32_t n, uint8_t *__restrict__ bits,
                                                     float *__restrict__ llr_out) {
    __shared__ float tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int v0 = blockIdx.x * 64, s0 = blockIdx.y * 64;
    for (int i = ty; i < 64; i += 4) {
        const int v = v0 + i;
        tile[i][tx] = v >= n ? 0.f
                      : llr_out ? Lpost[size_t(v) * S + s0 + tx]
                                : Codec<CodecOf<PT>::kMsg>::dec(post[size_t(v) * S + s0 + tx]);
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int f = s0 + i, v = v0 + tx;
        if (f < F && v < n) {
            const float x = tile[tx][i];
            bits[size_t(f) * n + v] = x < 0.f;
            if (llr_out) llr_out[size_t(f) * n + v] = x;
        }
    }
}

// ------------------------------------------------------------------ driver

// ------------------------------------------------------- Monte-Carlo runs

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds, each two
// 32x32 -> 64-bit products of counter words with fixed multipliers, mixed with
// the other words and the round key; the key advances by two Weyl constants.
__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
        const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
        const uint32_t n0 = uint32_t(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = uint32_t(p0 >> 32) ^ c[3] ^ k1;
        c[1] = uint32_t(p1);
        c[3] = uint32_t(p0);
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform in (0, 1) from the top 23 bits (exact in FP32), then Box-Muller.
__device__ __forceinline__ float unit_open(uint32_t x) { return (float(x >> 9) + 0.5f) * 0x1p-23f; }

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float &z0, float &z1) {
    const float r = sqrtf(-2.f * logf(unit_open(a)));
    float sn, cs;
    sincospif(2.f * unit_open(b), &sn, &cs);
    z0 = r * cs;
    z1 = r * sn;
}

// Channel LLRs of the all-zero codeword over BPSK/AWGN, written straight into
// the slot-major channel array: thread = frame slot, 4 bits per counter value
// (L = k0 + k1 z with k0 = 2/sigma^2, k1 = 2/sigma).  Padding slots get 0.
__global__ __launch_bounds__(256) void channel_kernel(float *__restrict__ Lch, int32_t S, int32_t F, int32_t n,
                                                      uint32_t key0, uint32_t key1, uint64_t first_frame, float k0,
                                                      float k1, float *__restrict__ llr_out,
                                                      _Float16 *__restrict__ post16) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const int quads = (n + 3) / 4;
    const uint64_t f = first_frame + uint64_t(s);
    for (int q = blockIdx.y; q < quads; q += gridDim.y) {
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        if (s < F) {
            uint32_t c[4] = {uint32_t(q), uint32_t(f), uint32_t(f >> 32), 0u};
            philox4x32_10(c, key0, key1);
            box_muller(c[0], c[1], z[0], z[1]);
            box_muller(c[2], c[3], z[2], z[3]);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int v = 4 * q + j;
            if (v < n) {
                const float L = s < F ? canon_llr(fmaf(k1, z[j], k0)) : 0.f;
                Lch[size_t(v) * S + s] = L;
                if (post16) post16[size_t(v) * S + s] = post16_enc(L);
                if (llr_out && s < F) llr_out[size_t(s) * n + v] = L;
            }
        }
    }
}

__global__ __launch_bounds__(256) void zero_kernel(int32_t *__restrict__ x, int32_t count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) x[i] = 0;
}

// Bit errors of each frame's estimate against the all-zero codeword: bits whose
// hard decision is 1 (Lpost < 0, Algorithm 6).  Thread = frame, 64 bits per
// workgroup row; counts are added into err[frame].
template <typename PT>
__global__ __launch_bounds__(256) void count_errors_kernel(const PT *__restrict__ Lpost, int32_t S, int32_t F,
                                                           int32_t n, int32_t *__restrict__ err) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= F) return;
    for (int v0 = blockIdx.y * 64; v0 < n; v0 += gridDim.y * 64) {
        const int v1 = min(n, v0 + 64);
        int cnt = 0;
        for (int v = v0; v < v1; v++) cnt += Codec<CodecOf<PT>::kMsg>::dec(Lpost[size_t(v) * S + s]) < 0.f;
        if (cnt) atomicAdd(err + s, cnt);
    }
}

// Per-frame results into the run's counts: one atomic per counter per workgroup.
__global__ __launch_bounds__(256) void tally_kernel(const int32_t *__restrict__ err,
                                                    const int32_t *__restrict__ iters,
                                                    const uint8_t *__restrict__ ok, int32_t F,
                                                    ldpc_sim_counts *__restrict__ out) {
    __shared__ unsigned long long part[5][4];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v[5] = {0ull, 0ull, 0ull, 0ull, 0ull};
    if (s < F) {
        const int e = err[s];
        v[0] = 1ull;
        v[1] = e > 0;
        v[2] = unsigned(e);
        v[3] = e > 0 && ok[s];
        v[4] = unsigned(iters[s]);
    }
#pragma unroll
    for (int k = 0; k < 5; k++) {
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off);
        if ((threadIdx.x & 63) == 0) part[k][threadIdx.x >> 6] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int k = threadIdx.x;
        const unsigned long long sum = part[k][0] + part[k][1] + part[k][2] + part[k][3];
        uint64_t *dst = k == 0 ? &out->frames : k == 1 ? &out->frame_errors : k == 2 ? &out->bit_errors
                      : k == 3 ? &out->undetected : &out->iterations;
        static_assert(sizeof(uint64_t) == sizeof(unsigned long long), "64-bit counters");
        if (sum) atomicAdd(reinterpret_cast<unsigned long long *>(dst), sum);
    }
}

// ------------------------------------------------------- tail compaction
//
// Once few frames of a call are still running, their state is copied into a
// smaller slot range (slot k of the copy holds slot map[k] of the state it
// came from) and the remaining iterations run there.  Level 0 is the full
// state (S slots, V per lane); level l = 1, 2 is a copy of S_l <= S >> l slots
// (a multiple of 64) at V_l = max(1, V >> l) slots per lane, so that no
// level's grid is larger than the full state's.  The device takes every
// decision: every few iterations one workgroup counts the running frames and,
// once they fit a smaller level, lists them and switches the level word; a
// gather kernel then moves them (it exits at once when no move was decided);
// every pass kernel after the first count reads the level word and works on
// that level's state.  Only the running frames move and the per-frame
// arithmetic is unchanged, so results are identical; the host never waits.
// A frame runs while iters[s] == 0.

constexpr int kLevels = 3;

// The state of one level as the kernels address it.
struct LevelView {
    float *lch;
    void *post;       // posterior in the check pass's storage (Post<M>)
    float *lpost;     // fp32 posterior output (16-bit formats with llr_out), else NULL
    void *r;
    int32_t *iters, *fail;
    int32_t *map;     // slot k of this level holds slot map[k] of the level it came from
    int32_t S;        // slots (0: the level does not exist)
    int32_t V;        // slots per lane of the launch's check class (or of the bit pass)
};

// Every level of a call, and the device word that names the current one.
struct Levels {
    LevelView lv[kLevels];
    const int32_t *level;
};

// Control words of a call, in its workspace.
struct LevelCtl {
    int32_t level;            // the level the running frames are in
    int32_t from, to;         // the move the last count decided (to < 0: none)
    int32_t running;          // frames running at the last count
    int32_t src[kLevels];     // the level each level's frames came from (-1: not entered)
    int32_t count[kLevels];   // frames moved into each level
};

__device__ __forceinline__ const LevelView &level_at(const Levels &a, int l) {
    return l == 0 ? a.lv[0] : l == 1 ? a.lv[1] : a.lv[2];
}

// The level the frames are in (the same word for the whole grid).
__device__ __forceinline__ const LevelView &current_level(const Levels &a) {
    return level_at(a, wave_uniform(cload(a.level)));
}

// Pass kernels on the current level.  The grid is the full state's for the
// launch's class; at a smaller level the wavefronts beyond its slot groups
// exit at once.
template <int M, int V0, int DMAX, int RULE, bool QC>
__global__ __launch_bounds__(256, 4) void check_rows_level_kernel(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx, int32_t nrows, Levels a, int32_t syn_iter,
    float rp, const int32_t *__restrict__ rows, const int32_t *__restrict__ qc_row_ptr,
    const int32_t *__restrict__ qc_ent, int32_t Z) {
    const LevelView &x = current_level(a);
    const auto *L = static_cast<const CheckL<M, kIter> *>(x.post);
    auto *R = static_cast<typename Codec<M>::T *>(x.r);
    if constexpr (V0 >= 4) {
        if (x.V == 4) {
            check_rows_body<M, 4, DMAX, kIter, RULE, QC>(rd, col_idx, nrows, L, R, x.iters, x.fail, x.S, x.S / 256,
                                                         syn_iter, rp, rows, qc_row_ptr, qc_ent, Z);
            return;
        }
    }
    if constexpr (V0 >= 2) {
        if (x.V == 2) {
            check_rows_body<M, 2, DMAX, kIter, RULE, QC>(rd, col_idx, nrows, L, R, x.iters, x.fail, x.S, x.S / 128,
                                                         syn_iter, rp, rows, qc_row_ptr, qc_ent, Z);
            return;
        }
    }
    check_rows_body<M, 1, DMAX, kIter, RULE, QC>(rd, col_idx, nrows, L, R, x.iters, x.fail, x.S, x.S / 64, syn_iter,
                                                 rp, rows, qc_row_ptr, qc_ent, Z);
}

template <int M, int V0, int WPR, int RULE>
__global__ __launch_bounds__(256) void check_chunk_level_kernel(const int32_t *__restrict__ rd,
                                                                const int32_t *__restrict__ col_idx, int32_t nrows,
                                                                Levels a, int32_t syn_iter, float rp) {
    constexpr int NE = chunk_share_entries<WPR>();
    __shared__ ChunkShare<V0, NE> sh;   // the largest of the levels' shares
    const LevelView &x = current_level(a);
    const auto *L = static_cast<const CheckL<M, kIter> *>(x.post);
    auto *R = static_cast<typename Codec<M>::T *>(x.r);
    if constexpr (V0 >= 4) {
        if (x.V == 4) {
            check_chunk_body<M, 4, WPR, kIter, RULE>(rd, col_idx, nrows, L, R, x.iters, x.fail, x.S, x.S / 256,
                                                     syn_iter, rp, reinterpret_cast<ChunkShare<4, NE> &>(sh));
            return;
        }
    }
    if constexpr (V0 >= 2) {
        if (x.V == 2) {
            check_chunk_body<M, 2, WPR, kIter, RULE>(rd, col_idx, nrows, L, R, x.iters, x.fail, x.S, x.S / 128,
                                                     syn_iter, rp, reinterpret_cast<ChunkShare<2, NE> &>(sh));
            return;
        }
    }
    check_chunk_body<M, 1, WPR, kIter, RULE>(rd, col_idx, nrows, L, R, x.iters, x.fail, x.S, x.S / 64, syn_iter, rp,
                                             reinterpret_cast<ChunkShare<1, NE> &>(sh));
}

template <int M, int RULE>
__global__ __launch_bounds__(1024) void check_wide_level_kernel(const int32_t *__restrict__ rd,
                                                                const int32_t *__restrict__ col_idx, int32_t nrows,
                                                                Levels a, int32_t syn_iter, float rp) {
    __shared__ ChunkShare<1, kWideWaves> sh;
    const LevelView &x = current_level(a);
    check_wide_body<M, kIter, RULE>(rd, col_idx, nrows, static_cast<const CheckL<M, kIter> *>(x.post),
                                    static_cast<typename Codec<M>::T *>(x.r), x.iters, x.fail, x.S, x.S / 64,
                                    syn_iter, rp, sh);
}

template <int M, int RULE>
__global__ __launch_bounds__(256) void check_hub_level_kernel(
    const int32_t *__restrict__ rd, const int32_t *__restrict__ col_idx, int32_t nrows,
    const int32_t *__restrict__ chunk_base, Levels a, int32_t syn_iter, float *__restrict__ aggD,
    float *__restrict__ aggPre, int32_t *__restrict__ aggBits, float rp) {
    __shared__ int32_t total_bits[64];
    const LevelView &x = current_level(a);
    check_hub_body<M, kIter, RULE>(rd, col_idx, nrows, chunk_base, static_cast<const CheckL<M, kIter> *>(x.post),
                                   static_cast<typename Codec<M>::T *>(x.r), x.iters, x.fail, x.S, x.S / 64,
                                   syn_iter, aggD, aggPre, aggBits, rp, total_bits);
}

template <int M, int V0>
__global__ __launch_bounds__(256) void bit_level_kernel(const int32_t *__restrict__ col_ptr,
                                                        const int32_t *__restrict__ csc_to_csr, int32_t n, Levels a,
                                                        int32_t t, int32_t early_stop, float bscale) {
    const LevelView &x = current_level(a);
    const auto *R = static_cast<const typename Codec<M>::T *>(x.r);
    auto *post = static_cast<typename Post<M>::T *>(x.post);
    if constexpr (V0 >= 4) {
        if (x.V == 4) {
            bit_body<M, 4>(col_ptr, csc_to_csr, n, x.lch, R, post, x.lpost, x.iters, x.fail, x.S, x.S / 256, t,
                           early_stop, bscale);
            return;
        }
    }
    if constexpr (V0 >= 2) {
        if (x.V == 2) {
            bit_body<M, 2>(col_ptr, csc_to_csr, n, x.lch, R, post, x.lpost, x.iters, x.fail, x.S, x.S / 128, t,
                           early_stop, bscale);
            return;
        }
    }
    bit_body<M, 1>(col_ptr, csc_to_csr, n, x.lch, R, post, x.lpost, x.iters, x.fail, x.S, x.S / 64, t, early_stop,
                   bscale);
}

// One workgroup: counts the frames running at the current level and, when
// they fit a smaller level (the smallest that holds them), lists them in slot
// order into that level's map and switches the level word.
__global__ __launch_bounds__(1024) void level_decide_kernel(LevelCtl *__restrict__ ctl, Levels a) {
    __shared__ int32_t part[16];
    __shared__ int32_t base;
    const int l = ctl->level;
    const LevelView &x = level_at(a, l);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // count
    int32_t mine = 0;
    for (int s = threadIdx.x; s < x.S; s += blockDim.x) mine += x.iters[s] == 0;
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
    if (lane == 0) part[w] = mine;
    __syncthreads();
    int32_t K = 0;
    for (int i = 0; i < nw; i++) K += part[i];
    int to = -1;
    for (int c = kLevels - 1; c > l; c--) {
        if (K > 0 && level_at(a, c).S > 0 && K <= level_at(a, c).S) {
            to = c;
            break;
        }
    }
    if (to >= 0) {
        // list: running slots in slot order
        int32_t *map = level_at(a, to).map;
        if (threadIdx.x == 0) base = 0;
        __syncthreads();
        for (int s0 = 0; s0 < x.S; s0 += blockDim.x) {
            const int s = s0 + int(threadIdx.x);
            const bool run = s < x.S && x.iters[s] == 0;
            const uint64_t m = __ballot(run);
            if (lane == 0) part[w] = __popcll(m);
            __syncthreads();
            int before = base;
            for (int i = 0; i < w; i++) before += part[i];
            if (run) map[before + __popcll(m & ((uint64_t(1) << lane) - 1u))] = s;
            __syncthreads();
            if (threadIdx.x == 0) {
                int tot = 0;
                for (int i = 0; i < nw; i++) tot += part[i];
                base += tot;
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        ctl->running = K;
        ctl->to = to;
        if (to >= 0) {
            ctl->from = l;
            ctl->src[to] = l;
            ctl->count[to] = K;
            ctl->level = to;
        }
    }
}

// dst[r][k] = src[r][map[k]] for k < K, 0 above (rows x St elements).
template <typename W>
__device__ __forceinline__ void gather_rows(const W *__restrict__ src, int32_t Sf, W *__restrict__ dst, int32_t St,
                                            int64_t rows, const int32_t *__restrict__ map, int32_t K) {
    const int64_t total = rows * St;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t r = i / St;
        const int k = int(i - r * St);
        dst[i] = k < K ? src[r * Sf + map[k]] : W(0);
    }
}

// The move the last count decided, if any: messages, channel LLRs, posteriors
// and fail marks of the running frames into the new level; its slots above
// the running count are padding.
template <typename W, typename PW>
__global__ __launch_bounds__(256) void level_move_kernel(const LevelCtl *__restrict__ ctl, Levels a, int64_t E,
                                                         int64_t n, int32_t keep32) {
    const int to = wave_uniform(cload(&ctl->to));
    if (to < 0) return;
    const int from = wave_uniform(cload(&ctl->from));
    const int32_t K = wave_uniform(cload(&ctl->count[to]));
    const LevelView &f = level_at(a, from);
    const LevelView &d = level_at(a, to);
    gather_rows<W>(static_cast<const W *>(f.r), f.S, static_cast<W *>(d.r), d.S, E, d.map, K);
    gather_rows<float>(f.lch, f.S, d.lch, d.S, n, d.map, K);
    gather_rows<PW>(static_cast<const PW *>(f.post), f.S, static_cast<PW *>(d.post), d.S, n, d.map, K);
    if (keep32) gather_rows<float>(f.lpost, f.S, d.lpost, d.S, n, d.map, K);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d.S; k += gridDim.x * blockDim.x) {
        d.iters[k] = k < K ? 0 : kPadSlot;
        d.fail[k] = k < K ? f.fail[d.map[k]] : 0;
    }
}

// Level l back into the level its frames came from, if it was entered:
// posteriors, iteration counts and fail marks (messages are not needed after
// the last iteration).  Deeper levels go first.
template <typename PT>
__global__ __launch_bounds__(256) void level_scatter_kernel(const LevelCtl *__restrict__ ctl, Levels a, int32_t l,
                                                            int64_t n, int32_t keep32) {
    const int up = wave_uniform(cload(&ctl->src[l]));
    if (up < 0) return;
    const int32_t K = wave_uniform(cload(&ctl->count[l]));
    const LevelView &x = level_at(a, l);
    const LevelView &u = level_at(a, up);
    const int64_t total = n * x.S;
    const PT *xp = static_cast<const PT *>(x.post);
    PT *upost = static_cast<PT *>(u.post);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t v = i / x.S;
        const int k = int(i - v * x.S);
        if (k < K) {
            upost[v * u.S + x.map[k]] = xp[i];
            if (keep32) u.lpost[v * u.S + x.map[k]] = x.lpost[i];
        }
    }
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        u.iters[x.map[k]] = x.iters[k];
        u.fail[x.map[k]] = x.fail[k];
    }
}

struct Plan {
    int msg = kF32;
    int V = 1;
    int32_t S = 0;
    size_t off_lch = 0, off_lpost = 0, off_post = 0, off_r = 0, off_iters = 0, off_fail = 0;
    size_t off_aggd = 0, off_aggpre = 0, off_aggbits = 0, total = 0;
    size_t off_err = 0, off_it = 0, off_ok = 0;   // Monte-Carlo runs only
    // tail compaction (LDPC_COMPACT_TAIL): two copies of the state, for S/2
    // and S/4 slots (level 1 and 2), and the control words (LevelCtl)
    struct Level {
        int32_t Sc = 0;
        size_t off_lch = 0, off_lpost = 0, off_post = 0, off_r = 0, off_iters = 0, off_fail = 0, off_map = 0;
    } lv[2];
    size_t off_ctl = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr uint32_t kLaneSlotFlags = LDPC_LANE_SLOTS_1 | LDPC_LANE_SLOTS_2 | LDPC_LANE_SLOTS_4;

bool flags_ok(uint32_t flags) {
    const uint32_t known =
        LDPC_NO_EARLY_STOP | LDPC_MSG_FP16 | LDPC_MSG_BF16 | LDPC_MSG_Q8 | kLaneSlotFlags | LDPC_COMPACT_TAIL;
    if (flags & ~known) return false;
    if (__builtin_popcount(flags & (LDPC_MSG_FP16 | LDPC_MSG_BF16 | LDPC_MSG_Q8)) > 1) return false;
    if (__builtin_popcount(flags & kLaneSlotFlags) > 1) return false;
    return true;
}

Plan make_plan(const ldpc_graph *g, int32_t F, uint32_t flags, bool sim = false) {
    Plan p;
    p.msg = (flags & LDPC_MSG_FP16) ? kF16 : (flags & LDPC_MSG_BF16) ? kBF16 : (flags & LDPC_MSG_Q8) ? kQ8 : kF32;
    if (flags & LDPC_LANE_SLOTS_1) p.V = 1;
    else if (flags & LDPC_LANE_SLOTS_2) p.V = 2;
    else if (flags & LDPC_LANE_SLOTS_4) p.V = 4;
    else p.V = F > 128 ? 4 : F > 64 ? 2 : 1;
    const int32_t unit = 64 * p.V;
    p.S = (std::max<int32_t>(F, 1) + unit - 1) / unit * unit;
    const size_t S = size_t(p.S);
    const size_t msg_bytes = p.msg == kF32 ? 4 : p.msg == kQ8 ? 1 : 2;
    size_t off = 0;
    p.off_lch = off;     off = align256(off + size_t(g->n) * S * 4);
    p.off_lpost = off;   off = align256(off + size_t(g->n) * S * 4);
    // 16-bit message formats keep a 16-bit copy of the posterior for the check pass
    const bool post16 = p.msg == kF16 || p.msg == kBF16;
    p.off_post = p.off_lpost;
    if (post16) { p.off_post = off; off = align256(off + size_t(g->n) * S * 2); }
    p.off_r = off;       off = align256(off + size_t(g->E) * S * msg_bytes);
    p.off_iters = off;   off = align256(off + S * 4);
    p.off_fail = off;    off = align256(off + S * 4);
    p.off_aggd = off;    off = align256(off + size_t(g->hub_chunks) * S * 4);
    p.off_aggpre = off;  off = align256(off + size_t(g->hub_chunks) * S * 4);
    p.off_aggbits = off; off = align256(off + size_t(g->hub_chunks) * S * 4);
    if (sim) {
        p.off_err = off; off = align256(off + S * 4);
        p.off_it = off;  off = align256(off + S * 4);
        p.off_ok = off;  off = align256(off + S);
    }
    // Pools below 256 slots are left as they are.  A copy uses the largest
    // multiple of 64 slots within its capacity (S/2, S/4).
    if ((flags & LDPC_COMPACT_TAIL) && !(flags & LDPC_NO_EARLY_STOP) && p.S >= 256) {
        for (int l = 0; l < 2; l++) {
            Plan::Level &L = p.lv[l];
            L.Sc = p.S / (2 << l);
            const size_t Sc = size_t(L.Sc);
            L.off_lch = off;   off = align256(off + size_t(g->n) * Sc * 4);
            L.off_lpost = off; off = align256(off + size_t(g->n) * Sc * 4);
            L.off_post = L.off_lpost;
            if (post16) { L.off_post = off; off = align256(off + size_t(g->n) * Sc * 2); }
            L.off_r = off;     off = align256(off + size_t(g->E) * Sc * msg_bytes);
            L.off_iters = off; off = align256(off + Sc * 4);
            L.off_fail = off;  off = align256(off + Sc * 4);
            L.off_map = off;   off = align256(off + Sc * 4);
        }
        p.off_ctl = off; off = align256(off + sizeof(LevelCtl));
    }
    p.total = off;
    return p;
}

struct Bufs {
    float *lch, *lpost;
    void *post;             // posterior in the check pass's storage (Post<M>); lpost for 32/8-bit messages
    void *r;
    int32_t *iters, *fail;
    float *aggd, *aggpre;
    int32_t *aggbits;
    char *base = nullptr;   // the workspace (for the compaction copy's offsets)
};

inline unsigned blocks_for_waves(int64_t waves) { return unsigned((waves + 3) / 4); }

template <int M, int V, int DMAX, int RULE>
void launch_rows(const ldpc_graph *g, int cls, int mode, const void *L, const Bufs &b, int32_t S, int32_t syn_iter,
                 float rp, hipStream_t st) {
    const int32_t nrows = g->class_begin[cls + 1] - g->class_begin[cls];
    if (nrows == 0) return;
    const int32_t groups = S / (64 * V);
    const unsigned blocks = blocks_for_waves(int64_t(nrows) * groups);
    using T = typename Codec<M>::T;
    T *R = static_cast<T *>(b.r);
    const int32_t *rd = g->d_class_rd + 2 * g->class_begin[cls];
    const int32_t *rows = g->d_class_rows + g->class_begin[cls];
    // quasi-cyclic graphs take their bits from the base matrix (sum-product rule)
    if constexpr (RULE == kRuleSP) {
        if (g->qc_Z > 0) {
            if (mode == kFirst)
                hipLaunchKernelGGL((check_rows_kernel<M, V, DMAX, kFirst, RULE, true>), dim3(blocks), dim3(256), 0,
                                   st, rd, g->d_col_idx, nrows, static_cast<const CheckL<M, kFirst> *>(L), R,
                                   b.iters, b.fail, S, groups, 0, rp, rows, g->d_qc_row_ptr, g->d_qc_ent, g->qc_Z);
            else
                hipLaunchKernelGGL((check_rows_kernel<M, V, DMAX, kIter, RULE, true>), dim3(blocks), dim3(256), 0,
                                   st, rd, g->d_col_idx, nrows, static_cast<const CheckL<M, kIter> *>(L), R,
                                   b.iters, b.fail, S, groups, syn_iter, rp, rows, g->d_qc_row_ptr, g->d_qc_ent,
                                   g->qc_Z);
            return;
        }
    }
    if (mode == kFirst)
        hipLaunchKernelGGL((check_rows_kernel<M, V, DMAX, kFirst, RULE, false>), dim3(blocks), dim3(256), 0, st, rd,
                           g->d_col_idx, nrows, static_cast<const CheckL<M, kFirst> *>(L), R, b.iters, b.fail, S,
                           groups, 0, rp, nullptr, nullptr, nullptr, 0);
    else
        hipLaunchKernelGGL((check_rows_kernel<M, V, DMAX, kIter, RULE, false>), dim3(blocks), dim3(256), 0, st, rd,
                           g->d_col_idx, nrows, static_cast<const CheckL<M, kIter> *>(L), R, b.iters, b.fail, S,
                           groups, syn_iter, rp, nullptr, nullptr, nullptr, 0);
}

template <int M, int V, int WPR, int RULE>
void launch_chunked(const ldpc_graph *g, int cls, int mode, const void *L, const Bufs &b, int32_t S,
                    int32_t syn_iter, float rp, hipStream_t st) {
    const int32_t nrows = g->class_begin[cls + 1] - g->class_begin[cls];
    if (nrows == 0) return;
    const int32_t groups = S / (64 * V);
    const int64_t items = int64_t(nrows) * groups;
    const unsigned blocks = unsigned((items + (4 / WPR) - 1) / (4 / WPR));
    using T = typename Codec<M>::T;
    T *R = static_cast<T *>(b.r);
    const int32_t *rd = g->d_class_rd + 2 * g->class_begin[cls];
    if (mode == kFirst)
        hipLaunchKernelGGL((check_chunk_kernel<M, V, WPR, kFirst, RULE>), dim3(blocks), dim3(256), 0, st, rd,
                           g->d_col_idx, nrows, static_cast<const CheckL<M, kFirst> *>(L), R, b.iters, b.fail, S,
                           groups, 0, rp);
    else
        hipLaunchKernelGGL((check_chunk_kernel<M, V, WPR, kIter, RULE>), dim3(blocks), dim3(256), 0, st, rd,
                           g->d_col_idx, nrows, static_cast<const CheckL<M, kIter> *>(L), R, b.iters, b.fail, S,
                           groups, syn_iter, rp);
}

template <int M, int RULE>
void launch_hub(const ldpc_graph *g, int mode, const void *L, const Bufs &b, int32_t S, int32_t syn_iter, float rp,
                hipStream_t st) {
    const int32_t nrows = g->class_begin[ldpc::kClassHub + 1] - g->class_begin[ldpc::kClassHub];
    if (nrows == 0) return;
    const int32_t groups = S / 64;
    using T = typename Codec<M>::T;
    T *R = static_cast<T *>(b.r);
    const int32_t *rd = g->d_class_rd + 2 * g->class_begin[ldpc::kClassHub];
    // rows above kWideRowMax lead the class (longest first): segmented path
    const int32_t nseg = g->hub_seg_rows, nwide = nrows - nseg;
    if (nseg > 0) {
        const unsigned blocks = unsigned(int64_t(nseg) * groups);
        if (mode == kFirst)
            hipLaunchKernelGGL((check_hub_kernel<M, kFirst, RULE>), dim3(blocks), dim3(256), 0, st, rd, g->d_col_idx,
                               nseg, g->d_hub_chunk_base, static_cast<const CheckL<M, kFirst> *>(L), R, b.iters,
                               b.fail, S, groups, 0, b.aggd, b.aggpre, b.aggbits, rp);
        else
            hipLaunchKernelGGL((check_hub_kernel<M, kIter, RULE>), dim3(blocks), dim3(256), 0, st, rd, g->d_col_idx,
                               nseg, g->d_hub_chunk_base, static_cast<const CheckL<M, kIter> *>(L), R, b.iters,
                               b.fail, S, groups, syn_iter, b.aggd, b.aggpre, b.aggbits, rp);
    }
    if (nwide > 0) {
        const unsigned blocks = unsigned(int64_t(nwide) * groups);
        const dim3 block(64 * kWideWaves);
        if (mode == kFirst)
            hipLaunchKernelGGL((check_wide_kernel<M, kFirst, RULE>), dim3(blocks), block, 0, st, rd + 2 * nseg,
                               g->d_col_idx, nwide, static_cast<const CheckL<M, kFirst> *>(L), R, b.iters, b.fail, S,
                               groups, 0, rp);
        else
            hipLaunchKernelGGL((check_wide_kernel<M, kIter, RULE>), dim3(blocks), block, 0, st, rd + 2 * nseg,
                               g->d_col_idx, nwide, static_cast<const CheckL<M, kIter> *>(L), R, b.iters, b.fail, S,
                               groups, syn_iter, rp);
    }
}

template <int M, int V, int RULE>
void launch_check_pass(const ldpc_graph *g, int mode, const void *L, const Bufs &b, int32_t S, int32_t syn_iter,
                       float rp, hipStream_t st) {
    launch_rows<M, V, 8, RULE>(g, ldpc::kClassD8, mode, L, b, S, syn_iter, rp, st);
    launch_rows<M, ldpc::class_lane_slots(ldpc::kClassD16, V), 16, RULE>(g, ldpc::kClassD16, mode, L, b, S, syn_iter,
                                                                         rp, st);
    launch_chunked<M, V, ldpc::class_waves_per_row(ldpc::kClassD128), RULE>(g, ldpc::kClassD128, mode, L, b, S,
                                                                             syn_iter, rp, st);
    launch_hub<M, RULE>(g, mode, L, b, S, syn_iter, rp, st);
}

// The check rule of a decode call: kind (RuleKind) and parameter.
struct RuleSel {
    int kind = kRuleSP;
    float param = 0.f;
};

template <int M, int V>
void launch_check_pass_rule(const ldpc_graph *g, int mode, const void *L, const Bufs &b, int32_t S,
                            int32_t syn_iter, const RuleSel &rule, hipStream_t st) {
    switch (rule.kind) {
        case kRuleNMS: launch_check_pass<M, V, kRuleNMS>(g, mode, L, b, S, syn_iter, rule.param, st); break;
        case kRuleOMS: launch_check_pass<M, V, kRuleOMS>(g, mode, L, b, S, syn_iter, rule.param, st); break;
        default: launch_check_pass<M, V, kRuleSP>(g, mode, L, b, S, syn_iter, 0.f, st); break;
    }
}

// Optional event marks for the profiled entry point: mark(i) records event i
// on the decode stream.  Layout: 0 start, 1 after ingest, then per iteration
// t (1-based) 2t after the check pass and 2t+1 after the bit pass, and
// 2T+2 after the syndrome/finalize/egress tail.
struct Marks {
    hipEvent_t *ev = nullptr;
    void mark(int i, hipStream_t st) const {
        if (ev) (void)hipEventRecord(ev[i], st);
    }
};

// A Monte-Carlo run (ldpc_simulate): the channel LLRs are drawn on the device
// instead of read from llr_in, and the per-frame outputs are counted instead
// of written out.
struct SimRun {
    bool on = false;
    uint32_t key0 = 0, key1 = 0;
    uint64_t first_frame = 0;
    float k0 = 0.f, k1 = 0.f;
    float *llr_out = nullptr;
    int32_t *err = nullptr, *it = nullptr;
    uint8_t *ok = nullptr;
    ldpc_sim_counts *counts = nullptr;
};

// The levels of a call's tail compaction (LDPC_COMPACT_TAIL): views of the
// full state and of its copies, and the control words.  Off when the plan has
// no copies (too few slots, no early stop).
struct LevelSet {
    bool on = false;
    Levels a{};                 // views; V is per launch (with_class_v)
    int32_t V[kLevels] = {};    // slots per lane of the register rows and the bit pass
    LevelCtl *ctl = nullptr;
};

LevelSet level_set(const Plan &p, const Bufs &b, bool wanted, bool keep32) {
    LevelSet ls;
    if (!wanted || p.lv[0].Sc == 0 || !b.base) return ls;
    char *ws = b.base;
    LevelView &z = ls.a.lv[0];
    z.lch = b.lch;
    z.post = b.post;
    z.lpost = keep32 ? b.lpost : nullptr;
    z.r = b.r;
    z.iters = b.iters;
    z.fail = b.fail;
    z.map = nullptr;
    z.S = p.S;
    ls.V[0] = p.V;
    for (int l = 1; l < kLevels; l++) {
        const Plan::Level &L = p.lv[l - 1];
        LevelView &x = ls.a.lv[l];
        x.lch = reinterpret_cast<float *>(ws + L.off_lch);
        x.post = ws + L.off_post;
        x.lpost = keep32 ? reinterpret_cast<float *>(ws + L.off_lpost) : nullptr;
        x.r = ws + L.off_r;
        x.iters = reinterpret_cast<int32_t *>(ws + L.off_iters);
        x.fail = reinterpret_cast<int32_t *>(ws + L.off_fail);
        x.map = reinterpret_cast<int32_t *>(ws + L.off_map);
        x.S = L.Sc / 64 * 64;
        int v = std::max(1, p.V >> l);
        if (x.S % (64 * v) != 0) v = 1;
        ls.V[l] = v;
        if (x.S < 64) x.S = 0;
    }
    ls.ctl = reinterpret_cast<LevelCtl *>(ws + p.off_ctl);
    ls.a.level = &ls.ctl->level;
    ls.on = ls.a.lv[1].S > 0;
    return ls;
}

// The views with the slots per lane of check class `cls` (every level's grid
// must fit in the full state's: checked by the caller through fits()).
Levels with_class_v(const LevelSet &ls, int cls) {
    Levels a = ls.a;
    for (int l = 0; l < kLevels; l++) a.lv[l].V = cls < 0 ? ls.V[l] : ldpc::class_lane_slots(cls, ls.V[l]);
    return a;
}

bool fits(const Levels &a) {
    for (int l = 1; l < kLevels; l++)
        if (a.lv[l].S > 0 && (a.lv[l].S % (64 * a.lv[l].V) != 0 ||
                              int64_t(a.lv[l].S) * a.lv[0].V > int64_t(a.lv[0].S) * a.lv[l].V))
            return false;
    return true;
}

__global__ __launch_bounds__(64) void level_init_kernel(LevelCtl *ctl) {
    if (threadIdx.x == 0) {
        ctl->level = 0;
        ctl->from = 0;
        ctl->to = -1;
        ctl->running = -1;
        for (int l = 0; l < kLevels; l++) {
            ctl->src[l] = -1;
            ctl->count[l] = 0;
        }
    }
}

// The check pass on the current level (iterations after the first count).
template <int M, int V, int RULE>
void launch_check_pass_levels(const ldpc_graph *g, const LevelSet &ls, int32_t syn_iter, float rp, const Bufs &b,
                              hipStream_t st) {
    const int32_t S = ls.a.lv[0].S;
    {
        constexpr int cls = ldpc::kClassD8;
        const int32_t nrows = g->class_begin[cls + 1] - g->class_begin[cls];
        if (nrows > 0) {
            const Levels a = with_class_v(ls, cls);
            const unsigned blocks = blocks_for_waves(int64_t(nrows) * (S / (64 * V)));
            const int32_t *rd = g->d_class_rd + 2 * g->class_begin[cls];
            const bool qc = RULE == kRuleSP && g->qc_Z > 0;
            if (qc)
                hipLaunchKernelGGL((check_rows_level_kernel<M, V, 8, RULE, true>), dim3(blocks), dim3(256), 0, st, rd,
                                   g->d_col_idx, nrows, a, syn_iter, rp, g->d_class_rows + g->class_begin[cls],
                                   g->d_qc_row_ptr, g->d_qc_ent, g->qc_Z);
            else
                hipLaunchKernelGGL((check_rows_level_kernel<M, V, 8, RULE, false>), dim3(blocks), dim3(256), 0, st,
                                   rd, g->d_col_idx, nrows, a, syn_iter, rp, nullptr, nullptr, nullptr, 0);
        }
    }
    {
        constexpr int cls = ldpc::kClassD16;
        constexpr int V16 = ldpc::class_lane_slots(cls, V);
        const int32_t nrows = g->class_begin[cls + 1] - g->class_begin[cls];
        if (nrows > 0) {
            const Levels a = with_class_v(ls, cls);
            const unsigned blocks = blocks_for_waves(int64_t(nrows) * (S / (64 * V16)));
            const int32_t *rd = g->d_class_rd + 2 * g->class_begin[cls];
            const bool qc = RULE == kRuleSP && g->qc_Z > 0;
            if (qc)
                hipLaunchKernelGGL((check_rows_level_kernel<M, V16, 16, RULE, true>), dim3(blocks), dim3(256), 0, st,
                                   rd, g->d_col_idx, nrows, a, syn_iter, rp, g->d_class_rows + g->class_begin[cls],
                                   g->d_qc_row_ptr, g->d_qc_ent, g->qc_Z);
            else
                hipLaunchKernelGGL((check_rows_level_kernel<M, V16, 16, RULE, false>), dim3(blocks), dim3(256), 0, st,
                                   rd, g->d_col_idx, nrows, a, syn_iter, rp, nullptr, nullptr, nullptr, 0);
        }
    }
    {
        constexpr int cls = ldpc::kClassD128;
        constexpr int WPR = ldpc::class_waves_per_row(cls);
        const int32_t nrows = g->class_begin[cls + 1] - g->class_begin[cls];
        if (nrows > 0) {
            const Levels a = with_class_v(ls, cls);
            const int64_t items = int64_t(nrows) * (S / (64 * V));
            const unsigned blocks = unsigned((items + (4 / WPR) - 1) / (4 / WPR));
            hipLaunchKernelGGL((check_chunk_level_kernel<M, V, WPR, RULE>), dim3(blocks), dim3(256), 0, st,
                               g->d_class_rd + 2 * g->class_begin[cls], g->d_col_idx, nrows, a, syn_iter, rp);
        }
    }
    {
        const int32_t nrows = g->class_begin[ldpc::kClassHub + 1] - g->class_begin[ldpc::kClassHub];
        if (nrows > 0) {
            const Levels a = with_class_v(ls, ldpc::kClassHub);
            const int32_t groups = S / 64;
            const int32_t *rd = g->d_class_rd + 2 * g->class_begin[ldpc::kClassHub];
            const int32_t nseg = g->hub_seg_rows, nwide = nrows - nseg;
            if (nseg > 0)
                hipLaunchKernelGGL((check_hub_level_kernel<M, RULE>), dim3(unsigned(int64_t(nseg) * groups)),
                                   dim3(256), 0, st, rd, g->d_col_idx, nseg, g->d_hub_chunk_base, a, syn_iter, b.aggd,
                                   b.aggpre, b.aggbits, rp);
            if (nwide > 0)
                hipLaunchKernelGGL((check_wide_level_kernel<M, RULE>), dim3(unsigned(int64_t(nwide) * groups)),
                                   dim3(64 * kWideWaves), 0, st, rd + 2 * nseg, g->d_col_idx, nwide, a, syn_iter, rp);
        }
    }
}

template <int M, int V>
void launch_check_pass_levels_rule(const ldpc_graph *g, const LevelSet &ls, int32_t syn_iter, const RuleSel &rule,
                                   const Bufs &b, hipStream_t st) {
    switch (rule.kind) {
        case kRuleNMS: launch_check_pass_levels<M, V, kRuleNMS>(g, ls, syn_iter, rule.param, b, st); break;
        case kRuleOMS: launch_check_pass_levels<M, V, kRuleOMS>(g, ls, syn_iter, rule.param, b, st); break;
        default: launch_check_pass_levels<M, V, kRuleSP>(g, ls, syn_iter, 0.f, b, st); break;
    }
}

// Every launch class of the decode fits the level grid rule.
bool level_set_fits(const LevelSet &ls) {
    return fits(with_class_v(ls, -1)) && fits(with_class_v(ls, ldpc::kClassD8)) &&
           fits(with_class_v(ls, ldpc::kClassD16)) && fits(with_class_v(ls, ldpc::kClassD128)) &&
           fits(with_class_v(ls, ldpc::kClassHub));
}

template <int M, int V>
void run_decode(const ldpc_graph *g, const Plan &p, const Bufs &b, const float *llr_in, int32_t F, int32_t T,
                bool early_stop, uint8_t *bits, uint8_t *ok, int32_t *iters_out, float *llr_out, hipStream_t st,
                const Marks &mk, const SimRun &sim, const RuleSel &rule) {
    using MT = typename Codec<M>::T;
    using PT = typename Post<M>::T;
    const int32_t S = p.S;
    const int32_t groups = S / (64 * V);
    // 16-bit message formats write the fp32 posterior only when it is an output
    const bool keep32 = kPost16<M> && llr_out && !sim.on;
    _Float16 *post16 = kPost16<M> ? static_cast<_Float16 *>(b.post) : nullptr;
    // factor of a bit's message sum in its posterior (the messages' units)
    const float bscale = rule.kind == kRuleNMS   ? MsgUnits<M, kRuleNMS>::kBitScale
                         : rule.kind == kRuleOMS ? MsgUnits<M, kRuleOMS>::kBitScale
                                                 : MsgUnits<M, kRuleSP>::kBitScale;
    mk.mark(0, st);
    hipLaunchKernelGGL(init_state_kernel, dim3((S + 255) / 256), dim3(256), 0, st, b.iters, b.fail, F, S);
    const dim3 tgrid((g->n + 63) / 64, S / 64);
    if (sim.on) {
        const unsigned quads = unsigned(std::min(65535, (g->n + 3) / 4));
        hipLaunchKernelGGL(channel_kernel, dim3(unsigned((S + 255) / 256), quads), dim3(256), 0, st, b.lch, S, F,
                           g->n, sim.key0, sim.key1, sim.first_frame, sim.k0, sim.k1, sim.llr_out, post16);
        hipLaunchKernelGGL(zero_kernel, dim3(unsigned((S + 255) / 256)), dim3(256), 0, st, sim.err, S);
    } else {
        hipLaunchKernelGGL(ingest_kernel, tgrid, dim3(256), 0, st, llr_in, F, g->n, b.lch, S, post16);
    }
    mk.mark(1, st);
    const unsigned bit_blocks = blocks_for_waves(int64_t(g->n) * groups);

    // Tail compaction: after iteration kFirstCheck and every kEvery
    // iterations after it, the device counts the running frames and moves
    // them into a smaller level once they fit one; the passes after the first
    // count run on whichever level the frames are in.
    constexpr int32_t kFirstCheck = 8, kEvery = 4;
    LevelSet ls = level_set(p, b, early_stop, keep32);
    if (ls.on && !level_set_fits(ls)) ls.on = false;
    if (ls.on) hipLaunchKernelGGL(level_init_kernel, dim3(1), dim3(64), 0, st, ls.ctl);
    const Levels bit_levels = with_class_v(ls, -1);
    for (int32_t t = 1; t <= T; t++) {
        const int32_t syn_iter = (early_stop && t > 1) ? t - 1 : 0;
        if (ls.on && t > kFirstCheck) {
            launch_check_pass_levels_rule<M, V>(g, ls, syn_iter, rule, b, st);
            mk.mark(2 * t, st);
            hipLaunchKernelGGL((bit_level_kernel<M, V>), dim3(bit_blocks), dim3(256), 0, st, g->d_col_ptr,
                               g->d_csc_to_csr, g->n, bit_levels, t, int32_t(early_stop), bscale);
            mk.mark(2 * t + 1, st);
        } else {
            const void *L1 = kPost16<M> ? b.post : static_cast<const void *>(b.lch);
            launch_check_pass_rule<M, V>(g, t == 1 ? kFirst : kIter, t == 1 ? L1 : b.post, b, S, syn_iter, rule,
                                         st);
            mk.mark(2 * t, st);
            hipLaunchKernelGGL((bit_kernel<M, V>), dim3(bit_blocks), dim3(256), 0, st, g->d_col_ptr, g->d_csc_to_csr,
                               g->n, b.lch, static_cast<const MT *>(b.r), static_cast<PT *>(b.post),
                               keep32 ? b.lpost : nullptr, b.iters, b.fail, S, groups, t,
                               int32_t(early_stop), bscale);
            mk.mark(2 * t + 1, st);
        }
        if (ls.on && t >= kFirstCheck && (t - kFirstCheck) % kEvery == 0 && t < T) {
            using W = typename Raw<sizeof(MT)>::T;
            using PW = typename Raw<sizeof(PT)>::T;
            hipLaunchKernelGGL(level_decide_kernel, dim3(1), dim3(1024), 0, st, ls.ctl, ls.a);
            hipLaunchKernelGGL((level_move_kernel<W, PW>), dim3(2048), dim3(256), 0, st, ls.ctl, ls.a, int64_t(g->E),
                               int64_t(g->n), int32_t(keep32));
        }
    }
    // posteriors, iteration counts and fail marks back to the full state
    if (ls.on && T > kFirstCheck) {
        for (int l = kLevels - 1; l > 0; l--)
            hipLaunchKernelGGL((level_scatter_kernel<PT>), dim3(2048), dim3(256), 0, st, ls.ctl, ls.a, l,
                               int64_t(g->n), int32_t(keep32));
    }
    const int32_t nrows = g->class_begin[ldpc::kNumClasses];
    if (nrows > 0) {
        hipLaunchKernelGGL((syndrome_kernel<V, PT>), dim3(blocks_for_waves(int64_t(nrows) * groups)), dim3(256), 0, st,
                           g->d_class_rd, g->d_col_idx, nrows, static_cast<const PT *>(b.post), b.iters, b.fail, S,
                           groups, T);
    }
    if (sim.on) {
        hipLaunchKernelGGL(finalize_kernel, dim3((F + 255) / 256), dim3(256), 0, st, b.iters, b.fail, F, T, sim.it,
                           sim.ok);
        const unsigned rows = unsigned(std::min(4096, (g->n + 63) / 64));
        hipLaunchKernelGGL((count_errors_kernel<PT>), dim3(unsigned((F + 255) / 256), rows), dim3(256), 0, st,
                           static_cast<const PT *>(b.post), S, F, g->n, sim.err);
        hipLaunchKernelGGL(tally_kernel, dim3(unsigned((F + 255) / 256)), dim3(256), 0, st, sim.err, sim.it, sim.ok, F,
                           sim.counts);
    } else {
        hipLaunchKernelGGL(finalize_kernel, dim3((F + 255) / 256), dim3(256), 0, st, b.iters, b.fail, F, T, iters_out,
                           ok);
        hipLaunchKernelGGL((egress_kernel<PT>), tgrid, dim3(256), 0, st, static_cast<const PT *>(b.post), b.lpost, S, F,
                           g->n, bits, llr_out);
    }
    mk.mark(2 * T + 2, st);
}

template <int M>
void run_decode_v(const ldpc_graph *g, const Plan &p, const Bufs &b, const float *llr_in, int32_t F, int32_t T,
                  bool es, uint8_t *bits, uint8_t *ok, int32_t *it, float *lo, hipStream_t st, const Marks &mk,
                  const SimRun &sim, const RuleSel &rule) {
    switch (p.V) {
        case 4: run_decode<M, 4>(g, p, b, llr_in, F, T, es, bits, ok, it, lo, st, mk, sim, rule); break;
        case 2: run_decode<M, 2>(g, p, b, llr_in, F, T, es, bits, ok, it, lo, st, mk, sim, rule); break;
        default: run_decode<M, 1>(g, p, b, llr_in, F, T, es, bits, ok, it, lo, st, mk, sim, rule); break;
    }
}

// Validate an ldpc_rule (NULL: sum-product) into `out`.
bool rule_from(const ldpc_rule *r, RuleSel &out, std::string &why) {
    out = RuleSel{};
    if (!r) return true;
    for (int32_t x : r->reserved)
        if (x != 0) { why = "reserved rule fields must be 0"; return false; }
    if (!ldpc::rule_ok(r->kind, r->param, why)) return false;
    out.kind = r->kind == LDPC_RULE_MIN_SUM_NORMALIZED ? kRuleNMS : r->kind == LDPC_RULE_MIN_SUM_OFFSET ? kRuleOMS : kRuleSP;
    out.param = out.kind == kRuleSP ? 0.f : r->param;
    return true;
}

}  // namespace

using ldpc::set_error;

extern "C" ldpc_status ldpc_decode_workspace_size(const ldpc_graph *g, int32_t frames, uint32_t flags, size_t *bytes) {
    if (!g || !bytes) { set_error("ldpc_decode_workspace_size: NULL argument"); return LDPC_E_INVAL; }
    if (frames < 0) { set_error("ldpc_decode_workspace_size: frames < 0"); return LDPC_E_INVAL; }
    if (!flags_ok(flags)) { set_error("ldpc_decode_workspace_size: bad flags"); return LDPC_E_INVAL; }
    *bytes = frames == 0 ? 0 : make_plan(g, frames, flags).total;
    return LDPC_OK;
}

namespace {

Bufs bufs_at(char *ws, const Plan &p) {
    Bufs b;
    b.lch = reinterpret_cast<float *>(ws + p.off_lch);
    b.lpost = reinterpret_cast<float *>(ws + p.off_lpost);
    b.post = ws + p.off_post;
    b.r = ws + p.off_r;
    b.iters = reinterpret_cast<int32_t *>(ws + p.off_iters);
    b.fail = reinterpret_cast<int32_t *>(ws + p.off_fail);
    b.aggd = reinterpret_cast<float *>(ws + p.off_aggd);
    b.aggpre = reinterpret_cast<float *>(ws + p.off_aggpre);
    b.aggbits = reinterpret_cast<int32_t *>(ws + p.off_aggbits);
    b.base = ws;
    return b;
}

ldpc_status decode_core(const char *fn, const ldpc_graph *g, const float *llr_in, int32_t frames, int32_t max_iter,
                        uint32_t flags, const ldpc_rule *rule_in, uint8_t *bits_out, uint8_t *syndrome_ok,
                        int32_t *iters, float *llr_out, void *workspace, size_t workspace_bytes, void *hip_stream,
                        const Marks &mk) {
    const std::string f(fn);
    if (!g) { set_error(f + ": graph is NULL"); return LDPC_E_INVAL; }
    RuleSel rule;
    std::string why;
    if (!rule_from(rule_in, rule, why)) { set_error(f + ": " + why); return LDPC_E_INVAL; }
    if (g->host_only) { set_error(f + ": graph was built host-only"); return LDPC_E_INVAL; }
    if (frames < 0) { set_error(f + ": frames < 0"); return LDPC_E_INVAL; }
    if (max_iter < 1) { set_error(f + ": max_iter must be >= 1"); return LDPC_E_INVAL; }
    if (!flags_ok(flags)) { set_error(f + ": bad flags"); return LDPC_E_INVAL; }
    if (frames == 0) return LDPC_OK;
    if (!llr_in || !bits_out || !syndrome_ok || !iters || !workspace) {
        set_error(f + ": NULL buffer");
        return LDPC_E_INVAL;
    }
    if (reinterpret_cast<uintptr_t>(workspace) & 255u) {
        set_error(f + ": workspace must be 256-byte aligned");
        return LDPC_E_INVAL;
    }
    const Plan p = make_plan(g, frames, flags);
    if (workspace_bytes < p.total) {
        set_error(f + ": workspace too small (" + std::to_string(workspace_bytes) + " < " + std::to_string(p.total) +
                  ")");
        return LDPC_E_INVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g->device) {
        (void)hipGetLastError();
        set_error(f + ": the current device is not the graph's device");
        return LDPC_E_INVAL;
    }
    const Bufs b = bufs_at(static_cast<char *>(workspace), p);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const bool es = !(flags & LDPC_NO_EARLY_STOP);
    (void)hipGetLastError();
    switch (p.msg) {
        case kF16:
            run_decode_v<kF16>(g, p, b, llr_in, frames, max_iter, es, bits_out, syndrome_ok, iters, llr_out, st, mk,
                               SimRun{}, rule);
            break;
        case kBF16:
            run_decode_v<kBF16>(g, p, b, llr_in, frames, max_iter, es, bits_out, syndrome_ok, iters, llr_out, st, mk,
                                SimRun{}, rule);
            break;
        case kQ8:
            run_decode_v<kQ8>(g, p, b, llr_in, frames, max_iter, es, bits_out, syndrome_ok, iters, llr_out, st, mk,
                              SimRun{}, rule);
            break;
        default:
            run_decode_v<kF32>(g, p, b, llr_in, frames, max_iter, es, bits_out, syndrome_ok, iters, llr_out, st, mk,
                               SimRun{}, rule);
            break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(f + ": launch failed: " + hipGetErrorString(e));
        return LDPC_E_DEVICE;
    }
    return LDPC_OK;
}

}  // namespace

extern "C" ldpc_status ldpc_decode(const ldpc_graph *g, const float *llr_in, int32_t frames, int32_t max_iter,
                                   uint32_t flags, uint8_t *bits_out, uint8_t *syndrome_ok, int32_t *iters,
                                   float *llr_out, void *workspace, size_t workspace_bytes, void *hip_stream) {
    return decode_core("ldpc_decode", g, llr_in, frames, max_iter, flags, nullptr, bits_out, syndrome_ok, iters,
                       llr_out, workspace, workspace_bytes, hip_stream, Marks{});
}

extern "C" ldpc_status ldpc_decode_rule(const ldpc_graph *g, const float *llr_in, int32_t frames, int32_t max_iter,
                                        uint32_t flags, const ldpc_rule *rule, uint8_t *bits_out,
                                        uint8_t *syndrome_ok, int32_t *iters, float *llr_out, void *workspace,
                                        size_t workspace_bytes, void *hip_stream) {
    return decode_core("ldpc_decode_rule", g, llr_in, frames, max_iter, flags, rule, bits_out, syndrome_ok, iters,
                       llr_out, workspace, workspace_bytes, hip_stream, Marks{});
}

extern "C" ldpc_status ldpc_decode_profiled(const ldpc_graph *g, const float *llr_in, int32_t frames,
                                            int32_t max_iter, uint32_t flags, uint8_t *bits_out,
                                            uint8_t *syndrome_ok, int32_t *iters, float *llr_out, void *workspace,
                                            size_t workspace_bytes, void *hip_stream, float *check_ms,
                                            float *bit_ms, float *edge_ms) {
    if (!check_ms || !bit_ms || !edge_ms) { set_error("ldpc_decode_profiled: NULL timing array"); return LDPC_E_INVAL; }
    if (frames <= 0 || max_iter < 1)
        return decode_core("ldpc_decode_profiled", g, llr_in, frames, max_iter, flags, nullptr, bits_out, syndrome_ok,
                           iters, llr_out, workspace, workspace_bytes, hip_stream, Marks{});
    const int nev = 2 * max_iter + 3;
    std::vector<hipEvent_t> ev(size_t(nev), nullptr);
    for (int i = 0; i < nev; i++) {
        if (hipEventCreate(&ev[size_t(i)]) != hipSuccess) {
            (void)hipGetLastError();
            for (int k = 0; k < i; k++) (void)hipEventDestroy(ev[size_t(k)]);
            set_error("ldpc_decode_profiled: hipEventCreate failed");
            return LDPC_E_DEVICE;
        }
    }
    Marks mk;
    mk.ev = ev.data();
    ldpc_status stt = decode_core("ldpc_decode_profiled", g, llr_in, frames, max_iter, flags, nullptr, bits_out,
                                  syndrome_ok, iters, llr_out, workspace, workspace_bytes, hip_stream, mk);
    if (stt == LDPC_OK) {
        if (hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("ldpc_decode_profiled: stream synchronization failed");
            stt = LDPC_E_DEVICE;
        } else {
            auto span = [&](int a, int b) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, ev[size_t(a)], ev[size_t(b)]);
                return ms;
            };
            edge_ms[0] = span(0, 1);
            for (int t = 1; t <= max_iter; t++) {
                check_ms[t - 1] = span(2 * t - 1, 2 * t);
                bit_ms[t - 1] = span(2 * t, 2 * t + 1);
            }
            edge_ms[1] = span(2 * max_iter + 1, 2 * max_iter + 2);
        }
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    return stt;
}

extern "C" ldpc_status ldpc_simulate_workspace_size(const ldpc_graph *g, int32_t frames, uint32_t flags,
                                                    size_t *bytes) {
    if (!g || !bytes) { set_error("ldpc_simulate_workspace_size: NULL argument"); return LDPC_E_INVAL; }
    if (frames < 0) { set_error("ldpc_simulate_workspace_size: frames < 0"); return LDPC_E_INVAL; }
    if (!flags_ok(flags)) { set_error("ldpc_simulate_workspace_size: bad flags"); return LDPC_E_INVAL; }
    *bytes = frames == 0 ? 0 : make_plan(g, frames, flags, true).total;
    return LDPC_OK;
}

namespace {

ldpc_status simulate_core(const char *fn, const ldpc_graph *g, int32_t frames, double ebn0_db, uint64_t seed,
                          uint64_t first_frame, int32_t max_iter, uint32_t flags, const ldpc_rule *rule_in,
                          ldpc_sim_counts *counts, float *llr_out, void *workspace, size_t workspace_bytes,
                          void *hip_stream) {
    const std::string f(fn);
    if (!g || !counts) { set_error(f + ": NULL graph or counts"); return LDPC_E_INVAL; }
    RuleSel rule;
    std::string why;
    if (!rule_from(rule_in, rule, why)) { set_error(f + ": " + why); return LDPC_E_INVAL; }
    if (g->host_only) { set_error(f + ": graph was built host-only"); return LDPC_E_INVAL; }
    if (frames < 0) { set_error(f + ": frames < 0"); return LDPC_E_INVAL; }
    if (max_iter < 1) { set_error(f + ": max_iter must be >= 1"); return LDPC_E_INVAL; }
    if (!flags_ok(flags)) { set_error(f + ": bad flags"); return LDPC_E_INVAL; }
    if (g->n <= g->m) { set_error(f + ": the nominal rate (n - m)/n must be positive"); return LDPC_E_INVAL; }
    if (!std::isfinite(ebn0_db)) { set_error(f + ": Eb/N0 must be finite"); return LDPC_E_INVAL; }
    if (frames == 0) return LDPC_OK;
    if (!workspace) { set_error(f + ": NULL workspace"); return LDPC_E_INVAL; }
    if (reinterpret_cast<uintptr_t>(workspace) & 255u) {
        set_error(f + ": workspace must be 256-byte aligned");
        return LDPC_E_INVAL;
    }
    const Plan p = make_plan(g, frames, flags, true);
    if (workspace_bytes < p.total) {
        set_error(f + ": workspace too small (" + std::to_string(workspace_bytes) + " < " + std::to_string(p.total) +
                  ")");
        return LDPC_E_INVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g->device) {
        (void)hipGetLastError();
        set_error(f + ": the current device is not the graph's device");
        return LDPC_E_INVAL;
    }
    char *ws = static_cast<char *>(workspace);
    const Bufs b = bufs_at(ws, p);
    // sigma^2 = 1 / (2 R 10^(EbN0/10)) with the nominal rate R = (n - m)/n (Eqs. (3)-(4));
    // L = 2y/sigma^2 = 2/sigma^2 + (2/sigma) z for y = 1 + sigma z
    const double rate = double(g->n - g->m) / double(g->n);
    const double sigma2 = 1.0 / (2.0 * rate * std::pow(10.0, ebn0_db / 10.0));
    SimRun sim;
    sim.on = true;
    sim.key0 = uint32_t(seed);
    sim.key1 = uint32_t(seed >> 32);
    sim.first_frame = first_frame;
    sim.k0 = float(2.0 / sigma2);
    sim.k1 = float(2.0 / std::sqrt(sigma2));
    sim.llr_out = llr_out;
    sim.err = reinterpret_cast<int32_t *>(ws + p.off_err);
    sim.it = reinterpret_cast<int32_t *>(ws + p.off_it);
    sim.ok = reinterpret_cast<uint8_t *>(ws + p.off_ok);
    sim.counts = counts;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const bool es = !(flags & LDPC_NO_EARLY_STOP);
    (void)hipGetLastError();
    switch (p.msg) {
        case kF16:
            run_decode_v<kF16>(g, p, b, nullptr, frames, max_iter, es, nullptr, nullptr, nullptr, nullptr, st, Marks{},
                               sim, rule);
            break;
        case kBF16:
            run_decode_v<kBF16>(g, p, b, nullptr, frames, max_iter, es, nullptr, nullptr, nullptr, nullptr, st,
                                Marks{}, sim, rule);
            break;
        case kQ8:
            run_decode_v<kQ8>(g, p, b, nullptr, frames, max_iter, es, nullptr, nullptr, nullptr, nullptr, st, Marks{},
                              sim, rule);
            break;
        default:
            run_decode_v<kF32>(g, p, b, nullptr, frames, max_iter, es, nullptr, nullptr, nullptr, nullptr, st, Marks{},
                               sim, rule);
            break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(f + ": launch failed: " + hipGetErrorString(e));
        return LDPC_E_DEVICE;
    }
    return LDPC_OK;
}

}  // namespace

extern "C" ldpc_status ldpc_simulate(const ldpc_graph *g, int32_t frames, double ebn0_db, uint64_t seed,
                                     uint64_t first_frame, int32_t max_iter, uint32_t flags,
                                     ldpc_sim_counts *counts, float *llr_out, void *workspace,
                                     size_t workspace_bytes, void *hip_stream) {
    return simulate_core("ldpc_simulate", g, frames, ebn0_db, seed, first_frame, max_iter, flags, nullptr, counts,
                         llr_out, workspace, workspace_bytes, hip_stream);
}

extern "C" ldpc_status ldpc_simulate_rule(const ldpc_graph *g, int32_t frames, double ebn0_db, uint64_t seed,
                                          uint64_t first_frame, int32_t max_iter, uint32_t flags,
                                          const ldpc_rule *rule, ldpc_sim_counts *counts, float *llr_out,
                                          void *workspace, size_t workspace_bytes, void *hip_stream) {
    return simulate_core("ldpc_simulate_rule", g, frames, ebn0_db, seed, first_frame, max_iter, flags, rule, counts,
                         llr_out, workspace, workspace_bytes, hip_stream);
}

// ---------------------------------------------------------------------------
// Decoding without allocation (ldpc_decode_noalloc): the workspace of
// ldpc_decode is this file-scope device array instead of caller memory.  Each
// device the library runs on holds its own copy until the process ends.  In
// host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device with that device current, and only
// that address is ever handed to a kernel.
static __device__ __align__(256) unsigned char scratch[LDPC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on device `dev` (the current device), looked up
// on the first call for that device; NULL (with the error set) on failure.
void *scratch_address(int dev, const std::string &f) {
    if (dev < 0 || dev >= kMaxScratchDevices) {
        set_error(f + ": device ordinal " + std::to_string(dev) + " is beyond the scratch table");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error(f + ": hipGetSymbolAddress(scratch) failed: " + hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" ldpc_status ldpc_decode_noalloc(const ldpc_graph *g, const float *llr_in, int32_t frames,
                                           int32_t max_iter, uint32_t flags, uint8_t *bits_out,
                                           uint8_t *syndrome_ok, int32_t *iters, float *llr_out,
                                           void *hip_stream) {
    const std::string f("ldpc_decode_noalloc");
    if (!g) { set_error(f + ": graph is NULL"); return LDPC_E_INVAL; }
    if (g->host_only) { set_error(f + ": graph was built host-only"); return LDPC_E_INVAL; }
    if (frames < 0) { set_error(f + ": frames < 0"); return LDPC_E_INVAL; }
    if (!flags_ok(flags)) { set_error(f + ": bad flags"); return LDPC_E_INVAL; }
    if (frames == 0 || max_iter < 1)   // no-op or an argument error, reported by the decode itself
        return decode_core(f.c_str(), g, llr_in, frames, max_iter, flags, nullptr, bits_out, syndrome_ok, iters,
                           llr_out, nullptr, 0, hip_stream, Marks{});
    const size_t need = make_plan(g, frames, flags).total;
    if (need > size_t(LDPC_NOALLOC_SCRATCH_BYTES)) {
        set_error(f + ": " + std::to_string(frames) + " frames need " + std::to_string(need) +
                  " bytes of state; the static scratch holds " + std::to_string(size_t(LDPC_NOALLOC_SCRATCH_BYTES)));
        return LDPC_E_RANGE;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g->device) {
        (void)hipGetLastError();
        set_error(f + ": the current device is not the graph's device");
        return LDPC_E_INVAL;
    }
    void *ws = scratch_address(dev, f);
    if (!ws) return LDPC_E_DEVICE;
    return decode_core(f.c_str(), g, llr_in, frames, max_iter, flags, nullptr, bits_out, syndrome_ok, iters, llr_out,
                       ws, size_t(LDPC_NOALLOC_SCRATCH_BYTES), hip_stream, Marks{});
}
