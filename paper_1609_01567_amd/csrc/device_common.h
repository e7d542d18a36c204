// Device-side building blocks shared by the plain decoder (decode.hip) and the
// batched engine (engine.hip): message storage codecs, vector loads/stores over
// a lane's frame slots, and the check-rule arithmetic.
//
// Check rule (Algorithm 1, second half, in LLR form).  With
// u = 1 - tanh(|Q|/2) = 2w/(1+w), w = exp(-|Q|), the product of tanh's over a
// set of edges is 1 - D, where D combines the u's with a (+) b = a + b(1 - a)
// (the complement of a product of complements), and the message magnitude is
// 2 atanh(1 - D) = ln((2 - D)/D).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace ldpc_dev {

constexpr float kLmax = 64.f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr int32_t kPadSlot = 0x7fffffff;   // iters value of a padding slot: never active

enum MsgType { kF32 = 0, kF16 = 1, kBF16 = 2, kQ8 = 3 };
enum Mode { kFirst = 0, kIter = 1 };

// ----------------------------------------------------------------- storage

template <int M> struct Codec;
template <> struct Codec<kF32> {
    using T = float;
    __device__ static float dec(T x) { return x; }
    __device__ static T enc(float x) { return x; }
};
template <> struct Codec<kF16> {
    using T = _Float16;
    __device__ static float dec(T x) { return static_cast<float>(x); }
    __device__ static T enc(float x) { return static_cast<_Float16>(x); }   // round to nearest even
};
template <> struct Codec<kBF16> {
    using T = uint16_t;
    __device__ static float dec(T x) { return __uint_as_float(uint32_t(x) << 16); }
    __device__ static T enc(float x) {                                     // round to nearest even
        const uint32_t b = __float_as_uint(x);
        return static_cast<T>((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
    }
};
// 8-bit fixed point: steps of 1/2, saturating at +-63.5 (127 steps).
template <> struct Codec<kQ8> {
    using T = int8_t;
    __device__ static float dec(T x) { return float(x) * 0.5f; }
    __device__ static T enc(float x) {                                     // round to nearest even, saturate
        return static_cast<T>(fminf(fmaxf(rintf(x * 2.f), -127.f), 127.f));
    }
};

// Storage of the posterior that the check pass gathers to form the bit->check
// messages Q = L - R_old (in a frame's first iteration it holds the channel
// LLRs, the messages of Algorithm 3).  With 16-bit messages it is kept at 16
// bits too (IEEE fp16, for fp16 and bf16 messages alike); otherwise fp32.  The fp16
// value is rounded so that its sign is that of the fp32 sum it came from: a
// negative sum that rounds to zero is stored as the smallest negative
// subnormal, and a zero sum of either sign as +0.  The hard decision
// (posterior < 0, Algorithm 6) is the same read from either copy.
template <int M> struct Post { using T = float; static constexpr int kMsg = kF32; };
template <> struct Post<kF16> { using T = _Float16; static constexpr int kMsg = kF16; };
template <> struct Post<kBF16> { using T = _Float16; static constexpr int kMsg = kF16; };
template <int M> constexpr bool kPost16 = Post<M>::kMsg == kF16;

template <typename T> struct CodecOf;
template <> struct CodecOf<float> { static constexpr int kMsg = kF32; };
template <> struct CodecOf<_Float16> { static constexpr int kMsg = kF16; };

__device__ __forceinline__ _Float16 post16_enc(float x) {
    uint16_t b = __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));   // round to nearest even
    if ((b & 0x7fffu) == 0u) b = x < 0.f ? uint16_t(0x8001u) : uint16_t(0u);
    return __builtin_bit_cast(_Float16, b);
}

// Device arrays by address space.  A pointer that reaches a kernel through
// memory (a table of per-graph arrays, a frame descriptor) is generic to the
// compiler, which then emits flat accesses; flat loads also count against the
// scalar/LDS wait counter, so a row's index loads end up waiting behind its
// message loads.  Every array here is in global memory: gmem() states that for
// data arrays, cload() reads an entry of a read-only table (graph indices) as
// constant memory, which uniform addresses turn into scalar loads.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ T cload(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <int B> struct Raw;
template <> struct Raw<1> { using T = uint8_t; };
template <> struct Raw<2> { using T = uint16_t; };
template <> struct Raw<4> { using T = uint32_t; };
template <> struct Raw<8> { using T = u32x2; };
template <> struct Raw<16> { using T = u32x4; };

template <int M, int V>
__device__ __forceinline__ void load_vec(const typename Codec<M>::T *p, float (&out)[V]) {
    using T = typename Codec<M>::T;
    using W = typename Raw<sizeof(T) * V>::T;
    const W raw = *gmem(reinterpret_cast<const W *>(p));
    T e[V];
    __builtin_memcpy(e, &raw, sizeof(W));
#pragma unroll
    for (int k = 0; k < V; k++) out[k] = Codec<M>::dec(e[k]);
}

template <int M, int V>
__device__ __forceinline__ void store_vec(typename Codec<M>::T *p, const float (&in)[V]) {
    using T = typename Codec<M>::T;
    using W = typename Raw<sizeof(T) * V>::T;
    T e[V];
#pragma unroll
    for (int k = 0; k < V; k++) e[k] = Codec<M>::enc(in[k]);
    W raw;
    __builtin_memcpy(&raw, e, sizeof(W));
    *gmem(reinterpret_cast<W *>(p)) = raw;
}

// Store a lane's V posterior values in the check pass's storage (Post).
template <int V, typename T>
__device__ __forceinline__ void store_post(T *p, const float (&in)[V]) {
    if constexpr (sizeof(T) == 4) {
        store_vec<kF32, V>(reinterpret_cast<float *>(p), in);
    } else {
        using W = typename Raw<2 * V>::T;
        _Float16 e[V];
#pragma unroll
        for (int k = 0; k < V; k++) e[k] = post16_enc(in[k]);
        W raw;
        __builtin_memcpy(&raw, e, sizeof(W));
        *gmem(reinterpret_cast<W *>(p)) = raw;
    }
}

template <typename T>
__device__ __forceinline__ void store_post1(T *p, float x) {
    if constexpr (sizeof(T) == 4) *gmem(p) = x;
    else *gmem(p) = post16_enc(x);
}

// Element s0 of row `row` as a base plus a 32-bit per-lane byte offset.  With
// UNIFORM (every lane of the wavefront on the same row) the base is read from
// lane 0 into scalar registers, so the access takes the scalar-base form:
// without it the compiler folds the lane offset into one 64-bit address per
// row and lane, two registers per edge that stay live from a message's load
// to its store.
template <bool UNIFORM, typename T>
__device__ __forceinline__ T *lane_elem(T *row, int s0) {
    using B = std::conditional_t<std::is_const_v<T>, const char, char>;
    B *base = reinterpret_cast<B *>(row);
    if constexpr (UNIFORM) {
        const uint64_t a = reinterpret_cast<uint64_t>(row);
        const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
        const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
        base = reinterpret_cast<B *>((uint64_t(hi) << 32) | lo);
    }
    return reinterpret_cast<T *>(base + uint32_t(s0) * uint32_t(sizeof(T)));
}

template <int V>
__device__ __forceinline__ void load_i32(const int32_t *p, int32_t (&out)[V]) {
    using W = typename Raw<4 * V>::T;
    const W raw = *gmem(reinterpret_cast<const W *>(p));
    __builtin_memcpy(out, &raw, sizeof(W));
}

template <int V>
__device__ __forceinline__ void store_i32(int32_t *p, const int32_t (&in)[V]) {
    using W = typename Raw<4 * V>::T;
    W raw;
    __builtin_memcpy(&raw, in, sizeof(W));
    *gmem(reinterpret_cast<W *>(p)) = raw;
}

// -------------------------------------------------------------- check math

// u = 1 - tanh(x/2) = 2 / (1 + e^x) = 1 / ((1 + 2^y)/2) with y = x log2(e), for
// 0 <= x = |Q| <= LMAX, the argument given as y (2^(64 log2 e) is a normal fp32
// number; the halved denominator is one fma).
__device__ __forceinline__ float tanh_complement_b2(float y) {
    return __builtin_amdgcn_rcpf(fmaf(0.5f, __builtin_amdgcn_exp2f(y), 0.5f));
}

// Complement of a product of complements: 1 - (1-a)(1-b) = a + b(1-a).
__device__ __forceinline__ float dplus(float a, float b) { return fmaf(b, 1.f - a, a); }

// |R| log2(e) = 2 atanh(1 - D) log2(e) = log2((2 - D)/D) = log2(2/D - 1); D = 0
// (empty product) gives +inf, which the caller clamps.  For 0 < D <= 1 the
// ratio is >= 1, so the one rounding of 2/D - 1 in the fma adds no cancellation.
__device__ __forceinline__ float magnitude_from_complement_b2(float D) {
    return __builtin_amdgcn_logf(fmaf(2.f, __builtin_amdgcn_rcpf(D), -1.f));
}

// Q clamped to [-LMAX, LMAX] (one v_med3; Q is never NaN).
__device__ __forceinline__ float clamp_msg(float q) { return __builtin_amdgcn_fmed3f(q, -kLmax, kLmax); }

// Signs travel in the sign bit of the rule inputs: u carries the sign of its
// Q, the row's sign parity is bit 31 of the XOR of the Q words (the other bits
// of that word are never read), and an output magnitude (>= 0) takes its sign
// from bit 31 of a word.  The values a check pass
// reads never hold -0 (channel LLRs are stored with -0 replaced by +0, and
// sums and differences of such values round exact zeros to +0), so the sign
// bit of Q is exactly Q < 0, the sign Algorithm 1 uses (sgn(0) = +1).
// (FP16 messages: one bit-field insert; the other formats OR the masked sign
// bit in, which keeps their kernels within their register budget.)
template <int M>
__device__ __forceinline__ float signed_mag(float mag, uint32_t sign) {
    if constexpr (M == kF16) return copysignf(mag, __uint_as_float(sign));
    else return __uint_as_float(__float_as_uint(mag) | (sign & 0x80000000u));
}
// A channel LLR as the check and bit passes store it: -0 becomes +0.
__device__ __forceinline__ float canon_llr(float x) { return x + 0.f; }

// Check-node rules.  Every rule takes the sign of R from the other inputs' sign
// product and its magnitude from an aggregate of the other inputs, formed with
// an associative operation (exclusive prefix/suffix combinations, never "total
// minus own"):
//   kRuleSP   sum-product (Algorithm 1): input u = 1 - tanh(|Q|/2), aggregate
//             D = 1 - prod(1 - u), |R| = ln((2 - D)/D);
//   kRuleNMS  normalized Min-Sum: aggregate min |Q|, |R| = alpha * min
//             (alpha = 1: plain Min-Sum);
//   kRuleOMS  offset Min-Sum: aggregate min |Q|, |R| = max(min - beta, 0);
// the derived decoders Section 3.1 names for the edge-level approach (after
// Wu, Song, Jiang and Zhao, IEEE Commun. Lett. 14(7), 2010).  |R| is clamped to
// LMAX; an empty aggregate (degree-1 check) gives LMAX under every rule.
enum RuleKind { kRuleSP = 0, kRuleNMS = 1, kRuleOMS = 2 };

template <int RULE> struct CheckRule;

// Sum-product works on LLRs in base-2 units (|Q| log2 e in, |R| log2 e out):
// the hardware's transcendentals are exp2 and log2.  See MsgUnits for where
// the scaling happens.
template <> struct CheckRule<kRuleSP> {
    static __device__ __forceinline__ float identity() { return 0.f; }
    static __device__ __forceinline__ float input(float qa2) { return tanh_complement_b2(qa2); }
    static __device__ __forceinline__ float combine(float a, float b) { return dplus(a, b); }
    static __device__ __forceinline__ float magnitude_b2(float agg) { return magnitude_from_complement_b2(agg); }
};

template <> struct CheckRule<kRuleNMS> {
    static __device__ __forceinline__ float identity() { return __builtin_inff(); }
    static __device__ __forceinline__ float input(float qa) { return qa; }
    static __device__ __forceinline__ float combine(float a, float b) { return fminf(a, b); }
    static __device__ __forceinline__ float magnitude(float m, float alpha) { return fminf(alpha * m, kLmax); }
};

template <> struct CheckRule<kRuleOMS> {
    static __device__ __forceinline__ float identity() { return __builtin_inff(); }
    static __device__ __forceinline__ float input(float qa) { return qa; }
    static __device__ __forceinline__ float combine(float a, float b) { return fminf(a, b); }
    static __device__ __forceinline__ float magnitude(float m, float beta) {
        return fminf(fmaxf(m - beta, 0.f), kLmax);
    }
};

// Units of the stored messages.  With the sum-product rule and FP16 or BF16
// storage a message is stored as R log2(e): the check pass then forms the
// rule's input Q log2(e) = L log2(e) - R log2(e) with one fma and stores the
// rule's output as it comes, and the bit pass adds ln(2) times the sum of a
// bit's messages to its channel LLR.  Posteriors and channel LLRs stay in
// natural units.  FP32 messages (whose check pass is bound by memory, not by
// its arithmetic), 8-bit fixed-point messages (steps of 1/2) and the Min-Sum
// rules store R itself, and the sum-product rule scales on the way in and
// out.  LMAX bounds |Q| and |R| in natural units either way.
template <int M, int RULE>
struct MsgUnits {
    static constexpr bool kRuleB2 = RULE == kRuleSP;                              // base-2 rule magnitudes
    static constexpr bool kStoredB2 = kRuleB2 && (M == kF16 || M == kBF16);      // base-2 stored messages
    static constexpr float kLim = kStoredB2 ? kLmax * kLog2e : kLmax;   // |Q|, |R| bound in stored units
    // factor of the sum of a bit's messages in its posterior
    static constexpr float kBitScale = kStoredB2 ? kLn2 : 1.f;
};

// Q (clamped, in stored units) from a posterior L and a stored message R.
template <int M, int RULE>
__device__ __forceinline__ float rule_q(float L, float R) {
    using U = MsgUnits<M, RULE>;
    if constexpr (U::kStoredB2) return __builtin_amdgcn_fmed3f(fmaf(L, kLog2e, -R), -U::kLim, U::kLim);
    else return clamp_msg(L - R);
}

// The rule's input from |Q| in stored units.
template <int M, int RULE>
__device__ __forceinline__ float rule_in(float qa) {
    using U = MsgUnits<M, RULE>;
    if constexpr (U::kStoredB2) return CheckRule<RULE>::input(qa);
    else if constexpr (U::kRuleB2) return CheckRule<RULE>::input(qa * kLog2e);
    else return CheckRule<RULE>::input(qa);
}

// The stored magnitude of an outgoing message from the rule's aggregate.
template <int M, int RULE>
__device__ __forceinline__ float rule_mag(float agg, float rp) {
    using U = MsgUnits<M, RULE>;
    if constexpr (U::kStoredB2) return fminf(CheckRule<RULE>::magnitude_b2(agg), U::kLim);
    else if constexpr (U::kRuleB2) return fminf(CheckRule<RULE>::magnitude_b2(agg) * kLn2, kLmax);
    else return CheckRule<RULE>::magnitude(agg, rp);
}

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }


// ----------------------------------------------------------- row building blocks

// Where a check pass takes each edge's inputs (a compile-time choice, so the
// common case carries no per-slot selection):
//   kInFirst   first iteration of every slot: L is the channel array and every
//              previous message is 0 (Algorithm 3's q = p);
//   kInSteady  every slot past its first iteration: L is the posterior, R_old
//              is read;
//   kInMixed   as kInSteady, except slots with SlotSrc::alt set, which are in
//              their first iteration: their previous messages count as 0 (the
//              caller has placed the channel LLRs in their posterior entries),
//              so the common case pays one branch per lane (SlotSrc::any).
enum Inputs { kInFirst = 0, kInSteady = 1, kInMixed = 2 };

// Whether a row's message and posterior accesses take scalar bases
// (lane_elem).  The engine's 8-bit rows (first-iteration slots mixed in) need
// more registers with them than without, so they keep per-lane addresses.
template <int M, bool UNIFORM, int IN>
constexpr bool scalar_base() { return UNIFORM && !(M == kQ8 && IN == kInMixed); }

template <int V>
struct SlotSrc {
    bool alt[V];
    bool any;   // some alt[k] is set
};

// L * a - R for fp16 L and R held as halves of 32-bit words (half 0: bits
// 0-15, half 1: bits 16-31) and an fp32 factor a: one mixed-precision fma
// converts both halves to fp32 on the fly and rounds the result once.
template <int HALF>
__device__ __forceinline__ float fma_f16_halves(uint32_t l, float a, uint32_t r) {
    float q;
    if constexpr (HALF == 0)
        asm("v_fma_mix_f32 %0, %1, %2, -%3 op_sel_hi:[1,0,1]" : "=v"(q) : "v"(l), "s"(a), "v"(r));
    else
        asm("v_fma_mix_f32 %0, %1, %2, -%3 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(q) : "v"(l), "s"(a), "v"(r));
    return q;
}

// rule_q for fp16 posteriors and messages held as word halves.
template <int HALF, int RULE>
__device__ __forceinline__ float rule_q_f16_halves(uint32_t l, uint32_t r) {
    using U = MsgUnits<kF16, RULE>;
    return __builtin_amdgcn_fmed3f(fma_f16_halves<HALF>(l, U::kStoredB2 ? kLog2e : 1.f, r), -U::kLim, U::kLim);
}

// Column index of a check-sorted edge position: read from the column table,
// or, for a row of a quasi-cyclic code, computed from its base row.  Edge
// e0 + k of check i*Z + t joins bit J_k + ((t + s_k) mod Z), where (J_k = j_k Z,
// s_k) is the k-th entry of base row i (the graph keeps base-column order).
struct QcCols {
    const int32_t *ent;   // (J, s) pairs of the row's base row
    int32_t e0, t, Z;     // first edge of the row, its offset in the block, lifting size
};
template <bool UNIFORM>
__device__ __forceinline__ int col_at(const int32_t *col_idx, int e) {
    return UNIFORM ? wave_uniform(cload(col_idx + e)) : cload(col_idx + e);
}
template <bool UNIFORM>
__device__ __forceinline__ int col_at(const QcCols &q, int e) {
    const int k = e - q.e0;
    const int u = q.t + cload(q.ent + 2 * k + 1);
    return cload(q.ent + 2 * k) + (u >= q.Z ? u - q.Z : u);
}

// Inputs of edges j0 .. j0+count-1 (1 <= count <= C) for the lane's slots:
// Q = clamp(L - R_old) and the rule's input u (1 - tanh(|Q|/2) for
// sum-product, |Q| for Min-Sum) carrying the sign of Q in its sign bit; the
// XOR of those sign bits goes into par (bit 31);
// the sign of L feeds the syndrome of the estimate that L holds (Algorithm 7).
// Every index load and then every message load is issued before any value is
// used: positions past `count` repeat the last edge (same addresses, no
// branch), so the loads of a row are in flight together instead of one edge
// at a time.  UNIFORM: all lanes walk the same row (indices read once per
// wavefront).
template <int M, int V, int C, bool UNIFORM, int IN, int RULE = kRuleSP, typename LT, typename CI>
__device__ __forceinline__ void gather_edges(CI col_idx, int j0, int count,
                                             const LT *__restrict__ L,
                                             const typename Codec<M>::T *__restrict__ R, int32_t S, int s0,
                                             const SlotSrc<V> &src, float (&u)[C][V], uint32_t (&par)[V],
                                             int (&syn)[V]) {
    constexpr bool SB = scalar_base<M, UNIFORM, IN>();
    int vix[C];
#pragma unroll
    for (int j = 0; j < C; j++) {
        const int e = j0 + (j < count ? j : count - 1);
        vix[j] = col_at<UNIFORM>(col_idx, e);
    }
    if constexpr (M == kF16 && CodecOf<LT>::kMsg == kF16 && V % 2 == 0) {
        // fp16 posterior and messages: the words as loaded, two slots each
        constexpr int W = V / 2;
        uint32_t lw[C][W], rw[C][W];
#pragma unroll
        for (int j = 0; j < C; j++) {
            const int e = j0 + (j < count ? j : count - 1);
            using RawW = typename Raw<4 * W>::T;
            const RawW a = *gmem(reinterpret_cast<const RawW *>(lane_elem<SB>(L + size_t(vix[j]) * S, s0)));
            __builtin_memcpy(lw[j], &a, sizeof(RawW));
            if (IN != kInFirst) {
                const RawW b = *gmem(reinterpret_cast<const RawW *>(lane_elem<SB>(R + size_t(e) * S, s0)));
                __builtin_memcpy(rw[j], &b, sizeof(RawW));
            } else {
#pragma unroll
                for (int w = 0; w < W; w++) rw[j][w] = 0u;
            }
        }
        if (IN == kInMixed && src.any) {
            uint32_t keep[W];   // first-iteration slots: previous message 0
#pragma unroll
            for (int w = 0; w < W; w++)
                keep[w] = (src.alt[2 * w] ? 0u : 0x0000ffffu) | (src.alt[2 * w + 1] ? 0u : 0xffff0000u);
#pragma unroll
            for (int j = 0; j < C; j++) {
#pragma unroll
                for (int w = 0; w < W; w++) rw[j][w] &= keep[w];
            }
        }
        uint32_t sw[W];   // syndrome: XOR of the posterior words (stored signs are the decisions)
#pragma unroll
        for (int w = 0; w < W; w++) sw[w] = 0u;
#pragma unroll
        for (int j = 0; j < C; j++) {
            if (j < count) {
#pragma unroll
                for (int w = 0; w < W; w++) {
                    sw[w] ^= lw[j][w];
                    const float q0 = rule_q_f16_halves<0, RULE>(lw[j][w], rw[j][w]);
                    const float q1 = rule_q_f16_halves<1, RULE>(lw[j][w], rw[j][w]);
                    par[2 * w] ^= __float_as_uint(q0);
                    par[2 * w + 1] ^= __float_as_uint(q1);
                    u[j][2 * w] = copysignf(rule_in<M, RULE>(fabsf(q0)), q0);
                    u[j][2 * w + 1] = copysignf(rule_in<M, RULE>(fabsf(q1)), q1);
                }
            }
        }
#pragma unroll
        for (int w = 0; w < W; w++) {
            syn[2 * w] ^= int((sw[w] >> 15) & 1u);
            syn[2 * w + 1] ^= int(sw[w] >> 31);
        }
        return;
    }
    float lv[C][V], r[C][V];
#pragma unroll
    for (int j = 0; j < C; j++) {
        const int e = j0 + (j < count ? j : count - 1);
        load_vec<CodecOf<LT>::kMsg, V>(lane_elem<SB>(L + size_t(vix[j]) * S, s0), lv[j]);
        if (IN != kInFirst) {
            load_vec<M, V>(lane_elem<SB>(R + size_t(e) * S, s0), r[j]);
        } else {
#pragma unroll
            for (int k = 0; k < V; k++) r[j][k] = 0.f;
        }
    }
    if (IN == kInMixed && src.any) {
#pragma unroll
        for (int j = 0; j < C; j++) {
#pragma unroll
            for (int k = 0; k < V; k++)
                if (src.alt[k]) r[j][k] = 0.f;
        }
    }
#pragma unroll
    for (int j = 0; j < C; j++) {
        if (j < count) {
#pragma unroll
            for (int k = 0; k < V; k++) {
                syn[k] ^= (lv[j][k] < 0.f);
                const float q = rule_q<M, RULE>(lv[j][k], r[j][k]);
                // bit 31 only: keeping whole words here costs the FP32 kernels registers
                const uint32_t sq = __float_as_uint(q) & 0x80000000u;
                par[k] ^= sq;
                u[j][k] = __uint_as_float(__float_as_uint(rule_in<M, RULE>(fabsf(q))) | sq);
            }
        }
    }
}

// Check rule for a whole row of d <= DMAX edges held in registers: exclusive
// suffixes, then exclusive prefixes combined on the fly; R is updated in place.
// UNIFORM: every lane of the wavefront works on the same row (indices are read
// once per wavefront); otherwise each lane walks its own row.
template <int M, int V, int DMAX, bool UNIFORM, int IN, int RULE = kRuleSP, typename LT, typename CI>
__device__ __forceinline__ void row_rule_n(CI col_idx, int e0, int d,
                                         const LT *__restrict__ L,
                                         typename Codec<M>::T *__restrict__ R, int32_t S, int s0,
                                         const SlotSrc<V> &src, int (&syn)[V], float rp = 0.f) {
    using Rule = CheckRule<RULE>;
    float u[DMAX][V];
    float suf[DMAX][V];
    uint32_t par[V];
#pragma unroll
    for (int k = 0; k < V; k++) par[k] = 0u;
    gather_edges<M, V, DMAX, UNIFORM, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, u, par, syn);
    float run[V];
#pragma unroll
    for (int k = 0; k < V; k++) run[k] = Rule::identity();
#pragma unroll
    for (int j = DMAX - 1; j >= 0; j--) {
        if (j < d) {
#pragma unroll
            for (int k = 0; k < V; k++) {
                suf[j][k] = run[k];
                run[k] = Rule::combine(fabsf(u[j][k]), run[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < V; k++) run[k] = Rule::identity();
#pragma unroll
    for (int j = 0; j < DMAX; j++) {
        if (j < d) {
            float out[V];
#pragma unroll
            for (int k = 0; k < V; k++) {
                const float mag = rule_mag<M, RULE>(Rule::combine(run[k], suf[j][k]), rp);
                out[k] = signed_mag<M>(mag, par[k] ^ __float_as_uint(u[j][k]));   // sign of the other inputs
                run[k] = Rule::combine(run[k], fabsf(u[j][k]));
            }
            store_vec<M, V>(lane_elem<scalar_base<M, UNIFORM, IN>()>(R + size_t(e0 + j) * S, s0), out);
        }
    }
}

// row_rule_n with the degree as a compile-time constant when every lane works
// on the same row of at most 8 edges: the row's code is then straight-line
// (no per-position test of the degree).  Other rows take the generic form.
template <int M, int V, int D, bool UNIFORM, int IN, int RULE, typename LT, typename CI>
__device__ __forceinline__ bool row_rule_fixed(CI col_idx, int e0, int d,
                                               const LT *__restrict__ L, typename Codec<M>::T *__restrict__ R,
                                               int32_t S, int s0, const SlotSrc<V> &src, int (&syn)[V], float rp) {
    if (d != D) return false;
    row_rule_n<M, V, D, UNIFORM, IN, RULE>(col_idx, e0, D, L, R, S, s0, src, syn, rp);
    return true;
}

template <int M, int V, int DMAX, bool UNIFORM, int IN, int RULE = kRuleSP, typename LT, typename CI>
__device__ __forceinline__ void row_rule(CI col_idx, int e0, int d,
                                         const LT *__restrict__ L,
                                         typename Codec<M>::T *__restrict__ R, int32_t S, int s0,
                                         const SlotSrc<V> &src, int (&syn)[V], float rp = 0.f) {
    if constexpr (UNIFORM && DMAX == 8) {
        if (row_rule_fixed<M, V, 8, UNIFORM, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, syn, rp) ||
            row_rule_fixed<M, V, 7, UNIFORM, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, syn, rp) ||
            row_rule_fixed<M, V, 6, UNIFORM, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, syn, rp) ||
            row_rule_fixed<M, V, 5, UNIFORM, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, syn, rp) ||
            row_rule_fixed<M, V, 4, UNIFORM, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, syn, rp) ||
            row_rule_fixed<M, V, 3, UNIFORM, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, syn, rp))
            return;
    }
    row_rule_n<M, V, DMAX, UNIFORM, IN, RULE>(col_idx, e0, d, L, R, S, s0, src, syn, rp);
}

// Posterior sum Lch + sum of the bit's incoming messages, added in column
// order (positions a .. b-1 of the bit-sorted edge list, mapped to message
// rows by csc_to_csr).  Edges are fetched four at a time with all their loads
// in flight; positions past b repeat the last edge and are not added.
constexpr int kBitBatch = 4;

template <int M, int V, bool UNIFORM>
__device__ __forceinline__ void bit_sum(const int32_t *__restrict__ csc_to_csr, int a, int b,
                                        const typename Codec<M>::T *__restrict__ R, int32_t S, int s0,
                                        float (&sum)[V]) {
    for (int k0 = a; k0 < b; k0 += kBitBatch) {
        int e[kBitBatch];
#pragma unroll
        for (int j = 0; j < kBitBatch; j++) {
            const int k = k0 + j < b ? k0 + j : b - 1;
            e[j] = UNIFORM ? wave_uniform(cload(csc_to_csr + k)) : cload(csc_to_csr + k);
        }
        float r[kBitBatch][V];
#pragma unroll
        for (int j = 0; j < kBitBatch; j++) load_vec<M, V>(R + size_t(e[j]) * S + s0, r[j]);
#pragma unroll
        for (int j = 0; j < kBitBatch; j++) {
            if (k0 + j < b) {
#pragma unroll
                for (int z = 0; z < V; z++) sum[z] += r[j][z];
            }
        }
    }
}

// Posterior of a bit from its channel LLRs (row `lch` of the [n][S] array):
// scale 1 adds the bit's messages to Lch in column order; any other scale
// (base-2 messages) sums the messages first and adds scale times the sum to
// Lch with one fma.  The branch is uniform over the wavefront.
template <int M, int V, bool UNIFORM>
__device__ __forceinline__ void bit_posterior(const int32_t *__restrict__ csc_to_csr, int a, int b,
                                              const typename Codec<M>::T *__restrict__ R, int32_t S, int s0,
                                              const float *__restrict__ lch, float scale, float (&sum)[V]) {
    float l[V];
    load_vec<kF32, V>(lch + s0, l);
    if (scale == 1.f) {
#pragma unroll
        for (int k = 0; k < V; k++) sum[k] = l[k];
        bit_sum<M, V, UNIFORM>(csc_to_csr, a, b, R, S, s0, sum);
    } else {
#pragma unroll
        for (int k = 0; k < V; k++) sum[k] = 0.f;
        bit_sum<M, V, UNIFORM>(csc_to_csr, a, b, R, S, s0, sum);
#pragma unroll
        for (int k = 0; k < V; k++) sum[k] = fmaf(scale, sum[k], l[k]);
    }
}

// Chunked rows: a row is cut into chunks of C edges handled by different
// wavefronts.  chunk_load forms a chunk's u's, exclusive in-chunk suffixes and
// its aggregate (the u's combined), sign bits and syndrome parity;
// chunk_store finishes the chunk given the aggregate of the chunks before it
// (pre), of the chunks after it (post) and the row's total sign parity.
constexpr int kRowChunk = 8;

template <int M, int V, int C, int IN, int RULE = kRuleSP, typename LT>
__device__ __forceinline__ void chunk_load(const int32_t *__restrict__ col_idx, int j0, int dc,
                                           const LT *__restrict__ L,
                                           const typename Codec<M>::T *__restrict__ R, int32_t S, int s0,
                                           const SlotSrc<V> &src, float (&u)[C][V], float (&suf)[C][V],
                                           float (&agg)[V], uint32_t (&par)[V], int (&syn)[V]) {
#pragma unroll
    for (int k = 0; k < V; k++) { par[k] = 0u; syn[k] = 0; }
    gather_edges<M, V, C, true, IN, RULE>(col_idx, j0, dc, L, R, S, s0, src, u, par, syn);
#pragma unroll
    for (int k = 0; k < V; k++) agg[k] = CheckRule<RULE>::identity();
#pragma unroll
    for (int j = C - 1; j >= 0; j--) {
        if (j < dc) {
#pragma unroll
            for (int k = 0; k < V; k++) {
                suf[j][k] = agg[k];
                agg[k] = CheckRule<RULE>::combine(fabsf(u[j][k]), agg[k]);
            }
        }
    }
}

template <int M, int V, int C, int RULE = kRuleSP>
__device__ __forceinline__ void chunk_store(int j0, int dc, const float (&u)[C][V], const float (&suf)[C][V],
                                            const float (&pre)[V], const float (&post)[V],
                                            const uint32_t (&parity)[V], typename Codec<M>::T *__restrict__ R,
                                            int32_t S, int s0, float rp = 0.f) {
    using Rule = CheckRule<RULE>;
    float run[V];
#pragma unroll
    for (int k = 0; k < V; k++) run[k] = pre[k];
#pragma unroll
    for (int j = 0; j < C; j++) {
        if (j < dc) {
            float out[V];
#pragma unroll
            for (int k = 0; k < V; k++) {
                const float mag = rule_mag<M, RULE>(Rule::combine(run[k], Rule::combine(suf[j][k], post[k])), rp);
                out[k] = signed_mag<M>(mag, (parity[k] << 31) ^ __float_as_uint(u[j][k]));
                run[k] = Rule::combine(run[k], fabsf(u[j][k]));
            }
            store_vec<M, V>(R + size_t(j0 + j) * S + s0, out);
        }
    }
}

// Chunk aggregates of one row exchanged through LDS: each entry is a lane's
// V aggregates plus packed sign parities (bits 0..V-1) and syndrome parities
// (bits 8..8+V-1).
template <int V, int ENTRIES>
struct ChunkShare {
    float agg[ENTRIES][64][V];
    uint32_t bits[ENTRIES][64];
};

template <int V>
__device__ __forceinline__ uint32_t pack_bits(const uint32_t (&par)[V], const int (&syn)[V]) {
    uint32_t b = 0u;
#pragma unroll
    for (int k = 0; k < V; k++) b |= ((par[k] >> 31) << k) | (uint32_t(syn[k] & 1) << (8 + k));
    return b;
}

// pre/post aggregates and total parities of chunk `ch` of a row of nch chunks
// whose entries start at `base` in the shared table.
template <int V, int ENTRIES, int RULE = kRuleSP>
__device__ __forceinline__ void chunk_context(const ChunkShare<V, ENTRIES> &sh, int base, int nch, int ch, int lane,
                                              float (&pre)[V], float (&post)[V], uint32_t (&parity)[V],
                                              int (&syn)[V]) {
    using Rule = CheckRule<RULE>;
    uint32_t tot = 0u;
#pragma unroll
    for (int k = 0; k < V; k++) { pre[k] = Rule::identity(); post[k] = Rule::identity(); }
    for (int c = 0; c < nch; c++) {
        tot ^= sh.bits[base + c][lane];
        if (c < ch) {
#pragma unroll
            for (int k = 0; k < V; k++) pre[k] = Rule::combine(pre[k], sh.agg[base + c][lane][k]);
        }
    }
    for (int c = nch - 1; c > ch; c--) {
#pragma unroll
        for (int k = 0; k < V; k++) post[k] = Rule::combine(sh.agg[base + c][lane][k], post[k]);
    }
#pragma unroll
    for (int k = 0; k < V; k++) { parity[k] = (tot >> k) & 1u; syn[k] = int((tot >> (8 + k)) & 1u); }
}

// Rows of up to kWideWaves chunks of C edges on one workgroup of kWideWaves
// wavefronts, one chunk each, for one 64-slot group at one slot per lane: the
// chunk aggregates, sign parities and syndrome parities go through LDS, and
// each wavefront finishes its chunk from the inputs it still holds, so every
// input is read once.  Every wavefront of the workgroup must call it (it
// synchronises the workgroup).  Returns the row's syndrome parity for the
// lane (meaningful in wavefronts wv < number of chunks).
constexpr int kWideWaves = 16;
constexpr int kWideChunk = 32;   // edges per wavefront: rows of up to 512 edges

template <int M, int C, int IN, int RULE, typename LT>
__device__ __forceinline__ bool wide_row(const int32_t *__restrict__ col_idx, int e0, int d,
                                         const LT *__restrict__ L, typename Codec<M>::T *__restrict__ R, int32_t S,
                                         int s, const SlotSrc<1> &src, bool active, ChunkShare<1, kWideWaves> &sh,
                                         int wv, int lane, float rp) {
    using Rule = CheckRule<RULE>;
    const int nch = (d + C - 1) / C;
    const int dc = min(C, d - wv * C);
    float u[C][1], suf[C][1], agg[1];
    uint32_t par[1];
    int syn[1];
    const bool mine = wv < nch && active;
    if (mine) {
        chunk_load<M, 1, C, IN, RULE>(col_idx, e0 + wv * C, dc, L, R, S, s, src, u, suf, agg, par, syn);
    } else {
        agg[0] = Rule::identity();
        par[0] = 0u;
        syn[0] = 0;
    }
    if (wv < nch) {
        sh.agg[wv][lane][0] = agg[0];
        sh.bits[wv][lane] = pack_bits<1>(par, syn);
    }
    __syncthreads();
    int syn_row[1] = {0};
    if (mine) {
        float pre[1], post[1];
        uint32_t parity[1];
        chunk_context<1, kWideWaves, RULE>(sh, 0, nch, wv, lane, pre, post, parity, syn_row);
        chunk_store<M, 1, C, RULE>(e0 + wv * C, dc, u, suf, pre, post, parity, R, S, s, rp);
    }
    return syn_row[0] != 0;
}

}  // namespace ldpc_dev
