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

namespace ldpc_dev {

constexpr float kLmax = 64.f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr int32_t kPadSlot = 0x7fffffff;   // iters value of a padding slot: never active

enum MsgType { kF32 = 0, kF16 = 1, kBF16 = 2 };
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

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <int B> struct Raw;
template <> struct Raw<2> { using T = uint16_t; };
template <> struct Raw<4> { using T = uint32_t; };
template <> struct Raw<8> { using T = u32x2; };
template <> struct Raw<16> { using T = u32x4; };

template <int M, int V>
__device__ __forceinline__ void load_vec(const typename Codec<M>::T *p, float (&out)[V]) {
    using T = typename Codec<M>::T;
    using W = typename Raw<sizeof(T) * V>::T;
    const W raw = *reinterpret_cast<const W *>(p);
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
    *reinterpret_cast<W *>(p) = raw;
}

template <int V>
__device__ __forceinline__ void load_i32(const int32_t *p, int32_t (&out)[V]) {
    using W = typename Raw<4 * V>::T;
    const W raw = *reinterpret_cast<const W *>(p);
    __builtin_memcpy(out, &raw, sizeof(W));
}

// -------------------------------------------------------------- check math

// u = 1 - tanh(x/2) = 2w/(1+w) with w = e^-x, for x = |Q| >= 0.
__device__ __forceinline__ float tanh_complement(float x) {
    const float w = __builtin_amdgcn_exp2f(-x * kLog2e);
    return 2.f * w * __builtin_amdgcn_rcpf(1.f + w);
}

// Complement of a product of complements: 1 - (1-a)(1-b) = a + b(1-a).
__device__ __forceinline__ float dplus(float a, float b) { return fmaf(b, 1.f - a, a); }

// |R| = 2 atanh(1 - D) = ln((2 - D)/D), clamped to LMAX; D = 0 (empty product) gives LMAX.
__device__ __forceinline__ float magnitude_from_complement(float D) {
    const float ratio = (2.f - D) * __builtin_amdgcn_rcpf(D);
    return fminf(__builtin_amdgcn_logf(ratio) * kLn2, kLmax);
}

__device__ __forceinline__ float clamp_msg(float q) { return fminf(fmaxf(q, -kLmax), kLmax); }

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

}  // namespace ldpc_dev
