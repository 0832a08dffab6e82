// Device helpers shared by the evaluation kernels: the absorption kernel and level bookkeeping.
#pragma once

#include <hip/hip_runtime.h>

#include "ph_internal.h"

namespace ph {

// K(r) = g(r) / (4 pi r^2), g of Sec. 2.1 eq. (3):
//   K(r) = exp(-a r) (1 - exp(-(b - a) r)) / (4 pi L r^3),  a = chi_min pO2, b = chi_max pO2.
template <class T>
struct KParams {
    T a, bma, inv4piL;   // a, b - a, 1 / (4 pi L)
    T na_l2, nbma_l2;    // -a log2(e), -(b - a) log2(e) for the exp2 form
};

template <class T>
inline KParams<T> make_kparams(const Gas &g)
{
    const double log2e = 1.4426950408889634;
    KParams<T> k;
    k.a = (T)g.a;
    k.bma = (T)(g.b - g.a);
    k.inv4piL = (T)(1.0 / (4.0 * M_PI * g.L));
    k.na_l2 = (T)(-g.a * log2e);
    k.nbma_l2 = (T)(-(g.b - g.a) * log2e);
    return k;
}

// FP32: hardware rsqrt and exp2.  1 - exp(-t) loses relative accuracy for small t,
// so below t = 1/4 it is summed as the alternating Taylor series (truncation < 4e-10).
// NEAR selects that guarded form; far-field callers (t >= 1 by construction) may skip it.
template <bool NEAR>
__device__ __forceinline__ float kernel_eval(float r2, const KParams<float> &k)
{
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * rinv;
    const float e1 = __builtin_amdgcn_exp2f(k.na_l2 * r);
    float om = 1.0f - __builtin_amdgcn_exp2f(k.nbma_l2 * r);
    if (NEAR) {
        const float t = k.bma * r;
        // t (1 - t/2 (1 - t/3 (1 - t/4 (1 - t/5 (1 - t/6 (1 - t/7))))))
        float s = 1.0f - t * (1.0f / 7.0f);
        s = 1.0f - t * (1.0f / 6.0f) * s;
        s = 1.0f - t * (1.0f / 5.0f) * s;
        s = 1.0f - t * (1.0f / 4.0f) * s;
        s = 1.0f - t * (1.0f / 3.0f) * s;
        s = 1.0f - t * 0.5f * s;
        om = (t < 0.25f) ? t * s : om;
    }
    return e1 * om * (rinv * rinv * rinv) * k.inv4piL;
}

template <bool NEAR>
__device__ __forceinline__ double kernel_eval(double r2, const KParams<double> &k)
{
    const double r = sqrt(r2);
    return exp(-k.a * r) * (-expm1(-k.bma * r)) * k.inv4piL / (r2 * r);
}

template <class T>
struct Vec4T;
template <>
struct Vec4T<float> {
    using type = float4;
};
template <>
struct Vec4T<double> {
    using type = double4;
};

struct LevelTable {
    int32_t base[kMaxDepth + 2];
    int32_t cap[kMaxDepth + 2];
    double hw[kMaxDepth + 2];
    int32_t depth;
};

inline LevelTable make_level_table(const Plan &p)
{
    LevelTable t{};
    for (int l = 0; l <= p.max_depth; ++l) {
        t.base[l] = (int32_t)p.level_base[l];
        t.cap[l] = (int32_t)p.level_cap[l];
        t.hw[l] = p.hw[l];
    }
    t.base[p.max_depth + 1] = (int32_t)p.level_base[p.max_depth + 1];
    t.depth = p.max_depth;
    return t;
}

// Box b is live if it lies in its level's slot range below that level's count.
__device__ __forceinline__ bool box_live(const LevelTable &lt, const CallScalars *sc, int32_t b, int &level)
{
    for (int l = 0; l <= lt.depth; ++l) {
        const int32_t i = b - lt.base[l];
        if (i >= 0 && i < lt.cap[l]) {
            level = l;
            return i < sc->lvl_count[l];
        }
    }
    return false;
}

// Index of a well-separated offset t in [-3,3]^3 minus [-1,1]^3, in x-major order (0..315).
__host__ __device__ __forceinline__ int m2l_slot(int dx, int dy, int dz)
{
    const int X = dx + 3, Y = dy + 3, Z = dz + 3;
    const int full = X * 49 + Y * 7 + Z;
    auto inner_before = [](int v) { return v < 2 ? 0 : (v > 4 ? 3 : v - 2); };
    const bool xin = X >= 2 && X <= 4, yin = Y >= 2 && Y <= 4;
    const int skipped = inner_before(X) * 9 + (xin ? (inner_before(Y) * 3 + (yin ? inner_before(Z) : 0)) : 0);
    return full - skipped;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;

// v_mfma_f32_16x16x4_f32: A lane l = A[l%16][l/16], B lane l = B[l/16][l%16],
// D register r of lane l = D[4 (l/16) + r][l%16]
template <>
struct Mfma<float> {
    using acc_t = f32x4;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// v_mfma_f64_16x16x4_f64: same operand layout, D register r of lane l = D[(l/16) + 4 r][l%16]
template <>
struct Mfma<double> {
    using acc_t = f64x4;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};

// Start of a call, by workgroup 0 of the call's first kernel (no other kernel of the call has
// run yet, and no other workgroup of that kernel touches the scalars): clear the call's
// scalars and, with gen, advance the call number kept on the device and store it in sc.
// Append val to list for the lanes with pred: one atomic per wave, lanes in lane order.
template <class V>
__device__ __forceinline__ void wave_append(bool pred, V *__restrict__ list, int32_t *counter, V val)
{
    const uint64_t m = __ballot(pred);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, leader);
    if (pred) list[base + __popcll(m & ((1ull << lane) - 1ull))] = val;
}

__device__ __forceinline__ void begin_call(CallScalars *sc, int32_t *gen)
{
    int32_t *w = reinterpret_cast<int32_t *>(sc);
    for (int i = threadIdx.x; i < (int)(sizeof(CallScalars) / 4); i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0 && gen) {
        int32_t g = *gen + 1;
        if (g <= 0) g = 1;
        *gen = g;
        sc->gen = g;
    }
}

// An error of the call: in the call's scalars (read by a call that fetches its statistics) and in
// the plan's sticky word (read and cleared by the next check, whatever calls came in between).
__device__ __forceinline__ void flag_error(CallScalars *sc, int32_t *sticky, int bits)
{
    atomicOr(&sc->err, bits);
    if (sticky) atomicOr(sticky, bits);
}

// The list range (begin, begin + count) cut at the list's capacity: never past the stored entries.
__host__ __device__ __forceinline__ uint2 clamp_range(uint32_t begin, uint32_t count, int64_t cap)
{
    const int64_t b = begin < cap ? (int64_t)begin : cap;
    const int64_t e = (int64_t)begin + count < cap ? (int64_t)begin + count : cap;
    return make_uint2((uint32_t)b, (uint32_t)e);
}

// Per-workgroup maxima of I carry a bad source value seen by the workgroup as -(max + 1)
__device__ __forceinline__ double mark_bad(double m, bool bad) { return bad ? -(m + 1.0) : m; }
__device__ __forceinline__ double partial_max(double v, bool &bad)
{
    if (v < 0.0) {
        bad = true;
        return -v - 1.0;
    }
    return v;
}

// A source value the method cannot use: negative, NaN or infinite.
template <class T>
__device__ __forceinline__ bool bad_value(T v)
{
    return !(v >= T(0)) || isinf(v);
}

// Order key of |E| at caller index i: the float's bits (|E| >= 0 orders like its bits) above the
// complemented index, so the largest key is the largest |E|, first in caller order among ties.
__device__ __forceinline__ uint64_t e_key(float e, int64_t i)
{
    const float c = e > 0.f ? e : 0.f;  // NaN and negative values rank lowest
    return ((uint64_t)__float_as_uint(c) << 32) | (uint64_t)(0xffffffffu - (uint32_t)i);
}

// LDS written by some lanes of a wave and then read by others of the same wave
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- wave scans

template <class T>
__device__ __forceinline__ T shfl_up_t(T v, int d)
{
    if constexpr (sizeof(T) == 8) {
        const uint32_t lo = __shfl_up((uint32_t)v, (unsigned)d), hi = __shfl_up((uint32_t)(v >> 32), (unsigned)d);
        return ((T)hi << 32) | lo;
    } else {
        return (T)__shfl_up((uint32_t)v, (unsigned)d);
    }
}

// Workgroups are handed to the eight XCDs in turn (workgroup b to XCD b mod 8), and each XCD
// has its own L2.  This maps workgroup b of nb to a logical index such that every XCD takes
// one contiguous range of them (a bijection on [0, nb)): work items that share cache lines
// (neighbouring tiles of sorted points, whose grid rows interleave) then meet in one L2
// instead of each XCD fetching, or writing back, its own copy of the line.
__device__ __forceinline__ int32_t xcd_contiguous(uint32_t b, uint32_t nb)
{
    const uint32_t x = b & 7u, q = nb >> 3, r = nb & 7u;
    return (int32_t)(x * q + min(x, r) + (b >> 3));
}

template <class T>
__device__ __forceinline__ T lane_value(T v, int l)
{
    if constexpr (sizeof(T) == 8) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
        return ((T)hi << 32) | lo;
    } else {
        return (T)(uint32_t)__builtin_amdgcn_readlane((int)v, l);
    }
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int o)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o), hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
    return ((uint64_t)hi << 32) | lo;
}

// inclusive scan across the 64 lanes
template <class T>
__device__ __forceinline__ T wave_inclusive(T v, int lane)
{
    for (int d = 1; d < 64; d <<= 1) {
        const T y = shfl_up_t(v, d);
        if (lane >= d) v += y;
    }
    return v;
}

}  // namespace ph
