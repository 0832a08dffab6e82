// Device code of the learned leaf selector shared by the selection pass and the network
// kernels: the 8 -> 64 -> 64 -> 1 GELU network's inference, and the per-leaf statistics and
// features it reads.  One definition, so that the evaluation path and the training entry
// points compute the same features and logits bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include "k_common.h"

namespace ph {
namespace mlp {

constexpr int NIN = PH_MLP_NIN, NH = PH_MLP_NHID, NP = PH_MLP_NPARAM;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH;

__device__ __forceinline__ float round_bf16(float x)
{
    // round to nearest even on the upper 16 bits
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float a)
{
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * expf(-0.5f * a * a);
}

template <bool BF16>
__device__ __forceinline__ float q(float x)
{
    return BF16 ? round_bf16(x) : x;
}

// Inference, one wave per row: lane i owns hidden unit i of both layers.  The first two
// weight matrices are staged in LDS as groups of four consecutive inputs per hidden unit
// (w[(k / 4) NH + i][k % 4] is weight (i, k)), so a lane reads four weights in one 16-byte
// load and the 64 lanes read consecutive words.  The hidden activations of layer 1 are
// broadcast lane by lane through scalar registers, and the output layer is a fixed butterfly
// sum over the wave.  Every inference (the evaluation path and the standalone forward call)
// runs mlp_row, so their logits agree bit for bit; every sum runs over its inputs in order.
struct MlpLds {
    float4 w1[NIN / 4 * NH], w2[NH / 4 * NH];
    float b1[NH], b2[NH], w3[NH], b3;
};
static_assert(NIN % 4 == 0 && NH % 4 == 0, "weights are staged four inputs at a time");

template <bool BF16>
__device__ void stage_weights(const float *__restrict__ params, MlpLds &L)
{
    // walk the parameters in order (consecutive threads, consecutive addresses) and regroup
    // on the LDS side; eight loads per thread in flight before their stores (one round trip
    // per batch, not one per element).  Weight (o, i) of a layer with NI inputs sits at
    // o NI + i in the parameters.
    constexpr int kB = 8;
    float *w1 = reinterpret_cast<float *>(L.w1), *w2 = reinterpret_cast<float *>(L.w2);
    for (int t0 = threadIdx.x; t0 < NH * NIN; t0 += kB * blockDim.x) {
        float v[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) v[b] = params[OFF_W1 + min(t0 + b * (int)blockDim.x, NH * NIN - 1)];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int u = t0 + b * (int)blockDim.x, o = u / NIN, i = u % NIN;
            if (u < NH * NIN) w1[((i >> 2) * NH + o) * 4 + (i & 3)] = q<BF16>(v[b]);
        }
    }
    for (int t0 = threadIdx.x; t0 < NH * NH; t0 += kB * blockDim.x) {
        float v[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) v[b] = params[OFF_W2 + min(t0 + b * (int)blockDim.x, NH * NH - 1)];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int u = t0 + b * (int)blockDim.x, o = u / NH, i = u % NH;
            if (u < NH * NH) w2[((i >> 2) * NH + o) * 4 + (i & 3)] = q<BF16>(v[b]);
        }
    }
    if (threadIdx.x < NH) {
        L.b1[threadIdx.x] = q<BF16>(params[OFF_B1 + threadIdx.x]);
        L.b2[threadIdx.x] = q<BF16>(params[OFF_B2 + threadIdx.x]);
        L.w3[threadIdx.x] = q<BF16>(params[OFF_W3 + threadIdx.x]);
    }
    if (threadIdx.x == 0) L.b3 = q<BF16>(params[OFF_B3]);
}

// The same staging with every load of a thread in flight at once (KW blockDim >= NP), in two
// halves so that a kernel can issue the loads early and place the values later: parameter
// t + k blockDim goes to thread t (indices past the end read the last parameter: no per-lane
// branch, which would make each load wait on its own), then to its LDS place with the
// rounding of stage_weights (the LDS contents are identical)
template <int KW>
__device__ __forceinline__ void load_weights(const float *__restrict__ params, float (&v)[KW])
{
#pragma unroll
    for (int k = 0; k < KW; ++k) v[k] = params[min((int)threadIdx.x + k * (int)blockDim.x, NP - 1)];
}

template <bool BF16, int KW>
__device__ __forceinline__ void store_weights(const float (&v)[KW], MlpLds &L)
{
    float *w1 = reinterpret_cast<float *>(L.w1), *w2 = reinterpret_cast<float *>(L.w2);
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const int idx = (int)threadIdx.x + k * (int)blockDim.x;
        const float x = q<BF16>(v[k]);
        if (idx < OFF_B1) {
            const int o = idx / NIN, i = idx % NIN;
            w1[((i >> 2) * NH + o) * 4 + (i & 3)] = x;
        } else if (idx < OFF_W2) {
            L.b1[idx - OFF_B1] = x;
        } else if (idx < OFF_B2) {
            const int u = idx - OFF_W2, o = u / NH, i = u % NH;
            w2[((i >> 2) * NH + o) * 4 + (i & 3)] = x;
        } else if (idx < OFF_W3) {
            L.b2[idx - OFF_B2] = x;
        } else if (idx < OFF_B3) {
            L.w3[idx - OFF_W3] = x;
        } else if (idx == OFF_B3) {
            L.b3 = x;
        }
    }
}

template <bool BF16, int KW>
__device__ __forceinline__ void stage_weights_at_once(const float *__restrict__ params, MlpLds &L)
{
    float v[KW];
    load_weights<KW>(params, v);
    store_weights<BF16, KW>(v, L);
}

// value of lane j (uniform j) in every lane
__device__ __forceinline__ float lane_bcast(float v, int j)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// x: the row's 8 inputs, the same values in every lane.  Returns the logit in every lane.
template <bool BF16>
__device__ __forceinline__ float mlp_row(const float (&x)[NIN], const MlpLds &L, int lane)
{
    float a = L.b1[lane];
#pragma unroll
    for (int k4 = 0; k4 < NIN / 4; ++k4) {
        const float4 wq = L.w1[k4 * NH + lane];
        a += wq.x * q<BF16>(x[4 * k4 + 0]);
        a += wq.y * q<BF16>(x[4 * k4 + 1]);
        a += wq.z * q<BF16>(x[4 * k4 + 2]);
        a += wq.w * q<BF16>(x[4 * k4 + 3]);
    }
    const float h1 = q<BF16>(gelu(a));
    float a2 = L.b2[lane];
#pragma unroll 4
    for (int j4 = 0; j4 < NH / 4; ++j4) {
        const float4 wq = L.w2[j4 * NH + lane];
        a2 += wq.x * lane_bcast(h1, 4 * j4 + 0);
        a2 += wq.y * lane_bcast(h1, 4 * j4 + 1);
        a2 += wq.z * lane_bcast(h1, 4 * j4 + 2);
        a2 += wq.w * lane_bcast(h1, 4 * j4 + 3);
    }
    float z = L.w3[lane] * q<BF16>(gelu(a2));
    for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o);
    return z + L.b3;
}

// Up to four rows at once (x[r] for r < nr, every lane the same values): four independent
// chains in flight, each row's operations in the order of mlp_row, so every logit equals
// mlp_row's bit for bit.
template <bool BF16>
__device__ __forceinline__ void mlp_rows4(const float (&x)[4][NIN], const MlpLds &L, int lane, float (&z)[4])
{
    float a[4], h1[4], a2[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = L.b1[lane];
#pragma unroll
    for (int k4 = 0; k4 < NIN / 4; ++k4) {
        const float4 wq = L.w1[k4 * NH + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a[r] += wq.x * q<BF16>(x[r][4 * k4 + 0]);
            a[r] += wq.y * q<BF16>(x[r][4 * k4 + 1]);
            a[r] += wq.z * q<BF16>(x[r][4 * k4 + 2]);
            a[r] += wq.w * q<BF16>(x[r][4 * k4 + 3]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        h1[r] = q<BF16>(gelu(a[r]));
        a2[r] = L.b2[lane];
    }
#pragma unroll 4
    for (int j4 = 0; j4 < NH / 4; ++j4) {
        const float4 wq = L.w2[j4 * NH + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a2[r] += wq.x * lane_bcast(h1[r], 4 * j4 + 0);
            a2[r] += wq.y * lane_bcast(h1[r], 4 * j4 + 1);
            a2[r] += wq.z * lane_bcast(h1[r], 4 * j4 + 2);
            a2[r] += wq.w * lane_bcast(h1[r], 4 * j4 + 3);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float zz = L.w3[lane] * q<BF16>(gelu(a2[r]));
        for (int o = 32; o > 0; o >>= 1) zz += __shfl_xor(zz, o);
        z[r] = zz + L.b3;
    }
}

// ---------------------------------------------------------------- per-leaf statistics and features

// wave reductions in a fixed butterfly order
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// The source rule of the plan: the same expression as the selection's
__device__ __forceinline__ bool candidate(double v, double src_rel, double imax)
{
    return (src_rel <= 0.0) || (v >= src_rel * imax);
}

// Statistics of one plan leaf (sorted points [st, en)) by one wave: over the candidates (the
// plan's source rule) the largest I, the sum of w I and their count; over all points the
// largest, the sum and the sum of squares of |E|.  fetch(k, v, e) gives I and |E| of sorted
// point k.  Lane l takes points st + l, st + l + 64, ... in order, and the lanes are combined
// by a fixed butterfly, which leaves the same bits in every lane; so the statistics do not
// depend on where the values come from, and every caller of this function agrees bit for bit.
struct LeafStats {
    double imax_c, swi_c, n_c, emax, es, es2, n;
};

template <class F>
__device__ __forceinline__ LeafStats leaf_stats_wave(F &&fetch, const double *__restrict__ w, double w_ref,
                                                     int32_t st, int32_t en, double src_rel, double imax, int lane)
{
    LeafStats s{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, (double)(en - st)};
    for (int32_t k = st + lane; k < en; k += 64) {
        double v, e;
        fetch(k, v, e);
        if (candidate(v, src_rel, imax)) {
            s.imax_c = fmax(s.imax_c, v);
            s.swi_c += v * (w ? w[k] : w_ref);
            s.n_c += 1.0;
        }
        s.emax = fmax(s.emax, e);
        s.es += e;
        s.es2 += e * e;
    }
    s.imax_c = wave_max(s.imax_c);
    s.swi_c = wave_sum(s.swi_c);
    s.n_c = wave_sum(s.n_c);
    s.emax = wave_max(s.emax);
    s.es = wave_sum(s.es);
    s.es2 = wave_sum(s.es2);
    return s;
}

// Reference points and scales of a call's features.
struct FeatureRefs {
    double imax, emax, w_ref;
    double xi[3];       // position of the largest I
    double xe[3];       // position of the largest |E|
    double lo[3], cube; // root cube
    bool efeat;         // |E| given and not all zero
};

// The eight inputs of a candidate leaf (level, anchor ax/ay/az):
//   0 log10(max I / I_max) over its candidates       1 log10(sum w I / (I_max w_ref)) over them
//   2 log10(candidates / points of the leaf)
//   3 log10(1 + |centre - x_Imax| / side)             4 log10(1 + |centre - x_Emax| / side)
//   5 max |E| / E_max     6 mean |E| / E_max     7 std |E| / E_max   (over the leaf's points;
//   features 4-7 are 0 without |E|)
__device__ __forceinline__ void leaf_features(const LeafStats &s, const FeatureRefs &r, int level, int ax, int ay,
                                              int az, float (&fe)[NIN])
{
    const double side = r.cube / (double)(1 << level), hw = 0.5 * side;
    const double c0 = r.lo[0] + (2.0 * ax + 1.0) * hw, c1 = r.lo[1] + (2.0 * ay + 1.0) * hw,
                 c2 = r.lo[2] + (2.0 * az + 1.0) * hw;
    fe[0] = (float)log10(fmax(s.imax_c / r.imax, 1e-300));
    fe[1] = (float)log10(fmax(s.swi_c / (r.imax * r.w_ref), 1e-300));
    fe[2] = (float)log10(fmax(s.n_c / s.n, 1e-300));
    const double d0 = c0 - r.xi[0], d1 = c1 - r.xi[1], d2 = c2 - r.xi[2];
    fe[3] = (float)log10(1.0 + sqrt(d0 * d0 + d1 * d1 + d2 * d2) / side);
    for (int q = 4; q < NIN; ++q) fe[q] = 0.0f;
    if (r.efeat) {
        const double e0 = c0 - r.xe[0], e1 = c1 - r.xe[1], e2 = c2 - r.xe[2];
        fe[4] = (float)log10(1.0 + sqrt(e0 * e0 + e1 * e1 + e2 * e2) / side);
        const double mean = s.es / r.emax / s.n;
        fe[5] = (float)(s.emax / r.emax);
        fe[6] = (float)mean;
        fe[7] = (float)sqrt(fmax(s.es2 / (r.emax * r.emax) / s.n - mean * mean, 0.0));
    }
}

}  // namespace mlp
}  // namespace ph
