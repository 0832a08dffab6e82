// Learned leaf selector: the 8 -> 64 -> 64 -> 1 GELU network (inference, training, Adam)
// and the per-leaf features, contributions and keep decisions of the adaptive FMM.
//
// Parameter layout (PH_MLP_NPARAM floats): W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.
// GELU is the exact erf form.  Training loss: mean binary cross-entropy with logits,
// positive rows weighted by pos_weight.  Gradients are summed per block of rows and the
// block partials reduced in block order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <mutex>

#include "k_fmm_args.h"

namespace ph {

namespace {

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
// weight matrices are staged transposed in LDS so that the 64 lanes read consecutive words;
// the hidden activations of layer 1 are broadcast lane by lane, and the output layer is a
// fixed butterfly sum over the wave.  Every inference (the evaluation path and the
// standalone forward call) runs mlp_row, so their logits agree bit for bit.
struct MlpLds {
    float w1t[NIN * NH], w2t[NH * NH], b1[NH], b2[NH], w3[NH], b3;
};

template <bool BF16>
__device__ void stage_weights(const float *__restrict__ params, MlpLds &L)
{
    // walk the parameters in order (consecutive threads, consecutive addresses) and transpose
    // on the LDS side; eight loads per thread in flight
    // before their stores (one round trip per batch, not one per element).  Weight (o, i) of a
    // layer with NI inputs sits at o NI + i in the parameters and at i NH + o in LDS.
    constexpr int kB = 8;
    for (int t0 = threadIdx.x; t0 < NH * NIN; t0 += kB * blockDim.x) {
        float v[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) v[b] = params[OFF_W1 + min(t0 + b * (int)blockDim.x, NH * NIN - 1)];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int u = t0 + b * (int)blockDim.x;
            if (u < NH * NIN) L.w1t[(u % NIN) * NH + u / NIN] = q<BF16>(v[b]);
        }
    }
    for (int t0 = threadIdx.x; t0 < NH * NH; t0 += kB * blockDim.x) {
        float v[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) v[b] = params[OFF_W2 + min(t0 + b * (int)blockDim.x, NH * NH - 1)];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int u = t0 + b * (int)blockDim.x;
            if (u < NH * NH) L.w2t[(u % NH) * NH + u / NH] = q<BF16>(v[b]);
        }
    }
    if (threadIdx.x < NH) {
        L.b1[threadIdx.x] = q<BF16>(params[OFF_B1 + threadIdx.x]);
        L.b2[threadIdx.x] = q<BF16>(params[OFF_B2 + threadIdx.x]);
        L.w3[threadIdx.x] = q<BF16>(params[OFF_W3 + threadIdx.x]);
    }
    if (threadIdx.x == 0) L.b3 = q<BF16>(params[OFF_B3]);
}

// x: the row's 8 inputs, the same values in every lane.  Returns the logit in every lane.
template <bool BF16>
__device__ __forceinline__ float mlp_row(const float (&x)[NIN], const MlpLds &L, int lane)
{
    float a = L.b1[lane];
#pragma unroll
    for (int k = 0; k < NIN; ++k) a += L.w1t[k * NH + lane] * q<BF16>(x[k]);
    const float h1 = q<BF16>(gelu(a));
    float a2 = L.b2[lane];
#pragma unroll 16
    for (int j = 0; j < NH; ++j) a2 += L.w2t[j * NH + lane] * __shfl(h1, j);
    float z = L.w3[lane] * q<BF16>(gelu(a2));
    for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o);
    return z + L.b3;
}

// m_dev (nullable) caps the row count from the device.
template <bool BF16>
__global__ __launch_bounds__(256) void mlp_rows_kernel(const float *__restrict__ params, const float *__restrict__ X,
                                                       int64_t m, const int32_t *__restrict__ m_dev,
                                                       float *__restrict__ logits)
{
    __shared__ MlpLds L;
    stage_weights<BF16>(params, L);
    __syncthreads();
    const int64_t rows = m_dev ? min(m, (int64_t)*m_dev) : m;
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < rows; r += (int64_t)gridDim.x * 4) {
        float x[NIN];
#pragma unroll
        for (int k = 0; k < NIN; ++k) x[k] = X[r * NIN + k];
        const float z = mlp_row<BF16>(x, L, lane);
        if (lane == 0) logits[r] = z;
    }
}

constexpr int kRows = 32;  // rows per backward block

// Per block of kRows rows: forward, loss, and the block's gradient partial (NP values + loss).
__global__ __launch_bounds__(256) void mlp_backward_kernel(const float *__restrict__ params,
                                                           const float *__restrict__ X, const float *__restrict__ y,
                                                           float pos_weight, int64_t m, float *__restrict__ partial)
{
    __shared__ float w[NP];
    __shared__ float sx[kRows][NIN], sh1[kRows][NH], sda1[kRows][NH], sda2[kRows][NH], sh2[kRows][NH];
    __shared__ float sdz[kRows], sloss[kRows];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = params[i];
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * kRows;
    const int t = threadIdx.x;
    if (t < kRows) {
        const int64_t r = r0 + t;
        if (r < m) {
            float x[NIN], h1[NH], a1[NH];
            for (int k = 0; k < NIN; ++k) x[k] = sx[t][k] = X[r * NIN + k];
            for (int i = 0; i < NH; ++i) {
                float a = w[OFF_B1 + i];
                for (int k = 0; k < NIN; ++k) a += w[OFF_W1 + i * NIN + k] * x[k];
                a1[i] = a;
                h1[i] = gelu(a);
                sh1[t][i] = h1[i];
            }
            float z = w[OFF_B3];
            for (int i = 0; i < NH; ++i) {
                float a = w[OFF_B2 + i];
                for (int j = 0; j < NH; ++j) a += w[OFF_W2 + i * NH + j] * h1[j];
                const float h2 = gelu(a);
                sh2[t][i] = h2;
                sda2[t][i] = a;  // pre-activation for now
                z += w[OFF_W3 + i] * h2;
            }
            const float yy = y[r];
            const float sg = 1.0f / (1.0f + expf(-z));
            // mean weighted BCE with logits, stable log-sigmoid
            const float ls = -(fmaxf(-z, 0.0f) + log1pf(expf(-fabsf(z))));
            const float l1s = -(fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))));
            sloss[t] = -(pos_weight * yy * ls + (1.0f - yy) * l1s) / (float)m;
            const float dz = (pos_weight * yy * (sg - 1.0f) + (1.0f - yy) * sg) / (float)m;
            sdz[t] = dz;
            float dh1[NH];
            for (int j = 0; j < NH; ++j) dh1[j] = 0.0f;
            for (int i = 0; i < NH; ++i) {
                const float da2 = dz * w[OFF_W3 + i] * gelu_grad(sda2[t][i]);
                sda2[t][i] = da2;
                for (int j = 0; j < NH; ++j) dh1[j] += w[OFF_W2 + i * NH + j] * da2;
            }
            for (int j = 0; j < NH; ++j) sda1[t][j] = dh1[j] * gelu_grad(a1[j]);
        } else {
            for (int k = 0; k < NIN; ++k) sx[t][k] = 0.0f;
            for (int i = 0; i < NH; ++i) sh1[t][i] = sda1[t][i] = sda2[t][i] = sh2[t][i] = 0.0f;
            sdz[t] = 0.0f;
            sloss[t] = 0.0f;
        }
    }
    __syncthreads();
    float *out = partial + (size_t)blockIdx.x * (NP + 1);
    for (int p = t; p < NP + 1; p += blockDim.x) {
        float g = 0.0f;
        if (p < OFF_B1) {
            const int i = p / NIN, k = p % NIN;
            for (int rr = 0; rr < kRows; ++rr) g += sda1[rr][i] * sx[rr][k];
        } else if (p < OFF_W2) {
            const int i = p - OFF_B1;
            for (int rr = 0; rr < kRows; ++rr) g += sda1[rr][i];
        } else if (p < OFF_B2) {
            const int i = (p - OFF_W2) / NH, j = (p - OFF_W2) % NH;
            for (int rr = 0; rr < kRows; ++rr) g += sda2[rr][i] * sh1[rr][j];
        } else if (p < OFF_W3) {
            const int i = p - OFF_B2;
            for (int rr = 0; rr < kRows; ++rr) g += sda2[rr][i];
        } else if (p < OFF_B3) {
            const int i = p - OFF_W3;
            for (int rr = 0; rr < kRows; ++rr) g += sdz[rr] * sh2[rr][i];
        } else if (p == OFF_B3) {
            for (int rr = 0; rr < kRows; ++rr) g += sdz[rr];
        } else {
            for (int rr = 0; rr < kRows; ++rr) g += sloss[rr];
        }
        out[p] = g;
    }
}

// grad[p] = sum over blocks (in block order) of partial[b][p]; loss from the extra slot
__global__ void mlp_reduce_kernel(const float *__restrict__ partial, int nblocks, float *__restrict__ grad,
                                  float *__restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NP) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += (double)partial[(size_t)b * (NP + 1) + p];
    if (p < NP) grad[p] = (float)s;
    else *loss = (float)s;
}

__global__ void adam_kernel(float *__restrict__ params, float *__restrict__ m1, float *__restrict__ m2,
                            const float *__restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    params[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

std::mutex g_partial_mutex;
float *g_partial = nullptr;
size_t g_partial_bytes = 0;

// Gradient partials of the allocation-free backward call: kNoAllocMaxBlocks blocks of
// NP + 1 floats (4.9 MB), in the code object's own device memory on every GPU the library
// runs on, held until the process ends.  Host code never passes this name to a kernel: its
// device address, looked up once per device, is what the launches take.
constexpr int kNoAllocMaxBlocks = PH_MLP_NOALLOC_MAX_ROWS / kRows;
static_assert(PH_MLP_NOALLOC_MAX_ROWS % kRows == 0, "whole blocks of rows");
static __device__ __align__(256) float scratch[(size_t)kNoAllocMaxBlocks * (NP + 1)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
float *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (looked up at the first call there)
float *scratch_on_current_device()
{
    int dev = 0;
    PH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error{PH_EDEVICE, "device index beyond the scratch table"};
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        PH_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error{PH_EDEVICE, "no device address for the backward scratch"};
        g_scratch_ptr[dev] = static_cast<float *>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

void launch_mlp_forward(const float *params, const float *X, int64_t m, const int32_t *m_dev, float *logits,
                        int bf16, hipStream_t s)
{
    if (m == 0) return;
    // a device-side row count is small (selector rows): fewer blocks stage the weights
    const unsigned g = (unsigned)std::min<int64_t>((m + 3) / 4, m_dev ? 256 : 1024);
    if (bf16) mlp_rows_kernel<true><<<g, 256, 0, s>>>(params, X, m, m_dev, logits);
    else mlp_rows_kernel<false><<<g, 256, 0, s>>>(params, X, m, m_dev, logits);
}

void launch_mlp_backward(const float *params, const float *X, const float *y, float pos_weight, int64_t m,
                         float *grad, float *loss, hipStream_t s)
{
    const int nblocks = (int)((m + kRows - 1) / kRows);
    const size_t need = (size_t)nblocks * (NP + 1) * sizeof(float);
    std::lock_guard<std::mutex> lock(g_partial_mutex);
    if (need > g_partial_bytes) {
        // training scratch, kept for the life of the process and grown on demand
        PH_HIP(hipStreamSynchronize(s));
        if (g_partial) PH_HIP(hipFree(g_partial));
        g_partial = nullptr;
        g_partial_bytes = 0;
        PH_HIP(hipMalloc(&g_partial, need));
        g_partial_bytes = need;
    }
    mlp_backward_kernel<<<nblocks, 256, 0, s>>>(params, X, y, pos_weight, m, g_partial);
    mlp_reduce_kernel<<<(NP + 1 + 255) / 256, 256, 0, s>>>(g_partial, nblocks, grad, loss);
}

void launch_mlp_backward_noalloc(const float *params, const float *X, const float *y, float pos_weight, int64_t m,
                                 float *grad, float *loss, hipStream_t s)
{
    if (m < 1 || m > PH_MLP_NOALLOC_MAX_ROWS) throw Error{PH_EINVAL, "rows must be in 1..PH_MLP_NOALLOC_MAX_ROWS"};
    float *part = scratch_on_current_device();
    const int nblocks = (int)((m + kRows - 1) / kRows);
    // every block writes its whole partial (rows past m count zero), so nothing needs clearing
    mlp_backward_kernel<<<nblocks, 256, 0, s>>>(params, X, y, pos_weight, m, part);
    mlp_reduce_kernel<<<(NP + 1 + 255) / 256, 256, 0, s>>>(part, nblocks, grad, loss);
}

void launch_adam(float *params, float *m1, float *m2, const float *grad, int64_t n, float lr, float b1, float b2,
                 float eps, int64_t step, hipStream_t s)
{
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(params, m1, m2, grad, n, lr, b1, b2, eps, c1, c2);
}


// ---------------------------------------------------------------- selector rows, features, decisions
//
// The selector decides on the leaves of the plan's tree (the tree over all points, fixed at
// plan time), straight from the sorted arrays, before any selection of the call: a row is a
// plan leaf holding at least one candidate source (I >= src_rel I_max, the threshold rule of
// the plan), and a dropped row removes all its candidates from the call's source set.
// Two passes over the plan leaves: per-leaf statistics, then features and decisions.

namespace {

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

__device__ __forceinline__ bool candidate(double v, double src_rel, double imax)
{
    // the same expression as the selection kernel's source rule
    return (src_rel <= 0.0) || (v >= src_rel * imax);
}

struct LeafArgs {
    BoxArrays bx;
    const int32_t *pleaf, *pleaf_of_box, *perm, *iperm;
    const int4 *pinfo, *pinfo2;  // per plan leaf: (box, first, end, 0), (anchor x, y, z, level)
    const int32_t *pcoll;        // per plan leaf, 27: C (a plan leaf), -2 - C (split), -1 (none)
    int32_t n_pleaf;
    const double *xyz;
    const double *w;  // sorted quadrature weights, null on uniform grids (w = w_ref)
    const float *E;
    CallScalars *sc;
    int32_t *sticky;         // the plan's sticky error word
    uint32_t *flag, *flag2;  // candidate flags (flag2: a copy for the row compaction, nullable)
    int32_t *list;           // candidate leaves (plan-leaf indices, any order)
    double *lstat;           // per leaf: max I, sum |E|, sum |E|^2, max |E|
    float *box_emax;         // per leaf box: max |E|
    float *feats;
    int32_t *cnt;
    double lo0, lo1, lo2, cube, w_ref, src_rel;
    // decisions (evaluation path)
    const float *params;
    float threshold;
    float *logits;
    uint8_t *drop;
};

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o), hi = __shfl_xor((uint32_t)(v >> 32), o);
        const uint64_t u = ((uint64_t)hi << 32) | lo;
        v = u > v ? u : v;
    }
    return v;
}

constexpr int kLPW = 4;  // plan leaves per wave in the statistics pass: 16 lanes each

// sum / max over the 16 lanes of a quarter-wave (butterfly, fixed order)
__device__ __forceinline__ double quarter_sum(double v)
{
    for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double quarter_max(double v)
{
    for (int o = 8; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Pass 1, over the plan leaves in sorted order (grid-stride; a wave takes kLPW leaves, 16
// lanes each, so one set of 16-lane reductions serves four leaves): per leaf the largest I and
// the sum, sum of squares and maximum of |E|; per block the partial maxima of I and of the
// |E| order key over all points (the same maxima as the plain reduction).
template <class T>
__global__ __launch_bounds__(256) void leaf_reduce_kernel(LeafArgs a, const T *__restrict__ I,
                                                          double *__restrict__ partial,
                                                          uint64_t *__restrict__ partial_key, int32_t *gen)
{
    if (blockIdx.x == 0 && gen) begin_call(a.sc, gen);
    __shared__ double smI[4];
    __shared__ uint64_t smE[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int slot = lane >> 4, sub = lane & 15;
    const bool has_e = a.E != nullptr;
    double gmax = 0.0;
    uint64_t gkey = 0;
    int bad = 0;
    for (int64_t base = ((int64_t)blockIdx.x * 4 + wv) * kLPW; base < a.n_pleaf;
         base += (int64_t)gridDim.x * 4 * kLPW) {
        const int64_t i = base + slot;
        const int4 inf = i < a.n_pleaf ? a.pinfo[i] : make_int4(-1, 0, 0, 0);  // box, first, end
        const int32_t f = inf.x, st = inf.y, en = inf.z;
        double mx = 0.0, es = 0.0, es2 = 0.0;
        float emx = 0.0f;
        for (int32_t k0 = st; k0 < en; k0 += 64) {
            // up to four points per lane, all loads issued before use
            int32_t o[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int32_t k = k0 + sub + 16 * m;
                o[m] = k < en ? a.perm[k] : -1;
            }
            T v[4];
            float e[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                v[m] = o[m] >= 0 ? I[o[m]] : T(0);
                e[m] = (has_e && o[m] >= 0) ? a.E[o[m]] : 0.0f;
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (o[m] < 0) continue;
                if (bad_value(v[m])) bad = 1;
                else mx = fmax(mx, (double)v[m]);
                if (has_e) {
                    gkey = max(gkey, e_key(e[m], o[m]));
                    emx = fmaxf(emx, e[m]);
                    es += (double)e[m];
                    es2 += (double)e[m] * (double)e[m];
                }
            }
        }
        gmax = fmax(gmax, mx);
        mx = quarter_max(mx);
        es = quarter_sum(es);
        es2 = quarter_sum(es2);
        const double em = quarter_max((double)emx);
        if (sub == 0 && f >= 0) {
            double *L = a.lstat + (size_t)i * 4;
            L[0] = mx;
            L[1] = es;
            L[2] = es2;
            L[3] = em;
            a.box_emax[f] = (float)em;
        }
    }
    __shared__ int anybad;
    if (threadIdx.x == 0) anybad = 0;
    __syncthreads();
    if (bad) anybad = 1;
    gmax = wave_max(gmax);
    gkey = wave_max_u64(gkey);
    if (lane == 0) {
        smI[wv] = gmax;
        smE[wv] = gkey;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = smI[0];
        uint64_t k = smE[0];
        for (int q = 1; q < 4; ++q) {
            m = fmax(m, smI[q]);
            k = max(k, smE[q]);
        }
        partial[blockIdx.x] = mark_bad(m, anybad != 0);
        partial_key[blockIdx.x] = k;
    }
}

// Pass 2, one thread per plan leaf: it is a row iff its largest I passes the source rule.
// Every workgroup first reduces pass 1's per-workgroup maxima itself (nb of them, a few KB
// from L2) for the largest I; workgroup 0 also stores the maxima for the later kernels.
__global__ __launch_bounds__(256) void leaf_pick_kernel(LeafArgs a, const double *__restrict__ partial,
                                                        const uint64_t *__restrict__ partial_key, int nb)
{
    __shared__ double smI[4];
    __shared__ uint64_t smE[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double mi = 0.0;
    uint64_t me = 0;
    bool bad = false;
    // eight of each per thread in flight (a zero partial is neutral: not marked, no larger)
    for (int j0 = threadIdx.x; j0 < nb; j0 += 8 * blockDim.x) {
        double pv[8];
        uint64_t kv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + u * (int)blockDim.x;
            pv[u] = j < nb ? partial[j] : 0.0;
            kv[u] = j < nb ? partial_key[j] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            mi = fmax(mi, partial_max(pv[u], bad));
            me = max(me, kv[u]);
        }
    }
    if (bad && blockIdx.x == 0) flag_error(a.sc, a.sticky, 1);
    mi = wave_max(mi);
    me = wave_max_u64(me);
    if (lane == 0) {
        smI[wv] = mi;
        smE[wv] = me;
    }
    __syncthreads();
    double imax = smI[0];
    uint64_t ekey = smE[0];
    for (int q = 1; q < 4; ++q) {
        imax = fmax(imax, smI[q]);
        ekey = max(ekey, smE[q]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double emax = (double)__uint_as_float((uint32_t)(ekey >> 32));
        a.sc->imax = imax;
        a.sc->emax = emax;
        a.sc->emax_key = ekey;
        // the position of the largest |E| (the distance feature's reference point)
        double ex = 0.0, ey = 0.0, ez = 0.0;
        if (a.E && emax > 0.0) {
            const int64_t kp = a.iperm[0xffffffffu - (uint32_t)(ekey & 0xffffffffu)];
            ex = a.xyz[3 * kp];
            ey = a.xyz[3 * kp + 1];
            ez = a.xyz[3 * kp + 2];
        }
        a.sc->emax_xyz[0] = ex;
        a.sc->emax_xyz[1] = ey;
        a.sc->emax_xyz[2] = ez;
    }
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && a.flag2) a.flag2[a.n_pleaf] = 0;
    if (i >= a.n_pleaf) return;
    const bool cand = candidate(a.lstat[(size_t)i * 4], a.src_rel, imax);
    a.flag[i] = cand ? 1u : 0u;
    if (a.flag2) a.flag2[i] = cand ? 1u : 0u;
    if (cand) a.list[atomicAdd(&a.sc->n_srcleaf, 1)] = i;
}

// Pass 3, one wave per row (grid-stride over the candidate list): the candidates' count and
// sum of w I, the eight features; with DECIDE also the network (BF16) and the keep/drop
// decision, keep iff logit >= threshold.  The drop byte of every point of a decided leaf is
// written (0 or 1), so the mask needs no clearing: points outside candidate leaves fail the
// source rule anyway.  A non-finite logit switches the call to the fallback rule.  Sums run
// in a fixed lane/stride/butterfly order; results do not depend on the list's order.
template <class T, bool DECIDE>
__global__ __launch_bounds__(256) void leaf_features_kernel(LeafArgs a, const T *__restrict__ I)
{
    __shared__ MlpLds L;
    const int lane = threadIdx.x & 63;
    const int32_t nrow = a.sc->n_srcleaf;
    if ((int32_t)blockIdx.x * 4 >= nrow) return;  // the whole block
    if (DECIDE) {
        stage_weights<true>(a.params, L);
        __syncthreads();
    }
    const double imax = a.sc->imax, emax = a.sc->emax;
    const double ex = a.sc->emax_xyz[0], ey = a.sc->emax_xyz[1], ez = a.sc->emax_xyz[2];
    const bool efeat = a.E && emax > 0.0;
    for (int32_t r = blockIdx.x * 4 + (threadIdx.x >> 6); r < nrow; r += gridDim.x * 4) {
        const int32_t i = a.list[r];
        // the row's records, all loaded together
        const int4 inf = a.pinfo[i], inf2 = a.pinfo2[i];
        const int32_t cq = (efeat && lane < 27) ? a.pcoll[(size_t)i * 27 + lane] : -1;
        const double *S = a.lstat + (size_t)i * 4;
        const double S0 = S[0], S1 = S[1], S2 = S[2], S3 = S[3];
        const int32_t st = inf.y, en = inf.z;
        double swi = 0.0, cnt = 0.0;
        for (int32_t k = st + lane; k < en; k += 64) {
            const double v = (double)I[a.perm[k]];
            if (!candidate(v, a.src_rel, imax)) continue;
            swi += v * (a.w ? a.w[k] : a.w_ref);
            cnt += 1.0;
        }
        swi = wave_sum(swi);
        cnt = wave_sum(cnt);
        const int level = inf2.w;
        const double side = a.cube / (double)(1 << level), hw = 0.5 * side;
        float fe[8];
        fe[0] = (float)log10(fmax(S0 / imax, 1e-300));
        fe[1] = (float)log10(fmax(swi / (imax * a.w_ref), 1e-300));
        fe[2] = (float)log2(side / cbrt(a.w_ref));
        for (int q = 3; q < 8; ++q) fe[q] = 0.0f;
        if (efeat) {
            const double cx = a.lo0 + (2.0 * inf2.x + 1.0) * hw, cy = a.lo1 + (2.0 * inf2.y + 1.0) * hw,
                         cz = a.lo2 + (2.0 * inf2.z + 1.0) * hw;
            const double dx = cx - ex, dy = cy - ey, dz = cz - ez;
            fe[3] = (float)log10(1.0 + sqrt(dx * dx + dy * dy + dz * dz) / side);
            const double nn = (double)(en - st);
            const double mean = S1 / emax / nn;
            fe[4] = (float)(S3 / emax);
            fe[5] = (float)mean;
            fe[6] = (float)sqrt(fmax(S2 / (emax * emax) / nn - mean * mean, 0.0));
            // the 27 boxes around the leaf, one lane each: a leaf's stored maximum, or the box's range
            double nmx = 0.0;
            if (cq >= 0) {
                nmx = (double)a.box_emax[cq];
            } else if (cq < -1) {
                const int32_t C = -2 - cq;
                for (int32_t k = a.bx.start[C]; k < a.bx.end[C]; ++k) nmx = fmax(nmx, (double)a.E[a.perm[k]]);
            }
            fe[7] = (float)(wave_max(nmx) / emax);
        }
        if (lane < 8) a.feats[(size_t)i * 8 + lane] = fe[lane];
        if (lane == 0) a.cnt[i] = (int32_t)cnt;
        if (DECIDE) {
            const float z = mlp_row<true>(fe, L, lane);
            if (lane == 0) a.logits[i] = z;
            if (!isfinite(z)) {
                if (lane == 0) atomicOr(&a.sc->fallback, 1);
                continue;
            }
            if (lane == 0) atomicAdd(&a.sc->n_src_base, (int32_t)cnt);
            const uint8_t d = z >= a.threshold ? 0 : 1;
            for (int32_t k = st + lane; k < en; k += 64) a.drop[k] = d;
        }
    }
}

// Row compaction for the training entry points: rows in box order, with their features.
__global__ void rows_kernel(const int32_t *__restrict__ pleaf, int32_t n_pleaf, const uint32_t *__restrict__ scanned,
                            const float *__restrict__ feats, int32_t *__restrict__ rows,
                            float *__restrict__ row_feats)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pleaf) return;
    if (scanned[i + 1] == scanned[i]) return;
    const uint32_t r = scanned[i];
    rows[r] = pleaf[i];
    for (int k = 0; k < 8; ++k) row_feats[(size_t)r * 8 + k] = feats[(size_t)i * 8 + k];
}

// Field of each row's candidate sources at the given targets, in the units of S:
// out[r ld + t] = P 2^e sum_{k in row r} (w_k I_k 2^-e K(|x_t - x_k|), or c_self I_k 2^-e when
// x_t is x_k).  Kernel values in FP32 (FP64 plans: FP64), sums in FP64.
struct FieldArgs {
    BoxArrays bx;
    const int32_t *perm, *iperm, *rows;
    const double *xyz, *w;
    const CallScalars *sc;
    double w_ref, c_self, src_rel, P;
};

constexpr int kFieldTargets = 2048;  // targets per block (eight passes of 256)

template <class T>
__global__ __launch_bounds__(256) void fields_kernel(FieldArgs a, KParams<T> kp, const T *__restrict__ I,
                                                     const int32_t *__restrict__ targets, int64_t nt,
                                                     float *__restrict__ out, int64_t ld)
{
    __shared__ V4<T> tile[256];
    __shared__ int32_t tpos[256];
    const int32_t r = blockIdx.y;
    const int32_t f = a.rows[r];
    const int32_t st = a.bx.start[f], en = a.bx.end[f];
    const double imax = a.sc->imax;
    int e = 0;
    if (imax > 0.0) {
        (void)frexp(imax, &e);
        e -= 1;
    }
    const double scale = ldexp(1.0, -e);
    const bool one_tile = en - st <= 256;
    auto load_tile = [&](int32_t base) {
        const int32_t k = base + (int32_t)threadIdx.x;
        if (k < en) {
            const double v = (double)I[a.perm[k]];
            const double wk = a.w ? a.w[k] : a.w_ref;
            V4<T> y;
            y.x = (T)a.xyz[3 * (int64_t)k];
            y.y = (T)a.xyz[3 * (int64_t)k + 1];
            y.z = (T)a.xyz[3 * (int64_t)k + 2];
            y.w = candidate(v, a.src_rel, imax) ? (T)(wk * v * scale) : T(0);
            tile[threadIdx.x] = y;
            tpos[threadIdx.x] = k;
        }
    };
    if (one_tile) {
        load_tile(st);
        __syncthreads();
    }
    const double own = a.w ? 0.0 : a.c_self / a.w_ref;  // own cell on uniform grids only
    const int64_t t0 = (int64_t)blockIdx.x * kFieldTargets;
    for (int64_t tb = t0; tb < min(nt, t0 + kFieldTargets); tb += 256) {
        const int64_t t = tb + threadIdx.x;
        const bool act = t < nt;
        int32_t kt = -1;
        T x = 0, y = 0, z = 0;
        if (act) {
            kt = a.iperm[targets[t]];
            x = (T)a.xyz[3 * (int64_t)kt];
            y = (T)a.xyz[3 * (int64_t)kt + 1];
            z = (T)a.xyz[3 * (int64_t)kt + 2];
        }
        double acc = 0.0;
        for (int32_t base = st; base < en; base += 256) {
            if (!one_tile) {
                __syncthreads();
                load_tile(base);
                __syncthreads();
            }
            const int m = min(256, en - base);
            if (act)
                for (int j = 0; j < m; ++j) {
                    const V4<T> s = tile[j];
                    if (s.w == T(0)) continue;
                    if (tpos[j] == kt) {
                        acc += own * (double)s.w;
                        continue;
                    }
                    const T dx = x - s.x, dy = y - s.y, dz = z - s.z;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 > T(0)) acc += (double)(kernel_eval<true>(r2, kp) * s.w);
                }
        }
        if (act) out[(int64_t)r * ld + t] = (float)(a.P * ldexp(acc, e));
    }
}

}  // namespace

static LeafArgs leaf_args(Plan &p, const float *E)
{
    LeafArgs a{};
    a.bx = p.box;
    a.pleaf = p.d_pleaf;
    a.pleaf_of_box = p.d_pleaf_of_box;
    a.pinfo = p.d_pinfo;
    a.pinfo2 = p.d_pinfo2;
    a.pcoll = p.d_pcoll;
    a.perm = p.d_perm;
    a.iperm = p.d_iperm;
    a.n_pleaf = p.n_pleaf;
    a.xyz = p.d_xyz;
    a.w = p.d_w;
    a.E = E;
    a.sc = p.d_sc;
    a.sticky = p.d_sticky;
    a.flag = p.d_leafflag;
    a.list = p.d_cand_list;
    a.lstat = p.d_lstat;
    a.box_emax = p.d_box_emax;
    a.feats = p.d_feat;
    a.cnt = p.d_feat_cnt;
    a.lo0 = p.cube_lo[0];
    a.lo1 = p.cube_lo[1];
    a.lo2 = p.cube_lo[2];
    a.cube = p.cube_size;
    a.w_ref = p.uniform_w ? p.w_uniform : p.cube_size * p.cube_size * p.cube_size / (double)p.n;
    a.src_rel = p.thr.src_rel;
    return a;
}

static unsigned feature_blocks(const Plan &p) { return (unsigned)std::min<int64_t>((p.n_pleaf + 3) / 4, 256); }

// the maxima of I and |E| and the per-leaf statistics in one pass (scalars reset)
void selector_reduce(Plan &p, const void *I, const float *E, int32_t *gen, hipStream_t s)
{
    LeafArgs a = leaf_args(p, E);
    const int nb = (int)std::min<int64_t>((p.n_pleaf + 4 * kLPW - 1) / (4 * kLPW), kLeafPartials);
    double *partial = reinterpret_cast<double *>(p.d_scan_tmp);
    uint64_t *partial_key = reinterpret_cast<uint64_t *>(partial + kLeafPartials);
    if (p.precision == PH_FP64)
        leaf_reduce_kernel<double><<<nb, 256, 0, s>>>(a, (const double *)I, partial, partial_key, gen);
    else
        leaf_reduce_kernel<float><<<nb, 256, 0, s>>>(a, (const float *)I, partial, partial_key, gen);
    // the maxima over the workgroups' partials: reduced by each workgroup of the pick pass
}

// the pick pass over the plan leaves, with the maxima of pass 1's partials (see selector_reduce)
static void launch_leaf_pick(Plan &p, const LeafArgs &a, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((p.n_pleaf + 4 * kLPW - 1) / (4 * kLPW), kLeafPartials);
    const double *partial = reinterpret_cast<const double *>(p.d_scan_tmp);
    const uint64_t *partial_key = reinterpret_cast<const uint64_t *>(partial + kLeafPartials);
    leaf_pick_kernel<<<(unsigned)((p.n_pleaf + 255) / 256), 256, 0, s>>>(a, partial, partial_key, nb);
}

// rows, their features, and the rows compacted in box order (after selector_reduce)
void selector_features(Plan &p, const void *I, const float *E, hipStream_t s)
{
    LeafArgs a = leaf_args(p, E);
    a.flag2 = p.d_leafscan;
    launch_leaf_pick(p, a, s);
    if (p.precision == PH_FP64) leaf_features_kernel<double, false><<<feature_blocks(p), 256, 0, s>>>(a, (const double *)I);
    else leaf_features_kernel<float, false><<<feature_blocks(p), 256, 0, s>>>(a, (const float *)I);
    exclusive_scan_u32(p.d_leafscan, p.n_pleaf + 1, p.d_scan_tmp, nullptr, s);
    rows_kernel<<<(unsigned)((p.n_pleaf + 255) / 256), 256, 0, s>>>(p.d_pleaf, p.n_pleaf, p.d_leafscan, p.d_feat,
                                                                    p.d_row_box, p.d_row_feat);
}

// the evaluation path after selector_reduce: rows, features, network and drop mask
void selector_decide(Plan &p, const void *I, const float *E, hipStream_t s)
{
    LeafArgs a = leaf_args(p, E);
    a.params = p.d_sel_params;
    a.threshold = p.sel_threshold;
    a.logits = p.d_logit;
    a.drop = p.d_drop;
    launch_leaf_pick(p, a, s);
    if (p.precision == PH_FP64) leaf_features_kernel<double, true><<<feature_blocks(p), 256, 0, s>>>(a, (const double *)I);
    else leaf_features_kernel<float, true><<<feature_blocks(p), 256, 0, s>>>(a, (const float *)I);
}

}  // namespace ph

extern "C" ph_status ph_selector_features(ph_plan *plan, const void *I, const float *absE, float *feats,
                                          int64_t cap_leaves, int64_t *n_leaves, void *stream)
{
    using namespace ph;
    if (!plan || !I || !n_leaves || cap_leaves < 0) {
        set_last_error("plan, I and n_leaves must be non-null and cap_leaves >= 0");
        return PH_EINVAL;
    }
    Plan &p = *reinterpret_cast<Plan *>(plan);
    try {
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PH_HIP(hipSetDevice(p.device));
        launch_reset_scalars(p.d_sc, nullptr, s);
        selector_reduce(p, I, absE, nullptr, s);
        selector_features(p, I, absE, s);
        int32_t nrow = 0;
        PH_HIP(hipMemcpyAsync(&nrow, &p.d_sc->n_srcleaf, 4, hipMemcpyDeviceToHost, s));
        PH_HIP(hipStreamSynchronize(s));
        *n_leaves = nrow;
        const int64_t k = std::min<int64_t>(nrow, cap_leaves);
        if (feats && k > 0)
            PH_HIP(hipMemcpyAsync(feats, p.d_row_feat, (size_t)k * 8 * 4, hipMemcpyDeviceToDevice, s));
        PH_HIP(hipStreamSynchronize(s));
        return PH_OK;
    } catch (const Error &e) {
        set_last_error(e.what);
        return e.status;
    }
}

extern "C" ph_status ph_selector_fields(ph_plan *plan, const void *I, const int32_t *targets, int64_t n_targets,
                                        float *out, int64_t ld, int64_t n_rows, void *stream)
{
    using namespace ph;
    if (!plan || !I || !targets || !out || n_targets < 1 || ld < n_targets || n_rows < 0) {
        set_last_error("bad selector_fields arguments (null pointer, n_targets < 1, ld < n_targets or n_rows < 0)");
        return PH_EINVAL;
    }
    Plan &p = *reinterpret_cast<Plan *>(plan);
    try {
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PH_HIP(hipSetDevice(p.device));
        int32_t nrow = 0;
        PH_HIP(hipMemcpyAsync(&nrow, &p.d_sc->n_srcleaf, 4, hipMemcpyDeviceToHost, s));
        PH_HIP(hipStreamSynchronize(s));
        if (n_rows > nrow) throw Error{PH_EINVAL, "n_rows exceeds the rows of the last ph_selector_features call"};
        if (n_rows == 0) return PH_OK;
        FieldArgs fa;
        fa.bx = p.box;
        fa.perm = p.d_perm;
        fa.iperm = p.d_iperm;
        fa.rows = p.d_row_box;
        fa.xyz = p.d_xyz;
        fa.w = p.d_w;
        fa.sc = p.d_sc;
        fa.w_ref = p.uniform_w ? p.w_uniform : 0.0;
        fa.c_self = p.c_self;
        fa.src_rel = p.thr.src_rel;
        fa.P = p.gas.P;
        const dim3 grid((unsigned)((n_targets + kFieldTargets - 1) / kFieldTargets), (unsigned)n_rows);
        if (p.precision == PH_FP64)
            fields_kernel<double><<<grid, 256, 0, s>>>(fa, make_kparams<double>(p.gas), (const double *)I, targets,
                                                       n_targets, out, ld);
        else
            fields_kernel<float><<<grid, 256, 0, s>>>(fa, make_kparams<float>(p.gas), (const float *)I, targets,
                                                      n_targets, out, ld);
        PH_HIP(hipGetLastError());
        PH_HIP(hipStreamSynchronize(s));
        return PH_OK;
    } catch (const Error &e) {
        set_last_error(e.what);
        return e.status;
    }
}
