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
#include "k_mlp_dev.h"

namespace ph {

namespace {

using namespace mlp;

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


// ---------------------------------------------------------------- selector rows and features
//
// The selector decides on the leaves of the plan's tree (the tree over all points, fixed at
// plan time): a row is a plan leaf holding at least one candidate source (I >= src_rel I_max,
// the plan's source rule), and a dropped row removes all its candidates from the call's source
// set.  On the evaluation path the decisions are made inside the selection pass; the training
// entry points below compute the same rows and features (the same device functions) over the
// plan leaves in box order.

namespace {

struct RowArgs {
    const int4 *pinfo, *pinfo2;  // per plan leaf: (box, first, end, 0), (anchor x, y, z, level)
    const int32_t *perm;
    const double *w;
    const CallScalars *sc;
    int32_t n_pleaf;
    double src_rel;
    mlp::FeatureRefs base;       // everything but the call's maxima and positions
    float *feats;
    uint32_t *flag, *flag2;
    int32_t *cnt;
};

// One wave per plan leaf (box order): its statistics (the same function as the evaluation
// path's), and for a candidate leaf its features; flag (and flag2, the compaction's copy) 1 for
// a candidate leaf, else 0.
template <class T>
__global__ __launch_bounds__(256) void leaf_rows_kernel(RowArgs a, const T *__restrict__ I, const float *__restrict__ E)
{
    mlp::FeatureRefs r = a.base;
    r.imax = a.sc->imax;
    r.emax = a.sc->emax;
    r.efeat = E && r.emax > 0.0;
    for (int d = 0; d < 3; ++d) {
        r.xi[d] = a.sc->imax_xyz[d];
        r.xe[d] = a.sc->emax_xyz[d];
    }
    const int lane = threadIdx.x & 63;
    const int32_t i = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (i == 0 && lane == 0 && a.flag2) a.flag2[a.n_pleaf] = 0;
    if (i >= a.n_pleaf) return;
    const int4 inf = a.pinfo[i], g = a.pinfo2[i];
    auto fetch = [&](int32_t k, double &v, double &e) {
        const int32_t o = a.perm[k];
        v = (double)I[o];
        e = E ? (double)E[o] : 0.0;
    };
    const mlp::LeafStats s = mlp::leaf_stats_wave(fetch, a.w, r.w_ref, inf.y, inf.z, a.src_rel, r.imax, lane);
    const bool cand = s.n_c > 0.0;
    if (cand) {
        float fe[PH_MLP_NIN];
        mlp::leaf_features(s, r, g.w, g.x, g.y, g.z, fe);
        if (lane < PH_MLP_NIN) {
            float f = fe[0];
#pragma unroll
            for (int q = 1; q < PH_MLP_NIN; ++q) f = lane == q ? fe[q] : f;
            a.feats[(size_t)i * PH_MLP_NIN + lane] = f;
        }
    }
    if (lane == 0) {
        a.flag[i] = cand ? 1u : 0u;
        if (a.flag2) a.flag2[i] = cand ? 1u : 0u;
        a.cnt[i] = (int32_t)s.n_c;
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

// rows and their features in box order (the maxima first, as the evaluation path finds them)
void selector_features(Plan &p, const void *I, const float *E, hipStream_t s)
{
    launch_reset_scalars(p.d_sc, nullptr, s);
    launch_reduce_max(p, I, E, nullptr, s);
    launch_maxima_store(p, E != nullptr, s);
    RowArgs a{};
    a.pinfo = p.d_pinfo;
    a.pinfo2 = p.d_pinfo2;
    a.perm = p.d_perm;
    a.w = p.d_w;
    a.sc = p.d_sc;
    a.n_pleaf = p.n_pleaf;
    a.src_rel = p.thr.src_rel;
    a.base.w_ref = p.uniform_w ? p.w_uniform : p.cube_size * p.cube_size * p.cube_size / (double)p.n;
    for (int d = 0; d < 3; ++d) a.base.lo[d] = p.cube_lo[d];
    a.base.cube = p.cube_size;
    a.feats = p.d_feat;
    a.flag = p.d_leafflag;
    a.flag2 = p.d_leafscan;
    a.cnt = p.d_feat_cnt;
    const unsigned g = (unsigned)((p.n_pleaf + 3) / 4);  // a wave per plan leaf
    if (p.precision == PH_FP64) leaf_rows_kernel<double><<<g, 256, 0, s>>>(a, (const double *)I, E);
    else leaf_rows_kernel<float><<<g, 256, 0, s>>>(a, (const float *)I, E);
    exclusive_scan_u32(p.d_leafscan, p.n_pleaf + 1, p.d_scan_tmp, reinterpret_cast<uint32_t *>(&p.d_sc->n_srcleaf), s);
    rows_kernel<<<(unsigned)((p.n_pleaf + 255) / 256), 256, 0, s>>>(p.d_pleaf, p.n_pleaf, p.d_leafscan, p.d_feat,
                                                                    p.d_row_box, p.d_row_feat);
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
