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

template <bool BF16>
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ params, const float *__restrict__ X,
                                                          int64_t m, float *__restrict__ logits)
{
    __shared__ float w[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = q<BF16>(params[i]);
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    float x[NIN];
    for (int k = 0; k < NIN; ++k) x[k] = q<BF16>(X[r * NIN + k]);
    float h1[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        float a = w[OFF_B1 + i];
        for (int k = 0; k < NIN; ++k) a += w[OFF_W1 + i * NIN + k] * x[k];
        h1[i] = q<BF16>(gelu(a));
    }
    float z = w[OFF_B3];
    for (int i = 0; i < NH; ++i) {
        float a = w[OFF_B2 + i];
#pragma unroll
        for (int j = 0; j < NH; ++j) a += w[OFF_W2 + i * NH + j] * h1[j];
        z += w[OFF_W3 + i] * q<BF16>(gelu(a));
    }
    logits[r] = z;
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

}  // namespace

void launch_mlp_forward(const float *params, const float *X, int64_t m, float *logits, int bf16, hipStream_t s)
{
    if (m == 0) return;
    const unsigned g = (unsigned)((m + 255) / 256);
    if (bf16) mlp_forward_kernel<true><<<g, 256, 0, s>>>(params, X, m, logits);
    else mlp_forward_kernel<false><<<g, 256, 0, s>>>(params, X, m, logits);
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

void launch_adam(float *params, float *m1, float *m2, const float *grad, int64_t n, float lr, float b1, float b2,
                 float eps, int64_t step, hipStream_t s)
{
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(params, m1, m2, grad, n, lr, b1, b2, eps, c1, c2);
}

// ---------------------------------------------------------------- selector rows and features

namespace {

__global__ void leaf_flag_kernel(BoxArrays bx, int32_t nbox, uint32_t *__restrict__ flag)
{
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f == 0) flag[nbox] = 0;
    if (f >= nbox) return;
    flag[f] = ((bx.flags[f] & kBoxLeaf) && bx.s_cnt[f] > 0) ? 1u : 0u;
}

__global__ void leaf_rows_kernel(int32_t nbox, const uint32_t *__restrict__ scanned, int32_t *__restrict__ rows,
                                 CallScalars *__restrict__ sc)
{
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f == 0) sc->n_srcleaf = (int32_t)scanned[nbox];
    if (f >= nbox) return;
    if (scanned[f + 1] != scanned[f]) rows[scanned[f]] = f;
}

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

struct FeatArgs {
    BoxArrays bx;
    const int32_t *s_pos, *perm, *rows;
    const double *xyz;
    const double *w;  // sorted quadrature weights, null on uniform grids (w = w_ref)
    const float *E;
    const CallScalars *sc;
    float *feats;
    double lo0, lo1, lo2, cube, w_ref;
    int64_t n;
};

// one wave per source leaf; the wave sums in a fixed lane/stride order
template <class T>
__global__ __launch_bounds__(256) void features_kernel(FeatArgs a, const T *__restrict__ I)
{
    const int lane = threadIdx.x & 63;
    const int32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= a.sc->n_srcleaf) return;
    const int32_t f = a.rows[r];
    const double imax = a.sc->imax, emax = a.sc->emax;
    const int level = a.bx.level[f];
    const double side = a.cube / (double)(1 << level), hw = 0.5 * side;
    const double cx = a.lo0 + (2.0 * a.bx.ax[f] + 1.0) * hw, cy = a.lo1 + (2.0 * a.bx.ay[f] + 1.0) * hw,
                 cz = a.lo2 + (2.0 * a.bx.az[f] + 1.0) * hw;
    // sources: max I and sum of w I over the leaf
    double mx = 0.0, swi = 0.0;
    const int32_t sf = a.bx.s_first[f], sn = a.bx.s_cnt[f];
    for (int32_t j = lane; j < sn; j += 64) {
        const int32_t k = a.s_pos[sf + j];
        const double v = (double)I[a.perm[k]];
        mx = fmax(mx, v);
        swi += v * (a.w ? a.w[k] : a.w_ref);
    }
    mx = wave_max(mx);
    swi = wave_sum(swi);
    float fe[8];
    fe[0] = (float)log10(fmax(mx / imax, 1e-300));
    fe[1] = (float)log10(fmax(swi / (imax * a.w_ref), 1e-300));
    fe[2] = (float)log2(side / cbrt(a.w_ref));
    for (int q = 3; q < 8; ++q) fe[q] = 0.0f;
    if (a.E && emax > 0.0) {
        const int64_t kp = a.n - a.sc->emax_pos_rev;
        const double dx = cx - a.xyz[3 * kp], dy = cy - a.xyz[3 * kp + 1], dz = cz - a.xyz[3 * kp + 2];
        fe[3] = (float)log10(1.0 + sqrt(dx * dx + dy * dy + dz * dz) / side);
        const int32_t st = a.bx.start[f], en = a.bx.end[f];
        double emx = 0.0, es = 0.0, es2 = 0.0;
        for (int32_t k = st + lane; k < en; k += 64) {
            const double e = (double)a.E[a.perm[k]] / emax;
            emx = fmax(emx, e);
            es += e;
            es2 += e * e;
        }
        emx = wave_max(emx);
        es = wave_sum(es);
        es2 = wave_sum(es2);
        const double cnt = (double)(en - st);
        const double mean = es / cnt;
        fe[4] = (float)emx;
        fe[5] = (float)mean;
        fe[6] = (float)sqrt(fmax(es2 / cnt - mean * mean, 0.0));
        double nmx = 0.0;
        for (int d = 0; d < 27; ++d) {
            const int32_t C = a.bx.coll[(size_t)f * 27 + d];
            if (C < 0) continue;
            const int32_t cs = a.bx.start[C], ce = a.bx.end[C];
            for (int32_t k = cs + lane; k < ce; k += 64) nmx = fmax(nmx, (double)a.E[a.perm[k]] / emax);
        }
        fe[7] = (float)wave_max(nmx);
    }
    if (lane < 8) a.feats[(size_t)r * 8 + lane] = fe[lane];
}

// ||field of leaf b||_2 over the sampled targets, in the units of S (one workgroup per row)
template <class T>
__global__ __launch_bounds__(256) void contrib_kernel(BoxArrays bx, const int32_t *__restrict__ rows,
                                                      const CallScalars *__restrict__ sc,
                                                      const V4<T> *__restrict__ s_dat, const int32_t *__restrict__ s_pos,
                                                      const int32_t *__restrict__ iperm, const double *__restrict__ xyz,
                                                      const int32_t *__restrict__ targets, int64_t nt, KParams<T> kp,
                                                      double c_self_over_w, double P, float *__restrict__ out,
                                                      int64_t cap)
{
    __shared__ V4<T> tile[256];
    __shared__ int32_t tpos[256];
    __shared__ double red[256];
    const int32_t r = blockIdx.x;
    if (r >= sc->n_srcleaf || r >= cap) return;
    const int32_t f = rows[r];
    const int32_t sf = bx.s_first[f], sn = bx.s_cnt[f];
    double acc = 0.0;
    for (int64_t t0 = 0; t0 < nt; t0 += 256) {
        const int64_t t = t0 + threadIdx.x;
        const bool act = t < nt;
        int32_t kt = 0;
        T x = 0, y = 0, z = 0;
        if (act) {
            kt = iperm[targets[t]];
            x = (T)xyz[3 * (int64_t)kt];
            y = (T)xyz[3 * (int64_t)kt + 1];
            z = (T)xyz[3 * (int64_t)kt + 2];
        }
        double sfield = 0.0;
        for (int base = 0; base < sn; base += 256) {
            const int m = min(256, sn - base);
            __syncthreads();
            if ((int)threadIdx.x < m) {
                tile[threadIdx.x] = s_dat[sf + base + threadIdx.x];
                tpos[threadIdx.x] = s_pos[sf + base + threadIdx.x];
            }
            __syncthreads();
            if (act)
                for (int j = 0; j < m; ++j) {
                    const V4<T> yj = tile[j];
                    const T dx = x - yj.x, dy = y - yj.y, dz = z - yj.z;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    if (tpos[j] == kt) sfield += c_self_over_w * (double)yj.w;
                    else if (r2 > T(0)) sfield += (double)(kernel_eval<true>(r2, kp) * yj.w);
                }
        }
        acc += sfield * sfield;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = (float)(sqrt(red[0]) * P * ldexp(1.0, sc->scale_exp));
}

__global__ void zero_bytes_kernel(uint8_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// keep a source leaf iff its logit >= threshold; sources of dropped leaves are marked.
// A non-finite logit switches the call to the threshold fallback.
__global__ void decide_kernel(BoxArrays bx, const int32_t *__restrict__ rows, const float *__restrict__ logits,
                              float thr, const int32_t *__restrict__ s_pos, uint8_t *__restrict__ drop,
                              CallScalars *__restrict__ sc)
{
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) sc->n_src_base = sc->n_src;
    if (r >= sc->n_srcleaf) return;
    const float z = logits[r];
    if (!isfinite(z)) {
        atomicOr(&sc->fallback, 1);
        return;
    }
    if (z >= thr) return;
    const int32_t f = rows[r];
    const int32_t sf = bx.s_first[f], sn = bx.s_cnt[f];
    for (int32_t j = 0; j < sn; ++j) drop[s_pos[sf + j]] = 1;
}

}  // namespace

void selector_features(Plan &p, const void *I, const float *E, hipStream_t s)
{
    const int32_t nbox = (int32_t)p.box_cap;
    const unsigned g = (unsigned)((nbox + 256) / 256);
    leaf_flag_kernel<<<g, 256, 0, s>>>(p.box, nbox, p.d_leafflag);
    exclusive_scan_u32(p.d_leafflag, nbox + 1, p.d_scan_tmp, nullptr, s);
    leaf_rows_kernel<<<g, 256, 0, s>>>(nbox, p.d_leafflag, p.d_feat_box, p.d_sc);
    FeatArgs fa;
    fa.bx = p.box;
    fa.s_pos = p.d_s_pos;
    fa.perm = p.d_perm;
    fa.rows = p.d_feat_box;
    fa.xyz = p.d_xyz;
    fa.w = p.d_w;
    fa.E = E;
    fa.sc = p.d_sc;
    fa.feats = p.d_feat;
    fa.lo0 = p.cube_lo[0];
    fa.lo1 = p.cube_lo[1];
    fa.lo2 = p.cube_lo[2];
    fa.cube = p.cube_size;
    fa.w_ref = p.uniform_w ? p.w_uniform : p.cube_size * p.cube_size * p.cube_size / (double)p.n;
    fa.n = p.n;
    const unsigned gr = (unsigned)((p.box_cap + 3) / 4);
    if (p.precision == PH_FP64) features_kernel<double><<<gr, 256, 0, s>>>(fa, (const double *)I);
    else features_kernel<float><<<gr, 256, 0, s>>>(fa, (const float *)I);
}

void selector_apply(Plan &p, const void *I, const float *E, void *S_out, hipStream_t s)
{
    selector_features(p, I, E, s);
    launch_mlp_forward(p.d_sel_params, p.d_feat, p.box_cap, p.d_logit, 1, s);
    zero_bytes_kernel<<<1024, 256, 0, s>>>(p.d_drop, p.n);
    decide_kernel<<<(unsigned)((p.box_cap + 255) / 256), 256, 0, s>>>(p.box, p.d_feat_box, p.d_logit,
                                                                       p.sel_threshold, p.d_s_pos, p.d_drop, p.d_sc);
    launch_select_flags(p, I, E, S_out, s, p.d_drop);
    exclusive_scan_u64(p.d_flag, p.n, p.d_scan_tmp, &p.d_sc->packed_total, s);
    launch_compact(p, I, s);
    build_tree(p, s);
}

}  // namespace ph

extern "C" ph_status ph_selector_features(ph_plan *plan, const void *I, const float *absE, float *feats,
                                          int64_t cap_leaves, int64_t *n_leaves, void *stream)
{
    using namespace ph;
    if (!plan || !I || !n_leaves) {
        set_last_error("plan, I and n_leaves must be non-null");
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
            PH_HIP(hipMemcpyAsync(feats, p.d_feat, (size_t)k * 8 * 4, hipMemcpyDeviceToDevice, s));
        PH_HIP(hipStreamSynchronize(s));
        return PH_OK;
    } catch (const Error &e) {
        set_last_error(e.what);
        return e.status;
    }
}

extern "C" ph_status ph_selector_contrib(ph_plan *plan, const int32_t *targets, int64_t n_targets, float *contrib,
                                         int64_t cap_rows, void *stream)
{
    using namespace ph;
    if (!plan || !targets || !contrib || n_targets < 1 || cap_rows < 0) {
        set_last_error("bad selector_contrib arguments");
        return PH_EINVAL;
    }
    Plan &p = *reinterpret_cast<Plan *>(plan);
    try {
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PH_HIP(hipSetDevice(p.device));
        const double csw = p.uniform_w && p.w_uniform > 0 ? p.c_self / p.w_uniform : 0.0;
        const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(p.box_cap, cap_rows));
        if (p.precision == PH_FP64)
            contrib_kernel<double><<<g, 256, 0, s>>>(p.box, p.d_feat_box, p.d_sc, (const double4 *)p.d_s_dat,
                                                     p.d_s_pos, p.d_iperm, p.d_xyz, targets, n_targets,
                                                     make_kparams<double>(p.gas), csw, p.gas.P, contrib, cap_rows);
        else
            contrib_kernel<float><<<g, 256, 0, s>>>(p.box, p.d_feat_box, p.d_sc, (const float4 *)p.d_s_dat, p.d_s_pos,
                                                    p.d_iperm, p.d_xyz, targets, n_targets,
                                                    make_kparams<float>(p.gas), csw, p.gas.P, contrib,
                                                    cap_rows);
        PH_HIP(hipGetLastError());
        PH_HIP(hipStreamSynchronize(s));
        return PH_OK;
    } catch (const Error &e) {
        set_last_error(e.what);
        return e.status;
    }
}
