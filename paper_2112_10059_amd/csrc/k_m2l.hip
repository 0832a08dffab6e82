// Downward pass: well-separated translations (M2L) as one MFMA GEMM per level,
// then a per-box gather that adds the parent's field (L2L) and coarse-leaf sources (P2L).
//
// For every well-separated offset t (316 per level) the translation is a dense
// n_lam x n_lam kernel matrix between lattices, K(c_B + h Lambda_i, c_A + h Lambda_j)
// with c_A - c_B = 2 h t (Sec. 2.4: far interactions through artificial sources).
// Stacking the 316 matrices gives M_all (316 n_lam x n_lam); for the boxes of a
// level that hold sources, Y = M_all * [phi_A ...] holds every translation a
// source box can send.  A target box B then sums, in a fixed candidate order,
// the columns Y[A][slot(A - B)] of its V list (children of the parent's
// colleagues that are not adjacent to B).  The GEMM runs on the matrix cores:
// computed as Y^T = Phi^T M_all^T so that each wave writes contiguous rows of Y.
#include <hip/hip_runtime.h>

#include "k_fmm_args.h"

namespace ph {

namespace {

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

constexpr int kTile = 64;     // tile of source boxes (rows of Y) and of stacked rows m
constexpr int kTK = kGemmK;   // K chunk staged in LDS
constexpr int kPad = 4;       // LDS row padding (bank spread)

// Y[col][m] = sum_k phi_{src_box(r0 + col)}[k] * M_all[m][k],  m < M = 316 n_lam
template <class T>
__global__ __launch_bounds__(256) void m2l_gemm_kernel(const T *__restrict__ M_all, int k_pad, int M, int nl,
                                                       const T *__restrict__ phi, const int32_t *__restrict__ src_box,
                                                       const CallScalars *__restrict__ sc, int level, int32_t lvl_base,
                                                       int32_t r0, int32_t ccap, T *__restrict__ Y)
{
    __shared__ T As[kTK][kTile + kPad];  // phi^T tile, k-major
    __shared__ T Bs[kTK][kTile + kPad];  // M_all^T tile, k-major
    const int32_t ns = sc->lvl_src[level];
    const int32_t ncols = min(ccap, ns - r0);
    const int m0 = blockIdx.x * kTile;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wn = w >> 1, wm = w & 1;
    using acc_t = typename Mfma<T>::acc_t;
    // blockIdx.y strides over the tiles of source boxes (a bounded grid for any count)
    for (int n0 = blockIdx.y * kTile; n0 < ncols; n0 += gridDim.y * kTile) {
    acc_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < k_pad; k0 += kTK) {
        __syncthreads();
        for (int e = t; e < kTK * kTile; e += 256) {
            const int n = e / kTK, k = e % kTK;
            const int gn = n0 + n, gk = k0 + k;
            T v = T(0);
            if (gn < ncols && gk < nl) v = phi[(size_t)src_box[lvl_base + r0 + gn] * nl + gk];
            As[k][n] = v;
            const int gm = m0 + n;
            Bs[k][n] = gm < M ? M_all[(size_t)gm * k_pad + gk] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kTK; ks += 4) {
            const int kk = ks + (lane >> 4);
            T a[2], b[2];
            for (int i = 0; i < 2; ++i) a[i] = As[kk][wn * 32 + i * 16 + (lane & 15)];
            for (int j = 0; j < 2; ++j) b[j] = Bs[kk][wm * 32 + j * 16 + (lane & 15)];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::mma(a[i], b[j], acc[i][j]);
        }
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int gm = m0 + wm * 32 + j * 16 + (lane & 15);
            for (int r = 0; r < 4; ++r) {
                const int gn = n0 + wn * 32 + i * 16 + Mfma<T>::row(lane, r);
                if (gn < ncols && gm < M) Y[(size_t)gn * M + gm] = acc[i][j][r];
            }
        }
    }
}

// u_B = [first chunk: l2l u_parent + X-list sources] + sum over V(B) in this chunk of Y
template <class T>
__global__ void down_gather_kernel(FmmArgs<T> a, int level, const T *__restrict__ Y, int M, int32_t r0,
                                   int32_t ccap, int first)
{
    const int32_t i = blockIdx.x;
    if (i >= a.sc->lvl_count[level]) return;
    const int32_t b = a.lt.base[level] + i;
    if (a.bx.t_cnt[b] == 0) return;
    const int32_t ns = a.sc->lvl_src[level];
    const int32_t ncols = min(ccap, ns - r0);
    if (!first && ncols <= 0) return;
    __shared__ T vec[kMaxLattice];
    __shared__ V4<T> tile[128];
    __shared__ int32_t cand[216];
    const int nl = a.n_lam;
    const size_t nn = (size_t)nl * nl;
    T acc[4] = {0, 0, 0, 0};
    unsigned long long n_m2l = 0, n_p2l = 0;
    const int32_t par = a.bx.parent[b];
    if (first) {
        if (level >= 3) {
            for (int li = threadIdx.x; li < nl; li += blockDim.x) vec[li] = a.u[(size_t)par * nl + li];
            __syncthreads();
            const int oct = ((a.bx.ax[b] & 1) << 2) | ((a.bx.ay[b] & 1) << 1) | (a.bx.az[b] & 1);
            const T *Ml = a.l2l + ((size_t)level * 8 + oct) * nn;
            for (int k = 0; k < 4; ++k) {
                const int li = threadIdx.x + k * blockDim.x;
                if (li >= nl) break;
                T s = 0;
                for (int j = 0; j < nl; ++j) s += Ml[(size_t)j * nl + li] * vec[j];
                acc[k] = s;
            }
        }
        // X list: sources of coarser leaves straight onto the check points
        const uint32_t x0 = a.L.x_off[b], x1 = a.L.x_off[b + 1];
        if (x1 > x0) {
            const double hw = a.lt.hw[level];
            T cx, cy, cz;
            box_centre(a, b, hw, cx, cy, cz);
            const T h = (T)hw;
            for (uint32_t e = x0; e < x1; ++e) {
                const int32_t C = a.L.x[e];
                const int32_t sf = a.bx.s_first[C], sn = a.bx.s_cnt[C];
                n_p2l += (unsigned long long)sn * nl;
                for (int base = 0; base < sn; base += 128) {
                    const int m = min(128, sn - base);
                    __syncthreads();
                    for (int q = threadIdx.x; q < m; q += blockDim.x) tile[q] = a.s_dat[sf + base + q];
                    __syncthreads();
                    for (int k = 0; k < 4; ++k) {
                        const int li = threadIdx.x + k * blockDim.x;
                        if (li >= nl) break;
                        const T px = cx + h * a.lat[3 * li], py = cy + h * a.lat[3 * li + 1],
                                pz = cz + h * a.lat[3 * li + 2];
                        T s = 0;
                        for (int j = 0; j < m; ++j) {
                            const V4<T> y = tile[j];
                            const T ddx = px - y.x, ddy = py - y.y, ddz = pz - y.z;
                            s += kernel_eval<true>(ddx * ddx + ddy * ddy + ddz * ddz, a.kp) * y.w;
                        }
                        acc[k] += s;
                    }
                }
            }
        }
    } else {
        for (int k = 0; k < 4; ++k) {
            const int li = threadIdx.x + k * blockDim.x;
            if (li < nl) acc[k] = a.u[(size_t)b * nl + li];
        }
    }
    // V list, resolved in parallel: candidate c = (parent colleague c/8, child octant c%8)
    const int bx0 = a.bx.ax[b], by0 = a.bx.ay[b], bz0 = a.bx.az[b];
    for (int c = threadIdx.x; c < 216; c += blockDim.x) {
        const int32_t P = a.bx.coll[(size_t)par * 27 + (c >> 3)];
        const int32_t A = P >= 0 ? a.bx.child[(size_t)P * 8 + (c & 7)] : -1;
        int32_t code = -1;
        if (A >= 0) {
            const int32_t rk = a.bx.src_rank[A] - r0;
            const int dx = a.bx.ax[A] - bx0, dy = a.bx.ay[A] - by0, dz = a.bx.az[A] - bz0;
            const bool far = !(dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1);
            if (far && a.bx.src_rank[A] >= 0 && rk >= 0 && rk < ncols) code = rk * kNumM2L + m2l_slot(dx, dy, dz);
        }
        cand[c] = code;
    }
    __syncthreads();
    for (int c = 0; c < 216; ++c) {
        const int32_t code = cand[c];
        if (code < 0) continue;
        ++n_m2l;
        const T *y = Y + (size_t)(code / kNumM2L) * M + (size_t)(code % kNumM2L) * nl;
        for (int k = 0; k < 4; ++k) {
            const int li = threadIdx.x + k * blockDim.x;
            if (li < nl) acc[k] += y[li];
        }
    }
    for (int k = 0; k < 4; ++k) {
        const int li = threadIdx.x + k * blockDim.x;
        if (li < nl) a.u[(size_t)b * nl + li] = acc[k];
    }
    if (a.work && threadIdx.x == 0) {
        if (n_m2l) atomicAdd(&a.work[5], n_m2l);
        if (n_p2l) atomicAdd(&a.work[4], n_p2l);
        if (first && level >= 3) atomicAdd(&a.work[7], 1ull);
    }
}

template <class T>
void fmm_downward_t(Plan &p, hipStream_t s)
{
    FmmArgs<T> a = make_args<T>(p);
    const int nl = p.n_lam;
    const int M = kNumM2L * nl;
    const int threads = nl <= 64 ? 64 : (nl <= 128 ? 128 : 256);
    for (int l = 2; l <= p.max_depth; ++l) {
        const int64_t cap = p.level_cap[l];
        const int64_t ccap = std::min<int64_t>((int64_t)p.y_cap_cols, cap);
        const int nchunk = (int)((cap + ccap - 1) / ccap);
        const T *Ml = (const T *)p.ops.m2l + (size_t)l * M * p.k_pad;
        for (int c = 0; c < nchunk; ++c) {
            const int32_t r0 = (int32_t)(c * ccap);
            dim3 g((M + kTile - 1) / kTile, (unsigned)std::min<int64_t>(32, (ccap + kTile - 1) / kTile));
            m2l_gemm_kernel<T><<<g, 256, 0, s>>>(Ml, p.k_pad, M, nl, (const T *)p.d_phi, p.box.src_box, p.d_sc, l,
                                                 (int32_t)p.level_base[l], r0, (int32_t)ccap, (T *)p.d_y);
            down_gather_kernel<T><<<(unsigned)cap, threads, 0, s>>>(a, l, (const T *)p.d_y, M, r0, (int32_t)ccap,
                                                                     c == 0 ? 1 : 0);
        }
    }
}

}  // namespace

void fmm_downward(Plan &p, hipStream_t s)
{
    if (p.precision == PH_FP64) fmm_downward_t<double>(p, s);
    else fmm_downward_t<float>(p, s);
}

}  // namespace ph
