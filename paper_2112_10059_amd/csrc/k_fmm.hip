// Upward pass, translations, downward pass and leaf evaluation of the adaptive FMM.
//
// Sec. 2.4: near interactions (eq. (16), box B and its neighbours) are summed
// exactly; far interactions go through artificial sources whose intensities
// solve the check-point fit of eq. (17), recursively over the octree.
// Representation per box of level l (half-width h_l, centre c):
//   phi  (upward)   : intensities of artificial sources at c + h_l * lattice   (n_lam)
//   u    (downward) : far-field values at the check points c + h_l * lattice   (n_lam)
//   psi  (leaf)     : uc2e_l^T u, intensities of artificial sources at c + h_l * shell (n_sig)
// Kernels:
//   p2m     leaf sources -> check values on the shell -> phi = uc2e_l * check
//   m2m     phi_parent = sum_c m2m_{l+1,c} phi_child_c
//   down    u_B = l2l_{l,oct} u_parent + sum_{A in V(B)} m2l_{l,A-B} phi_A + sum_{X(B)} K(lattice, y) q
//   leaf    targets of leaf B: K(x, shell) psi + sum_{W(B)} K(x, lattice_A) phi_A
//           + sum_{U(B)} K(x, y) q (Kahan in FP32) + own-cell term, combined in FP64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "k_fmm_args.h"

namespace ph {

namespace {

// ---------------------------------------------------------------- leaf evaluation

template <class T>
struct Acc;
template <>
struct Acc<float> {
    float s = 0.f, c = 0.f;  // Kahan sum and compensation
    __device__ __forceinline__ void add(float v)
    {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};
template <>
struct Acc<double> {
    double s = 0.0;
    __device__ __forceinline__ void add(double v) { s += v; }
    __device__ __forceinline__ double value() const { return s; }
};

// broadcast of lane j's value to the whole wave (scalar register)
__device__ __forceinline__ float lane_bcast(float v, int j)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ __forceinline__ double lane_bcast(double v, int j)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), j);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), j);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------- upward pass

constexpr int kUpThreads = 256;
constexpr int kUpGroups = kUpThreads / 64;

// Artificial sources of source leaf b (Sec. 2.4): on a grid level, phi = G q with G the
// level's lattice operator over the box's cells; elsewhere the sources' field at the check
// shell, then the level's pseudo-inverse.  Wave g takes every kUpGroups-th source (or check
// point) and the partial sums are added in wave order.
static_assert(kMaxShell <= 2 * kUpThreads, "two check points per thread");

template <class T>
__device__ void p2m_box(const FmmArgs<T> &a, int32_t b, int level, V4<T> *tile, int32_t *rloc, T *chk,
                        T (*part)[kMaxLattice])
{
    const int t = threadIdx.x, lane = t & 63, g = t >> 6;
    const int nl = a.n_lam, nk = (nl + 63) / 64;
    const int32_t sf = a.bx.s_first[b], sn = a.bx.s_cnt[b];
    const int gm = a.grid_m[level];
    T acc[kMaxLattice / 64];
#pragma unroll
    for (int k = 0; k < kMaxLattice / 64; ++k) acc[k] = T(0);
    if (gm > 0) {
        const T *G = a.grid_gt + a.grid_off[level];  // [cell][lambda]
        for (int base = 0; base < sn; base += 128) {
            const int m = min(128, sn - base);
            __syncthreads();
            if (t < m) {
                tile[t] = a.s_dat[sf + base + t];
                rloc[t] = local_cell(a, a.s_cell[sf + base + t], b, gm);
            }
            __syncthreads();
            for (int j = g; j < m; j += kUpGroups)
#pragma unroll
                for (int k = 0; k < kMaxLattice / 64; ++k) {
                    const int li = lane + 64 * k;
                    if (k < nk && li < nl) acc[k] += G[(size_t)rloc[j] * nl + li] * tile[j].w;
                }
        }
        if (a.work && t == 0) atomicAdd(&a.work[9], (unsigned long long)sn * nl);
    } else {
        const double hw = a.lt.hw[level];
        T cx, cy, cz;
        box_centre(a, b, hw, cx, cy, cz);
        const T h = (T)hw;
        // n_sig <= kMaxShell <= 2 kUpThreads: check points t and t + kUpThreads
        const bool own = t < a.n_sig, own2 = t + kUpThreads < a.n_sig;
        T px = 0, py = 0, pz = 0, qx = 0, qy = 0, qz = 0, s = 0, s2 = 0;
        if (own) {
            px = cx + h * a.shell[3 * t];
            py = cy + h * a.shell[3 * t + 1];
            pz = cz + h * a.shell[3 * t + 2];
        }
        if (own2) {
            const int u = t + kUpThreads;
            qx = cx + h * a.shell[3 * u];
            qy = cy + h * a.shell[3 * u + 1];
            qz = cz + h * a.shell[3 * u + 2];
        }
        for (int base = 0; base < sn; base += 128) {
            const int m = min(128, sn - base);
            __syncthreads();
            if (t < m) tile[t] = a.s_dat[sf + base + t];
            __syncthreads();
            if (own)
                for (int j = 0; j < m; ++j) {
                    const V4<T> y = tile[j];
                    const T dx = px - y.x, dy = py - y.y, dz = pz - y.z;
                    s += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * y.w;
                }
            if (own2)
                for (int j = 0; j < m; ++j) {
                    const V4<T> y = tile[j];
                    const T dx = qx - y.x, dy = qy - y.y, dz = qz - y.z;
                    s2 += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * y.w;
                }
        }
        if (own) chk[t] = s;
        if (own2) chk[t + kUpThreads] = s2;
        __syncthreads();
        const T *U = a.uc2e_cm + (size_t)level * a.n_sig * nl;  // [check point][lambda]
        for (int sg = g; sg < a.n_sig; sg += kUpGroups)
#pragma unroll
            for (int k = 0; k < kMaxLattice / 64; ++k) {
                const int li = lane + 64 * k;
                if (k < nk && li < nl) acc[k] += U[(size_t)sg * nl + li] * chk[sg];
            }
        if (a.work && t == 0) atomicAdd(&a.work[3], (unsigned long long)sn * a.n_sig);
    }
#pragma unroll
    for (int k = 0; k < kMaxLattice / 64; ++k) {
        const int li = lane + 64 * k;
        if (k < nk && li < nl) part[g][li] = acc[k];
    }
    __syncthreads();
    for (int li = t; li < nl; li += kUpThreads) {
        T v = part[0][li];
        for (int o = 1; o < kUpGroups; ++o) v += part[o][li];
        a.phi[(size_t)b * nl + li] = v;
    }
}

// P2M of every source leaf of levels >= 2 in one launch: the source boxes of those levels are
// dealt to the workgroups as one flat range (boxes that are not leaves get their densities
// from their children afterwards).
// The same launch also clears the check values of every box of levels >= 3 (u_zero .. u_end
// elements) where the per-level L2L runs: the downward gather then stores only the level-local
// parts of the boxes with a V or X list, and the L2L products add whatever their children
// hold.  (The composite L2L reads only the parts the gather wrote: an empty range there.)
template <class T>
__global__ __launch_bounds__(kUpThreads) void p2m_kernel(FmmArgs<T> a, int depth, int64_t u_zero, int64_t u_end)
{
    __shared__ V4<T> tile[128];
    __shared__ int32_t rloc[128];
    __shared__ T chk[kMaxShell];
    __shared__ T part[kUpGroups][kMaxLattice];
    for (int64_t i = u_zero + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < u_end;
         i += (int64_t)gridDim.x * blockDim.x)
        a.u[i] = T(0);
    static_assert(kMaxDepth + 2 <= 64, "a lane per level");
    // the call's per-level counts, lane l holding level l's (read once, picked by readlane)
    const int lane = threadIdx.x & 63;
    const int32_t src_l = lane < kMaxDepth + 2 ? a.sc->lvl_src[lane] : 0;
    for (int32_t idx = blockIdx.x;; idx += gridDim.x) {
        int level = -1;
        int32_t r = idx;
        for (int l = 2; l <= depth; ++l) {
            const int32_t c = __builtin_amdgcn_readlane(src_l, l);
            if (r < c) {
                level = l;
                break;
            }
            r -= c;
        }
        if (level < 0) break;
        const int32_t b = a.bx.src_box[a.lt.base[level] + r];
        if (a.bx.flags[b] & kBoxLeaf) p2m_box(a, b, level, tile, rloc, chk, part);
    }
}

// M2M for the split source boxes of one level when n_lam <= 64: one workgroup per parent, wave
// o translating the child in octant o (lane = parent lattice index; the octant's operator rows
// are read from L2 a batch at a time), the translations summed in octant order.
constexpr int kM2MThreads = 512;

template <class T>
__global__ __launch_bounds__(kM2MThreads) void m2m_kernel(FmmArgs<T> a, int level)
{
    __shared__ T mpart[8][64];
    __shared__ int32_t kids[8];
    const int t = threadIdx.x, lane = t & 63, o = t >> 6;
    const int nl = a.n_lam;
    for (int32_t rk = blockIdx.x; rk < a.sc->lvl_src[level]; rk += gridDim.x) {
        const int32_t P = a.bx.src_box[a.lt.base[level] + rk];
        // the children's indices loaded with the parent's flags (a leaf has none)
        const int32_t fl = a.bx.flags[P];
        const int32_t Ct = t < 8 ? a.bx.child[(size_t)P * 8 + t] : -1;
        if (fl & kBoxLeaf) continue;
        __syncthreads();  // the previous parent's kids and partial sums have been read
        if (t < 8) kids[t] = (Ct >= 0 && a.bx.s_cnt[Ct] > 0) ? Ct : -1;
        __syncthreads();
        const int32_t C = kids[o];
        T acc = T(0);
        if (C >= 0) {
            const T ph = lane < nl ? a.phi[(size_t)C * nl + lane] : T(0);
            const T *op = a.l2l + ((size_t)(level + 1) * 8 + o) * nl * a.k_pad;  // [child j][parent i]
            // rows addressed as a uniform row pointer plus the lane's 32-bit offset, so that a
            // batch in flight holds only the loaded values (the kernel runs beside the near
            // field, whose waves leave about 190 registers per SIMD)
            constexpr int kRB = sizeof(T) == 4 ? 32 : 16;  // operator rows in flight
            const unsigned ln = (unsigned)min(lane, nl - 1);
            const int kp = a.k_pad;
#pragma unroll 1
            for (int j0 = 0; j0 < nl; j0 += kRB) {
                T v[kRB];
#pragma unroll
                for (int u = 0; u < kRB; ++u) {
                    const T *row = op + (size_t)min(j0 + u, nl - 1) * kp;
                    v[u] = row[ln];
                }
#pragma unroll
                for (int u = 0; u < kRB; ++u)
                    if (j0 + u < nl) acc += v[u] * lane_bcast(ph, j0 + u);
            }
            if (lane >= nl) acc = T(0);
        }
        mpart[o][lane] = acc;
        __syncthreads();
        if (t < nl) {
            T v = T(0);
            int nc = 0;
            for (int q = 0; q < 8; ++q)
                if (kids[q] >= 0) {
                    v += mpart[q][t];
                    ++nc;
                }
            a.phi[(size_t)P * nl + t] = v;
            if (a.work && t == 0) atomicAdd(&a.work[6], (unsigned long long)nc);
        }
    }
}

// Output of a target whose sums are complete: S = P 2^e (far + near + own cell), in FP64.
template <class TO>
__device__ __forceinline__ void put_output(TO *__restrict__ S_out, int32_t o, double P, double tot, int scale_exp)
{
    S_out[o] = (TO)(P * ldexp(tot, scale_exp));
}

// Third strategy of Sec. 3: an upper bound of the W-list sources' field anywhere in leaf b.
// Box A of the W list (not adjacent to b) holds selected sources of total weighted strength
// Q_A; their field at any point of b is at most Q_A K(d_min), d_min the smallest distance
// between the two cubes, because K decreases with r.  Sum over A in FP64, in the units of the
// scaled strengths (2^-e).  At a target of b the W list is left out when this bound is below
// r_s times the rest of S there (far field, near field and own cell).
template <class T>
__device__ double w_list_bound(const FmmArgs<T> &a, int32_t b)
{
    const int lb = a.bx.level[b];
    const double hb = a.lt.hw[lb];
    const double cb0 = a.lo0 + (2.0 * a.bx.ax[b] + 1.0) * hb, cb1 = a.lo1 + (2.0 * a.bx.ay[b] + 1.0) * hb,
                 cb2 = a.lo2 + (2.0 * a.bx.az[b] + 1.0) * hb;
    double bound = 0.0;
    for (uint32_t e = a.L.w_rng[b].x; e < a.L.w_rng[b].y; ++e) {
        const int32_t A = a.L.w[e];
        const double ha = a.lt.hw[a.bx.level[A]];
        const double g0 = fmax(fabs(a.lo0 + (2.0 * a.bx.ax[A] + 1.0) * ha - cb0) - ha - hb, 0.0);
        const double g1 = fmax(fabs(a.lo1 + (2.0 * a.bx.ay[A] + 1.0) * ha - cb1) - ha - hb, 0.0);
        const double g2 = fmax(fabs(a.lo2 + (2.0 * a.bx.az[A] + 1.0) * ha - cb2) - ha - hb, 0.0);
        const int32_t s0 = a.bx.s_first[A], s1 = s0 + a.bx.s_cnt[A];
        double q = 0.0;
        for (int32_t j = s0; j < s1; ++j) q += (double)a.s_dat[j].w;
        const double d2 = g0 * g0 + g1 * g1 + g2 * g2;
        if (q > 0.0) bound += d2 > 0.0 ? q * kernel_eval<false>(d2, a.kp64) : INFINITY;
    }
    return bound;
}

// true when the W list of a leaf with bound bnd is left out at a target whose other terms sum
// to rest (scaled units); records the decision for the target (sorted point k)
template <class T>
__device__ __forceinline__ bool w_list_skipped(const FmmArgs<T> &a, double bnd, double rest, int32_t k)
{
    const bool skip = bnd < a.r_s * rest;
    if (a.rs_flag) a.rs_flag[k] = skip ? 1 : 0;
    return skip;
}

// The bounds of every target leaf with a W list (third strategy), before the far-field
// kernels read them: the leaves of the per-level grid segments and of the shell list
template <class T>
__global__ __launch_bounds__(256) void w_bound_kernel(FmmArgs<T> a, double *__restrict__ bound)
{
    const int32_t stride = (int32_t)(gridDim.x * blockDim.x), t0 = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    for (int32_t i = t0; i < a.sc->n_far_b; i += stride) {
        const int32_t b = a.L.far_b[i];
        if (a.L.w_rng[b].y > a.L.w_rng[b].x) bound[b] = w_list_bound(a, b);
    }
#pragma unroll
    for (int l = 0; l < kMaxDepth + 2; ++l) {
        if (l > a.lt.depth) break;
        const int32_t n = a.sc->n_far_a_lvl[l], base = a.lt.base[l];
        for (int32_t i = t0; i < n; i += stride) {
            const int4 en = a.L.far_a[base + i];
            if (en.w & 2) bound[en.x] = w_list_bound(a, en.x);
        }
    }
}

// W list of target leaf b for the lanes' targets: artificial sources of smaller non-adjacent
// boxes.  The wave holds the source box's densities in registers, lane li of slot k holding
// phi[64 k + li], and broadcasts them lane by lane.
template <class T, int NK>
__device__ __forceinline__ T w_list_far(const FmmArgs<T> &a, int32_t b, const V4<T> &x, bool act, int lane)
{
    T far = 0;
    const uint32_t w0 = a.L.w_rng[b].x, w1 = a.L.w_rng[b].y;
    const int nl = a.n_lam;
    for (uint32_t e = w0; e < w1; ++e) {
        const int32_t A = a.L.w[e];
        const double hwa = a.lt.hw[a.bx.level[A]];
        T ax, ay, az;
        box_centre(a, A, hwa, ax, ay, az);
        const T ha = (T)hwa;
        T ph[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) ph[k] = 64 * k + lane < nl ? a.phi[(size_t)A * nl + 64 * k + lane] : T(0);
#pragma unroll
        for (int k = 0; k < NK; ++k)
            for (int j = 0; j < 64 && 64 * k + j < nl; ++j) {
                const int li = 64 * k + j;
                const T wv = lane_bcast(ph[k], j);
                const T dx = x.x - (ax + ha * a.lat[3 * li]);
                const T dy = x.y - (ay + ha * a.lat[3 * li + 1]);
                const T dz = x.z - (az + ha * a.lat[3 * li + 2]);
                if (act) far += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * wv;
            }
    }
    return far;
}

// This workgroup's level and the first entry of its slice of that level's far_a segment, for
// the levels in mask, at per leaves per workgroup; false if the workgroup has no slice.
__device__ __forceinline__ bool far_slice(const CallScalars *sc, int depth, uint32_t mask, int per, int32_t slice,
                                          int &level, int32_t &first)
{
    int32_t cnt[kMaxDepth + 2];
#pragma unroll
    for (int l = 0; l < kMaxDepth + 2; ++l) cnt[l] = sc->n_far_a_lvl[l];  // loads issued together
    int32_t acc = 0;
#pragma unroll
    for (int l = 0; l < kMaxDepth + 2; ++l) {
        if (l > depth || !((mask >> l) & 1u)) continue;
        const int32_t nb = (cnt[l] + per - 1) / per;
        if (slice < acc + nb) {
            level = l;
            first = (slice - acc) * per;
            return true;
        }
        acc += nb;
    }
    return false;
}

// Far field of grid-operator leaves with n_lam <= 64 and at most 4^3 cells (FP32), on the
// matrix cores.  A workgroup takes kFarMLeaves leaves of one level: with their check values
// U (leaves x n_lam) in LDS and the level operator G (n_lam x cells) read by each wave as its
// MFMA operand fragment, C = U G is a 16 x 64 x 64 product (wave j: the 16 x 16 tile of cells 16 j .. 16 j + 15,
// v_mfma_f32_16x16x4_f32 over k), written back to LDS; then the 256 threads walk the
// workgroup's points (each leaf's sorted range) in one flat range, their loads issued
// together, and finish the targets among them as the wave kernel does (far = C[leaf][cell],
// W list, near field, own cell, output).  Many small
// workgroups keep many dependent load chains in flight.
constexpr int kFarMLeaves = 16;

template <class TO>
__device__ void far_mfma_body(const FmmArgs<float> &a, TO *__restrict__ S_out, const double *__restrict__ t_near,
                              uint32_t level_mask, int32_t bid)
{
    __shared__ float Us[kFarMLeaves][65];  // U, then C = U G
    __shared__ int32_t lbox[kFarMLeaves], lt0[kFarMLeaves], loff[kFarMLeaves + 1];
    __shared__ int32_t lorg[kFarMLeaves][3];  // the leaves' first cells (anchor * m)
    __shared__ uint8_t lnear[kFarMLeaves], lw[kFarMLeaves];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int level;
    int32_t first;
    if (!far_slice(a.sc, a.lt.depth, level_mask, kFarMLeaves, bid, level, first)) return;
    const int32_t cnt = min(kFarMLeaves, a.sc->n_far_a_lvl[level] - first);
    const int nl = a.n_lam;
    const int gm = level >= 2 ? a.grid_m[level] : 0;  // 0: no far field at this level
    const int R = gm * gm * gm;
    const float *G = a.grid_g + a.grid_off[level];
    // this wave's B operand straight from memory, all 16 loads in flight at once: lane l holds
    // G[4 kk + l / 16][16 w + l % 16] for step kk of the product
    float gb[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        const int li = 4 * kk + (lane >> 4), c = 16 * w + (lane & 15);
        gb[kk] = (li < nl && c < R) ? G[li * R + c] : 0.0f;
    }
    if (w == 0 && lane < kFarMLeaves) {
        const bool valid = lane < cnt;
        const int4 en = valid ? a.L.far_a[a.lt.base[level] + first + lane] : make_int4(-1, 0, 0, 0);
        lbox[lane] = en.x;
        lt0[lane] = en.y;
        lnear[lane] = (en.w & 1) != 0;
        lw[lane] = (en.w & 2) != 0;
        // inclusive scan of the target counts over the 16 lanes
        int32_t v = en.z;
        for (int o = 1; o < kFarMLeaves; o <<= 1) {
            const int32_t y = __shfl_up(v, o, kFarMLeaves);
            if (lane >= o) v += y;
        }
        loff[lane + 1] = v;
        if (lane == 0) loff[0] = 0;
        const int32_t b = en.x;
        lorg[lane][0] = b >= 0 ? a.bx.ax[b] * gm : 0;
        lorg[lane][1] = b >= 0 ? a.bx.ay[b] * gm : 0;
        lorg[lane][2] = b >= 0 ? a.bx.az[b] * gm : 0;
    }
    __syncthreads();
    const int32_t total = loff[cnt];
    // the points' data (issued with the check values: one round trip for both)
    constexpr int kU = 4;  // points per thread, kU x 256 >= kFarMLeaves x 64
    const int32_t *__restrict__ pcell = a.pcell;
    const int32_t *__restrict__ perm = a.perm;
    const uint8_t *__restrict__ sel = a.sel;
    // per point only what the product's registers leave room for (the sorted position is
    // recomputed from the leaf, the flags ride in the top bits of the cell, the near-field sum
    // is read after the product): held across it, more would spill to scratch memory
    int32_t q[kU], k[kU], cell[kU], out[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int32_t f = u * 256 + t;
        q[u] = -1;
        if (f < total) {
            // the leaf of flat point f: the last q with loff[q] <= f
            int lo = 0, hi = cnt - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (loff[mid] <= f) lo = mid;
                else hi = mid - 1;
            }
            q[u] = lo;
            k[u] = lt0[lo] + (f - loff[lo]);
        }
    }
    constexpr int kUR = kFarMLeaves * 64 / 256;  // check values per thread
    float uv[kUR];
#pragma unroll
    for (int r = 0; r < kUR; ++r) {
        const int i = t + 256 * r, qq = i >> 6, li = i & 63;
        const int32_t b = lbox[qq];
        uv[r] = (b >= 0 && li < nl) ? a.u[(size_t)b * nl + li] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
        if (q[u] >= 0) {
            // cells pack three 10-bit coordinates: the two flag bits go above them
            cell[u] = (gm > 0 ? pcell[k[u]] : 0) | ((int32_t)sel[k[u]] << 30);
            out[u] = perm[k[u]];
        }
#pragma unroll
    for (int r = 0; r < kUR; ++r) Us[(t + 256 * r) >> 6][(t + 256 * r) & 63] = uv[r];
    __syncthreads();
    f32x4 acc = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < 64; k0 += 4)
        acc = Mfma<float>::mma(Us[lane & 15][k0 + (lane >> 4)], gb[k0 / 4], acc);
    __syncthreads();  // every wave has read U
#pragma unroll
    for (int r = 0; r < 4; ++r) Us[Mfma<float>::row(lane, r)][16 * w + (lane & 15)] = acc[r];
    __syncthreads();
    const int scale_exp = a.sc->scale_exp;
    auto finish = [&](int qq, int32_t cl, int32_t ot, int32_t kk, uint32_t sbit, double tnr) {
        cl &= 0x3fffffff;
        if (!(sbit & 2u)) return;  // not a target (its output was cleared at selection)
        const int32_t b = lbox[qq];
        float far = 0.0f;
        if (gm > 0) {
            const int i = (cl & 1023) - lorg[qq][0], j = ((cl >> 10) & 1023) - lorg[qq][1],
                      kz = ((cl >> 20) & 1023) - lorg[qq][2];
            far = Us[qq][(i * gm + j) * gm + kz];
        }
        const double rest = (double)far + tnr + own_term(a, sbit, ot, scale_exp);
        const bool skip_w = lw[qq] && a.r_s > 0.0 && w_list_skipped(a, a.rs_bound[b], rest, kk);
        if (lw[qq] && !skip_w) {
            // W list (rare on grids): the source boxes' lattice densities, one thread per target
            const V4<float> xx = point_xyz(a, kk);
            for (uint32_t e = a.L.w_rng[b].x; e < a.L.w_rng[b].y; ++e) {
                const int32_t A = a.L.w[e];
                const double hwa = a.lt.hw[a.bx.level[A]];
                float ax, ay, az;
                box_centre(a, A, hwa, ax, ay, az);
                const float ha = (float)hwa;
                for (int li = 0; li < nl; ++li) {
                    const float dx = xx.x - (ax + ha * a.lat[3 * li]);
                    const float dy = xx.y - (ay + ha * a.lat[3 * li + 1]);
                    const float dz = xx.z - (az + ha * a.lat[3 * li + 2]);
                    far += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * a.phi[(size_t)A * nl + li];
                }
            }
        }
        const double tot = lw[qq] && !skip_w ? (double)far + tnr + own_term(a, sbit, ot, scale_exp) : rest;
        S_out[ot] = (TO)(a.P * ldexp(tot, scale_exp));
    };
    double tnear[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int32_t kk = q[u] >= 0 ? lt0[q[u]] + (u * 256 + t - loff[q[u]]) : 0;
        tnear[u] = (q[u] >= 0 && lnear[q[u]]) ? t_near[kk] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
        if (q[u] >= 0)
            finish(q[u], cell[u], out[u], lt0[q[u]] + (u * 256 + t - loff[q[u]]), (uint32_t)cell[u] >> 30, tnear[u]);
    // points beyond the first kU x 256 (leaves of levels without an operator may hold more)
    for (int32_t f = kU * 256 + t; f < total; f += 256) {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (loff[mid] <= f) lo = mid;
            else hi = mid - 1;
        }
        const int32_t kk = lt0[lo] + (f - loff[lo]);
        finish(lo, gm > 0 ? pcell[kk] : 0, perm[kk], kk, sel[kk], lnear[lo] ? t_near[kk] : 0.0);
    }
    if (a.work && t < cnt) {
        const int32_t b = lbox[t];
        const int32_t tn = a.bx.t_cnt[b];  // targets (the entry counts all the leaf's points)
        unsigned long long near_src = 0, tab_src = 0;
        const bool tab_b = a.near_tab != nullptr && a.bx.level[b] == a.near_level;
        for (uint32_t e = a.L.u_rng[b].x; e < a.L.u_rng[b].y; ++e) {
            const int32_t C = a.L.u[e];
            near_src += a.bx.s_cnt[C];
            if (tab_b && a.bx.level[C] == a.near_level) tab_src += a.bx.s_cnt[C];
        }
        atomicAdd(&a.work[0], near_src * tn);
        if (tab_src) atomicAdd(&a.work[11], tab_src * tn);
        if (lnear[t]) atomicAdd(&a.work[10], (unsigned long long)tn);
        if (gm > 0) atomicAdd(&a.work[8], (unsigned long long)tn * nl);
        const uint32_t nw = a.L.w_rng[b].y - a.L.w_rng[b].x;
        if (nw) atomicAdd(&a.work[2], (unsigned long long)nw * nl * tn);
    }
}

// Far field of the target leaves whose level has a grid operator (uniform grids).  A workgroup
// takes up to kFarLeaves leaves of one level (the list's per-level segments), stages that
// level's operator G_l (n_lam x m^3) in LDS once, and gives one wave per leaf:
// far(t) = sum_li G_l[li][cell(t)] u[li], with the leaf's u in registers (lane li of slot k
// holds u[64 k + li]) broadcast lane by lane, plus the W list, the near field of leaves with a
// U list (computed beforehand) and the own-cell term, which gives the output.  Leaves of more
// than 64 points (m^3 > 64: coarse leaves, where a target rule leaves few targets in a box) are
// shared out instead: a workgroup takes one leaf and a group of four of its 64-point chunks, a
// chunk per wave, so that a few coarse leaves do not hold the whole launch one wave each.
constexpr int kFarLeaves = 4;      // leaves per workgroup: one per wave, all in flight at once
constexpr int kGridStage = 8192;   // operator entries staged in LDS (larger operators stay in L2)

// 64-point chunks of a leaf of a level with m cells per axis, and groups of four of them
__host__ __device__ __forceinline__ int far_chunks(int m) { return m > 0 ? (m * m * m + 63) / 64 : 1; }
__host__ __device__ __forceinline__ int far_groups(int m) { return (far_chunks(m) + 3) / 4; }

// This workgroup's level and its slice of that level's far_a segment for the wave kernel: up to
// kFarLeaves leaves from the first (group -1), or, on levels whose leaves span several chunks,
// the leaf first and its chunk group; false if the workgroup has no slice.
template <class T>
__device__ __forceinline__ bool far_slice_w(const FmmArgs<T> &a, uint32_t mask, int32_t slice, int &level,
                                            int32_t &first, int &group)
{
    int32_t cnt[kMaxDepth + 2];
#pragma unroll
    for (int l = 0; l < kMaxDepth + 2; ++l) cnt[l] = a.sc->n_far_a_lvl[l];  // loads issued together
    int32_t acc = 0;
#pragma unroll
    for (int l = 0; l < kMaxDepth + 2; ++l) {
        if (l > a.lt.depth || !((mask >> l) & 1u)) continue;
        const int gm = l >= 2 ? a.grid_m[l] : 0;
        const int gr = far_chunks(gm) > 1 ? far_groups(gm) : 0;
        const int32_t nb = gr > 0 ? cnt[l] * gr : (cnt[l] + kFarLeaves - 1) / kFarLeaves;
        if (slice < acc + nb) {
            level = l;
            if (gr > 0) {
                first = (slice - acc) / gr;
                group = (slice - acc) % gr;
            } else {
                first = (slice - acc) * kFarLeaves;
                group = -1;
            }
            return true;
        }
        acc += nb;
    }
    return false;
}

template <class T, int NK, bool LDSG>
__device__ __forceinline__ T grid_far(const T *__restrict__ G, int R, int nl, int r, const T (&uv)[NK])
{
    // four independent partial sums (latency), added in a fixed order
    T f4[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < NK; ++k)
#pragma unroll 16
        for (int j = 0; j < 64; ++j)
            if (64 * k + j < nl) f4[j & 3] += G[(64 * k + j) * R + r] * lane_bcast(uv[k], j);
    return (f4[0] + f4[1]) + (f4[2] + f4[3]);
}

// The body as a workgroup function: workgroup bid of nblk taking part, Gs the LDS staging area
template <class T, class TO, int NK>
__device__ void far_grid_body(const FmmArgs<T> &a, TO *__restrict__ S_out, const double *__restrict__ t_near,
                              int stage_cap, uint32_t level_mask, int32_t bid, int32_t nblk, T *Gs)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // slices of the per-level leaf lists, grid-stride (a small grid costs little when the lists
    // are empty)
    for (int32_t slice = bid;; slice += nblk) {
        int level, group;
        int32_t first;
        if (!far_slice_w(a, level_mask, slice, level, first, group)) return;  // the whole workgroup
        if (slice != bid) __syncthreads();  // the previous slice is done with Gs
        // group < 0: up to kFarLeaves leaves, a wave each, every chunk; else the leaf first, the
        // chunk 4 group + w of it for wave w
        const int32_t cnt = group < 0 ? min(kFarLeaves, a.sc->n_far_a_lvl[level] - first) : 1;
        const int nl = a.n_lam;
        const int gm = level >= 2 ? level_pick(a.grid_m, level) : 0;
        const int R = gm * gm * gm;
        const int64_t goff = level_pick(a.grid_off, level);
        const T *G = a.grid_g + goff;
        const bool staged = gm > 0 && nl * R <= stage_cap;
        if (staged) {
            // 16-byte loads, all issued before any store (one round trip to L2, not one per element);
            // the level offsets are multiples of 16 bytes whenever n_lam m^3 is a multiple of 4
            const int ne = nl * R;
            if ((ne & 3) == 0 && (goff & 3) == 0) {
                using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
                constexpr int per = 16 / sizeof(T);
                const V *src = reinterpret_cast<const V *>(G);
                V *dst = reinterpret_cast<V *>(Gs);
                const int nv = ne / per;
                V buf[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    // an index clamped into the operator keeps every load unconditional
                    const int i = min((int)(threadIdx.x + u * blockDim.x), nv - 1);
                    buf[u] = src[i];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = threadIdx.x + u * blockDim.x;
                    if (i < nv) dst[i] = buf[u];
                }
                for (int i = threadIdx.x + 8 * blockDim.x; i < nv; i += blockDim.x) dst[i] = src[i];
            } else {
                for (int i = threadIdx.x; i < ne; i += blockDim.x) Gs[i] = G[i];
            }
            __syncthreads();
        }
        const int scale_exp = a.sc->scale_exp;
        for (int32_t q = group < 0 ? w : 0; q < cnt; q += 4) {
            const int32_t b = a.L.far_a[level_pick(a.lt.base, level) + first + q].x;
            T uv[NK];
#pragma unroll
            for (int k = 0; k < NK; ++k)
                uv[k] = (gm > 0 && 64 * k + lane < nl) ? a.u[(size_t)b * nl + 64 * k + lane] : T(0);
            const int32_t p0 = a.bx.start[b], np = a.bx.end[b] - p0, tn = a.bx.t_cnt[b];
            const bool near = a.L.u_rng[b].y > a.L.u_rng[b].x;
            const bool has_w = a.L.w_rng[b].y > a.L.w_rng[b].x;
            const double bnd = (has_w && a.r_s > 0.0) ? a.rs_bound[b] : 0.0;
            if (a.work && lane == 0 && (group < 0 || (group == 0 && w == 0))) {  // once per leaf
                unsigned long long near_src = 0;
                for (uint32_t e = a.L.u_rng[b].x; e < a.L.u_rng[b].y; ++e) near_src += a.bx.s_cnt[a.L.u[e]];
                atomicAdd(&a.work[0], near_src * tn);
                if (near) atomicAdd(&a.work[10], (unsigned long long)tn);
                if (gm > 0) atomicAdd(&a.work[8], (unsigned long long)tn * nl);
                if (has_w) atomicAdd(&a.work[2], (unsigned long long)(a.L.w_rng[b].y - a.L.w_rng[b].x) * nl * tn);
            }
            // the leaf's points in sorted order, the targets among them flagged: every chunk, or
            // chunk 4 group + w and those a whole round of the leaf's groups later (none when a
            // leaf holds at most m^3 points)
            const int tb0 = group < 0 ? 0 : 64 * (4 * group + w), tstep = group < 0 ? 64 : 256 * far_groups(gm);
            for (int tb = tb0; tb < np; tb += tstep) {
                const int32_t k = p0 + tb + lane;
                const uint32_t sb = tb + lane < np ? a.sel[k] : 0u;
                const bool act = (sb & 2u) != 0;
                V4<T> x;
                if (act && has_w) x = point_xyz(a, k);
                else x.x = x.y = x.z = x.w = T(0);
                T far = 0;
                if (gm > 0) {
                    const int r = act ? local_cell(a, a.pcell[k], b, gm) : 0;
                    far = staged ? grid_far<T, NK, true>(Gs, R, nl, r, uv) : grid_far<T, NK, false>(G, R, nl, r, uv);
                }
                bool skip_w = false;
                if (has_w && a.r_s > 0.0 && act) {
                    const double rest = (double)far + (near ? t_near[k] : 0.0) + own_term(a, sb, a.perm[k], scale_exp);
                    skip_w = w_list_skipped(a, bnd, rest, k);
                }
                if (has_w) far += w_list_far<T, NK>(a, b, x, act && !skip_w, lane);
                if (act) {
                    const int32_t o = a.perm[k];
                    put_output(S_out, o, a.P, (double)far + (near ? t_near[k] : 0.0) + own_term(a, sb, o, scale_exp),
                               scale_exp);
                }
            }
        }
    }
}

// Far field of the other target leaves (point clouds, or grid levels without an operator),
// one workgroup per leaf over the list: the leaf's check values give the intensities of its
// shell points, which are then evaluated at every target; plus the W list and the own cell.
// The body as a workgroup function (any workgroup size): workgroup bid of nblk taking part
template <class T, class TO>
__device__ void far_shell_body(const FmmArgs<T> &a, TO *__restrict__ S_out, const double *__restrict__ t_near,
                               int32_t bid, int32_t nblk)
{
    __shared__ T uvec[kMaxLattice];
    __shared__ T wphi[kMaxLattice];
    __shared__ V4<T> shp[kMaxShell];  // shell point position and its intensity
    const int32_t n = a.sc->n_far_b;
    const int nl = a.n_lam, ns = a.n_sig;
    const int scale_exp = a.sc->scale_exp;
    for (int32_t idx = bid; idx < n; idx += nblk) {
        const int32_t b = a.L.far_b[idx];
        const int level = a.bx.level[b];
        const bool has_far = level >= 2;
        const double hw = a.lt.hw[level];
        T cx, cy, cz;
        box_centre(a, b, hw, cx, cy, cz);
        const T h = (T)hw;
        __syncthreads();  // the previous leaf's use of the shared arrays is over
        if (has_far) {
            for (int li = threadIdx.x; li < nl; li += blockDim.x) uvec[li] = a.u[(size_t)b * nl + li];
            __syncthreads();
            const T *U = a.uc2e_rm + (size_t)level * nl * ns;
            for (int sg = threadIdx.x; sg < ns; sg += blockDim.x) {
                T s = 0;
                for (int li = 0; li < nl; ++li) s += U[(size_t)li * ns + sg] * uvec[li];
                V4<T> q;
                q.x = cx + h * a.shell[3 * sg];
                q.y = cy + h * a.shell[3 * sg + 1];
                q.z = cz + h * a.shell[3 * sg + 2];
                q.w = s;
                shp[sg] = q;
            }
            __syncthreads();
        }
        const int32_t p0 = a.bx.start[b], np = a.bx.end[b] - p0, tn = a.bx.t_cnt[b];
        const uint32_t u0 = a.L.u_rng[b].x, u1 = a.L.u_rng[b].y;
        const uint32_t w0 = a.L.w_rng[b].x, w1 = a.L.w_rng[b].y;
        const double bnd = (w1 > w0 && a.r_s > 0.0) ? a.rs_bound[b] : 0.0;
        if (a.work && threadIdx.x == 0) {
            unsigned long long near_src = 0;
            for (uint32_t e = u0; e < u1; ++e) near_src += a.bx.s_cnt[a.L.u[e]];
            atomicAdd(&a.work[0], near_src * tn);
            if (u1 > u0) atomicAdd(&a.work[10], (unsigned long long)tn);
            if (has_far) atomicAdd(&a.work[1], (unsigned long long)tn * ns);
            if (w1 > w0) atomicAdd(&a.work[2], (unsigned long long)(w1 - w0) * nl * tn);
        }
        // the leaf's points in sorted order, the targets among them flagged
        for (int tb = 0; tb < np; tb += blockDim.x) {
            const int32_t k = p0 + tb + threadIdx.x;
            const uint32_t sb = tb + (int)threadIdx.x < np ? a.sel[k] : 0u;
            const bool act = (sb & 2u) != 0;
            V4<T> x;
            if (act) x = point_xyz(a, k);
            else x.x = x.y = x.z = x.w = T(0);
            T far = 0;
            if (has_far && act)
                for (int sg = 0; sg < ns; ++sg) {
                    const V4<T> q = shp[sg];
                    const T dx = x.x - q.x, dy = x.y - q.y, dz = x.z - q.z;
                    far += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * q.w;
                }
            bool skip_w = false;
            if (w1 > w0 && a.r_s > 0.0 && act) {
                const double rest = (double)far + (u1 > u0 ? t_near[k] : 0.0) + own_term(a, sb, a.perm[k], scale_exp);
                skip_w = w_list_skipped(a, bnd, rest, k);
            }
            for (uint32_t e = w0; e < w1; ++e) {
                const int32_t A = a.L.w[e];
                const double hwa = a.lt.hw[a.bx.level[A]];
                T ax, ay, az;
                box_centre(a, A, hwa, ax, ay, az);
                const T ha = (T)hwa;
                __syncthreads();
                for (int li = threadIdx.x; li < nl; li += blockDim.x) wphi[li] = a.phi[(size_t)A * nl + li];
                __syncthreads();
                if (act && !skip_w)
                    for (int li = 0; li < nl; ++li) {
                        const T dx = x.x - (ax + ha * a.lat[3 * li]);
                        const T dy = x.y - (ay + ha * a.lat[3 * li + 1]);
                        const T dz = x.z - (az + ha * a.lat[3 * li + 2]);
                        far += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * wphi[li];
                    }
            }
            if (act) {
                const int32_t o = a.perm[k];
                put_output(S_out, o, a.P, (double)far + (u1 > u0 ? t_near[k] : 0.0) + own_term(a, sb, o, scale_exp),
                           scale_exp);
            }
        }
    }
}

template <class T, class TO, int NK>
__global__ __launch_bounds__(256) void far_grid_kernel(FmmArgs<T> a, TO *__restrict__ S_out,
                                                       const double *__restrict__ t_near,
                                                       int stage_cap, uint32_t level_mask)
{
    extern __shared__ __align__(16) unsigned char far_lds[];  // stage_cap operator entries
    far_grid_body<T, TO, NK>(a, S_out, t_near, stage_cap, level_mask, (int32_t)blockIdx.x, (int32_t)gridDim.x,
                             reinterpret_cast<T *>(far_lds));
}

template <class T, class TO>
__global__ void far_shell_kernel(FmmArgs<T> a, TO *__restrict__ S_out, const double *__restrict__ t_near)
{
    far_shell_body<T, TO>(a, S_out, t_near, (int32_t)blockIdx.x, (int32_t)gridDim.x);
}

// The far field of every kind of grid leaf in one launch (uniform grids): the first g_mfma
// workgroups take the matrix-core leaves (FP32), the next g_grid the other grid-operator
// leaves, the rest the shell-point leaves
template <class T, class TO, int NK>
__global__ __launch_bounds__(256, 8) void far_rest_kernel(FmmArgs<T> a, TO *__restrict__ S_out,
                                                       const double *__restrict__ t_near, int stage_cap,
                                                       uint32_t level_mask, uint32_t mfma_mask, int32_t g_mfma,
                                                       int32_t g_grid)
{
    extern __shared__ __align__(16) unsigned char far_lds[];
    if ((int32_t)blockIdx.x < g_mfma) {
        if constexpr (std::is_same<T, float>::value)
            far_mfma_body<TO>(a, S_out, t_near, mfma_mask, (int32_t)blockIdx.x);
        return;
    }
    const int32_t bid = (int32_t)blockIdx.x - g_mfma;
    if (bid < g_grid)
        far_grid_body<T, TO, NK>(a, S_out, t_near, stage_cap, level_mask, bid, g_grid,
                                 reinterpret_cast<T *>(far_lds));
    else
        far_shell_body<T, TO>(a, S_out, t_near, bid - g_grid, (int32_t)gridDim.x - g_mfma - g_grid);
}

// Exact near field (Sec. 2.4 eq. (16)) of the leaves with a U list, one workgroup of
// kNearWaves waves per leaf over the list.  The leaf's work items are (U entry, chunk of 64
// of its sources), dealt to the waves in turn (the entries' source ranges are read into LDS
// 64 at a time, so that walking the list costs no dependent loads); a wave stages an item's
// sources in LDS, reads them back with broadcast reads, sums the item's terms per target in
// a plain FP32 sum (at most 64 terms) and adds that to a Kahan-compensated FP32 total (FP64
// throughout in the FP64 form).  On uniform grids the kernel between two finest-level
// leaves is read from a table indexed by the integer cell offset (built in FP64 at plan
// time, held in LDS) instead of being evaluated from FP32 coordinates.  The partial sums are combined in FP64 in wave order (so the result does not
// depend on scheduling) into t_near, which the far-field kernels add to the far field and
// the own-cell term.  The kernel reads only the tree and the lists, so it can run beside
// the upward and downward passes.
constexpr int kNearWaves = 4;
constexpr int32_t kNearTabMark = 0x7fc0dab5;  // a NaN pattern: the staged source is read from the table

template <class T, bool GUARD>
__global__ __launch_bounds__(64 * kNearWaves) void near_kernel(FmmArgs<T> a, double *__restrict__ t_near)
{
    constexpr int kNB = sizeof(T) == 4 ? 2 : 1;  // items staged together per wave
    __shared__ double part[kNearWaves][64];
    __shared__ V4<T> ysh[kNearWaves][kNB][64];  // per wave: the current items' sources
    __shared__ int32_t esf[64], esn[64];          // a chunk of the U list: first sources, run offsets
    __shared__ uint8_t etab[64];                  // and whether the table serves the entry
    __shared__ int32_t ecnt;                      // the chunk's sources
    extern __shared__ __align__(16) float ntab[];  // the near-field kernel table, when present
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t n = a.sc->n_near;
    // the workgroup's leaves: each XCD (workgroup b runs on XCD b mod 8) takes one contiguous run
    // of the list, so that neighbouring leaves, whose U lists share their sources, read them
    // through one L2 (with fewer than 8 workgroups: every gridDim-th leaf)
    const uint32_t G = gridDim.x, xcd = blockIdx.x & 7u;
    int32_t idx0 = (int32_t)blockIdx.x, idx1 = n, step = (int32_t)G;
    if (G >= 8) {
        idx0 = (int32_t)((int64_t)n * xcd / 8) + (int32_t)(blockIdx.x >> 3);
        idx1 = (int32_t)((int64_t)n * (xcd + 1) / 8);
        step = (int32_t)((G >> 3) + (xcd < (G & 7u) ? 1u : 0u));
    }
    if (idx0 >= idx1) return;  // the whole workgroup
    // uniform grids (FP32): between two leaves of the table's level the kernel is read from the
    // table at the integer cell offset instead of being evaluated
    const bool tab = sizeof(T) == 4 && a.near_tab != nullptr;
    const int TR = a.near_R, sx = a.near_sx, sy = a.near_sy, sz = a.near_sz, TN = a.near_n;
    // the table's loads (float4, zero padded) all issued before the first leaf's, and written to
    // LDS once they have arrived (the chunk staging's barrier publishes them)
    constexpr int kTabV = (kNearTabMax + 4 * 64 * kNearWaves - 1) / (4 * 64 * kNearWaves);
    const int TN4 = (TN + 3) >> 2;
    float4 tv[kTabV];
    if (tab) {
#pragma unroll
        for (int u = 0; u < kTabV; ++u) {
            const int i4 = (int)threadIdx.x + u * 64 * kNearWaves;
            tv[u] = i4 < TN4 ? reinterpret_cast<const float4 *>(a.near_tab)[i4] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    bool staged = !tab;
    for (int32_t idx = idx0; idx < idx1; idx += step) {
        const int32_t b = a.L.near_leaves[idx];
        const uint32_t u0 = a.L.u_rng[b].x, u1 = a.L.u_rng[b].y;
        const int32_t p0 = a.bx.start[b], np = a.bx.end[b] - p0;
        const bool tab_b = tab && a.bx.level[b] == a.near_level;
        if (!staged) {
#pragma unroll
            for (int u = 0; u < kTabV; ++u) {
                const int i4 = (int)threadIdx.x + u * 64 * kNearWaves;
                if (i4 < TN4) reinterpret_cast<float4 *>(ntab)[i4] = tv[u];
            }
            staged = true;
        }
        // the leaf's points in sorted order, the targets among them flagged
        for (int tb = 0; tb < np; tb += 64) {
            const int t = tb + lane;
            const int32_t k = p0 + min(t, np - 1);
            const bool act = t < np && (a.sel[k] & 2u) != 0;
            V4<T> x;
            if (act) x = point_xyz(a, k);
            else x.x = x.y = x.z = x.w = T(0);
            // table index of the point's cell with every offset bias folded in (lanes past the
            // leaf's end take its last point, so that their reads stay inside the table)
            int tl = 0;
            if (tab_b) {
                const int32_t c = a.pcell[k];
                tl = ((c & 1023) + TR) * sx + (((c >> 10) & 1023) + TR) * sy + ((c >> 20) + TR) * sz;
            }
            Acc<T> near;
            // the U list a chunk of 64 entries at a time: the entries' source ranges (whether
            // the table serves them, and where each starts in the chunk's run of sources) are
            // read in parallel into LDS; the chunk's sources, packed 64 to a batch across entry
            // boundaries, are then shared out to the waves batch by batch, kNB batches at a time
            // (their source loads issued together)
            for (uint32_t c0 = u0; c0 < u1; c0 += 64) {
                const int ne = (int)min(64u, u1 - c0);
                __syncthreads();  // every wave is done with the previous chunk
                if (w == 0) {
                    int32_t sf = 0, sn = 0;
                    uint8_t et = 0;
                    if (lane < ne) {
                        const int32_t C = a.L.u[c0 + lane];
                        sf = a.bx.s_first[C];
                        sn = a.bx.s_cnt[C];
                        et = tab_b && a.bx.level[C] == a.near_level;
                    }
                    const int32_t incl = wave_inclusive(sn, lane);
                    esf[lane] = sf;
                    esn[lane] = incl - sn;  // the entry's first position in the run
                    etab[lane] = et;
                    if (lane == 63) ecnt = incl;
                }
                __syncthreads();
                const int32_t S = ecnt, nbat = (S + 63) >> 6;
                for (int b0 = w; b0 < nbat; b0 += kNearWaves * kNB) {
                    int cnt[kNB];
                    uint8_t kind[kNB];  // 0 direct, 1 table, 2 both (a branch per source)
#pragma unroll
                    for (int q = 0; q < kNB; ++q) {
                        const int bi = b0 + q * kNearWaves;
                        cnt[q] = bi < nbat ? min(64, S - bi * 64) : 0;
                        const int32_t sp = bi * 64 + lane;  // the lane's source in the run
                        const bool live = lane < cnt[q];
                        // the entry holding it: the last one starting at or before it (every
                        // entry holds at least one source)
                        int e = 0;
#pragma unroll
                        for (int st = 32; st > 0; st >>= 1)
                            if (e + st < ne && esn[e + st] <= sp) e += st;
                        const int32_t src = esf[e] + (sp - esn[e]);
                        const bool st = sizeof(T) == 4 && live && etab[e];
                        const uint64_t m_live = __ballot(live), m_tab = __ballot(st);
                        kind[q] = m_tab == 0 ? 0 : (m_tab == m_live ? 1 : 2);
                        if (kind[q] == 1) {
                            // table sources only: the linear index of the cell in the table's
                            // strides and the weight, two sources to 16 bytes (lanes past the
                            // batch stage a zero weight)
                            float2 y2 = make_float2(0.f, 0.f);
                            if (live) {
                                const int32_t c = a.s_cell[src];
                                y2.x = __int_as_float((c & 1023) * sx + ((c >> 10) & 1023) * sy + (c >> 20) * sz);
                                y2.y = (float)a.s_dat[src].w;
                            }
                            reinterpret_cast<float2 *>(&ysh[w][q][0])[lane] = y2;
                        } else if (live) {
                            if (st) {
                                // a table source among others: index, weight and the table mark
                                const int32_t c = a.s_cell[src];
                                V4<T> y;
                                y.x = __int_as_float((c & 1023) * sx + ((c >> 10) & 1023) * sy + (c >> 20) * sz);
                                y.y = a.s_dat[src].w;
                                y.z = __int_as_float(kNearTabMark);
                                y.w = T(0);
                                ysh[w][q][lane] = y;
                            } else {
                                ysh[w][q][lane] = a.s_dat[src];
                            }
                        }
                    }
                    wave_lds_sync();
#pragma unroll
                    for (int q = 0; q < kNB; ++q) {
                        // the batch's terms in a plain sum (at most 64), added to the compensated total
                        T blk = T(0);
                        if (sizeof(T) == 4 && kind[q] == 1) {
                            const float4 *y4 = reinterpret_cast<const float4 *>(&ysh[w][q][0]);
#pragma unroll 4
                            for (int j = 0; j < (cnt[q] + 1) / 2; ++j) {
                                const float4 y = y4[j];  // two sources, a broadcast read
                                // adjacent leaves keep the offsets inside the table; the clamp
                                // keeps every read inside it regardless
                                const int i0 = min(max(tl - __float_as_int(y.x), 0), TN - 1);
                                const int i1 = min(max(tl - __float_as_int(y.z), 0), TN - 1);
                                blk += (T)ntab[i0] * (T)y.y;
                                blk += (T)ntab[i1] * (T)y.w;
                            }
                        } else if (kind[q] == 0) {
#pragma unroll 8
                            for (int j = 0; j < cnt[q]; ++j) {
                                const V4<T> y = ysh[w][q][j];  // one address for the wave: a broadcast read
                                const T dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                                const T r2 = dx * dx + dy * dy + dz * dz;
                                const T v = kernel_eval<GUARD>(r2, a.kp) * y.w;
                                blk += r2 > T(0) ? v : T(0);
                            }
                        } else {
                            for (int j = 0; j < cnt[q]; ++j) {
                                const V4<T> y = ysh[w][q][j];
                                if (__float_as_int((float)y.z) == kNearTabMark) {
                                    const int i0 = min(max(tl - __float_as_int((float)y.x), 0), TN - 1);
                                    blk += (T)ntab[i0] * y.y;
                                } else {
                                    const T dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                                    const T r2 = dx * dx + dy * dy + dz * dz;
                                    const T v = kernel_eval<GUARD>(r2, a.kp) * y.w;
                                    blk += r2 > T(0) ? v : T(0);
                                }
                            }
                        }
                        if (cnt[q] > 0) near.add(blk);
                    }
                    wave_lds_sync();  // the batches' sources have been read
                }
            }
            __syncthreads();  // the previous pass's partial sums have been read
            part[w][lane] = near.value();
            __syncthreads();
            if (w == 0 && act) {
                double tot = 0.0;
                for (int q = 0; q < kNearWaves; ++q) tot += part[q][lane];
                t_near[k] = tot;
            }
        }
    }
}

template <class T>
void fmm_p2m_t(Plan &p, hipStream_t s)
{
    FmmArgs<T> a = make_args<T>(p);
    const int D = p.max_depth;
    int64_t cap = 0;
    for (int l = 2; l <= D; ++l) cap += p.level_cap[l];
    if (cap == 0) return;
    // the composite L2L reads only the check values the gather wrote this call: nothing to clear
    const bool comp = std::is_same<T, float>::value && p.l2l_comp;
    const int64_t u_zero = D >= 3 ? p.level_base[3] * (int64_t)p.n_lam : 0;
    const int64_t u_end = (D >= 3 && !comp) ? p.box_cap * (int64_t)p.n_lam : u_zero;
    p2m_kernel<T><<<(unsigned)std::min<int64_t>(cap, 4096), kUpThreads, 0, s>>>(a, D, u_zero, u_end);
}

template <class T>
void fmm_m2m_t(Plan &p, hipStream_t s)
{
    FmmArgs<T> a = make_args<T>(p);
    const int D = p.max_depth;
    for (int l = D - 1; l >= 2; --l) {
        // a direct product per parent for small lattices; the level GEMM (all eight octant
        // translations of every child, on the matrix cores) for large ones
        if (p.n_lam <= 64)
            m2m_kernel<T><<<(unsigned)std::min<int64_t>(p.level_cap[l], 2048), kM2MThreads, 0, s>>>(a, l);
        else
            fmm_m2m_level(p, l, s);
    }
}

template <class T>
void fmm_leaf_t(Plan &p, void *S_out, hipStream_t s, hipStream_t s_aux)
{
    FmmArgs<T> a = make_args<T>(p);
    // third strategy: the W lists' bounds first (the leaf kernels compare them per target)
    if (p.thr.r_s > 0 && p.d_rs_bound) w_bound_kernel<T><<<256, 256, 0, s>>>(a, p.d_rs_bound);
    // upper bounds on the list lengths (the counts are on the device)
    const int64_t B = p.box_cap;
    if (p.grid_mode) {
        // levels of the grid-operator lists: the matrix-core kernel where the operator is at most
        // 64 x 64 (FP32), the wave kernel elsewhere (and for levels without a far field)
        uint32_t mfma_levels = 0, wave_levels = 0;
        for (int l = 0; l <= p.max_depth; ++l) {
            if (!(l < 2 || p.grid_m[l] > 0)) continue;
            const bool mf = std::is_same<T, float>::value && (l < 2 || p.grid_m[l] <= 4) && p.n_lam <= 64;
            (mf ? mfma_levels : wave_levels) |= 1u << l;
        }
        int64_t gm_blocks = 0, gw_blocks = 0;
        for (int l = 0; l <= p.max_depth; ++l) {
            if ((mfma_levels >> l) & 1u) gm_blocks += (p.level_cap[l] + kFarMLeaves - 1) / kFarMLeaves;
            if ((wave_levels >> l) & 1u) {
                const int gm = l >= 2 ? p.grid_m[l] : 0;
                gw_blocks += far_chunks(gm) > 1 ? p.level_cap[l] * far_groups(gm)
                                                : (p.level_cap[l] + kFarLeaves - 1) / kFarLeaves;
            }
        }
        if (!std::is_same<T, float>::value) gm_blocks = 0;
        // LDS for the largest wave-kernel level operator that fits the staging cap
        int cap = 0;
        for (int l = 2; l <= p.max_depth; ++l) {
            const int e = p.n_lam * p.grid_m[l] * p.grid_m[l] * p.grid_m[l];
            if (((wave_levels >> l) & 1u) && p.grid_m[l] > 0 && e <= kGridStage) cap = std::max(cap, e);
        }
        const size_t lds = (size_t)cap * sizeof(T);
        const int32_t gmb = (int32_t)gm_blocks;
        const int32_t g = (int32_t)std::min<int64_t>(gw_blocks, 256);
        // on grids the shell list holds only leaves of levels >= 2 without an operator
        bool shell_leaves = false;
        for (int l = 2; l <= p.max_depth; ++l) shell_leaves = shell_leaves || p.grid_m[l] == 0;
        const unsigned gt = (unsigned)(gmb + g + (shell_leaves ? (int32_t)std::min<int64_t>(B, 64) : 0));
        if (gt == 0) return;
        switch ((p.n_lam + 63) / 64) {
        case 1: far_rest_kernel<T, T, 1><<<gt, 256, lds, s>>>(a, (T *)S_out, p.d_t_near, cap, wave_levels, mfma_levels, gmb, g); break;
        case 2: far_rest_kernel<T, T, 2><<<gt, 256, lds, s>>>(a, (T *)S_out, p.d_t_near, cap, wave_levels, mfma_levels, gmb, g); break;
        case 3:
        case 4: far_rest_kernel<T, T, 4><<<gt, 256, lds, s>>>(a, (T *)S_out, p.d_t_near, cap, wave_levels, mfma_levels, gmb, g); break;
        default: far_rest_kernel<T, T, 8><<<gt, 256, lds, s>>>(a, (T *)S_out, p.d_t_near, cap, wave_levels, mfma_levels, gmb, g); break;
        }
        return;
    }
    // point clouds (or grids without grid-operator leaves): the shell-point leaves alone
    bool shell_leaves = !p.grid_mode;
    for (int l = 2; l <= p.max_depth; ++l) shell_leaves = shell_leaves || p.grid_m[l] == 0;
    if (shell_leaves)
        far_shell_kernel<T, T><<<(unsigned)std::min<int64_t>(B, p.grid_mode ? 256 : 4096), 64, 0, s>>>(
            a, (T *)S_out, p.d_t_near);
}

template <class T>
void fmm_near_t(Plan &p, hipStream_t s)
{
    FmmArgs<T> a = make_args<T>(p);
    // at most four workgroups (16 waves) per CU: the upward and downward passes run beside this
    // kernel on the other stream, and a full grid would hold every wave slot until it drains
    const unsigned g = (unsigned)std::min<int64_t>(p.box_cap, 1024);
    // the table is stored padded with zeros to a whole number of float4
    const size_t lds =
        (std::is_same<T, float>::value && p.ops.near_tab) ? (size_t)((p.ops.near_n + 3) & ~3) * sizeof(float) : 0;
    if (p.near_guard) near_kernel<T, true><<<g, 64 * kNearWaves, lds, s>>>(a, p.d_t_near);
    else near_kernel<T, false><<<g, 64 * kNearWaves, lds, s>>>(a, p.d_t_near);
}

}  // namespace

void fmm_p2m(Plan &p, hipStream_t s)
{
    if (p.precision == PH_FP64) fmm_p2m_t<double>(p, s);
    else fmm_p2m_t<float>(p, s);
}

void fmm_m2m(Plan &p, hipStream_t s)
{
    if (p.precision == PH_FP64) fmm_m2m_t<double>(p, s);
    else fmm_m2m_t<float>(p, s);
}

void fmm_upward(Plan &p, hipStream_t s)
{
    fmm_p2m(p, s);
    fmm_m2m(p, s);
}

void fmm_leaf(Plan &p, void *S_out, hipStream_t s, hipStream_t s_aux)
{
    if (p.precision == PH_FP64) fmm_leaf_t<double>(p, S_out, s, s_aux);
    else fmm_leaf_t<float>(p, S_out, s, s_aux);
}

void fmm_near(Plan &p, hipStream_t s)
{
    if (p.precision == PH_FP64) fmm_near_t<double>(p, s);
    else fmm_near_t<float>(p, s);
}

}  // namespace ph
