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

#include "k_fmm_args.h"

namespace ph {

namespace {

// ---------------------------------------------------------------- P2M

template <class T>
__global__ void p2m_kernel(FmmArgs<T> a, int level)
{
  for (int32_t rk = blockIdx.x; rk < a.sc->lvl_src[level]; rk += gridDim.x) {
    const int32_t b = a.bx.src_box[a.lt.base[level] + rk];
    if (!(a.bx.flags[b] & kBoxLeaf) || a.bx.s_cnt[b] == 0) continue;
    __shared__ V4<T> tile[128];
    __shared__ T chk[kMaxShell];
    __shared__ int32_t rloc[128];
    const int32_t sf = a.bx.s_first[b], sn = a.bx.s_cnt[b];
    const int gm = a.grid_m[level];
    if (gm > 0) {
        // grid box: phi = G q over the box's cells (G = uc2e K(shell, cells))
        const T *G = a.grid_gt + a.grid_off[level];
        T accg[4] = {0, 0, 0, 0};
        for (int base = 0; base < sn; base += 128) {
            const int m = min(128, sn - base);
            __syncthreads();
            if ((int)threadIdx.x < m) {
                tile[threadIdx.x] = a.s_dat[sf + base + threadIdx.x];
                rloc[threadIdx.x] = local_cell(a, a.s_cell[sf + base + threadIdx.x], b, gm);
            }
            __syncthreads();
            for (int k = 0; k < 4; ++k) {
                const int li = threadIdx.x + k * blockDim.x;
                if (li >= a.n_lam) break;
                T sacc = 0;
                for (int j = 0; j < m; ++j) sacc += G[(size_t)rloc[j] * a.n_lam + li] * tile[j].w;
                accg[k] += sacc;
            }
        }
        for (int k = 0; k < 4; ++k) {
            const int li = threadIdx.x + k * blockDim.x;
            if (li < a.n_lam) a.phi[(size_t)b * a.n_lam + li] = accg[k];
        }
        if (a.work && threadIdx.x == 0) atomicAdd(&a.work[9], (unsigned long long)sn * a.n_lam);
        continue;
    }
    const double hw = a.lt.hw[level];
    T cx, cy, cz;
    box_centre(a, b, hw, cx, cy, cz);
    const T h = (T)hw;
    T acc[4] = {0, 0, 0, 0};  // n_sig <= 4 * 128 check points per thread slot
    for (int base = 0; base < sn; base += 128) {
        const int m = min(128, sn - base);
        __syncthreads();
        if ((int)threadIdx.x < m) tile[threadIdx.x] = a.s_dat[sf + base + threadIdx.x];
        __syncthreads();
        for (int r = 0; r < 4; ++r) {
            const int sg = threadIdx.x + r * 128;
            if (sg >= a.n_sig) break;
            const T px = cx + h * a.shell[3 * sg], py = cy + h * a.shell[3 * sg + 1], pz = cz + h * a.shell[3 * sg + 2];
            T s = 0;
            for (int j = 0; j < m; ++j) {
                const V4<T> y = tile[j];
                const T dx = px - y.x, dy = py - y.y, dz = pz - y.z;
                s += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * y.w;
            }
            acc[r] += s;
        }
    }
    for (int r = 0; r < 4; ++r) {
        const int sg = threadIdx.x + r * 128;
        if (sg < a.n_sig) chk[sg] = acc[r];
    }
    __syncthreads();
    const T *U = a.uc2e_cm + (size_t)level * a.n_sig * a.n_lam;
    for (int li = threadIdx.x; li < a.n_lam; li += blockDim.x) {
        T s = 0;
        for (int sg = 0; sg < a.n_sig; ++sg) s += U[(size_t)sg * a.n_lam + li] * chk[sg];
        a.phi[(size_t)b * a.n_lam + li] = s;
    }
    if (a.work && threadIdx.x == 0) atomicAdd(&a.work[3], (unsigned long long)sn * a.n_sig);
  }
}

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

// Far field of every target leaf (lattice or shell L2P, W list) plus the own-cell term.
// Leaves without near sources are finished here; the others leave their far field in
// t_far for the near-field kernel.
template <class T, class TO, bool GRIDF>
__global__ void leaf_kernel(FmmArgs<T> a, TO *__restrict__ S_out, T *__restrict__ t_far, int role)
{
    const int32_t b = blockIdx.x;
    int level;
    if (!box_live(a.lt, a.sc, b, level)) return;
    if (!(a.bx.flags[b] & kBoxLeaf) || a.bx.t_cnt[b] == 0) return;
    __shared__ T uvec[kMaxLattice];
    __shared__ T wphi[kMaxLattice];
    __shared__ V4<T> shp[GRIDF ? 1 : kMaxShell];  // shell point position and its intensity psi
    const int nl = a.n_lam, ns = a.n_sig;
    const bool has_far = level >= 2;
    const int gm = has_far ? a.grid_m[level] : 0;
    // role 1: boxes with a lattice operator (or no far field); role 2: the others; role 0: all
    if (role == 1 && has_far && gm == 0) return;
    if (role == 2 && !(has_far && gm == 0)) return;
    const double hw = a.lt.hw[level];
    T cx, cy, cz;
    box_centre(a, b, hw, cx, cy, cz);
    const T h = (T)hw;
    if (has_far) {
        for (int li = threadIdx.x; li < nl; li += blockDim.x) uvec[li] = a.u[(size_t)b * nl + li];
        __syncthreads();
        if (!GRIDF && gm == 0) {
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
    }
    const int32_t tf = a.bx.t_first[b], tn = a.bx.t_cnt[b];
    const uint32_t u0 = a.L.u_off[b], u1 = a.L.u_off[b + 1];
    const uint32_t w0 = a.L.w_off[b], w1 = a.L.w_off[b + 1];
    const int scale_exp = a.sc->scale_exp;
    if (a.work && threadIdx.x == 0) {
        unsigned long long near_src = 0, w_eval = 0;
        for (uint32_t e = u0; e < u1; ++e) near_src += a.bx.s_cnt[a.L.u[e]];
        w_eval = (unsigned long long)(w1 - w0) * nl;
        atomicAdd(&a.work[0], near_src * tn);
        if (u1 > u0) atomicAdd(&a.work[10], (unsigned long long)tn);  // targets the near-field kernel visits
        if (has_far && gm == 0) atomicAdd(&a.work[1], (unsigned long long)tn * ns);
        if (has_far && gm > 0) atomicAdd(&a.work[8], (unsigned long long)tn * nl);
        if (w_eval) atomicAdd(&a.work[2], w_eval * tn);
    }
    for (int tb = 0; tb < tn; tb += blockDim.x) {
        const int t = tb + threadIdx.x;
        const bool act = t < tn;
        V4<T> x;
        if (act) x = a.t_dat[tf + t];
        else x.x = x.y = x.z = x.w = T(0);
        T far = 0;
        if (has_far && act) {
            if (GRIDF || gm > 0) {
                const T *G = a.grid_g + a.grid_off[level];
                const int R = gm * gm * gm;
                const int r = local_cell(a, a.t_cell[tf + t], b, gm);
                for (int li = 0; li < nl; ++li) far += G[(size_t)li * R + r] * uvec[li];
            } else if (!GRIDF) {
                for (int sg = 0; sg < ns; ++sg) {
                    const V4<T> q = shp[GRIDF ? 0 : sg];
                    const T dx = x.x - q.x, dy = x.y - q.y, dz = x.z - q.z;
                    far += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * q.w;
                }
            }
        }
        // W list: artificial sources of smaller non-adjacent boxes
        for (uint32_t e = w0; e < w1; ++e) {
            const int32_t A = a.L.w[e];
            const int la = a.bx.level[A];
            const double hwa = a.lt.hw[la];
            T ax, ay, az;
            box_centre(a, A, hwa, ax, ay, az);
            const T ha = (T)hwa;
            __syncthreads();
            for (int li = threadIdx.x; li < nl; li += blockDim.x) wphi[li] = a.phi[(size_t)A * nl + li];
            __syncthreads();
            if (act)
                for (int li = 0; li < nl; ++li) {
                    const T dx = x.x - (ax + ha * a.lat[3 * li]);
                    const T dy = x.y - (ay + ha * a.lat[3 * li + 1]);
                    const T dz = x.z - (az + ha * a.lat[3 * li + 2]);
                    far += kernel_eval<false>(dx * dx + dy * dy + dz * dz, a.kp) * wphi[li];
                }
        }
        if (act) {
            if (u1 > u0) {
                t_far[tf + t] = far;
            } else {
                const double tot = (double)far + (double)x.w;
                S_out[a.perm[a.t_pos[tf + t]]] = (TO)(a.P * ldexp(tot, scale_exp));
            }
        }
    }
}

// Exact near field (Sec. 2.4 eq. (16)) of leaves with a U list: four waves per leaf,
// wave w sums the U entries w, w+4, ...; each wave keeps a Kahan-compensated FP32 sum
// (FP64 in the FP64 form); the partial sums, the far field and the own-cell term are
// combined in FP64 in a fixed order.  Sources are broadcast lane by lane from registers.
template <class T, class TO, bool GUARD>
__global__ __launch_bounds__(256) void near_kernel(FmmArgs<T> a, TO *__restrict__ S_out,
                                                   const T *__restrict__ t_far)
{
    const int32_t b = blockIdx.x;
    int level;
    if (!box_live(a.lt, a.sc, b, level)) return;
    if (!(a.bx.flags[b] & kBoxLeaf) || a.bx.t_cnt[b] == 0) return;
    const uint32_t u0 = a.L.u_off[b], u1 = a.L.u_off[b + 1];
    if (u1 == u0) return;
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t tf = a.bx.t_first[b], tn = a.bx.t_cnt[b];
    const int scale_exp = a.sc->scale_exp;
    for (int tb = 0; tb < tn; tb += 64) {
        const int t = tb + lane;
        const bool act = t < tn;
        V4<T> x;
        if (act) x = a.t_dat[tf + t];
        else x.x = x.y = x.z = x.w = T(0);
        Acc<T> near;
        for (uint32_t e = u0 + w; e < u1; e += 4) {
            const int32_t C = a.L.u[e];
            const int32_t sf = a.bx.s_first[C], sn = a.bx.s_cnt[C];
            for (int base = 0; base < sn; base += 64) {
                const int m = min(64, sn - base);
                V4<T> y;
                if (lane < m) y = a.s_dat[sf + base + lane];
                else y.x = y.y = y.z = y.w = T(0);
                for (int j = 0; j < m; ++j) {
                    const T yx = lane_bcast(y.x, j), yy = lane_bcast(y.y, j), yz = lane_bcast(y.z, j),
                            yw = lane_bcast(y.w, j);
                    const T dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    if (act && r2 > T(0)) near.add(kernel_eval<GUARD>(r2, a.kp) * yw);
                }
            }
        }
        part[w][lane] = near.value();
        __syncthreads();
        if (w == 0 && act) {
            const double tot = (double)t_far[tf + t] + part[0][lane] + part[1][lane] + part[2][lane] +
                               part[3][lane] + (double)x.w;
            S_out[a.perm[a.t_pos[tf + t]]] = (TO)(a.P * ldexp(tot, scale_exp));
        }
        __syncthreads();
    }
}

template <class T>
void fmm_upward_t(Plan &p, hipStream_t s)
{
    FmmArgs<T> a = make_args<T>(p);
    const int D = p.max_depth;
    const int threads = std::max(128, ((p.n_lam + 63) / 64) * 64);
    for (int l = 2; l <= D; ++l)
        p2m_kernel<T><<<(unsigned)std::min<int64_t>(p.level_cap[l], 4096), 128, 0, s>>>(a, l);
    for (int l = D - 1; l >= 2; --l) fmm_m2m_level(p, l, s);
}

template <class T>
void fmm_leaf_t(Plan &p, void *S_out, hipStream_t s)
{
    FmmArgs<T> a = make_args<T>(p);
    bool shell_levels = !p.grid_mode;
    for (int l = 2; l <= p.max_depth; ++l) shell_levels = shell_levels || p.grid_m[l] == 0;
    if (p.grid_mode) {
        leaf_kernel<T, T, true><<<(unsigned)p.box_cap, 64, 0, s>>>(a, (T *)S_out, (T *)p.d_t_far, 1);
        if (shell_levels) leaf_kernel<T, T, false><<<(unsigned)p.box_cap, 64, 0, s>>>(a, (T *)S_out, (T *)p.d_t_far, 2);
    } else {
        leaf_kernel<T, T, false><<<(unsigned)p.box_cap, 64, 0, s>>>(a, (T *)S_out, (T *)p.d_t_far, 0);
    }
}

template <class T>
void fmm_near_t(Plan &p, void *S_out, hipStream_t s)
{
    FmmArgs<T> a = make_args<T>(p);
    if (p.near_guard)
        near_kernel<T, T, true><<<(unsigned)p.box_cap, 256, 0, s>>>(a, (T *)S_out, (const T *)p.d_t_far);
    else
        near_kernel<T, T, false><<<(unsigned)p.box_cap, 256, 0, s>>>(a, (T *)S_out, (const T *)p.d_t_far);
}

}  // namespace

void fmm_upward(Plan &p, hipStream_t s)
{
    if (p.precision == PH_FP64) fmm_upward_t<double>(p, s);
    else fmm_upward_t<float>(p, s);
}

void fmm_leaf(Plan &p, void *S_out, hipStream_t s)
{
    if (p.precision == PH_FP64) fmm_leaf_t<double>(p, S_out, s);
    else fmm_leaf_t<float>(p, S_out, s);
}

void fmm_near(Plan &p, void *S_out, hipStream_t s)
{
    if (p.precision == PH_FP64) fmm_near_t<double>(p, S_out, s);
    else fmm_near_t<float>(p, S_out, s);
}

}  // namespace ph
