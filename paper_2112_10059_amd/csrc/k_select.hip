// Adaptive selection and compaction (Sec. 3 strategies 1-2; Sec. 4.3 eq. (22); Sec. 5 field rule).
//
// Source j is kept iff I_j >= src_rel * max_k I_k (the maximum over every
// point); target i is kept iff |E_i| >= e_abs and/or
// |E_i| >= E_applied + eps (max|E| - E_applied).  Every comparison is made in
// FP64 between the stored value (exactly widened) and an FP64 threshold.
// Compaction walks the Morton order, so the selected lists stay sorted and
// every octree box is a contiguous run in each list.
#include <hip/hip_runtime.h>

#include "k_common.h"

namespace ph {

namespace {

__global__ void reset_scalars_kernel(CallScalars *sc)
{
    int32_t *w = reinterpret_cast<int32_t *>(sc);
    for (int i = threadIdx.x; i < (int)(sizeof(CallScalars) / 4); i += blockDim.x) w[i] = 0;
}

// Maxima of I and |E| (with the position of the largest |E|): each block reduces its
// grid-stride share into partials, one block then reduces the partials (no contended atomics).
template <class T>
__global__ void reduce_max_kernel(const T *__restrict__ I, const float *__restrict__ E, int64_t n,
                                  double *__restrict__ partial, uint64_t *__restrict__ partial_key, CallScalars *sc)
{
    __shared__ double smI[256];
    __shared__ uint64_t smE[256];
    double mi = 0.0;
    uint64_t me = 0;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        T v = I[i];
        if (bad_value(v)) bad = 1;
        else mi = fmax(mi, (double)v);
        if (E) {
            const uint64_t k = e_key(E[i], i);
            if (k > me) me = k;
        }
    }
    smI[threadIdx.x] = mi;
    smE[threadIdx.x] = me;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            smI[threadIdx.x] = fmax(smI[threadIdx.x], smI[threadIdx.x + o]);
            smE[threadIdx.x] = max(smE[threadIdx.x], smE[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (bad) atomicOr(&sc->err, 1);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = smI[0];
        partial_key[blockIdx.x] = smE[0];
    }
}

__global__ void reduce_max_final_kernel(const double *__restrict__ partial, const uint64_t *__restrict__ partial_key,
                                        int nb, CallScalars *sc)
{
    __shared__ double a[256];
    __shared__ uint64_t b[256];
    double mi = 0.0;
    uint64_t me = 0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        mi = fmax(mi, partial[i]);
        me = max(me, partial_key[i]);
    }
    a[threadIdx.x] = mi;
    b[threadIdx.x] = me;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            a[threadIdx.x] = fmax(a[threadIdx.x], a[threadIdx.x + o]);
            b[threadIdx.x] = max(b[threadIdx.x], b[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->imax = a[0];
        sc->emax = (double)__uint_as_float((uint32_t)(b[0] >> 32));
        sc->emax_key = b[0];
    }
}

struct SelectParams {
    double src_rel, e_abs, e_applied, e_rel;
    double fallback_rel;          // source rule used when the learned selector falls back
};

// drop: per sorted point, 1 if a learned decision removed its source leaf (null: none).
// When the selector has fallen back (sc->fallback) the source rule is fallback_rel instead.
template <class T>
__global__ void select_flags_kernel(const T *__restrict__ I, const float *__restrict__ E,
                                    const int32_t *__restrict__ perm, int64_t n, SelectParams sp,
                                    CallScalars *__restrict__ sc, uint64_t *__restrict__ flag,
                                    T *__restrict__ S_out, const uint8_t *__restrict__ drop)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t o = perm[k];
    const double v = (double)I[o];
    bool src;
    if (drop && sc->fallback) {
        src = (sp.fallback_rel <= 0.0) || (v >= sp.fallback_rel * sc->imax);
    } else {
        src = (sp.src_rel <= 0.0) || (v >= sp.src_rel * sc->imax);
        if (drop) src = src && !drop[k];
    }
    bool tgt = true;
    if (E) {
        const double e = (double)E[o];
        if (sp.e_abs >= 0.0) tgt = tgt && (e >= sp.e_abs);
        if (sp.e_rel >= 0.0) tgt = tgt && (e >= sp.e_applied + sp.e_rel * (sc->emax - sp.e_applied));
    }
    flag[k] = (uint64_t)(src ? 1u : 0u) | ((uint64_t)(tgt ? 1u : 0u) << 32);
    if (!tgt) S_out[o] = T(0);
}

template <class T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};

// flag[] now holds the exclusive scan of the packed (src, tgt) indicators and
// sc->packed_total the packed totals, so element k is selected iff its scan
// value differs from the next one.
template <class T, class TI>
__global__ void compact_kernel(const TI *__restrict__ I, const int32_t *__restrict__ perm,
                               const uint64_t *__restrict__ key, const double *__restrict__ xyz,
                               const double *__restrict__ w, double w_uniform, double c_self, int64_t n,
                               CallScalars *__restrict__ sc, const uint64_t *__restrict__ scanned,
                               int32_t *__restrict__ s_pos, int32_t *__restrict__ t_pos,
                               int32_t *__restrict__ t_out,
                               typename Vec4<T>::type *__restrict__ s_dat, typename Vec4<T>::type *__restrict__ t_dat,
                               const int32_t *__restrict__ cell, int32_t *__restrict__ s_cell,
                               int32_t *__restrict__ t_cell)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double imax = sc->imax;
    // scale I by 2^-e, e = floor(log2(max I)), so FP32 sums stay near unit magnitude
    int e = 0;
    if (imax > 0.0) {
        (void)frexp(imax, &e);
        e -= 1;
    }
    const uint64_t total = sc->packed_total;
    if (k == 0) {
        sc->scale_exp = e;
        sc->n_src = (int32_t)(total & 0xffffffffu);
        sc->n_tgt = (int32_t)(total >> 32);
    }
    if (k >= n) return;
    const uint64_t here = scanned[k];
    const uint64_t next = (k + 1 < n) ? scanned[k + 1] : total;
    const uint32_t sp_lo = (uint32_t)(here & 0xffffffffu), sp_hi = (uint32_t)(here >> 32);
    const bool is_src = (uint32_t)(next & 0xffffffffu) != sp_lo;
    const bool is_tgt = (uint32_t)(next >> 32) != sp_hi;
    if (!is_src && !is_tgt) return;
    const int32_t o = perm[k];
    const double scale = ldexp(1.0, -e);
    const double Iv = (double)I[o] * scale;
    const double x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
    if (is_src) {
        const double wk = w ? w[k] : w_uniform;
        s_pos[sp_lo] = (int32_t)k;
        typename Vec4<T>::type d;
        d.x = (T)x;
        d.y = (T)y;
        d.z = (T)z;
        d.w = (T)(wk * Iv);
        s_dat[sp_lo] = d;
        if (cell) s_cell[sp_lo] = cell[k];
    }
    if (is_tgt) {
        t_pos[sp_hi] = (int32_t)k;
        t_out[sp_hi] = o;
        typename Vec4<T>::type d;
        d.x = (T)x;
        d.y = (T)y;
        d.z = (T)z;
        d.w = is_src ? (T)(c_self * Iv) : T(0);
        t_dat[sp_hi] = d;
        if (cell) t_cell[sp_hi] = cell[k];
    }
}

}  // namespace

void launch_reset_scalars(CallScalars *sc, hipStream_t s) { reset_scalars_kernel<<<1, 256, 0, s>>>(sc); }

void launch_reduce_max_final(const double *partial, const uint64_t *partial_key, int nb, CallScalars *sc,
                             hipStream_t s)
{
    reduce_max_final_kernel<<<1, 256, 0, s>>>(partial, partial_key, nb, sc);
}

void launch_reduce_max(const void *I, bool fp64, const float *E, bool need_e, int64_t n, CallScalars *sc,
                       void *tmp, hipStream_t s)
{
    int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
    double *partial = reinterpret_cast<double *>(tmp);
    uint64_t *partial_key = reinterpret_cast<uint64_t *>(partial + 1024);
    if (fp64)
        reduce_max_kernel<double><<<blocks, 256, 0, s>>>((const double *)I, need_e ? E : nullptr, n, partial,
                                                         partial_key, sc);
    else
        reduce_max_kernel<float><<<blocks, 256, 0, s>>>((const float *)I, need_e ? E : nullptr, n, partial,
                                                        partial_key, sc);
    reduce_max_final_kernel<<<1, 256, 0, s>>>(partial, partial_key, blocks, sc);
}

static SelectParams params_of(const Plan &p)
{
    return SelectParams{p.thr.src_rel, p.thr.e_abs, p.thr.e_applied, p.thr.e_rel, p.fallback_rel};
}

void launch_select_flags(const Plan &p, const void *I, const float *E, void *S_out, hipStream_t s,
                         const uint8_t *drop)
{
    const bool need_e = p.thr.e_abs >= 0 || p.thr.e_rel >= 0;
    unsigned g = (unsigned)((p.n + 255) / 256);
    if (p.precision == PH_FP64)
        select_flags_kernel<double><<<g, 256, 0, s>>>((const double *)I, need_e ? E : nullptr, p.d_perm, p.n,
                                                      params_of(p), p.d_sc, p.d_flag, (double *)S_out, drop);
    else
        select_flags_kernel<float><<<g, 256, 0, s>>>((const float *)I, need_e ? E : nullptr, p.d_perm, p.n,
                                                     params_of(p), p.d_sc, p.d_flag, (float *)S_out, drop);
}

void launch_compact(const Plan &p, const void *I, hipStream_t s)
{
    unsigned g = (unsigned)((p.n + 255) / 256);
    if (p.precision == PH_FP64)
        compact_kernel<double, double><<<g, 256, 0, s>>>(
            (const double *)I, p.d_perm, p.d_key, p.d_xyz, p.d_w, p.w_uniform, p.c_self, p.n, p.d_sc, p.d_flag,
            p.d_s_pos, p.d_t_pos, p.d_t_out, (double4 *)p.d_s_dat, (double4 *)p.d_t_dat,
            p.grid_mode ? p.d_cell : nullptr, p.d_s_cell, p.d_t_cell);
    else
        compact_kernel<float, float><<<g, 256, 0, s>>>(
            (const float *)I, p.d_perm, p.d_key, p.d_xyz, p.d_w, p.w_uniform, p.c_self, p.n, p.d_sc, p.d_flag,
            p.d_s_pos, p.d_t_pos, p.d_t_out, (float4 *)p.d_s_dat, (float4 *)p.d_t_dat,
            p.grid_mode ? p.d_cell : nullptr, p.d_s_cell, p.d_t_cell);
}

}  // namespace ph
