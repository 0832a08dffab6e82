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

__global__ void reset_scalars_kernel(CallScalars *sc, int32_t *gen)
{
    int32_t *w = reinterpret_cast<int32_t *>(sc);
    for (int i = threadIdx.x; i < (int)(sizeof(CallScalars) / 4); i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0 && gen) {
        // the call's number, kept on the device so that a replayed launch sequence advances it
        int32_t g = *gen + 1;
        if (g <= 0) g = 1;
        *gen = g;
        sc->gen = g;
    }
}

// Maxima of I and |E| (with the position of the largest |E|): each block reduces its
// grid-stride share into partials, one block then reduces the partials (no contended atomics).
template <class T>
__global__ void reduce_max_kernel(const T *__restrict__ I, const float *__restrict__ E, int64_t n,
                                  double *__restrict__ partial, uint64_t *__restrict__ partial_key, CallScalars *sc,
                                  int32_t *gen)
{
    if (blockIdx.x == 0 && gen) begin_call(sc, gen);
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
    __shared__ int anybad;
    if (threadIdx.x == 0) anybad = 0;
    __syncthreads();
    if (bad) anybad = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = mark_bad(smI[0], anybad != 0);
        partial_key[blockIdx.x] = smE[0];
    }
}

__global__ void reduce_max_final_kernel(const double *__restrict__ partial, const uint64_t *__restrict__ partial_key,
                                        int nb, CallScalars *sc, int32_t *sticky)
{
    __shared__ double a[256];
    __shared__ uint64_t b[256];
    double mi = 0.0;
    uint64_t me = 0;
    bool bad = false;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        mi = fmax(mi, partial_max(partial[i], bad));
        me = max(me, partial_key[i]);
    }
    if (bad) flag_error(sc, sticky, 1);
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

// Selection flags of sorted point k (bit 0 source, bit 1 target).  drop: per sorted point, 1
// if a learned decision removed its source leaf (null: none).  When the selector has fallen
// back (sc->fallback) the source rule is fallback_rel instead.  tmask: the caller's target set
// per sorted point (null: every point), intersected with the field rules.
template <class T>
__device__ __forceinline__ uint32_t select_one(const T *__restrict__ I, const float *__restrict__ E, int32_t o,
                                               int64_t k, const SelectParams &sp, const CallScalars *__restrict__ sc,
                                               const uint8_t *__restrict__ drop, const uint8_t *__restrict__ tmask)
{
    const double v = (double)I[o];
    bool src;
    if (drop && sc->fallback) {
        src = (sp.fallback_rel <= 0.0) || (v >= sp.fallback_rel * sc->imax);
    } else {
        src = (sp.src_rel <= 0.0) || (v >= sp.src_rel * sc->imax);
        if (drop) src = src && !drop[k];
    }
    bool tgt = tmask ? tmask[k] != 0 : true;
    if (E) {
        const double e = (double)E[o];
        if (sp.e_abs >= 0.0) tgt = tgt && (e >= sp.e_abs);
        if (sp.e_rel >= 0.0) tgt = tgt && (e >= sp.e_applied + sp.e_rel * (sc->emax - sp.e_applied));
    }
    return (src ? 1u : 0u) | (tgt ? 2u : 0u);
}

__device__ __forceinline__ uint64_t packed_of(uint32_t f)
{
    return (uint64_t)(f & 1u) | ((uint64_t)(f >> 1) << 32);
}

// Selection in two passes over tiles of kSelTile sorted points (1024 threads; wave w owns a
// contiguous sixteenth, read as kSelStrips coalesced strips of 64), with a scan of the tile
// sums between them.  Pass one: the flags of every point (one byte each), S = 0 at points that
// are not targets, and each tile's packed count (sources | targets << 32).
constexpr int kSelWaves = 16;
constexpr int kSelStrips = 4;
constexpr int kSelSpan = 64 * kSelStrips;  // points per wave in a tile
constexpr int kSelTile = kSelWaves * kSelSpan;

template <class T>
__global__ __launch_bounds__(64 * kSelWaves) void select_tiles_kernel(const T *__restrict__ I, const float *__restrict__ E,
                                                           const int32_t *__restrict__ perm, int64_t n,
                                                           SelectParams sp, const CallScalars *__restrict__ sc,
                                                           const uint8_t *__restrict__ drop,
                                                           const uint8_t *__restrict__ tmask, uint8_t *__restrict__ sel,
                                                           T *__restrict__ S_out, uint64_t *__restrict__ partial)
{
    __shared__ uint64_t wsum[kSelWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSelTile + (int64_t)w * kSelSpan;
    int32_t o[kSelStrips];
#pragma unroll
    for (int st = 0; st < kSelStrips; ++st) {
        const int64_t k = base + st * 64 + lane;
        o[st] = k < n ? perm[k] : 0;
    }
    uint64_t acc = 0;
#pragma unroll
    for (int st = 0; st < kSelStrips; ++st) {
        const int64_t k = base + st * 64 + lane;
        if (k < n) {
            const uint32_t f = select_one(I, E, o[st], k, sp, sc, drop, tmask);
            sel[k] = (uint8_t)f;
            if (!(f & 2u)) S_out[o[st]] = T(0);
            acc += packed_of(f);
        }
    }
    acc = lane_value(wave_inclusive(acc, lane), 63);
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int q = 0; q < kSelWaves; ++q) t += wsum[q];
        partial[blockIdx.x] = t;
    }
}

// Pass two: the exclusive scan of the packed counts where the tree build reads it (the first
// point of a box and the point after a box: bnd), and the compaction of the selected points in
// Morton order: sources (x, y, z, w I 2^-e) and, with tgt_compact (the direct method), targets
// (x, y, z, own-cell term c_self I 2^-e if the point is also a source) with their caller
// indices and grid cells; the FMM reads its targets in place.  Coordinates come from the
// plan's sorted copy in the working precision (C: float4, FP64: three doubles).
template <class TI, class T, class C>
__global__ __launch_bounds__(64 * kSelWaves) void select_compact_kernel(
    const TI *__restrict__ I, const int32_t *__restrict__ perm, const C *__restrict__ xyz,
    const double *__restrict__ w, double w_uniform, double c_self, int64_t n, CallScalars *__restrict__ sc,
    const uint8_t *__restrict__ sel, const uint8_t *__restrict__ bnd, const uint64_t *__restrict__ partial,
    int64_t nb, int tile_sums, int tgt_compact, uint64_t *__restrict__ scanned, int32_t *__restrict__ t_out,
    typename Vec4T<T>::type *__restrict__ s_dat, typename Vec4T<T>::type *__restrict__ t_dat,
    const int32_t *__restrict__ cell, int32_t *__restrict__ s_cell, int32_t *__restrict__ t_cell)
{
    __shared__ uint64_t wsum[kSelWaves];
    constexpr int kStrips = kSelStrips;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double imax = sc->imax;
    // scale I by 2^-e, e = floor(log2(max I)), so FP32 sums stay near unit magnitude
    int e = 0;
    if (imax > 0.0) {
        (void)frexp(imax, &e);
        e -= 1;
    }
    // the tile's offset: partial holds the tile sums (tile_sums: each workgroup adds up those of
    // the earlier tiles, and workgroup 0 all of them for the totals) or their exclusive scan
    uint64_t tile_off;
    if (tile_sums) {
        const int64_t upto = blockIdx.x == 0 ? nb : blockIdx.x;
        uint64_t acc = 0;
        for (int64_t j = threadIdx.x; j < upto; j += blockDim.x) acc += partial[j];
        acc = lane_value(wave_inclusive(acc, lane), 63);
        if (lane == 0) wsum[wv] = acc;
        __syncthreads();
        uint64_t sum = 0;
        for (int q = 0; q < kSelWaves; ++q) sum += wsum[q];
        __syncthreads();  // wsum is reused below
        tile_off = blockIdx.x == 0 ? 0 : sum;
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->packed_total = sum;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->n_src = (int32_t)(sum & 0xffffffffu);
            sc->n_tgt = (int32_t)(sum >> 32);
        }
    } else {
        tile_off = partial[blockIdx.x];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const uint64_t total = sc->packed_total;
            sc->n_src = (int32_t)(total & 0xffffffffu);
            sc->n_tgt = (int32_t)(total >> 32);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->scale_exp = e;
    const double scale = ldexp(1.0, -e);
    const int64_t base = (int64_t)blockIdx.x * kSelTile + (int64_t)wv * kSelSpan;
    uint32_t f[kStrips], bd[kStrips];  // flags and box-boundary marks, loaded together
    uint64_t acc = 0;
#pragma unroll
    for (int st = 0; st < kStrips; ++st) {
        const int64_t k = base + st * 64 + lane;
        f[st] = k < n ? sel[k] : 0u;
        bd[st] = k < n ? bnd[k] : 0u;
    }
#pragma unroll
    for (int st = 0; st < kStrips; ++st) acc += packed_of(f[st]);
    acc = lane_value(wave_inclusive(acc, lane), 63);
    if (lane == 0) wsum[wv] = acc;
    __syncthreads();
    uint64_t carry = tile_off;
    for (int q = 0; q < wv; ++q) carry += wsum[q];
#pragma unroll
    for (int st = 0; st < kStrips; ++st) {
        const uint64_t v = packed_of(f[st]);
        const uint64_t incl = wave_inclusive(v, lane);
        const uint64_t here = carry + incl - v;
        carry += lane_value(incl, 63);
        const int64_t k = base + st * 64 + lane;
        if (k >= n) continue;
        if (bd[st]) scanned[k] = here;
        // points that are only targets need nothing more unless targets are compacted
        if (!(tgt_compact ? f[st] : (f[st] & 1u))) continue;
        const uint32_t sp_lo = (uint32_t)(here & 0xffffffffu), sp_hi = (uint32_t)(here >> 32);
        const int32_t o = perm[k];
        const double Iv = (double)I[o] * scale;
        T x, y, z;
        if constexpr (sizeof(C) == 8) {
            x = (T)xyz[3 * k];
            y = (T)xyz[3 * k + 1];
            z = (T)xyz[3 * k + 2];
        } else {
            const C q = xyz[k];
            x = q.x;
            y = q.y;
            z = q.z;
        }
        const bool is_src = f[st] & 1u;
        if (is_src) {
            const double wk = w ? w[k] : w_uniform;
            typename Vec4T<T>::type d;
            d.x = (T)x;
            d.y = (T)y;
            d.z = (T)z;
            d.w = (T)(wk * Iv);
            s_dat[sp_lo] = d;
            if (cell) s_cell[sp_lo] = cell[k];
        }
        if ((f[st] & 2u) && tgt_compact) {
            t_out[sp_hi] = o;
            typename Vec4T<T>::type d;
            d.x = (T)x;
            d.y = (T)y;
            d.z = (T)z;
            d.w = is_src ? (T)(c_self * Iv) : T(0);
            t_dat[sp_hi] = d;
            if (cell) t_cell[sp_hi] = cell[k];
        }
    }
}

// plan time: the sorted coordinates rounded to FP32, as float4 (x, y, z, 0)
__global__ void pack_xyzf_kernel(const double *__restrict__ xyz, int64_t n, float4 *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = make_float4((float)xyz[3 * k], (float)xyz[3 * k + 1], (float)xyz[3 * k + 2], 0.f);
}

}  // namespace

void launch_pack_xyzf(const double *xyz, int64_t n, float4 *out, hipStream_t s)
{
    if (n > 0) pack_xyzf_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xyz, n, out);
}

void launch_reset_scalars(CallScalars *sc, int32_t *gen, hipStream_t s)
{
    reset_scalars_kernel<<<1, 256, 0, s>>>(sc, gen);
}

void launch_reduce_max_final(const double *partial, const uint64_t *partial_key, int nb, CallScalars *sc,
                             int32_t *sticky, hipStream_t s)
{
    reduce_max_final_kernel<<<1, 256, 0, s>>>(partial, partial_key, nb, sc, sticky);
}

void launch_reduce_max(const void *I, bool fp64, const float *E, bool need_e, int64_t n, CallScalars *sc,
                       int32_t *gen, int32_t *sticky, void *tmp, hipStream_t s)
{
    int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
    double *partial = reinterpret_cast<double *>(tmp);
    uint64_t *partial_key = reinterpret_cast<uint64_t *>(partial + 1024);
    if (fp64)
        reduce_max_kernel<double><<<blocks, 256, 0, s>>>((const double *)I, need_e ? E : nullptr, n, partial,
                                                         partial_key, sc, gen);
    else
        reduce_max_kernel<float><<<blocks, 256, 0, s>>>((const float *)I, need_e ? E : nullptr, n, partial,
                                                        partial_key, sc, gen);
    reduce_max_final_kernel<<<1, 256, 0, s>>>(partial, partial_key, blocks, sc, sticky);
}

static SelectParams params_of(const Plan &p, double src_rel)
{
    return SelectParams{src_rel >= 0.0 ? src_rel : p.thr.src_rel, p.thr.e_abs, p.thr.e_applied, p.thr.e_rel,
                        p.fallback_rel};
}

void launch_select(const Plan &p, const void *I, const float *E, void *S_out, hipStream_t s, const uint8_t *drop,
                   double src_rel)
{
    const bool need_e = p.thr.e_abs >= 0 || p.thr.e_rel >= 0;
    if (p.n <= 0) return;
    const int64_t nb = (p.n + kSelTile - 1) / kSelTile;
    uint64_t *partial = (uint64_t *)p.d_scan_tmp;
    const SelectParams sp = params_of(p, src_rel);
    if (p.precision == PH_FP64)
        select_tiles_kernel<double><<<(unsigned)nb, 64 * kSelWaves, 0, s>>>((const double *)I, need_e ? E : nullptr, p.d_perm,
                                                                  p.n, sp, p.d_sc, drop, p.d_tmask, p.d_sel, (double *)S_out,
                                                                  partial);
    else
        select_tiles_kernel<float><<<(unsigned)nb, 64 * kSelWaves, 0, s>>>((const float *)I, need_e ? E : nullptr, p.d_perm,
                                                                 p.n, sp, p.d_sc, drop, p.d_tmask, p.d_sel, (float *)S_out,
                                                                 partial);
    // up to 2048 tiles the compaction adds up the earlier tiles' sums itself; beyond, one
    // workgroup scans them first
    const int tile_sums = nb <= 2048 ? 1 : 0;
    if (!tile_sums) scan_tile_sums_u64(partial, nb, &p.d_sc->packed_total, s);
    if (p.precision == PH_FP64)
        select_compact_kernel<double, double, double><<<(unsigned)nb, 64 * kSelWaves, 0, s>>>(
            (const double *)I, p.d_perm, p.d_xyz, p.d_w, p.w_uniform, p.c_self, p.n, p.d_sc, p.d_sel, p.d_bnd,
            partial, nb, tile_sums, p.method == PH_METHOD_DIRECT ? 1 : 0, p.d_flag, p.d_t_out, (double4 *)p.d_s_dat, (double4 *)p.d_t_dat,
            p.grid_mode ? p.d_cell : nullptr, p.d_s_cell, p.d_t_cell);
    else
        select_compact_kernel<float, float, float4><<<(unsigned)nb, 64 * kSelWaves, 0, s>>>(
            (const float *)I, p.d_perm, p.d_xyzf, p.d_w, p.w_uniform, p.c_self, p.n, p.d_sc, p.d_sel, p.d_bnd,
            partial, nb, tile_sums, p.method == PH_METHOD_DIRECT ? 1 : 0, p.d_flag, p.d_t_out, (float4 *)p.d_s_dat, (float4 *)p.d_t_dat,
            p.grid_mode ? p.d_cell : nullptr, p.d_s_cell, p.d_t_cell);
}

// ---------------------------------------------------------------- validation of a learned call
//
// The learned result S_l (in S_out) against the threshold rule's S_t (the plain FMM of the
// same call): rel = ||S_l - S_t||_2 / ||S_t||_2 over every point (non-targets are 0 in both),
// summed in FP64 in a fixed order.  If rel > tol, or rel is not finite, the threshold result
// replaces the learned one and the call counts as fallen back.

namespace {

constexpr int kValBlocks = 512;

template <class T>
__global__ __launch_bounds__(256) void validate_partials_kernel(const T *__restrict__ Sl, const T *__restrict__ Sr,
                                                                int64_t n, double *__restrict__ partial)
{
    __shared__ double sd[256], sr[256];
    double d2 = 0.0, r2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)Sl[i], b = (double)Sr[i];
        d2 += (a - b) * (a - b);
        r2 += b * b;
    }
    sd[threadIdx.x] = d2;
    sr[threadIdx.x] = r2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sd[threadIdx.x] += sd[threadIdx.x + o];
            sr[threadIdx.x] += sr[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sd[0];
        partial[2 * blockIdx.x + 1] = sr[0];
    }
}

// every workgroup reduces the partials (the same order, so the same decision), then copies
template <class T>
__global__ __launch_bounds__(256) void validate_apply_kernel(T *__restrict__ Sl, const T *__restrict__ Sr, int64_t n,
                                                             const double *__restrict__ partial, int nb, double tol,
                                                             CallScalars *__restrict__ sc)
{
    __shared__ double rel_s;
    if (threadIdx.x == 0) {
        double d2 = 0.0, r2 = 0.0;
        for (int b = 0; b < nb; ++b) {
            d2 += partial[2 * b];
            r2 += partial[2 * b + 1];
        }
        rel_s = r2 > 0.0 ? sqrt(d2 / r2) : (d2 > 0.0 ? INFINITY : 0.0);
        if (blockIdx.x == 0) sc->check_rel = rel_s;
    }
    __syncthreads();
    const double rel = rel_s;
    const bool back = !(rel <= tol);
    if (!back) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->fallback = 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        Sl[i] = Sr[i];
}

}  // namespace

void launch_validate(const Plan &p, void *S_out, const void *S_ref, double tol, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>(kValBlocks, (p.n + 255) / 256);
    double *partial = reinterpret_cast<double *>(p.d_scan_tmp);
    if (p.precision == PH_FP64) {
        validate_partials_kernel<double><<<nb, 256, 0, s>>>((const double *)S_out, (const double *)S_ref, p.n, partial);
        validate_apply_kernel<double><<<nb, 256, 0, s>>>((double *)S_out, (const double *)S_ref, p.n, partial, nb, tol,
                                                         p.d_sc);
    } else {
        validate_partials_kernel<float><<<nb, 256, 0, s>>>((const float *)S_out, (const float *)S_ref, p.n, partial);
        validate_apply_kernel<float><<<nb, 256, 0, s>>>((float *)S_out, (const float *)S_ref, p.n, partial, nb, tol,
                                                        p.d_sc);
    }
}

}  // namespace ph
