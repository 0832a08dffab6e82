// Adaptive selection and compaction (Sec. 3 strategies 1-2; Sec. 4.3 eq. (22); Sec. 5 field rule).
//
// Source j is kept iff I_j >= src_rel * max_k I_k (the maximum over every
// point); target i is kept iff |E_i| >= e_abs and/or
// |E_i| >= E_applied + eps (max|E| - E_applied).  Every comparison is made in
// FP64 between the stored value (exactly widened) and an FP64 threshold.
// Compaction walks the Morton order, so the selected lists stay sorted and
// every octree box is a contiguous run in each list.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "k_common.h"
#include "k_mlp_dev.h"

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

// Maxima of I and |E| and the order keys that locate them.  Each of at most kRedBlocks blocks
// reduces its grid-stride share (eight elements per thread in flight) into partials: the
// largest I, marked if a bad value was seen, and the order keys of |E| and of I (value bits
// above the complemented caller index: the largest key is the largest value, first in caller
// order among ties).  The consumers reduce the few partials themselves: maxima do not depend on
// the order of reduction, and no two blocks write one address.
constexpr int kRedUnroll = 8;
constexpr int kRedBlocks = 1024;

template <class T>
__global__ __launch_bounds__(256) void reduce_max_kernel(const T *__restrict__ I, const float *__restrict__ E,
                                                         int64_t n, double *__restrict__ partial,
                                                         uint64_t *__restrict__ pkey, uint64_t *__restrict__ pikey,
                                                         CallScalars *sc, int32_t *gen)
{
    if (blockIdx.x == 0 && gen) begin_call(sc, gen);
    __shared__ double smI[4];
    __shared__ uint64_t smE[4], smK[4];
    __shared__ int anybad;
    double mi = 0.0;
    uint64_t me = 0, mk = 0;
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += kRedUnroll * stride) {
        T v[kRedUnroll];
        float e[kRedUnroll];
#pragma unroll
        for (int u = 0; u < kRedUnroll; ++u) {
            const int64_t i = i0 + u * stride;
            v[u] = i < n ? I[i] : T(0);
            e[u] = (E && i < n) ? E[i] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kRedUnroll; ++u) {
            const int64_t i = i0 + u * stride;
            if (i >= n) continue;
            if (bad_value(v[u])) {
                bad = 1;
            } else {
                mi = fmax(mi, (double)v[u]);
                mk = max(mk, e_key((float)v[u], i));
            }
            if (E) me = max(me, e_key(e[u], i));
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mi = fmax(mi, __shfl_xor(mi, o));
        me = max(me, shfl_xor_u64(me, o));
        mk = max(mk, shfl_xor_u64(mk, o));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) anybad = 0;
    __syncthreads();
    if (bad) anybad = 1;
    if (lane == 0) {
        smI[wv] = mi;
        smE[wv] = me;
        smK[wv] = mk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = smI[0];
        uint64_t k = smE[0], q = smK[0];
        for (int w = 1; w < 4; ++w) {
            m = fmax(m, smI[w]);
            k = max(k, smE[w]);
            q = max(q, smK[w]);
        }
        partial[blockIdx.x] = mark_bad(m, anybad != 0);
        pkey[blockIdx.x] = k;
        pikey[blockIdx.x] = q;
    }
}

// Sorted position of the point an order key names (caller index in the complemented low word)
__device__ __forceinline__ int64_t key_point(uint64_t key, const int32_t *__restrict__ iperm)
{
    return iperm[0xffffffffu - (uint32_t)(key & 0xffffffffu)];
}

struct Maxima {
    double imax, emax;
    uint64_t ekey, ikey;
    int bad;
};

// The maxima over the nb partials at red, by a whole workgroup (every thread gets them)
__device__ Maxima block_maxima(const double *__restrict__ red, int nb)
{
    const double *partial = red;
    const uint64_t *pkey = reinterpret_cast<const uint64_t *>(red + kRedBlocks), *pikey = pkey + kRedBlocks;
    __shared__ double sI[16];
    __shared__ uint64_t sE[16], sK[16];
    __shared__ int sbad;
    double mi = 0.0;
    uint64_t me = 0, mk = 0;
    bool b = false;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
        mi = fmax(mi, partial_max(partial[j], b));
        me = max(me, pkey[j]);
        mk = max(mk, pikey[j]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mi = fmax(mi, __shfl_xor(mi, o));
        me = max(me, shfl_xor_u64(me, o));
        mk = max(mk, shfl_xor_u64(mk, o));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();
    if (b) sbad = 1;
    if (lane == 0) {
        sI[wv] = mi;
        sE[wv] = me;
        sK[wv] = mk;
    }
    __syncthreads();
    Maxima m{0.0, 0.0, 0, 0, 0};
    const int nw = (int)(blockDim.x >> 6);
    for (int q = 0; q < nw; ++q) {
        m.imax = fmax(m.imax, sI[q]);
        m.ekey = max(m.ekey, sE[q]);
        m.ikey = max(m.ikey, sK[q]);
    }
    m.emax = (double)__uint_as_float((uint32_t)(m.ekey >> 32));
    m.bad = sbad;
    return m;
}

// The call's maxima, their keys and the positions of the two points into its scalars (one thread)
__device__ void store_maxima(const Maxima &m, CallScalars *sc, int32_t *sticky, const int32_t *__restrict__ iperm,
                             const double *__restrict__ xyz, bool has_e)
{
    if (m.bad) flag_error(sc, sticky, 1);
    sc->imax = m.imax;
    sc->emax = m.emax;
    sc->emax_key = m.ekey;
    sc->imax_key = m.ikey;
    double xe[3] = {0.0, 0.0, 0.0}, xi[3] = {0.0, 0.0, 0.0};
    if (has_e && m.emax > 0.0) {
        const int64_t k = key_point(m.ekey, iperm);
        for (int d = 0; d < 3; ++d) xe[d] = xyz[3 * k + d];
    }
    if (m.imax > 0.0) {
        const int64_t k = key_point(m.ikey, iperm);
        for (int d = 0; d < 3; ++d) xi[d] = xyz[3 * k + d];
    }
    for (int d = 0; d < 3; ++d) {
        sc->emax_xyz[d] = xe[d];
        sc->imax_xyz[d] = xi[d];
    }
}

// First kernel of a call on the previous call's sets: the call's work counters, error bits and
// validation figure start from zero; the sets, the tree, the lists and the call number stay.
__global__ void reuse_begin_kernel(CallScalars *sc)
{
    for (int i = threadIdx.x; i < 12; i += blockDim.x) sc->work[i] = 0ull;
    if (threadIdx.x == 0) {
        sc->err = 0;
        sc->check_rel = 0.0;
    }
}

// The training entry points' step between the reduction and their own passes
__global__ __launch_bounds__(256) void maxima_store_kernel(const double *__restrict__ red, int nb, CallScalars *sc,
                                                           int32_t *sticky, const int32_t *__restrict__ iperm,
                                                           const double *__restrict__ xyz, int has_e)
{
    const Maxima m = block_maxima(red, nb);
    if (threadIdx.x == 0) store_maxima(m, sc, sticky, iperm, xyz, has_e != 0);
}

struct SelectParams {
    double src_rel, e_abs, e_applied, e_rel;
    double fallback_rel;          // source rule of a leaf whose learned decision is not finite
};

__device__ __forceinline__ bool src_rule(double v, double rel, double imax) { return (rel <= 0.0) || (v >= rel * imax); }

// Target flag of a point: the caller's set (tmask, null: every point) and the field rules
__device__ __forceinline__ bool tgt_rule(const SelectParams &sp, float ev, bool has_e, double emax, uint8_t tm)
{
    bool tgt = tm != 0;
    if (has_e) {
        const double e = (double)ev;
        if (sp.e_abs >= 0.0) tgt = tgt && (e >= sp.e_abs);
        if (sp.e_rel >= 0.0) tgt = tgt && (e >= sp.e_applied + sp.e_rel * (emax - sp.e_applied));
    }
    return tgt;
}

__device__ __forceinline__ uint64_t packed_of(uint32_t f)
{
    return (uint64_t)(f & 1u) | ((uint64_t)(f >> 1) << 32);
}

// Selection in two passes over tiles of kSelTile sorted points (1024 threads; wave w owns a
// contiguous sixteenth, read as kSelStrips coalesced strips of 64), with a scan of the tile
// sums between them.  Pass one: the flags of every point (one byte each: bit 0 source, bit 1
// target), S = 0 at points that are not targets, and each tile's packed count (sources |
// targets << 32).  With the learned selector it also decides on the plan leaves that hold
// candidates (below).
constexpr int kSelWaves = 16;
constexpr int kSelStrips = 4;
constexpr int kSelSpan = 64 * kSelStrips;  // points per wave in a tile
constexpr int kSelTile = kSelWaves * kSelSpan;
static_assert(kSelTile == kSelTilePoints, "the plan's tile table uses the same tile");

// The learned selector, around the selection pass.  The plan leaves are listed by first point
// (leaf_pos: first, end, plan-leaf index), and each tile knows the range of them that overlaps
// it (tile_leaves).  The learned variant of the pass flags the sources by the plan's rule (the
// candidates) as the plain pass does, and in addition lists every plan leaf that holds a
// candidate (the rows), once, by the tile that holds the leaf's first point.  A second pass
// (learned_decide_kernel) then takes the rows a wave each, all of them at once across the
// device: statistics, features, the network's BF16 logit; keep iff logit >= threshold, else
// the leaf's candidates lose their source flag; a non-finite logit puts the leaf under the
// fallback rule.  The tile counts are corrected there, before the compaction reads them.
struct LearnArgs {
    const int2 *tile_leaves;     // per tile: [first, end) in leaf_pos
    const int4 *leaf_pos;        // plan leaves by first point: (first, end, plan-leaf index, 0)
    const int4 *pinfo2;          // per plan leaf: anchor x, y, z, level
    const double *w;             // sorted weights (null on grids)
    const float *params;         // network weights (FP32; BF16 in use)
    float threshold;
    double w_ref, lo0, lo1, lo2, cube;
    float *feats;                // per plan leaf: its features (candidate leaves)
    uint32_t *leafflag;          // per plan leaf: 1 if it held a candidate in this call
    int32_t *featcnt;            // per plan leaf: candidates
    int4 *rows;                  // the call's rows: (first, end, plan-leaf index, 0)
    int count;                   // count rows and candidates into the scalars (calls with statistics)
};

// Is a candidate among the tile's points [a, b) (tile-relative)?  cand: a word per 64 points.
__device__ __forceinline__ bool any_cand(const uint64_t *cand, int a, int b)
{
    for (int q = a >> 6; q <= (b - 1) >> 6; ++q) {
        uint64_t wq = cand[q];
        const int lo = q * 64;
        if (a > lo) wq &= ~0ull << (a - lo);
        if (b < lo + 64) wq &= (1ull << (b - lo)) - 1ull;
        if (wq) return true;
    }
    return false;
}

template <class T, bool LEARNED>
__global__ __launch_bounds__(64 * kSelWaves, 8) void select_tiles_kernel(
    const T *__restrict__ I, const float *__restrict__ E, const int32_t *__restrict__ perm, int64_t n,
    SelectParams sp, CallScalars *__restrict__ sc, const double *__restrict__ red, int red_nb, int32_t *sticky,
    const int32_t *__restrict__ iperm, const double *__restrict__ xyz, const uint8_t *__restrict__ tmask,
    uint8_t *__restrict__ sel, T *__restrict__ S_out, uint64_t *__restrict__ partial, LearnArgs la)
{
    __shared__ uint64_t wsum[kSelWaves];
    __shared__ uint64_t cand[LEARNED ? kSelTile / 64 : 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // the tile: consecutive tiles on one XCD (their points' rows share cache lines)
    const int64_t bt = xcd_contiguous(blockIdx.x, gridDim.x);
    const int64_t tile0 = bt * kSelTile;
    const int64_t base = tile0 + (int64_t)w * kSelSpan;
    // the tile's values first (they do not depend on the maxima), then the maxima from the partials
    int32_t o[kSelStrips];
    T v[kSelStrips];
    float e[kSelStrips];
    uint8_t tm[kSelStrips];
    int2 lrange = make_int2(0, 0);
    if constexpr (LEARNED) lrange = la.tile_leaves[bt];
    // (lanes past the end read the last point, so that the loads need no per-lane branch, each
    // of which would cost a round trip of its own, and go out together; the flags below test k)
#pragma unroll
    for (int st = 0; st < kSelStrips; ++st) o[st] = perm[min(base + st * 64 + lane, n - 1)];
    if (tmask) {
#pragma unroll
        for (int st = 0; st < kSelStrips; ++st) tm[st] = tmask[min(base + st * 64 + lane, n - 1)];
    } else {
#pragma unroll
        for (int st = 0; st < kSelStrips; ++st) tm[st] = 1;
    }
    // the learned variant's leaf records, in flight with the tile's values
    int4 lpre = make_int4(0, 0, 0, 0);
    if constexpr (LEARNED) {
        if ((int)threadIdx.x < lrange.y - lrange.x) lpre = la.leaf_pos[lrange.x + threadIdx.x];
    }
#pragma unroll
    for (int st = 0; st < kSelStrips; ++st) v[st] = I[o[st]];
    if (E) {
#pragma unroll
        for (int st = 0; st < kSelStrips; ++st) e[st] = E[o[st]];
    } else {
#pragma unroll
        for (int st = 0; st < kSelStrips; ++st) e[st] = 0.0f;
    }
    const Maxima mx = block_maxima(red, red_nb);
    const double imax = mx.imax, emax = mx.emax;
    uint64_t acc = 0;
#pragma unroll
    for (int st = 0; st < kSelStrips; ++st) {
        const int64_t k = base + st * 64 + lane;
        const bool src = k < n && src_rule((double)v[st], sp.src_rel, imax);
        if constexpr (LEARNED) {
            const uint64_t cw = __ballot(src);
            if (lane == 0) cand[w * kSelStrips + st] = cw;
        }
        if (k < n) {
            const bool tgt = tgt_rule(sp, e[st], E != nullptr, emax, tm[st]);
            const uint32_t f = (src ? 1u : 0u) | (tgt ? 2u : 0u);
            sel[k] = (uint8_t)f;
            if (!tgt) S_out[o[st]] = T(0);
            acc += packed_of(f);
        }
    }
    if constexpr (LEARNED) {
        // the rows: leaves whose first point is in this tile and that hold a candidate
        __syncthreads();
        const int64_t t1 = min(n, tile0 + kSelTile);
        for (int32_t li = lrange.x + (int32_t)threadIdx.x; li < lrange.y; li += (int32_t)blockDim.x) {
            const int4 lp = li - lrange.x < (int32_t)blockDim.x ? lpre : la.leaf_pos[li];
            bool c = false;
            if (lp.x >= tile0) {
                c = any_cand(cand, (int)(lp.x - tile0), (int)(min((int64_t)lp.y, t1) - tile0));
                // a leaf that runs into the next tile: the rest of its points from memory
                for (int32_t k = (int32_t)t1; k < lp.y && !c; ++k) c = src_rule((double)I[perm[k]], sp.src_rel, imax);
                la.leafflag[lp.z] = c ? 1u : 0u;
            }
            wave_append(c, la.rows, &sc->n_rows, lp);
        }
    }
    // workgroup 0 publishes the maxima for the later kernels (after its own points)
    if (blockIdx.x == 0 && threadIdx.x == 0) store_maxima(mx, sc, sticky, iperm, xyz, E != nullptr);
    acc = lane_value(wave_inclusive(acc, lane), 63);
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int q = 0; q < kSelWaves; ++q) t += wsum[q];
        partial[bt] = t;
    }
}

// The decisions on the rows, a wave per row over the whole device (the rows of a call are few
// and independent).  The leaf's statistics read I and |E| through the permutation, with the
// same function as the training entry points, so the features are those the network was
// trained on, bit for bit; the logit is mlp_row's.  A dropped leaf's candidates lose their
// source flag, a leaf under the fallback rule gets the flags of that rule, and the tiles'
// source counts follow (one atomic per tile the leaf touches).
constexpr int kDecideWaves = 4;

template <class T>
__global__ __launch_bounds__(64 * kDecideWaves) void learned_decide_kernel(
    const T *__restrict__ I, const float *__restrict__ E, const int32_t *__restrict__ perm, SelectParams sp,
    CallScalars *__restrict__ sc, LearnArgs la, uint8_t *__restrict__ sel, uint64_t *__restrict__ partial)
{
    __shared__ mlp::MlpLds net;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t nrows = sc->n_rows;
    if ((int32_t)blockIdx.x * kDecideWaves >= nrows) return;  // the whole workgroup: no row for it
    // the wave's first row: its record, then its geometry and the permutation of its first 64
    // points, then their values, with the network's weights in flight behind the record (a
    // wave past the rows, or a lane past its leaf, reads the last row or point: every load is
    // unconditional, so that none waits on its own, and the values go unused)
    // the call's maxima and their positions first: the kernel also writes the scalars, so these
    // are vector loads, and issued here they share the first round trip
    mlp::FeatureRefs r;
    r.imax = sc->imax;
    r.emax = sc->emax;
    r.w_ref = la.w_ref;
    r.lo[0] = la.lo0;
    r.lo[1] = la.lo1;
    r.lo[2] = la.lo2;
    r.cube = la.cube;
    r.efeat = E && r.emax > 0.0;
    for (int d = 0; d < 3; ++d) {
        r.xi[d] = sc->imax_xyz[d];
        r.xe[d] = sc->emax_xyz[d];
    }
    int32_t row = (int32_t)blockIdx.x * kDecideWaves + wv;
    int4 lp = la.rows[min(row, nrows - 1)];
    constexpr int kW = (PH_MLP_NPARAM + 64 * kDecideWaves - 1) / (64 * kDecideWaves);
    float wts[kW];
    mlp::load_weights<kW>(la.params, wts);
    int4 g = la.pinfo2[lp.z];
    double pv, pe = 0.0;
    {
        const int32_t o = perm[min(lp.x + lane, lp.y - 1)];
        pv = (double)I[o];
        if (E) pe = (double)E[o];
    }
    mlp::store_weights<true, kW>(wts, net);
    __syncthreads();
    bool first = true;
    for (; row < nrows; row += (int32_t)gridDim.x * kDecideWaves) {
        if (!first) {
            lp = la.rows[row];
            g = la.pinfo2[lp.z];
        }
        const bool pre = first;
        first = false;
        auto fetch = [&](int32_t k, double &v, double &e) {
            if (pre && k < lp.x + 64) {  // this lane's prefetched point
                v = pv;
                e = pe;
                return;
            }
            const int32_t o = perm[k];
            v = (double)I[o];
            e = E ? (double)E[o] : 0.0;
        };
        const mlp::LeafStats st = mlp::leaf_stats_wave(fetch, la.w, la.w_ref, lp.x, lp.y, sp.src_rel, r.imax, lane);
        float fe[PH_MLP_NIN];
        mlp::leaf_features(st, r, g.w, g.x, g.y, g.z, fe);
        if (lane < PH_MLP_NIN) {
            float f = fe[0];
#pragma unroll
            for (int q = 1; q < PH_MLP_NIN; ++q) f = lane == q ? fe[q] : f;
            la.feats[(size_t)lp.z * PH_MLP_NIN + lane] = f;
        }
        if (lane == 0) {
            la.featcnt[lp.z] = (int32_t)st.n_c;
            if (la.count) {  // calls that report statistics: the rows and their candidates
                atomicAdd(&sc->n_src_base, (int32_t)st.n_c);
                atomicAdd(&sc->n_srcleaf, 1);
            }
        }
        const float z = mlp::mlp_row<true>(fe, net, lane);
        if (isfinite(z) && z >= la.threshold) continue;  // kept: the flags stand
        const bool fb = !isfinite(z);
        if (fb && lane == 0) atomicOr(&sc->fallback, 1);
        // new source flags on the leaf's points; the change of each tile's count (a leaf touches
        // at most two tiles: it holds fewer points than a tile)
        const int64_t tA = (int64_t)lp.x / kSelTile;
        int32_t dA = 0, dB = 0;
        for (int32_t k = lp.x + lane; k < lp.y; k += 64) {
            const uint32_t f = sel[k];
            const uint32_t was = f & 1u;
            const uint32_t now = fb ? (src_rule((double)I[perm[k]], sp.fallback_rel, r.imax) ? 1u : 0u) : 0u;
            if (was == now) continue;
            sel[k] = (uint8_t)((f & ~1u) | now);
            const int32_t d = (int32_t)now - (int32_t)was;
            if ((int64_t)k / kSelTile == tA) dA += d;
            else dB += d;
        }
        for (int off = 32; off > 0; off >>= 1) {
            dA += __shfl_xor(dA, off);
            dB += __shfl_xor(dB, off);
        }
        if (lane == 0) {
            // the count sits in the low word of the packed value, which stays >= 0
            if (dA) atomicAdd((unsigned long long *)&partial[tA], (unsigned long long)(int64_t)dA);
            if (dB) atomicAdd((unsigned long long *)&partial[tA + 1], (unsigned long long)(int64_t)dB);
        }
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
    const int32_t *__restrict__ cell, int32_t *__restrict__ s_cell, int32_t *__restrict__ t_cell,
    TI *__restrict__ S_zero, int32_t *sticky)
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
    // the tile's flags and box-boundary marks first (they do not depend on the offset)
    // (lanes past the end read the last point, so that the loads need no branch and go out together)
    const int64_t base = (int64_t)blockIdx.x * kSelTile + (int64_t)wv * kSelSpan;
    uint32_t f[kStrips], bd[kStrips];
#pragma unroll
    for (int st = 0; st < kStrips; ++st) {
        const int64_t k = min(base + st * 64 + lane, n - 1);
        f[st] = sel[k];
        bd[st] = bnd[k];
    }
#pragma unroll
    for (int st = 0; st < kStrips; ++st)
        if (base + st * 64 + lane >= n) f[st] = bd[st] = 0u;
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
    uint64_t acc = 0;
#pragma unroll
    for (int st = 0; st < kStrips; ++st) acc += packed_of(f[st]);
    acc = lane_value(wave_inclusive(acc, lane), 63);
    if (lane == 0) wsum[wv] = acc;
    __syncthreads();
    uint64_t carry = tile_off;
    for (int q = 0; q < wv; ++q) carry += wsum[q];
    uint64_t here[kStrips];
    bool wr[kStrips], any = false;
#pragma unroll
    for (int st = 0; st < kStrips; ++st) {
        const uint64_t v = packed_of(f[st]);
        const uint64_t incl = wave_inclusive(v, lane);
        here[st] = carry + incl - v;
        carry += lane_value(incl, 63);
        const int64_t k = base + st * 64 + lane;
        // points that are only targets need nothing more unless targets are compacted
        wr[st] = k < n && (tgt_compact ? f[st] != 0u : (f[st] & 1u) != 0u);
        any = any || wr[st];
        if (k >= n) continue;
        if (bd[st]) scanned[k] = here[st];
        // a call on the previous call's sets (S_zero set): the output at the points that are
        // not targets is cleared here, as the selection pass would have done
        if (S_zero && !(f[st] & 2u)) S_zero[perm[k]] = TI(0);
    }
    // the written points' data for all strips in two batches of loads (the permutation and
    // the point's record, then I through the permutation), in the waves that write any
    if (!__ballot(any)) return;
    int32_t o[kStrips], ce[kStrips];
    T x[kStrips], y[kStrips], z[kStrips];
#pragma unroll
    for (int st = 0; st < kStrips; ++st) {
        const int64_t k = min(base + st * 64 + lane, n - 1);
        o[st] = perm[k];
        ce[st] = cell ? cell[k] : 0;
        if constexpr (sizeof(C) == 8) {
            x[st] = (T)xyz[3 * k];
            y[st] = (T)xyz[3 * k + 1];
            z[st] = (T)xyz[3 * k + 2];
        } else {
            const C q = xyz[k];
            x[st] = q.x;
            y[st] = q.y;
            z[st] = q.z;
        }
    }
    TI Iraw[kStrips];
#pragma unroll
    for (int st = 0; st < kStrips; ++st) Iraw[st] = I[o[st]];
#pragma unroll
    for (int st = 0; st < kStrips; ++st) {
        if (!wr[st]) continue;
        const int64_t k = base + st * 64 + lane;
        const uint32_t sp_lo = (uint32_t)(here[st] & 0xffffffffu), sp_hi = (uint32_t)(here[st] >> 32);
        if (S_zero && bad_value(Iraw[st])) flag_error(sc, sticky, 1);  // no maxima pass checked it
        const double Iv = (double)Iraw[st] * scale;
        const bool is_src = f[st] & 1u;
        if (is_src) {
            const double wk = w ? w[k] : w_uniform;
            typename Vec4T<T>::type d;
            d.x = x[st];
            d.y = y[st];
            d.z = z[st];
            d.w = (T)(wk * Iv);
            s_dat[sp_lo] = d;
            if (cell) s_cell[sp_lo] = ce[st];
        }
        if ((f[st] & 2u) && tgt_compact) {
            t_out[sp_hi] = o[st];
            typename Vec4T<T>::type d;
            d.x = x[st];
            d.y = y[st];
            d.z = z[st];
            d.w = is_src ? (T)(c_self * Iv) : T(0);
            t_dat[sp_hi] = d;
            if (cell) t_cell[sp_hi] = ce[st];
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


int reduce_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (n + 2047) / 2048)); }
static_assert(kRedBytes == (size_t)kRedBlocks * 24, "partials buffer sized for the reduction's blocks");

void launch_reduce_max(const Plan &p, const void *I, const float *E, int32_t *gen, hipStream_t s)
{
    const int blocks = reduce_blocks(p.n);
    double *red = p.d_red;
    uint64_t *key = reinterpret_cast<uint64_t *>(red + kRedBlocks), *ikey = key + kRedBlocks;
    if (p.precision == PH_FP64)
        reduce_max_kernel<double><<<blocks, 256, 0, s>>>((const double *)I, E, p.n, red, key, ikey, p.d_sc, gen);
    else
        reduce_max_kernel<float><<<blocks, 256, 0, s>>>((const float *)I, E, p.n, red, key, ikey, p.d_sc, gen);
}

void launch_maxima_store(const Plan &p, bool has_e, hipStream_t s)
{
    maxima_store_kernel<<<1, 256, 0, s>>>(p.d_red, reduce_blocks(p.n), p.d_sc, p.d_sticky, p.d_iperm, p.d_xyz,
                                          has_e ? 1 : 0);
}

static SelectParams params_of(const Plan &p, double src_rel)
{
    return SelectParams{src_rel >= 0.0 ? src_rel : p.thr.src_rel, p.thr.e_abs, p.thr.e_applied, p.thr.e_rel,
                        p.fallback_rel};
}

void launch_select(const Plan &p, const void *I, const float *E, void *S_out, hipStream_t s, bool learned,
                   double src_rel, hipEvent_t after_tiles)
{
    if (p.n <= 0) return;
    const int64_t nb = (p.n + kSelTile - 1) / kSelTile;
    uint64_t *partial = p.d_tile_sum;
    const SelectParams sp = params_of(p, src_rel);
    LearnArgs la{};
    if (learned) {
        la.tile_leaves = p.d_tile_leaves;
        la.leaf_pos = p.d_leaf_pos;
        la.pinfo2 = p.d_pinfo2;
        la.w = p.d_w;
        la.params = p.d_sel_params;
        la.threshold = p.sel_threshold;
        la.w_ref = p.uniform_w ? p.w_uniform : p.cube_size * p.cube_size * p.cube_size / (double)p.n;
        la.lo0 = p.cube_lo[0];
        la.lo1 = p.cube_lo[1];
        la.lo2 = p.cube_lo[2];
        la.cube = p.cube_size;
        la.feats = p.d_feat;
        la.leafflag = p.d_leafflag;
        la.featcnt = p.d_feat_cnt;
        la.rows = p.d_rows;
        la.count = p.count_work ? 1 : 0;
    }
    const unsigned g = (unsigned)nb, bs = 64 * kSelWaves;
    const int rnb = reduce_blocks(p.n);
    if (p.precision == PH_FP64) {
        if (learned)
            select_tiles_kernel<double, true><<<g, bs, 0, s>>>((const double *)I, E, p.d_perm, p.n, sp, p.d_sc, p.d_red, rnb, p.d_sticky, p.d_iperm, p.d_xyz, p.d_tmask,
                                                               p.d_sel, (double *)S_out, partial, la);
        else
            select_tiles_kernel<double, false><<<g, bs, 0, s>>>((const double *)I, E, p.d_perm, p.n, sp, p.d_sc, p.d_red, rnb, p.d_sticky, p.d_iperm, p.d_xyz, p.d_tmask, p.d_sel, (double *)S_out, partial, la);
    } else {
        if (learned)
            select_tiles_kernel<float, true><<<g, bs, 0, s>>>((const float *)I, E, p.d_perm, p.n, sp, p.d_sc, p.d_red, rnb, p.d_sticky, p.d_iperm, p.d_xyz, p.d_tmask,
                                                              p.d_sel, (float *)S_out, partial, la);
        else
            select_tiles_kernel<float, false><<<g, bs, 0, s>>>((const float *)I, E, p.d_perm, p.n, sp, p.d_sc, p.d_red, rnb, p.d_sticky, p.d_iperm, p.d_xyz, p.d_tmask,
                                                               p.d_sel, (float *)S_out, partial, la);
    }
    if (after_tiles) PH_HIP(hipEventRecord(after_tiles, s));
    if (learned) {
        // the rows' decisions: a wave per row; workgroups beyond the call's rows return at once
        const unsigned gd = (unsigned)std::max<int64_t>(1, std::min<int64_t>((p.n_pleaf + kDecideWaves - 1) / kDecideWaves, 1024));
        if (p.precision == PH_FP64)
            learned_decide_kernel<double><<<gd, 64 * kDecideWaves, 0, s>>>((const double *)I, E, p.d_perm, sp, p.d_sc, la,
                                                                          p.d_sel, partial);
        else
            learned_decide_kernel<float><<<gd, 64 * kDecideWaves, 0, s>>>((const float *)I, E, p.d_perm, sp, p.d_sc, la,
                                                                         p.d_sel, partial);
    }
    // up to 2048 tiles the compaction adds up the earlier tiles' sums itself; beyond, one
    // workgroup scans them first (in place: a call on the same sets reads the scan)
    if (nb > 2048) scan_tile_sums_u64(partial, nb, &p.d_sc->packed_total, s);
    launch_compact(p, I, nullptr, s);
}

// The compaction pass over the flags of the last selection pass.  S_zero: a call on the
// previous call's sets, whose output at the points that are not targets is cleared here.
void launch_compact(const Plan &p, const void *I, void *S_zero, hipStream_t s)
{
    const int64_t nb = (p.n + kSelTile - 1) / kSelTile;
    const uint64_t *partial = p.d_tile_sum;
    const int tile_sums = nb <= 2048 ? 1 : 0;
    if (p.precision == PH_FP64)
        select_compact_kernel<double, double, double><<<(unsigned)nb, 64 * kSelWaves, 0, s>>>(
            (const double *)I, p.d_perm, p.d_xyz, p.d_w, p.w_uniform, p.c_self, p.n, p.d_sc, p.d_sel, p.d_bnd,
            partial, nb, tile_sums, p.method == PH_METHOD_DIRECT ? 1 : 0, p.d_flag, p.d_t_out, (double4 *)p.d_s_dat, (double4 *)p.d_t_dat,
            p.grid_mode ? p.d_cell : nullptr, p.d_s_cell, p.d_t_cell, (double *)S_zero, p.d_sticky);
    else
        select_compact_kernel<float, float, float4><<<(unsigned)nb, 64 * kSelWaves, 0, s>>>(
            (const float *)I, p.d_perm, p.d_xyzf, p.d_w, p.w_uniform, p.c_self, p.n, p.d_sc, p.d_sel, p.d_bnd,
            partial, nb, tile_sums, p.method == PH_METHOD_DIRECT ? 1 : 0, p.d_flag, p.d_t_out, (float4 *)p.d_s_dat, (float4 *)p.d_t_dat,
            p.grid_mode ? p.d_cell : nullptr, p.d_s_cell, p.d_t_cell, (float *)S_zero, p.d_sticky);
}

void launch_reuse_begin(const Plan &p, hipStream_t s)
{
    reuse_begin_kernel<<<1, 64, 0, s>>>(p.d_sc);
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
