// Per-call adaptive octree over the selected sources and targets, and its interaction lists.
//
// Sec. 2.4: the octree is refined until every leaf holds at most a
// prescribed number of points; near interactions N(B) are summed exactly and
// far interactions F(B) go through the hierarchy.  Here a box is split while
// max(#selected sources, #selected targets) > leaf capacity.  The plan holds
// the tree over all points; since selected counts only shrink down the tree,
// the per-call tree is that tree pruned: a box belongs to it iff it holds
// selected points and its parent is split.  The selected lists are sorted by
// Morton key, so a box's range in each list is read off the selection scan at
// the ends of its range in the sorted point order.
//
// Lists (kernel-independent FMM of [ying2004], cited in Sec. 2.4):
//   U(B), leaf B : source leaves adjacent to B (any level, B included)
//   W(B), leaf B : descendants of B's colleagues not adjacent to B whose parent is
//                  adjacent to B (their artificial sources act on B's targets)
//   X(B), any B  : leaves not adjacent to B but adjacent to B's parent, coarser than B
//                  (their sources act on B's check points)
//   V(B)         : children of the parent's colleagues not adjacent to B; enumerated
//                  on the fly by the translation gather, not stored (the boxes with a
//                  non-empty V or X list are listed per level).
#include <hip/hip_runtime.h>

#include "k_common.h"

namespace ph {

namespace {

struct LevelInfo {
    int32_t base[kMaxDepth + 2];
    int32_t cap[kMaxDepth + 2];
    int32_t tbase[kMaxDepth + 2];  // first 64-slot tile of each level's source list
    int32_t depth;                 // deepest level
};

// Slot of each lane with pred in a list whose length is *counter: one atomic per wave, lanes in
// lane order; -1 for the other lanes.
__device__ __forceinline__ int32_t wave_slot(bool pred, int32_t *counter)
{
    const uint64_t m = __ballot(pred);
    if (m == 0) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, leader);
    return pred ? base + (int32_t)__popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// Per-call tree: the plan's tree over all points, pruned to the selected sets.
// Box ranges come from the exclusive scan of the packed (source | target << 32)
// selection indicators at the box's sorted-order range ends.
__device__ __forceinline__ uint64_t scan_at(const uint64_t *__restrict__ scanned, int32_t k, int64_t n,
                                            uint64_t total)
{
    // (the load is unconditional, at the last point past the end, so that it needs no branch
    // and goes out with the caller's other loads)
    const uint64_t v = scanned[k < n ? k : n - 1];
    return k < n ? v : total;
}

__global__ void tree_status_kernel(BoxArrays bx, LevelInfo li, int32_t nbox, int leaf_cap, int max_depth,
                                   const uint64_t *__restrict__ scanned, int64_t n, CallScalars *__restrict__ sc,
                                   uint32_t *__restrict__ tile_use, int32_t n_tile_words)
{
    const int32_t f0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (int32_t i = f0; i < n_tile_words; i += gridDim.x * blockDim.x) tile_use[i] = 0u;  // filled by the lists
    const int32_t f = f0 < nbox ? f0 : nbox - 1;  // whole waves reach the reduction below
    const bool mine = f0 < nbox;
    const uint64_t total = sc->packed_total;
    if (f == 0) {
        for (int l = 0; l <= li.depth; ++l) sc->lvl_count[l] = li.cap[l];
        for (int l = 0; l <= li.depth + 1; ++l) sc->lvl_start[l] = li.base[l];
    }
    // the box's and its parent's ranges and their scanned counts, each set of loads together
    const int32_t st = bx.start[f], en = bx.end[f], par = bx.parent[f], lev = bx.level[f];
    const int32_t pc = par >= 0 ? par : f;
    const int32_t pst = bx.start[pc], pen = bx.end[pc];
    const uint64_t a = scan_at(scanned, st, n, total), b = scan_at(scanned, en, n, total);
    const uint64_t pa = scan_at(scanned, pst, n, total), pb = scan_at(scanned, pen, n, total);
    const int32_t s0 = (int32_t)(a & 0xffffffffu), t0 = (int32_t)(a >> 32);
    const int32_t sn = (int32_t)(b & 0xffffffffu) - s0, tn = (int32_t)(b >> 32) - t0;
    bool exists = true;
    if (par >= 0) {
        const int32_t psn = (int32_t)(pb & 0xffffffffu) - (int32_t)(pa & 0xffffffffu);
        const int32_t ptn = (int32_t)(pb >> 32) - (int32_t)(pa >> 32);
        exists = (sn + tn > 0) && (max(psn, ptn) > leaf_cap);
    }
    // split in the plan's tree iff it holds more than leaf_cap points above the depth limit
    const bool split = exists && (en - st > leaf_cap) && (lev < max_depth) && (max(sn, tn) > leaf_cap);
    if (mine) {
        bx.s_first[f] = exists ? s0 : 0;
        bx.s_cnt[f] = exists ? sn : 0;
        bx.t_first[f] = exists ? t0 : 0;
        bx.t_cnt[f] = exists ? tn : 0;
        bx.flags[f] = exists ? (kBoxExists | (split ? 0 : kBoxLeaf)) : 0;
    }
    // per level: the boxes with sources and the split boxes with targets (the parents whose
    // local fields the next level needs), each with its slot in the level's list.  The slots
    // come from atomic appends (a wave rarely spans two levels): the order of the boxes within
    // a level enters no result, only the layout of the per-level products.
    const bool has_src = mine && exists && sn > 0, is_tpar = mine && split && tn > 0;
    int32_t srank = -1, trank = -1;
    uint64_t pending = __ballot(has_src || is_tpar);
    while (pending) {
        const int l0 = __shfl(lev, __ffsll((long long)pending) - 1);
        const bool here = lev == l0;
        const int32_t rs = wave_slot(has_src && here, &sc->lvl_src[l0]);
        const int32_t rt = wave_slot(is_tpar && here, &sc->lvl_tpar[l0]);
        if (here) {
            srank = rs;
            trank = rt;
        }
        pending &= ~__ballot(here);
    }
    if (mine) {
        bx.src_rank[f] = srank;
        if (srank >= 0) bx.src_box[li.base[lev] + srank] = f;
        if (trank >= 0) bx.tpar_box[li.base[lev] + trank] = f;
    }
    // lowest level holding a leaf with sources, as max of (depth + 1 - level), one atomic per wave
    int v = (mine && exists && !split && sn > 0) ? (li.depth + 1 - lev) : 0;
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0 && v > 0) atomicMax(&sc->min_leafsrc_level, v);
}

// ---------------------------------------------------------------- lists

__device__ __forceinline__ bool adjacent(const BoxArrays &bx, int32_t A, int32_t B)
{
    // closed intervals in units of the finest Morton cell
    const int la = bx.level[A], lb = bx.level[B];
    const int sa = kMortonBits - la, sb = kMortonBits - lb;
    const int a0 = bx.ax[A] << sa, a1 = (bx.ax[A] + 1) << sa;
    const int b0 = bx.ax[B] << sb, b1 = (bx.ax[B] + 1) << sb;
    if (a0 > b1 || b0 > a1) return false;
    const int c0 = bx.ay[A] << sa, c1 = (bx.ay[A] + 1) << sa;
    const int d0 = bx.ay[B] << sb, d1 = (bx.ay[B] + 1) << sb;
    if (c0 > d1 || d0 > c1) return false;
    const int e0 = bx.az[A] << sa, e1 = (bx.az[A] + 1) << sa;
    const int f0 = bx.az[B] << sb, f1 = (bx.az[B] + 1) << sb;
    return !(e0 > f1 || f0 > e1);
}

__device__ __forceinline__ int32_t box_of_thread(const LevelInfo &li, const CallScalars *sc, int32_t gid)
{
    for (int l = 0; l <= li.depth; ++l) {
        const int32_t i = gid - li.base[l];
        if (i >= 0 && i < li.cap[l]) return (i < sc->lvl_count[l]) ? gid : -1;
    }
    return -1;
}

enum { kListU = 0, kListW = 1, kListX = 2 };

// The first existing child of P after child `after` (any child if after < 0), or -1
__device__ __forceinline__ int32_t first_child(const BoxArrays &bx, int32_t P, int32_t after)
{
    const int32_t *ch = bx.child + (size_t)P * 8;
    int o = 0;
    if (after >= 0)
        while (o < 8 && ch[o] != after) ++o;
    for (o = after >= 0 ? o + 1 : 0; o < 8; ++o)
        if (ch[o] >= 0) return ch[o];
    return -1;
}

template <class F>
__device__ void enumerate_lists(const BoxArrays &bx, int32_t b, int min_leaf_level, F &&emit)
{
    if (bx.t_cnt[b] == 0) return;
    const bool leaf = bx.flags[b] & kBoxLeaf;
    if (leaf) {
        // the colleagues, then their counts and flags, each set of loads issued together
        int32_t Cs[27];
#pragma unroll
        for (int d = 0; d < 27; ++d) Cs[d] = bx.coll[(size_t)b * 27 + d];
        uint32_t lmask = 0, smask = 0;  // colleagues with sources: leaves, split boxes
#pragma unroll
        for (int d = 0; d < 27; ++d) {
            const int32_t C = Cs[d];
            const int32_t sn = C >= 0 ? bx.s_cnt[C] : 0;
            const int32_t fl = C >= 0 ? bx.flags[C] : 0;
            if (sn > 0) {
                if (fl & kBoxLeaf) lmask |= 1u << d;
                else smask |= 1u << d;
            }
        }
        for (uint32_t m = lmask | smask; m; m &= m - 1) {
            const int d = __ffs((int)m) - 1;
            const int32_t C = bx.coll[(size_t)b * 27 + d];
            if ((lmask >> d) & 1u) {
                emit(kListU, C);
                continue;
            }
            // the split colleague's descendants depth first in child order, walked through
            // the parent and child links (no stack): a box with sources that is not adjacent
            // to b joins W, an adjacent leaf joins U, an adjacent split box is descended into
            int32_t D = first_child(bx, C, -1);
            while (D >= 0) {
                bool down = false;
                if (bx.s_cnt[D] > 0) {
                    if (!adjacent(bx, D, b)) emit(kListW, D);
                    else if (bx.flags[D] & kBoxLeaf) emit(kListU, D);
                    else down = true;
                }
                const int32_t E = down ? first_child(bx, D, -1) : -1;
                if (E >= 0) {
                    D = E;
                    continue;
                }
                // the next sibling, else that of the nearest ancestor below C that has one
                while (true) {
                    const int32_t P = bx.parent[D];
                    const int32_t S = first_child(bx, P, D);
                    if (S >= 0) {
                        D = S;
                        break;
                    }
                    if (P == C) {
                        D = -1;
                        break;
                    }
                    D = P;
                }
            }
        }
    }
    // coarser leaves around the ancestors (none if every leaf with sources is this deep)
    if (bx.level[b] <= min_leaf_level) return;
    const int32_t par = bx.parent[b];
    for (int32_t A = par; A >= 0; A = bx.parent[A]) {
        for (int d = 0; d < 27; ++d) {
            const int32_t C = bx.coll[(size_t)A * 27 + d];
            if (C < 0 || C == A || !(bx.flags[C] & kBoxLeaf) || bx.s_cnt[C] == 0) continue;
            if (adjacent(bx, C, b)) {
                if (leaf) emit(kListU, C);
            } else if (adjacent(bx, C, par)) {
                emit(kListX, C);
            }
        }
    }
}

constexpr int kListBlock = 256;

// Space for n entries per lane from a shared counter: one atomic per wave, lanes in order.
// Every lane of the wave takes part.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t n, int32_t *counter)
{
    const int lane = threadIdx.x & 63;
    const uint32_t incl = wave_inclusive(n, lane);
    const uint32_t tot = lane_value(incl, 63);
    uint32_t base = 0;
    if (lane == 63 && tot) base = atomicAdd(reinterpret_cast<unsigned int *>(counter), tot);
    return lane_value(base, 63) + incl - n;
}

// The interaction lists of every box in one pass.  A workgroup takes 64 boxes; each half wave
// resolves 8 of them with one lane per colleague (lane c < 27: colleague c), all their loads
// issued together.  A leaf with targets whose colleagues with sources are all leaves, and whose
// level needs no look at coarser leaves (the common case), has only a U list: those colleagues
// in colleague order, written from the lanes.  Any other box with targets is enumerated by one
// lane of its half (descents into split colleagues, coarser leaves around the ancestors),
// counting first and writing after the reservation.  Wave 0 then reserves the workgroup's
// space (one atomic per list) and enters its boxes into the leaf lists of the target-side
// kernels (one atomic per list), a box per lane.  Each box stores its ranges.  grid_levels:
// bit l set when leaves of level l take their far field from a grid operator (or have none).
constexpr int kLBoxes = 64;               // boxes per workgroup
constexpr int kLPer = kLBoxes / 8;        // boxes per half wave

__global__ __launch_bounds__(kListBlock) void list_build_kernel(BoxArrays bx, LevelInfo li,
                                                                CallScalars *__restrict__ sc, int32_t nbox, Lists L,
                                                                uint32_t grid_levels, int32_t *sticky)
{
    static_assert(kListBlock == 256, "eight half waves");
    __shared__ int32_t sbox[kLBoxes], slev[kLBoxes];
    __shared__ uint32_t su[kLBoxes], sw[kLBoxes], sx[kLBoxes];     // counts, then first entries
    __shared__ uint32_t sumask[kLBoxes];                           // U colleagues (simple boxes)
    __shared__ uint8_t sser[kLBoxes], sleaf[kLBoxes];
    const int gen = sc->gen;
    const int t = threadIdx.x, lane = t & 63, half = lane >> 5, hl = lane & 31;
    const int hw = t >> 5;  // half wave 0..7
    const int mll = li.depth + 1 - sc->min_leafsrc_level;
    const int32_t g0 = (int32_t)blockIdx.x * kLBoxes;
    // the half's boxes, their colleagues and the colleagues' counts, each set of loads together
    int32_t bq[kLPer], C[kLPer];
    int32_t lv[kLPer];
    bool tg[kLPer], lf[kLPer];
#pragma unroll
    for (int i = 0; i < kLPer; ++i) {
        const int32_t gid = g0 + hw * kLPer + i;
        bq[i] = gid < nbox ? box_of_thread(li, sc, gid) : -1;
    }
#pragma unroll
    for (int i = 0; i < kLPer; ++i) {
        const int32_t b = bq[i];
        tg[i] = b >= 0 && bx.t_cnt[b] > 0;
        const int32_t fl = b >= 0 ? bx.flags[b] : 0;
        lv[i] = b >= 0 ? bx.level[b] : 0;
        lf[i] = tg[i] && (fl & kBoxLeaf);
    }
#pragma unroll
    for (int i = 0; i < kLPer; ++i) C[i] = (lf[i] && hl < 27) ? bx.coll[(size_t)bq[i] * 27 + hl] : -1;
    uint32_t um[kLPer], sm[kLPer];
#pragma unroll
    for (int i = 0; i < kLPer; ++i) {
        bool isu = false, iss = false;
        if (C[i] >= 0) {
            const int32_t sn = bx.s_cnt[C[i]], cf = bx.flags[C[i]];
            isu = sn > 0 && (cf & kBoxLeaf);
            iss = sn > 0 && !(cf & kBoxLeaf);
        }
        um[i] = (uint32_t)(__ballot(isu) >> (32 * half));
        sm[i] = (uint32_t)(__ballot(iss) >> (32 * half));
    }
    // the half's boxes to LDS (lane i for box i)
#pragma unroll
    for (int i = 0; i < kLPer; ++i) {
        if (hl == i) {
            const int j = hw * kLPer + i;
            const bool ser = tg[i] && (sm[i] != 0 || lv[i] > mll);
            sbox[j] = bq[i];
            slev[j] = lv[i];
            su[j] = ser ? 0u : (uint32_t)__popc(um[i]);
            sw[j] = 0;
            sx[j] = 0;
            sumask[j] = um[i];
            sser[j] = ser;
            sleaf[j] = lf[i];
        }
    }
    __syncthreads();
    // boxes that need the full enumeration: counted by lane i of the half for its box i
    const int jm = hw * kLPer + (hl & (kLPer - 1));
    const bool my_ser = hl < kLPer && sser[jm];
    if (my_ser) {
        uint32_t nu = 0, nw = 0, nx = 0;
        enumerate_lists(bx, sbox[jm], mll, [&](int kind, int32_t) {
            if (kind == kListU) ++nu;
            else if (kind == kListW) ++nw;
            else ++nx;
        });
        su[jm] = nu;
        sw[jm] = nw;
        sx[jm] = nx;
    }
    __syncthreads();
    // wave 0: the workgroup's space, a box per lane (one atomic per list)
    if (t < kLBoxes) {
        const uint32_t nu = su[t], nw = sw[t], nx = sx[t];
        const uint32_t ub = wave_reserve(nu, &sc->n_u);
        const uint32_t wb = wave_reserve(nw, &sc->n_w);
        const uint32_t xb = wave_reserve(nx, &sc->n_x);
        const int32_t gid = g0 + t;
        if (gid < nbox) {
            // ranges past a list's capacity are cut at it (their entries are not stored, and the
            // overflow is reported), so that no reader leaves the list
            L.u_rng[gid] = clamp_range(ub, nu, L.u_cap);
            L.w_rng[gid] = clamp_range(wb, nw, L.w_cap);
            L.x_rng[gid] = clamp_range(xb, nx, L.x_cap);
            if ((int64_t)ub + nu > L.u_cap || (int64_t)wb + nw > L.w_cap || (int64_t)xb + nx > L.x_cap)
                flag_error(sc, sticky, 2);
        }
        su[t] = ub;  // first entries from here on
        sw[t] = wb;
        sx[t] = xb;
        // the box's entries in the target-side lists
        const int32_t b = sbox[t];
        const int lev = slev[t];
        const bool tleaf = sleaf[t] != 0;
        const bool grid_leaf = tleaf && ((grid_levels >> lev) & 1u);
        // grid-operator leaves go to their level's segment (a wave rarely spans two levels)
        uint64_t pending = __ballot(grid_leaf);
        // the leaf's points in sorted order (its targets are those with the target flag)
        const int4 entry = make_int4(b, b >= 0 ? bx.start[b] : 0, b >= 0 ? bx.end[b] - bx.start[b] : 0,
                                     (nu > 0 ? 1 : 0) | (nw > 0 ? 2 : 0));
        while (pending) {
            const int l0 = __shfl(lev, __ffsll((long long)pending) - 1);
            const bool mine = grid_leaf && lev == l0;
            wave_append(mine, L.far_a + li.base[l0], &sc->n_far_a_lvl[l0], entry);
            pending &= ~__ballot(mine);
        }
        wave_append(tleaf && !grid_leaf, L.far_b, &sc->n_far_b, b);
        wave_append(tleaf && nu > 0, L.near_leaves, &sc->n_near, b);
        // boxes of levels >= 3 with an X list join their level's V/X target segment
        const bool xbox = nx > 0 && lev >= 3 && atomicExch(&L.vt_tag[b], gen) != gen;
        pending = __ballot(xbox);
        while (pending) {
            const int l0 = __shfl(lev, __ffsll((long long)pending) - 1);
            const bool mine = xbox && lev == l0;
            wave_append(mine, L.vt + li.base[l0], &sc->n_vt_lvl[l0], b);
            pending &= ~__ballot(mine);
        }
    }
    __syncthreads();
    // the entries: enumerated boxes by lane i of the half, simple boxes from the colleague lanes
    if (my_ser) {
        uint32_t pu = su[jm], pw = sw[jm], px = sx[jm];
        bool over = false;
        enumerate_lists(bx, sbox[jm], mll, [&](int kind, int32_t E) {
            if (kind == kListU) {
                if (pu < (uint32_t)L.u_cap) L.u[pu] = E;
                else over = true;
                ++pu;
            } else if (kind == kListW) {
                if (pw < (uint32_t)L.w_cap) L.w[pw] = E;
                else over = true;
                ++pw;
            } else {
                if (px < (uint32_t)L.x_cap) L.x[px] = E;
                else over = true;
                ++px;
            }
        });
        if (over) flag_error(sc, sticky, 2);
    }
#pragma unroll
    for (int i = 0; i < kLPer; ++i) {
        const int j = hw * kLPer + i;
        if (!sser[j] && hl < 27 && ((sumask[j] >> hl) & 1u)) {
            const uint32_t pos = su[j] + __popc(sumask[j] & ((1u << hl) - 1u));
            if (pos < (uint32_t)L.u_cap) L.u[pos] = C[i];
            else flag_error(sc, sticky, 2);
        }
    }
}

// Boxes of levels >= 3 that receive M2L translations, and the offsets each source box sends
// along.  B has source box S in its V list iff B is a child of a colleague of S's parent, not
// adjacent to S, at S's level; so one wave per source box S (levels >= 2) walks those
// candidates (the children of the parent's split colleagues), enters each one with targets
// once per call into its level's segment of vt (levels >= 3), stores the 316-bit mask of the
// offset slots used at S's slot, and ORs it into the mask of the 64-slot tile of the level's
// source list that holds S.
__global__ __launch_bounds__(256) void vtarget_kernel(BoxArrays bx, LevelInfo li, CallScalars *__restrict__ sc,
                                                      Lists L)
{
    const int gen = sc->gen;
    __shared__ uint32_t use[4][kUseWords];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    static_assert(kMaxDepth + 2 <= 64, "a lane per level");
    // the call's per-level counts, lane l holding level l's (read once, picked by readlane)
    const int32_t src_l = lane < kMaxDepth + 2 ? sc->lvl_src[lane] : 0;
    for (int32_t idx = blockIdx.x * 4 + wv;; idx += gridDim.x * 4) {
        int level = -1;
        int32_t r = idx;
        for (int l = 2; l <= li.depth; ++l) {
            const int32_t c = __builtin_amdgcn_readlane(src_l, l);
            if (r < c) {
                level = l;
                break;
            }
            r -= c;
        }
        if (level < 0) return;
        const int32_t S = bx.src_box[li.base[level] + r];
        const int32_t P = bx.parent[S];
        const int sx = bx.ax[S], sy = bx.ay[S], sz = bx.az[S];
        if (lane < kUseWords) use[wv][lane] = 0u;
        // the parent's colleagues; the children of those not split in this call have no
        // targets (every box outside the call's tree has zero counts), so the count test
        // below also stands for the colleague's own status
        const int32_t Qd = lane < 27 ? bx.coll[(size_t)P * 27 + lane] : -1;
        const uint64_t qmask = __ballot(Qd >= 0);
        const int nc = 8 * __popcll(qmask);
        __builtin_amdgcn_wave_barrier();
        // the candidates (8 children per colleague, up to 216): every child index, then every
        // child's target count and position, each batch of loads issued together
        constexpr int kC = (27 * 8 + 63) / 64;
        int32_t Bc[kC], dq[kC];
#pragma unroll
        for (int u = 0; u < kC; ++u) {
            const int f = 64 * u + lane;
            uint64_t m = qmask;
            for (int j = f < nc ? (f >> 3) : 0; j > 0; --j) m &= m - 1;
            const int d = m ? __ffsll((long long)m) - 1 : 0;
            const int32_t Q = __shfl(Qd, d);
            dq[u] = d;
            Bc[u] = f < nc ? bx.child[(size_t)Q * 8 + (f & 7)] : -1;
        }
        int32_t tc[kC], bxc[kC], byc[kC], bzc[kC];
#pragma unroll
        for (int u = 0; u < kC; ++u) {
            const int32_t B = Bc[u];
            tc[u] = B >= 0 ? bx.t_cnt[B] : 0;
            bxc[u] = B >= 0 ? bx.ax[B] : 0;
            byc[u] = B >= 0 ? bx.ay[B] : 0;
            bzc[u] = B >= 0 ? bx.az[B] : 0;
        }
#pragma unroll
        for (int u = 0; u < kC; ++u) {
            const int32_t B = Bc[u];
            bool fresh = false;
            if (B >= 0 && tc[u] > 0) {
                const int dx = sx - bxc[u], dy = sy - byc[u], dz = sz - bzc[u];
                const bool near = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
                if (!near) {
                    const int slot = m2l_slot(dx, dy, dz);
                    atomicOr(&use[wv][slot >> 5], 1u << (slot & 31));
                    // B's V-list entry for S: candidate slot 8 c + o, c the index of S's parent
                    // among B's parent's colleagues (the mirror of Q's index d among P's), o
                    // S's octant
                    const int o = ((sx & 1) << 2) | ((sy & 1) << 1) | (sz & 1);
                    L.vslot[(size_t)B * kVSlots + (26 - dq[u]) * 8 + o] =
                        ((uint64_t)(uint32_t)gen << 32) | (uint32_t)(r * kNumM2L + slot);
                    fresh = level >= 3 && atomicExch(&L.vt_tag[B], gen) != gen;
                }
            }
            wave_append(fresh, L.vt + li.base[level], &sc->n_vt_lvl[level], B);
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < kUseWords) {
            L.m2l_box_use[(size_t)(li.base[level] + r) * kUseWords + lane] = use[wv][lane];
            if (use[wv][lane])
                atomicOr(&L.m2l_tile_use[(size_t)(li.tbase[level] + r / 64) * kUseWords + lane], use[wv][lane]);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

LevelInfo level_info(const Plan &p)
{
    LevelInfo li{};
    for (int l = 0; l <= p.max_depth; ++l) {
        li.base[l] = (int32_t)p.level_base[l];
        li.cap[l] = (int32_t)p.level_cap[l];
    }
    li.base[p.max_depth + 1] = (int32_t)p.level_base[p.max_depth + 1];
    li.cap[p.max_depth + 1] = 0;
    for (int l = 0; l <= p.max_depth; ++l) li.tbase[l] = p.m2l_tile_base[l];
    li.depth = p.max_depth;
    return li;
}

}  // namespace

void build_tree(Plan &p, hipStream_t s)
{
    LevelInfo li = level_info(p);
    const int32_t nbox = (int32_t)p.box_cap;
    const unsigned g = (unsigned)((nbox + 255) / 256);
    tree_status_kernel<<<g, 256, 0, s>>>(p.box, li, nbox, p.leaf_cap, p.max_depth, p.d_flag, p.n, p.d_sc,
                                         p.lists.m2l_tile_use, p.m2l_tiles * kUseWords);
}

void build_vtargets(Plan &p, hipStream_t s)
{
    LevelInfo li = level_info(p);
    if (p.method == PH_METHOD_FMM && p.max_depth >= 2) {
        int64_t cap = 0;
        for (int l = 2; l <= p.max_depth; ++l) cap += p.level_cap[l];
        vtarget_kernel<<<(unsigned)std::min<int64_t>((cap + 3) / 4, 1024), 256, 0, s>>>(p.box, li, p.d_sc, p.lists);
    }
}

void build_lists(Plan &p, hipStream_t s)
{
    LevelInfo li = level_info(p);
    const int32_t nbox = (int32_t)p.box_cap;
    const unsigned g = (unsigned)((nbox + kLBoxes - 1) / kLBoxes);
    uint32_t grid_levels = 0;
    if (p.grid_mode)
        for (int l = 0; l <= p.max_depth; ++l)
            if (l < 2 || p.grid_m[l] > 0) grid_levels |= 1u << l;
    list_build_kernel<<<g, kListBlock, 0, s>>>(p.box, li, p.d_sc, nbox, p.lists, grid_levels, p.d_sticky);
}

}  // namespace ph
