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
//                  on the fly by the translation kernel, not stored.
#include <hip/hip_runtime.h>

#include "ph_internal.h"

namespace ph {

namespace {

struct LevelInfo {
    int32_t base[kMaxDepth + 2];
    int32_t cap[kMaxDepth + 2];
    int32_t depth;  // deepest level
};

// Per-call tree: the plan's tree over all points, pruned to the selected sets.
// Box ranges come from the exclusive scan of the packed (source | target << 32)
// selection indicators at the box's sorted-order range ends.
__device__ __forceinline__ uint64_t scan_at(const uint64_t *__restrict__ scanned, int32_t k, int64_t n,
                                            uint64_t total)
{
    return k < n ? scanned[k] : total;
}

__global__ void tree_status_kernel(BoxArrays bx, LevelInfo li, int32_t nbox, int leaf_cap, int max_depth,
                                   const uint64_t *__restrict__ scanned, int64_t n, CallScalars *__restrict__ sc)
{
    const int32_t f0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t f = f0 < nbox ? f0 : nbox - 1;  // whole waves reach the reduction below
    const bool mine = f0 < nbox;
    const uint64_t total = sc->packed_total;
    if (f == 0) {
        for (int l = 0; l <= li.depth; ++l) sc->lvl_count[l] = li.cap[l];
        for (int l = 0; l <= li.depth + 1; ++l) sc->lvl_start[l] = li.base[l];
        bx.srcflag[nbox] = 0;
    }
    const int32_t st = bx.start[f], en = bx.end[f];
    const uint64_t a = scan_at(scanned, st, n, total), b = scan_at(scanned, en, n, total);
    const int32_t s0 = (int32_t)(a & 0xffffffffu), t0 = (int32_t)(a >> 32);
    const int32_t sn = (int32_t)(b & 0xffffffffu) - s0, tn = (int32_t)(b >> 32) - t0;
    const int32_t par = bx.parent[f];
    bool exists = true;
    if (par >= 0) {
        const uint64_t pa = scan_at(scanned, bx.start[par], n, total), pb = scan_at(scanned, bx.end[par], n, total);
        const int32_t psn = (int32_t)(pb & 0xffffffffu) - (int32_t)(pa & 0xffffffffu);
        const int32_t ptn = (int32_t)(pb >> 32) - (int32_t)(pa >> 32);
        exists = (sn + tn > 0) && (max(psn, ptn) > leaf_cap);
    }
    // split in the plan's tree iff it holds more than leaf_cap points above the depth limit
    const bool split = exists && (en - st > leaf_cap) && (bx.level[f] < max_depth) && (max(sn, tn) > leaf_cap);
    if (mine) {
        bx.s_first[f] = exists ? s0 : 0;
        bx.s_cnt[f] = exists ? sn : 0;
        bx.t_first[f] = exists ? t0 : 0;
        bx.t_cnt[f] = exists ? tn : 0;
        bx.flags[f] = exists ? (kBoxExists | (split ? 0 : kBoxLeaf)) : 0;
        // low word: box with sources; high word: split box with targets (parent of target boxes)
        bx.srcflag[f] = (uint64_t)((exists && sn > 0) ? 1u : 0u) | ((uint64_t)((split && tn > 0) ? 1u : 0u) << 32);
    }
    // lowest level holding a leaf with sources, as max of (depth + 1 - level), one atomic per wave
    int v = (mine && exists && !split && sn > 0) ? (li.depth + 1 - bx.level[f]) : 0;
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0 && v > 0) atomicMax(&sc->min_leafsrc_level, v);
}

// srcflag holds its exclusive scan: per level, the rank of every box with sources and of
// every split box with targets (the parents whose local fields the next level needs)
__global__ void tree_srcrank_kernel(BoxArrays bx, LevelInfo li, int32_t nbox, CallScalars *__restrict__ sc)
{
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nbox) return;
    const int l = bx.level[f];
    const int32_t base = li.base[l];
    const uint64_t here = bx.srcflag[f], next = bx.srcflag[f + 1], first = bx.srcflag[base];
    if (f == base) {
        const uint64_t end = bx.srcflag[li.base[l + 1]];
        sc->lvl_src[l] = (int32_t)((end & 0xffffffffu) - (first & 0xffffffffu));
        sc->lvl_tpar[l] = (int32_t)((end >> 32) - (first >> 32));
    }
    if ((next & 0xffffffffu) != (here & 0xffffffffu)) {
        const int32_t rank = (int32_t)((here & 0xffffffffu) - (first & 0xffffffffu));
        bx.src_rank[f] = rank;
        bx.src_box[base + rank] = f;
    } else {
        bx.src_rank[f] = -1;
    }
    if ((next >> 32) != (here >> 32)) {
        const int32_t rank = (int32_t)((here >> 32) - (first >> 32));
        bx.tpar_rank[f] = rank;
        bx.tpar_box[base + rank] = f;
    } else {
        bx.tpar_rank[f] = -1;
    }
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

template <class F>
__device__ void enumerate_lists(const BoxArrays &bx, int32_t b, int min_leaf_level, F &&emit)
{
    if (bx.t_cnt[b] == 0) return;
    const bool leaf = bx.flags[b] & kBoxLeaf;
    if (leaf) {
        int32_t stack[8 * kMaxDepth];
        for (int d = 0; d < 27; ++d) {
            const int32_t C = bx.coll[(size_t)b * 27 + d];
            if (C < 0 || bx.s_cnt[C] == 0) continue;
            if (bx.flags[C] & kBoxLeaf) {
                emit(kListU, C);
                continue;
            }
            int top = 0;
            for (int o = 0; o < 8; ++o) {
                const int32_t D = bx.child[(size_t)C * 8 + o];
                if (D >= 0) stack[top++] = D;
            }
            while (top > 0) {
                const int32_t D = stack[--top];
                if (bx.s_cnt[D] == 0) continue;
                if (!adjacent(bx, D, b)) emit(kListW, D);
                else if (bx.flags[D] & kBoxLeaf) emit(kListU, D);
                else
                    for (int o = 0; o < 8; ++o) {
                        const int32_t E = bx.child[(size_t)D * 8 + o];
                        if (E >= 0 && top < 8 * kMaxDepth) stack[top++] = E;
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

// Append val to list for the lanes with pred: one atomic per wave, lanes in lane order.
template <class V>
__device__ __forceinline__ void wave_append(bool pred, V *__restrict__ list, int32_t *counter, V val)
{
    const uint64_t m = __ballot(pred);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, leader);
    if (pred) list[base + __popcll(m & ((1ull << lane) - 1ull))] = val;
}

// List lengths per box, and the leaf lists of the target-side kernels.  grid_levels: bit l
// set when leaves of level l take their far field from a grid operator (or have none).
__global__ void list_count_kernel(BoxArrays bx, LevelInfo li, CallScalars *__restrict__ sc, int32_t nbox,
                                  Lists L, uint32_t grid_levels)
{
    const int32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) L.u_off[nbox] = L.w_off[nbox] = L.x_off[nbox] = 0;  // scanned into the totals
    if (gid >= nbox) return;
    const int32_t b = box_of_thread(li, sc, gid);
    uint32_t nu = 0, nw = 0, nx = 0;
    const int mll = li.depth + 1 - sc->min_leafsrc_level;
    if (b >= 0)
        enumerate_lists(bx, b, mll, [&](int kind, int32_t) {
            if (kind == kListU) ++nu;
            else if (kind == kListW) ++nw;
            else ++nx;
        });
    L.u_off[gid] = nu;
    L.w_off[gid] = nw;
    L.x_off[gid] = nx;
    const bool tleaf = b >= 0 && (bx.flags[b] & kBoxLeaf) && bx.t_cnt[b] > 0;
    const int lev = b >= 0 ? bx.level[b] : 0;
    const bool grid_leaf = tleaf && ((grid_levels >> lev) & 1u);
    // grid-operator leaves go to their level's segment (a wave rarely spans two levels)
    uint64_t pending = __ballot(grid_leaf);
    const int4 entry = make_int4(b, b >= 0 ? bx.t_first[b] : 0, b >= 0 ? bx.t_cnt[b] : 0,
                                 (nu > 0 ? 1 : 0) | (nw > 0 ? 2 : 0));
    while (pending) {
        const int l0 = __shfl(lev, __ffsll((long long)pending) - 1);
        const bool mine = grid_leaf && lev == l0;
        wave_append(mine, L.far_a + li.base[l0], &sc->n_far_a_lvl[l0], entry);
        pending &= ~__ballot(mine);
    }
    wave_append(tleaf && !grid_leaf, L.far_b, &sc->n_far_b, b);
    wave_append(tleaf && nu > 0, L.near_leaves, &sc->n_near, b);
}

__global__ void list_fill_kernel(BoxArrays bx, LevelInfo li, CallScalars *__restrict__ sc, int32_t nbox, Lists L)
{
    const int32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nbox) return;
    const int32_t b = box_of_thread(li, sc, gid);
    if (b < 0) return;
    uint32_t pu = L.u_off[gid], pw = L.w_off[gid], px = L.x_off[gid];
    bool over = false;
    const int mll = li.depth + 1 - sc->min_leafsrc_level;
    enumerate_lists(bx, b, mll, [&](int kind, int32_t C) {
        if (kind == kListU) {
            if (pu < (uint32_t)L.u_cap) L.u[pu] = C;
            else over = true;
            ++pu;
        } else if (kind == kListW) {
            if (pw < (uint32_t)L.w_cap) L.w[pw] = C;
            else over = true;
            ++pw;
        } else {
            if (px < (uint32_t)L.x_cap) L.x[px] = C;
            else over = true;
            ++px;
        }
    });
    if (over) atomicOr(&sc->err, 2);
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
    li.depth = p.max_depth;
    return li;
}

}  // namespace

void build_tree(Plan &p, hipStream_t s)
{
    LevelInfo li = level_info(p);
    const int32_t nbox = (int32_t)p.box_cap;
    const unsigned g = (unsigned)((nbox + 255) / 256);
    tree_status_kernel<<<g, 256, 0, s>>>(p.box, li, nbox, p.leaf_cap, p.max_depth, p.d_flag, p.n, p.d_sc);
    exclusive_scan_u64(p.box.srcflag, nbox + 1, p.d_scan_tmp, nullptr, s);
    tree_srcrank_kernel<<<g, 256, 0, s>>>(p.box, li, nbox, p.d_sc);
}

void build_lists(Plan &p, hipStream_t s)
{
    LevelInfo li = level_info(p);
    const int32_t nbox = (int32_t)p.box_cap;
    const unsigned g = (unsigned)((nbox + 255) / 256);
    uint32_t grid_levels = 0;
    if (p.grid_mode)
        for (int l = 0; l <= p.max_depth; ++l)
            if (l < 2 || p.grid_m[l] > 0) grid_levels |= 1u << l;
    list_count_kernel<<<g, 256, 0, s>>>(p.box, li, p.d_sc, nbox, p.lists, grid_levels);
    // nbox + 1 entries: the last one (0 before the scan) receives the total
    exclusive_scan3_u32(p.lists.u_off, reinterpret_cast<uint32_t *>(&p.d_sc->n_u), p.lists.w_off,
                        reinterpret_cast<uint32_t *>(&p.d_sc->n_w), p.lists.x_off,
                        reinterpret_cast<uint32_t *>(&p.d_sc->n_x), nbox + 1, p.d_scan_tmp, s);
    list_fill_kernel<<<g, 256, 0, s>>>(p.box, li, p.d_sc, nbox, p.lists);
}

}  // namespace ph
