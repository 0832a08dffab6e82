// Per-call adaptive octree over the selected sources and targets, and its interaction lists.
//
// Sec. 2.4: the octree is refined until every leaf holds at most a
// prescribed number of points; near interactions N(B) are summed exactly and
// far interactions F(B) go through the hierarchy.  Here a box is split while
// max(#selected sources, #selected targets) > leaf capacity.  Since the
// selected lists are sorted by Morton key, every box is a contiguous range of
// each list and a child range is found by binary search on the next key digit.
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

__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t prefix_of(int ax, int ay, int az)
{
    return (spread3((uint32_t)ax) << 2) | (spread3((uint32_t)ay) << 1) | spread3((uint32_t)az);
}

// first index in [lo, hi) with (key >> shift) >= target
__device__ __forceinline__ int32_t lower_bound_prefix(const uint64_t *__restrict__ keys, int32_t lo, int32_t hi,
                                                      int shift, uint64_t target)
{
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if ((keys[mid] >> shift) < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void init_root_kernel(BoxArrays bx, LevelInfo li, CallScalars *sc)
{
    if (threadIdx.x == 0) {
        const int b = li.base[0];
        bx.level[b] = 0;
        bx.ax[b] = bx.ay[b] = bx.az[b] = 0;
        bx.s_first[b] = 0;
        bx.s_cnt[b] = sc->n_src;
        bx.t_first[b] = 0;
        bx.t_cnt[b] = sc->n_tgt;
        bx.parent[b] = -1;
        bx.flags[b] = 0;
        bx.src_rank[b] = sc->n_src > 0 ? 0 : -1;
        bx.src_box[b] = b;
        sc->lvl_count[0] = 1;
        sc->lvl_src[0] = sc->n_src > 0 ? 1 : 0;
        for (int l = 0; l <= li.depth + 1 && l < kMaxDepth + 3; ++l) sc->lvl_start[l] = li.base[l];
    }
    if (threadIdx.x < 27) bx.coll[(size_t)li.base[0] * 27 + threadIdx.x] = (threadIdx.x == 13) ? li.base[0] : -1;
}

__global__ void split_count_kernel(BoxArrays bx, LevelInfo li, int level, int leaf_cap, int may_split,
                                   const CallScalars *__restrict__ sc, const uint64_t *__restrict__ s_key,
                                   const uint64_t *__restrict__ t_key)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= li.cap[level]) return;
    if (i >= sc->lvl_count[level]) {
        bx.child_cnt[i] = 0;
        return;
    }
    const int32_t b = li.base[level] + i;
    const int32_t sf = bx.s_first[b], sn = bx.s_cnt[b], tf = bx.t_first[b], tn = bx.t_cnt[b];
    const bool split = may_split && (max(sn, tn) > leaf_cap);
    bx.flags[b] = split ? 0 : kBoxLeaf;
    if (!split) {
        bx.child_cnt[i] = 0;
        return;
    }
    const int shift = 3 * (kMortonBits - (level + 1));
    const uint64_t pre = prefix_of(bx.ax[b], bx.ay[b], bx.az[b]) << 3;
    int32_t sb[9], tb[9];
    sb[0] = sf;
    sb[8] = sf + sn;
    tb[0] = tf;
    tb[8] = tf + tn;
    for (int o = 1; o < 8; ++o) {
        sb[o] = lower_bound_prefix(s_key, sb[o - 1], sf + sn, shift, pre | (uint64_t)o);
        tb[o] = lower_bound_prefix(t_key, tb[o - 1], tf + tn, shift, pre | (uint64_t)o);
    }
    uint64_t cnt = 0, cnt_s = 0;
    for (int o = 0; o < 8; ++o) {
        int4 r = make_int4(sb[o], sb[o + 1] - sb[o], tb[o], tb[o + 1] - tb[o]);
        bx.child_tmp[(size_t)i * 8 + o] = r;
        cnt += (r.y + r.w) > 0 ? 1u : 0u;
        cnt_s += r.y > 0 ? 1u : 0u;
    }
    bx.child_cnt[i] = cnt | (cnt_s << 32);
}

// child_cnt now holds packed exclusive offsets; lvl_count/lvl_src[level+1] the totals.
__global__ void split_emit_kernel(BoxArrays bx, LevelInfo li, int level, CallScalars *__restrict__ sc)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc->lvl_count[level]) return;
    if (i == 0) {
        const uint64_t v = sc->lvl_pack[level + 1];
        sc->lvl_count[level + 1] = (int32_t)(v & 0xffffffffu);
        sc->lvl_src[level + 1] = (int32_t)(v >> 32);
    }
    const int32_t b = li.base[level] + i;
    int32_t *ch = bx.child + (size_t)b * 8;
    if (bx.flags[b] & kBoxLeaf) {
        for (int o = 0; o < 8; ++o) ch[o] = -1;
        return;
    }
    const uint64_t off = bx.child_cnt[i];
    int32_t c = li.base[level + 1] + (int32_t)(off & 0xffffffffu);
    int32_t rs = (int32_t)(off >> 32);  // next source rank at level + 1
    const int ax = bx.ax[b], ay = bx.ay[b], az = bx.az[b];
    for (int o = 0; o < 8; ++o) {
        int4 r = bx.child_tmp[(size_t)i * 8 + o];
        if (r.y + r.w == 0) {
            ch[o] = -1;
            continue;
        }
        ch[o] = c;
        bx.level[c] = level + 1;
        bx.ax[c] = 2 * ax + ((o >> 2) & 1);
        bx.ay[c] = 2 * ay + ((o >> 1) & 1);
        bx.az[c] = 2 * az + (o & 1);
        bx.s_first[c] = r.x;
        bx.s_cnt[c] = r.y;
        bx.t_first[c] = r.z;
        bx.t_cnt[c] = r.w;
        bx.parent[c] = b;
        bx.flags[c] = 0;
        if (r.y > 0) {
            bx.src_rank[c] = rs;
            bx.src_box[li.base[level + 1] + rs] = c;
            ++rs;
        } else {
            bx.src_rank[c] = -1;
        }
        ++c;
    }
}

__global__ void mark_last_level_kernel(BoxArrays bx, LevelInfo li, int level, const CallScalars *__restrict__ sc)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc->lvl_count[level]) return;
    const int32_t b = li.base[level] + i;
    bx.flags[b] = kBoxLeaf;
    for (int o = 0; o < 8; ++o) bx.child[(size_t)b * 8 + o] = -1;
}

// Colleagues (the 27 same-level boxes around B, B included) from the parent's colleagues.
__global__ void colleagues_kernel(BoxArrays bx, LevelInfo li, int level, const CallScalars *__restrict__ sc)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc->lvl_count[level]) return;
    const int32_t b = li.base[level] + i;
    const int ax = bx.ax[b], ay = bx.ay[b], az = bx.az[b];
    const int32_t p = bx.parent[b];
    const int lim = 1 << level;
    for (int d = 0; d < 27; ++d) {
        const int nx = ax + d / 9 - 1, ny = ay + (d / 3) % 3 - 1, nz = az + d % 3 - 1;
        int32_t res = -1;
        if (nx >= 0 && ny >= 0 && nz >= 0 && nx < lim && ny < lim && nz < lim) {
            const int dpx = (nx >> 1) - (ax >> 1), dpy = (ny >> 1) - (ay >> 1), dpz = (nz >> 1) - (az >> 1);
            const int32_t P = bx.coll[(size_t)p * 27 + (dpx + 1) * 9 + (dpy + 1) * 3 + (dpz + 1)];
            if (P >= 0) res = bx.child[(size_t)P * 8 + (((nx & 1) << 2) | ((ny & 1) << 1) | (nz & 1))];
        }
        bx.coll[(size_t)b * 27 + d] = res;
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
__device__ void enumerate_lists(const BoxArrays &bx, int32_t b, F &&emit)
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
    // coarser leaves around the ancestors
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

__global__ void list_count_kernel(BoxArrays bx, LevelInfo li, const CallScalars *__restrict__ sc, int32_t nbox,
                                  Lists L)
{
    const int32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) L.u_off[nbox] = L.w_off[nbox] = L.x_off[nbox] = 0;  // scanned into the totals
    if (gid >= nbox) return;
    const int32_t b = box_of_thread(li, sc, gid);
    uint32_t nu = 0, nw = 0, nx = 0;
    if (b >= 0)
        enumerate_lists(bx, b, [&](int kind, int32_t) {
            if (kind == kListU) ++nu;
            else if (kind == kListW) ++nw;
            else ++nx;
        });
    L.u_off[gid] = nu;
    L.w_off[gid] = nw;
    L.x_off[gid] = nx;
}

__global__ void list_fill_kernel(BoxArrays bx, LevelInfo li, CallScalars *__restrict__ sc, int32_t nbox, Lists L)
{
    const int32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nbox) return;
    const int32_t b = box_of_thread(li, sc, gid);
    if (b < 0) return;
    uint32_t pu = L.u_off[gid], pw = L.w_off[gid], px = L.x_off[gid];
    bool over = false;
    enumerate_lists(bx, b, [&](int kind, int32_t C) {
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
    init_root_kernel<<<1, 64, 0, s>>>(p.box, li, p.d_sc);
    for (int l = 0; l < p.max_depth; ++l) {
        const int cap = (int)p.level_cap[l];
        const unsigned g = (unsigned)((cap + 255) / 256);
        split_count_kernel<<<g, 256, 0, s>>>(p.box, li, l, p.leaf_cap, 1, p.d_sc, p.d_s_key, p.d_t_key);
        exclusive_scan_u64(p.box.child_cnt, cap, p.d_scan_tmp, &p.d_sc->lvl_pack[l + 1], s);
        split_emit_kernel<<<g, 256, 0, s>>>(p.box, li, l, p.d_sc);
        const unsigned g1 = (unsigned)((p.level_cap[l + 1] + 255) / 256);
        colleagues_kernel<<<g1, 256, 0, s>>>(p.box, li, l + 1, p.d_sc);
    }
    const unsigned g = (unsigned)((p.level_cap[p.max_depth] + 255) / 256);
    mark_last_level_kernel<<<g, 256, 0, s>>>(p.box, li, p.max_depth, p.d_sc);
}

void build_lists(Plan &p, hipStream_t s)
{
    LevelInfo li = level_info(p);
    const int32_t nbox = (int32_t)p.box_cap;
    const unsigned g = (unsigned)((nbox + 255) / 256);
    list_count_kernel<<<g, 256, 0, s>>>(p.box, li, p.d_sc, nbox, p.lists);
    // nbox + 1 entries: the last one (0 before the scan) receives the total
    exclusive_scan_u32(p.lists.u_off, nbox + 1, p.d_scan_tmp, reinterpret_cast<uint32_t *>(&p.d_sc->n_u), s);
    exclusive_scan_u32(p.lists.w_off, nbox + 1, p.d_scan_tmp, reinterpret_cast<uint32_t *>(&p.d_sc->n_w), s);
    exclusive_scan_u32(p.lists.x_off, nbox + 1, p.d_scan_tmp, reinterpret_cast<uint32_t *>(&p.d_sc->n_x), s);
    list_fill_kernel<<<g, 256, 0, s>>>(p.box, li, p.d_sc, nbox, p.lists);
}

}  // namespace ph
