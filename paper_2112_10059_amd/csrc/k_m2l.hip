// Translation operators on the matrix cores: M2M (upward), L2L and M2L (downward) as
// stacked-operator GEMMs per level, then a per-box gather in a fixed order.
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

#include <type_traits>

#include "k_fmm_args.h"

namespace ph {

namespace {

constexpr int kTile = 64;     // tile of source boxes (rows of Y) and of stacked rows m
constexpr int kTK = kGemmK;   // K chunk staged in LDS
constexpr int kPad = 4;       // LDS row padding (bank spread)

enum { kModeM2L = 0, kModeL2L = 1, kModeM2M = 2 };

// One level's part of a translation GEMM: the columns are the boxes list[list_base + r0 + n],
// n < min(ccap, count[count_idx] - r0); the operator starts op_off elements in; column n
// goes to row out_row + n of the output.
struct GemmSeg {
    int32_t count_idx, list_base, r0, ccap;
    int64_t op_off, out_row;
    int32_t tile_base;  // M2L: the segment's first tile in the per-tile offset masks
};
struct GemmSegs {
    int n;
    GemmSeg s[kMaxDepth + 1];
};

// Column tile `tile` of the segments taken in order: its segment and first column, or false
__device__ __forceinline__ bool seg_tile(const GemmSegs &sg, const int32_t *__restrict__ count, int32_t tile,
                                         int &si, int32_t &n0, int32_t &ncols)
{
    for (si = 0; si < sg.n; ++si) {
        ncols = max(0, min(sg.s[si].ccap, count[sg.s[si].count_idx] - sg.s[si].r0));
        const int32_t nt = (ncols + kTile - 1) / kTile;
        if (tile < nt) {
            n0 = tile * kTile;
            return true;
        }
        tile -= nt;
    }
    return false;
}

// Whether a source box of the column tile (slots r0 + n0 .. + 63 of its level, r0 + n0 a
// multiple of 64) sends one of the offsets of rows m0 .. m0 + 63 to a target; a tile that
// reaches no target is not computed (the gathers never read those rows).  One mask word per
// offset range, the same for the whole workgroup.
__device__ __forceinline__ bool tile_used(const uint32_t *__restrict__ tuse, const GemmSeg &sg, int32_t n0, int m0,
                                          int M, int nl)
{
    const uint32_t *tu = tuse + (size_t)(sg.tile_base + (sg.r0 + n0) / kTile) * kUseWords;
    const int o_lo = m0 / nl, o_hi = min(M - 1, m0 + kTile - 1) / nl;
    for (int o = o_lo; o <= o_hi; ++o)
        if ((tu[o >> 5] >> (o & 31)) & 1u) return true;
    return false;
}

// The offsets of the row tile at m0 (rows o n_lam + i) that the column's source box sends
// along, as bits from o_lo: its stored mask (slot: the box's index in the source list)
__device__ __forceinline__ uint32_t col_offsets(const uint32_t *__restrict__ buse, int32_t slot, int m0, int M,
                                                int nl)
{
    const uint32_t *bu = buse + (size_t)slot * kUseWords;
    const int o_lo = m0 / nl, o_hi = min(M - 1, m0 + kTile - 1) / nl;
    uint32_t bits = 0;
    for (int o = o_lo; o <= o_hi; ++o) bits |= ((bu[o >> 5] >> (o & 31)) & 1u) << (o - o_lo);
    return bits;
}

// Translation GEMM on the matrix cores, out^T = X^T Op^T with Op (M x kp, row-major) a
// stacked translation operator and X (kp x ncols) the gathered columns, over one or more
// levels (segments) in one launch:
//   X[:, n] = vec of the n-th listed box of the segment, out[n][m] row per box:
//   M2L: phi of the boxes with sources, Op = 316 stacked offsets   -> Y
//   L2L: u of the split boxes with targets, Op = 8 stacked octants -> u of child c
//   M2M: phi of the boxes with sources, Op = 8 stacked octants     -> Z (child c to parent)
// Stage loads of a GEMM tile, all issued before any use (one round trip), into v[u] for the
// tile element e = t + 256 u (row e / KT, column e % KT).  With KT = 64 a wave covers whole
// rows (row ws + 4 u, column = lane), so each row's base address is a scalar and a load costs
// one register for its value.
// Rows m0 + n of a row-major matrix (row length ld), columns k0 + k below kcols.
template <class T, int KT>
__device__ __forceinline__ void load_rows(T (&v)[KT * kTile / 256], const T *__restrict__ A, int ld, int m0,
                                          int M, int kcols, int k0, int ws, int t)
{
    constexpr int kV = KT * kTile / 256;
    const int lane = t & 63;
#pragma unroll
    for (int u = 0; u < kV; ++u) {
        if constexpr (KT == 64) {
            const int gm = m0 + ws + 4 * u;
            const T *row = A + (size_t)(gm < M ? gm : 0) * ld + k0;
            v[u] = (gm < M && k0 + lane < kcols) ? row[lane] : T(0);
        } else {
            const int e = t + 256 * u, gm = m0 + e / KT, gk = k0 + e % KT;
            v[u] = (gm < M && gk < kcols) ? A[(size_t)gm * ld + gk] : T(0);
        }
    }
}
// Rows of the boxes listed in LDS (box < 0: zero row), columns k0 + k below nl.
template <class T, int KT>
__device__ __forceinline__ void load_box_rows(T (&v)[KT * kTile / 256], const T *__restrict__ X, int nl,
                                              const int32_t *boxes, int k0, int ws, int t)
{
    constexpr int kV = KT * kTile / 256;
    static_assert(kV <= 64, "one row per lane of the box read");
    const int lane = t & 63;
    // with KT = 64 lane u reads row u's box, all of them in one LDS access
    const int32_t rb = KT == 64 ? boxes[ws + 4 * (lane % kV)] : -1;
#pragma unroll
    for (int u = 0; u < kV; ++u) {
        if constexpr (KT == 64) {
            const int32_t bx = __builtin_amdgcn_readlane(rb, u);
            const T *row = X + (size_t)(bx >= 0 ? bx : 0) * nl + k0;
            v[u] = (bx >= 0 && k0 + lane < nl) ? row[lane] : T(0);
        } else {
            const int e = t + 256 * u, gk = k0 + e % KT;
            const int32_t bx = boxes[e / KT];
            v[u] = (bx >= 0 && gk < nl) ? X[(size_t)bx * nl + gk] : T(0);
        }
    }
}

template <class T, int MODE>
__global__ __launch_bounds__(256) void tgemm_kernel(const T *__restrict__ Op0, int kp, int M, int nl,
                                                    const T *__restrict__ vec, const int32_t *__restrict__ list,
                                                    const int32_t *__restrict__ count, GemmSegs segs,
                                                    T *__restrict__ out0, const int32_t *__restrict__ child,
                                                    const int32_t *__restrict__ t_cnt,
                                                    unsigned long long *__restrict__ work,
                                                    const uint32_t *__restrict__ use,
                                                    const uint32_t *__restrict__ buse)
{
    // K staged 64 deep for FP32 (one LDS fill when n_lam <= 64), 32 for FP64
    constexpr int KT = sizeof(T) == 4 ? 2 * kTK : kTK;
    // tiles row-major (a row of K per box / per operator row), rows KT + kPad apart: the staging
    // writes (K fastest) and the matrix-core operand reads (16 rows x 4 K per wave) both spread
    // over all 64 LDS banks
    __shared__ T As[kTile][KT + kPad];  // X^T tile
    __shared__ T Bs[kTile][KT + kPad];  // Op tile
    __shared__ int32_t boxes[kTile];
    __shared__ int32_t kid[MODE == kModeL2L ? kTile : 1][8];  // L2L: children of the column boxes
    __shared__ uint32_t cols_used[MODE == kModeM2L ? kTile : 1];  // M2L: offsets each column sends
    const int m0 = blockIdx.x * kTile;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int ws = __builtin_amdgcn_readfirstlane(w);  // the wave index in a scalar register
    const int wn = w >> 1, wm = w & 1;
    using acc_t = typename Mfma<T>::acc_t;
    // blockIdx.y strides over the column tiles of all segments (a bounded grid for any count);
    // when K fits one stage the operator tile stays in LDS while the segment does not change
    const bool resident = kp <= KT;
    int bseg = -1;
    for (int32_t tile = blockIdx.y;; tile += gridDim.y) {
        int si;
        int32_t n0, ncols;
        if (!seg_tile(segs, count, tile, si, n0, ncols)) break;
        const GemmSeg sg = segs.s[si];
        const T *Op = Op0 + sg.op_off;
        T *out = out0 + (size_t)sg.out_row * M;
        if (MODE == kModeM2L && use && !tile_used(use, sg, n0, m0, M, nl)) continue;
        // the operator's first K stage does not depend on the column boxes: its loads go out
        // before the boxes' (into registers, stored to LDS with the boxes' values)
        constexpr int kBV = KT * kTile / 256;
        T breg[kBV];
        const bool load_b0 = !resident || si != bseg;
        if (load_b0) load_rows<T, KT>(breg, Op, kp, m0, M, kp, 0, ws, t);
        __syncthreads();
        if (t < kTile) {
            const bool in = n0 + t < ncols;
            const int32_t slot = sg.list_base + sg.r0 + n0 + t;
            boxes[t] = in ? list[slot] : -1;
            if (MODE == kModeM2L) cols_used[t] = (in && buse) ? col_offsets(buse, slot, m0, M, nl) : ~0u;
        }
        acc_t acc[2][2];
        T own[2][2][4];  // L2L: the children's level-local parts
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
        for (int k0 = 0; k0 < kp; k0 += KT) {
            __syncthreads();
            // every load of the stage goes out before the first LDS store (one round trip)
            constexpr int kKid = kTile * 8 / 256;
            int32_t kreg[MODE == kModeL2L ? kKid : 1];
            if (MODE == kModeL2L && k0 == 0)
#pragma unroll
                for (int u = 0; u < kKid; ++u) {
                    const int e = t + 256 * u;
                    const int32_t bx = boxes[e >> 3];
                    kreg[u] = bx >= 0 ? child[(size_t)bx * 8 + (e & 7)] : -1;
                }
            T areg[kBV];
            load_box_rows<T, KT>(areg, vec, nl, boxes, k0, ws, t);
            if (k0 > 0) load_rows<T, KT>(breg, Op, kp, m0, M, kp, k0, ws, t);
            if (MODE == kModeL2L && k0 == 0)
#pragma unroll
                for (int u = 0; u < kKid; ++u) {
                    const int e = t + 256 * u;
                    kid[e >> 3][e & 7] = kreg[u];
                }
#pragma unroll
            for (int u = 0; u < kBV; ++u) {
                const int e = t + 256 * u;
                As[e / KT][e % KT] = areg[u];
            }
            if (k0 > 0 || load_b0)
#pragma unroll
                for (int u = 0; u < kBV; ++u) {
                    const int e = t + 256 * u;
                    Bs[e / KT][e % KT] = breg[u];
                }
            bseg = si;
            __syncthreads();
            if (MODE == kModeL2L && k0 == 0) {
                // the children's level-local parts (cleared where none), loaded while the products run
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) {
                        const int gm = m0 + wm * 32 + j * 16 + (lane & 15);
                        const int c = gm / nl, li = gm - c * nl;
                        for (int r = 0; r < 4; ++r) {
                            const int nl_ = wn * 32 + i * 16 + Mfma<T>::row(lane, r);
                            const int32_t C = (n0 + nl_ < ncols && gm < M) ? kid[nl_][c] : -1;
                            own[i][j][r] = C >= 0 ? out0[(size_t)C * nl + li] : T(0);
                        }
                    }
            }
#pragma unroll
            for (int ks = 0; ks < KT; ks += 4) {
                const int kk = ks + (lane >> 4);
                T a[2], b[2];
                for (int i = 0; i < 2; ++i) a[i] = As[wn * 32 + i * 16 + (lane & 15)][kk];
                for (int j = 0; j < 2; ++j) b[j] = Bs[wm * 32 + j * 16 + (lane & 15)][kk];
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::mma(a[i], b[j], acc[i][j]);
            }
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                const int gm = m0 + wm * 32 + j * 16 + (lane & 15);
                for (int r = 0; r < 4; ++r) {
                    const int nl_ = wn * 32 + i * 16 + Mfma<T>::row(lane, r);
                    const int gn = n0 + nl_;
                    if (gn >= ncols || gm >= M) continue;
                    if (MODE == kModeL2L) {
                        // row c n_lam + li is the check potential li of child c: into its u, plus
                        // the level-local part already there (zero unless it has a V or X list)
                        const int c = gm / nl, li = gm - c * nl;
                        const int32_t C = kid[nl_][c];
                        if (C < 0) continue;
                        out0[(size_t)C * nl + li] = acc[i][j][r] + own[i][j][r];
                        if (work && li == 0 && t_cnt[C] > 0) atomicAdd(&work[7], 1ull);
                    } else {
                        // only the offsets some target of the box's V lists reads
                        if (MODE == kModeM2L && !((cols_used[nl_] >> (gm / nl - m0 / nl)) & 1u)) continue;
                        out[(size_t)gn * M + gm] = acc[i][j][r];
                    }
                }
            }
    }
}

// M2L products in FP32 when a row tile's K fits one stage (k_pad <= 64): the workgroup keeps
// one 64-row tile of the stacked offset slots and walks the column tiles blockIdx.y,
// blockIdx.y + gridDim.y, ... of all levels.  Their boxes, and the offsets each box sends
// along, are listed in LDS kPipeTiles tiles at a time; then the next used tile's densities
// (and its operator tile, when its level differs) are loaded into registers while the current
// tile's products run and its columns are stored, so that loads, matrix-core work and stores
// of consecutive tiles overlap.
constexpr int kPipeTiles = 8;

__global__ __launch_bounds__(256) void m2l_pipe_kernel(const float *__restrict__ Op0, int kp, int M, int nl,
                                                       const float *__restrict__ phi,
                                                       const int32_t *__restrict__ list,
                                                       const int32_t *__restrict__ count, GemmSegs segs,
                                                       float *__restrict__ out0,
                                                       const uint32_t *__restrict__ use,
                                                       const uint32_t *__restrict__ buse)
{
    constexpr int KT = 64, kV = KT * kTile / 256;
    __shared__ float As[kTile][KT + kPad];  // the current tile's densities, a row per box
    __shared__ float Bs[kTile][KT + kPad];  // the operator tile, a row per offset slot row
    __shared__ int32_t boxes[kPipeTiles][kTile];
    __shared__ uint32_t cols[kPipeTiles][kTile];
    __shared__ int32_t tseg[kPipeTiles], tn0[kPipeTiles], tnc[kPipeTiles];
    const int m0 = blockIdx.x * kTile;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int ws = __builtin_amdgcn_readfirstlane(w);
    const int wn = w >> 1, wm = w & 1;
    for (int32_t tb = blockIdx.y;; tb += kPipeTiles * (int32_t)gridDim.y) {
        __syncthreads();  // the previous batch's lists have been read
        if (t < kPipeTiles) {
            int si;
            int32_t n0, nc;
            const bool ok = seg_tile(segs, count, tb + t * (int32_t)gridDim.y, si, n0, nc);
            // -1: past the last tile, -2: a tile whose offsets no target reads
            tseg[t] = !ok ? -1 : ((use && !tile_used(use, segs.s[si], n0, m0, M, nl)) ? -2 : si);
            tn0[t] = ok ? n0 : 0;
            tnc[t] = ok ? nc : 0;
        }
        __syncthreads();
        if (tseg[0] == -1) return;
        // every listed column's box and offset bits, the loads issued together
        constexpr int kL = kPipeTiles * kTile / 256;
        int32_t bv[kL];
        uint32_t cv[kL];
#pragma unroll
        for (int u = 0; u < kL; ++u) {
            const int e = t + 256 * u, j = e / kTile, c = e % kTile;
            const int si = tseg[j];
            bv[u] = -1;
            cv[u] = 0u;
            if (si >= 0 && tn0[j] + c < tnc[j]) {
                const int32_t slot = segs.s[si].list_base + segs.s[si].r0 + tn0[j] + c;
                bv[u] = list[slot];
                cv[u] = buse ? col_offsets(buse, slot, m0, M, nl) : ~0u;
            }
        }
#pragma unroll
        for (int u = 0; u < kL; ++u) {
            const int e = t + 256 * u;
            boxes[e / kTile][e % kTile] = bv[u];
            cols[e / kTile][e % kTile] = cv[u];
        }
        __syncthreads();
        int j = 0;
        while (j < kPipeTiles && tseg[j] == -2) ++j;
        if (j >= kPipeTiles || tseg[j] < 0) continue;
        float areg[kV], breg[kV];
        load_box_rows<float, KT>(areg, phi, nl, boxes[j], 0, ws, t);
        load_rows<float, KT>(breg, Op0 + segs.s[tseg[j]].op_off, kp, m0, M, kp, 0, ws, t);
        int bseg = -1;  // the segment whose operator tile is in Bs
        while (true) {
            const int sj = tseg[j];
            int jn = j + 1;
            while (jn < kPipeTiles && tseg[jn] == -2) ++jn;
            const bool has_next = jn < kPipeTiles && tseg[jn] >= 0;
#pragma unroll
            for (int u = 0; u < kV; ++u) As[ws + 4 * u][lane] = areg[u];
            if (sj != bseg)
#pragma unroll
                for (int u = 0; u < kV; ++u) Bs[ws + 4 * u][lane] = breg[u];
            __syncthreads();
            bseg = sj;
            // the next tile's loads go out before this tile's products
            if (has_next) {
                load_box_rows<float, KT>(areg, phi, nl, boxes[jn], 0, ws, t);
                if (tseg[jn] != sj) load_rows<float, KT>(breg, Op0 + segs.s[tseg[jn]].op_off, kp, m0, M, kp, 0, ws, t);
            }
            f32x4 acc[2][2];
            for (int i = 0; i < 2; ++i)
                for (int q = 0; q < 2; ++q) acc[i][q] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < KT; ks += 4) {
                const int kk = ks + (lane >> 4);
                float a[2], b[2];
                for (int i = 0; i < 2; ++i) a[i] = As[wn * 32 + i * 16 + (lane & 15)][kk];
                for (int q = 0; q < 2; ++q) b[q] = Bs[wm * 32 + q * 16 + (lane & 15)][kk];
                for (int i = 0; i < 2; ++i)
                    for (int q = 0; q < 2; ++q) acc[i][q] = Mfma<float>::mma(a[i], b[q], acc[i][q]);
            }
            float *out = out0 + (size_t)segs.s[sj].out_row * M;
            const int32_t n0 = tn0[j], nc = tnc[j];
            for (int i = 0; i < 2; ++i)
                for (int q = 0; q < 2; ++q) {
                    const int gm = m0 + wm * 32 + q * 16 + (lane & 15);
                    for (int r = 0; r < 4; ++r) {
                        const int cn = wn * 32 + i * 16 + Mfma<float>::row(lane, r), gn = n0 + cn;
                        if (gn >= nc || gm >= M) continue;
                        // only the offsets some target of the box's V lists reads
                        if (!((cols[j][cn] >> (gm / nl - m0 / nl)) & 1u)) continue;
                        out[(size_t)gn * M + gm] = acc[i][q][r];
                    }
                }
            __syncthreads();  // every wave is done with As and Bs
            if (!has_next) break;
            j = jn;
        }
    }
}

// Check values of the target leaves of levels 3 .. depth in one launch (FP32, n_lam <= 64):
// u_B = w_B + sum over the ancestors A of B at levels 2 .. m - 1 of T(l -> m, pos) w_A, with
// T the composite of the L2L steps from A down to B (the L2L chain unrolled, by linearity) and
// w the level-local parts (V and X lists) the gather stored in u.  Leaves are nobody's
// ancestors, so their u is written in place while the ancestors' w are read.  A workgroup
// takes the 64 boxes of level m whose coordinates are congruent to its class c modulo
// 2^(m-2) (one below each level-2 box); they share every composite, so each ancestor level is
// one 64 x 64 x 64 product on the matrix cores (the next level's loads go out before the
// current product), accumulated in registers.
struct CompArgs {
    const float *ops;
    const int32_t *map;  // boxes by level and coordinates
    int64_t map_off[kCompMaxDepth + 1];
    int64_t off[kCompMaxDepth + 1][kCompMaxDepth + 1];  // levels up to kCompMaxDepth only
    int depth;
};

__global__ __launch_bounds__(256) void l2l_comp_kernel(FmmArgs<float> a, CompArgs ca, int kp)
{
    constexpr int KT = 64, kV = KT * kTile / 256;
    __shared__ float As[kTile][KT + kPad];
    __shared__ float Bs[kTile][KT + kPad];
    __shared__ int32_t anc[kMaxDepth + 2][kTile];  // per ancestor level, each column's ancestor
    __shared__ int32_t leafb[kTile];               // the column's leaf (-1: none)
    __shared__ uint8_t lown[kTile];                // whether the leaf holds a level-local part
    __shared__ int anyv;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int ws = __builtin_amdgcn_readfirstlane(w);
    const int wn = w >> 1, wm = w & 1;
    const int nl = a.n_lam;
    int m = -1, cls = blockIdx.x;
    for (int l = 3; l <= ca.depth; ++l) {
        const int n = 1 << (3 * (l - 2));
        if (cls < n) {
            m = l;
            break;
        }
        cls -= n;
    }
    if (m < 0) return;
    const int sh = m - 2, side = 1 << sh;
    const int cx = cls >> (2 * sh), cy = (cls >> sh) & (side - 1), cz = cls & (side - 1);
    if (t == 0) anyv = 0;
    __syncthreads();
    if (t < kTile) {
        // column t: below the level-2 box (t / 16, t / 4 % 4, t % 4)
        const int X = (t >> 4) * side + cx, Y = ((t >> 2) & 3) * side + cy, Z = (t & 3) * side + cz;
        const int64_t nm = (int64_t)1 << m;
        const int32_t B = ca.map[ca.map_off[m] + ((int64_t)X * nm + Y) * nm + Z];
        // the ancestors' look-ups issued with the box's (they need only its coordinates)
        int32_t an[kCompMaxDepth];
#pragma unroll
        for (int l = 2; l < kCompMaxDepth; ++l) {
            const int lc = min(l, m - 1), s2 = m - lc;
            const int64_t n2 = (int64_t)1 << lc;
            an[l] = ca.map[ca.map_off[lc] + ((int64_t)(X >> s2) * n2 + (Y >> s2)) * n2 + (Z >> s2)];
        }
        // a box of level >= 3 holds a level-local part only if the gather wrote one this call
        // (a V/X target: tagged with the call number); the others count as zero, so their
        // check values need no clearing.  Every box of level 2 is written.
        // (all read unconditionally, box 0 standing in for an absent box: a short-circuit test
        // would make each read a round trip of its own)
        const int gen = a.sc->gen;
        const int32_t Bc = max(B, 0);
        const int32_t fl = a.bx.flags[Bc], tc = a.bx.t_cnt[Bc], tg = a.L.vt_tag[Bc];
        int32_t tga[kCompMaxDepth];
#pragma unroll
        for (int l = 2; l < kCompMaxDepth; ++l) tga[l] = a.L.vt_tag[max(an[l], 0)];
        const bool v = B >= 0 && (fl & kBoxLeaf) && tc > 0;
        const bool vo = B >= 0 && tg == gen;
        bool va[kCompMaxDepth];
#pragma unroll
        for (int l = 2; l < kCompMaxDepth; ++l) va[l] = l == 2 || (an[l] >= 0 && tga[l] == gen);
        leafb[t] = v ? B : -1;
        lown[t] = v && vo;
#pragma unroll
        for (int l = 2; l < kCompMaxDepth; ++l)
            if (l < m) anc[l][t] = (v && va[l]) ? an[l] : -1;
        if (v) anyv = 1;
    }
    __syncthreads();
    if (!anyv) return;
    // the leaves' own level-local parts, for the epilogue
    float own[2][2][4];
    for (int i = 0; i < 2; ++i)
        for (int q = 0; q < 2; ++q) {
            const int gm = wm * 32 + q * 16 + (lane & 15);
            for (int r = 0; r < 4; ++r) {
                const int col = wn * 32 + i * 16 + Mfma<float>::row(lane, r);
                const int32_t B = leafb[col];
                own[i][q][r] = (B >= 0 && lown[col] && gm < nl) ? a.u[(size_t)B * nl + gm] : 0.0f;
            }
        }
    auto op_of = [&](int l) {
        const int s2 = m - l, sd = 1 << s2, msk = sd - 1;
        const int pos = ((cx & msk) * sd + (cy & msk)) * sd + (cz & msk);
        return ca.ops + ca.off[m][l] + (int64_t)pos * nl * kp;
    };
    float areg[kV], breg[kV];
    load_box_rows<float, KT>(areg, a.u, nl, anc[2], 0, ws, t);
    load_rows<float, KT>(breg, op_of(2), kp, 0, nl, kp, 0, ws, t);
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int q = 0; q < 2; ++q) acc[i][q] = f32x4{0, 0, 0, 0};
    for (int l = 2; l < m; ++l) {
#pragma unroll
        for (int u = 0; u < kV; ++u) {
            As[ws + 4 * u][lane] = areg[u];
            Bs[ws + 4 * u][lane] = breg[u];
        }
        __syncthreads();
        if (l + 1 < m) {
            load_box_rows<float, KT>(areg, a.u, nl, anc[l + 1], 0, ws, t);
            load_rows<float, KT>(breg, op_of(l + 1), kp, 0, nl, kp, 0, ws, t);
        }
#pragma unroll
        for (int ks = 0; ks < KT; ks += 4) {
            const int kk = ks + (lane >> 4);
            float av[2], bv[2];
            for (int i = 0; i < 2; ++i) av[i] = As[wn * 32 + i * 16 + (lane & 15)][kk];
            for (int q = 0; q < 2; ++q) bv[q] = Bs[wm * 32 + q * 16 + (lane & 15)][kk];
            for (int i = 0; i < 2; ++i)
                for (int q = 0; q < 2; ++q) acc[i][q] = Mfma<float>::mma(av[i], bv[q], acc[i][q]);
        }
        __syncthreads();  // every wave is done with As and Bs
    }
    for (int i = 0; i < 2; ++i)
        for (int q = 0; q < 2; ++q) {
            const int gm = wm * 32 + q * 16 + (lane & 15);
            for (int r = 0; r < 4; ++r) {
                const int cn = wn * 32 + i * 16 + Mfma<float>::row(lane, r);
                const int32_t B = leafb[cn];
                if (B < 0 || gm >= nl) continue;
                a.u[(size_t)B * nl + gm] = acc[i][q][r] + own[i][q][r];
                if (a.work && gm == 0) atomicAdd(&a.work[7], 1ull);
            }
        }
}

// M2L GEMM of the split-BF16 form (same tiling and output as tgemm_kernel in M2L mode):
// every operand x is taken as hi + lo with hi = bf16(x), lo = bf16(x - hi) (the operator's
// parts precomputed in FP64, the densities split while staged), and
//   Y = Phi^T (Op_hi + Op_lo)^T ~ Phi_hi Op_hi + Phi_hi Op_lo + Phi_lo Op_hi
// runs as three v_mfma_f32_16x16x32_bf16 per 32-deep k step with FP32 accumulation; the
// dropped lo * lo term is below 2^-16 of the product.
// Operand layout of v_mfma_f32_16x16x32_bf16: A lane l holds A[l%16][8 (l/16) + v],
// B lane l holds B[8 (l/16) + v][l%16] (v = 0..7); D as for the FP32 form.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kPadB = 8;  // LDS row padding (bfloat16 elements; rows stay 16-byte aligned)
static_assert(kTK % 32 == 0 && ((kTK + kPadB) * 2) % 16 == 0, "whole 16x16x32 steps, 16-byte aligned LDS rows");

__device__ __forceinline__ uint16_t bf16_rne(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void tgemm_m2l_bf16s_kernel(const uint16_t *__restrict__ Oh0,
                                                              const uint16_t *__restrict__ Ol0, int kp, int M,
                                                              int nl, const float *__restrict__ vec,
                                                              const int32_t *__restrict__ list,
                                                              const int32_t *__restrict__ count, GemmSegs segs,
                                                              float *__restrict__ out0,
                                                              const uint32_t *__restrict__ use,
                                                              const uint32_t *__restrict__ buse)
{
    __shared__ __align__(16) uint16_t Ah[kTile][kTK + kPadB], Al[kTile][kTK + kPadB];
    __shared__ __align__(16) uint16_t Bh[kTile][kTK + kPadB], Bl[kTile][kTK + kPadB];
    __shared__ int32_t boxes[kTile];
    __shared__ uint32_t cols_used[kTile];
    const int m0 = blockIdx.x * kTile;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wn = w >> 1, wm = w & 1;
    for (int32_t tile = blockIdx.y;; tile += gridDim.y) {
        int si;
        int32_t n0, ncols;
        if (!seg_tile(segs, count, tile, si, n0, ncols)) break;
        const GemmSeg sg = segs.s[si];
        const uint16_t *Oh = Oh0 + sg.op_off, *Ol = Ol0 + sg.op_off;
        float *out = out0 + (size_t)sg.out_row * M;
        if (use && !tile_used(use, sg, n0, m0, M, nl)) continue;
        __syncthreads();
        if (t < kTile) {
            const bool in = n0 + t < ncols;
            const int32_t slot = sg.list_base + sg.r0 + n0 + t;
            boxes[t] = in ? list[slot] : -1;
            cols_used[t] = (in && buse) ? col_offsets(buse, slot, m0, M, nl) : ~0u;
        }
        f32x4 acc[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
        for (int k0 = 0; k0 < kp; k0 += kTK) {
            __syncthreads();
            for (int e = t; e < kTK * kTile; e += 256) {
                const int n = e / kTK, k = e % kTK;
                const int gk = k0 + k;
                const int32_t bx = boxes[n];
                const float v = (bx >= 0 && gk < nl) ? vec[(size_t)bx * nl + gk] : 0.0f;
                const uint16_t h = bf16_rne(v);
                Ah[n][k] = h;
                Al[n][k] = bf16_rne(v - __uint_as_float((unsigned)h << 16));
                const int gm = m0 + n;
                Bh[n][k] = gm < M ? Oh[(size_t)gm * kp + gk] : (uint16_t)0;
                Bl[n][k] = gm < M ? Ol[(size_t)gm * kp + gk] : (uint16_t)0;
            }
            __syncthreads();
            // v_mfma_f32_16x16x32_bf16: lane l holds row l % 16, k = 8 (l / 16) .. + 7 of A and
            // the same of B (column l % 16); three products per step (hi hi, hi lo, lo hi)
#pragma unroll
            for (int ks = 0; ks < kTK; ks += 32) {
                const int kk = ks + 8 * (lane >> 4);
                bf16x8 ah[2], al[2], bh[2], bl[2];
                for (int i = 0; i < 2; ++i) {
                    const int n = wn * 32 + i * 16 + (lane & 15);
                    ah[i] = *reinterpret_cast<const bf16x8 *>(&Ah[n][kk]);
                    al[i] = *reinterpret_cast<const bf16x8 *>(&Al[n][kk]);
                }
                for (int j = 0; j < 2; ++j) {
                    const int m = wm * 32 + j * 16 + (lane & 15);
                    bh[j] = *reinterpret_cast<const bf16x8 *>(&Bh[m][kk]);
                    bl[j] = *reinterpret_cast<const bf16x8 *>(&Bl[m][kk]);
                }
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    }
            }
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                const int gm = m0 + wm * 32 + j * 16 + (lane & 15);
                for (int r = 0; r < 4; ++r) {
                    const int nl_ = wn * 32 + i * 16 + 4 * (lane >> 4) + r, gn = n0 + nl_;
                    if (gn >= ncols || gm >= M) continue;
                    if (!((cols_used[nl_] >> (gm / nl - m0 / nl)) & 1u)) continue;
                    out[(size_t)gn * M + gm] = acc[i][j][r];
                }
            }
    }
}

// The level-local part of the check values, one wave (a workgroup of 64) per target box B:
//   w_B = base + [first chunk: X-list sources of B] + sum over V(B) in this chunk of Y,
// base = 0 in the first chunk, else the earlier chunks' sum; w_B is stored in u_B, and the L2L
// product of the next level adds the parent's expansion to it.  V(B) = children of the
// parent's colleagues not adjacent to B: the V-target pass stored each pair's translation code
// at B's candidate slot 8 c + o (216 slots, tagged with the call's number), so the wave reads
// the slots in 64-slot slices (lane = slot), compacts a slice's translations in candidate order
// and reads them kB at a time (loads in flight together), added in candidate order.  A box's
// work is a chain of dependent loads, so a wave per box keeps many boxes in flight.
// The boxes: every box of level 2 and the listed boxes (V or X list) of the deeper levels in
// gl.lo .. gl.hi, dealt to the workgroups as one flat range.
struct GatherLevels {
    int lo, hi;                      // levels
    int64_t y_row[kMaxDepth + 2];    // first row of each level's products in Y
};

template <class T, int NK>
__global__ __launch_bounds__(64) void down_gather_kernel(FmmArgs<T> a, GatherLevels gl, const T *__restrict__ Y0,
                                                         int M, int32_t r0, int32_t ccap, int init, int with_x)
{
    __shared__ int32_t cds[kVSlots];  // the box's translations, in candidate order
    const int lane = threadIdx.x & 63;
    const int nl = a.n_lam;
    const int gen = a.sc->gen;  // this call's tag of the V-list slots
    constexpr int nk = NK;  // lattice values per lane: n_lam <= 64 NK
    static_assert(kMaxDepth + 2 <= 64, "a lane per level");
    // the call's per-level counts, lane l holding level l's (read once, picked by readlane)
    const int32_t cnt_l = (lane >= gl.lo && lane <= gl.hi)
                              ? (lane == 2 ? a.sc->lvl_count[2] : a.sc->n_vt_lvl[lane]) : 0;
    const int32_t src_l = lane < kMaxDepth + 2 ? a.sc->lvl_src[lane] : 0;
    for (int32_t idx = blockIdx.x;; idx += gridDim.x) {
        int level = -1;
        int32_t i = idx;
        for (int l = gl.lo; l <= gl.hi; ++l) {
            const int32_t c = __builtin_amdgcn_readlane(cnt_l, l);
            if (i < c) {
                level = l;
                break;
            }
            i -= c;
        }
        if (level < 0) break;
        const int32_t ncols = min(ccap, __builtin_amdgcn_readlane(src_l, level) - r0);
        if (!with_x && ncols <= 0) continue;  // nothing of this level in the chunk
        const int32_t b = level == 2 ? a.lt.base[2] + i : a.L.vt[a.lt.base[level] + i];
        // the box's target count, X range and V-list slots (the children of the parent's
        // colleagues, in candidate order, filled by this call's V-target pass), loaded together
        // (no branch on them before their use: a box without targets only writes nothing)
        const int32_t tcnt = a.bx.t_cnt[b];
        const uint2 xrng = a.L.x_rng[b];
        const uint64_t *__restrict__ vs = a.L.vslot + (size_t)b * kVSlots;
        uint64_t ve[(kVSlots + 63) / 64];
#pragma unroll
        for (int q = 0; q < (kVSlots + 63) / 64; ++q) ve[q] = vs[min(64 * q + lane, kVSlots - 1)];
        const bool live = tcnt != 0;
#pragma unroll
        for (int q = 0; q < (kVSlots + 63) / 64; ++q)
            if (64 * q + lane >= kVSlots || !live) ve[q] = 0ull;
        const uint2 xr = (with_x && live) ? xrng : make_uint2(0u, 0u);
        int64_t yrow = 0;  // constant indices only (no private copy of the argument block)
#pragma unroll
        for (int l = 0; l < kMaxDepth + 2; ++l)
            if (l == level) yrow = gl.y_row[l];
        const T *__restrict__ Y = Y0 + (size_t)yrow * M;
        T acc[NK];
        for (int k = 0; k < NK; ++k) acc[k] = T(0);
        unsigned long long n_m2l = 0, n_p2l = 0;
        if (with_x) {
            // X list: sources of coarser leaves straight onto the check points
            const uint32_t x0 = xr.x, x1 = xr.y;
            if (x1 > x0) {
                const double hw = a.lt.hw[level];
                T cx, cy, cz;
                box_centre(a, b, hw, cx, cy, cz);
                const T h = (T)hw;
                for (uint32_t e = x0; e < x1; ++e) {
                    const int32_t C = a.L.x[e];
                    const int32_t sf = a.bx.s_first[C], sn = a.bx.s_cnt[C];
                    n_p2l += (unsigned long long)sn * nl;
                    for (int j = 0; j < sn; ++j) {
                        const V4<T> y = a.s_dat[sf + j];
#pragma unroll
                        for (int k = 0; k < NK; ++k) {
                            const int li = lane + 64 * k;
                            if (k >= nk || li >= nl) break;
                            const T ddx = cx + h * a.lat[3 * li] - y.x, ddy = cy + h * a.lat[3 * li + 1] - y.y,
                                    ddz = cz + h * a.lat[3 * li + 2] - y.z;
                            acc[k] += kernel_eval<true>(ddx * ddx + ddy * ddy + ddz * ddz, a.kp) * y.w;
                        }
                    }
                }
            }
        }
        // V list: the box's candidate slots, read above in one sweep
        const uint64_t below = (1ull << lane) - 1ull;
        // the box's translations compacted in candidate order (all slices first, so that the
        // reads below run across slice boundaries), then read kB at a time (loads issued
        // together, added in order)
        int n = 0;
#pragma unroll
        for (int q = 0; q < (kVSlots + 63) / 64; ++q) {
            int32_t code = -1;  // rank * 316 + slot, chunk-relative
            if ((uint32_t)(ve[q] >> 32) == (uint32_t)gen) {
                const int32_t full = (int32_t)(uint32_t)ve[q];
                const int32_t rk = full / kNumM2L - r0;
                if (rk >= 0 && rk < ncols) code = rk * kNumM2L + full % kNumM2L;
            }
            const uint64_t mask = __ballot(code >= 0);
            if (code >= 0) cds[n + __popcll(mask & below)] = code;
            n += __popcll(mask);
        }
        n_m2l += n;
        wave_lds_sync();
        constexpr int kB = sizeof(T) == 4 ? 32 : 8;
        for (int u0 = 0; u0 < n; u0 += kB) {
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                if (k >= nk) break;
                const int li = lane + 64 * k;
                T v[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int32_t c = u0 + u < n ? cds[u0 + u] : 0;
                    v[u] = (u0 + u < n && li < nl)
                               ? Y[(size_t)(c / kNumM2L) * M + (size_t)(c % kNumM2L) * nl + li]
                               : T(0);
                }
#pragma unroll
                for (int u = 0; u < kB; ++u)
                    if (u0 + u < n && li < nl) acc[k] += v[u];
            }
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int li = lane + 64 * k;
            if (live && k < nk && li < nl) {
                const size_t o = (size_t)b * nl + li;
                a.u[o] = init ? acc[k] : a.u[o] + acc[k];
            }
        }
        wave_lds_sync();  // qs and cds are free for the next box
        if (a.work && lane == 0) {
            if (n_m2l) atomicAdd(&a.work[5], n_m2l);
            if (n_p2l) atomicAdd(&a.work[4], n_p2l);
        }
    }
}

template <class T>
void launch_gather(Plan &p, const FmmArgs<T> &a, unsigned grid, const GatherLevels &gl, int M, int32_t r0,
                   int32_t ccap, int init, int with_x, hipStream_t s)
{
    const T *Y = (const T *)p.d_y;
    switch ((p.n_lam + 63) / 64) {
    case 1: down_gather_kernel<T, 1><<<grid, 64, 0, s>>>(a, gl, Y, M, r0, ccap, init, with_x); break;
    case 2: down_gather_kernel<T, 2><<<grid, 64, 0, s>>>(a, gl, Y, M, r0, ccap, init, with_x); break;
    case 3:
    case 4: down_gather_kernel<T, 4><<<grid, 64, 0, s>>>(a, gl, Y, M, r0, ccap, init, with_x); break;
    default: down_gather_kernel<T, 8><<<grid, 64, 0, s>>>(a, gl, Y, M, r0, ccap, init, with_x); break;
    }
}

GemmSegs one_seg(int32_t count_idx, int64_t list_base, int64_t r0, int64_t ccap, int64_t op_off, int64_t out_row,
                 int32_t tile_base = 0)
{
    GemmSegs sg{};
    sg.n = 1;
    sg.s[0] = GemmSeg{count_idx, (int32_t)list_base, (int32_t)r0, (int32_t)ccap, op_off, out_row, tile_base};
    return sg;
}

// Y = M2L products of the segments' source boxes (FP32 / FP64 operator, or its split-BF16 form)
template <class T>
void m2l_product(Plan &p, const GemmSegs &sg, int64_t col_tiles, hipStream_t s)
{
    const int nl = p.n_lam, M = kNumM2L * nl;
    // a bounded grid striding over the column tiles (an empty segment costs little)
    dim3 g((M + kTile - 1) / kTile, (unsigned)std::max<int64_t>(1, std::min<int64_t>(16, col_tiles)));
    if (std::is_same<T, float>::value && p.precision == PH_FP32_BF16SPLIT)
        tgemm_m2l_bf16s_kernel<<<g, 256, 0, s>>>((const uint16_t *)p.ops.m2l_hi, (const uint16_t *)p.ops.m2l_lo,
                                                 p.k_pad, M, nl, (const float *)p.d_phi, p.box.src_box,
                                                 p.d_sc->lvl_src, sg, (float *)p.d_y, p.lists.m2l_tile_use,
                                                 p.lists.m2l_box_use);
    else if (std::is_same<T, float>::value && p.k_pad <= 64) {
        // two workgroups per row tile, each walking every second column tile
        dim3 gp((M + kTile - 1) / kTile, (unsigned)std::max<int64_t>(1, std::min<int64_t>(2, col_tiles)));
        m2l_pipe_kernel<<<gp, 256, 0, s>>>((const float *)p.ops.m2l, p.k_pad, M, nl, (const float *)p.d_phi,
                                           p.box.src_box, p.d_sc->lvl_src, sg, (float *)p.d_y,
                                           p.lists.m2l_tile_use, p.lists.m2l_box_use);
    } else
        tgemm_kernel<T, kModeM2L><<<g, 256, 0, s>>>((const T *)p.ops.m2l, p.k_pad, M, nl, (const T *)p.d_phi,
                                                    p.box.src_box, p.d_sc->lvl_src, sg, (T *)p.d_y, nullptr,
                                                    nullptr, nullptr, p.lists.m2l_tile_use, p.lists.m2l_box_use);
}

template <class T>
void fmm_downward_t(Plan &p, hipStream_t s, hipEvent_t m2l_ready, hipEvent_t side_ready, hipEvent_t m2l_begin,
                    hipEvent_t m2l_end)
{
    FmmArgs<T> a = make_args<T>(p);
    const int nl = p.n_lam;
    const int M = kNumM2L * nl;
    const int D = p.max_depth;
    // the levels' M2L products in one launch (they depend on the upward pass and on the offset
    // masks only); the deepest level's were launched on another stream when every level has
    // its products (m2l_ready then follows them there, else the offset masks and V/X targets)
    const bool deep = p.y_all_levels && D >= 2;
    const int top = deep ? D - 1 : D;
    PH_HIP(hipStreamWaitEvent(s, m2l_ready, 0));
    if (p.y_all_levels && top >= 2) {
        GemmSegs sg{};
        int64_t tiles = 0;
        for (int l = 2; l <= top; ++l) {
            sg.s[sg.n++] = GemmSeg{l,           (int32_t)p.level_base[l], 0, (int32_t)p.level_cap[l],
                                   (int64_t)l * M * p.k_pad, p.y_lvl_col[l], p.m2l_tile_base[l]};
            tiles += (p.level_cap[l] + kTile - 1) / kTile;
        }
        if (m2l_begin) PH_HIP(hipEventRecord(m2l_begin, s));
        m2l_product<T>(p, sg, tiles, s);
        if (m2l_end) PH_HIP(hipEventRecord(m2l_end, s));
    } else if (m2l_begin) {
        PH_HIP(hipEventRecord(m2l_begin, s));
        PH_HIP(hipEventRecord(m2l_end, s));
    }
    PH_HIP(hipStreamWaitEvent(s, side_ready, 0));  // the gathers read the X lists (built before it)
    // level-local parts (V and X lists) of every level: no dependence between levels
    int64_t gcap = 0;
    for (int l = 2; l <= D; ++l) gcap += p.level_cap[l];
    // one wave per box: 8192 single-wave workgroups fill every wave slot of the chip
    const unsigned gg = (unsigned)std::max<int64_t>(1, std::min<int64_t>(gcap, 8192));
    if (p.y_all_levels) {
        GatherLevels gl{};
        gl.lo = 2;
        gl.hi = D;
        for (int l = 2; l <= D; ++l) gl.y_row[l] = p.y_lvl_col[l];
        if (D >= 2) launch_gather<T>(p, a, gg, gl, M, 0, INT32_MAX, 1, 1, s);
    } else {
        for (int l = 2; l <= D; ++l) {
            GatherLevels gl{};
            gl.lo = gl.hi = l;
            const int64_t cap = p.level_cap[l];
            const int64_t ccap = std::min<int64_t>((int64_t)p.y_cap_cols, cap);
            const int nchunk = (int)((cap + ccap - 1) / ccap);
            const unsigned gl_grid = (unsigned)std::min<int64_t>(cap, 8192);
            for (int c = 0; c < nchunk; ++c) {
                const int64_t r0 = c * ccap;
                m2l_product<T>(p, one_seg(l, p.level_base[l], r0, ccap, (int64_t)l * M * p.k_pad, 0, p.m2l_tile_base[l]),
                               (ccap + kTile - 1) / kTile, s);
                launch_gather<T>(p, a, gl_grid, gl, M, (int32_t)r0, (int32_t)ccap, c == 0, c == 0, s);
            }
        }
    }
    if (std::is_same<T, float>::value && p.l2l_comp) {
        // every target leaf of levels >= 3 from its ancestors' level-local parts in one launch
        CompArgs ca{};
        ca.ops = (const float *)p.ops.l2l_comp;
        ca.map = p.d_boxmap;
        if (D > kCompMaxDepth) throw Error{PH_EINVAL, "composite translations built for a deeper tree"};
        for (int l = 0; l <= kCompMaxDepth; ++l) {
            ca.map_off[l] = p.boxmap_off[l];
            for (int k = 0; k <= kCompMaxDepth; ++k) ca.off[l][k] = p.comp_off[l][k];
        }
        ca.depth = D;
        int64_t classes = 0;
        for (int l = 3; l <= D; ++l) classes += (int64_t)1 << (3 * (l - 2));
        if (classes > 0)
            l2l_comp_kernel<<<(unsigned)classes, 256, 0, s>>>(*reinterpret_cast<FmmArgs<float> *>(&a), ca, p.k_pad);
        return;
    }
    // u of every child of the split boxes with targets at level l - 1 = L2L_all (8 n_lam x n_lam)
    // applied to the parent's u, plus the child's level-local part
    for (int l = 3; l <= D; ++l) {
        const int Mz = 8 * nl;
        const int64_t pcap = p.level_cap[l - 1];
        dim3 gz((Mz + kTile - 1) / kTile, (unsigned)std::min<int64_t>(1024, (pcap + kTile - 1) / kTile));
        tgemm_kernel<T, kModeL2L><<<gz, 256, 0, s>>>(
            (const T *)p.ops.l2l, p.k_pad, Mz, nl, (const T *)p.d_u, p.box.tpar_box, p.d_sc->lvl_tpar,
            one_seg(l - 1, p.level_base[l - 1], 0, pcap, (int64_t)l * Mz * p.k_pad, 0), (T *)p.d_u, p.box.child,
            p.box.t_cnt, a.work, nullptr, nullptr);
    }
}

// phi_P = sum over children c with sources of W[child c][c n_lam + i], in octant order
template <class T>
__global__ void m2m_gather_kernel(FmmArgs<T> a, int level, const T *__restrict__ W)
{
    const int nl = a.n_lam;
    for (int32_t rk = blockIdx.x; rk < a.sc->lvl_src[level]; rk += gridDim.x) {
        const int32_t P = a.bx.src_box[a.lt.base[level] + rk];
        if (a.bx.flags[P] & kBoxLeaf) continue;
        T acc[4] = {0, 0, 0, 0};
        unsigned long long nc = 0;
        for (int o = 0; o < 8; ++o) {
            const int32_t C = a.bx.child[(size_t)P * 8 + o];
            if (C < 0 || a.bx.src_rank[C] < 0) continue;
            ++nc;
            const T *w = W + ((size_t)a.bx.src_rank[C] * 8 + o) * nl;
            for (int k = 0; k < 4; ++k) {
                const int li = threadIdx.x + k * blockDim.x;
                if (li < nl) acc[k] += w[li];
            }
        }
        for (int k = 0; k < 4; ++k) {
            const int li = threadIdx.x + k * blockDim.x;
            if (li < nl) a.phi[(size_t)P * nl + li] = acc[k];
        }
        if (a.work && threadIdx.x == 0) atomicAdd(&a.work[6], nc);
    }
}

template <class T>
void m2m_level_t(Plan &p, int l, hipStream_t s)
{
    // W = M2M_all (8 n_lam x n_lam) applied to every box with sources at level l + 1,
    // then each non-leaf box with sources at level l sums its children's columns
    FmmArgs<T> a = make_args<T>(p);
    const int nl = p.n_lam;
    const int Mw = 8 * nl;
    const int64_t ccap = p.level_cap[l + 1];
    dim3 g((Mw + kTile - 1) / kTile, (unsigned)std::min<int64_t>(1024, (ccap + kTile - 1) / kTile));
    tgemm_kernel<T, kModeM2M><<<g, 256, 0, s>>>(
        (const T *)p.ops.m2m, p.k_pad, Mw, nl, (const T *)p.d_phi, p.box.src_box, p.d_sc->lvl_src,
        one_seg(l + 1, p.level_base[l + 1], 0, ccap, (int64_t)(l + 1) * Mw * p.k_pad, 0), (T *)p.d_z, nullptr,
        nullptr, nullptr, nullptr, nullptr);
    const int threads = nl <= 64 ? 64 : (nl <= 128 ? 128 : 256);
    m2m_gather_kernel<T><<<(unsigned)std::min<int64_t>(p.level_cap[l], 8192), threads, 0, s>>>(a, l,
                                                                                              (const T *)p.d_z);
}

}  // namespace

bool fmm_m2l_deepest(Plan &p, hipStream_t s)
{
    const int D = p.max_depth;
    if (!p.y_all_levels || D < 2) return false;
    const int M = kNumM2L * p.n_lam;
    GemmSegs sg{};
    sg.s[sg.n++] = GemmSeg{D,           (int32_t)p.level_base[D], 0, (int32_t)p.level_cap[D],
                           (int64_t)D * M * p.k_pad, p.y_lvl_col[D], p.m2l_tile_base[D]};
    const int64_t tiles = (p.level_cap[D] + kTile - 1) / kTile;
    if (p.precision == PH_FP64) m2l_product<double>(p, sg, tiles, s);
    else m2l_product<float>(p, sg, tiles, s);
    return true;
}

void fmm_downward(Plan &p, hipStream_t s, hipEvent_t m2l_ready, hipEvent_t side_ready, hipEvent_t m2l_begin,
                  hipEvent_t m2l_end)
{
    if (p.precision == PH_FP64) fmm_downward_t<double>(p, s, m2l_ready, side_ready, m2l_begin, m2l_end);
    else fmm_downward_t<float>(p, s, m2l_ready, side_ready, m2l_begin, m2l_end);
}

void fmm_m2m_level(Plan &p, int l, hipStream_t s)
{
    if (p.precision == PH_FP64) m2m_level_t<double>(p, l, s);
    else m2m_level_t<float>(p, l, s);
}

}  // namespace ph
