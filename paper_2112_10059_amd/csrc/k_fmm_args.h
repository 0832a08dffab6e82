// Argument block shared by the FMM kernels (upward pass, translations, leaf evaluation).
#pragma once

#include "k_common.h"

namespace ph {

template <class T>
using V4 = typename Vec4T<T>::type;

template <class T>
struct FmmArgs {
    BoxArrays bx;
    Lists L;
    LevelTable lt;
    KParams<T> kp;
    const CallScalars *sc;
    const V4<T> *s_dat;
    const V4<T> *t_dat;
    const int32_t *t_out;  // caller index of each selected target
    const int32_t *perm;
    const T *uc2e_rm;   // levels x n_lam x n_sig
    const T *uc2e_cm;   // levels x n_sig x n_lam
    const T *m2m;       // levels x 8 x n_lam^2 (column-major)
    const T *l2l;
    const T *m2l;       // levels x (316 n_lam) x k_pad (row-major GEMM operand)
    const T *lat;       // n_lam x 3
    const T *shell;     // n_sig x 3
    T *phi;
    T *u;
    unsigned long long *work;
    // uniform-grid lattice operators (grid_g [lambda][r], grid_gt [r][lambda] per level)
    const T *grid_g;
    const T *grid_gt;
    const int32_t *s_cell;
    const int32_t *t_cell;
    // targets are read in place: the points of a target leaf in sorted order, flagged by sel
    // (bit 0 source, bit 1 target), with their plan-time cells and coordinates
    const uint8_t *sel;
    const int32_t *pcell;   // sorted packed cells (uniform grids), else null
    const float4 *xyzf;     // FP32 plans: sorted coordinates
    const double *xyzd;     // sorted coordinates (n x 3)
    const T *I;             // source intensities in caller order (own-cell term)
    double c_self;
    // near-field kernel table (uniform grids, FP32): entries at the cell offsets of adjacent
    // leaves of level near_level, offsets within [-near_R, near_R] per axis; null if absent
    const float *near_tab;
    int near_R, near_level, near_sx, near_sy, near_sz, near_n;
    int grid_m[kMaxDepth + 2];
    int64_t grid_off[kMaxDepth + 2];
    int n_lam, n_sig;
    int k_pad;  // padded row length of the stacked translation operators
    double lo0, lo1, lo2;
    double P;
    // third strategy of Sec. 3 (0 = off): the W list of a target leaf is left out at a target
    // where its bound is below r_s times the rest of S there; rs_flag (per sorted point) records
    // the targets of leaves with a W list at which that happened
    double r_s;
    uint8_t *rs_flag;
    const double *rs_bound;  // per box: the bound of its W list (leaves with one)
    KParams<double> kp64;    // the kernel in FP64, for the bound
};

template <class T>
__device__ __forceinline__ void box_centre(const FmmArgs<T> &a, int32_t b, double hw, T &cx, T &cy, T &cz)
{
    cx = (T)(a.lo0 + (2.0 * a.bx.ax[b] + 1.0) * hw);
    cy = (T)(a.lo1 + (2.0 * a.bx.ay[b] + 1.0) * hw);
    cz = (T)(a.lo2 + (2.0 * a.bx.az[b] + 1.0) * hw);
}

// cell index of a grid point inside its level-l box of m^3 cells
template <class T>
__device__ __forceinline__ int local_cell(const FmmArgs<T> &a, int32_t cell, int32_t b, int m)
{
    const int i = (cell & 1023) - a.bx.ax[b] * m;
    const int j = ((cell >> 10) & 1023) - a.bx.ay[b] * m;
    const int k = ((cell >> 20) & 1023) - a.bx.az[b] * m;
    return (i * m + j) * m + k;
}

// arr[level] with constant indices only (a dynamic index into the kernel's argument block makes
// the compiler copy the block to scratch)
template <class A>
__device__ __forceinline__ A level_pick(const A (&arr)[kMaxDepth + 2], int level)
{
    A v{};
#pragma unroll
    for (int l = 0; l < kMaxDepth + 2; ++l)
        if (l == level) v = arr[l];
    return v;
}

// coordinates of sorted point k in the working precision
template <class T>
__device__ __forceinline__ V4<T> point_xyz(const FmmArgs<T> &a, int64_t k)
{
    V4<T> x;
    if constexpr (sizeof(T) == 4) {
        x = a.xyzf[k];
    } else {
        x.x = a.xyzd[3 * k];
        x.y = a.xyzd[3 * k + 1];
        x.z = a.xyzd[3 * k + 2];
    }
    x.w = T(0);
    return x;
}

// own-cell term of a target that is also a source (Sec. 2.4): c_self I 2^-e, rounded to the
// working precision as the source's other terms are; o is the point's caller index
template <class T>
__device__ __forceinline__ double own_term(const FmmArgs<T> &a, uint8_t sel, int32_t o, int scale_exp)
{
    if (!(sel & 1u)) return 0.0;
    return (double)(T)(a.c_self * ldexp((double)a.I[o], -scale_exp));
}

template <class T>
inline FmmArgs<T> make_args(Plan &p)
{
    FmmArgs<T> a;
    a.bx = p.box;
    a.L = p.lists;
    a.lt = make_level_table(p);
    a.kp = make_kparams<T>(p.gas);
    a.sc = p.d_sc;
    a.s_dat = (const V4<T> *)p.d_s_dat;
    a.t_dat = (const V4<T> *)p.d_t_dat;
    a.t_out = p.d_t_out;
    a.perm = p.d_perm;
    a.uc2e_rm = (const T *)p.ops.uc2e_rm;
    a.uc2e_cm = (const T *)p.ops.uc2e_cm;
    a.m2m = (const T *)p.ops.m2m;
    a.l2l = (const T *)p.ops.l2l;
    a.m2l = (const T *)p.ops.m2l;
    a.lat = (const T *)p.ops.lat_unit;
    a.shell = (const T *)p.ops.shell_unit;
    a.phi = (T *)p.d_phi;
    a.u = (T *)p.d_u;
    a.work = p.count_work ? p.d_sc->work : nullptr;
    a.grid_g = (const T *)p.ops.grid_g;
    a.grid_gt = (const T *)p.ops.grid_gt;
    a.s_cell = p.d_s_cell;
    a.t_cell = p.d_t_cell;
    a.sel = p.d_sel;
    a.pcell = p.grid_mode ? p.d_cell : nullptr;
    a.xyzf = p.d_xyzf;
    a.xyzd = p.d_xyz;
    a.I = (const T *)p.cur_I;
    a.c_self = p.c_self;
    a.near_tab = (const float *)p.ops.near_tab;
    a.near_R = p.ops.near_R;
    a.near_level = p.ops.near_level;
    a.near_sx = p.ops.near_sx;
    a.near_sy = p.ops.near_sy;
    a.near_sz = p.ops.near_sz;
    a.near_n = p.ops.near_n;
    for (int l = 0; l < kMaxDepth + 2; ++l) {
        a.grid_m[l] = p.grid_mode ? p.grid_m[l] : 0;
        a.grid_off[l] = p.grid_off[l];
    }
    a.n_lam = p.n_lam;
    a.n_sig = p.n_sig;
    a.k_pad = p.k_pad;
    a.lo0 = p.cube_lo[0];
    a.lo1 = p.cube_lo[1];
    a.lo2 = p.cube_lo[2];
    a.P = p.gas.P;
    a.r_s = p.thr.r_s;
    a.rs_flag = p.d_rs_flag;
    a.rs_bound = p.d_rs_bound;
    a.kp64 = make_kparams<double>(p.gas);
    return a;
}


}  // namespace ph
