// Internal declarations of libph: the plan object, device buffers and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/ph.h"

namespace ph {

// ------------------------------------------------------------------ errors

struct Error {
    ph_status status;
    std::string what;
};

void set_last_error(const std::string &s);

#define PH_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            throw ::ph::Error{PH_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)};   \
    } while (0)

// ------------------------------------------------------------------ constants

constexpr int kMortonBits = 21;                 // bits per axis of the Morton key
constexpr int kMaxDepth = 16;                   // deepest octree level supported
constexpr int kNumM2L = 316;                    // 7^3 - 3^3 well-separated offsets
constexpr int kUseWords = (kNumM2L + 31) / 32;  // words of a per-box offset mask
constexpr int kMaxLattice = 512;                // q <= 8
constexpr int kMaxShell = 6 * 8 * 8 + 2;        // shell of q+1 <= 9 points per edge

// Box flag bits (per call)
constexpr int kBoxLeaf = 1;    // a leaf of the per-call tree
constexpr int kBoxExists = 2;  // the box belongs to the per-call tree

// Device-resident per-call scalars (one struct, one allocation)
struct CallScalars {
    double imax;          // max of I over all points
    double emax;          // max of |E| over all points
    int32_t err;          // bit 0: bad source value seen
    int32_t scale_exp;    // e with I scaled by 2^-e in the FP32 forms
    int32_t n_src;
    int32_t n_tgt;
    int32_t lvl_count[kMaxDepth + 2];   // boxes per level
    int32_t lvl_src[kMaxDepth + 2];     // boxes with sources per level
    int32_t lvl_tpar[kMaxDepth + 2];    // split boxes with targets per level
    int32_t lvl_start[kMaxDepth + 3];   // first box of each level
    int32_t n_u, n_w, n_x;              // list lengths
    int32_t n_far_a, n_far_b, n_near;   // leaf lists of the target-side kernels
    int32_t n_far_a_lvl[kMaxDepth + 2]; // grid-operator leaves per level (segments of far_a)
    int32_t n_vt_lvl[kMaxDepth + 2];    // boxes with a V or X list per level (segments of vt)
    int32_t n_src_dropped;              // learned selector
    int32_t min_leafsrc_level;          // lowest level holding a leaf with sources
    int32_t fallback;                   // learned selector fell back to the threshold rule
    int32_t n_srcleaf;                  // selector rows: plan leaves holding candidate sources
    int32_t n_src_base;                 // candidate sources of the learned decisions (kept + dropped)
    int32_t n_rows;                     // learned selector: rows listed by the selection pass
    int32_t gen;                        // number of the call (never 0): V/X target tags
    uint64_t packed_total;              // selected (sources | targets << 32)
    uint64_t emax_key;                  // |E| bits << 32 | ~caller index of the largest |E|
    double emax_xyz[3];                 // that point's position
    uint64_t imax_key;                  // I bits (as FP32) << 32 | ~caller index of the largest I
    double imax_xyz[3];                 // that point's position
    double check_rel;                   // validated calls: rel-L2 of learned vs threshold result
    // algorithmic work of the call (integer counters, order independent)
    unsigned long long work[12];        // p2p pairs, l2p evals, m2p evals, p2m evals,
                                        // p2l evals, m2l pairs, m2m children, l2l boxes,
                                        // grid l2p multiply-adds, grid p2m multiply-adds,
                                        // near-field targets, table near pairs
};

// Box table (structure of arrays, capacity box_cap).  Structure fields come from the
// plan's tree over all points; per-call fields mark the pruned per-call tree.
struct BoxArrays {
    // plan time
    int32_t *level = nullptr;
    int32_t *ax = nullptr, *ay = nullptr, *az = nullptr;
    int32_t *start = nullptr, *end = nullptr;  // range of the box in the sorted point order
    int32_t *parent = nullptr;
    int32_t *child = nullptr;       // box_cap x 8, -1 if absent
    int32_t *coll = nullptr;        // box_cap x 27 colleagues, -1 if absent
    // per call (boxes outside the per-call tree have zero counts and no flags)
    int32_t *s_first = nullptr, *s_cnt = nullptr, *t_first = nullptr, *t_cnt = nullptr;
    int32_t *flags = nullptr;
    int32_t *src_rank = nullptr;    // slot of a box among its level's boxes with sources (-1 if none)
    int32_t *src_box = nullptr;     // per-level slots: box of each source rank
    int32_t *tpar_box = nullptr;    // per-level slots: the split boxes with targets
};

// Interaction lists over all boxes: each box's entries are contiguous, in enumeration order,
// at the range (begin, end) stored for the box (ranges of different boxes in any order)
struct Lists {
    uint2 *u_rng = nullptr, *w_rng = nullptr, *x_rng = nullptr;
    int32_t *u = nullptr, *w = nullptr, *x = nullptr;
    int64_t u_cap = 0, w_cap = 0, x_cap = 0;
    // leaves with targets (any order within a list): far field by a grid operator (a, in
    // per-level segments at the level's box base) or by shell points (b), and the leaves with a
    // non-empty U list (near field); box_cap entries each
    int32_t *far_b = nullptr, *near_leaves = nullptr;
    int4 *far_a = nullptr;  // (box, first target, target count, 1 near | 2 W list)
    // boxes of levels >= 3 with targets and a non-empty V or X list, per-level segments at the
    // level's box base; a box is entered once per call through vt_tag (the call's number)
    int32_t *vt = nullptr, *vt_tag = nullptr;
    // M2L offsets that reach a target, per tile of 64 slots of a level's source list (316 bits
    // in kUseWords words; the tiles of level l start at Plan::m2l_tile_base[l])
    uint32_t *m2l_tile_use = nullptr;
    // the same per source box (at the box's slot in the level's source list), so that the
    // products store only the columns some target reads
    uint32_t *m2l_box_use = nullptr;
    // per target box, its V list as translation codes (source rank * 316 + offset slot) at fixed
    // candidate slots: 8 c + o for the source box in octant o of the c-th colleague of the box's
    // parent (216 per box), each tagged with the number of the call that wrote it (high word)
    uint64_t *vslot = nullptr;
};

constexpr int kVSlots = 216;

struct Gas {
    double a, b, L, P;   // chi_min pO2, chi_max pO2, ln(chi_max/chi_min), prefactor
};

// Per-level FMM operators on the device; T is float or double.
struct OperatorsDev {
    void *uc2e_rm = nullptr;   // levels x n_lam x n_sig (row i = lattice index)
    void *uc2e_cm = nullptr;   // levels x n_sig x n_lam (transposed copy)
    void *m2m = nullptr;       // per child level: (8 n_lam) x k_pad, row c n_lam + i, column j (M2M_c[i][j])
    void *l2l = nullptr;       // per child level: (8 n_lam) x k_pad, row c n_lam + i, column j (L2L_c[i][j])
    void *m2l = nullptr;       // levels x (316 n_lam) x k_pad, row m = slot n_lam + i, column k = j
    void *lat_unit = nullptr;  // n_lam x 3 lattice nodes on [-1,1]^3 (T)
    void *shell_unit = nullptr;// n_sig x 3 shell points (radius included) in units of the half-width
    // BF16 split copies of m2l (hi, lo), row-major tiles for MFMA
    void *m2l_hi = nullptr, *m2l_lo = nullptr;
    // uniform-grid lattice operators per level (cells of a box at fixed offsets):
    //   grid_g  [lambda][r] = (uc2e_l K(shell_l, cells_l))[lambda][r]   (L2P reads columns)
    //   grid_gt [r][lambda] = same matrix transposed                      (P2M reads rows)
    void *grid_g = nullptr, *grid_gt = nullptr;
    // uniform grids, FP32: the kernel at the cell offsets of two adjacent finest-level leaves,
    // near_tab[(i + R) sx + (j + R) sy + (k + R) sz] = K(h |(i, j, k)|), 0 at the origin
    void *near_tab = nullptr;
    int near_R = 0;        // offsets per axis within [-R, R] (R = 2 m - 1 for leaves of m^3 cells)
    int near_level = -1;   // level of the leaves the table serves
    int near_sx = 0, near_sy = 0, near_sz = 0, near_n = 0;  // strides and entries
    // composite L2L translations (FP32 forms): from a box of level l to its descendant at level m
    // in relative position pos (coordinates mod 2^(m-l), pos = (x 2^(m-l) + y) 2^(m-l) + z),
    // the product of the L2L steps along the path; n_lam rows x k_pad columns each, the ones of
    // (m, l) from element comp_off[m][l]
    void *l2l_comp = nullptr;
};

constexpr int kLeafPartials = 2048;  // scan space the selector's row compaction may use
constexpr int kSelTilePoints = 4096;  // sorted points per workgroup of the selection pass
constexpr size_t kRedBytes = 1024 * 24;  // maxima partials: 1024 x (max I, |E| key, I key)
constexpr int kCompMaxDepth = 6;  // composite translations for trees of at most this depth

constexpr int kNearTabMaxR = 7;     // table for leaves of at most 4^3 cells
constexpr int kNearTabMax = 4800;   // entries kept in LDS

constexpr int kGridMaxCells = 16;  // lattice operators for boxes of at most 16^3 cells

// Far-field operators of one level in the units of the level at which they were built.  The
// kernel depends on the pressure only through a r and b r (eq. (3)), so two levels with equal
// a hw and b hw (hw the half-width; for instance level l at pressure 2p and level l - 1 at p)
// have operators that differ by powers of hw only: with f = hw_built / hw (a power of two),
// K and the M2L operators scale by f^3, the check-to-equivalent maps by f^-3, and M2M is
// unchanged.  Scaling by a power of two is exact, so a rescaled level equals a fresh build bit
// for bit.
struct CachedLevel {
    double hw = 0.0;
    uint64_t stamp = 0;                  // last build that used it (the oldest is evicted first)
    std::vector<double> uc2e, m2l, m2m;  // m2m empty when the level was built as the coarsest
};
struct OperatorCache {
    std::map<std::tuple<double, double, double>, CachedLevel> levels;  // key (a hw, b hw, ln(chi_max/chi_min))
    size_t bytes = 0;                     // host memory held by the cached levels
    size_t max_bytes = (size_t)1 << 30;   // beyond this the least recently used levels are dropped
    uint64_t clock = 0;                   // builds so far
};

struct Plan {
    // configuration
    bool self_coeff_given = false;   // the caller fixed c_self (else it follows the gas)
    int levels_reused = 0;           // far-field levels of the last operator build taken from the cache
    OperatorCache op_cache;          // far-field operators by (a hw, b hw, L), over the plan's gases
    std::map<void **, size_t> upload_bytes;  // sizes of the uploaded operator buffers
    int64_t n = 0;
    int device = 0;
    ph_precision precision = PH_FP32;
    ph_method method = PH_METHOD_FMM;
    ph_selector selector = PH_SEL_THRESHOLD;
    int q = 4, n_lam = 64, n_sig = 98;
    int k_pad = 64;          // n_lam rounded up to the GEMM K chunk
    int k_pad8 = 512;        // 8 n_lam rounded up to the GEMM K chunk
    size_t z_cap_cols = 0;   // target parents per level (Z buffer columns)
    void *d_z = nullptr;     // parent-to-child (and child-to-parent) translations: z_cap_cols x (8 n_lam)
    size_t y_cap_cols = 0;   // source boxes per translation chunk (Y buffer columns)
    bool y_all_levels = false;            // Y holds every level at once (one M2L product)
    int32_t m2l_tile_base[kMaxDepth + 2] = {};  // first tile of each level's source list
    int32_t m2l_tiles = 0;                      // tiles of all levels
    int64_t y_lvl_col[kMaxDepth + 2] = {};  // ... at these first columns
    void *d_y = nullptr;     // translation products: y_cap_cols x (316 n_lam)
    int leaf_cap = 64;
    int max_depth = 0;       // deepest level any per-call tree may reach
    double pinv_cut = 0;
    double cube_lo[3] = {0, 0, 0};
    double cube_size = 1;
    double h = 0;
    double c_self = 0;
    const void *cur_I = nullptr;             // the evaluation's source intensities (caller order)
    Gas gas{};
    ph_thresholds thr{};
    bool uniform_w = true;
    double w_uniform = 0;
    // uniform cell-centred grid aligned with the root cube: points carry integer cell indices
    bool grid_mode = false;
    int grid_n = 0;                          // cells per root-cube edge
    int grid_m[kMaxDepth + 2] = {};          // cells per box edge at each level (0 = no operator)
    int64_t grid_off[kMaxDepth + 2] = {};    // offset of each level's operator (elements)
    int32_t *d_cell = nullptr;               // sorted packed cell index ix | iy << 10 | iz << 20
    // learned selector
    std::vector<float> sel_weights;
    float sel_threshold = 0.f;
    double fallback_rel = 1e-4;     // threshold rule of the learned selector's fallback
    bool validate = false;          // learned calls also run the threshold rule and compare
    double validate_tol = 1e-3;     // ... falling back when the relative L2 difference exceeds this
    uint32_t *d_leafflag = nullptr; // per plan leaf: 1 if it holds a candidate source
    int32_t n_pleaf = 0;            // leaves of the plan's tree over all points
    int32_t *d_pleaf = nullptr;     // their box ids in box order
    std::vector<int32_t> h_pleaf;   // host copy
    int4 *d_pinfo = nullptr;           // per plan leaf: box, first point, end, 0
    int4 *d_pinfo2 = nullptr;          // per plan leaf: anchor x, y, z, level
    uint32_t *d_leafscan = nullptr; // per plan leaf: candidate flag, scanned by the row compaction
    int4 *d_rows = nullptr;         // learned selector: the call's rows (first, end, plan leaf, 0)
    int32_t *d_row_box = nullptr;   // compacted rows (training entry points): plan-leaf box ids
    float *d_row_feat = nullptr;    // and their features
    int2 *d_tile_leaves = nullptr;  // per selection tile (4096 sorted points): its plan leaves in d_leaf_pos
    int4 *d_leaf_pos = nullptr;     // plan leaves by first point: (first, end, plan-leaf index, 0)
    double *d_red = nullptr;        // partials of the call's maxima (kRedBytes)

    // plan-time device arrays
    uint64_t *d_key = nullptr;      // sorted Morton keys (n)
    int32_t *d_perm = nullptr;      // sorted -> caller index (n)
    int32_t *d_iperm = nullptr;     // caller -> sorted index (n)
    double *d_xyz = nullptr;        // sorted coordinates (n x 3)
    double *d_w = nullptr;          // sorted weights (n), null on uniform grids
    std::vector<int64_t> level_cap; // max boxes per level (from the tree over all points)
    std::vector<int64_t> level_base;// first slot of each level in the box table
    int64_t box_cap = 0;
    OperatorsDev ops;
    std::vector<double> hw;         // half-width of boxes per level

    // per-call workspace
    CallScalars *d_sc = nullptr;
    CallScalars h_sc{};             // host mirror of the last fetched scalars
    uint64_t *d_flag = nullptr;     // n packed (src | tgt << 32) flags, scanned in place
    void *d_scan_tmp = nullptr;     // scan partials
    size_t scan_tmp_bytes = 0;
    float4 *d_xyzf = nullptr;       // FP32 plans: sorted coordinates as float4 (x, y, z, 0)
    uint8_t *d_bnd = nullptr;       // 1 at the first point of a box and at the point after a box
    int32_t *d_t_out = nullptr;     // caller index of each selected target (output position)
    void *d_s_dat = nullptr;        // sources: (x, y, z, q = w * I * 2^-e), float4 or double4
    void *d_t_dat = nullptr;        // targets: (x, y, z, self = c_self * I * 2^-e or 0)
    uint8_t *d_sel = nullptr;       // selection flags per sorted point (bit 0 source, bit 1 target)
    int32_t *d_s_cell = nullptr, *d_t_cell = nullptr; // packed cell indices (grid mode)
    double *d_t_near = nullptr;     // near field (P2P) of targets whose leaf has a U list
    void *d_sref = nullptr;         // validated learned calls: the threshold rule's S (caller order)
    BoxArrays box;
    Lists lists;
    void *d_phi = nullptr;          // box_cap x n_lam upward densities
    void *d_u = nullptr;            // box_cap x n_lam downward check potentials
    float *d_feat = nullptr;        // learned selector features per plan leaf (n_pleaf x 8)
    int32_t *d_feat_cnt = nullptr;  // candidate sources per plan leaf
    float *d_sel_params = nullptr;  // device copy of the selector weights
    // per-phase timing: a ring of event sets, one set per recorded call
    static constexpr int kRing = 32;
    // marks 0..7 on the caller's stream, 8..10 on the plan's second stream (lists, near field)
    static constexpr int kMarks = 15;  // 11..14: around the M2L product launches (third, main stream)
    hipEvent_t ring[kRing][kMarks] = {};
    bool ring_used[kRing] = {};
    int ring_pos = 0;
    bool recording = false;
    double phase_sum[PH_NPHASES] = {};
    int64_t phase_calls = 0;
    bool events_ready = false;
    // the interaction lists and the near field run on a second stream, the V/X targets, offset
    // masks and deepest level's M2L products on a third, both forked from the caller's stream
    // after the tree (ev_fork); the gathers (and so the far field) wait for the near field
    // (ev_join, after the lists), the other levels' M2L products for the deepest level's
    // (ev_m2l, after the offset masks; ev_vt when that level runs with the others)
    hipStream_t side = nullptr;
    hipStream_t side2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_vt = nullptr;                     // V/X targets and M2L offset masks known
    hipEvent_t ev_p2m = nullptr, ev_m2l = nullptr;  // leaf densities known (main); deepest M2L done
    // check values of the leaves of levels >= 3 in one launch from the level-local parts of their
    // ancestors (composite translations) in place of the level-by-level L2L chain
    bool l2l_comp = false;
    int32_t *d_boxmap = nullptr;                  // boxes of level l >= 2 by coordinates (8^l, -1)
    int64_t boxmap_off[kMaxDepth + 2] = {};
    int64_t comp_off[kMaxDepth + 2][kMaxDepth + 2] = {};
    int32_t *d_gen = nullptr;  // device: number of the last call (the reset kernel advances it)
    int32_t *d_sticky = nullptr; // device: error bits of every call since the last ph_plan_check
    bool count_work = false;        // algorithmic work counters (only for calls that fetch stats)
    bool near_guard = true;         // near pairs may have (b - a) r < 1/4: small-argument series needed
    // the per-call arrays live in one workspace: the plan's own (zero-filled at creation) or,
    // for the duration of a ph_evaluate_ws call, the caller's
    char *d_ws_own = nullptr;
    std::mutex mu;                  // one call at a time enqueues on the plan
    size_t ws_bytes = 0;
    // caller-supplied target set (sorted order, 1 = may be a target), or null for every point
    uint8_t *d_tmask = nullptr;
    uint8_t *d_rs_flag = nullptr;   // per sorted point: the W list was left out there (r_s > 0)
    uint64_t *d_tile_sum = nullptr; // per selection tile: packed (sources | targets << 32) counts
    bool sets_ready = false;        // the own workspace holds a call's sets, tree and lists
    double *d_rs_bound = nullptr;   // per box: bound of its W list's field (r_s > 0)
    size_t bytes_allocated = 0;
    size_t workspace_cap = 0;
};

// ------------------------------------------------------------------ host-side helpers

// The octree over all points (every point both a source and a target), split
// while a box holds more than leaf_cap points.  Any per-call tree over selected
// subsets is this tree pruned: a box survives iff it holds selected points and
// its parent is split in the per-call tree (counts shrink monotonically down the
// tree, so the parent's test implies every ancestor's).
struct FullTree {
    std::vector<int32_t> level, ax, ay, az, start, end, parent, child, coll;
    std::vector<int64_t> level_cap;
};

void build_full_tree(const std::vector<uint64_t> &keys, int leaf_cap, int depth_limit, FullTree &T);


void *dev_alloc(Plan &p, size_t bytes);
void dev_free(void *ptr);

// Operators (ph_operators.cpp): FP64 on the host
struct HostOperators {
    int q = 0, n_lam = 0, n_sig = 0;
    std::vector<double> lat_unit, shell_unit;            // n x 3
    std::vector<std::vector<double>> uc2e;               // per level: n_lam x n_sig (row-major)
    std::vector<std::vector<double>> m2m;                // per level: 8 x n_lam x n_lam (row-major)
    std::vector<std::vector<double>> m2l;                // per level: 316 x n_lam x n_lam (row-major)
};

// cache (nullable): levels found there are rescaled instead of built, and new levels are added;
// *reused (nullable) counts the levels taken from the cache.
void build_operators(const Gas &gas, int q, double root_size, int max_depth, double cut,
                     HostOperators &out, OperatorCache *cache = nullptr, int *reused = nullptr);
double cube_self_integral(const Gas &gas, double h);
void build_near_table(const Gas &gas, double h, int R, int sx, int sy, int sz, int n, std::vector<double> &tab);
void build_grid_operator(const Gas &gas, const HostOperators &H, int level, double hw, double h, int m,
                         std::vector<double> &G);
int m2l_index(int dx, int dy, int dz);  // -1 unless the offset is well separated
void m2l_offset(int idx, int &dx, int &dy, int &dz);

// ------------------------------------------------------------------ launchers (device code)

// sort / scan (k_sort.hip)
void launch_morton_keys(const double *xyz, int64_t n, double lo0, double lo1, double lo2,
                        double size, uint64_t *keys, int32_t *idx, hipStream_t s);
void radix_sort_pairs(uint64_t *keys, int32_t *vals, uint64_t *keys_tmp, int32_t *vals_tmp, int64_t n,
                      uint32_t *hist_tmp, size_t hist_bytes, int key_bits, hipStream_t s);
size_t radix_sort_tmp_bytes(int64_t n);
size_t scan_tmp_bytes(int64_t n, size_t elem);
void exclusive_scan_u32(uint32_t *data, int64_t n, void *tmp, uint32_t *total, hipStream_t s);
void exclusive_scan_u64(uint64_t *data, int64_t n, void *tmp, uint64_t *total, hipStream_t s);
// three independent scans of n elements (totals nullable)
void launch_gather_sorted(const double *xyz, const double *w, const int32_t *perm, int64_t n,
                          double *xyz_sorted, double *w_sorted, int32_t *iperm, hipStream_t s);

// selection (k_select.hip)
// Clears the call's scalars; with gen, also advances the call number there and stores it in sc
void launch_reset_scalars(CallScalars *sc, int32_t *gen, hipStream_t s);
// partials of the call's maxima of I and |E| and of the order keys of the largest of each into
// d_red (at most 256 blocks); with gen the kernel also starts the call (clears the scalars,
// advances the call number).  The selection pass reduces the partials in every workgroup.
int reduce_blocks(int64_t n);
void launch_reduce_max(const Plan &p, const void *I, const float *E, int32_t *gen, hipStream_t s);
// the training entry points' reduction of those partials into the scalars (the selection pass
// does it itself on the evaluation path)
void launch_maxima_store(const Plan &p, bool has_e, hipStream_t s);
// selection flags (with the learned decisions on the plan leaves when learned), their scan (kept
// in d_flag for the tree build) and the compaction.  src_rel >= 0 replaces the plan's source rule
// for this pass (the threshold run of a validated call).
void launch_select(const Plan &p, const void *I, const float *E, void *S_out, hipStream_t s, bool learned,
                   double src_rel, hipEvent_t after_tiles = nullptr);
void launch_compact(const Plan &p, const void *I, void *S_zero, hipStream_t s);
void launch_reuse_begin(const Plan &p, hipStream_t s);
// validated learned call: S_out (learned) against S_ref (threshold rule); S_ref replaces S_out
// and the call is marked fallen back when their relative L2 difference exceeds tol
void launch_validate(const Plan &p, void *S_out, const void *S_ref, double tol, hipStream_t s);
void scan_tile_sums_u64(uint64_t *partial, int64_t nb, uint64_t *total, hipStream_t s);
void launch_pack_xyzf(const double *xyz, int64_t n, float4 *out, hipStream_t s);

// tree (k_tree.hip)
void build_tree(Plan &p, hipStream_t s);
// V/X targets and M2L offset masks, and the interaction lists: independent of each other (both
// enter boxes into the V/X target lists through atomics), so they may run on different streams
void build_vtargets(Plan &p, hipStream_t s);
void build_lists(Plan &p, hipStream_t s);

// fmm (k_fmm.hip, k_m2l.hip)
void fmm_upward(Plan &p, hipStream_t s);
void fmm_p2m(Plan &p, hipStream_t s);  // the upward pass split: leaf densities ...
void fmm_m2m(Plan &p, hipStream_t s);  // ... and the M2M chain
// The deepest level's M2L products on s (after the leaf densities and the offset masks);
// false if this plan computes that level with the others (then nothing is launched)
bool fmm_m2l_deepest(Plan &p, hipStream_t s);
// waits for m2l_ready (the offset masks, and the deepest level's M2L products when they run on
// another stream) before the M2L products and for side_ready (the lists and the near field) before the gathers
void fmm_downward(Plan &p, hipStream_t s, hipEvent_t m2l_ready, hipEvent_t side_ready,
                  hipEvent_t m2l_begin = nullptr, hipEvent_t m2l_end = nullptr);
void fmm_m2m_level(Plan &p, int level, hipStream_t s);  // parents at level, children at level + 1
constexpr int kGemmK = 32;  // K chunk of the translation GEMM
// far field at targets (L2P, M2P, own cell) + output: the matrix-core kernel on s, the other
// leaf kernels on s_aux (both streams must already be ordered after the downward pass and
// the near field)
void fmm_leaf(Plan &p, void *S_out, hipStream_t s, hipStream_t s_aux);
void fmm_near(Plan &p, hipStream_t s);  // near field (P2P) of the targets of leaves with a U list

// direct sum (k_direct.hip)
void run_direct(Plan &p, void *S_out, hipStream_t s);

// learned selector (k_mlp.hip)
// training entry points: the call's maxima, then the rows (candidate plan leaves in box order) and
// their features, compacted into d_row_box / d_row_feat (resets the call's scalars)
void selector_features(Plan &p, const void *I, const float *E, hipStream_t s);
void launch_mlp_forward(const float *params, const float *X, int64_t m, const int32_t *m_dev, float *logits,
                        int bf16, hipStream_t s);
void launch_mlp_backward(const float *params, const float *X, const float *y, float pos_weight,
                         int64_t m, float *grad, float *loss, hipStream_t s);
// the same with the block partials in the library's static device scratch (no allocation)
void launch_mlp_backward_noalloc(const float *params, const float *X, const float *y, float pos_weight,
                                 int64_t m, float *grad, float *loss, hipStream_t s);
void launch_adam(float *params, float *m1, float *m2, const float *grad, int64_t nparam, float lr,
                 float b1, float b2, float eps, int64_t step, hipStream_t s);

}  // namespace ph
