// C ABI entry points of libph: validation, plan construction, evaluation sequencing.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <thread>
#include <vector>

#include "k_common.h"
#include "ph_internal.h"

namespace ph {

namespace {
thread_local std::string g_last_error;

template <class T>
void upload(Plan &p, void **dst, const std::vector<T> &src)
{
    const size_t bytes = src.size() * sizeof(T);
    if (*dst) {  // a rebuild for a new gas: same operator, same size
        auto it = p.upload_bytes.find(dst);
        if (it == p.upload_bytes.end() || it->second != bytes)
            throw Error{PH_EDEVICE, "internal: rebuilt operator changed size"};
        PH_HIP(hipMemcpy(*dst, src.data(), bytes, hipMemcpyHostToDevice));
        return;
    }
    *dst = dev_alloc(p, bytes);
    p.upload_bytes[dst] = bytes;
    PH_HIP(hipMemcpy(*dst, src.data(), bytes, hipMemcpyHostToDevice));
}

// f(i) for i in [0, n) over up to 16 host threads
template <class F>
void parallel_for_host(int n, F &&f)
{
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 4 || nt == 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int i = (int)t; i < n; i += (int)nt) f(i);
        });
    for (auto &x : th) x.join();
}

template <class T>
std::vector<T> convert(const std::vector<double> &v)
{
    std::vector<T> out(v.size());
    for (size_t i = 0; i < v.size(); ++i) out[i] = (T)v[i];
    return out;
}

bool finite(double x) { return std::isfinite(x); }

// bfloat16 bits of x, round to nearest even (x finite)
uint16_t bf16_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

// x = hi + lo + O(2^-16 |x|): the two bfloat16 terms of each value
void split_bf16(const std::vector<double> &v, std::vector<uint16_t> &hi, std::vector<uint16_t> &lo)
{
    hi.resize(v.size());
    lo.resize(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        hi[i] = bf16_bits((float)v[i]);
        lo[i] = bf16_bits((float)(v[i] - (double)bf16_value(hi[i])));
    }
}

// The gas parameters (Sec. 2.1, eq. (3)): positive pressures and 0 < chi_min < chi_max
void validate_gas(const ph_gas *gas)
{
    auto bad = [](const char *m) { throw Error{PH_EINVAL, m}; };
    auto finite = [](double v) { return std::isfinite(v); };
    if (!gas) bad("gas is null");
    if (!(gas->p_torr > 0) || !finite(gas->p_torr)) bad("gas.p_torr must be > 0");
    if (!(gas->o2_fraction > 0) || !(gas->o2_fraction <= 1)) bad("gas.o2_fraction must be in (0, 1]");
    if (!(gas->pq_torr >= 0) || !finite(gas->pq_torr)) bad("gas.pq_torr must be >= 0");
    if (!(gas->xi_omega_over_alpha >= 0) || !finite(gas->xi_omega_over_alpha))
        bad("gas.xi_omega_over_alpha must be >= 0");
    if (!(gas->chi_min > 0) || !(gas->chi_max > gas->chi_min) || !finite(gas->chi_max))
        bad("gas needs 0 < chi_min < chi_max");
}

// Validation happens entirely on the host, before any device call.
void validate(const ph_points *pts, const ph_gas *gas, const ph_thresholds *thr, const ph_options *opt)
{
    auto bad = [](const std::string &s) { throw Error{PH_EINVAL, s}; };
    if (!pts || !gas || !thr || !opt) bad("null argument");
    if (pts->n < 1) bad("points.n must be >= 1");
    if (pts->n > (int64_t)1 << 30) bad("points.n exceeds 2^30");
    if (!pts->xyz) bad("points.xyz is null");
    for (int64_t i = 0; i < 3 * pts->n; ++i)
        if (!finite(pts->xyz[i])) bad("points.xyz has a non-finite coordinate");
    if (pts->w) {
        for (int64_t i = 0; i < pts->n; ++i)
            if (!finite(pts->w[i]) || pts->w[i] < 0) bad("points.w must be finite and >= 0");
    } else if (!(pts->h > 0) || !finite(pts->h)) {
        bad("points.h must be > 0 when points.w is null");
    }
    if (pts->h < 0 || !finite(pts->h)) bad("points.h must be finite and >= 0");
    if (std::isnan(pts->self_coeff)) {
        if (!(pts->h > 0)) bad("self_coeff NaN needs h > 0");
    } else if (!finite(pts->self_coeff) || pts->self_coeff < 0) {
        bad("points.self_coeff must be NaN or finite and >= 0");
    }
    if (pts->cube_size > 0) {
        for (int d = 0; d < 3; ++d)
            if (!finite(pts->cube_lo[d])) bad("points.cube_lo must be finite");
        for (int64_t i = 0; i < pts->n; ++i)
            for (int d = 0; d < 3; ++d) {
                double x = pts->xyz[3 * i + d];
                if (x < pts->cube_lo[d] || x > pts->cube_lo[d] + pts->cube_size)
                    bad("a point lies outside the root cube");
            }
    } else if (!finite(pts->cube_size)) {
        bad("points.cube_size must be finite");
    }
    validate_gas(gas);
    if (!finite(thr->src_rel) || thr->src_rel < 0 || thr->src_rel > 1) bad("thresholds.src_rel must be in [0, 1]");
    if (!finite(thr->e_abs)) bad("thresholds.e_abs must be finite");
    if (!finite(thr->e_rel) || thr->e_rel > 1) bad("thresholds.e_rel must be <= 1 (negative = off)");
    if (!finite(thr->e_applied) || thr->e_applied < 0) bad("thresholds.e_applied must be >= 0");
    if (!std::isfinite(thr->r_s) || thr->r_s < 0) bad("thresholds.r_s (third strategy) must be finite and >= 0");
    if (opt->precision < PH_FP64 || opt->precision > PH_FP32_BF16SPLIT) bad("options.precision out of range");
    if (opt->method < PH_METHOD_FMM || opt->method > PH_METHOD_DIRECT) bad("options.method out of range");
    if (opt->selector < PH_SEL_THRESHOLD || opt->selector > PH_SEL_LEARNED) bad("options.selector out of range");
    if (opt->order_q != 0 && (opt->order_q < 2 || opt->order_q > 8)) bad("options.order_q must be 0 or 2..8");
    if (opt->leaf_capacity < 0 || opt->leaf_capacity > 4096) bad("options.leaf_capacity must be 0..4096");
    if (opt->max_depth < 0 || opt->max_depth > kMaxDepth) bad("options.max_depth must be 0..16");
    if (!(opt->pinv_rel_cutoff >= 0) || opt->pinv_rel_cutoff >= 1) bad("options.pinv_rel_cutoff must be in [0, 1)");
    if (opt->selector == PH_SEL_LEARNED) {
        if (!opt->selector_weights) bad("learned selector needs selector_weights");
        for (int i = 0; i < PH_MLP_NPARAM; ++i)
            if (!std::isfinite(opt->selector_weights[i])) bad("selector_weights has a non-finite value");
        if (opt->method != PH_METHOD_FMM) bad("the learned selector needs the FMM method");
        if (!std::isfinite(opt->selector_logit_threshold)) bad("selector_logit_threshold must be finite");
        if (!(opt->selector_fallback_rel >= 0) || opt->selector_fallback_rel > 1)
            bad("selector_fallback_rel must be in [0, 1]");
        if (!(opt->tol >= 0) || !std::isfinite(opt->tol)) bad("options.tol must be finite and >= 0");
    }
}

// Capacities of the per-call arrays (lists, translation buffers, scan space): fixed per plan.
void size_workspace(Plan &p)
{
    const int64_t n = p.n;
    const size_t rs = p.precision == PH_FP64 ? sizeof(double) : sizeof(float);
    const int64_t B = p.box_cap;
    // also the list build's per-workgroup totals (3 words per 256 boxes)
    p.scan_tmp_bytes = std::max({scan_tmp_bytes(n, 8), scan_tmp_bytes(p.box_cap + 1, 4),
                                 (size_t)12 * ((p.box_cap + 255) / 256) + 256, (size_t)16 * kLeafPartials});
    Lists &L = p.lists;
    L.u_cap = std::max<int64_t>(1024, 64 * B);
    L.w_cap = std::max<int64_t>(1024, 32 * B);
    L.x_cap = std::max<int64_t>(1024, 32 * B);
    if (const char *env = std::getenv("PH_LIST_ENTRIES_PER_BOX")) {  // small lists: overflow handling tests
        const int64_t k = std::max<int64_t>(0, std::atoll(env));
        L.u_cap = L.w_cap = L.x_cap = std::max<int64_t>(1, k * B);
    }
    p.m2l_tiles = 0;
    for (int l = 0; l <= p.max_depth; ++l) {
        p.m2l_tile_base[l] = p.m2l_tiles;
        p.m2l_tiles += (int32_t)((p.level_cap[l] + 63) / 64);
    }
    if (p.method == PH_METHOD_FMM) {
        // translation products: the source boxes of every level at once (one M2L product for
        // all levels) if that takes at most an eighth of the device memory (a quarter of a
        // workspace cap); else one level at a time, in chunks of at most that size (at least
        // one tile of source boxes)
        const size_t col_bytes = (size_t)kNumM2L * p.n_lam * rs;
        int64_t widest2 = 1;
        for (int l = 2; l <= p.max_depth; ++l) widest2 = std::max<int64_t>(widest2, p.level_cap[l]);
        size_t total_mem = 0;
        PH_HIP(hipDeviceTotalMem(&total_mem, p.device));
        size_t budget = std::max<size_t>(total_mem / 8, 256ull << 20);
        if (p.workspace_cap) budget = std::min<size_t>(budget, p.workspace_cap / 4);
        if (const char *env = std::getenv("PH_TRANSLATION_BUFFER_MB")) budget = (size_t)std::atoll(env) << 20;
        int64_t all_cols = 0;
        for (int l = 2; l <= p.max_depth; ++l) {
            p.y_lvl_col[l] = all_cols;
            all_cols += p.level_cap[l];
        }
        p.y_all_levels = all_cols > 0 && (size_t)all_cols * col_bytes <= budget;
        if (p.y_all_levels) p.y_cap_cols = (size_t)all_cols;
        else p.y_cap_cols = (size_t)std::max<int64_t>(64, std::min<int64_t>(widest2, (int64_t)(budget / col_bytes)) / 64 * 64);
        p.z_cap_cols = (size_t)widest2;
    }
}

// Points every per-call array of the plan into the workspace at base, in 256-byte aligned
// slices, and returns the workspace size.  assign = false only measures (no pointer changes).
// A workspace must be all zero before its first call: call numbers, box tags and the
// selection flags of "no earlier call" are zeros.
size_t layout_workspace(Plan &p, char *base, bool assign)
{
    size_t off = 0;
    auto take = [&](auto **dst, size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        if (assign) *dst = reinterpret_cast<std::remove_pointer_t<decltype(dst)>>(base + off);
        off += std::max<size_t>(bytes, 16);
    };
    const int64_t n = p.n;
    const size_t rs = p.precision == PH_FP64 ? sizeof(double) : sizeof(float);
    const int64_t B = p.box_cap;
    take(&p.d_sc, sizeof(CallScalars));
    take(&p.d_gen, sizeof(int32_t));
    take(&p.d_flag, (size_t)n * sizeof(uint64_t));
    take(&p.d_sel, (size_t)n);
    take(&p.d_scan_tmp, p.scan_tmp_bytes);
    take(&p.d_tile_sum, (size_t)((n + kSelTilePoints - 1) / kSelTilePoints) * 8);
    take(&p.d_red, kRedBytes);
    take(&p.d_t_out, (size_t)n * 4);
    take(&p.d_s_dat, (size_t)n * 4 * rs);
    take(&p.d_t_dat, (size_t)n * 4 * rs);
    take(&p.d_t_near, (size_t)n * 8);
    take(&p.d_sref, (size_t)n * rs);
    if (p.grid_mode) {
        take(&p.d_s_cell, (size_t)n * 4);
        take(&p.d_t_cell, (size_t)n * 4);
    }
    BoxArrays &b = p.box;
    for (int32_t **f : {&b.s_first, &b.s_cnt, &b.t_first, &b.t_cnt, &b.flags, &b.tpar_box, &b.src_rank, &b.src_box})
        take(f, (size_t)B * 4);
    Lists &L = p.lists;
    take(&L.u_rng, (size_t)B * sizeof(uint2));
    take(&L.w_rng, (size_t)B * sizeof(uint2));
    take(&L.x_rng, (size_t)B * sizeof(uint2));
    take(&L.u, (size_t)L.u_cap * 4);
    take(&L.w, (size_t)L.w_cap * 4);
    take(&L.x, (size_t)L.x_cap * 4);
    take(&L.far_a, (size_t)B * sizeof(int4));
    take(&L.far_b, (size_t)B * 4);
    take(&L.near_leaves, (size_t)B * 4);
    take(&L.vt, (size_t)B * 4);
    take(&L.vt_tag, (size_t)B * 4);
    take(&L.m2l_tile_use, (size_t)std::max(p.m2l_tiles, 1) * kUseWords * 4);
    take(&L.m2l_box_use, (size_t)B * kUseWords * 4);
    take(&L.vslot, (size_t)B * kVSlots * 8);
    if (p.method == PH_METHOD_FMM) {
        take(&p.d_phi, (size_t)B * p.n_lam * rs);
        take(&p.d_u, (size_t)B * p.n_lam * rs);
        take(&p.d_y, p.y_cap_cols * (size_t)kNumM2L * p.n_lam * rs);
        take(&p.d_z, p.z_cap_cols * 8 * (size_t)p.n_lam * rs);
    }
    const int64_t NL = std::max<int32_t>(p.n_pleaf, 1);
    take(&p.d_feat, (size_t)NL * 8 * 4);
    take(&p.d_feat_cnt, (size_t)NL * 4);
    take(&p.d_leafscan, (size_t)(NL + 1) * 4);
    take(&p.d_rows, (size_t)NL * sizeof(int4));
    take(&p.d_row_box, (size_t)NL * 4);
    take(&p.d_row_feat, (size_t)NL * 8 * 4);
    take(&p.d_leafflag, (size_t)(NL + 1) * 4);
    if (p.thr.r_s > 0) {
        take(&p.d_rs_flag, (size_t)n);
        take(&p.d_rs_bound, (size_t)B * 8);
    }
    return (off + 255) & ~(size_t)255;
}

// The plan's own workspace (zero-filled) and its plan-time neighbours
void alloc_workspace(Plan &p)
{
    size_workspace(p);
    p.ws_bytes = layout_workspace(p, nullptr, false);
    p.d_ws_own = (char *)dev_alloc(p, p.ws_bytes);
    PH_HIP(hipMemset(p.d_ws_own, 0, p.ws_bytes));
    layout_workspace(p, p.d_ws_own, true);
    p.d_sticky = (int32_t *)dev_alloc(p, sizeof(int32_t));
    PH_HIP(hipMemset(p.d_sticky, 0, sizeof(int32_t)));
    p.d_sel_params = (float *)dev_alloc(p, PH_MLP_NPARAM * 4);
    if (!p.sel_weights.empty())
        PH_HIP(hipMemcpy(p.d_sel_params, p.sel_weights.data(), PH_MLP_NPARAM * 4, hipMemcpyHostToDevice));
}

// The second and third streams of the plans on one device, shared by them all (default
// priority).  A process with several plans would otherwise hold more streams than the device
// has hardware queues, and streams that share a queue run one after the other.  Calls on
// different plans enqueue their work on these streams one call at a time (side_mu).
struct SideStreams {
    hipStream_t side = nullptr, side2 = nullptr;
    int refs = 0;
    std::mutex enqueue;  // held while a call enqueues its work
};
static std::mutex g_side_mu;
static std::map<int, SideStreams> g_side;

static SideStreams &acquire_side_streams(int device)
{
    std::lock_guard<std::mutex> lock(g_side_mu);
    SideStreams &ss = g_side[device];
    if (ss.refs == 0) {
        PH_HIP(hipStreamCreateWithFlags(&ss.side, hipStreamNonBlocking));
        PH_HIP(hipStreamCreateWithFlags(&ss.side2, hipStreamNonBlocking));
    }
    ++ss.refs;
    return ss;
}

static void release_side_streams(int device)
{
    std::lock_guard<std::mutex> lock(g_side_mu);
    auto it = g_side.find(device);
    if (it == g_side.end()) return;
    if (--it->second.refs == 0) {
        (void)hipStreamDestroy(it->second.side);
        (void)hipStreamDestroy(it->second.side2);
        g_side.erase(it);
    }
}

std::mutex &side_enqueue_mutex(int device)
{
    std::lock_guard<std::mutex> lock(g_side_mu);
    return g_side[device].enqueue;
}

void free_plan(Plan *p)
{
    if (!p) return;
    // every pointer member that came from dev_alloc
    void *ptrs[] = {p->d_key, p->d_perm, p->d_iperm, p->d_xyz, p->d_w, p->ops.uc2e_rm, p->ops.uc2e_cm,
                    p->ops.m2m, p->ops.l2l, p->ops.m2l, p->ops.lat_unit, p->ops.shell_unit, p->ops.m2l_hi,
                    p->ops.m2l_lo, p->d_xyzf, p->d_bnd, p->box.level, p->box.ax, p->box.ay, p->box.az,
                    p->box.parent, p->box.child, p->box.coll, p->box.start, p->box.end, p->d_ws_own,
                    p->d_sel_params, p->d_pleaf, p->d_pinfo, p->d_pinfo2,
                    p->d_cell, p->ops.grid_g, p->ops.grid_gt, p->ops.near_tab, p->d_sticky, p->ops.l2l_comp,
                    p->d_boxmap, p->d_tmask, p->d_leaf_pos, p->d_tile_leaves};
    // events and streams first, then the memory the work on them used
    if (p->events_ready)
        for (auto &set : p->ring)
            for (auto &e : set) (void)hipEventDestroy(e);
    for (hipEvent_t e : {p->ev_fork, p->ev_join, p->ev_vt, p->ev_p2m, p->ev_m2l})
        if (e) (void)hipEventDestroy(e);
    if (p->side) release_side_streams(p->device);
    for (void *q : ptrs) dev_free(q);
    delete p;
}

ph_status fail(const Error &e)
{
    g_last_error = e.what;
    return e.status;
}

}  // namespace

void set_last_error(const std::string &s) { g_last_error = s; }

void *dev_alloc(Plan &p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (p.workspace_cap && p.bytes_allocated + bytes > p.workspace_cap)
        throw Error{PH_ENOMEM, "workspace cap exceeded (" + std::to_string(p.bytes_allocated + bytes) + " bytes)"};
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) throw Error{PH_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    p.bytes_allocated += bytes;
    return ptr;
}

void dev_free(void *ptr)
{
    if (ptr) (void)hipFree(ptr);
}

// Everything that depends on the gas (Sec. 2.1, eqs. (1)-(3)): the constants a, b, L and P,
// the own-cell coefficient, and the far-field operators with the grid operators and the near
// table.  Called at plan creation and again for each new gas of ph_plan_set_gas; operator
// buffers keep their sizes (the tree and the order are fixed by the plan), so a rebuild
// copies into them.  Levels whose a hw and b hw were built before come from the plan's cache.
static void build_gas_state(Plan &p, const ph_gas *gas)
{
    const double pO2 = gas->o2_fraction * gas->p_torr;
    p.gas.a = gas->chi_min * pO2;
    p.gas.b = gas->chi_max * pO2;
    p.gas.L = std::log(gas->chi_max / gas->chi_min);
    p.gas.P = gas->pq_torr / (gas->p_torr + gas->pq_torr) * gas->xi_omega_over_alpha;
    if (!p.self_coeff_given) p.c_self = cube_self_integral(p.gas, p.h);
    // on a grid the closest distinct pair is h apart: the guarded form is needed only if (b - a) h < 1/4
    p.near_guard = !(p.grid_mode && (p.gas.b - p.gas.a) * p.h >= 0.25);
    p.levels_reused = 0;
    if (p.method == PH_METHOD_FMM) {
        HostOperators H;
        build_operators(p.gas, p.q, p.cube_size, std::max(p.max_depth, 2), p.pinv_cut, H, &p.op_cache,
                        &p.levels_reused);
        p.n_lam = H.n_lam;
        p.n_sig = H.n_sig;
        const int nl = p.n_lam, ns = p.n_sig, L = p.max_depth + 1;
        std::vector<double> rm((size_t)L * nl * ns, 0.0), cm((size_t)L * nl * ns, 0.0);
        p.k_pad8 = ((8 * nl + kGemmK - 1) / kGemmK) * kGemmK;
        const int kp8 = p.k_pad8;
        const int kpl = ((nl + kGemmK - 1) / kGemmK) * kGemmK;
        std::vector<double> m2m((size_t)L * 8 * nl * kpl, 0.0), l2l((size_t)L * 8 * nl * kpl, 0.0);
        (void)kp8;
        p.k_pad = ((nl + kGemmK - 1) / kGemmK) * kGemmK;
        const int kp = p.k_pad;
        std::vector<double> m2l((size_t)L * kNumM2L * nl * kp, 0.0);
        for (int l = 2; l < L; ++l) {
            const std::vector<double> &U = H.uc2e[l];
            for (int i = 0; i < nl; ++i)
                for (int k = 0; k < ns; ++k) {
                    rm[(size_t)l * nl * ns + (size_t)i * ns + k] = U[(size_t)i * ns + k];
                    cm[(size_t)l * nl * ns + (size_t)k * nl + i] = U[(size_t)i * ns + k];
                }
            if (l >= 3)
                for (int c = 0; c < 8; ++c)
                    for (int i = 0; i < nl; ++i)
                        for (int j = 0; j < nl; ++j) {
                            const double v = H.m2m[l][(size_t)c * nl * nl + (size_t)i * nl + j];
                            // M2M stacked operand: row c nl + i (parent lattice, as seen from octant c),
                            // column j (child lattice)
                            m2m[((size_t)l * 8 * nl + (size_t)c * nl + i) * kpl + j] = v;
                            // L2L = M2M^T: row c nl + j (child c check point), column i (parent)
                            l2l[((size_t)l * 8 * nl + (size_t)c * nl + j) * kpl + i] = v;
                        }
            // stacked GEMM operand: row slot * nl + i, column j (zero padded to k_pad)
            for (int t = 0; t < kNumM2L; ++t)
                for (int i = 0; i < nl; ++i)
                    for (int j = 0; j < nl; ++j)
                        m2l[((size_t)l * kNumM2L * nl + (size_t)t * nl + i) * kp + j] =
                            H.m2l[l][(size_t)t * nl * nl + (size_t)i * nl + j];
        }
        std::vector<double> shell = H.shell_unit, lat = H.lat_unit;
        // lattice operators of uniform-grid boxes
        std::vector<double> gg, ggt;
        if (p.grid_mode) {
            for (int l = 2; l < L; ++l) {
                const int m = (p.grid_n % (1 << l) == 0) ? (p.grid_n >> l) : 0;
                if (m < 1 || m > kGridMaxCells) continue;
                std::vector<double> G;
                build_grid_operator(p.gas, H, l, p.hw[l], p.h, m, G);
                const int R = m * m * m;
                p.grid_m[l] = m;
                p.grid_off[l] = (int64_t)gg.size();
                gg.insert(gg.end(), G.begin(), G.end());
                ggt.resize(gg.size());
                for (int li = 0; li < nl; ++li)
                    for (int r = 0; r < R; ++r) ggt[p.grid_off[l] + (size_t)r * nl + li] = G[(size_t)li * R + r];
            }
            if (gg.empty()) gg.push_back(0.0), ggt.push_back(0.0);
        }
        // near-field kernel table (FP32 forms): offsets between two adjacent leaves of the
        // finest level, m^3 cells each, lie within [-(2m - 1), 2m - 1] per axis
        if (p.grid_mode && p.precision != PH_FP64) {
            const int D = p.max_depth;
            const int m = (p.grid_n % (1 << D) == 0) ? (p.grid_n >> D) : 0;
            const int R = 2 * m - 1;
            if (m >= 1 && R <= kNearTabMaxR) {
                // strides: y 1, x 16, z chosen so that a leaf's targets (the lanes of a wave, in
                // the sorted order of the first finest-level box, which holds the first m^3
                // points) read the table without LDS bank conflicts (32 banks per half wave, 64
                // per wave), or with as few as any z stride in range allows
                const int S = 2 * R + 1, mc = (int)std::min<int64_t>(m * m * m, p.n);
                std::vector<int32_t> c0(mc);
                PH_HIP(hipMemcpy(c0.data(), p.d_cell, (size_t)mc * 4, hipMemcpyDeviceToHost));
                int lo[3] = {1 << 30, 1 << 30, 1 << 30};
                for (int32_t c : c0)
                    for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], (c >> (10 * d)) & 1023);
                const int sx = 16, sy = 1;
                int sz = S * sx, worst_best = 1 << 30;
                for (int cand = S * sx; cand < S * sx + 64; ++cand) {
                    int worst = 0;
                    for (int nb : {32, 64}) {
                        const int group = nb == 32 ? 32 : 64;
                        for (int g0 = 0; g0 < mc; g0 += group) {
                            std::vector<std::vector<int>> banks(nb);
                            for (int l = g0; l < std::min(mc, g0 + group); ++l) {
                                const int x = ((c0[l] & 1023) - lo[0]), y = (((c0[l] >> 10) & 1023) - lo[1]),
                                          z = (((c0[l] >> 20) & 1023) - lo[2]);
                                const int idx = x * sx + y * sy + z * cand;
                                auto &bk = banks[idx % nb];
                                if (std::find(bk.begin(), bk.end(), idx) == bk.end()) bk.push_back(idx);
                            }
                            for (auto &bk : banks) worst = std::max(worst, (int)bk.size());
                        }
                    }
                    if (worst < worst_best) worst_best = worst, sz = cand;
                }
                const int n_tab = S * sz;
                if (n_tab <= kNearTabMax) {
                    std::vector<double> tab;
                    build_near_table(p.gas, p.h, R, sx, sy, sz, n_tab, tab);
                    std::vector<float> tf = convert<float>(tab);
                    tf.resize((tf.size() + 3) & ~(size_t)3, 0.0f);  // whole float4 for the kernel's loads
                    upload(p, &p.ops.near_tab, tf);
                    p.ops.near_R = R;
                    p.ops.near_level = D;
                    p.ops.near_sx = sx;
                    p.ops.near_sy = sy;
                    p.ops.near_sz = sz;
                    p.ops.near_n = n_tab;
                }
            }
        }
        if (p.precision == PH_FP64) {
            upload(p, &p.ops.uc2e_rm, rm);
            upload(p, &p.ops.uc2e_cm, cm);
            upload(p, &p.ops.m2m, m2m);
            upload(p, &p.ops.l2l, l2l);
            upload(p, &p.ops.m2l, m2l);
            upload(p, &p.ops.lat_unit, lat);
            upload(p, &p.ops.shell_unit, shell);
            if (p.grid_mode) {
                upload(p, &p.ops.grid_g, gg);
                upload(p, &p.ops.grid_gt, ggt);
            }
        } else {
            upload(p, &p.ops.uc2e_rm, convert<float>(rm));
            upload(p, &p.ops.uc2e_cm, convert<float>(cm));
            upload(p, &p.ops.m2m, convert<float>(m2m));
            upload(p, &p.ops.l2l, convert<float>(l2l));
            if (p.d_boxmap && nl <= 64 && p.k_pad <= 64) {
                // composite translations, level by level in FP64: the one from level l to level m
                // at position pos is L2L(m, o) times the one from l to m - 1 at the parent's
                // position (pos / 2 per axis), o the octant of the last step; L2L(m, o)[j][i] =
                // M2M(m, o)[i][j]
                const int D = p.max_depth, kp = p.k_pad;
                std::vector<std::vector<double>> prev(D + 1), cur(D + 1);
                std::vector<float> comp;
                for (int m = 3; m <= D; ++m) {
                    for (int l = 2; l < m; ++l) {
                        const int side = 1 << (m - l), npos = side * side * side;
                        cur[l].assign((size_t)npos * nl * nl, 0.0);
                        parallel_for_host(npos, [&](int pos) {
                            const int rx = pos / (side * side), ry = (pos / side) % side, rz = pos % side;
                            const int o = ((rx & 1) << 2) | ((ry & 1) << 1) | (rz & 1);
                            const double *M = &H.m2m[m][(size_t)o * nl * nl];
                            double *dst = &cur[l][(size_t)pos * nl * nl];
                            if (l == m - 1) {
                                for (int j = 0; j < nl; ++j)
                                    for (int i = 0; i < nl; ++i) dst[(size_t)j * nl + i] = M[(size_t)i * nl + j];
                                return;
                            }
                            const int hs = side / 2;
                            const int ppos = ((rx >> 1) * hs + (ry >> 1)) * hs + (rz >> 1);
                            const double *Tp = &prev[l][(size_t)ppos * nl * nl];
                            for (int k = 0; k < nl; ++k)
                                for (int j = 0; j < nl; ++j) {
                                    const double mkj = M[(size_t)k * nl + j];
                                    const double *tk = Tp + (size_t)k * nl;
                                    double *dj = dst + (size_t)j * nl;
                                    for (int i = 0; i < nl; ++i) dj[i] += mkj * tk[i];
                                }
                        });
                        p.comp_off[m][l] = (int64_t)comp.size();
                        comp.resize(comp.size() + (size_t)npos * nl * kp, 0.0f);
                        float *out = comp.data() + p.comp_off[m][l];
                        for (int pos = 0; pos < npos; ++pos)
                            for (int j = 0; j < nl; ++j)
                                for (int i = 0; i < nl; ++i)
                                    out[((size_t)pos * nl + j) * kp + i] =
                                        (float)cur[l][((size_t)pos * nl + j) * nl + i];
                    }
                    std::swap(prev, cur);
                }
                upload(p, &p.ops.l2l_comp, comp);
                p.l2l_comp = true;
            }
            upload(p, &p.ops.m2l, convert<float>(m2l));
            if (p.precision == PH_FP32_BF16SPLIT) {
                std::vector<uint16_t> hi, lo;
                split_bf16(m2l, hi, lo);
                upload(p, &p.ops.m2l_hi, hi);
                upload(p, &p.ops.m2l_lo, lo);
            }
            upload(p, &p.ops.lat_unit, convert<float>(lat));
            upload(p, &p.ops.shell_unit, convert<float>(shell));
            if (p.grid_mode) {
                upload(p, &p.ops.grid_g, convert<float>(gg));
                upload(p, &p.ops.grid_gt, convert<float>(ggt));
            }
        }
    }
}

static void create_plan(Plan &p, const ph_points *pts, const ph_gas *gas, const ph_thresholds *thr,
                        const ph_options *opt)
{
    p.n = pts->n;
    PH_HIP(hipGetDevice(&p.device));
    p.precision = opt->precision;
    p.method = opt->method;
    p.selector = opt->selector;
    p.q = opt->order_q ? opt->order_q : (p.precision == PH_FP64 ? 6 : 4);
    p.leaf_cap = opt->leaf_capacity ? opt->leaf_capacity : 64;
    p.pinv_cut = opt->pinv_rel_cutoff > 0 ? opt->pinv_rel_cutoff : (p.precision == PH_FP64 ? 1e-15 : 1e-7);
    p.thr = *thr;
    p.workspace_cap = opt->workspace_cap_bytes;
    p.h = pts->h;
    p.self_coeff_given = !std::isnan(pts->self_coeff);
    p.c_self = pts->self_coeff;
    p.uniform_w = pts->w == nullptr;
    p.w_uniform = p.uniform_w ? pts->h * pts->h * pts->h : 0.0;
    if (opt->selector == PH_SEL_LEARNED) {
        p.validate = opt->validate != 0;
        p.validate_tol = opt->tol > 0 ? opt->tol : (opt->tol == 0 && opt->validate ? 0.0 : 1e-3);
        p.sel_weights.assign(opt->selector_weights, opt->selector_weights + PH_MLP_NPARAM);
        p.sel_threshold = opt->selector_logit_threshold;
        p.fallback_rel = opt->selector_fallback_rel > 0 ? opt->selector_fallback_rel : 1e-4;
    }
    // root cube
    if (pts->cube_size > 0) {
        for (int d = 0; d < 3; ++d) p.cube_lo[d] = pts->cube_lo[d];
        p.cube_size = pts->cube_size;
    } else {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t i = 0; i < p.n; ++i)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], pts->xyz[3 * i + d]);
                hi[d] = std::max(hi[d], pts->xyz[3 * i + d]);
            }
        double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
        if (!(ext > 0)) ext = 1.0;
        ext *= 1.0 + 1e-9;
        for (int d = 0; d < 3; ++d) p.cube_lo[d] = lo[d] - 1e-12 * ext;
        p.cube_size = ext * (1.0 + 2e-12);
    }
    // points to the device, keys, sort
    const int64_t n = p.n;
    double *d_xyz_in = (double *)dev_alloc(p, (size_t)n * 3 * 8);
    double *d_w_in = nullptr;
    PH_HIP(hipMemcpy(d_xyz_in, pts->xyz, (size_t)n * 3 * 8, hipMemcpyHostToDevice));
    if (pts->w) {
        d_w_in = (double *)dev_alloc(p, (size_t)n * 8);
        PH_HIP(hipMemcpy(d_w_in, pts->w, (size_t)n * 8, hipMemcpyHostToDevice));
    }
    p.d_key = (uint64_t *)dev_alloc(p, (size_t)n * 8);
    p.d_perm = (int32_t *)dev_alloc(p, (size_t)n * 4);
    uint64_t *ktmp = (uint64_t *)dev_alloc(p, (size_t)n * 8);
    int32_t *vtmp = (int32_t *)dev_alloc(p, (size_t)n * 4);
    size_t hb = radix_sort_tmp_bytes(n);
    uint32_t *htmp = (uint32_t *)dev_alloc(p, hb);
    hipStream_t s = nullptr;
    launch_morton_keys(d_xyz_in, n, p.cube_lo[0], p.cube_lo[1], p.cube_lo[2], p.cube_size, p.d_key, p.d_perm, s);
    radix_sort_pairs(p.d_key, p.d_perm, ktmp, vtmp, n, htmp, hb, 3 * kMortonBits, s);
    p.d_xyz = (double *)dev_alloc(p, (size_t)n * 3 * 8);
    p.d_iperm = (int32_t *)dev_alloc(p, (size_t)n * 4);
    if (d_w_in) p.d_w = (double *)dev_alloc(p, (size_t)n * 8);
    launch_gather_sorted(d_xyz_in, d_w_in, p.d_perm, n, p.d_xyz, p.d_w, p.d_iperm, s);
    if (p.precision != PH_FP64) {
        p.d_xyzf = (float4 *)dev_alloc(p, (size_t)n * sizeof(float4));
        launch_pack_xyzf(p.d_xyz, n, p.d_xyzf, s);
    }
    PH_HIP(hipStreamSynchronize(s));
    dev_free(ktmp);
    dev_free(vtmp);
    dev_free(htmp);
    dev_free(d_xyz_in);
    dev_free(d_w_in);
    p.bytes_allocated -= (size_t)n * 8 + (size_t)n * 4 + hb + (size_t)n * 24 + (d_w_in ? (size_t)n * 8 : 0);
    // uniform grid aligned with the root cube: every point at a cell centre
    if (!pts->w && pts->h > 0) {
        const double Nf = p.cube_size / pts->h;
        const long N = std::lround(Nf);
        bool ok = N >= 1 && N <= 1024 && std::fabs(Nf - (double)N) < 1e-9 * (double)N;
        std::vector<int32_t> cell(ok ? n : 0);
        for (int64_t i = 0; ok && i < n; ++i) {
            int32_t c = 0;
            for (int d = 0; d < 3; ++d) {
                const double f = (pts->xyz[3 * i + d] - p.cube_lo[d]) / pts->h - 0.5;
                const long ci = std::lround(f);
                if (std::fabs(f - (double)ci) > 1e-6 || ci < 0 || ci >= N) {
                    ok = false;
                    break;
                }
                c |= (int32_t)ci << (10 * d);
            }
            if (ok) cell[i] = c;
        }
        if (ok) {
            std::vector<int32_t> perm(n), sorted(n);
            PH_HIP(hipMemcpy(perm.data(), p.d_perm, (size_t)n * 4, hipMemcpyDeviceToHost));
            for (int64_t k = 0; k < n; ++k) sorted[k] = cell[perm[k]];
            p.d_cell = (int32_t *)dev_alloc(p, (size_t)n * 4);
            PH_HIP(hipMemcpy(p.d_cell, sorted.data(), (size_t)n * 4, hipMemcpyHostToDevice));
            p.grid_mode = true;
            p.grid_n = (int)N;
        }
    }
    // default order from measured error: the FP64 form reaches 1e-7 at q = 6 on uniform grids
    // but needs q = 7 on clustered point clouds (1.0e-6 at q = 6, 2.6e-7 at q = 7)
    if (!opt->order_q && p.precision == PH_FP64 && !p.grid_mode) p.q = 7;
    // FP32 forms: the pseudo-inverses are regularised so that FP32 rounding is not amplified by
    // their conditioning; on clustered clouds (boxes over many absorption lengths, and at low
    // pressure few) 1e-4 sigma_max keeps the error near 1e-4 at 40 and 760 Torr, where 1e-7
    // reaches 1.5e-3 at 40 Torr; uniform grids at 760 Torr are best at 1e-7 (5e-5)
    if (opt->pinv_rel_cutoff <= 0 && p.precision != PH_FP64 && !p.grid_mode) p.pinv_cut = 1e-4;
    // tree bound from the tree over all points
    std::vector<uint64_t> hkeys(n);
    PH_HIP(hipMemcpy(hkeys.data(), p.d_key, (size_t)n * 8, hipMemcpyDeviceToHost));
    int depth_limit = opt->max_depth ? opt->max_depth : kMaxDepth;
    FullTree FT;
    build_full_tree(hkeys, p.leaf_cap, depth_limit, FT);
    p.level_cap = FT.level_cap;
    p.max_depth = (int)p.level_cap.size() - 1;
    {
        // the tree structure is fixed for the plan: upload it once
        BoxArrays &bx = p.box;
        auto up = [&](int32_t **dst, const std::vector<int32_t> &v) {
            *dst = (int32_t *)dev_alloc(p, v.size() * 4);
            PH_HIP(hipMemcpy(*dst, v.data(), v.size() * 4, hipMemcpyHostToDevice));
        };
        up(&bx.level, FT.level);
        up(&bx.ax, FT.ax);
        up(&bx.ay, FT.ay);
        up(&bx.az, FT.az);
        up(&bx.start, FT.start);
        up(&bx.end, FT.end);
        // the points where the tree build reads the selection scan: box starts and ends
        std::vector<uint8_t> bnd((size_t)n, 0);
        for (size_t f = 0; f < FT.start.size(); ++f) {
            if (FT.start[f] < n) bnd[FT.start[f]] = 1;
            if (FT.end[f] < n) bnd[FT.end[f]] = 1;
        }
        p.d_bnd = (uint8_t *)dev_alloc(p, (size_t)n);
        PH_HIP(hipMemcpy(p.d_bnd, bnd.data(), (size_t)n, hipMemcpyHostToDevice));
        up(&bx.parent, FT.parent);
        up(&bx.child, FT.child);
        up(&bx.coll, FT.coll);
        // leaves of the full tree (no child), in box order: the rows of the learned selector
        std::vector<int32_t> leaves;
        for (size_t f = 0; f < FT.level.size(); ++f) {
            bool leaf = true;
            for (int o = 0; o < 8 && leaf; ++o) leaf = FT.child[f * 8 + o] < 0;
            if (leaf) leaves.push_back((int32_t)f);
        }
        p.n_pleaf = (int32_t)leaves.size();
        up(&p.d_pleaf, leaves);
        // the selector's per-leaf look-ups in one record each (no chains of dependent loads)
        {
            std::vector<int4> info(leaves.size()), info2(leaves.size());
            for (size_t i = 0; i < leaves.size(); ++i) {
                const int32_t f = leaves[i];
                info[i] = make_int4(f, FT.start[f], FT.end[f], 0);
                info2[i] = make_int4(FT.ax[f], FT.ay[f], FT.az[f], FT.level[f]);
            }
            upload(p, reinterpret_cast<void **>(&p.d_pinfo), info);
            upload(p, reinterpret_cast<void **>(&p.d_pinfo2), info2);
        }
        // the plan leaves by first point, and per selection tile the range of them overlapping it
        {
            std::vector<int32_t> order(leaves.size());
            for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
            std::sort(order.begin(), order.end(),
                      [&](int32_t a, int32_t b) { return FT.start[leaves[a]] < FT.start[leaves[b]]; });
            std::vector<int4> pos(order.size());
            for (size_t j = 0; j < order.size(); ++j) {
                const int32_t f = leaves[order[j]];
                pos[j] = make_int4(FT.start[f], FT.end[f], order[j], 0);
            }
            const int64_t ntile = (n + kSelTilePoints - 1) / kSelTilePoints;
            std::vector<int2> tl((size_t)std::max<int64_t>(ntile, 1), make_int2(0, 0));
            size_t j = 0;
            for (int64_t tI = 0; tI < ntile; ++tI) {
                const int64_t t0 = tI * kSelTilePoints, t1 = std::min<int64_t>(n, t0 + kSelTilePoints);
                while (j < pos.size() && pos[j].y <= t0) ++j;  // leaves ending before the tile
                size_t e = j;
                while (e < pos.size() && pos[e].x < t1) ++e;
                tl[(size_t)tI] = make_int2((int32_t)j, (int32_t)e);
            }
            upload(p, reinterpret_cast<void **>(&p.d_leaf_pos), pos);
            upload(p, reinterpret_cast<void **>(&p.d_tile_leaves), tl);
        }
        p.h_pleaf = std::move(leaves);
        // boxes by level and coordinates, for the composite translations
        const int D = (int)FT.level_cap.size() - 1;
        if (D >= 3 && D <= kCompMaxDepth) {
            std::vector<int32_t> map;
            for (int l = 0; l <= D; ++l) {
                p.boxmap_off[l] = (int64_t)map.size();
                if (l < 2) continue;
                const int64_t nside = (int64_t)1 << l;
                map.resize(map.size() + (size_t)(nside * nside * nside), -1);
            }
            for (size_t f = 0; f < FT.level.size(); ++f) {
                const int l = FT.level[f];
                if (l < 2) continue;
                const int64_t nside = (int64_t)1 << l;
                map[(size_t)(p.boxmap_off[l] + ((int64_t)FT.ax[f] * nside + FT.ay[f]) * nside + FT.az[f])] = (int32_t)f;
            }
            up(&p.d_boxmap, map);
        }
    }
    p.level_base.assign(p.level_cap.size() + 1, 0);
    for (size_t l = 0; l < p.level_cap.size(); ++l) p.level_base[l + 1] = p.level_base[l] + p.level_cap[l];
    p.box_cap = p.level_base.back();
    p.hw.resize(p.max_depth + 1);
    for (int l = 0; l <= p.max_depth; ++l) p.hw[l] = p.cube_size / std::ldexp(1.0, l + 1);
    // far-field operators
    for (int t = 0; t < kNumM2L; ++t) {  // the device offset->slot map must match the host table
        int dx, dy, dz;
        m2l_offset(t, dx, dy, dz);
        if (m2l_slot(dx, dy, dz) != t || m2l_index(dx, dy, dz) != t)
            throw Error{PH_EDEVICE, "internal: translation slot table mismatch"};
    }
    build_gas_state(p, gas);
    alloc_workspace(p);
    // timing-only events: no system-scope fence, so a mark does not write back L2 (that
    // write-back would otherwise be charged to the next phase)
    for (auto &set : p.ring)
        for (auto &e : set) PH_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    p.events_ready = true;
    // second and third streams (shared by the device's plans) and their ordering events.  The events order
    // kernels of one device only: every kernel's completion already makes its writes visible to
    // later kernels on the device, so a record needs no system-scope fence (host visibility)
    constexpr unsigned kSyncEventFlags = hipEventDisableTiming | hipEventDisableSystemFence;
    {
        SideStreams &ss = acquire_side_streams(p.device);
        p.side = ss.side;
        p.side2 = ss.side2;
    }
    PH_HIP(hipEventCreateWithFlags(&p.ev_p2m, kSyncEventFlags));
    PH_HIP(hipEventCreateWithFlags(&p.ev_m2l, kSyncEventFlags));
    PH_HIP(hipEventCreateWithFlags(&p.ev_fork, kSyncEventFlags));
    PH_HIP(hipEventCreateWithFlags(&p.ev_join, kSyncEventFlags));
    PH_HIP(hipEventCreateWithFlags(&p.ev_vt, kSyncEventFlags));
}

}  // namespace ph

using namespace ph;

extern "C" {

const char *ph_status_string(ph_status s)
{
    switch (s) {
    case PH_OK: return "ok";
    case PH_EINVAL: return "invalid argument";
    case PH_ENOMEM: return "out of memory";
    case PH_EDEVICE: return "device error";
    case PH_ENUMERIC: return "non-finite or negative source value";
    case PH_EUNSUPPORTED: return "unsupported";
    case PH_EFALLBACK: return "learned selector fell back to the threshold rule";
    }
    return "unknown status";
}

const char *ph_last_error(void) { return g_last_error.c_str(); }

void ph_options_default(ph_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = PH_FP32;
    opt->selector = PH_SEL_THRESHOLD;
    opt->method = PH_METHOD_FMM;
    opt->selector_logit_threshold = 0.0f;
}

ph_status ph_plan_create(const ph_points *pts, const ph_gas *gas, const ph_thresholds *thr,
                         const ph_options *opt, ph_plan **out)
{
    g_last_error.clear();
    if (!out) return fail(Error{PH_EINVAL, "out is null"});
    Plan *p = nullptr;
    try {
        validate(pts, gas, thr, opt);
        p = new Plan();
        create_plan(*p, pts, gas, thr, opt);
        *out = reinterpret_cast<ph_plan *>(p);
        return PH_OK;
    } catch (const Error &e) {
        free_plan(p);
        return fail(e);
    } catch (const std::bad_alloc &) {
        free_plan(p);
        return fail(Error{PH_ENOMEM, "host allocation failed"});
    }
}

void ph_plan_destroy(ph_plan *plan)
{
    if (!plan) return;
    (void)hipDeviceSynchronize();
    free_plan(reinterpret_cast<Plan *>(plan));
}

int64_t ph_plan_size(const ph_plan *plan) { return plan ? reinterpret_cast<const Plan *>(plan)->n : -1; }

static void raise_error_bits(int32_t err)
{
    if (err & 2) throw Error{PH_ENOMEM, "interaction list capacity exceeded"};
    if (err & 1) throw Error{PH_ENUMERIC, "I holds a non-finite or negative value"};
}

// the scalars of the call just enqueued on s (waits for s); raises that call's errors
static void fetch_scalars(Plan &p, hipStream_t s)
{
    PH_HIP(hipMemcpyAsync(&p.h_sc, p.d_sc, sizeof(CallScalars), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    raise_error_bits(p.h_sc.err);
}

// Phase boundaries recorded per call (events 0..9): 0 start, 1 maxima reduced,
// 2 selection flags done, 3 learned decisions and compaction done, 4 tree done, 5 lists done,
// 6 upward done, 7 downward done, 8 far field at the targets done, 9 near field (or
// direct sum) done.
// Event k of a slot: 0..7 on the caller's stream (start, then the ends of reduce, selector,
// select, tree, upward, downward, far field); 8..10 on the second stream (start of the lists,
// end of the lists, end of the near field).
static float phase_ms(Plan &p, int slot, int k)
{
    static const int from[9] = {0, 1, 2, 3, 8, 4, 5, 6, 9};
    static const int to[9] = {1, 2, 3, 4, 9, 5, 6, 7, 10};
    float ms = 0;
    if (k == 9) {  // the M2L product launches: the deepest level's (third stream) and the others'
        float a = 0, b = 0;
        PH_HIP(hipEventElapsedTime(&a, p.ring[slot][11], p.ring[slot][12]));
        PH_HIP(hipEventElapsedTime(&b, p.ring[slot][13], p.ring[slot][14]));
        return a + b;
    }
    PH_HIP(hipEventElapsedTime(&ms, p.ring[slot][from[k]], p.ring[slot][to[k]]));
    return ms;
}

static void harvest_slot(Plan &p, int slot)
{
    if (!p.ring_used[slot]) return;
    PH_HIP(hipEventSynchronize(p.ring[slot][7]));
    PH_HIP(hipEventSynchronize(p.ring[slot][10]));
    for (int k = 0; k < 10; ++k) p.phase_sum[k] += phase_ms(p, slot, k);
    p.phase_calls += 1;
    p.ring_used[slot] = false;
}

namespace {

// One evaluation's launches on s (with the plan's second and third streams joined back into s
// before the end).  timed: phase events into ring slot `slot`.  threshold_run: a learned plan's
// plain threshold-rule evaluation (source rule fallback_rel, no network), the reference of a
// validated call.
void enqueue_call(Plan &p, const void *I, const float *absE, void *S_out, hipStream_t s, bool timed, int slot,
                  bool threshold_run = false, bool same_sets = false)
{
    auto mark = [&](int k, hipStream_t on) {
        if (timed) PH_HIP(hipEventRecord(p.ring[slot][k], on));
    };
    const bool learned = p.selector == PH_SEL_LEARNED && !threshold_run;
    p.cur_I = I;  // the target kernels read the own-cell term's intensity from it
    mark(0, s);
    // |E| is read where a field rule needs it, and by the learned selector's features
    const bool need_e = p.thr.e_abs >= 0 || p.thr.e_rel >= 0;
    const float *Eu = (need_e || learned) ? absE : nullptr;
    if (same_sets) {
        // the previous call's sets, tree and lists: new strengths compacted on the old flags
        launch_reuse_begin(p, s);
        mark(1, s);
        mark(2, s);
        launch_compact(p, I, S_out, s);
        mark(3, s);
    } else {
        // the first kernel clears the call's scalars and advances the call number
        launch_reduce_max(p, I, Eu, p.d_gen, s);
        mark(1, s);
        // event 2 closes the tile pass (flags, and the learned selector's rows)
        launch_select(p, I, Eu, S_out, s, learned, threshold_run ? p.fallback_rel : -1.0,
                      timed ? p.ring[slot][2] : nullptr);
        mark(3, s);
    }
    if (p.method == PH_METHOD_DIRECT) {
        for (int k = 4; k <= 7; ++k) mark(k, s);
        mark(8, s);
        mark(9, s);
        run_direct(p, S_out, s);
        mark(10, s);
        for (int k = 11; k <= 14; ++k) mark(k, s);
        return;
    }
    if (!same_sets) build_tree(p, s);
    mark(4, s);
    // The lists and the near field run on the second stream, the V/X targets and the deepest
    // level's M2L products on the third, the upward pass and the rest of the downward pass here.
    // Every event record or wait costs the host time and leaves the stream idle for several
    // microseconds (measured: 5-9 us between two kernels, even for an event that completed long
    // before), so each wait stands for everything before its event on that stream: the M2L
    // levels here wait for the deepest level's products (which follow the V/X targets), and the
    // gathers for the near field (which follows the lists), which also orders the far-field
    // kernels after it (they add the near field into the output).  On the 128^3 grid the lists
    // and the near field end about when the coarser levels' M2L products do, so the gathers
    // lose little.  The leaf densities are enqueued here before the other streams' work, so
    // that the host reaches them early; enqueued before the fork they would delay the third
    // stream's chain (V/X targets, deepest M2L products), which sets when the coarser M2L
    // products can start (measured: 9 us more per call).
    const bool deep = p.y_all_levels && p.max_depth >= 2;
    PH_HIP(hipEventRecord(p.ev_fork, s));
    fmm_p2m(p, s);
    if (deep) PH_HIP(hipEventRecord(p.ev_p2m, s));
    PH_HIP(hipStreamWaitEvent(p.side, p.ev_fork, 0));
    PH_HIP(hipStreamWaitEvent(p.side2, p.ev_fork, 0));
    if (!same_sets) build_vtargets(p, p.side2);
    if (!deep) PH_HIP(hipEventRecord(p.ev_vt, p.side2));
    mark(8, p.side);
    if (!same_sets) build_lists(p, p.side);
    mark(9, p.side);
    fmm_near(p, p.side);
    mark(10, p.side);
    PH_HIP(hipEventRecord(p.ev_join, p.side));
    // the deepest level's M2L products on the third stream (after the leaf densities) while
    // the M2M chain runs here
    if (deep) {
        PH_HIP(hipStreamWaitEvent(p.side2, p.ev_p2m, 0));
        mark(11, p.side2);
        fmm_m2l_deepest(p, p.side2);
        mark(12, p.side2);
        PH_HIP(hipEventRecord(p.ev_m2l, p.side2));
    } else {
        mark(11, p.side2);
        mark(12, p.side2);
    }
    fmm_m2m(p, s);
    mark(5, s);
    fmm_downward(p, s, deep ? p.ev_m2l : p.ev_vt, p.ev_join, timed ? p.ring[slot][13] : nullptr,
                 timed ? p.ring[slot][14] : nullptr);
    mark(6, s);
    // far field at the targets (every leaf kernel here, after the gathers and so after the near field)
    fmm_leaf(p, S_out, s, s);
    mark(7, s);
}

}  // namespace

static ph_status evaluate_locked(Plan &p, const void *I, const float *absE, void *S_out, hipStream_t s,
                                 ph_stats *stats, bool same_sets = false);

// One call on the plan's current workspace, with the arguments checked
static ph_status evaluate_checked(ph_plan *plan, const void *I, const float *absE, void *S_out, void *stream,
                                  ph_stats *stats, void *workspace, bool use_ws)
{
    g_last_error.clear();
    if (!plan) return fail(Error{PH_EINVAL, "plan is null"});
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (!I || !S_out) return fail(Error{PH_EINVAL, "I and S_out must be device pointers"});
    const bool need_e = p.thr.e_abs >= 0 || p.thr.e_rel >= 0;
    if (need_e && !absE) return fail(Error{PH_EINVAL, "absE is required when a field rule is on"});
    if (use_ws && (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)))
        return fail(Error{PH_EINVAL, "workspace must be a 256-byte aligned device pointer"});
    std::lock_guard<std::mutex> lock(p.mu);
    if (!use_ws) {
        // the own workspace holds this call's sets once the call is enqueued
        p.sets_ready = false;
        const ph_status st = evaluate_locked(p, I, absE, S_out, reinterpret_cast<hipStream_t>(stream), stats);
        p.sets_ready = (st == PH_OK || st == PH_EFALLBACK) && p.method == PH_METHOD_FMM;
        return st;
    }
    // the per-call arrays point into the caller's workspace for this call only
    struct Restore {
        Plan &p;
        ~Restore() { layout_workspace(p, p.d_ws_own, true); }
    } restore{p};
    layout_workspace(p, static_cast<char *>(workspace), true);
    return evaluate_locked(p, I, absE, S_out, reinterpret_cast<hipStream_t>(stream), stats);
}

ph_status ph_evaluate(ph_plan *plan, const void *I, const float *absE, void *S_out, void *stream,
                      ph_stats *stats)
{
    return evaluate_checked(plan, I, absE, S_out, stream, stats, nullptr, false);
}

ph_status ph_evaluate_same_sets(ph_plan *plan, const void *I, void *S_out, void *stream, ph_stats *stats)
{
    g_last_error.clear();
    if (!plan) return fail(Error{PH_EINVAL, "plan is null"});
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (!I || !S_out) return fail(Error{PH_EINVAL, "I and S_out must be device pointers"});
    if (p.method != PH_METHOD_FMM) return fail(Error{PH_EUNSUPPORTED, "calls on the previous sets need the FMM method"});
    std::lock_guard<std::mutex> lock(p.mu);
    if (!p.sets_ready)
        return fail(Error{PH_EINVAL, "no earlier ph_evaluate on this plan's own workspace to take the sets from"});
    return evaluate_locked(p, I, nullptr, S_out, reinterpret_cast<hipStream_t>(stream), stats, true);
}

size_t ph_evaluate_workspace_bytes(const ph_plan *plan)
{
    return plan ? reinterpret_cast<const Plan *>(plan)->ws_bytes : 0;
}

ph_status ph_evaluate_ws(ph_plan *plan, const void *I, const float *absE, void *S_out, void *workspace,
                         void *stream, ph_stats *stats)
{
    return evaluate_checked(plan, I, absE, S_out, stream, stats, workspace, true);
}

static ph_status evaluate_locked(Plan &p, const void *I, const float *absE, void *S_out, hipStream_t s,
                                 ph_stats *stats, bool same_sets)
{
    const bool learned_plan = p.selector == PH_SEL_LEARNED;
    (void)learned_plan;
    try {
        PH_HIP(hipSetDevice(p.device));
        const bool timed = stats != nullptr || p.recording;
        p.count_work = stats != nullptr;
        const int slot = p.ring_pos;
        if (timed) {
            harvest_slot(p, slot);  // a slot from kRing calls ago: long finished
            p.ring_pos = (p.ring_pos + 1) % Plan::kRing;
        }
        const bool learned = p.selector == PH_SEL_LEARNED;
        const bool validated = learned && p.validate && !same_sets;
        // the side streams are shared with the other plans of the device: one call's work at a time
        std::lock_guard<std::mutex> side_lock(side_enqueue_mutex(p.device));
        if (validated) {
            // the plain FMM under the threshold rule first (into the workspace), then the
            // learned call, then the comparison that keeps one of the two
            enqueue_call(p, I, absE, p.d_sref, s, false, slot, true);
            enqueue_call(p, I, absE, S_out, s, timed, slot);
            launch_validate(p, S_out, p.d_sref, p.validate_tol, s);
        } else {
            enqueue_call(p, I, absE, S_out, s, timed, slot, false, same_sets);
        }
        PH_HIP(hipGetLastError());
        if (timed) p.ring_used[slot] = true;
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            fetch_scalars(p, s);
            stats->n_src = p.h_sc.n_src;
            stats->n_tgt = p.h_sc.n_tgt;
            int levels = 0;
            int64_t nb = 0;
            for (int l = 0; l <= p.max_depth; ++l) {
                nb += p.h_sc.lvl_count[l];
                if (p.h_sc.lvl_count[l] > 0) levels = l + 1;
            }
            stats->n_boxes = p.method == PH_METHOD_FMM ? nb : 0;
            stats->levels = levels;
            stats->fell_back = p.h_sc.fallback;
            stats->n_src_dropped =
                (learned && !p.h_sc.fallback) ? (int64_t)p.h_sc.n_src_base - p.h_sc.n_src : 0;
            stats->n_leaves = learned ? p.h_sc.n_srcleaf : 0;
            for (int k = 0; k < 12; ++k) stats->work[k] = (int64_t)p.h_sc.work[k];
            for (int k = 0; k < 10; ++k) stats->t_ms[k] = phase_ms(p, slot, k);
            stats->check_rel_l2 = validated ? p.h_sc.check_rel : -1.0;
        }
        if (stats && stats->fell_back) return PH_EFALLBACK;
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_plan_set_targets(ph_plan *plan, const uint8_t *mask, int64_t n)
{
    g_last_error.clear();
    if (!plan) return fail(Error{PH_EINVAL, "plan is null"});
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (mask && n != p.n) return fail(Error{PH_EINVAL, "target mask length must equal the number of points"});
    try {
        std::lock_guard<std::mutex> lock(p.mu);
        PH_HIP(hipSetDevice(p.device));
        PH_HIP(hipDeviceSynchronize());  // no call still reads the old set
        p.sets_ready = false;             // the next call selects again
        if (!mask) {
            dev_free(p.d_tmask);
            if (p.d_tmask) p.bytes_allocated -= (size_t)p.n;
            p.d_tmask = nullptr;
            return PH_OK;
        }
        std::vector<int32_t> perm((size_t)p.n);
        PH_HIP(hipMemcpy(perm.data(), p.d_perm, (size_t)p.n * 4, hipMemcpyDeviceToHost));
        std::vector<uint8_t> sorted((size_t)p.n);
        for (int64_t k = 0; k < p.n; ++k) sorted[k] = mask[perm[k]] ? 1 : 0;
        if (!p.d_tmask) p.d_tmask = (uint8_t *)dev_alloc(p, (size_t)p.n);
        PH_HIP(hipMemcpy(p.d_tmask, sorted.data(), (size_t)p.n, hipMemcpyHostToDevice));
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_plan_set_gas(ph_plan *plan, const ph_gas *gas, int *levels_reused)
{
    g_last_error.clear();
    if (!plan) return fail(Error{PH_EINVAL, "plan is null"});
    Plan &p = *reinterpret_cast<Plan *>(plan);
    try {
        validate_gas(gas);
        std::lock_guard<std::mutex> lock(p.mu);
        PH_HIP(hipSetDevice(p.device));
        PH_HIP(hipDeviceSynchronize());  // no call still reads the old operators
        build_gas_state(p, gas);
        PH_HIP(hipDeviceSynchronize());
        if (levels_reused) *levels_reused = p.levels_reused;
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_plan_set_graph(ph_plan *plan, int enable)
{
    g_last_error.clear();
    if (!plan) return fail(Error{PH_EINVAL, "plan is null"});
    if (enable) return fail(Error{PH_EUNSUPPORTED, "graph replay is not available in this library"});
    return PH_OK;
}

ph_status ph_phase_times(ph_plan *plan, int record, double *ms_sum, int64_t *n_calls)
{
    g_last_error.clear();
    if (!plan) return fail(Error{PH_EINVAL, "plan is null"});
    Plan &p = *reinterpret_cast<Plan *>(plan);
    try {
        PH_HIP(hipSetDevice(p.device));
        for (int k = 0; k < Plan::kRing; ++k) harvest_slot(p, k);
        if (ms_sum)
            for (int k = 0; k < PH_NPHASES; ++k) ms_sum[k] = k < 10 ? p.phase_sum[k] : 0.0;
        if (n_calls) *n_calls = p.phase_calls;
        for (double &v : p.phase_sum) v = 0.0;
        p.phase_calls = 0;
        if (record >= 0) p.recording = record != 0;
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_plan_check(ph_plan *plan, void *stream)
{
    g_last_error.clear();
    if (!plan) return fail(Error{PH_EINVAL, "plan is null"});
    Plan &p = *reinterpret_cast<Plan *>(plan);
    try {
        PH_HIP(hipSetDevice(p.device));
        // the error bits of every call since the last check, then cleared
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        int32_t sticky = 0;
        PH_HIP(hipMemcpyAsync(&sticky, p.d_sticky, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PH_HIP(hipMemsetAsync(p.d_sticky, 0, sizeof(int32_t), s));
        PH_HIP(hipStreamSynchronize(s));
        raise_error_bits(sticky);
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_debug_fetch(ph_plan *plan, int what, void *dst, int64_t cap_bytes, int64_t *n_out)
{
    g_last_error.clear();
    if (!plan || !n_out) return fail(Error{PH_EINVAL, "plan and n_out must be non-null"});
    Plan &p = *reinterpret_cast<Plan *>(plan);
    try {
        PH_HIP(hipSetDevice(p.device));
        PH_HIP(hipDeviceSynchronize());
        PH_HIP(hipMemcpy(&p.h_sc, p.d_sc, sizeof(CallScalars), hipMemcpyDeviceToHost));
        auto copy = [&](const void *src, int64_t count, size_t elem) {
            *n_out = count;
            size_t bytes = std::min<size_t>((size_t)count * elem, cap_bytes > 0 ? (size_t)cap_bytes : 0);
            if (bytes && dst) PH_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        };
        int64_t nb = 0;
        for (int l = 0; l <= p.max_depth; ++l) nb += p.h_sc.lvl_count[l];
        switch (what) {
        case 0: copy(p.d_key, p.n, 8); break;
        case 1: copy(p.d_perm, p.n, 4); break;
        case 2:
        case 3: {
            // sorted positions of the selected sources (2) or targets (3), from the flags
            std::vector<uint8_t> sel((size_t)p.n);
            PH_HIP(hipMemcpy(sel.data(), p.d_sel, (size_t)p.n, hipMemcpyDeviceToHost));
            const uint8_t bit = what == 2 ? 1 : 2;
            std::vector<int32_t> pos;
            for (int64_t k = 0; k < p.n; ++k)
                if (sel[k] & bit) pos.push_back((int32_t)k);
            *n_out = (int64_t)pos.size();
            size_t bytes = std::min<size_t>(pos.size() * 4, cap_bytes > 0 ? (size_t)cap_bytes : 0);
            if (bytes && dst) std::memcpy(dst, pos.data(), bytes);
            break;
        }
        case 4: {
            // assemble the box table level by level (levels are stored at fixed bases)
            std::vector<int32_t> tab;
            int32_t *fields[PH_BOX_FIELDS] = {p.box.level, p.box.ax, p.box.ay, p.box.az, p.box.s_first,
                                              p.box.s_cnt, p.box.t_first, p.box.t_cnt, p.box.parent,
                                              p.box.flags};
            // boxes of the per-call tree (the plan's tree pruned), level by level in Morton order
            std::vector<std::vector<int32_t>> cols(PH_BOX_FIELDS, std::vector<int32_t>(nb));
            for (int f = 0; f < PH_BOX_FIELDS; ++f)
                PH_HIP(hipMemcpy(cols[f].data(), fields[f], (size_t)nb * 4, hipMemcpyDeviceToHost));
            int64_t row = 0;
            tab.reserve((size_t)nb * PH_BOX_FIELDS);
            for (int64_t k = 0; k < nb; ++k) {
                if (!(cols[9][k] & kBoxExists)) continue;
                for (int f = 0; f < PH_BOX_FIELDS; ++f) tab.push_back(cols[f][k]);
                ++row;
            }
            *n_out = row;
            size_t bytes = std::min<size_t>(tab.size() * 4, cap_bytes > 0 ? (size_t)cap_bytes : 0);
            if (bytes && dst) std::memcpy(dst, tab.data(), bytes);
            break;
        }
        case 5: {
            std::vector<int32_t> v(p.max_depth + 2);
            for (int l = 0; l <= p.max_depth + 1; ++l) v[l] = p.h_sc.lvl_start[l];
            *n_out = (int64_t)v.size();
            size_t bytes = std::min<size_t>(v.size() * 4, cap_bytes > 0 ? (size_t)cap_bytes : 0);
            if (bytes && dst) std::memcpy(dst, v.data(), bytes);
            break;
        }
        case 6:
            *n_out = 1;
            if (dst && cap_bytes >= 8) std::memcpy(dst, &p.c_self, 8);
            break;
        case 7:
            *n_out = 1;
            if (dst && cap_bytes >= 4) std::memcpy(dst, &p.h_sc.scale_exp, 4);
            break;
        case 8:
        case 9: {
            // selector rows: the plan leaves flagged by the last selector pass, in box order
            std::vector<uint32_t> flag(p.n_pleaf);
            std::vector<float> feat((size_t)p.n_pleaf * 8);
            PH_HIP(hipMemcpy(flag.data(), p.d_leafflag, (size_t)p.n_pleaf * 4, hipMemcpyDeviceToHost));
            PH_HIP(hipMemcpy(feat.data(), p.d_feat, feat.size() * 4, hipMemcpyDeviceToHost));
            std::vector<float> rf;
            std::vector<int32_t> rb;
            for (int32_t i = 0; i < p.n_pleaf; ++i) {
                if (!flag[i]) continue;
                rb.push_back(p.h_pleaf[i]);
                rf.insert(rf.end(), feat.begin() + (size_t)i * 8, feat.begin() + (size_t)i * 8 + 8);
            }
            *n_out = (int64_t)rb.size();  // rows
            const size_t total = what == 8 ? rf.size() * 4 : rb.size() * 4;
            size_t bytes = std::min<size_t>(total, cap_bytes > 0 ? (size_t)cap_bytes : 0);
            if (bytes && dst) std::memcpy(dst, what == 8 ? (const void *)rf.data() : (const void *)rb.data(), bytes);
            break;
        }
        case 10: {
            // third strategy: per sorted point, 1 where the W list was left out (targets of leaves
            // with a W list; other entries are not defined)
            if (!p.d_rs_flag) throw Error{PH_EINVAL, "the plan has no third-strategy flags (r_s = 0)"};
            *n_out = p.n;
            const size_t bytes = std::min<size_t>((size_t)p.n, cap_bytes > 0 ? (size_t)cap_bytes : 0);
            if (bytes && dst) PH_HIP(hipMemcpy(dst, p.d_rs_flag, bytes, hipMemcpyDeviceToHost));
            break;
        }
        default: throw Error{PH_EINVAL, "unknown debug array"};
        }
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_mlp_forward(const float *params, const float *X, int64_t m, float *logits, int bf16, void *stream)
{
    g_last_error.clear();
    if (!params || !X || !logits || m < 0) return fail(Error{PH_EINVAL, "bad mlp_forward arguments"});
    try {
        launch_mlp_forward(params, X, m, nullptr, logits, bf16, reinterpret_cast<hipStream_t>(stream));
        PH_HIP(hipGetLastError());
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_mlp_backward(const float *params, const float *X, const float *y, float pos_weight, int64_t m,
                          float *grad, float *loss, void *stream)
{
    g_last_error.clear();
    if (!params || !X || !y || !grad || !loss || m < 1 || !(pos_weight > 0))
        return fail(Error{PH_EINVAL, "bad mlp_backward arguments"});
    try {
        launch_mlp_backward(params, X, y, pos_weight, m, grad, loss, reinterpret_cast<hipStream_t>(stream));
        PH_HIP(hipGetLastError());
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_mlp_backward_noalloc(const float *params, const float *X, const float *y, float pos_weight, int64_t m,
                                  float *grad, float *loss, void *stream)
{
    g_last_error.clear();
    if (!params || !X || !y || !grad || !loss || !(pos_weight > 0))
        return fail(Error{PH_EINVAL, "bad mlp_backward_noalloc arguments"});
    try {
        launch_mlp_backward_noalloc(params, X, y, pos_weight, m, grad, loss, reinterpret_cast<hipStream_t>(stream));
        PH_HIP(hipGetLastError());
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

ph_status ph_adam_step(float *params, float *m1, float *m2, const float *grad, int64_t nparam, float lr,
                       float beta1, float beta2, float eps, int64_t step, void *stream)
{
    g_last_error.clear();
    if (!params || !m1 || !m2 || !grad || nparam < 1 || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(Error{PH_EINVAL, "bad adam_step arguments"});
    try {
        launch_adam(params, m1, m2, grad, nparam, lr, beta1, beta2, eps, step, reinterpret_cast<hipStream_t>(stream));
        PH_HIP(hipGetLastError());
        return PH_OK;
    } catch (const Error &e) {
        return fail(e);
    }
}

}  // extern "C"
