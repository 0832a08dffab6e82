// Host-side checks of libph built with the address and undefined-behaviour sanitizers on the
// host code.  Runs without a GPU: every path here stops before the first device call or never
// makes one.  Prints one line per check and exits non-zero on the first failed expectation.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2112_10059_amd/csrc/ph_internal.h"
#include "../../paper_2112_10059_amd/csrc/k_common.h"

static int g_fail = 0;
#define EXPECT(cond, what)                                                     \
    do {                                                                       \
        if (!(cond)) {                                                         \
            std::printf("FAIL %s (%s:%d)\n", what, __FILE__, __LINE__);        \
            g_fail = 1;                                                        \
        } else {                                                               \
            std::printf("ok   %s\n", what);                                    \
        }                                                                      \
    } while (0)

static ph::Gas gas760()
{
    // 760 Torr air: pO2 = 152 Torr, chi_min = 0.035, chi_max = 2 (cm Torr)^-1
    ph::Gas g{};
    g.a = 0.035 * 152.0;
    g.b = 2.0 * 152.0;
    g.L = std::log(2.0 / 0.035);
    g.P = 30.0 / 790.0 * 0.06;
    return g;
}

static void check_validation()
{
    std::vector<double> xyz = {0.1, 0.1, 0.1, 0.2, 0.2, 0.2, 0.3, 0.3, 0.3, 0.4, 0.4, 0.4};
    ph_points pts{};
    pts.n = 4;
    pts.xyz = xyz.data();
    pts.h = 0.1;
    pts.self_coeff = NAN;
    pts.cube_size = 0.0;
    ph_gas gas{760.0, 0.2, 30.0, 0.06, 0.035, 2.0};
    ph_thresholds thr{1e-4, -1.0, 0.0, -1.0, 0.0};
    ph_options opt;
    ph_options_default(&opt);
    ph_plan *plan = nullptr;
    EXPECT(ph_plan_create(nullptr, &gas, &thr, &opt, &plan) == PH_EINVAL && !plan, "null points rejected");
    ph_thresholds bad = thr;
    bad.src_rel = 2.0;
    EXPECT(ph_plan_create(&pts, &gas, &bad, &opt, &plan) == PH_EINVAL && std::strstr(ph_last_error(), "src_rel"),
           "src_rel out of range rejected");
    ph_gas badg = gas;
    badg.chi_min = 5.0;
    EXPECT(ph_plan_create(&pts, &badg, &thr, &opt, &plan) == PH_EINVAL, "chi_min > chi_max rejected");
    std::vector<double> xyz2 = xyz;
    xyz2[4] = NAN;
    ph_points p2 = pts;
    p2.xyz = xyz2.data();
    EXPECT(ph_plan_create(&p2, &gas, &thr, &opt, &plan) == PH_EINVAL, "non-finite coordinate rejected");
    ph_options o2 = opt;
    o2.selector = PH_SEL_LEARNED;
    EXPECT(ph_plan_create(&pts, &gas, &thr, &o2, &plan) == PH_EINVAL, "learned selector without weights rejected");
    // a valid request stops at the first device call on a machine without a GPU, and the
    // partial plan is released (the sanitizers watch that teardown)
    const ph_status s = ph_plan_create(&pts, &gas, &thr, &opt, &plan);
    EXPECT(s != PH_OK || plan != nullptr, "valid request either builds a plan or reports a device error");
    if (plan) ph_plan_destroy(plan);
    ph_plan_destroy(nullptr);
    EXPECT(ph_plan_size(nullptr) == -1, "size of a null plan");
    for (int k = 0; k <= 7; ++k) EXPECT(ph_status_string((ph_status)k) != nullptr, "status string");
}

static void check_own_cell()
{
    const ph::Gas g = gas760();
    // integral of K over the cube of side h: values from an independent quadrature
    EXPECT(std::fabs(ph::cube_self_integral(g, 0.2 / 24) - 0.2660797372) < 2e-10, "c_self(1/120 cm)");
    EXPECT(std::fabs(ph::cube_self_integral(g, 1.0 / 128) - 0.2541680820) < 2e-10, "c_self(1/128 cm)");
    EXPECT(std::fabs(ph::cube_self_integral(g, 10.0) - 1.0) < 1e-10, "c_self of a huge cell is 1");
}

static void check_operators()
{
    const ph::Gas g = gas760();
    for (int q : {3, 4}) {
        ph::HostOperators H;
        ph::build_operators(g, q, 1.0, 4, 1e-7, H);
        bool finite = true;
        for (int l = 2; l <= 4; ++l) {
            for (double v : H.uc2e[l]) finite = finite && std::isfinite(v);
            for (double v : H.m2l[l]) finite = finite && std::isfinite(v);
            if (l >= 3)
                for (double v : H.m2m[l]) finite = finite && std::isfinite(v);
        }
        EXPECT(H.n_lam == q * q * q && H.n_sig == 6 * q * q + 2, "operator sizes");
        EXPECT(finite, "operators finite");
        EXPECT(H.uc2e[4].size() == (size_t)H.n_lam * H.n_sig && H.m2l[3].size() == (size_t)316 * H.n_lam * H.n_lam,
               "operator shapes");
        std::vector<double> G;
        ph::build_grid_operator(g, H, 3, 1.0 / 16, 1.0 / 32, 4, G);
        EXPECT(G.size() == (size_t)H.n_lam * 64, "grid operator shape");
    }
    std::vector<double> tab;
    ph::build_near_table(g, 1.0 / 128, 7, 16, 1, 16 * 15, 15 * 16 * 15, tab);
    EXPECT(tab.size() == (size_t)15 * 16 * 15 && tab[7 * 16 + 7 + 7 * 240] == 0.0, "near table origin is 0");
    int bad = 0;
    for (int t = 0; t < 316; ++t) {
        int dx, dy, dz;
        ph::m2l_offset(t, dx, dy, dz);
        bad += ph::m2l_index(dx, dy, dz) != t || ph::m2l_slot(dx, dy, dz) != t;
    }
    EXPECT(bad == 0, "316 well-separated offsets round-trip");
}

// Operators rescaled from the cache (another pressure, the same a hw and b hw at another level)
// equal a fresh build bit for bit: the kernel scales by an exact power of two.
static void check_operator_cache()
{
    auto at = [](double p_torr) {
        ph::Gas g{};
        g.a = 0.035 * (0.2 * p_torr);
        g.b = 2.0 * (0.2 * p_torr);
        g.L = std::log(2.0 / 0.035);
        g.P = 30.0 / (p_torr + 30.0) * 0.06;
        return g;
    };
    auto same = [](const std::vector<double> &x, const std::vector<double> &y) {
        return x.size() == y.size() && (x.empty() || std::memcmp(x.data(), y.data(), x.size() * 8) == 0);
    };
    const int q = 3, depth = 5;
    ph::OperatorCache cache;
    ph::HostOperators H0, H1, F1, H2, F2;
    int r0 = -1, r1 = -1, r2 = -1;
    ph::build_operators(at(400.0), q, 1.0, depth, 1e-7, H0, &cache, &r0);
    EXPECT(r0 == 0, "first build takes nothing from the cache");
    ph::build_operators(at(800.0), q, 1.0, depth, 1e-7, H1, &cache, &r1);
    ph::build_operators(at(800.0), q, 1.0, depth, 1e-7, F1);
    EXPECT(r1 == depth - 2, "doubled pressure: every level but the coarsest from the cache");
    ph::build_operators(at(200.0), q, 1.0, depth, 1e-7, H2, &cache, &r2);
    ph::build_operators(at(200.0), q, 1.0, depth, 1e-7, F2);
    EXPECT(r2 == depth - 2, "halved pressure: every level but the finest from the cache");
    bool eq1 = true, eq2 = true;
    for (int l = 2; l <= depth; ++l) {
        eq1 = eq1 && same(H1.uc2e[l], F1.uc2e[l]) && same(H1.m2l[l], F1.m2l[l]) && same(H1.m2m[l], F1.m2m[l]);
        eq2 = eq2 && same(H2.uc2e[l], F2.uc2e[l]) && same(H2.m2l[l], F2.m2l[l]) && same(H2.m2m[l], F2.m2m[l]);
    }
    EXPECT(eq1, "doubled pressure: rescaled operators equal a fresh build bit for bit");
    EXPECT(eq2, "halved pressure: rescaled operators equal a fresh build bit for bit");
    // a pressure ratio that is not a power of two shares nothing
    int r3 = -1;
    ph::HostOperators H3;
    ph::build_operators(at(760.0), q, 1.0, depth, 1e-7, H3, &cache, &r3);
    EXPECT(r3 == 0, "760 Torr after 200/400/800 Torr: no level in common");
}

static void check_full_tree()
{
    std::mt19937_64 rng(7);
    for (int n : {1, 2, 65, 5000}) {
        std::vector<uint64_t> keys(n);
        for (auto &k : keys) k = rng() >> 1;  // 63-bit keys
        if (n > 100)
            for (int i = 10; i < 40; ++i) keys[i] = keys[9];  // duplicates
        std::sort(keys.begin(), keys.end());
        ph::FullTree T;
        ph::build_full_tree(keys, 16, 16, T);
        const size_t nb = T.level.size();
        bool ok = T.start[0] == 0 && T.end[0] == n && T.child.size() == nb * 8 && T.coll.size() == nb * 27;
        for (size_t b = 0; b < nb && ok; ++b) {
            int64_t covered = 0, nch = 0;
            for (int o = 0; o < 8; ++o) {
                const int32_t c = T.child[b * 8 + o];
                if (c < 0) continue;
                ++nch;
                ok = ok && T.parent[c] == (int32_t)b && T.level[c] == T.level[b] + 1 && T.start[c] >= T.start[b] &&
                     T.end[c] <= T.end[b];
                covered += T.end[c] - T.start[c];
            }
            if (nch) ok = ok && covered == T.end[b] - T.start[b];
            else ok = ok && (T.end[b] - T.start[b] <= 16 || T.level[b] == 16);
            ok = ok && T.coll[b * 27 + 13] == (int32_t)b;
            for (int d = 0; d < 27 && ok; ++d) {
                const int32_t c = T.coll[b * 27 + d];
                if (c >= 0) ok = T.coll[(size_t)c * 27 + (26 - d)] == (int32_t)b && T.level[c] == T.level[b];
            }
        }
        EXPECT(ok, "plan tree: children partition their parent, leaves hold at most 16 points, colleagues symmetric");
    }
}

static void check_clamp()
{
    uint2 r = ph::clamp_range(10, 5, 100);
    EXPECT(r.x == 10 && r.y == 15, "range inside the capacity");
    r = ph::clamp_range(98, 5, 100);
    EXPECT(r.x == 98 && r.y == 100, "range cut at the capacity");
    r = ph::clamp_range(150, 5, 100);
    EXPECT(r.x == 100 && r.y == 100, "range past the capacity is empty");
    r = ph::clamp_range(0xfffffff0u, 0x20u, 100);
    EXPECT(r.x == 100 && r.y == 100, "no 32-bit wrap");
}

int main()
{
    check_validation();
    check_own_cell();
    check_operator_cache();
    check_operators();
    check_full_tree();
    check_clamp();
    std::printf(g_fail ? "host checks FAILED\n" : "host checks passed\n");
    return g_fail;
}
