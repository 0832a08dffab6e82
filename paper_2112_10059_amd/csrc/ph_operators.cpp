// Plan-time FP64 construction of the far-field operators (host side).
//
// The far field of eq. (16) is carried by artificial sources whose intensities
// are fitted so that they reproduce the true field at check points
// (Sec. 2.4 eq. (17) and the figure of artificial/check points), applied
// recursively over the octree (Sec. 2.4, last paragraph).  For the
// absorption kernel K(r) = g(r)/(4 pi r^2) of eq. (3) a single enclosing
// surface of artificial sources does not converge (K is not harmonic, so
// matching on one surface does not fix the field elsewhere).  The artificial
// sources therefore sit on a q^3 Chebyshev lattice filling the box, and the
// check points on the cube surface of half-width 3.5 h_l (q+1 points per
// edge).  The downward (local) representation is the transpose: check points
// on the lattice inside the box, artificial sources on the surface.
//
// Per level l (box half-width h_l):
//   uc2e_l = pinv(K(shell_l, lattice_l))            n_lam x n_sig (truncated SVD)
//   m2m_{l,c} = uc2e_{l-1} K(shell_{l-1}, lattice_l + off_c)   child c -> parent
//   l2l_{l,c} = m2m_{l,c}^T                          parent check values -> child
//   m2l_{l,t} = K(lattice_l, lattice_l + 2 h_l t)    316 well-separated offsets t
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "ph_internal.h"

namespace ph {

namespace {

double kernel_fp64(double r, const Gas &g)
{
    return std::exp(-g.a * r) * (-std::expm1(-(g.b - g.a) * r)) / (4.0 * M_PI * g.L * r * r * r);
}

template <class F>
void parallel_for(int n, F &&f)
{
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
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

// Threads that meet at a barrier between rounds (sense-reversing, spinning): the rounds of
// the Jacobi sweeps below are short, so threads stay alive across them.
class SpinBarrier {
public:
    explicit SpinBarrier(unsigned n) : n_(n) {}
    void wait()
    {
        const unsigned gen = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
            count_.store(0, std::memory_order_relaxed);
            gen_.fetch_add(1, std::memory_order_acq_rel);
        } else {
            while (gen_.load(std::memory_order_acquire) == gen) std::this_thread::yield();
        }
    }

private:
    const unsigned n_;
    std::atomic<unsigned> count_{0}, gen_{0};
};

// One-sided Jacobi SVD of the m x n matrix A (column-major, m >= n).
// On exit A holds U * diag(s); s the singular values; V (n x n, column-major).
// The columns are split into nb blocks (a fixed count, at most 32); each sweep runs the rounds
// of a round-robin tournament over the blocks (circle method), and in a round every pair of
// blocks rotates all pairs of its columns (in the first round also the pairs inside each of
// its two blocks), in a fixed order.  The block pairs of a round are disjoint, so they run in
// parallel, and no bit of the result depends on the number of threads.  A column pair is
// rotated when it is not yet orthogonal to 1e-16 relative; the sweeps stop when no pair
// exceeds 1e-15.
void jacobi_svd(int m, int n, std::vector<double> &A, std::vector<double> &s, std::vector<double> &V)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto rotate_pair = [&](int p, int q) -> double {
        double *ap = &A[(size_t)p * m], *aq = &A[(size_t)q * m];
        double al = 0, be = 0, ga = 0;
        for (int i = 0; i < m; ++i) {
            al += ap[i] * ap[i];
            be += aq[i] * aq[i];
            ga += ap[i] * aq[i];
        }
        if (ga == 0.0) return 0.0;
        const double rel = std::fabs(ga) / std::sqrt(al * be);
        if (!(rel > 1e-16)) return 0.0;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < m; ++i) {
            const double x = ap[i], y = aq[i];
            ap[i] = c * x - sn * y;
            aq[i] = sn * x + c * y;
        }
        double *vp = &V[(size_t)p * n], *vq = &V[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
            const double x = vp[i], y = vq[i];
            vp[i] = c * x - sn * y;
            vq[i] = sn * x + c * y;
        }
        return rel;
    };
    const int nb = std::max(2, std::min(32, n - (n & 1)));  // even block count
    auto first = [&](int b) { return (int)((int64_t)b * n / nb); };
    std::vector<int> pos(nb);
    for (int i = 0; i < nb; ++i) pos[i] = i;
    const int npair = nb / 2;
    const unsigned nt = std::max(1u, std::min({16u, std::thread::hardware_concurrency(), (unsigned)npair}));
    SpinBarrier bar(nt);
    std::vector<double> off_t(nt, 0.0);
    std::atomic<bool> done{false};
    auto worker = [&](unsigned tid) {
        for (int sweep = 0; sweep < 80; ++sweep) {
            double off = 0.0;
            for (int r = 0; r < nb - 1; ++r) {
                for (int i = (int)tid; i < npair; i += (int)nt) {
                    const int P = std::min(pos[i], pos[nb - 1 - i]), Q = std::max(pos[i], pos[nb - 1 - i]);
                    if (r == 0)
                        for (int B : {P, Q})
                            for (int p = first(B); p < first(B + 1); ++p)
                                for (int q = p + 1; q < first(B + 1); ++q) off = std::max(off, rotate_pair(p, q));
                    for (int p = first(P); p < first(P + 1); ++p)
                        for (int q = first(Q); q < first(Q + 1); ++q) off = std::max(off, rotate_pair(p, q));
                }
                bar.wait();
                if (tid == 0) {  // next round: every position but the first moves one place
                    const int last = pos[nb - 1];
                    for (int i = nb - 1; i > 1; --i) pos[i] = pos[i - 1];
                    pos[1] = last;
                }
                bar.wait();
            }
            off_t[tid] = off;
            bar.wait();
            if (tid == 0) {
                double mx = 0.0;
                for (double v : off_t) mx = std::max(mx, v);
                done.store(mx < 1e-15, std::memory_order_relaxed);
            }
            bar.wait();
            if (done.load(std::memory_order_relaxed)) break;
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(worker, t);
    worker(0);
    for (auto &x : th) x.join();
    s.resize(n);
    for (int j = 0; j < n; ++j) {
        double acc = 0;
        for (int i = 0; i < m; ++i) acc += A[(size_t)j * m + i] * A[(size_t)j * m + i];
        s[j] = std::sqrt(acc);
    }
}

// Pseudo-inverse of the m x n row-major matrix M (m >= n) by truncated SVD:
// returns the n x m row-major matrix V diag(1/s) U^T, dropping s < cut * s_max.
std::vector<double> pinv_rowmajor(int m, int n, const std::vector<double> &M, double cut)
{
    std::vector<double> A((size_t)m * n);  // column-major copy
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)j * m + i] = M[(size_t)i * n + j];
    std::vector<double> s, V;
    jacobi_svd(m, n, A, s, V);
    double smax = 0;
    for (double x : s) smax = std::max(smax, x);
    std::vector<double> P((size_t)n * m, 0.0);
    for (int k = 0; k < n; ++k) {
        if (!(s[k] > cut * smax) || s[k] == 0.0) continue;
        double inv2 = 1.0 / (s[k] * s[k]);  // A column k = U_k s_k  ->  U_k / s_k = A_k / s_k^2
        const double *ak = &A[(size_t)k * m];
        const double *vk = &V[(size_t)k * n];
        for (int r = 0; r < n; ++r) {
            double vr = vk[r] * inv2;
            if (vr == 0.0) continue;
            double *pr = &P[(size_t)r * m];
            for (int c = 0; c < m; ++c) pr[c] += vr * ak[c];
        }
    }
    return P;
}

void kernel_matrix(const std::vector<double> &X, const std::vector<double> &Y, int nx, int ny,
                   double sx, double sy, const double *shift_y, const Gas &g, std::vector<double> &out)
{
    // out[i*ny + j] = K(|sx X_i - (sy Y_j + shift)|)
    out.resize((size_t)nx * ny);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double d0 = sx * X[3 * i] - (sy * Y[3 * j] + shift_y[0]);
            double d1 = sx * X[3 * i + 1] - (sy * Y[3 * j + 1] + shift_y[1]);
            double d2 = sx * X[3 * i + 2] - (sy * Y[3 * j + 2] + shift_y[2]);
            out[(size_t)i * ny + j] = kernel_fp64(std::sqrt(d0 * d0 + d1 * d1 + d2 * d2), g);
        }
}

}  // namespace

int m2l_index(int dx, int dy, int dz)
{
    if (dx < -3 || dx > 3 || dy < -3 || dy > 3 || dz < -3 || dz > 3) return -1;
    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) return -1;
    int k = 0;
    for (int x = -3; x <= 3; ++x)
        for (int y = -3; y <= 3; ++y)
            for (int z = -3; z <= 3; ++z) {
                if (std::abs(x) <= 1 && std::abs(y) <= 1 && std::abs(z) <= 1) continue;
                if (x == dx && y == dy && z == dz) return k;
                ++k;
            }
    return -1;
}

void m2l_offset(int idx, int &dx, int &dy, int &dz)
{
    int k = 0;
    for (int x = -3; x <= 3; ++x)
        for (int y = -3; y <= 3; ++y)
            for (int z = -3; z <= 3; ++z) {
                if (std::abs(x) <= 1 && std::abs(y) <= 1 && std::abs(z) <= 1) continue;
                if (k == idx) {
                    dx = x;
                    dy = y;
                    dz = z;
                    return;
                }
                ++k;
            }
    dx = dy = dz = 0;
}

void build_operators(const Gas &gas, int q, double root_size, int max_depth, double cut, HostOperators &out,
                     OperatorCache *cache, int *reused)
{
    const double kShellRadius = 3.5;
    out.q = q;
    out.n_lam = q * q * q;
    // lattice: tensor Chebyshev nodes of the first kind on [-1,1]
    std::vector<double> t(q);
    for (int k = 0; k < q; ++k) t[k] = std::cos(M_PI * (k + 0.5) / q);
    out.lat_unit.clear();
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k) {
                out.lat_unit.push_back(t[i]);
                out.lat_unit.push_back(t[j]);
                out.lat_unit.push_back(t[k]);
            }
    // shell: boundary points of the (q+1)^3 uniform grid on [-1,1]^3, times the shell radius
    int e = q + 1;
    out.shell_unit.clear();
    for (int i = 0; i < e; ++i)
        for (int j = 0; j < e; ++j)
            for (int k = 0; k < e; ++k) {
                if (i != 0 && i != e - 1 && j != 0 && j != e - 1 && k != 0 && k != e - 1) continue;
                out.shell_unit.push_back(kShellRadius * (-1.0 + 2.0 * i / (e - 1)));
                out.shell_unit.push_back(kShellRadius * (-1.0 + 2.0 * j / (e - 1)));
                out.shell_unit.push_back(kShellRadius * (-1.0 + 2.0 * k / (e - 1)));
            }
    out.n_sig = (int)out.shell_unit.size() / 3;
    const int nl = out.n_lam, ns = out.n_sig;
    const int L = max_depth + 1;
    out.uc2e.assign(L, {});
    out.m2m.assign(L, {});
    out.m2l.assign(L, {});
    const double zero[3] = {0, 0, 0};
    std::vector<double> hwl(L);
    for (int l = 0; l < L; ++l) hwl[l] = root_size / std::ldexp(1.0, l + 1);
    // levels found in the cache (same a hw and b hw): rescaled by the power of two between the
    // half-widths, exactly
    std::vector<const CachedLevel *> hit(L, nullptr);
    std::vector<int> fexp(L, 0);  // f = 2^fexp = hw_built / hw
    int n_hit = 0;
    if (cache) {
        for (int l = 2; l < L; ++l) {
            auto it = cache->levels.find(std::make_tuple(gas.a * hwl[l], gas.b * hwl[l], gas.L));
            if (it == cache->levels.end()) continue;
            int ex = 0;
            const double fr = std::frexp(it->second.hw / hwl[l], &ex);
            if (fr != 0.5) continue;  // not a power of two (cannot happen within one root cube)
            hit[l] = &it->second;
            fexp[l] = ex - 1;
            ++n_hit;
        }
    }
    if (reused) *reused = n_hit;
    auto scaled = [](const std::vector<double> &v, int ex) {
        std::vector<double> o(v.size());
        const size_t chunk = 1 << 16, nc = (v.size() + chunk - 1) / chunk;
        parallel_for((int)nc, [&](int c) {
            const size_t e = std::min(v.size(), (c + 1) * chunk);
            for (size_t i = c * chunk; i < e; ++i) o[i] = std::ldexp(v[i], ex);
        });
        return o;
    };
    // check-to-equivalent pseudo-inverse per level (K scales by f^3, its pseudo-inverse by
    // f^-3); one level after the other, each SVD on every thread
    for (int l = 2; l < L; ++l) {
        if (hit[l]) {
            out.uc2e[l] = scaled(hit[l]->uc2e, -3 * fexp[l]);
            continue;
        }
        std::vector<double> Kmat;
        kernel_matrix(out.shell_unit, out.lat_unit, ns, nl, hwl[l], hwl[l], zero, gas, Kmat);
        out.uc2e[l] = pinv_rowmajor(ns, nl, Kmat, cut);
    }
    // child -> parent translations (child level l, parent level l-1 >= 2); dimensionless
    for (int l = 3; l < L; ++l) {
        if (hit[l] && !hit[l]->m2m.empty()) {
            out.m2m[l] = hit[l]->m2m;
            continue;
        }
        out.m2m[l].assign((size_t)8 * nl * nl, 0.0);
        parallel_for(8, [&](int c) {
            double off[3] = {(((c >> 2) & 1) ? 1.0 : -1.0) * hwl[l], (((c >> 1) & 1) ? 1.0 : -1.0) * hwl[l],
                             ((c & 1) ? 1.0 : -1.0) * hwl[l]};
            std::vector<double> Kmat;  // shell of the parent vs lattice of the child
            kernel_matrix(out.shell_unit, out.lat_unit, ns, nl, hwl[l - 1], hwl[l], off, gas, Kmat);
            const std::vector<double> &P = out.uc2e[l - 1];
            double *dst = &out.m2m[l][(size_t)c * nl * nl];
            for (int i = 0; i < nl; ++i)
                for (int k = 0; k < ns; ++k) {
                    double pik = P[(size_t)i * ns + k];
                    const double *kr = &Kmat[(size_t)k * nl];
                    for (int j = 0; j < nl; ++j) dst[(size_t)i * nl + j] += pik * kr[j];
                }
        });
    }
    // well-separated translations, pure kernel values between lattices (scale by f^3)
    for (int l = 2; l < L; ++l) {
        if (hit[l]) {
            out.m2l[l] = scaled(hit[l]->m2l, 3 * fexp[l]);
            continue;
        }
        out.m2l[l].assign((size_t)kNumM2L * nl * nl, 0.0);
        parallel_for(kNumM2L, [&](int k) {
            int dx, dy, dz;
            m2l_offset(k, dx, dy, dz);
            double sh[3] = {2.0 * hwl[l] * dx, 2.0 * hwl[l] * dy, 2.0 * hwl[l] * dz};
            std::vector<double> Kmat;
            kernel_matrix(out.lat_unit, out.lat_unit, nl, nl, hwl[l], hwl[l], sh, gas, Kmat);
            std::copy(Kmat.begin(), Kmat.end(), out.m2l[l].begin() + (size_t)k * nl * nl);
        });
    }
    // new levels into the cache, in the units of this operator set; the levels this call used
    // are the most recent, and the least recently used go first when the cache is full
    if (cache) {
        const uint64_t now = ++cache->clock;
        auto level_bytes = [](const CachedLevel &c) { return 8 * (c.uc2e.size() + c.m2l.size() + c.m2m.size()); };
        for (int l = 2; l < L; ++l) {
            auto key = std::make_tuple(gas.a * hwl[l], gas.b * hwl[l], gas.L);
            auto it = cache->levels.find(key);
            if (it == cache->levels.end()) {
                CachedLevel c;
                c.hw = hwl[l];
                c.uc2e = out.uc2e[l];
                c.m2l = out.m2l[l];
                c.m2m = out.m2m[l];
                c.stamp = now;
                cache->bytes += level_bytes(c);
                cache->levels.emplace(key, std::move(c));
            } else {
                it->second.stamp = now;
                if (it->second.m2m.empty() && !out.m2m[l].empty()) {
                    // a level first built as the coarsest gains its child -> parent translations
                    // (dimensionless, so no rescaling)
                    it->second.m2m = out.m2m[l];
                    cache->bytes += 8 * out.m2m[l].size();
                }
            }
        }
        while (cache->bytes > cache->max_bytes && !cache->levels.empty()) {
            auto old = cache->levels.begin();
            for (auto i = cache->levels.begin(); i != cache->levels.end(); ++i)
                if (i->second.stamp < old->second.stamp) old = i;
            cache->bytes -= level_bytes(old->second);
            cache->levels.erase(old);
        }
    }
}

// Near-field kernel values of a uniform grid of spacing h (Sec. 2.4, eq. (16)): two cells
// whose indices differ by (i, j, k) are h |(i, j, k)| apart, so the sum over a leaf's
// neighbours needs the kernel only at the (2R + 1)^3 integer offsets with |i|, |j|, |k| <= R.
// tab[(i + R) sx + (j + R) sy + (k + R) sz] = K(h |(i, j, k)|) in a table of n entries (the
// strides leave unused entries, 0); the origin holds 0 (a coincident pair is the own-cell
// term, handled apart).
void build_near_table(const Gas &gas, double h, int R, int sx, int sy, int sz, int n, std::vector<double> &tab)
{
    tab.assign((size_t)n, 0.0);
    for (int i = -R; i <= R; ++i)
        for (int j = -R; j <= R; ++j)
            for (int k = -R; k <= R; ++k) {
                if (i == 0 && j == 0 && k == 0) continue;
                const double r = h * std::sqrt((double)(i * i + j * j + k * k));
                tab[(size_t)(i + R) * sx + (size_t)(j + R) * sy + (size_t)(k + R) * sz] = kernel_fp64(r, gas);
            }
}

// Lattice operator of a box of m^3 grid cells (uniform cell-centred grids):
// G = uc2e_l K(shell_l, cells_l), n_lam x m^3, cell r = (i m + j) m + k at offset
// ((i + 1/2) h - hw, (j + 1/2) h - hw, (k + 1/2) h - hw) from the box centre.
// P2M of sources q on the cells is G q; the far field at the cells is G^T u, since
// uc2e_l^T is the check-to-equivalent map of the downward pass and K is symmetric.
void build_grid_operator(const Gas &gas, const HostOperators &H, int level, double hw, double h, int m,
                         std::vector<double> &G)
{
    const int nl = H.n_lam, ns = H.n_sig, R = m * m * m;
    std::vector<double> cells((size_t)R * 3);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            for (int k = 0; k < m; ++k) {
                const int r = (i * m + j) * m + k;
                cells[3 * r] = (i + 0.5) * h - hw;
                cells[3 * r + 1] = (j + 0.5) * h - hw;
                cells[3 * r + 2] = (k + 0.5) * h - hw;
            }
    const double zero[3] = {0, 0, 0};
    std::vector<double> Kmat;  // n_sig x R
    kernel_matrix(H.shell_unit, cells, ns, R, hw, 1.0, zero, gas, Kmat);
    G.assign((size_t)nl * R, 0.0);
    const std::vector<double> &U = H.uc2e[level];
    parallel_for(nl, [&](int li) {
        for (int sg = 0; sg < ns; ++sg) {
            const double u = U[(size_t)li * ns + sg];
            const double *kr = &Kmat[(size_t)sg * R];
            double *g = &G[(size_t)li * R];
            for (int r = 0; r < R; ++r) g[r] += u * kr[r];
        }
    });
}

// ------------------------------------------------------------------ own-cell coefficient

namespace {

// Exponential integral E1(x) = integral_x^inf e^-t / t dt, x >= 1.  The even part of Euler's
// continued fraction for E1,
//   e^x E1(x) = 1 / (x + 1 - 1^2 / (x + 3 - 2^2 / (x + 5 - 3^2 / (x + 7 - ...)))),
// is evaluated from a fixed depth upwards (backward recurrence); at x >= 1 its truncation
// error after 96 levels is far below double rounding.  Below 1 the power series is used
// (absorbed_within).
double expint_e1_cf(double x)
{
    constexpr int kDepth = 96;
    double den = x + 2.0 * kDepth + 1.0;
    for (int k = kDepth; k >= 1; --k) den = x + (2.0 * k - 1.0) - (double)k * (double)k / den;
    return std::exp(-x) / den;
}

// Series part of E1 without the logarithm: sum_{k>=1} (-1)^(k+1) x^k/(k k!)
double e1_series_tail(double x)
{
    double term = 1.0, sum = 0.0;
    for (int k = 1; k < 80; ++k) {
        term *= -x / k;
        double add = -term / k;
        sum += add;
        if (std::fabs(add) < 1e-18 * std::fabs(sum)) break;
    }
    return sum;
}

// Fraction of photons absorbed within radius R: integral_0^R g = 1 - (E1(aR) - E1(bR)) / L
double absorbed_within(double R, const Gas &g)
{
    double xa = g.a * R, xb = g.b * R;
    if (xb < 1.0) {
        // E1(xa) - E1(xb) = ln(b/a) + tail(xa) - tail(xb); ln(b/a) = L cancels the leading 1
        return -(e1_series_tail(xa) - e1_series_tail(xb)) / g.L;
    }
    if (xa < 1.0)  // E1(xa) from its series: -gamma - ln(xa) + tail(xa)
        return 1.0 - (-0.57721566490153286061 - std::log(xa) + e1_series_tail(xa) - expint_e1_cf(xb)) / g.L;
    return 1.0 - (expint_e1_cf(xa) - expint_e1_cf(xb)) / g.L;
}

// Legendre polynomial P_n(z) and its derivative, from the three-term recurrence
// (k + 1) P_{k+1} = (2k + 1) z P_k - k P_{k-1} and (1 - z^2) P_n' = n (P_{n-1} - z P_n).
void legendre_with_derivative(int n, double z, double &pn, double &dpn)
{
    double prev = 1.0, cur = z;  // P_0, P_1
    for (int k = 1; k < n; ++k) {
        const double next = ((2.0 * k + 1.0) * z * cur - k * prev) / (k + 1.0);
        prev = cur;
        cur = next;
    }
    pn = cur;
    dpn = n * (prev - z * cur) / (1.0 - z * z);
}

// n-point Gauss-Legendre rule on [-1, 1]: each root of P_n by Newton's method from Tricomi's
// asymptotic estimate x_k ~ (1 - 1/(8n^2) + 1/(8n^3)) cos(pi (4k - 1) / (4n + 2)); weight
// 2 / ((1 - x_k^2) P_n'(x_k)^2).  Roots come in +- pairs, so half are computed.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double nn = (double)n;
    for (int k = 1; k <= (n + 1) / 2; ++k) {
        double z = (1.0 - 1.0 / (8.0 * nn * nn) + 1.0 / (8.0 * nn * nn * nn)) * std::cos(M_PI * (4.0 * k - 1.0) / (4.0 * nn + 2.0));
        double pn = 0.0, dpn = 1.0;
        for (int it = 0; it < 50; ++it) {
            legendre_with_derivative(n, z, pn, dpn);
            const double step = pn / dpn;
            z -= step;
            if (std::fabs(step) <= 4e-16) break;
        }
        legendre_with_derivative(n, z, pn, dpn);
        const double wk = 2.0 / ((1.0 - z * z) * dpn * dpn);
        x[k - 1] = z;
        w[k - 1] = wk;
        x[n - k] = -z;
        w[n - k] = wk;
    }
}

}  // namespace

// c_self(h) = integral of K over the cube of side h centred at the evaluation point.
// Over directions the radial integral gives A(R(direction))/(4 pi); the six faces give
// (6/4pi) * integral over the face z = h/2 of A(rho) (h/2) / rho^3, computed on the
// eighth of the face 0 <= v <= u <= h/2 (times 8) with a Gauss-Legendre product rule.
double cube_self_integral(const Gas &gas, double h)
{
    std::vector<double> x, w;
    gauss_legendre(48, x, w);
    const double half = 0.5 * h;
    double acc = 0.0;
    for (int i = 0; i < 48; ++i) {
        double u = 0.5 * half * (x[i] + 1.0), wu = 0.5 * half * w[i];
        for (int j = 0; j < 48; ++j) {
            double v = 0.5 * u * (x[j] + 1.0), wv = 0.5 * u * w[j];
            double rho = std::sqrt(u * u + v * v + half * half);
            acc += wu * wv * absorbed_within(rho, gas) * half / (rho * rho * rho);
        }
    }
    return 6.0 / (4.0 * M_PI) * 8.0 * acc;
}

}  // namespace ph
