/*
 * FP64 direct quadrature of the photoionization sum (oracle, test infrastructure only).
 *
 * Lin & Zhuang, Sec. 2.4 eq. (15): S(x_i) = sum_j G(x_i, y_j) I_h(y_j), with the
 * discrete kernel read as G(x_i, y_j) I_h(y_j) = w_j I_j K(|x_i - y_j|) for i != j,
 * K(r) = g(r) / (4 pi r^2) from eqs. (1) and (3), and the own-cell term c_self * I_i
 * when the target is itself a selected source (I constant over the own cell).
 * Pairs with r == 0 between distinct points are excluded (point clouds).
 *
 * Every target is summed over every selected source in fixed source order with
 * Neumaier-compensated FP64 accumulation.  OpenMP parallelises over targets only,
 * so the result does not depend on the thread count.
 *
 * This file shares nothing with the GPU library and is built on its own by gcc.
 */
#include <math.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline double kernel_K(double r, double a, double b, double four_pi_L)
{
    /* exp(-a r) - exp(-b r) written without cancellation */
    return exp(-a * r) * (-expm1(-(b - a) * r)) / (four_pi_L * r * r * r);
}

/*
 * src_xyz: ns x 3 (cm); src_q: ns weights w_j * I_j; src_id: ns point identifiers
 * tgt_xyz: nt x 3;       tgt_id: nt identifiers;   tgt_self: nt values c_self * I_i
 *          for targets that are selected sources (0 otherwise)
 * out: nt values  P * (sum_{j: id_j != id_i, r > 0} q_j K(r_ij) + tgt_self_i)
 * Returns the number of OpenMP threads used.
 */
int oracle_direct_sum(int64_t ns, const double *src_xyz, const double *src_q, const int64_t *src_id,
                      int64_t nt, const double *tgt_xyz, const int64_t *tgt_id, const double *tgt_self,
                      double a, double b, double L, double P, int nthreads, double *out)
{
    const double four_pi_L = 4.0 * M_PI * L;
    int used = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < nt; ++i) {
        const double xi = tgt_xyz[3 * i], yi = tgt_xyz[3 * i + 1], zi = tgt_xyz[3 * i + 2];
        const int64_t id = tgt_id[i];
        double s = 0.0, c = 0.0;        /* Neumaier sum and its compensation */
        for (int64_t j = 0; j < ns; ++j) {
            if (src_id[j] == id) continue;
            const double dx = xi - src_xyz[3 * j];
            const double dy = yi - src_xyz[3 * j + 1];
            const double dz = zi - src_xyz[3 * j + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0) continue;
            const double t = src_q[j] * kernel_K(r, a, b, four_pi_L);
            const double u = s + t;
            if (fabs(s) >= fabs(t)) c += (s - u) + t;
            else c += (t - u) + s;
            s = u;
        }
        out[i] = P * ((s + c) + tgt_self[i]);
    }
    return used;
}
