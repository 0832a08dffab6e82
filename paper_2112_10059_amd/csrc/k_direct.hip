// All-pairs evaluation of the quadrature sum (Sec. 2.4 eq. (15)) over the selected sets.
//
// Every selected target against every selected source; sources are staged
// through LDS in tiles of 256 and each lane owns one target.  FP32 sums are
// Kahan-compensated; the own-cell term and the prefactor are applied in FP64.
#include <hip/hip_runtime.h>

#include "k_common.h"

namespace ph {

namespace {

template <class T>
using V4 = typename Vec4T<T>::type;

template <class T, class TO>
__global__ __launch_bounds__(256) void direct_kernel(const V4<T> *__restrict__ s_dat, const V4<T> *__restrict__ t_dat,
                                                     const int32_t *__restrict__ t_out,
                                                     const CallScalars *__restrict__ sc, KParams<T> kp, double P,
                                                     TO *__restrict__ S_out, unsigned long long *work)
{
    __shared__ V4<T> tile[256];
    const int32_t ns = sc->n_src, nt = sc->n_tgt;
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if ((int32_t)(blockIdx.x * blockDim.x) >= nt) return;  // whole block idle
    const bool act = t < nt;
    V4<T> x;
    if (act) x = t_dat[t];
    else x.x = x.y = x.z = x.w = T(0);
    T s = 0, c = 0;
    for (int32_t base = 0; base < ns; base += 256) {
        const int m = min(256, ns - base);
        __syncthreads();
        if ((int)threadIdx.x < m) tile[threadIdx.x] = s_dat[base + threadIdx.x];
        __syncthreads();
        if (act)
            for (int j = 0; j < m; ++j) {
                const V4<T> y = tile[j];
                const T dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                const T r2 = dx * dx + dy * dy + dz * dz;
                if (r2 > T(0)) {
                    const T v = kernel_eval<true>(r2, kp) * y.w - c;
                    const T u = s + v;
                    c = (u - s) - v;
                    s = u;
                }
            }
    }
    if (work && threadIdx.x == 0) {
        const int32_t nt_here = min(256, nt - (int32_t)(blockIdx.x * blockDim.x));
        atomicAdd(&work[0], (unsigned long long)nt_here * ns);
    }
    if (act) {
        const double tot = (double)s - (double)c + (double)x.w;
        S_out[t_out[t]] = (TO)(P * ldexp(tot, sc->scale_exp));
    }
}

}  // namespace

void run_direct(Plan &p, void *S_out, hipStream_t s)
{
    // grid sized for the largest possible target count; idle blocks exit at once
    const unsigned g = (unsigned)((p.n + 255) / 256);
    if (p.precision == PH_FP64)
        direct_kernel<double, double><<<g, 256, 0, s>>>((const double4 *)p.d_s_dat, (const double4 *)p.d_t_dat,
                                                        p.d_t_out, p.d_sc, make_kparams<double>(p.gas),
                                                        p.gas.P, (double *)S_out,
                                                        p.count_work ? p.d_sc->work : nullptr);
    else
        direct_kernel<float, float><<<g, 256, 0, s>>>((const float4 *)p.d_s_dat, (const float4 *)p.d_t_dat, p.d_t_out,
                                                      p.d_sc, make_kparams<float>(p.gas), p.gas.P,
                                                      (float *)S_out,
                                                      p.count_work ? p.d_sc->work : nullptr);
}

}  // namespace ph
