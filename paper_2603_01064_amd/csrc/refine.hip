// Outer iteration in residual-driven form (Sec. 2.3 outer loop
// x^{t+1} = MG(x^t, b)): since every cycle step only sees residuals,
// MG(x, b) = x + MG(0, b - A x); the correction is computed from the
// normalised residual r/||r|| and scaled back, x += ||r|| d.  Converged
// right-hand sides get a zero input (hence a zero correction) and are left
// unchanged.
#include "nmg_internal.h"

namespace nmg {

namespace {
constexpr int kBlock = 256;

template <typename R, typename T>
__global__ void __launch_bounds__(kBlock) k_refine_scale(const R* __restrict__ r, T* __restrict__ y,
                                                         const double* __restrict__ rn2, const double* __restrict__ bn2,
                                                         double tol2, int* __restrict__ active, size_t per) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int b = blockIdx.y;
    const double q = rn2[b];
    const bool act = (q > tol2 * bn2[b]) && isfinite(q);
    if (e == 0) active[b] = act ? 1 : 0;
    if (e >= per) return;
    const double inv = act ? 1.0 / sqrt(q) : 0.0;
    y[(size_t)b * per + e] = (T)((double)r[(size_t)b * per + e] * inv);
}

template <typename X, typename T>
__global__ void __launch_bounds__(kBlock) k_refine_update(X* __restrict__ x, const T* __restrict__ d,
                                                          const double* __restrict__ rn2,
                                                          const int* __restrict__ active, size_t per) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int b = blockIdx.y;
    if (e >= per || !active[b]) return;
    const X rho = (X)sqrt(rn2[b]);
    x[(size_t)b * per + e] += rho * (X)d[(size_t)b * per + e];
}
}  // namespace

template <typename R, typename T>
nmg_status launch_refine_scale(int batch, size_t per, const R* r, T* y, const double* rn2, const double* bn2,
                               double rtol, int* active, hipStream_t s) {
    dim3 grid((unsigned)((per + kBlock - 1) / kBlock), batch);
    hipLaunchKernelGGL((k_refine_scale<R, T>), grid, dim3(kBlock), 0, s, r, y, rn2, bn2, rtol * rtol, active, per);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename X, typename T>
nmg_status launch_refine_update(int batch, size_t per, X* x, const T* d, const double* rn2, const int* active,
                                hipStream_t s) {
    dim3 grid((unsigned)((per + kBlock - 1) / kBlock), batch);
    hipLaunchKernelGGL((k_refine_update<X, T>), grid, dim3(kBlock), 0, s, x, d, rn2, active, per);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template nmg_status launch_refine_scale<double, double>(int, size_t, const double*, double*, const double*,
                                                        const double*, double, int*, hipStream_t);
template nmg_status launch_refine_scale<double, float>(int, size_t, const double*, float*, const double*,
                                                       const double*, double, int*, hipStream_t);
template nmg_status launch_refine_scale<float, float>(int, size_t, const float*, float*, const double*,
                                                      const double*, double, int*, hipStream_t);
template nmg_status launch_refine_update<double, double>(int, size_t, double*, const double*, const double*,
                                                         const int*, hipStream_t);
template nmg_status launch_refine_update<double, float>(int, size_t, double*, const float*, const double*,
                                                        const int*, hipStream_t);
template nmg_status launch_refine_update<float, float>(int, size_t, float*, const float*, const double*, const int*,
                                                       hipStream_t);

}  // namespace nmg
