// Outer iteration in residual-driven form (Sec. 2.3 outer loop
// x^{t+1} = MG(x^t, b)): since every cycle step only sees residuals,
// MG(x, b) = x + MG(0, b - A x); the correction is computed from the
// normalised residual r/||r|| and scaled back, x += ||r|| d.  Converged
// right-hand sides get a zero input (hence a zero correction) and are left
// unchanged.
#include "nmg_internal.h"
#include "tree_sum.h"

namespace nmg {

namespace {
constexpr int kBlock = 256;

// One block per (chunk, right-hand side) with the chunks of the norm
// partials: block ch covers elements [ch len, (ch + 1) len) of the image,
// len = ceil(per / norm_chunks(per)) (the grid's x size), and with part it
// also writes the sum
// of squares of its outputs (each thread's elements in order, then a fixed
// tree), the first stage of ||y||^2 for the cycle's first BF16 smoothing
// step, in the same order as a separate partial-sum pass over y.
template <typename R, typename T>
__global__ void __launch_bounds__(kBlock) k_refine_scale(const R* __restrict__ r, T* __restrict__ y,
                                                         const double* __restrict__ rn2, const double* __restrict__ bn2,
                                                         double tol2, int* __restrict__ active, size_t per,
                                                         double* __restrict__ part) {
    __shared__ double red[kBlock];
    const int b = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
    const double q = rn2[b];
    const bool act = (q > tol2 * bn2[b]) && isfinite(q);
    if (ch == 0 && threadIdx.x == 0) active[b] = act ? 1 : 0;
    const double inv = act ? 1.0 / sqrt(q) : 0.0;
    const size_t len = (per + nch - 1) / nch;
    const size_t e0 = (size_t)ch * len, e1 = e0 + len < per ? e0 + len : per;
    const R* src = r + (size_t)b * per;
    T* dst = y + (size_t)b * per;
    double acc = 0.0;
    // (unrolled: a thread's loads are in flight together; its sum keeps its order)
#pragma unroll 8
    for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
        const T v = (T)((double)src[e] * inv);
        dst[e] = v;
        const double t = (double)v;
        acc += t * t;
    }
    if (!part) return;
    red[threadIdx.x] = acc;
    __syncthreads();
    const double tot = tree_sum<kBlock, kBlock>(red, threadIdx.x);
    if (threadIdx.x == 0) part[(size_t)b * nch + ch] = tot;
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

// Active-set compaction: moves[2m] = destination slot, moves[2m+1] = source
// slot; up to three arrays of [slots][per] move together.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_move_slots(T* __restrict__ a, T* __restrict__ b, T* __restrict__ c,
                                                       const int* __restrict__ moves, size_t per) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    const size_t dst = (size_t)moves[2 * blockIdx.y] * per + e;
    const size_t src = (size_t)moves[2 * blockIdx.y + 1] * per + e;
    a[dst] = a[src];
    if (b) b[dst] = b[src];
    if (c) c[dst] = c[src];
}

// Final iterates of finished slots: pairs[2m] = slot, pairs[2m+1] = right-hand side.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scatter_slots(const T* __restrict__ xc, double* __restrict__ x,
                                                          const int* __restrict__ pairs, size_t per) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    x[(size_t)pairs[2 * blockIdx.y + 1] * per + e] = (double)xc[(size_t)pairs[2 * blockIdx.y] * per + e];
}

// Finished iterates to their owners: dst[m] receives slot slots[m].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scatter_ptrs(const T* __restrict__ xc, double* const* __restrict__ dst,
                                                         const int* __restrict__ slots, size_t per) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    dst[blockIdx.y][e] = (double)xc[(size_t)slots[blockIdx.y] * per + e];
}

// Device wall clock (constant rate) into one slot: a profiler stamp inside graphs.
__global__ void k_stamp(long long* slot) {
    if (threadIdx.x == 0) *slot = wall_clock64();
}
}  // namespace

void launch_stamp(long long* slot, hipStream_t s) { hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, slot); }

template <typename T>
nmg_status launch_move_slots(int count, size_t per, T* a, T* b, T* c, const int* moves, hipStream_t s) {
    if (count <= 0) return NMG_OK;
    dim3 grid((unsigned)((per + kBlock - 1) / kBlock), count);
    hipLaunchKernelGGL((k_move_slots<T>), grid, dim3(kBlock), 0, s, a, b, c, moves, per);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_scatter_slots(int count, size_t per, const T* xc, double* x, const int* pairs, hipStream_t s) {
    if (count <= 0) return NMG_OK;
    dim3 grid((unsigned)((per + kBlock - 1) / kBlock), count);
    hipLaunchKernelGGL((k_scatter_slots<T>), grid, dim3(kBlock), 0, s, xc, x, pairs, per);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_scatter_ptrs(int count, size_t per, const T* xc, double* const* dst, const int* slots,
                               hipStream_t s) {
    if (count <= 0) return NMG_OK;
    dim3 grid((unsigned)((per + kBlock - 1) / kBlock), count);
    hipLaunchKernelGGL((k_scatter_ptrs<T>), grid, dim3(kBlock), 0, s, xc, dst, slots, per);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}
template nmg_status launch_scatter_ptrs<double>(int, size_t, const double*, double* const*, const int*, hipStream_t);
template nmg_status launch_scatter_ptrs<float>(int, size_t, const float*, double* const*, const int*, hipStream_t);

template nmg_status launch_move_slots<double>(int, size_t, double*, double*, double*, const int*, hipStream_t);
template nmg_status launch_move_slots<float>(int, size_t, float*, float*, float*, const int*, hipStream_t);
template nmg_status launch_scatter_slots<double>(int, size_t, const double*, double*, const int*, hipStream_t);
template nmg_status launch_scatter_slots<float>(int, size_t, const float*, double*, const int*, hipStream_t);

template <typename R, typename T>
nmg_status launch_refine_scale(int batch, size_t per, const R* r, T* y, const double* rn2, const double* bn2,
                               double rtol, int* active, hipStream_t s, double* part) {
    dim3 grid((unsigned)norm_chunks(per), batch);
    hipLaunchKernelGGL((k_refine_scale<R, T>), grid, dim3(kBlock), 0, s, r, y, rn2, bn2, rtol * rtol, active, per,
                       part);
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

// Rollout step j of the training-data generation: e[b] -= d[b] for the
// samples still rolling out (j < k[b]); the others keep their error.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rollout_sub(T* __restrict__ e, const T* __restrict__ d,
                                                        const int* __restrict__ k, int j, size_t per) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= per || j >= k[b]) return;
    e[(size_t)b * per + i] -= d[(size_t)b * per + i];
}

template <typename T>
nmg_status launch_rollout_sub(int batch, size_t per, T* e, const T* d, const int* k, int j, hipStream_t s) {
    dim3 grid((unsigned)((per + kBlock - 1) / kBlock), batch);
    hipLaunchKernelGGL((k_rollout_sub<T>), grid, dim3(kBlock), 0, s, e, d, k, j, per);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}
template nmg_status launch_rollout_sub<double>(int, size_t, double*, const double*, const int*, int, hipStream_t);
template nmg_status launch_rollout_sub<float>(int, size_t, float*, const float*, const int*, int, hipStream_t);

template nmg_status launch_refine_scale<double, double>(int, size_t, const double*, double*, const double*,
                                                        const double*, double, int*, hipStream_t, double*);
template nmg_status launch_refine_scale<double, float>(int, size_t, const double*, float*, const double*,
                                                       const double*, double, int*, hipStream_t, double*);
template nmg_status launch_refine_scale<float, float>(int, size_t, const float*, float*, const double*,
                                                      const double*, double, int*, hipStream_t, double*);
template nmg_status launch_refine_update<double, double>(int, size_t, double*, const double*, const double*,
                                                         const int*, hipStream_t);
template nmg_status launch_refine_update<double, float>(int, size_t, double*, const float*, const double*,
                                                        const int*, hipStream_t);
template nmg_status launch_refine_update<float, float>(int, size_t, float*, const float*, const double*, const int*,
                                                       hipStream_t);

}  // namespace nmg
