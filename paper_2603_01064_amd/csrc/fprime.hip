// Frequency filter F'_l on the level grid (Algorithms 3 and 4):
//   F'_l(h) = C^T (m'_l .* (C h C^T)) C      (2D; 1D: C^T (m'_l .* (C h)))
// with C the orthonormal DCT-II of the level size n (frequencies pi k / n)
// and the ramp m'_l = sqrt(max(k1, k2) / n) over the range visible on the
// level (Sec. 3.2 / 3.3 mask m_l sampled on the level grid).  Evaluated as
// dense axis passes in the cycle's precision.
#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kBlock = 256;

// Row axis : out[b][i][k] = sum_j Op(k, j) in[b][i][j]
// Col axis : out[b][k][j] = sum_i Op(k, i) in[b][i][j]
// Op(k, j) = C[k][j] (forward) or C[j][k] (inverse).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dense_axis(const T* __restrict__ in, T* __restrict__ out,
                                                       const T* __restrict__ C, int n, int ny, int col_axis,
                                                       int inverse, int apply_mask) {
    const size_t per = (size_t)ny * n;
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    const int b = blockIdx.y;
    const int i = (int)(e / n), j = (int)(e % n);
    const T* src = in + (size_t)b * per;
    T acc = 0;
    if (!col_axis) {
        const T* row = src + (size_t)i * n;
        for (int q = 0; q < n; ++q) acc += (inverse ? C[(size_t)q * n + j] : C[(size_t)j * n + q]) * row[q];
    } else {
        for (int q = 0; q < n; ++q) acc += (inverse ? C[(size_t)q * n + i] : C[(size_t)i * n + q]) * src[(size_t)q * n + j];
    }
    if (apply_mask) {
        const int kmax = ny == 1 ? j : max(i, j);
        acc *= (T)sqrt((double)kmax / (double)n);
    }
    out[(size_t)b * per + e] = acc;
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

template <typename T>
nmg_status launch_fprime(const Ctx* c, int l, int batch, const T* h, T* dst, int accumulate, Work<T>& w,
                         hipStream_t s) {
    const int n = c->n[l];
    const int ny = c->p.dim == 2 ? n : 1;
    const size_t per = (size_t)ny * n;
    const T* C = w.dct + w.dct_off[l];
    T* t1 = w.lv[l].t1;
    T* t2 = w.lv[l].t2;
    dim3 grid(blocks_for(per), batch);
    if (ny == 1) {
        hipLaunchKernelGGL(k_dense_axis<T>, grid, dim3(kBlock), 0, s, h, t1, C, n, ny, 0, 0, 1);
        hipLaunchKernelGGL(k_dense_axis<T>, grid, dim3(kBlock), 0, s, t1, t2, C, n, ny, 0, 1, 0);
    } else {
        hipLaunchKernelGGL(k_dense_axis<T>, grid, dim3(kBlock), 0, s, h, t1, C, n, ny, 0, 0, 0);
        hipLaunchKernelGGL(k_dense_axis<T>, grid, dim3(kBlock), 0, s, t1, t2, C, n, ny, 1, 0, 1);
        hipLaunchKernelGGL(k_dense_axis<T>, grid, dim3(kBlock), 0, s, t2, t1, C, n, ny, 0, 1, 0);
        hipLaunchKernelGGL(k_dense_axis<T>, grid, dim3(kBlock), 0, s, t1, t2, C, n, ny, 1, 1, 0);
    }
    NMG_HIP(hipGetLastError());
    return launch_axpy<T>(batch, per, t2, dst, accumulate, s);
}

template <typename T>
nmg_status launch_dense_axis(const T* in, T* out, const T* C, int n, int ny, int batch, int col_axis, int inverse,
                             hipStream_t s) {
    const size_t per = (size_t)ny * n;
    hipLaunchKernelGGL(k_dense_axis<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, in, out, C, n, ny, col_axis,
                       inverse, 0);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}
template nmg_status launch_dense_axis<float>(const float*, float*, const float*, int, int, int, int, int, hipStream_t);
template nmg_status launch_dense_axis<double>(const double*, double*, const double*, int, int, int, int, int,
                                              hipStream_t);

template nmg_status launch_fprime<float>(const Ctx*, int, int, const float*, float*, int, Work<float>&, hipStream_t);
template nmg_status launch_fprime<double>(const Ctx*, int, int, const double*, double*, int, Work<double>&,
                                          hipStream_t);

}  // namespace nmg
