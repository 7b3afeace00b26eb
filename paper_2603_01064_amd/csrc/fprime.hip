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

// The same axis transforms of n x n images as LDS-tiled batched products
// OUT_b = A_b B_b (r, c < n): element (r, k) of A at A[r sar + k sak] and
// element (k, c) of B at B[k sbk + c sbc], with per-image strides (0 for the
// shared transform matrix).  A workgroup computes a 64 x 64 output tile, each
// thread 4 x 4 of it, over K chunks of 16 staged in LDS.  apply_mask scales
// output (r, c) by the ramp sqrt(max(r, c) / n).
constexpr int kGT = 64, kGK = 16;
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ void __launch_bounds__(kBlock) k_axis_gemm(const T* __restrict__ A, const T* __restrict__ B,
                                                      T* __restrict__ out, int n, size_t a_img, size_t b_img,
                                                      int sar, int sak, int sbk, int sbc, int tiles, int apply_mask) {
    __shared__ T As[kGK][kGT + 1];
    __shared__ T Bs[kGK][kGT + 1];
    const int img = blockIdx.y;
    const int r0 = (blockIdx.x / tiles) * kGT, c0 = (blockIdx.x % tiles) * kGT;
    const T* Ab = A + (size_t)img * a_img;
    const T* Bb = B + (size_t)img * b_img;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    // FP32 on the MFMA (v_mfma_f32_16x16x4f32): wave w takes the 32 x 32
    // quarter (w >> 1, w & 1) of the tile as 2 x 2 blocks of 16 x 16; FP64 on
    // the VALU, 4 x 4 outputs per thread
    constexpr bool kMfma = std::is_same<T, float>::value;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    floatx4 macc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) macc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0;
    for (int k0 = 0; k0 < n; k0 += kGK) {
        // 64 x 16 of A and 16 x 64 of B: four elements of each per thread
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + q * kBlock;
            {
                const int r = e / kGK, k = e % kGK;
                const int gr = r0 + r, gk = k0 + k;
                As[k][r] = (gr < n && gk < n) ? Ab[(size_t)gr * sar + (size_t)gk * sak] : (T)0;
            }
            {
                const int k = e / kGT, c = e % kGT;
                const int gk = k0 + k, gc = c0 + c;
                Bs[k][c] = (gk < n && gc < n) ? Bb[(size_t)gk * sbk + (size_t)gc * sbc] : (T)0;
            }
        }
        __syncthreads();
        if constexpr (kMfma) {
            // A[m][k] = As[k][row], lane (m = lane & 15, k = lane >> 4); B[k][n] = Bs[k][col]
#pragma unroll
            for (int k4 = 0; k4 < kGK; k4 += 4) {
                const int k = k4 + (lane >> 4);
                float a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = As[k][(wave >> 1) * 32 + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 2; ++j) b[j] = Bs[k][(wave & 1) * 32 + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        macc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], macc[i][j], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int k = 0; k < kGK; ++k) {
                T a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[k][ty * 4 + i];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx * 4 + j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
            }
        }
        __syncthreads();
    }
    T* o = out + (size_t)img * n * n;
    if constexpr (kMfma) {
        // D lane: row 4 (lane >> 4) + q, column lane & 15 of each block
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = r0 + (wave >> 1) * 32 + i * 16 + 4 * (lane >> 4) + q;
                    const int c = c0 + (wave & 1) * 32 + j * 16 + (lane & 15);
                    if (r >= n || c >= n) continue;
                    T v = macc[i][j][q];
                    if (apply_mask) v *= (T)sqrt((double)(r > c ? r : c) / (double)n);
                    o[(size_t)r * n + c] = v;
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + ty * 4 + i;
        if (r >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = c0 + tx * 4 + j;
            if (c >= n) continue;
            T v = acc[i][j];
            if (apply_mask) v *= (T)sqrt((double)(r > c ? r : c) / (double)n);
            o[(size_t)r * n + c] = v;
        }
    }
}

// One axis pass of a 2D transform through k_axis_gemm:
//   row axis: out[b][i][k] = sum_j Op(k, j) in[b][i][j]
//   col axis: out[b][k][j] = sum_i Op(k, i) in[b][i][j]
// Op(k, j) = C[k][j] (forward) or C[j][k] (inverse).
template <typename T>
void axis_pass(const T* in, T* out, const T* C, int n, int batch, int col_axis, int inverse, int apply_mask,
               hipStream_t s) {
    const int tiles = (n + kGT - 1) / kGT;
    const size_t img = (size_t)n * n;
    dim3 grid((unsigned)(tiles * tiles), (unsigned)batch);
    if (!col_axis) {
        // OUT = IN M with M[j][k] = Op(k, j)
        hipLaunchKernelGGL(k_axis_gemm<T>, grid, dim3(kBlock), 0, s, in, C, out, n, img, (size_t)0, n, 1,
                           inverse ? n : 1, inverse ? 1 : n, tiles, apply_mask);
    } else {
        // OUT = Mc IN with Mc[k][i] = Op(k, i)
        hipLaunchKernelGGL(k_axis_gemm<T>, grid, dim3(kBlock), 0, s, C, in, out, n, (size_t)0, img,
                           inverse ? 1 : n, inverse ? n : 1, n, 1, tiles, apply_mask);
    }
}

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
        axis_pass<T>(h, t1, C, n, batch, 0, 0, 0, s);
        axis_pass<T>(t1, t2, C, n, batch, 1, 0, 1, s);
        axis_pass<T>(t2, t1, C, n, batch, 0, 1, 0, s);
        axis_pass<T>(t1, t2, C, n, batch, 1, 1, 0, s);
    }
    NMG_HIP(hipGetLastError());
    return launch_axpy<T>(batch, per, t2, dst, accumulate, s);
}

template <typename T>
nmg_status launch_dense_axis(const T* in, T* out, const T* C, int n, int ny, int batch, int col_axis, int inverse,
                             hipStream_t s) {
    const size_t per = (size_t)ny * n;
    if (ny == n)
        axis_pass<T>(in, out, C, n, batch, col_axis, inverse, 0, s);
    else
        hipLaunchKernelGGL(k_dense_axis<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, in, out, C, n, ny,
                           col_axis, inverse, 0);
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
