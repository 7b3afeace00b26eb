// Coarsest-grid direct solve in FP64 (Algorithm 1, l = L: x_L = A_L^{-1} y_L).
//
// Per right-hand-side slot the dense matrix
//   A_L = alpha M_L (x) M_L + G_L (x) G_L   (1D: alpha M_L + G_L)
// is assembled from the dense Galerkin factors and factored by Cholesky,
// A_L = L L^T.  The FP64 cycle then performs the forward and back
// substitutions (one workgroup per slot; the factor is stored twice, L and
// L^T row-major, so both sweeps read contiguous rows).  FP32 and mixed
// cycles instead apply the FP64 inverse L^{-T} L^{-1}, formed once per
// factorisation, as a batched matrix-vector product: the substitutions are
// 2 n_L^2 dependent steps per cycle, the product has no serial chain.
#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kBlock = 256;

// Block k factors cache slot slots[k] for alpha alphas[k]; flags[k] reports
// a non-positive or non-finite pivot.
__global__ void __launch_bounds__(kBlock) k_cholesky(const double* __restrict__ Mc, const double* __restrict__ Gc,
                                                     const double* __restrict__ alphas, const int* __restrict__ slots,
                                                     double* __restrict__ chol, double* __restrict__ cholT,
                                                     int* __restrict__ flags, int nl, int two_d) {
    const int k_ = blockIdx.x;
    const int b = slots[k_];
    const int N = two_d ? nl * nl : nl;
    double* A = chol + (size_t)b * N * N;
    const double a = alphas[k_];
    for (int e = threadIdx.x; e < N * N; e += kBlock) {
        const int r = e / N, c = e % N;
        double v;
        if (two_d) {
            const int i1 = r / nl, j1 = r % nl, i2 = c / nl, j2 = c % nl;
            v = a * Mc[i1 * nl + i2] * Mc[j1 * nl + j2] + Gc[i1 * nl + i2] * Gc[j1 * nl + j2];
        } else {
            v = a * Mc[r * nl + c] + Gc[r * nl + c];
        }
        A[e] = v;
    }
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        if (threadIdx.x == 0) {
            double d = A[(size_t)k * N + k];
            if (!(d > 0.0) || !isfinite(d)) {
                bad = 1;
                d = 1.0;
            }
            A[(size_t)k * N + k] = sqrt(d);
        }
        __syncthreads();
        const double piv = A[(size_t)k * N + k];
        for (int i = k + 1 + threadIdx.x; i < N; i += kBlock) A[(size_t)i * N + k] /= piv;
        __syncthreads();
        const int m = N - k - 1;
        for (int e = threadIdx.x; e < m * m; e += kBlock) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j <= i) A[(size_t)i * N + j] -= A[(size_t)i * N + k] * A[(size_t)j * N + k];
        }
        __syncthreads();
    }
    double* AT = cholT + (size_t)b * N * N;
    for (int e = threadIdx.x; e < N * N; e += kBlock) {
        const int r = e / N, c = e % N;
        if (c > r) A[e] = 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += kBlock) {
        const int r = e / N, c = e % N;
        AT[(size_t)c * N + r] = A[e];
    }
    if (threadIdx.x == 0) flags[k_] = bad;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_solve(const double* __restrict__ chol,
                                                         const double* __restrict__ cholT, const int* __restrict__ fidx,
                                                         const T* __restrict__ y, T* __restrict__ x, int N) {
    extern __shared__ double z[];
    const int b = blockIdx.x;
    const double* Lr = chol + (size_t)fidx[b] * N * N;
    const double* Lt = cholT + (size_t)fidx[b] * N * N;
    for (int i = threadIdx.x; i < N; i += kBlock) z[i] = (double)y[(size_t)b * N + i];
    __syncthreads();
    // forward: L z = y, column-oriented (column j of L is row j of L^T)
    for (int j = 0; j < N; ++j) {
        if (threadIdx.x == 0) z[j] /= Lr[(size_t)j * N + j];
        __syncthreads();
        const double zj = z[j];
        for (int i = j + 1 + threadIdx.x; i < N; i += kBlock) z[i] -= Lt[(size_t)j * N + i] * zj;
        __syncthreads();
    }
    // backward: L^T x = z, column j of L^T is row j of L
    for (int j = N - 1; j >= 0; --j) {
        if (threadIdx.x == 0) z[j] /= Lr[(size_t)j * N + j];
        __syncthreads();
        const double xj = z[j];
        for (int i = threadIdx.x; i < j; i += kBlock) z[i] -= Lr[(size_t)j * N + i] * xj;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < N; i += kBlock) x[(size_t)b * N + i] = (T)z[i];
}

// W = L^{-1} by forward substitution on the identity, one column per thread
// (column c of W lives in W[.][c], so a row of W is read coalesced).
__global__ void __launch_bounds__(kBlock) k_lower_inverse(const double* __restrict__ chol, double* __restrict__ W,
                                                          const int* __restrict__ slots, int N) {
    const int b = slots[blockIdx.x];
    const double* Lr = chol + (size_t)b * N * N;
    double* Wb = W + (size_t)b * N * N;
    for (int c = threadIdx.x; c < N; c += kBlock) {
        for (int j = 0; j < N; ++j) {
            double acc = (j == c) ? 1.0 : 0.0;
            for (int k = c; k < j; ++k) acc -= Lr[(size_t)j * N + k] * Wb[(size_t)k * N + c];
            Wb[(size_t)j * N + c] = (j < c) ? 0.0 : acc / Lr[(size_t)j * N + j];
        }
    }
}

// Ainv = W^T W (symmetric), Ainv[i][j] = sum_{k >= max(i,j)} W[k][i] W[k][j].
__global__ void __launch_bounds__(kBlock) k_gram(const double* __restrict__ W, double* __restrict__ Ainv,
                                                 const int* __restrict__ slots, int N) {
    const int b = slots[blockIdx.y];
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= N * N) return;
    const int i = e / N, j = e % N;
    const double* Wb = W + (size_t)b * N * N;
    double acc = 0.0;
    for (int k = i > j ? i : j; k < N; ++k) acc += Wb[(size_t)k * N + i] * Wb[(size_t)k * N + j];
    Ainv[(size_t)b * N * N + e] = acc;
}

// x = Ainv y per right-hand side; Ainv is symmetric, so thread i reads column
// i (contiguous across threads for each k).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_inverse_apply(const double* __restrict__ Ainv, const int* __restrict__ fidx,
                                                          const T* __restrict__ y, T* __restrict__ x, int N) {
    extern __shared__ double yv[];
    const int b = blockIdx.x;
    for (int i = threadIdx.x; i < N; i += kBlock) yv[i] = (double)y[(size_t)b * N + i];
    __syncthreads();
    const double* A = Ainv + (size_t)fidx[b] * N * N;
    for (int i = threadIdx.x; i < N; i += kBlock) {
        double acc = 0.0;
        for (int k = 0; k < N; ++k) acc += A[(size_t)k * N + i] * yv[k];
        x[(size_t)b * N + i] = (T)acc;
    }
}

}  // namespace

nmg_status launch_coarse_inverse(Ctx* c, int count, const int* slots, hipStream_t s) {
    const int N = c->nc;
    hipLaunchKernelGGL(k_lower_inverse, dim3(count), dim3(kBlock), 0, s, c->chol, c->cwork, slots, N);
    hipLaunchKernelGGL(k_gram, dim3((N * N + kBlock - 1) / kBlock, count), dim3(kBlock), 0, s, c->cwork, c->cinv,
                       slots, N);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_coarse_apply_inverse(const Ctx* c, int batch, const T* y, T* x, hipStream_t s) {
    const int N = c->nc;
    hipLaunchKernelGGL(k_inverse_apply<T>, dim3(batch), dim3(kBlock), N * sizeof(double), s, c->cinv,
                       c->cycle_fidx ? c->cycle_fidx : c->coarse_idx,
                       y, x, N);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}
template nmg_status launch_coarse_apply_inverse<float>(const Ctx*, int, const float*, float*, hipStream_t);
template nmg_status launch_coarse_apply_inverse<double>(const Ctx*, int, const double*, double*, hipStream_t);

nmg_status launch_coarse_factor(Ctx* c, int count, const double* alphas, const int* slots, hipStream_t s) {
    const int nl = c->n[c->L - 1];
    hipLaunchKernelGGL(k_cholesky, dim3(count), dim3(kBlock), 0, s, c->Mc, c->Gc, alphas, slots, c->chol, c->cholT,
                       c->flags, nl, c->p.dim == 2 ? 1 : 0);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_coarse_solve(const Ctx* c, int batch, const T* y, T* x, hipStream_t s) {
    const int N = c->nc;
    hipLaunchKernelGGL(k_coarse_solve<T>, dim3(batch), dim3(kBlock), N * sizeof(double), s, c->chol, c->cholT,
                       c->cycle_fidx ? c->cycle_fidx : c->coarse_idx, y, x, N);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template nmg_status launch_coarse_solve<float>(const Ctx*, int, const float*, float*, hipStream_t);
template nmg_status launch_coarse_solve<double>(const Ctx*, int, const double*, double*, hipStream_t);

}  // namespace nmg
