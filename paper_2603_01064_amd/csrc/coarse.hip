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

// x = Ainv y per right-hand side; Ainv is symmetric, so output i reads
// column i (contiguous across threads for each k).  A workgroup takes 32
// outputs of one right-hand side and splits the sum over k into 8 slices of
// consecutive k (one per wave half), added in slice order: 8x shorter
// dependent chains and N/32 workgroups per right-hand side.
constexpr int kInvOut = 32, kInvSlices = kBlock / kInvOut;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_inverse_apply(const double* __restrict__ Ainv, const int* __restrict__ fidx,
                                                          const T* __restrict__ y, T* __restrict__ x, int N) {
    extern __shared__ double yv[];  // N values of y, then kBlock partial sums
    double* red = yv + N;
    const int b = blockIdx.y;
    for (int i = threadIdx.x; i < N; i += kBlock) yv[i] = (double)y[(size_t)b * N + i];
    __syncthreads();
    const double* A = Ainv + (size_t)fidx[b] * N * N;
    const int io = threadIdx.x % kInvOut, ks = threadIdx.x / kInvOut;
    const int i = blockIdx.x * kInvOut + io;
    const int len = (N + kInvSlices - 1) / kInvSlices, k0 = ks * len, k1 = min(N, k0 + len);
    double acc = 0.0;
    if (i < N)
        for (int k = k0; k < k1; ++k) acc += A[(size_t)k * N + i] * yv[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (ks == 0 && i < N) {
        double s = red[io];
        for (int q = 1; q < kInvSlices; ++q) s += red[q * kInvOut + io];
        x[(size_t)b * N + i] = (T)s;
    }
}

// One stage of the eigenbasis coarse solve, a batched n x n product
//   C[b](i, j) = sum_k A(b, i, k) B(b, k, j)   (FP64 accumulation)
// with element (b, r, c) of an operand at  ptr[b * sb + r * sr + c * sc]
// (sb = 0 for the shared basis V), so transposes are stride swaps.  With
// `lam`, the result is divided by alpha[b] + lam_i lam_j (the diagonal of the
// coarsest operator in that basis).  16 x 16 output tile per workgroup.
constexpr int kET = 16;

template <typename TA, typename TB, typename TC>
__global__ void __launch_bounds__(kET * kET) k_eig_stage(const TA* __restrict__ A, size_t sab, int sar, int sac,
                                                         const TB* __restrict__ B, size_t sbb, int sbr, int sbc,
                                                         TC* __restrict__ C, const double* __restrict__ lam,
                                                         const double* __restrict__ alpha, int n) {
    __shared__ double ta[kET][kET + 1], tb[kET][kET + 1];
    const int b = blockIdx.z;
    const int tiles = (n + kET - 1) / kET;
    const int i0 = (blockIdx.x / tiles) * kET, j0 = (blockIdx.x % tiles) * kET;
    const int ti = threadIdx.x / kET, tj = threadIdx.x % kET;
    const TA* Ab = A + (size_t)b * sab;
    const TB* Bb = B + (size_t)b * sbb;
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += kET) {
        const int ar = i0 + ti, ak = k0 + tj, bk = k0 + ti, bc = j0 + tj;
        ta[ti][tj] = (ar < n && ak < n) ? (double)Ab[(size_t)ar * sar + (size_t)ak * sac] : 0.0;
        tb[ti][tj] = (bk < n && bc < n) ? (double)Bb[(size_t)bk * sbr + (size_t)bc * sbc] : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kET; ++k) acc += ta[ti][k] * tb[k][tj];
        __syncthreads();
    }
    const int i = i0 + ti, j = j0 + tj;
    if (i >= n || j >= n) return;
    if (lam) acc /= alpha[b] + lam[i] * lam[j];
    C[(size_t)b * n * n + (size_t)i * n + j] = (TC)acc;
}

// The whole eigenbasis solve of one right-hand side in one workgroup for
// coarsest grids up to 32 x 32: V, y and the intermediate in LDS, the same
// four products as k_eig_stage (FP64, ascending k, the same division), so
// the result is the same; one launch instead of four.
constexpr int kEigSmall = 32;

// The one-workgroup eigenbasis solve of one right-hand side (NTH threads):
// y(e) gives element e of y, x receives the n x n solution.  sV, sA, sB hold
// kEigSmall^2 doubles each, sl kEigSmall.  With STAGED, sV and sl already
// hold V and the eigenvalues.
template <int NTH, bool STAGED = false, typename T, typename YF>
__device__ inline void eig_small_solve(const double* __restrict__ V, const double* __restrict__ lam, double a, YF y,
                                       T* __restrict__ x, int n, double* sV, double* sA, double* sB, double* sl) {
    const int nn = n * n;
    for (int e = threadIdx.x; e < nn; e += NTH) {
        if constexpr (!STAGED) sV[e] = V[e];
        sA[e] = y(e);
    }
    if constexpr (!STAGED)
        for (int i = threadIdx.x; i < n; i += NTH) sl[i] = lam[i];
    __syncthreads();
    // T1 = V^T y
    for (int e = threadIdx.x; e < nn; e += NTH) {
        const int i = e / n, j = e - (e / n) * n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += sV[k * n + i] * sA[k * n + j];
        sB[e] = acc;
    }
    __syncthreads();
    // T2 = (T1 V) / (alpha + lam_i lam_j)
    for (int e = threadIdx.x; e < nn; e += NTH) {
        const int i = e / n, j = e - (e / n) * n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += sB[i * n + k] * sV[k * n + j];
        sA[e] = acc / (a + sl[i] * sl[j]);
    }
    __syncthreads();
    // T3 = V T2
    for (int e = threadIdx.x; e < nn; e += NTH) {
        const int i = e / n, j = e - (e / n) * n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += sV[i * n + k] * sA[k * n + j];
        sB[e] = acc;
    }
    __syncthreads();
    // x = T3 V^T
    for (int e = threadIdx.x; e < nn; e += NTH) {
        const int i = e / n, j = e - (e / n) * n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += sB[i * n + k] * sV[j * n + k];
        x[e] = (T)acc;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_eig_small(const double* __restrict__ V, const double* __restrict__ lam,
                                                   const double* __restrict__ alpha, const T* __restrict__ y,
                                                   T* __restrict__ x, int n) {
    __shared__ double sV[kEigSmall * kEigSmall], sA[kEigSmall * kEigSmall], sB[kEigSmall * kEigSmall];
    __shared__ double sl[kEigSmall];
    const int b = blockIdx.x;
    const size_t nn = (size_t)n * n;
    const T* yb = y + b * nn;
    eig_small_solve<256>(V, lam, alpha[b], [&](int e) { return (double)yb[e]; }, x + b * nn, n, sV, sA, sB, sl);
}

// Restriction chain.  A cycle without pre-smoothing from x = 0 restricts its
// right-hand side through every level before any other work
// (y_{k+1} = R y_k).  From the first level whose restricted grids all fit
// in LDS, one workgroup per right-hand side takes the remaining
// restrictions in one launch: the first reads y_{k0} from global memory,
// each later one the grid the previous one left in LDS, and every y_k is
// written out (the post-smoothing residuals read them).  With the
// eigenbasis coarse solve on a grid of at most kEigSmall^2 points, the
// coarsest solve follows in the same workgroup.  Each point is the 3 x 3
// full weighting of the single-level restriction, in its order (weighted
// row sums, then their weighted sum), and the solve is the one of
// k_eig_small, so the values are those of the separate launches.
constexpr int kChainThreads = 1024;
static_assert(kEigSmall * kEigSmall <= kChainThreads, "one V element per thread");
constexpr int kChainUnroll = 4;  // outputs per thread whose loads are in flight together

template <typename T>
__device__ inline T restrict_point(const T* __restrict__ src, int nf, int i, int j) {
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    T acc = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T* row = src + (2 * i + a) * nf;
        T ra = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) ra += w[c] * row[2 * j + c];
        acc += w[a] * ra;
    }
    return acc;
}

template <typename T>
__global__ void __launch_bounds__(kChainThreads) k_restrict_chain(RestrictChain<T> ch, const double* __restrict__ V,
                                                                  const double* __restrict__ lam,
                                                                  const double* __restrict__ alpha) {
    __shared__ T bufA[kChainMax * kChainMax], bufB[(kChainMax / 2) * (kChainMax / 2)];
    __shared__ double sV[kEigSmall * kEigSmall], sA[kEigSmall * kEigSmall], sB[kEigSmall * kEigSmall];
    __shared__ double sl[kEigSmall];
    const int b = blockIdx.x, tid = threadIdx.x;
    // the coarsest solve's V and eigenvalues: loaded first (one element per
    // thread, n^2 <= kChainThreads), stored to LDS after the first restriction
    const int nL = ch.n[ch.levels - 1];
    const bool solve = ch.x_coarse != nullptr;
    const double vv = (solve && tid < nL * nL) ? V[tid] : 0.0;
    const double lv = (solve && tid < nL) ? lam[tid] : 0.0;
    // first restriction: y_{k0} (global) -> y_{k0 + 1}; the outputs of a
    // thread past the grid recompute its last point (their loads stay in
    // bounds and issue with the others) and store nothing
    {
        const int nf = ch.n[0], nc = ch.n[1], ncc = nc * nc;
        const T* src = ch.y[0] + (size_t)b * nf * nf;
        T* dst = ch.y[1] + (size_t)b * ncc;
        for (int e0 = 0; e0 < ncc; e0 += kChainThreads * kChainUnroll) {
            T v[kChainUnroll];
#pragma unroll
            for (int u = 0; u < kChainUnroll; ++u) {
                const int e = min(e0 + u * kChainThreads + tid, ncc - 1);
                const int i = e / nc, j = e - (e / nc) * nc;
                v[u] = restrict_point(src, nf, i, j);
            }
#pragma unroll
            for (int u = 0; u < kChainUnroll; ++u) {
                const int e = e0 + u * kChainThreads + tid;
                if (e < ncc) {
                    bufA[e] = v[u];
                    dst[e] = v[u];
                }
            }
        }
    }
    if (solve && tid < nL * nL) sV[tid] = vv;
    if (solve && tid < nL) sl[tid] = lv;
    __syncthreads();
    // later restrictions, LDS to LDS (levels alternate between the buffers)
    T* cur = bufA;
    T* nxt = bufB;
    for (int k = 1; k + 1 < ch.levels; ++k) {
        const int nf = ch.n[k], nc = ch.n[k + 1], ncc = nc * nc;
        T* dst = ch.y[k + 1] + (size_t)b * ncc;
        for (int e = tid; e < ncc; e += kChainThreads) {
            const int i = e / nc, j = e - (e / nc) * nc;
            const T v = restrict_point(cur, nf, i, j);
            nxt[e] = v;
            dst[e] = v;
        }
        __syncthreads();
        T* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (solve)
        eig_small_solve<kChainThreads, true>(V, lam, alpha[b], [&](int e) { return (double)cur[e]; },
                                             ch.x_coarse + (size_t)b * nL * nL, nL, sV, sA, sB, sl);
}

}  // namespace

// x = V [(V^T y V) / (alpha + lam_i lam_j)] V^T per right-hand side: four
// batched products through the FP64 stage scratch, or one workgroup per
// right-hand side for coarsest grids up to 32 x 32.
template <typename T>
nmg_status launch_eig_coarse(const Ctx* c, int batch, const double* alpha, const T* y, T* x, hipStream_t s) {
    const int n = c->n[(size_t)c->L - 1];
    if (n <= kEigSmall) {
        hipLaunchKernelGGL((k_eig_small<T>), dim3(batch), dim3(256), 0, s, c->eigV, c->eigLam, alpha, y, x, n);
        NMG_HIP(hipGetLastError());
        return NMG_OK;
    }
    const size_t nn = (size_t)n * n;
    const int tiles = (n + kET - 1) / kET;
    const dim3 grid(tiles * tiles, 1, batch), block(kET * kET);
    double* T1 = c->eigT;
    double* T2 = c->eigT + (size_t)c->p.max_batch * nn;
    const double* V = c->eigV;
    // T1 = V^T y
    hipLaunchKernelGGL((k_eig_stage<double, T, double>), grid, block, 0, s, V, (size_t)0, 1, n, y, nn, n, 1, T1,
                       (const double*)nullptr, alpha, n);
    // T2 = (T1 V) / (alpha + lam lam)
    hipLaunchKernelGGL((k_eig_stage<double, double, double>), grid, block, 0, s, T1, nn, n, 1, V, (size_t)0, n, 1,
                       T2, c->eigLam, alpha, n);
    // T1 = V T2
    hipLaunchKernelGGL((k_eig_stage<double, double, double>), grid, block, 0, s, V, (size_t)0, n, 1, T2, nn, n, 1,
                       T1, (const double*)nullptr, alpha, n);
    // x = T1 V^T
    hipLaunchKernelGGL((k_eig_stage<double, double, T>), grid, block, 0, s, T1, nn, n, 1, V, (size_t)0, 1, n, x,
                       (const double*)nullptr, alpha, n);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}
template <typename T>
nmg_status launch_restrict_chain(const Ctx* c, int batch, const double* alpha, const RestrictChain<T>& ch,
                                 hipStream_t s) {
    if (ch.levels < 2 || ch.levels > kChainLevels) return fail(NMG_ERR_ARG, "restriction chain: level count");
    for (int k = 0; k + 1 < ch.levels; ++k)
        if (ch.n[k + 1] != (ch.n[k] - 1) / 2 || ch.n[k + 1] < 1 || (k == 0 && 2 * ch.n[1] + 1 > ch.n[0]))
            return fail(NMG_ERR_SHAPE, "restriction chain: grid sizes do not halve");
    if (ch.n[1] > kChainMax) return fail(NMG_ERR_SHAPE, "restriction chain: restricted grid exceeds the LDS buffers");
    if (ch.x_coarse && (!c->eig_coarse || ch.n[ch.levels - 1] > kEigSmall))
        return fail(NMG_ERR_STATE, "restriction chain: the coarsest solve needs the small eigenbasis form");
    hipLaunchKernelGGL((k_restrict_chain<T>), dim3(batch), dim3(kChainThreads), 0, s, ch, c->eigV, c->eigLam, alpha);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}
template nmg_status launch_restrict_chain<float>(const Ctx*, int, const double*, const RestrictChain<float>&,
                                                 hipStream_t);
template nmg_status launch_restrict_chain<double>(const Ctx*, int, const double*, const RestrictChain<double>&,
                                                  hipStream_t);

int eig_small_max() { return kEigSmall; }

template nmg_status launch_eig_coarse<float>(const Ctx*, int, const double*, const float*, float*, hipStream_t);
template nmg_status launch_eig_coarse<double>(const Ctx*, int, const double*, const double*, double*, hipStream_t);

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
    hipLaunchKernelGGL(k_inverse_apply<T>, dim3((N + kInvOut - 1) / kInvOut, batch), dim3(kBlock),
                       (N + kBlock) * sizeof(double), s, c->cinv, c->cycle_fidx ? c->cycle_fidx : c->coarse_idx,
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
