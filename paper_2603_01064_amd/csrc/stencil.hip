// Residual / operator, norms and grid transfers on a level of the hierarchy.
//
// A_l X = alpha M_l X M_l + G_l X G_l (2D) and alpha M_l x + G_l x (1D),
// with banded, row-specific factors (Galerkin products, Algorithm 1).  The
// product is evaluated as two separable passes: a pass along each row
// (right multiplication by the symmetric factor) followed by a pass along
// each column that also forms y - A x.  Transfers are full weighting
// (1/4, 1/2, 1/4 per axis) and linear interpolation with zero boundary
// values (Sec. 2.3).
#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kBlock = 256;

// Row pass: tg[b][i][j] = sum_q G[j][q] x[b][i][q]; the same for M into tm.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rowpass(const T* __restrict__ x, T* __restrict__ tg,
                                                    T* __restrict__ tm, const T* __restrict__ G, int rg,
                                                    const T* __restrict__ M, int rm, int n, size_t per) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    const int b = blockIdx.y;
    const int i = (int)(e / n), j = (int)(e % n);
    const T* row = x + (size_t)b * per + (size_t)i * n;
    {
        const int w = 2 * rg + 1;
        const T* g = G + (size_t)j * w;
        const int t0 = max(0, rg - j), t1 = min(w - 1, n - 1 - j + rg);
        T acc = 0;
        for (int t = t0; t <= t1; ++t) acc += g[t] * row[j - rg + t];
        tg[(size_t)b * per + e] = acc;
    }
    {
        const int w = 2 * rm + 1;
        const T* m = M + (size_t)j * w;
        const int t0 = max(0, rm - j), t1 = min(w - 1, n - 1 - j + rm);
        T acc = 0;
        for (int t = t0; t <= t1; ++t) acc += m[t] * row[j - rm + t];
        tm[(size_t)b * per + e] = acc;
    }
}

// Column pass and combination.  2D: out = s0*y + s1*(alpha M tm + G tg)
// with the column factors applied along i; 1D: out = s0*y + s1*(alpha tm + tg).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_colcombine(const T* __restrict__ tg, const T* __restrict__ tm,
                                                       const T* __restrict__ y, T* __restrict__ out,
                                                       const T* __restrict__ G, int rg, const T* __restrict__ M,
                                                       int rm, const double* __restrict__ alpha, int n, int ny,
                                                       size_t per, int mode) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    const int b = blockIdx.y;
    const T a = (T)alpha[b];
    const size_t base = (size_t)b * per;
    T ax;
    if (ny == 1) {
        ax = a * tm[base + e] + tg[base + e];
    } else {
        const int i = (int)(e / n), j = (int)(e % n);
        T accg = 0, accm = 0;
        {
            const int w = 2 * rg + 1;
            const T* g = G + (size_t)i * w;
            const int t0 = max(0, rg - i), t1 = min(w - 1, n - 1 - i + rg);
            for (int t = t0; t <= t1; ++t) accg += g[t] * tg[base + (size_t)(i - rg + t) * n + j];
        }
        {
            const int w = 2 * rm + 1;
            const T* m = M + (size_t)i * w;
            const int t0 = max(0, rm - i), t1 = min(w - 1, n - 1 - i + rm);
            for (int t = t0; t <= t1; ++t) accm += m[t] * tm[base + (size_t)(i - rm + t) * n + j];
        }
        ax = a * accm + accg;
    }
    out[base + e] = (mode == 0) ? (y[base + e] - ax) : ax;
}

// Per right-hand-side sum of squares in FP64, fixed reduction order.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sumsq(const T* __restrict__ v, double* __restrict__ out, size_t per) {
    __shared__ double red[kBlock];
    const int b = blockIdx.x;
    const T* p = v + (size_t)b * per;
    double acc = 0.0;
    for (size_t e = threadIdx.x; e < per; e += kBlock) {
        const double t = (double)p[e];
        acc += t * t;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = red[0];
}

// Full weighting: coarse node i reads fine nodes 2i, 2i+1, 2i+2 (1/4, 1/2, 1/4).
template <typename T>
__device__ inline void restrict_taps(int i, int* idx, T* w) {
    idx[0] = 2 * i;
    idx[1] = 2 * i + 1;
    idx[2] = 2 * i + 2;
    w[0] = (T)0.25;
    w[1] = (T)0.5;
    w[2] = (T)0.25;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(const T* __restrict__ r, T* __restrict__ yc, int nf, int nc,
                                                     int two_d, T scale) {
    const int rows_c = two_d ? nc : 1;
    const size_t perc = (size_t)rows_c * nc;
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= perc) return;
    const int b = blockIdx.y;
    const size_t perf = (size_t)(two_d ? nf : 1) * nf;
    const int i = (int)(e / nc), j = (int)(e % nc);
    int ij[3], ii[3];
    T wj[3], wi[3];
    restrict_taps<T>(j, ij, wj);
    restrict_taps<T>(i, ii, wi);
    const T* src = r + (size_t)b * perf;
    T acc = 0;
    if (two_d) {
        for (int a = 0; a < 3; ++a) {
            const T* row = src + (size_t)ii[a] * nf;
            T ra = 0;
            for (int c = 0; c < 3; ++c) ra += wj[c] * row[ij[c]];
            acc += wi[a] * ra;
        }
    } else {
        for (int c = 0; c < 3; ++c) acc += wj[c] * src[ij[c]];
    }
    yc[(size_t)b * perc + e] = scale * acc;
}

// Linear interpolation and correction: x += P e (2D: P e P^T).
template <typename T>
__device__ inline int interp_taps(int p, int nc, int* idx, T* w) {
    if (p & 1) {
        idx[0] = (p - 1) >> 1;
        w[0] = (T)1;
        return 1;
    }
    int k = 0;
    const int c0 = (p >> 1) - 1, c1 = p >> 1;
    if (c0 >= 0) { idx[k] = c0; w[k] = (T)0.5; ++k; }
    if (c1 < nc) { idx[k] = c1; w[k] = (T)0.5; ++k; }
    return k;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_add(const T* __restrict__ ec, T* __restrict__ x, int nf, int nc,
                                                        int two_d) {
    const size_t perf = (size_t)(two_d ? nf : 1) * nf;
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= perf) return;
    const int b = blockIdx.y;
    const size_t perc = (size_t)(two_d ? nc : 1) * nc;
    const int p = (int)(e / nf), q = (int)(e % nf);
    const T* src = ec + (size_t)b * perc;
    int iq[2];
    T wq[2];
    const int kq = interp_taps<T>(q, nc, iq, wq);
    T acc = 0;
    if (two_d) {
        int ip[2];
        T wp[2];
        const int kp = interp_taps<T>(p, nc, ip, wp);
        for (int a = 0; a < kp; ++a) {
            T ra = 0;
            for (int c = 0; c < kq; ++c) ra += wq[c] * src[(size_t)ip[a] * nc + iq[c]];
            acc += wp[a] * ra;
        }
    } else {
        for (int c = 0; c < kq; ++c) acc += wq[c] * src[iq[c]];
    }
    x[(size_t)b * perf + e] += acc;
}

// Writes the index maps exactly as the transfer kernels compute them.
__global__ void k_export_maps(int nf, int nc, int kind, int32_t* __restrict__ idx, float* __restrict__ w) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (kind == 0) {
        if (e >= nc) return;
        int ii[3];
        float ww[3];
        restrict_taps<float>(e, ii, ww);
        for (int a = 0; a < 3; ++a) {
            idx[e * 3 + a] = ii[a];
            w[e * 3 + a] = ww[a];
        }
    } else {
        if (e >= nf) return;
        int ii[2] = {-1, -1};
        float ww[2] = {0.f, 0.f};
        interp_taps<float>(e, nc, ii, ww);
        for (int a = 0; a < 2; ++a) {
            idx[e * 2 + a] = ii[a];
            w[e * 2 + a] = ww[a];
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_axpy(const T* __restrict__ src, T* __restrict__ dst, size_t count,
                                                 int accumulate) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    dst[e] = accumulate ? dst[e] + src[e] : src[e];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill_zero(T* __restrict__ p, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < count) p[e] = (T)0;
}

template <typename A, typename B>
__global__ void __launch_bounds__(kBlock) k_convert(const A* __restrict__ src, B* __restrict__ dst, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < count) dst[e] = (B)src[e];
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

size_t level_elems(const Ctx* c, int l) { return (size_t)(c->p.dim == 2 ? c->n[l] : 1) * c->n[l]; }

template <typename T>
nmg_status launch_operator(const Ctx* c, int l, int batch, const double* alpha, const T* x, const T* y, T* out,
                           int mode, Work<T>& w, hipStream_t s) {
    const int n = c->n[l];
    const size_t per = level_elems(c, l);
    const HostLevel& hl = c->host[l];
    const T* G = w.Gd + w.g_off[l];
    const T* M = w.Md + w.m_off[l];
    dim3 grid(blocks_for(per), batch);
    hipLaunchKernelGGL(k_rowpass<T>, grid, dim3(kBlock), 0, s, x, w.lv[l].t1, w.lv[l].t2, G, hl.G.r, M, hl.M.r, n,
                       per);
    hipLaunchKernelGGL(k_colcombine<T>, grid, dim3(kBlock), 0, s, w.lv[l].t1, w.lv[l].t2, y, out, G, hl.G.r, M,
                       hl.M.r, alpha, n, c->p.dim == 2 ? n : 1, per, mode);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_sumsq(int batch, size_t elems, const T* v, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sumsq<T>, dim3(batch), dim3(kBlock), 0, s, v, out, elems);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_restrict(const Ctx* c, int l, int batch, const T* r, T* yc, hipStream_t s) {
    const int nf = c->n[l], nc = c->n[l + 1];
    const size_t perc = level_elems(c, l + 1);
    hipLaunchKernelGGL(k_restrict<T>, dim3(blocks_for(perc), batch), dim3(kBlock), 0, s, r, yc, nf, nc,
                       c->p.dim == 2 ? 1 : 0, (T)1);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

// P^T g = 2^d R g: the adjoint of linear interpolation (weights 1/2, 1, 1/2).
template <typename T>
nmg_status launch_prolong_transpose(const Ctx* c, int l, int batch, const T* g, T* out, hipStream_t s) {
    const int nf = c->n[l], nc = c->n[l + 1];
    const size_t perc = level_elems(c, l + 1);
    hipLaunchKernelGGL(k_restrict<T>, dim3(blocks_for(perc), batch), dim3(kBlock), 0, s, g, out, nf, nc,
                       c->p.dim == 2 ? 1 : 0, (T)(c->p.dim == 2 ? 4 : 2));
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_prolong_add(const Ctx* c, int l, int batch, const T* e, T* x, hipStream_t s) {
    const int nf = c->n[l], nc = c->n[l + 1];
    const size_t perf = level_elems(c, l);
    hipLaunchKernelGGL(k_prolong_add<T>, dim3(blocks_for(perf), batch), dim3(kBlock), 0, s, e, x, nf, nc,
                       c->p.dim == 2 ? 1 : 0);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

nmg_status launch_export_maps(const Ctx* c, int l, int kind, int32_t* idx, float* w, hipStream_t s) {
    const int nf = c->n[l], nc = c->n[l + 1];
    const int cnt = kind == 0 ? nc : nf;
    hipLaunchKernelGGL(k_export_maps, dim3((cnt + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nf, nc, kind, idx, w);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_axpy(int batch, size_t elems, const T* src, T* dst, int accumulate, hipStream_t s) {
    const size_t count = (size_t)batch * elems;
    hipLaunchKernelGGL(k_axpy<T>, dim3(blocks_for(count)), dim3(kBlock), 0, s, src, dst, count, accumulate);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_zero(T* p, size_t count, hipStream_t s) {
    if (count == 0) return NMG_OK;
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(blocks_for(count)), dim3(kBlock), 0, s, p, count);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename A, typename B>
nmg_status launch_convert(const A* src, B* dst, size_t count, hipStream_t s) {
    if (count == 0) return NMG_OK;
    hipLaunchKernelGGL((k_convert<A, B>), dim3(blocks_for(count)), dim3(kBlock), 0, s, src, dst, count);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

#define NMG_INST(T)                                                                                              \
    template nmg_status launch_operator<T>(const Ctx*, int, int, const double*, const T*, const T*, T*, int,     \
                                           Work<T>&, hipStream_t);                                               \
    template nmg_status launch_sumsq<T>(int, size_t, const T*, double*, hipStream_t);                            \
    template nmg_status launch_restrict<T>(const Ctx*, int, int, const T*, T*, hipStream_t);                     \
    template nmg_status launch_prolong_transpose<T>(const Ctx*, int, int, const T*, T*, hipStream_t);            \
    template nmg_status launch_prolong_add<T>(const Ctx*, int, int, const T*, T*, hipStream_t);                  \
    template nmg_status launch_axpy<T>(int, size_t, const T*, T*, int, hipStream_t);                             \
    template nmg_status launch_zero<T>(T*, size_t, hipStream_t);
NMG_INST(float)
NMG_INST(double)
#undef NMG_INST
template nmg_status launch_zero<int>(int*, size_t, hipStream_t);
template nmg_status launch_convert<float, double>(const float*, double*, size_t, hipStream_t);
template nmg_status launch_convert<double, float>(const double*, float*, size_t, hipStream_t);

}  // namespace nmg
