// Residual / operator, norms and grid transfers on a level of the hierarchy.
//
// A_l X = alpha M_l X M_l + G_l X G_l (2D) and alpha M_l x + G_l x (1D),
// with banded, row-specific factors (Galerkin products, Algorithm 1).  The
// product is evaluated as two separable passes: a pass along each row
// (right multiplication by the symmetric factor) followed by a pass along
// each column that also forms y - A x.  Transfers are full weighting
// (1/4, 1/2, 1/4 per axis) and linear interpolation with zero boundary
// values (Sec. 2.3).
#include <type_traits>

#include <algorithm>

#include "nmg_internal.h"
#include "tree_sum.h"

namespace nmg {

namespace {

constexpr int kBlock = 256;

// XCD-major numbering of a (gridDim.x, gridDim.y) grid.  Workgroups are
// dispatched round-robin over the 8 XCDs by linear id; numbering them so that
// XCD x takes a contiguous range of the (block, image) pairs, in order, puts
// the neighbouring blocks of one image on one XCD, where the halo rows and
// columns they share are read from its L2 instead of from memory.  Returns
// the logical block (bx) and image (by).
__device__ inline void xcd_major(int& bx, int& by) {
    const int G = gridDim.x * gridDim.y, i = blockIdx.x + blockIdx.y * gridDim.x;
    const int xc = i % 8, q = G / 8, rem = G % 8;
    const int p = xc * q + min(xc, rem) + i / 8;
    by = p / gridDim.x;
    bx = p - by * gridDim.x;
}

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

// Per right-hand-side sum of squares in FP64 with a fixed reduction order:
// stage 1 writes one partial per (chunk, rhs), stage 2 adds the chunks.
constexpr int kNormChunks = kNormChunksPerRhs;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sumsq_part(const T* __restrict__ v, double* __restrict__ part, size_t per) {
    __shared__ double red[kBlock];
    const int b = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
    const size_t len = (per + nch - 1) / nch;
    const size_t e0 = (size_t)ch * len, e1 = e0 + len < per ? e0 + len : per;
    const T* p = v + (size_t)b * per;
    double acc = 0.0;
    for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
        const double t = (double)p[e];
        acc += t * t;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    const double tot = tree_sum<kBlock, kBlock>(red, threadIdx.x);
    if (threadIdx.x == 0) part[(size_t)b * nch + ch] = tot;
}

// nparts partials per right-hand side (row stride `stride`), added in order
// mirror (optional): the same sums into pinned host memory, made visible at
// system scope, so the host reads them after the stream's work without a copy
__global__ void k_sumsq_final(const double* __restrict__ part, double* __restrict__ out, int batch, int nparts,
                              int stride, double* __restrict__ mirror = nullptr) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    double acc = 0.0;
    // (unrolled: the loads of eight partials are in flight together; the
    // sum keeps its ascending order)
#pragma unroll 8
    for (int c = 0; c < nparts; ++c) acc += part[(size_t)b * stride + c];
    out[b] = acc;
    if (mirror) {
        mirror[b] = acc;
        __threadfence_system();
    }
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
                                                     int two_d, T scale, double* __restrict__ part) {
    const int rows_c = two_d ? nc : 1;
    const size_t perc = (size_t)rows_c * nc;
    int bx, b;
    xcd_major(bx, b);
    const size_t perf = (size_t)(two_d ? nf : 1) * nf;
    const T* src = r + (size_t)b * perf;
    double sq = 0.0;
    // 32-bit indices (a level holds fewer than 2^31 points): a 64-bit division
    // per point cost more than the point's arithmetic
    for (int e = bx * kBlock + (int)threadIdx.x; e < (int)perc; e += (int)gridDim.x * kBlock) {
        const int i = e / nc, j = e - (e / nc) * nc;
        int ij[3], ii[3];
        T wj[3], wi[3];
        restrict_taps<T>(j, ij, wj);
        restrict_taps<T>(i, ii, wi);
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
        const T v = scale * acc;
        yc[(size_t)b * perc + e] = v;
        sq += (double)v * (double)v;
    }
    // optional: this block's partial sum of squares of the output (the first
    // stage of ||yc||^2, for a consumer that adds the gridDim.x partials)
    if (part) {
        __shared__ double red[kBlock];
        red[threadIdx.x] = sq;
        __syncthreads();
        const double tot = tree_sum<kBlock, kBlock>(red, threadIdx.x);
        if (threadIdx.x == 0) part[(size_t)b * gridDim.x + bx] = tot;
    }
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
                                                        int two_d, int set) {
    const size_t perf = (size_t)(two_d ? nf : 1) * nf;
    int bx, b;
    xcd_major(bx, b);
    const int e = bx * kBlock + (int)threadIdx.x;  // 32-bit: a level holds fewer than 2^31 points
    if (e >= (int)perf) return;
    const size_t perc = (size_t)(two_d ? nc : 1) * nc;
    const int p = e / nf, q = e - (e / nf) * nf;
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
    if (set)
        x[(size_t)b * perf + e] = acc;
    else
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

// ---------------------------------------------------------------------------
// Tiled residual: one workgroup per TH x TW output tile of one right-hand
// side.  Each factor is split into a Toeplitz interior (wave-uniform
// coefficients, zero-padded to a multiple of 4 taps) plus rc x rc corner
// corrections.  The input tile with a halo of rg rows/columns is staged in
// LDS, the row pass X G (and X M) is evaluated for the tile columns on every
// halo row, and the column pass G (X G) forms y - A x.  Each thread keeps
// four outputs in registers and slides a window of eight inputs over the
// taps, so every LDS read feeds four FMAs.
// ---------------------------------------------------------------------------
template <typename T>
struct Vec4 {
    T v[4];
};

template <typename T>
__device__ inline Vec4<T> lds_load4(const T* p) {
    Vec4<T> r;
    if constexpr (sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
    }
    return r;
}

// acc[o] += sum_t c[t] * row[base + o + t], o = 0..3, t < tp (tp % 4 == 0),
// stride = distance between consecutive elements of `row`.
template <typename T, bool CONTIG>
__device__ inline void slide4(const T* __restrict__ row, int stride, const T* __restrict__ c, int tp, T acc[4]) {
    T w[8];
    if constexpr (CONTIG) {
        const Vec4<T> a = lds_load4<T>(row);
        for (int k = 0; k < 4; ++k) w[k] = a.v[k];
    } else {
        for (int k = 0; k < 4; ++k) w[k] = row[k * stride];
    }
    for (int t4 = 0; t4 < tp; t4 += 4) {
        if constexpr (CONTIG) {
            const Vec4<T> b = lds_load4<T>(row + t4 + 4);
            for (int k = 0; k < 4; ++k) w[4 + k] = b.v[k];
        } else {
            for (int k = 0; k < 4; ++k) w[4 + k] = row[(t4 + 4 + k) * stride];
        }
        const T c0 = c[t4], c1 = c[t4 + 1], c2 = c[t4 + 2], c3 = c[t4 + 3];
#pragma unroll
        for (int o = 0; o < 4; ++o) acc[o] += c0 * w[o] + c1 * w[o + 1] + c2 * w[o + 2] + c3 * w[o + 3];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = w[4 + k];
    }
}

template <typename T, int TH, int TW>
__global__ void __launch_bounds__(kBlock) k_residual_tiled(
    const T* __restrict__ x, const T* __restrict__ y, T* __restrict__ out, const double* __restrict__ alpha, int n,
    int mode, const T* __restrict__ tg, int rg, int rgp, const T* __restrict__ dtl, const T* __restrict__ dbr, int rc,
    const T* __restrict__ tm, int rm, int rmp, int m_ident, int tiles_x) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int XW = TW + rgp;           // staged columns: image j0 - rg + c
    const int XH = TH + 2 * rg;        // staged rows:    image i0 - rg + r
    const int GH = TH + rgp;           // rows of X G (zero beyond XH)
    const int MH = TH + rmp;           // rows of X M
    T* X = sm;
    T* TGs = X + (size_t)XH * XW;
    T* TMs = TGs + (size_t)GH * TW;
    int tile, b;
    xcd_major(tile, b);
    const int i0 = (tile / tiles_x) * TH, j0 = (tile % tiles_x) * TW;
    const size_t per = (size_t)n * n;
    const T* xs = x + (size_t)b * per;
    const int tid = threadIdx.x;
    {
        // staging: 4 rows x 64 columns per pass, UNR passes of loads in flight
        // before their LDS stores (no integer division)
        constexpr int UNR = 8, KC = 4;  // XW <= 64 * KC (checked on the host)
        const int ty = tid >> 6, tx = tid & 63;
        for (int r0 = ty; r0 < XH; r0 += 4 * UNR) {
            T v[UNR][KC];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int r = r0 + 4 * u;
                const int gi = i0 - rg + r;
                const bool row_in = r < XH && gi >= 0 && gi < n;
                const T* src = xs + (size_t)(row_in ? gi : 0) * n;
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const int c = tx + 64 * k;
                    const int gj = j0 - rg + c;
                    v[u][k] = (row_in && c < XW && gj >= 0 && gj < n) ? src[gj] : (T)0;
                }
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int r = r0 + 4 * u;
                if (r < XH) {
#pragma unroll
                    for (int k = 0; k < KC; ++k)
                        if (tx + 64 * k < XW) X[r * XW + tx + 64 * k] = v[u][k];
                }
            }
        }
    }
    for (int e = tid + XH * TW; e < GH * TW; e += kBlock) TGs[e] = 0;
    if (!m_ident)
        for (int e = tid + (TH + 2 * rm) * TW; e < MH * TW; e += kBlock) TMs[e] = 0;
    __syncthreads();
    // ---- row passes
    constexpr int CG = TW / 4;
    for (int item = tid; item < XH * CG; item += kBlock) {
        const int r = item / CG, jj = (item % CG) * 4;
        T acc[4] = {0, 0, 0, 0};
        slide4<T, true>(X + (size_t)r * XW + jj, 1, tg, rgp, acc);
        const int j = j0 + jj;
        if (rc > 0 && (j < rc || j + 3 >= n - rc)) {
            for (int o = 0; o < 4; ++o) {
                const int jo = j + o;
                if (jo < rc) {
                    T s2 = 0;
                    for (int q = 0; q < rc; ++q) s2 += dtl[q * rc + jo] * X[(size_t)r * XW + (q - j0 + rg)];
                    acc[o] += s2;
                } else if (jo >= n - rc && jo < n) {
                    T s2 = 0;
                    const int jb = jo - (n - rc);
                    for (int q = 0; q < rc; ++q) s2 += dbr[q * rc + jb] * X[(size_t)r * XW + (n - rc + q - j0 + rg)];
                    acc[o] += s2;
                }
            }
        }
        for (int o = 0; o < 4; ++o) TGs[(size_t)r * TW + jj + o] = acc[o];
    }
    if (!m_ident) {
        const int RH = TH + 2 * rm;
        for (int item = tid; item < RH * CG; item += kBlock) {
            const int r = item / CG, jj = (item % CG) * 4;
            T acc[4] = {0, 0, 0, 0};
            slide4<T, false>(X + (size_t)(rg - rm + r) * XW + jj + rg - rm, 1, tm, rmp, acc);
            for (int o = 0; o < 4; ++o) TMs[(size_t)r * TW + jj + o] = acc[o];
        }
    }
    __syncthreads();
    // ---- column pass and combination
    const T a = (T)alpha[b];
    for (int item = tid; item < (TH / 4) * TW; item += kBlock) {
        const int ii = (item / TW) * 4, jj = item % TW;
        const int j = j0 + jj;
        T g4[4] = {0, 0, 0, 0}, m4[4] = {0, 0, 0, 0};
        slide4<T, false>(TGs + (size_t)ii * TW + jj, TW, tg, rgp, g4);
        if (m_ident) {
            for (int o = 0; o < 4; ++o) m4[o] = X[(size_t)(ii + o + rg) * XW + jj + rg];
        } else {
            slide4<T, false>(TMs + (size_t)ii * TW + jj, TW, tm, rmp, m4);
        }
        for (int o = 0; o < 4; ++o) {
            const int i = i0 + ii + o;
            if (i >= n || j >= n) continue;
            T corr = 0;
            if (i < rc) {
                for (int p = 0; p < rc; ++p) corr += dtl[i * rc + p] * TGs[(size_t)(p - i0 + rg) * TW + jj];
            } else if (i >= n - rc) {
                const int ib = i - (n - rc);
                for (int p = 0; p < rc; ++p) corr += dbr[ib * rc + p] * TGs[(size_t)(n - rc + p - i0 + rg) * TW + jj];
            }
            const T ax = a * m4[o] + (g4[o] + corr);
            const size_t idx = (size_t)b * per + (size_t)i * n + j;
            out[idx] = mode == 0 ? y[idx] - ax : ax;
        }
    }
}

// ---------------------------------------------------------------------------
// Tiled residual with a compile-time tap count TP (the Toeplitz interior of
// G_l, 2 r_g + 1 taps zero-padded to a multiple of 4).  The staged tile has
// TH + TP rows and TW + TP columns, so every loop has fixed trip counts and
// unrolls fully; the row pass X G overwrites the staged tile in place (its
// results are held in registers across a barrier), which keeps the LDS
// footprint at one tile and allows three or more workgroups per CU.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void lds_load4v(const T* p, T* w) {
    if constexpr (sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        w[0] = a.x; w[1] = a.y; w[2] = b.x; w[3] = b.y;
    }
}

// Corner corrections of the band factor (rc x rc blocks where G_l differs from
// its Toeplitz interior) for the row pass, in outer-product order: one pass
// over the rc coupled values with independent accumulators per output, so
// the loads pipeline instead of forming one dependent chain per output (every
// wave of a row pass holds corner columns).  Outputs j .. j+3 of a staged
// row; row[c + off] is image column c.
template <typename T>
__device__ inline void row_corners(const T* row, int off, const T* cs, int rc, int n, int j, T acc[4]) {
    const int rc2 = rc * rc;
    const bool left = j < rc, right = j + 3 >= n - rc;
    T cl[4] = {0, 0, 0, 0}, cr[4] = {0, 0, 0, 0};
    for (int p = 0; p < rc; ++p) {
        if (left) {
            const T xv = row[p + off];
#pragma unroll
            for (int o = 0; o < 4; ++o)
                if (j + o < rc) cl[o] += cs[p * rc + j + o] * xv;
        }
        if (right) {
            const T xv = row[n - rc + p + off];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int jo = j + o;
                if (jo >= rc && jo >= n - rc && jo < n) cr[o] += cs[rc2 + p * rc + (jo - (n - rc))] * xv;
            }
        }
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) acc[o] += (j + o < rc) ? cl[o] : cr[o];
}

constexpr int kNormBlock = 32;  // side of the blocks of the residual's norm partials

template <typename T, int TH, int TW, int TP, int OC, int NT, int WPE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) k_residual_fixed(
    const T* __restrict__ x, const T* __restrict__ y, T* __restrict__ out, const double* __restrict__ alpha, int n,
    int mode, const T* __restrict__ tg, int rg, const T* __restrict__ dtl, const T* __restrict__ dbr, int rc,
    const T* __restrict__ tm, int m_ident, int tiles_x, double* __restrict__ part = nullptr) {
    constexpr int XH = TH + TP, XW = TW + TP;     // staged rows / columns (image i0 - rg + r, j0 - rg + c)
    constexpr int CG = TW / 4;                     // row-pass items per row (4 outputs each)
    constexpr int RITEMS = (XH * CG + NT - 1) / NT;
    constexpr int CITEMS = (TH / OC) * TW;         // column-pass items (OC outputs each)
    constexpr int CPT = (CITEMS + NT - 1) / NT;
    constexpr int MH = TH + 4;                     // rows of X M (radius 1, 4 padded taps)
    constexpr int WAVES = NT / 64;
    constexpr int KC = (XW + 63) / 64;             // 64-column chunks per staged row
    constexpr int SU = (XH + WAVES - 1) / WAVES;   // staged rows per wave
    static_assert(TH % OC == 0 && TW % 4 == 0 && TP % 4 == 0, "tile shape");
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);
    T* TMs = X + XH * XW;
    // corner corrections staged next to the tile (rc x rc each)
    T* cs = TMs + (m_ident ? 0 : MH * TW);
    const int rc2 = rc * rc;
    int tile, b;
    xcd_major(tile, b);
    const int i0 = (tile / tiles_x) * TH, j0 = (tile % tiles_x) * TW;
    const size_t per = (size_t)n * n;
    const T* xs = x + (size_t)b * per;
    const int tid = threadIdx.x;
    const T* taps = tg;
    // corner corrections into LDS; called between the first staging batch's
    // loads and its stores, so their loads are in flight with the tile's
    auto copy_corners = [&]() {
        for (int e = threadIdx.x; e < rc2; e += NT) {
            cs[e] = dtl[e];
            cs[rc2 + e] = dbr[e];
        }
    };
    // ---- stage the tile with its halo (zero outside the grid); every load of
    // a thread is issued before the first LDS store
    {
        // batches of SB rows per wave keep the in-flight values within the register budget
        constexpr int SB = sizeof(T) == 4 ? SU : (SU + 1) / 2;
        const int tx = tid & 63, ty = tid / 64;
#pragma unroll
        for (int u0 = 0; u0 < SU; u0 += SB) {
            T v[SB][KC];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int r = ty + WAVES * (u0 + u);
                const int gi = i0 - rg + r;
                const bool row_in = u0 + u < SU && r < XH && gi >= 0 && gi < n;
                const T* src = xs + (size_t)(row_in ? gi : 0) * n;
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const int c = tx + 64 * k;
                    const int gj = j0 - rg + c;
                    v[u][k] = (row_in && c < XW && gj >= 0 && gj < n) ? src[gj] : (T)0;
                }
            }
            if (u0 == 0) copy_corners();
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int r = ty + WAVES * (u0 + u);
#pragma unroll
                for (int k = 0; k < KC; ++k)
                    if (u0 + u < SU && r < XH && tx + 64 * k < XW) X[r * XW + tx + 64 * k] = v[u][k];
            }
        }
    }
    // right-hand side of this thread's outputs, in flight during the passes
    T yv[CPT][OC];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int item = tid + q * NT;
        const int ii = (item / TW) * OC, jj = item % TW;
#pragma unroll
        for (int o = 0; o < OC; ++o) {
            const int i = i0 + ii + o, j = j0 + jj;
            yv[q][o] = (mode == 0 && item < CITEMS && i < n && j < n) ? y[(size_t)b * per + (size_t)i * n + j] : (T)0;
        }
    }
    __syncthreads();
    // ---- values the column pass needs from X before it is overwritten
    T xc[CPT][OC];
    if (m_ident) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int item = tid + q * NT;
            const int ii = (item / TW) * OC, jj = item % TW;
#pragma unroll
            for (int o = 0; o < OC; ++o) xc[q][o] = item < CITEMS ? X[(ii + o + rg) * XW + jj + rg] : (T)0;
        }
    } else {
        // X M on rows i0 - 1 .. i0 + TH (M has radius 1 and an exact Toeplitz form)
        const T m0 = tm[0], m1 = tm[1], m2 = tm[2];
        for (int e = tid; e < MH * TW; e += NT) {
            const int r = e / TW, jj = e % TW;
            T v = 0;
            if (r < TH + 2) {
                const T* row = X + (r + rg - 1) * XW + jj + rg - 1;
                v = m0 * row[0] + m1 * row[1] + m2 * row[2];
            }
            TMs[e] = v;
        }
    }
    // ---- row pass into registers
    T racc[RITEMS][4];
#pragma unroll
    for (int q = 0; q < RITEMS; ++q) {
        const int item = tid + q * NT;
        const int r = item / CG, jj = (item % CG) * 4;
#pragma unroll
        for (int o = 0; o < 4; ++o) racc[q][o] = 0;
        if (item < XH * CG) {
            const T* row = X + r * XW + jj;
            // sliding window of 8 values, refilled 4 at a time
            T w[8];
            lds_load4v<T>(row, w);
#pragma unroll
            for (int t4 = 0; t4 < TP; t4 += 4) {
                lds_load4v<T>(row + t4 + 4, w + 4);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const T ct = taps[t4 + t];
#pragma unroll
                    for (int o = 0; o < 4; ++o) racc[q][o] = fma(ct, w[o + t], racc[q][o]);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) w[k] = w[4 + k];
            }
            const int j = j0 + jj;
            if (rc > 0 && (j < rc || j + 3 >= n - rc))
                row_corners<T>(X + r * XW, rg - j0, cs, rc, n, j, racc[q]);
        }
    }
    __syncthreads();
    // X G replaces the staged tile: row r keeps its TW row-pass values in columns 0..TW-1
#pragma unroll
    for (int q = 0; q < RITEMS; ++q) {
        const int item = tid + q * NT;
        if (item < XH * CG) {
            const int r = item / CG, jj = (item % CG) * 4;
            T* dst = X + r * XW + jj;
#pragma unroll
            for (int o = 0; o < 4; ++o) dst[o] = racc[q][o];
        }
    }
    __syncthreads();
    // ---- column pass and combination
    const T a = (T)alpha[b];
    // sums of squares of the outputs per 4-row chunk of a column (OC / 4
    // chunks per item), for the norm partials below
    static_assert(OC % 4 == 0 && TH % kNormBlock == 0 && TW % kNormBlock == 0, "norm blocks");
    double sq4[CPT][OC / 4];
#pragma unroll
    for (int q = 0; q < CPT; ++q)
#pragma unroll
        for (int c4 = 0; c4 < OC / 4; ++c4) sq4[q][c4] = 0.0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int item = tid + q * NT;
        if (item >= CITEMS) continue;
        const int ii = (item / TW) * OC, jj = item % TW;
        const int j = j0 + jj;
        T g[OC];
#pragma unroll
        for (int o = 0; o < OC; ++o) g[o] = 0;
        {
            // sliding window of OC + 4 values down the column, refilled 4 at a time
            const T* col = X + ii * XW + jj;
            T w[OC + 4];
#pragma unroll
            for (int k = 0; k < OC; ++k) w[k] = col[k * XW];
#pragma unroll
            for (int t4 = 0; t4 < TP; t4 += 4) {
#pragma unroll
                for (int k = 0; k < 4; ++k) w[OC + k] = col[(t4 + OC + k) * XW];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const T ct = taps[t4 + t];
#pragma unroll
                    for (int o = 0; o < OC; ++o) g[o] = fma(ct, w[o + t], g[o]);
                }
#pragma unroll
                for (int k = 0; k < OC; ++k) w[k] = w[4 + k];
            }
        }
        T mv[OC];
        if (m_ident) {
#pragma unroll
            for (int o = 0; o < OC; ++o) mv[o] = xc[q][o];
        } else {
            const T m0 = tm[0], m1 = tm[1], m2 = tm[2];
#pragma unroll
            for (int o = 0; o < OC; ++o) {
                const T* col = TMs + (ii + o) * TW + jj;
                mv[o] = m0 * col[0] + m1 * col[TW] + m2 * col[2 * TW];
            }
        }
#pragma unroll
        for (int o = 0; o < OC; ++o) {
            const int i = i0 + ii + o;
            if (i >= n || j >= n) continue;
            // corner rows: first and last tile rows only, computed in place
            T corr = 0;
            if (i < rc) {
                for (int p = 0; p < rc; ++p) corr += cs[i * rc + p] * X[(p - i0 + rg) * XW + jj];
            } else if (i >= n - rc) {
                const int ib = i - (n - rc);
                for (int p = 0; p < rc; ++p) corr += cs[rc2 + ib * rc + p] * X[(n - rc + p - i0 + rg) * XW + jj];
            }
            const T ax = a * mv[o] + (g[o] + corr);
            const size_t idx = (size_t)b * per + (size_t)i * n + j;
            const T r = mode == 0 ? yv[q][o] - ax : ax;
            out[idx] = r;
            sq4[q][o / 4] += (double)r * (double)r;
        }
    }
    // With part: ||out||^2 partials, one per 32 x 32 block of the image (row
    // stride (n + 31) / 32), each in one fixed order whatever the tile shape:
    // the 4-row chunk sums of the block's 8 x 32 (chunk row, column) positions
    // t = chunk row * 32 + column, added by a binary tree over t.  A 32 x 32
    // tile holds one block (thread t owns position t), a 128 x 64 tile eight,
    // so the partials of an image do not depend on the launch's tile shape.
    if (part) {
        constexpr int BX = TW / kNormBlock, NB = (TH / kNormBlock) * BX, BP = kNormBlock * kNormBlock / 4;
        __syncthreads();  // every thread is done with the staged tile
        double* red = reinterpret_cast<double*>(smem_raw);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int item = tid + q * NT;
            if (item >= CITEMS) continue;
            const int ii = (item / TW) * OC, jj = item % TW;
#pragma unroll
            for (int c4 = 0; c4 < OC / 4; ++c4) {
                const int lr = ii + 4 * c4;
                const int blk = (lr / kNormBlock) * BX + jj / kNormBlock;
                red[blk * BP + ((lr % kNormBlock) / 4) * kNormBlock + jj % kNormBlock] = sq4[q][c4];
            }
        }
        __syncthreads();
        // the tree levels h >= 64 through LDS; the last six in one wave per
        // block by cross-lane shifts (the same pairs in the same order)
        for (int h = BP / 2; h >= 64; h >>= 1) {
            for (int e = tid; e < NB * h; e += NT) {
                const int blk = e / h, t = e - blk * h;
                red[blk * BP + t] += red[blk * BP + t + h];
            }
            __syncthreads();
        }
        const int nbx = (n + kNormBlock - 1) / kNormBlock;
        const int wv = tid >> 6, ln = tid & 63;
        for (int blk = wv; blk < NB; blk += NT / 64) {
            double v = red[blk * BP + ln];
#pragma unroll
            for (int h = 32; h > 0; h >>= 1) v += __shfl_down(v, h, 64);
            const int by = i0 / kNormBlock + blk / BX, bxg = j0 / kNormBlock + blk % BX;
            if (ln == 0 && by < nbx && bxg < nbx) part[(size_t)b * nbx * nbx + (size_t)by * nbx + bxg] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Two-launch operator for long bands and for FP64: the row pass writes X G
// (and X M) for whole rows of an image to the level scratch, then a column
// pass stages 64-column strips of it (with the band's halo rows) in LDS and
// forms y - A x.  Unlike the one-launch tile kernel, no row-pass output is
// computed twice, at the price of one extra round trip of X G through
// L2 / HBM.
// ---------------------------------------------------------------------------
constexpr int kRowsPerBlock = 4;

// With dcorr: the refinement update x += ||r|| d of right-hand sides marked
// active is applied to x (in place) as the rows are staged.  Every image
// element is staged by exactly one workgroup (rows are split between them and
// a row pass needs no neighbouring rows), so each is updated once, and the
// column pass that follows reads the updated x.
template <typename T, int TP, typename D = T>
__global__ void __launch_bounds__(kBlock) k_rows_fixed(T* x, T* __restrict__ tg,
                                                       T* __restrict__ tm, const T* __restrict__ taps, int rg,
                                                       const T* __restrict__ dtl, const T* __restrict__ dbr, int rc,
                                                       const T* __restrict__ mt, int m_ident, int n,
                                                       const D* __restrict__ dcorr = nullptr,
                                                       const double* __restrict__ rn2 = nullptr,
                                                       const int* __restrict__ active = nullptr) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    T* rows = reinterpret_cast<T*>(smem_raw);
    const int LW = (n + TP + 4 + 3) & ~3;  // staged column c <-> image column c - rg
    T* cs = rows + kRowsPerBlock * LW;     // corner corrections (rc x rc each)
    const int rc2 = rc * rc;
    for (int e = threadIdx.x; e < rc2; e += kBlock) {
        cs[e] = dtl[e];
        cs[rc2 + e] = dbr[e];
    }
    const int b = blockIdx.y, r0 = blockIdx.x * kRowsPerBlock;
    const size_t per = (size_t)n * n;
    T* xs = x + (size_t)b * per;
    const bool upd = dcorr && active[b];
    const T rho = upd ? (T)sqrt(rn2[b]) : (T)0;
    // staging: wave w loads row r0 + w, lane-contiguous, eight loads per lane in flight
    {
        const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int gi = r0 + r;
        const size_t roff = (size_t)(gi < n ? gi : 0) * n;
        T* src = xs + roff;
        static_assert(kRowsPerBlock * 64 == kBlock, "one wave per staged row");
        for (int q0 = 0; q0 * 64 < LW; q0 += 8) {
            T v[8];
            D dv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = lane + 64 * (q0 + u), gj = c - rg;
                v[u] = (c < LW && gi < n && gj >= 0 && gj < n) ? src[gj] : (T)0;
            }
            // the corrections are loaded together with x (all sixteen loads
            // in flight) before any of them is used: through a buffer
            // resource over this image, where an element outside the row
            // takes an out-of-range offset and reads zero (no branch per load)
            if (upd && per * sizeof(D) < 0x7FFFFFFFu) {
                const __amdgpu_buffer_rsrc_t dres = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<D*>(dcorr + (size_t)b * per), (short)0, (int)(per * sizeof(D)), 0x00020000);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = lane + 64 * (q0 + u), gj = c - rg;
                    const bool ok = c < LW && gi < n && gj >= 0 && gj < n;
                    const int off = ok ? (int)((roff + gj) * sizeof(D)) : (int)0x80000000;
                    if constexpr (sizeof(D) == 4) {
                        dv[u] = __builtin_bit_cast(D, __builtin_amdgcn_raw_buffer_load_b32(dres, off, 0, 0));
                    } else {
                        const auto w = __builtin_amdgcn_raw_buffer_load_b64(dres, off, 0, 0);
                        __builtin_memcpy(&dv[u], &w, sizeof(D));
                    }
                }
            } else if (upd) {  // images of 2 GiB and more: plain loads
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = lane + 64 * (q0 + u), gj = c - rg;
                    dv[u] = (c < LW && gi < n && gj >= 0 && gj < n) ? dcorr[(size_t)b * per + roff + gj] : (D)0;
                }
            }
            if (upd) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = lane + 64 * (q0 + u), gj = c - rg;
                    if (c < LW && gi < n && gj >= 0 && gj < n) {
                        v[u] += rho * (T)dv[u];
                        src[gj] = v[u];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = lane + 64 * (q0 + u);
                if (c < LW) rows[r * LW + c] = v[u];
            }
        }
    }
    __syncthreads();
    const int ngrp = (n + 3) / 4;
    for (int item = threadIdx.x; item < kRowsPerBlock * ngrp; item += kBlock) {
        const int r = item / ngrp, j = (item - r * ngrp) * 4;
        const int gi = r0 + r;
        if (gi >= n) continue;
        const T* row = rows + r * LW + j;
        T acc[4] = {0, 0, 0, 0};
        T w[8];
        lds_load4v<T>(row, w);
#pragma unroll
        for (int t4 = 0; t4 < TP; t4 += 4) {
            lds_load4v<T>(row + t4 + 4, w + 4);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const T ct = taps[t4 + t];
#pragma unroll
                for (int o = 0; o < 4; ++o) acc[o] = fma(ct, w[o + t], acc[o]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = w[4 + k];
        }
        if (rc > 0 && (j < rc || j + 3 >= n - rc)) row_corners<T>(rows + r * LW, rg, cs, rc, n, j, acc);
        T* trow = tg + (size_t)b * per + (size_t)gi * n;
        for (int o = 0; o < 4; ++o)
            if (j + o < n) trow[j + o] = acc[o];  // lanes write consecutive 4-value runs
        if (!m_ident) {
            T* mrow = tm + (size_t)b * per + (size_t)gi * n;
            for (int o = 0; o < 4; ++o)
                if (j + o < n) mrow[j + o] = mt[0] * row[rg - 1 + o] + mt[1] * row[rg + o] + mt[2] * row[rg + 1 + o];
        }
    }
}

// With part: this tile's sum of squares of its outputs (FP64, fixed order:
// each thread's rows in order, then a fixed tree over the threads) goes to
// part[b * kNormChunks + tile], the first stage of ||out||^2 with a partial
// layout that depends only on the level size.
template <typename T, int TP, int TW = 64>
__global__ void __launch_bounds__(kBlock) k_cols_fixed(const T* __restrict__ tg, const T* __restrict__ tm,
                                                       const T* __restrict__ x, const T* __restrict__ y,
                                                       T* __restrict__ out, const double* __restrict__ alpha, int n,
                                                       int mode, const T* __restrict__ taps, int rg,
                                                       const T* __restrict__ dtl, const T* __restrict__ dbr, int rc,
                                                       const T* __restrict__ mt, int m_ident, int tiles_x,
                                                       double* __restrict__ part = nullptr) {
    // TH x TW tile, TW columns x (TH / OC) row groups of threads: OC = 16 rows
    // each for 64 columns, 8 for 32 (more, smaller workgroups)
    constexpr int TH = 64, OC = TH * TW / kBlock;
    static_assert(OC * kBlock == TH * TW && OC % 4 == 0, "column-pass tile");
    constexpr int XH = TH + TP;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    T* G = reinterpret_cast<T*>(smem_raw);    // [XH][TW]: row r <-> image row i0 - rg + r
    T* Ms = G + XH * TW;                      // [TH + 4][TW]: row r <-> image row i0 - 1 + r
    T* cs = Ms + (m_ident ? 0 : (TH + 4) * TW);  // corner corrections (rc x rc each)
    const int rc2 = rc * rc;
    int bx, b;
    xcd_major(bx, b);
    // FP64: tiles numbered column-major, so the tiles that share a column
    // strip's halo rows (the pass has no horizontal halo) get consecutive
    // numbers and run together on one XCD, whose L2 serves the overlap; one
    // 117 KB workgroup per CU sweeping row-major evicts the halo before the
    // next tile row reads it (2047^2, radius 82: 1.67x the algorithmic bytes
    // row-major, 1.20x column-major).  FP32 (two workgroups per CU) keeps the
    // previous tile rows in L2 and does better row-major (1.07x against 1.21x).
    int i0, j0;
    if constexpr (sizeof(T) == 8) {
        const int tiles_y = (n + TH - 1) / TH;
        i0 = (bx % tiles_y) * TH;
        j0 = (bx / tiles_y) * TW;
    } else {
        i0 = (bx / tiles_x) * TH;
        j0 = (bx % tiles_x) * TW;
    }
    const size_t per = (size_t)n * n;
    const T* tgs = tg + (size_t)b * per;
    const int tid = threadIdx.x;
    // staging in batches of 16 loads per thread in flight (one batch for the
    // 44-tap band); the corner corrections go to LDS between the first
    // batch's loads and stores
    constexpr int SBT = 16;
    bool corners = false;
    for (int e0 = tid; e0 < XH * TW; e0 += SBT * kBlock) {
        T v[SBT];
#pragma unroll
        for (int u = 0; u < SBT; ++u) {
            const int e = e0 + u * kBlock;
            const int r = e / TW, c = e - r * TW;
            const int gi = i0 - rg + r, gj = j0 + c;
            v[u] = (e < XH * TW && gi >= 0 && gi < n && gj < n) ? tgs[(size_t)gi * n + gj] : (T)0;
        }
        if (!corners) {
            corners = true;
            for (int e = tid; e < rc2; e += kBlock) {
                cs[e] = dtl[e];
                cs[rc2 + e] = dbr[e];
            }
        }
#pragma unroll
        for (int u = 0; u < SBT; ++u)
            if (e0 + u * kBlock < XH * TW) G[e0 + u * kBlock] = v[u];
    }
    if (!corners)  // (a thread without a staging batch)
        for (int e = tid; e < rc2; e += kBlock) {
            cs[e] = dtl[e];
            cs[rc2 + e] = dbr[e];
        }
    if (!m_ident) {
        const T* tms = tm + (size_t)b * per;
        for (int e = tid; e < (TH + 4) * TW; e += kBlock) {
            const int r = e / TW, c = e - r * TW;
            const int gi = i0 - 1 + r, gj = j0 + c;
            Ms[e] = (r < TH + 2 && gi >= 0 && gi < n && gj < n) ? tms[(size_t)gi * n + gj] : (T)0;
        }
    }
    __syncthreads();
    const int jj = tid % TW, ii = (tid / TW) * OC;
    const int j = j0 + jj;
    // (threads of columns beyond n compute on zeros and store nothing: every
    // thread reaches the partial-sum barrier below)
    const bool colok = j < n;
    // the right-hand side (and x for M = I) of this thread's outputs, loaded before the pass
    T yv[OC], xv[OC];
#pragma unroll
    for (int o = 0; o < OC; ++o) {
        const int i = i0 + ii + o;
        const size_t idx = (size_t)b * per + (size_t)i * n + j;
        yv[o] = (mode == 0 && colok && i < n) ? y[idx] : (T)0;
        xv[o] = (m_ident && colok && i < n) ? x[idx] : (T)0;
    }
    T g[OC];
#pragma unroll
    for (int o = 0; o < OC; ++o) g[o] = 0;
    {
        const T* col = G + ii * TW + jj;
        T w[OC + 4];
#pragma unroll
        for (int k = 0; k < OC; ++k) w[k] = col[k * TW];
        // bands beyond 32 padded taps: 16 taps per unrolled body (fully
        // unrolled, the compiler holds every tap in scalar registers and
        // spills them: 44 FP64 taps took 204 VGPRs and two waves per SIMD, 164
        // FP32 taps 256 and one; unrolled four times, 130 and 82)
#pragma unroll(TP > 32 ? 4 : TP / 4)
        for (int t4 = 0; t4 < TP; t4 += 4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) w[OC + k] = col[(t4 + OC + k) * TW];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const T ct = taps[t4 + t];
#pragma unroll
                for (int o = 0; o < OC; ++o) g[o] = fma(ct, w[o + t], g[o]);
            }
#pragma unroll
            for (int k = 0; k < OC; ++k) w[k] = w[4 + k];
        }
    }
    const T a = (T)alpha[b];
    double sq = 0.0;
#pragma unroll
    for (int o = 0; o < OC; ++o) {
        const int i = i0 + ii + o;
        if (i >= n || !colok) break;
        // corner rows occur only in the first and last tile rows, for a quarter of
        // the threads; computed in place they cost no registers elsewhere
        T corr = 0;
        if (i < rc) {
            for (int p = 0; p < rc; ++p) corr += cs[i * rc + p] * G[(p - i0 + rg) * TW + jj];
        } else if (i >= n - rc) {
            const int ib = i - (n - rc);
            for (int p = 0; p < rc; ++p) corr += cs[rc2 + ib * rc + p] * G[(n - rc + p - i0 + rg) * TW + jj];
        }
        const size_t idx = (size_t)b * per + (size_t)i * n + j;
        T mv;
        if (m_ident) {
            mv = xv[o];
        } else {
            const T* c = Ms + (ii + o) * TW + jj;
            mv = mt[0] * c[0] + mt[1] * c[TW] + mt[2] * c[2 * TW];
        }
        const T ax = a * mv + (g[o] + corr);
        const T r = mode == 0 ? yv[o] - ax : ax;
        out[idx] = r;
        sq += (double)r * (double)r;
    }
    if (part) {
        __syncthreads();  // every thread is done with the staged tile
        double* red = reinterpret_cast<double*>(smem_raw);
        red[tid] = sq;
        __syncthreads();
        const double tot = tree_sum<kBlock, kBlock>(red, tid);
        if (tid == 0) part[(size_t)b * kNormChunks + bx] = tot;
    }
}

}  // namespace

size_t level_elems(const Ctx* c, int l) { return (size_t)(c->p.dim == 2 ? c->n[l] : 1) * c->n[l]; }

template <typename T>
constexpr int tile_w() { return sizeof(T) == 4 ? 64 : 32; }
template <typename T>
constexpr int tile_h() { return 64; }

template <typename T>
nmg_status launch_operator(const Ctx* c, int l, int batch, const double* alpha, const T* x, const T* y, T* out,
                           int mode, Work<T>& w, hipStream_t s, double* norm_part, int* nparts) {
    const int n = c->n[l];
    if (nparts) *nparts = 0;
    const size_t per = level_elems(c, l);
    const HostLevel& hl = c->host[l];
    const TiledOp<T>& op = w.tiled[(size_t)l];
    // FP64 (the refinement residual) and bands longer than 48 taps: two launches
    // (row pass through the level scratch, then the column pass)
    if (c->p.dim == 2 && op.ok && (op.m_ident || op.rm == 1) && (sizeof(T) == 8 || op.rgp > 48)) {
        bool launched = false;
        auto go2 = [&](auto tp_tag) {
            constexpr int TP = decltype(tp_tag)::value;
            if (launched || op.rgp != TP) return;
            launched = true;
            T* tg = w.lv[l].t1;
            T* tm = w.lv[l].t2;
            const int LW = (n + TP + 4 + 3) & ~3;
            // (no update: x is only read)
            hipLaunchKernelGGL((k_rows_fixed<T, TP>), dim3((n + kRowsPerBlock - 1) / kRowsPerBlock, batch),
                               dim3(kBlock), ((size_t)kRowsPerBlock * LW + 2 * (size_t)op.rc * op.rc) * sizeof(T), s,
                               const_cast<T*>(x), tg, tm, op.tg, op.rg, op.dtl, op.dbr, op.rc, op.tm, op.m_ident, n,
                               (const T*)nullptr, (const double*)nullptr, (const int*)nullptr);
            // FP64 and long bands (84 and 164 padded taps): 32-column strips, half
            // the LDS and registers of 64 columns at the same halo share, so more
            // workgroups per CU hide the staging latency that bounds this pass
            // (FP64 at 64 columns holds 202-251 VGPRs, two waves per SIMD; every
            // output's taps are added in the same order either way)
            constexpr int CW = (sizeof(T) == 8 || TP >= 84) ? 32 : 64;
            const int tiles_x = (n + CW - 1) / CW, tiles_y = (n + 63) / 64;
            const size_t lds = ((size_t)(64 + TP) * CW + (op.m_ident ? 0 : (size_t)68 * CW) +
                                2 * (size_t)op.rc * op.rc) * sizeof(T);
            hipLaunchKernelGGL((k_cols_fixed<T, TP, CW>), dim3(tiles_x * tiles_y, batch), dim3(kBlock), lds, s, tg,
                               tm, x, y, out, alpha, n, mode, op.tg, op.rg, op.dtl, op.dbr, op.rc, op.tm, op.m_ident,
                               tiles_x, (double*)nullptr);
        };
        go2(std::integral_constant<int, 8>{});
        go2(std::integral_constant<int, 12>{});
        go2(std::integral_constant<int, 16>{});
        go2(std::integral_constant<int, 20>{});
        go2(std::integral_constant<int, 24>{});
        go2(std::integral_constant<int, 28>{});
        go2(std::integral_constant<int, 32>{});
        go2(std::integral_constant<int, 36>{});
        go2(std::integral_constant<int, 40>{});
        go2(std::integral_constant<int, 44>{});
        go2(std::integral_constant<int, 48>{});
        go2(std::integral_constant<int, 84>{});
        go2(std::integral_constant<int, 164>{});
        if (launched) {
            NMG_HIP(hipGetLastError());
            return NMG_OK;
        }
    }
    if (c->p.dim == 2 && op.ok && op.rgp <= 48 && (op.m_ident || op.rm == 1)) {
        // fixed-tap kernel: TP = padded Toeplitz taps of G_l
        bool launched = false;
        // FP32: 128 x 64 tiles (512 threads, 4 waves per SIMD) when they give at
        // least 512 workgroups, else 32 x 32 tiles (256 threads) for more
        // parallelism at small batches and on coarse levels (64 x 64 tiles with
        // 256 threads, measured on level 1 at about 30 right-hand sides, took
        // 32 us against 21 us); FP64: 32 x 32 tiles
        const bool big = sizeof(T) == 4 && (long)((n + 63) / 64) * ((n + 127) / 128) * batch >= 512;
        auto launch = [&](auto cfg_tag, auto tp_tag) {
            constexpr int TP = decltype(tp_tag)::value;
            constexpr int CFG = decltype(cfg_tag)::value;  // 2: 128 x 64, 0: 32 x 32
            constexpr int TH = CFG == 2 ? 128 : 32, TW = CFG == 2 ? 64 : 32;
            constexpr int OC = CFG == 2 ? 8 : 4, NT = CFG == 2 ? 512 : 256;
            constexpr int WPE = CFG == 2 ? 4 : 1;
            const int tiles_x = (n + TW - 1) / TW, tiles_y = (n + TH - 1) / TH;
            size_t lds = ((size_t)(TH + TP) * (TW + TP) + (op.m_ident ? 0 : (size_t)(TH + 4) * TW) +
                          2 * (size_t)op.rc * op.rc) * sizeof(T);
            // the norm partials reuse the tile's LDS: (TH / 32) * (TW / 32) blocks of 256 doubles
            const int nb = (n + kNormBlock - 1) / kNormBlock;
            double* part = norm_part && nparts && nb * nb <= kResidualNormParts ? norm_part : nullptr;
            if (part) {
                lds = std::max(lds, (size_t)(TH / kNormBlock) * (TW / kNormBlock) * kNormBlock * kNormBlock / 4 *
                                        sizeof(double));
                *nparts = nb * nb;
            }
            hipLaunchKernelGGL((k_residual_fixed<T, TH, TW, TP, OC, NT, WPE>), dim3(tiles_x * tiles_y, batch), dim3(NT),
                               lds, s, x, y, out, alpha, n, mode, op.tg, op.rg, op.dtl, op.dbr, op.rc, op.tm,
                               op.m_ident, tiles_x, part);
        };
        auto go = [&](auto tp_tag) {
            constexpr int TP = decltype(tp_tag)::value;
            if (launched || op.rgp != TP) return;
            launched = true;
            if constexpr (sizeof(T) == 4) {
                if (big) {
                    launch(std::integral_constant<int, 2>{}, tp_tag);
                    return;
                }
            }
            launch(std::integral_constant<int, 0>{}, tp_tag);
        };
        go(std::integral_constant<int, 4>{});
        go(std::integral_constant<int, 8>{});
        go(std::integral_constant<int, 12>{});
        go(std::integral_constant<int, 16>{});
        go(std::integral_constant<int, 20>{});
        go(std::integral_constant<int, 24>{});
        go(std::integral_constant<int, 28>{});
        go(std::integral_constant<int, 32>{});
        go(std::integral_constant<int, 36>{});
        go(std::integral_constant<int, 40>{});
        go(std::integral_constant<int, 44>{});
        go(std::integral_constant<int, 48>{});
        if (launched) {
            NMG_HIP(hipGetLastError());
            return NMG_OK;
        }
    }
    if (c->p.dim == 2 && op.ok && op.fused_ok) {
        constexpr int TH = tile_h<T>(), TW = tile_w<T>();
        const int tiles_x = (n + TW - 1) / TW, tiles_y = (n + TH - 1) / TH;
        const int XW = TW + op.rgp, XH = TH + 2 * op.rg, GH = TH + op.rgp, MH = TH + op.rmp;
        const size_t lds = ((size_t)XH * XW + (size_t)GH * TW + (op.m_ident ? 0 : (size_t)MH * TW)) * sizeof(T);
        hipLaunchKernelGGL((k_residual_tiled<T, TH, TW>), dim3(tiles_x * tiles_y, batch), dim3(kBlock), lds, s, x, y,
                           out, alpha, n, mode, op.tg, op.rg, op.rgp, op.dtl, op.dbr, op.rc, op.tm, op.rm, op.rmp,
                           op.m_ident, tiles_x);
        NMG_HIP(hipGetLastError());
        return NMG_OK;
    }
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

// The FP64 refinement residual of one outer iteration, fused: x += ||r|| d
// for active right-hand sides inside the row pass, r = y - A x with the first
// stage of ||r||^2 in the column pass, then the per-image sums.  Returns
// false (and launches nothing) where the two-launch tile form does not apply
// or the partials would not fit; the caller then runs the separate kernels.
// The refinement residual's column pass runs on 64 x 32 tiles (8 rows per
// thread): twice the workgroups of 64 x 64 tiles at half the LDS each, for a
// pass that is bound by latency at the batch sizes of a solve's tail.
constexpr int kRefineTW = 32;

bool refine_residual_fusable(const Ctx* c, const Work<double>& w) {
    const int n = c->n[0];
    const TiledOp<double>& op = w.tiled[0];
    const int tiles = ((n + kRefineTW - 1) / kRefineTW) * ((n + 63) / 64);
    static const int kTaps[] = {8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 84, 164};
    bool tp_ok = false;
    for (int t : kTaps) tp_ok = tp_ok || op.rgp == t;
    return c->p.dim == 2 && op.ok && op.m_ident && tp_ok && tiles <= kNormChunks;
}

template <typename D>
bool launch_refine_residual(const Ctx* c, int batch, const double* alpha, double* x, const D* d,
                            const double* rn2, const int* active, const double* y, double* out, double* nrm2,
                            Work<double>& w, hipStream_t s, double* mirror) {
    const int l = 0, n = c->n[l];
    const TiledOp<double>& op = w.tiled[(size_t)l];
    const int tiles_x = (n + kRefineTW - 1) / kRefineTW, tiles = tiles_x * ((n + 63) / 64);
    if (!refine_residual_fusable(c, w)) return false;
    bool launched = false;
    auto go = [&](auto tp_tag) {
        constexpr int TP = decltype(tp_tag)::value;
        if (launched || op.rgp != TP) return;
        launched = true;
        double* tg = w.lv[l].t1;
        const int LW = (n + TP + 4 + 3) & ~3;
        hipLaunchKernelGGL((k_rows_fixed<double, TP, D>), dim3((n + kRowsPerBlock - 1) / kRowsPerBlock, batch),
                           dim3(kBlock), ((size_t)kRowsPerBlock * LW + 2 * (size_t)op.rc * op.rc) * sizeof(double), s,
                           x, tg, (double*)nullptr, op.tg, op.rg, op.dtl, op.dbr, op.rc, op.tm, op.m_ident, n, d, rn2,
                           active);
        const size_t lds = ((size_t)(64 + TP) * kRefineTW + 2 * (size_t)op.rc * op.rc) * sizeof(double);
        hipLaunchKernelGGL((k_cols_fixed<double, TP, kRefineTW>), dim3(tiles, batch), dim3(kBlock), lds, s, tg,
                           (const double*)nullptr, x, y, out, alpha, n, 0, op.tg, op.rg, op.dtl, op.dbr, op.rc, op.tm,
                           op.m_ident, tiles_x, c->norm_part);
        hipLaunchKernelGGL(k_sumsq_final, dim3((batch + 63) / 64), dim3(64), 0, s, c->norm_part, nrm2, batch, tiles,
                           kNormChunks, mirror);
    };
    go(std::integral_constant<int, 8>{});
    go(std::integral_constant<int, 12>{});
    go(std::integral_constant<int, 16>{});
    go(std::integral_constant<int, 20>{});
    go(std::integral_constant<int, 24>{});
    go(std::integral_constant<int, 28>{});
    go(std::integral_constant<int, 32>{});
    go(std::integral_constant<int, 36>{});
    go(std::integral_constant<int, 40>{});
    go(std::integral_constant<int, 44>{});
    go(std::integral_constant<int, 48>{});
    go(std::integral_constant<int, 84>{});
    go(std::integral_constant<int, 164>{});
    return launched;
}
template bool launch_refine_residual<float>(const Ctx*, int, const double*, double*, const float*, const double*,
                                            const int*, const double*, double*, double*, Work<double>&, hipStream_t,
                                            double*);
template bool launch_refine_residual<double>(const Ctx*, int, const double*, double*, const double*, const double*,
                                             const int*, const double*, double*, double*, Work<double>&, hipStream_t,
                                             double*);

template <typename T>
nmg_status launch_sumsq_part(const Ctx* c, int batch, size_t elems, const T* v, hipStream_t s) {
    hipLaunchKernelGGL(k_sumsq_part<T>, dim3((unsigned)norm_chunks(elems), batch), dim3(kBlock), 0, s, v,
                       c->norm_part, elems);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_sumsq(const Ctx* c, int batch, size_t elems, const T* v, double* out, hipStream_t s,
                        double* mirror) {
    double* part = c->norm_part;
    const int nch = norm_chunks(elems);
    hipLaunchKernelGGL(k_sumsq_part<T>, dim3((unsigned)nch, batch), dim3(kBlock), 0, s, v, part, elems);
    hipLaunchKernelGGL(k_sumsq_final, dim3((batch + 63) / 64), dim3(64), 0, s, part, out, batch, nch, nch, mirror);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

int restrict_norm_parts(const Ctx* c, int l) {
    return (int)std::min<unsigned>(blocks_for(level_elems(c, l + 1)), (unsigned)kNormChunksPerRhs);
}

template <typename T>
nmg_status launch_restrict(const Ctx* c, int l, int batch, const T* r, T* yc, hipStream_t s, double* norm_part) {
    const int nf = c->n[l], nc = c->n[l + 1];
    const size_t perc = level_elems(c, l + 1);
    // with partial sums: at most kNormChunksPerRhs blocks per image, grid-stride
    const unsigned gx = norm_part ? (unsigned)restrict_norm_parts(c, l) : blocks_for(perc);
    hipLaunchKernelGGL(k_restrict<T>, dim3(gx, batch), dim3(kBlock), 0, s, r, yc, nf, nc, c->p.dim == 2 ? 1 : 0,
                       (T)1, norm_part);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

// P^T g = 2^d R g: the adjoint of linear interpolation (weights 1/2, 1, 1/2).
template <typename T>
nmg_status launch_prolong_transpose(const Ctx* c, int l, int batch, const T* g, T* out, hipStream_t s) {
    const int nf = c->n[l], nc = c->n[l + 1];
    const size_t perc = level_elems(c, l + 1);
    hipLaunchKernelGGL(k_restrict<T>, dim3(blocks_for(perc), batch), dim3(kBlock), 0, s, g, out, nf, nc,
                       c->p.dim == 2 ? 1 : 0, (T)(c->p.dim == 2 ? 4 : 2), (double*)nullptr);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_prolong_add(const Ctx* c, int l, int batch, const T* e, T* x, hipStream_t s, bool set) {
    const int nf = c->n[l], nc = c->n[l + 1];
    const size_t perf = level_elems(c, l);
    hipLaunchKernelGGL(k_prolong_add<T>, dim3(blocks_for(perf), batch), dim3(kBlock), 0, s, e, x, nf, nc,
                       c->p.dim == 2 ? 1 : 0, set ? 1 : 0);
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
                                           Work<T>&, hipStream_t, double*, int*);                                \
    template nmg_status launch_sumsq<T>(const Ctx*, int, size_t, const T*, double*, hipStream_t, double*);                \
    template nmg_status launch_sumsq_part<T>(const Ctx*, int, size_t, const T*, hipStream_t);                    \
    template nmg_status launch_restrict<T>(const Ctx*, int, int, const T*, T*, hipStream_t, double*);            \
    template nmg_status launch_prolong_transpose<T>(const Ctx*, int, int, const T*, T*, hipStream_t);            \
    template nmg_status launch_prolong_add<T>(const Ctx*, int, int, const T*, T*, hipStream_t, bool);            \
    template nmg_status launch_axpy<T>(int, size_t, const T*, T*, int, hipStream_t);                             \
    template nmg_status launch_zero<T>(T*, size_t, hipStream_t);
NMG_INST(float)
NMG_INST(double)
#undef NMG_INST
template nmg_status launch_zero<int>(int*, size_t, hipStream_t);
template nmg_status launch_convert<float, double>(const float*, double*, size_t, hipStream_t);
template nmg_status launch_convert<double, float>(const double*, float*, size_t, hipStream_t);

}  // namespace nmg
