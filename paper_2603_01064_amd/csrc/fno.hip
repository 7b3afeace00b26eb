// Fourier-neural-operator smoother h = ||b|| N(b / ||b||) (Sec. 3.1; the
// appendix's network description): pointwise lift 1 -> C with bias, Fourier
// layers z <- GELU(DFT^-1 R DFT z + W z + B), pointwise projection C -> 1.
//
// Only the k lowest modes per axis are kept, so the transforms are evaluated
// as truncated DFT sums instead of full FFTs:
//   A (columns, 2D and 1D): T[x][j] = sum_y z[x][y] cos(2 pi j y / n) (j < k)
//                          and -sum_y z[x][y] sin(2 pi (j-k) y / n)   (j >= k)
//   B (rows, 2D): X[u][v] = sum_x e^{-2 pi i u x / n} T[x][v] for the 2k rows
//                          u in [0, k) and [n - k, n)
//   mix:          Y[co] = sum_ci X[ci] R[ci][co] per retained mode
//   D (rows, 2D): c[x][v] = (1/n) sum_u Y[u][v] e^{+2 pi i u x / n}
//   E (columns, fused into the layer's output kernel):
//                 s[x][y] = (1/n) sum_v w_v (Re c_v cos - Im c_v sin)(2 pi v y / n)
//                 with w_0 = 1 and w_v = 2 (the real inverse of a half spectrum)
// Twiddles come from one table of cos / sin (2 pi q / n), q < n, per level,
// indexed by (index product) mod n, so no angle is ever large.
// Activations are [B][C][ny][n] in the cycle's precision; weights follow the
// flat block layout documented with nmg_smoother_arch.
#include <cmath>
#include <type_traits>

#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kBlock = 256;
typedef float floatx4 __attribute__((ext_vector_type(4)));

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename T>
nmg_status falloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return NMG_OK;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(NMG_ERR_OOM, std::string("hipMalloc failed for FNO buffers: ") + hipGetErrorString(e));
    }
    return NMG_OK;
}

template <typename T>
__device__ inline T gelu(T x) {
    return (T)0.5 * x * ((T)1 + erf(x * (T)0.70710678118654752440));
}

struct FnoDims {
    int C, NL, m, ks, kk, dim;  // m = stored modes
    size_t rm, layer_stride;
};

inline FnoDims fno_dims(const Ctx* c) {
    FnoDims d;
    d.C = c->p.fno_width;
    d.NL = c->p.fno_layers;
    d.m = c->p.fno_modes;
    d.ks = c->p.fno_ksize;
    d.dim = c->p.dim;
    d.kk = d.dim == 2 ? d.ks * d.ks : d.ks;
    d.rm = d.dim == 2 ? (size_t)2 * d.C * d.C * d.m * d.m : (size_t)d.C * d.C * d.m;
    d.layer_stride = 2 * d.rm + (size_t)d.C * d.C * d.kk + d.C;
    return d;
}

template <typename T>
__device__ inline const T* set_block(const T* wl, size_t stride, const int* ws, int nsets, int img) {
    const int set = ws ? min(max(ws[img], 0), nsets - 1) : 0;
    return wl + (size_t)set * stride;
}

// z[b][c][p] = lift_w[c] * b[p] / ||b|| + lift_b[c]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_lift(const T* __restrict__ bres, const double* __restrict__ nrm2,
                                                     T* __restrict__ z, const T* __restrict__ wl, size_t stride,
                                                     const int* __restrict__ ws, int nsets, int C, size_t per) {
    const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int img = blockIdx.y;
    if (p >= per) return;
    const T* w = set_block(wl, stride, ws, nsets, img);
    const double q = nrm2[img];
    const T u = q > 0.0 ? (T)(bres[(size_t)img * per + p] / sqrt(q)) : (T)0;
    for (int c = 0; c < C; ++c) z[((size_t)img * C + c) * per + p] = w[c] * u + w[C + c];
}

// step A: one block per row (image, channel, x); thread j < 2k
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_dft_cols(const T* __restrict__ z, T* __restrict__ ta,
                                                         const T* __restrict__ cs, const T* __restrict__ sn, int n,
                                                         int k) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    T* row = reinterpret_cast<T*>(smem_raw);
    const size_t r = blockIdx.x;
    for (int y = threadIdx.x; y < n; y += kBlock) row[y] = z[r * n + y];
    __syncthreads();
    const int j = threadIdx.x;
    if (j >= 2 * k) return;
    const int f = j < k ? j : j - k;
    T acc = 0;
    int q = 0;  // f * y mod n
    for (int y = 0; y < n; ++y) {
        acc += row[y] * (j < k ? cs[q] : -sn[q]);
        q += f;
        if (q >= n) q -= n;
    }
    ta[r * 2 * k + j] = acc;
}

// step B (2D): X[img][c][u'][v] (re, im) for u' < 2k, v < k
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_dft_rows(const T* __restrict__ ta, T* __restrict__ xh,
                                                         const T* __restrict__ cs, const T* __restrict__ sn, int n,
                                                         int k, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    const int v = (int)(e % k);
    const int up = (int)((e / k) % (2 * k));
    const size_t bc = e / ((size_t)2 * k * k);
    const int u = up < k ? up : n - 2 * k + up;
    const T* t = ta + bc * (size_t)n * 2 * k;
    T xr = 0, xi = 0;
    int q = 0;
    for (int x = 0; x < n; ++x) {
        const T tr = t[(size_t)x * 2 * k + v], ti = t[(size_t)x * 2 * k + k + v];
        const T c = cs[q], s = sn[q];
        xr += c * tr + s * ti;
        xi += c * ti - s * tr;
        q += u;
        if (q >= n) q -= n;
    }
    xh[2 * e] = xr;
    xh[2 * e + 1] = xi;
}

// 1D: X[v] = T[v] + i T[k + v] laid out as (re, im) pairs
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_interleave(const T* __restrict__ ta, T* __restrict__ xh, int k,
                                                           size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    const size_t bc = e / k;
    const int v = (int)(e % k);
    xh[2 * e] = ta[bc * 2 * k + v];
    xh[2 * e + 1] = ta[bc * 2 * k + k + v];
}

// mode mixing: Y[img][co][mode] = sum_ci X[img][ci][mode] R[..ci][co][mode]
//   2D: mode = (u' < 2k, v < k), R index [corner][ci][co][u' mod k][v] with the
//       stored mode count m as the pitch; 1D: mode = v < k, R index [ci][co][v]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_mix(const T* __restrict__ xh, T* __restrict__ yh,
                                                    const T* __restrict__ wl, size_t stride, size_t r_off,
                                                    size_t rm, const int* __restrict__ ws, int nsets, int C, int k,
                                                    int m, int two_d, size_t modes, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    const size_t md = e % modes;
    const int co = (int)((e / modes) % C);
    const int img = (int)(e / (modes * C));
    const T* w = set_block(wl, stride, ws, nsets, img) + r_off;
    size_t ridx_base, cstride;
    if (two_d) {
        const int v = (int)(md % k), up = (int)(md / k);
        const int corner = up < k ? 0 : 1, u = up < k ? up : up - k;
        ridx_base = ((size_t)corner * C * C + co) * m * m + (size_t)u * m + v;  // + ci * C * m * m
        cstride = (size_t)C * m * m;
    } else {
        ridx_base = (size_t)co * m + md;  // + ci * C * m
        cstride = (size_t)C * m;
    }
    T yr = 0, yi = 0;
    for (int ci = 0; ci < C; ++ci) {
        const size_t xi_ = (((size_t)img * C + ci) * modes + md) * 2;
        const T ar = xh[xi_], ai = xh[xi_ + 1];
        const T rr = w[ridx_base + ci * cstride], ri = w[rm + ridx_base + ci * cstride];
        yr += ar * rr - ai * ri;
        yi += ar * ri + ai * rr;
    }
    yh[2 * e] = yr;
    yh[2 * e + 1] = yi;
}

// C[M x N] = A[M x K] B[K x N], row-major, 64 x 64 output tile per workgroup,
// 4 x 4 outputs per thread, K staged 16 at a time in LDS.  Used for the
// column transforms, whose twiddles form a dense [n x 2k] (forward) or
// [2k x n] (inverse) matrix per level.
template <typename T>
__global__ void __launch_bounds__(256) k_gemm_rm(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C,
                                                 int M, int N, int K, int transB = 0) {
    __shared__ T As[16][64 + 1], Bs[16][64 + 1];
    const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
    const size_t m0 = (size_t)blockIdx.x * 64;
    const int n0 = blockIdx.y * 64;
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = tid; e < 16 * 64; e += 256) {
            const int kk = e % 16, mm = e / 16;  // A tile: 64 rows x 16 columns
            const size_t gm = m0 + mm;
            As[kk][mm] = (gm < (size_t)M && k0 + kk < K) ? A[gm * K + k0 + kk] : (T)0;
            const int kb = e / 64, nn = e % 64;  // B tile: 16 rows x 64 columns
            Bs[kb][nn] = (k0 + kb < K && n0 + nn < N)
                             ? (transB ? B[(size_t)(n0 + nn) * K + k0 + kb] : B[(size_t)(k0 + kb) * N + n0 + nn])
                             : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tr * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const size_t gm = m0 + tr * 4 + i;
        if (gm >= (size_t)M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tc * 4 + j;
            if (gn < N) C[gm * N + gn] = acc[i][j];
        }
    }
}

// step D (2D) in split layout for the GEMM inverse: cd[row][v] = Re c_v and
// cd[row][k + v] = Im c_v with c_v(x) = (1/n) sum_u' Y[u'][v] e^{+2 pi i u x / n}
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_idft_rows_split(const T* __restrict__ yh, T* __restrict__ cd,
                                                                const T* __restrict__ cs, const T* __restrict__ sn,
                                                                int n, int k, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    const int v = (int)(e % k);
    const size_t row = e / k;  // (img, co, x)
    const int x = (int)(row % n);
    const size_t bc = row / n;
    const T* y = yh + bc * (size_t)2 * k * k * 2;
    T cr = 0, ci = 0;
    for (int up = 0; up < 2 * k; ++up) {
        const int u = up < k ? up : n - 2 * k + up;
        const int q = (int)(((long long)u * x) % n);
        const T c = cs[q], s = sn[q];
        const T yr = y[((size_t)up * k + v) * 2], yi = y[((size_t)up * k + v) * 2 + 1];
        cr += yr * c - yi * s;
        ci += yr * s + yi * c;
    }
    const T inv = (T)1 / (T)n;
    cd[row * 2 * k + v] = cr * inv;
    cd[row * 2 * k + k + v] = ci * inv;
}

// step D (2D): c[img][co][x][v] = (1/n) sum_u' Y[u'][v] e^{+2 pi i u x / n}
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_idft_rows(const T* __restrict__ yh, T* __restrict__ cd,
                                                          const T* __restrict__ cs, const T* __restrict__ sn, int n,
                                                          int k, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    const int v = (int)(e % k);
    const int x = (int)((e / k) % n);
    const size_t bc = e / ((size_t)n * k);
    const T* y = yh + bc * (size_t)2 * k * k * 2;
    T cr = 0, ci = 0;
    for (int up = 0; up < 2 * k; ++up) {
        const int u = up < k ? up : n - 2 * k + up;
        const int q = (int)(((long long)u * x) % n);
        const T c = cs[q], s = sn[q];
        const T yr = y[((size_t)up * k + v) * 2], yi = y[((size_t)up * k + v) * 2 + 1];
        cr += yr * c - yi * s;
        ci += yr * s + yi * c;
    }
    const T inv = (T)1 / (T)n;
    cd[2 * e] = cr * inv;
    cd[2 * e + 1] = ci * inv;
}

// Output of one Fourier layer: z1 = GELU(s + W z0 + B) with the spectral part
// s from step E.  cd holds c[img][co][x][v] (2D) or Y[img][co][v] (1D).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_layer_out(const T* __restrict__ z0, T* __restrict__ z1,
                                                          const T* __restrict__ cd, const T* __restrict__ wl,
                                                          size_t stride, size_t w_off, const int* __restrict__ ws,
                                                          int nsets, const T* __restrict__ cs,
                                                          const T* __restrict__ sn, int C, int ks, int ny, int n,
                                                          int k) {
    const size_t per = (size_t)ny * n;
    const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int co = blockIdx.y, img = blockIdx.z;
    if (p >= per) return;
    const int x = (int)(p / n), y = (int)(p % n);
    const T* w = set_block(wl, stride, ws, nsets, img) + w_off;
    const int kh = ny > 1 ? ks : 1, kw = ks;
    const T* Wc = w + (size_t)co * C * kh * kw;
    const T bias = w[(size_t)C * C * kh * kw + co];
    // spectral part
    const T* c = cd + (((size_t)img * C + co) * ny + x) * (size_t)k * 2;
    T s = 0;
    int q = 0;
    for (int v = 0; v < k; ++v) {
        const T term = c[2 * v] * cs[q] - c[2 * v + 1] * sn[q];
        s += v == 0 ? term : (T)2 * term;
        q += y;
        if (q >= n) q -= n;
    }
    s *= (T)1 / (T)n;
    // convolution (cross-correlation, zero "same" padding)
    T acc = 0;
    const int py = kh / 2, px = kw / 2;
    for (int ci = 0; ci < C; ++ci) {
        const T* zc = z0 + ((size_t)img * C + ci) * per;
        const T* wc = Wc + (size_t)ci * kh * kw;
        for (int dy = 0; dy < kh; ++dy) {
            const int yy = x + dy - py;
            if (yy < 0 || yy >= ny) continue;
            for (int dx = 0; dx < kw; ++dx) {
                const int xx = y + dx - px;
                if (xx < 0 || xx >= n) continue;
                acc += wc[dy * kw + dx] * zc[(size_t)yy * n + xx];
            }
        }
    }
    z1[((size_t)img * C + co) * per + p] = gelu(s + acc + bias);
}

// 2D Fourier-layer output on a 16 x 16 pixel tile for TCO output channels:
// the input tile plus a ks/2 halo is staged in LDS a few input channels at a
// time; each thread owns one pixel and TCO accumulators, and the weights of
// a (channel, tap) step are uniform across the workgroup, so they are read
// through scalar loads and used as scalar operands of the FMAs.
constexpr int kFT = 16;   // tile side
constexpr int kFCI = 8;   // input channels staged per step

template <typename T, int TCO>
__global__ void __launch_bounds__(kFT * kFT) k_fno_layer_out_tiled(
    const T* __restrict__ z0, T* __restrict__ z1, const T* __restrict__ cd, const T* __restrict__ wl, size_t stride,
    size_t w_off, const int* __restrict__ ws, int nsets, const T* __restrict__ cs, const T* __restrict__ sn, int C,
    int ks, int n, int k, int tiles_x) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    const int img = blockIdx.z, co0 = blockIdx.y * TCO;
    const int ty0 = (blockIdx.x / tiles_x) * kFT, tx0 = (blockIdx.x % tiles_x) * kFT;
    const int tid = threadIdx.x, ly = tid / kFT, lx = tid % kFT;
    const int x = ty0 + ly, y = tx0 + lx;  // x: row, y: column (as in the oracle's [row][col])
    const int r = ks / 2, S = kFT + 2 * r, kk = ks * ks;
    const size_t per = (size_t)n * n;
    const T* w = set_block(wl, stride, ws, nsets, img) + w_off;
    T acc[TCO];
#pragma unroll
    for (int j = 0; j < TCO; ++j) acc[j] = 0;
    for (int c0 = 0; c0 < C; c0 += kFCI) {
        const int cn = min(kFCI, C - c0);
        __syncthreads();
        for (int e = tid; e < cn * S * S; e += kFT * kFT) {
            const int cc = e / (S * S), rem = e % (S * S), sy = rem / S, sx = rem % S;
            const int gx = ty0 - r + sy, gy = tx0 - r + sx;
            tile[e] = (gx >= 0 && gx < n && gy >= 0 && gy < n)
                          ? z0[((size_t)img * C + c0 + cc) * per + (size_t)gx * n + gy]
                          : (T)0;
        }
        __syncthreads();
        for (int cc = 0; cc < cn; ++cc) {
            const T* tp = tile + cc * S * S + ly * S + lx;
            const T* wc = w + (size_t)co0 * C * kk + (size_t)(c0 + cc) * kk;
            for (int dy = 0; dy < ks; ++dy)
                for (int dx = 0; dx < ks; ++dx) {
                    const T v = tp[dy * S + dx];
                    const int t = dy * ks + dx;
#pragma unroll
                    for (int j = 0; j < TCO; ++j) acc[j] += wc[(size_t)j * C * kk + t] * v;
                }
        }
    }
    if (x >= n || y >= n) return;
    const T inv = (T)1 / (T)n;
    const T* bias = w + (size_t)C * C * kk;
#pragma unroll
    for (int j = 0; j < TCO; ++j) {
        const int co = co0 + j;
        const T* c = cd + (((size_t)img * C + co) * n + x) * (size_t)k * 2;
        T sp = 0;
        int q = 0;
        for (int v = 0; v < k; ++v) {
            const T term = c[2 * v] * cs[q] - c[2 * v + 1] * sn[q];
            sp += v == 0 ? term : (T)2 * term;
            q += y;
            if (q >= n) q -= n;
        }
        z1[((size_t)img * C + co) * per + (size_t)x * n + y] = gelu(sp * inv + acc[j] + bias[co]);
    }
}

// The same layer output with a 32 x 32 pixel tile and 2 x 2 pixels per
// thread (compile-time kernel size KS): per staged input channel and kernel
// row, a thread loads the KS + 1 input values of each of its two rows once
// and reuses them across the KS taps, its two columns and TCO channels.
constexpr int kFT2 = 32;

template <typename T, int TCO, int KS, int CI>
__global__ void __launch_bounds__(256) k_fno_layer_out_t2(
    const T* __restrict__ z0, T* __restrict__ z1, const T* __restrict__ sp_plane, const T* __restrict__ wl,
    size_t stride, size_t w_off, const int* __restrict__ ws, int nsets, int C, int n, int tiles_x) {
    constexpr int R = KS / 2, S = kFT2 + 2 * R, KK = KS * KS;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    const int img = blockIdx.z, co0 = blockIdx.y * TCO;
    const int ty0 = (blockIdx.x / tiles_x) * kFT2, tx0 = (blockIdx.x % tiles_x) * kFT2;
    const int tid = threadIdx.x, ly = tid / 16, lx = tid % 16;
    const size_t per = (size_t)n * n;
    const T* w = set_block(wl, stride, ws, nsets, img) + w_off;
    T acc[2][2][TCO];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int j = 0; j < TCO; ++j) acc[a][b][j] = 0;
    for (int c0 = 0; c0 < C; c0 += CI) {
        const int cn = min(CI, C - c0);
        __syncthreads();
        for (int e = tid; e < cn * S * S; e += 256) {
            const int cc = e / (S * S), rem = e % (S * S), sy = rem / S, sx = rem % S;
            const int gx = ty0 - R + sy, gy = tx0 - R + sx;
            tile[e] = (gx >= 0 && gx < n && gy >= 0 && gy < n)
                          ? z0[((size_t)img * C + c0 + cc) * per + (size_t)gx * n + gy]
                          : (T)0;
        }
        __syncthreads();
        for (int cc = 0; cc < cn; ++cc) {
            const T* wc = w + (size_t)co0 * C * KK + (size_t)(c0 + cc) * KK;
#pragma unroll
            for (int dy = 0; dy < KS; ++dy) {
                T in[2][KS + 1];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int t = 0; t <= KS; ++t) in[a][t] = tile[cc * S * S + (2 * ly + a + dy) * S + 2 * lx + t];
#pragma unroll
                for (int dx = 0; dx < KS; ++dx)
#pragma unroll
                    for (int j = 0; j < TCO; ++j) {
                        const T wv = wc[(size_t)j * C * KK + dy * KS + dx];
                        acc[0][0][j] += wv * in[0][dx];
                        acc[0][1][j] += wv * in[0][dx + 1];
                        acc[1][0][j] += wv * in[1][dx];
                        acc[1][1][j] += wv * in[1][dx + 1];
                    }
            }
        }
    }
    const T* bias = w + (size_t)C * C * KK;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int x = ty0 + 2 * ly + a;
        if (x >= n) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int y = tx0 + 2 * lx + b;
            if (y >= n) continue;
#pragma unroll
            for (int j = 0; j < TCO; ++j) {
                const size_t o = ((size_t)img * C + co0 + j) * per + (size_t)x * n + y;
                z1[o] = gelu(sp_plane[o] + acc[a][b][j] + bias[co0 + j]);
            }
        }
    }
}

// The layer's ks x ks convolution in FP32 on MFMA (float only): an implicit
// GEMM with the output channel as M (MB blocks of 16), 16 pixels of a row as N
// and K = 4 input channels at one tap per v_mfma_f32_16x16x4f32 (FP32 inputs,
// FP32 accumulation: the precision of the VALU kernels, at twice the
// non-packed VALU rate).  A workgroup owns a 32 x 8 pixel tile of one image
// and all C output channels; wave w takes rows 2w and 2w + 1, both 16-pixel
// halves (four N blocks).  Input channels are staged four at a time with the
// tile's halo (zero outside the image), and their weights from the per-set
// [ci][tap][co] copy (k_fno_wt).  Epilogue as in k_fno_layer_out_t2:
// z1 = GELU(spectral part + convolution + bias).
constexpr int kMW = 32, kMH = 8, kMCI = 4;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_wt(const T* __restrict__ wl, size_t stride, size_t w_off, int nsets,
                                                   int C, int KK, T* __restrict__ out) {
    const size_t per_set = (size_t)C * KK * C;
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per_set * nsets) return;
    const size_t set = e / per_set, r = e - set * per_set;
    const int ci = (int)(r / ((size_t)KK * C)), t = (int)((r / C) % KK), co = (int)(r % C);
    out[e] = wl[set * stride + w_off + ((size_t)co * C + ci) * KK + t];
}

template <int KS, int MB>
__global__ void __launch_bounds__(256) k_fno_layer_out_mfma(
    const float* __restrict__ z0, float* __restrict__ z1, const float* __restrict__ sp_plane,
    const float* __restrict__ wl, size_t stride, size_t w_off, const float* __restrict__ wt,
    const int* __restrict__ ws, int nsets, int n, int tiles_x) {
    constexpr int C = 16 * MB, R = KS / 2, KK = KS * KS;
    constexpr int SW = kMW + 2 * R, SH = kMH + 2 * R;  // staged columns / rows
    constexpr int IN_E = kMCI * SH * SW;               // staged input floats
    constexpr int W_E = kMCI * KK * C;                 // staged weight floats
    __shared__ float tin[IN_E];
    __shared__ float tw[W_E];
    const int img = blockIdx.y;
    const int ty0 = (blockIdx.x / tiles_x) * kMH, tx0 = (blockIdx.x % tiles_x) * kMW;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, kq = lane >> 4;
    const size_t per = (size_t)n * n;
    const int set = ws ? min(max(ws[img], 0), nsets - 1) : 0;
    const float* wts = wt + (size_t)set * C * KK * C;
    floatx4 acc[4][MB];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[nb][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
    // operand bases of this lane: B = staged input of channel kq, row 2 wave
    // (+ N block row + dy), column l16 (+ 16 x half + dx); A = staged weight of
    // channel kq, output channel l16 (+ 16 mb), tap 0
    const int bbase = (kq * SH + 2 * wave) * SW + l16;
    const int abase = kq * KK * C + l16;
    for (int c0 = 0; c0 < C; c0 += kMCI) {
        __syncthreads();  // every wave is done with the previous chunk
        for (int e = tid; e < IN_E; e += 256) {
            const int cc = e / (SH * SW), rem = e - cc * (SH * SW), sy = rem / SW, sx = rem - sy * SW;
            const int gy = ty0 - R + sy, gx = tx0 - R + sx;
            tin[e] = (gy >= 0 && gy < n && gx >= 0 && gx < n)
                         ? z0[((size_t)img * C + c0 + cc) * per + (size_t)gy * n + gx]
                         : 0.f;
        }
        const float* wsrc = wts + (size_t)c0 * KK * C;
        for (int e = tid; e < W_E; e += 256) tw[e] = wsrc[e];
        __syncthreads();
#pragma unroll
        for (int dy = 0; dy < KS; ++dy)
#pragma unroll
            for (int dx = 0; dx < KS; ++dx) {
                float a[MB];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) a[mb] = tw[abase + (dy * KS + dx) * C + 16 * mb];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    const float b = tin[bbase + ((nb >> 1) + dy) * SW + 16 * (nb & 1) + dx];
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
                        acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mb], b, acc[nb][mb], 0, 0, 0);
                }
            }
    }
    // acc[nb][mb][i]: output channel 16 mb + 4 kq + i of pixel (row 2 wave + (nb >> 1),
    // column 16 (nb & 1) + l16)
    const float* bias = set_block(wl, stride, ws, nsets, img) + w_off + (size_t)C * C * KK;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int y = ty0 + 2 * wave + (nb >> 1), x = tx0 + 16 * (nb & 1) + l16;
        if (y >= n || x >= n) continue;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = 16 * mb + 4 * kq + i;
                const size_t o = ((size_t)img * C + co) * per + (size_t)y * n + x;
                z1[o] = gelu(sp_plane[o] + acc[nb][mb][i] + bias[co]);
            }
    }
}

// h = ||b|| (sum_c proj_w[c] z[c] + proj_b), written or accumulated into dst
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_project(const T* __restrict__ z, const double* __restrict__ nrm2,
                                                        T* __restrict__ dst, const T* __restrict__ wl, size_t stride,
                                                        size_t p_off, const int* __restrict__ ws, int nsets, int C,
                                                        size_t per, int accumulate) {
    const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int img = blockIdx.y;
    if (p >= per) return;
    const T* w = set_block(wl, stride, ws, nsets, img) + p_off;
    const double q = nrm2[img];
    T h = 0;
    if (q > 0.0) {
        T acc = w[C];
        for (int c = 0; c < C; ++c) acc += w[c] * z[((size_t)img * C + c) * per + p];
        h = (T)sqrt(q) * acc;
    }
    T* o = dst + (size_t)img * per + p;
    *o = accumulate ? *o + h : h;
}


// ---------------------------------------------------------------------------
// Training: forward with stored activations, and the hand-written adjoint of
// the FNO for the level-wise loss (weights only; the smoother input b_l is a
// constant of level l's loss).  Every transform of a Fourier layer is a real
// linear map, so its adjoint is the transposed map:
//   forward  Z -> TA = Z Fc -> X (rows) -> Y = mix(X, R) -> CDs (inverse rows,
//            split re | im) -> S = CDs Finv;  pre = S + W * Z + B;  Z' = GELU(pre)
//   adjoint  gS = gPre -> gCDs = gS Finv^T -> gY -> (gX, dR) -> gTA -> gZ += gTA Fc^T
//            plus the transposed convolution, dW and dB.
// ---------------------------------------------------------------------------

// 1D: interleaved (re, im) pairs -> split layout (re block | im block); the
// adjoint of k_fno_interleave
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_deinterleave(const T* __restrict__ xi, T* __restrict__ sp, int k,
                                                             size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    const size_t bc = e / k;
    const int v = (int)(e % k);
    sp[bc * 2 * k + v] = xi[2 * e];
    sp[bc * 2 * k + k + v] = xi[2 * e + 1];
}

// pre = S + W * z + B and z' = GELU(pre) (any dim; direct convolution)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_pre(const T* __restrict__ z0, const T* __restrict__ sp_plane,
                                                    T* __restrict__ pre, T* __restrict__ z1, const T* __restrict__ wl,
                                                    size_t stride, size_t w_off, const int* __restrict__ ws, int nsets,
                                                    int C, int ks, int ny, int n) {
    const size_t per = (size_t)ny * n;
    const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int co = blockIdx.y, img = blockIdx.z;
    if (p >= per) return;
    const int x = (int)(p / n), y = (int)(p % n);
    const T* w = set_block(wl, stride, ws, nsets, img) + w_off;
    const int kh = ny > 1 ? ks : 1, kw = ks;
    const T* Wc = w + (size_t)co * C * kh * kw;
    T acc = w[(size_t)C * C * kh * kw + co];
    for (int ci = 0; ci < C; ++ci) {
        const T* zc = z0 + ((size_t)img * C + ci) * per;
        for (int dy = 0; dy < kh; ++dy) {
            const int yy = x + dy - kh / 2;
            if (yy < 0 || yy >= ny) continue;
            for (int dx = 0; dx < kw; ++dx) {
                const int xx = y + dx - kw / 2;
                if (xx < 0 || xx >= n) continue;
                acc += Wc[((size_t)ci * kh + dy) * kw + dx] * zc[(size_t)yy * n + xx];
            }
        }
    }
    const size_t o = ((size_t)img * C + co) * per + p;
    const T v = sp_plane[o] + acc;
    pre[o] = v;
    z1[o] = gelu(v);
}

// g_out = sign ||b|| upstream (per pixel); gZ[c] = proj_w[c] g_out
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_gout(const T* __restrict__ up, const double* __restrict__ nrm2,
                                                     T* __restrict__ gout, T* __restrict__ gz,
                                                     const T* __restrict__ wl, size_t stride, size_t p_off,
                                                     const int* __restrict__ ws, int nsets, int C, size_t per, T sign) {
    const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int img = blockIdx.y;
    if (p >= per) return;
    const T* w = set_block(wl, stride, ws, nsets, img) + p_off;
    const T g = sign * (T)sqrt(nrm2[img]) * up[(size_t)img * per + p];
    gout[(size_t)img * per + p] = g;
    for (int c = 0; c < C; ++c) gz[((size_t)img * C + c) * per + p] = w[c] * g;
}

// out[c] += sum_img sum_p A[img][c][p] * (B ? B[img][p] * scale(img) : 1), scale = 1/||b||
// when nrm2 is given; one workgroup per c, fixed reduction order.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_sum_prod(const T* __restrict__ A, const T* __restrict__ Bv,
                                                         const double* __restrict__ nrm2, T* __restrict__ out, int C,
                                                         size_t per, int batch) {
    __shared__ double red[kBlock];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int img = 0; img < batch; ++img) {
        const T* a = A + ((size_t)img * C + c) * per;
        const T* bv = Bv ? Bv + (size_t)img * per : nullptr;
        double part = 0.0;
        for (size_t p = threadIdx.x; p < per; p += kBlock) part += (double)a[p] * (bv ? (double)bv[p] : 1.0);
        if (bv && nrm2) part *= nrm2[img] > 0.0 ? 1.0 / sqrt(nrm2[img]) : 0.0;
        acc += part;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] += (T)red[0];
}

// gPre = gZ * GELU'(pre), GELU'(x) = Phi(x) + x phi(x)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_gelu_bwd(const T* __restrict__ gz, const T* __restrict__ pre,
                                                         T* __restrict__ gp, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    const T x = pre[e];
    const T cdf = (T)0.5 * ((T)1 + erf(x * (T)0.70710678118654752440));
    const T pdf = (T)0.39894228040143267794 * exp((T)-0.5 * x * x);
    gp[e] = gz[e] * (cdf + x * pdf);
}

// dW[co][ci][t] += sum_img sum_p gPre[img][co][p] Z[img][ci][p + off(t)];
// one workgroup per (co, ci), KK partial sums per thread
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_wgrad(const T* __restrict__ gp, const T* __restrict__ z,
                                                      T* __restrict__ dW, int C, int ks, int ny, int n, int batch) {
    __shared__ double red[kBlock];
    const int co = blockIdx.x / C, ci = blockIdx.x % C;
    const int kh = ny > 1 ? ks : 1, kw = ks, kk = kh * kw;
    const size_t per = (size_t)ny * n;
    double acc[49];
    for (int t = 0; t < kk; ++t) acc[t] = 0.0;
    for (int img = 0; img < batch; ++img) {
        const T* g = gp + ((size_t)img * C + co) * per;
        const T* zc = z + ((size_t)img * C + ci) * per;
        for (size_t p = threadIdx.x; p < per; p += kBlock) {
            const double gv = g[p];
            const int x = (int)(p / n), y = (int)(p % n);
            for (int dy = 0; dy < kh; ++dy) {
                const int yy = x + dy - kh / 2;
                if (yy < 0 || yy >= ny) continue;
                for (int dx = 0; dx < kw; ++dx) {
                    const int xx = y + dx - kw / 2;
                    if (xx < 0 || xx >= n) continue;
                    acc[dy * kw + dx] += gv * (double)zc[(size_t)yy * n + xx];
                }
            }
        }
    }
    for (int t = 0; t < kk; ++t) {
        red[threadIdx.x] = acc[t];
        __syncthreads();
        for (int k = kBlock / 2; k > 0; k >>= 1) {
            if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) dW[((size_t)co * C + ci) * kk + t] += (T)red[0];
        __syncthreads();
    }
}

// gZ[img][ci][p] = gS[img][ci][p] + sum_co sum_t W[co][ci][t] gPre[img][co][p - off(t)]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_conv_t_add(const T* __restrict__ gp, const T* __restrict__ gs,
                                                           T* __restrict__ gz, const T* __restrict__ wl, size_t stride,
                                                           size_t w_off, const int* __restrict__ ws, int nsets, int C,
                                                           int ks, int ny, int n) {
    const size_t per = (size_t)ny * n;
    const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int ci = blockIdx.y, img = blockIdx.z;
    if (p >= per) return;
    const int x = (int)(p / n), y = (int)(p % n);
    const T* w = set_block(wl, stride, ws, nsets, img) + w_off;
    const int kh = ny > 1 ? ks : 1, kw = ks;
    T acc = gs[((size_t)img * C + ci) * per + p];
    for (int co = 0; co < C; ++co) {
        const T* g = gp + ((size_t)img * C + co) * per;
        const T* wc = w + ((size_t)co * C + ci) * kh * kw;
        for (int dy = 0; dy < kh; ++dy) {
            const int yy = x - dy + kh / 2;
            if (yy < 0 || yy >= ny) continue;
            for (int dx = 0; dx < kw; ++dx) {
                const int xx = y - dx + kw / 2;
                if (xx < 0 || xx >= n) continue;
                acc += wc[dy * kw + dx] * g[(size_t)yy * n + xx];
            }
        }
    }
    gz[((size_t)img * C + ci) * per + p] = acc;
}

// adjoint of k_fno_idft_rows_split (2D): gY[bc][u'][v] (re, im) from gCDs
//   cr = (1/n) sum_u' (yr c - yi s), ci = (1/n) sum_u' (yr s + yi c), (c, s) of 2 pi u x / n
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_idft_rows_split_adj(const T* __restrict__ gcd, T* __restrict__ gy,
                                                                    const T* __restrict__ cs, const T* __restrict__ sn,
                                                                    int n, int k, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;  // (bc, u', v)
    if (e >= count) return;
    const int v = (int)(e % k);
    const int up = (int)((e / k) % (2 * k));
    const size_t bc = e / ((size_t)2 * k * k);
    const int u = up < k ? up : n - 2 * k + up;
    T gr = 0, gi = 0;
    int q = 0;
    for (int x = 0; x < n; ++x) {
        const T a = gcd[(bc * n + x) * 2 * k + v], b = gcd[(bc * n + x) * 2 * k + k + v];
        gr += a * cs[q] + b * sn[q];
        gi += -a * sn[q] + b * cs[q];
        q += u;
        if (q >= n) q -= n;
    }
    const T inv = (T)1 / (T)n;
    gy[2 * e] = gr * inv;
    gy[2 * e + 1] = gi * inv;
}

// adjoint of k_fno_dft_rows (2D): gTA[bc][x][j] from gX[bc][u'][v]
//   Xr = sum_x (c Tr + s Ti), Xi = sum_x (c Ti - s Tr)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_dft_rows_adj(const T* __restrict__ gx, T* __restrict__ gta,
                                                             const T* __restrict__ cs, const T* __restrict__ sn, int n,
                                                             int k, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;  // (bc, x, v)
    if (e >= count) return;
    const int v = (int)(e % k);
    const int x = (int)((e / k) % n);
    const size_t bc = e / ((size_t)n * k);
    T gtr = 0, gti = 0;
    for (int up = 0; up < 2 * k; ++up) {
        const int u = up < k ? up : n - 2 * k + up;
        const int q = (int)(((long long)u * x) % n);
        const T gr = gx[((bc * 2 * k + up) * k + v) * 2], gi = gx[((bc * 2 * k + up) * k + v) * 2 + 1];
        gtr += cs[q] * gr - sn[q] * gi;
        gti += sn[q] * gr + cs[q] * gi;
    }
    gta[(bc * n + x) * 2 * k + v] = gtr;
    gta[(bc * n + x) * 2 * k + k + v] = gti;
}

// adjoint of the mode mixing: gX[img][ci][m] = sum_co conj-style products with R
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_mix_adj_x(const T* __restrict__ gy, T* __restrict__ gx,
                                                          const T* __restrict__ wl, size_t stride, size_t r_off,
                                                          size_t rm, const int* __restrict__ ws, int nsets, int C,
                                                          int k, int m, int two_d, size_t modes, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;  // (img, ci, md)
    if (e >= count) return;
    const size_t md = e % modes;
    const int ci = (int)((e / modes) % C);
    const int img = (int)(e / (modes * C));
    const T* w = set_block(wl, stride, ws, nsets, img) + r_off;
    size_t base;
    if (two_d) {
        const int v = (int)(md % k), up = (int)(md / k);
        const int corner = up < k ? 0 : 1, u = up < k ? up : up - k;
        base = (((size_t)corner * C + ci) * C) * m * m + (size_t)u * m + v;  // + co * m * m
    } else {
        base = (size_t)ci * C * m + md;  // + co * m
    }
    const size_t cst = two_d ? (size_t)m * m : (size_t)m;
    T ar = 0, ai = 0;
    for (int co = 0; co < C; ++co) {
        const size_t yi = (((size_t)img * C + co) * modes + md) * 2;
        const T gr = gy[yi], gi = gy[yi + 1];
        const T rr = w[base + co * cst], ri = w[rm + base + co * cst];
        ar += rr * gr + ri * gi;
        ai += -ri * gr + rr * gi;
    }
    gx[2 * e] = ar;
    gx[2 * e + 1] = ai;
}

// dR: dRr[ci][co][m] += sum_img (Xr gYr + Xi gYi), dRi += sum_img (-Xi gYr + Xr gYi)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_mix_adj_r(const T* __restrict__ x, const T* __restrict__ gy,
                                                          T* __restrict__ dr, size_t rm, int C, int k, int m,
                                                          int two_d, size_t modes, int batch, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;  // (ci, co, md)
    if (e >= count) return;
    const size_t md = e % modes;
    const int co = (int)((e / modes) % C);
    const int ci = (int)(e / (modes * C));
    double sr = 0.0, si = 0.0;
    for (int img = 0; img < batch; ++img) {
        const size_t xi_ = (((size_t)img * C + ci) * modes + md) * 2;
        const size_t yi_ = (((size_t)img * C + co) * modes + md) * 2;
        const double xr = x[xi_], xim = x[xi_ + 1], gr = gy[yi_], gi = gy[yi_ + 1];
        sr += xr * gr + xim * gi;
        si += -xim * gr + xr * gi;
    }
    size_t idx;
    if (two_d) {
        const int v = (int)(md % k), up = (int)(md / k);
        const int corner = up < k ? 0 : 1, u = up < k ? up : up - k;
        idx = (((size_t)corner * C + ci) * C + co) * m * m + (size_t)u * m + v;
    } else {
        idx = ((size_t)ci * C + co) * m + md;
    }
    dr[idx] += (T)sr;
    dr[rm + idx] += (T)si;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fno_zero(T* __restrict__ p, size_t count) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < count) p[e] = 0;
}
}  // namespace

size_t fno_weight_count(const nmg_problem& p) {
    const size_t C = (size_t)p.fno_width, m = (size_t)p.fno_modes;
    const size_t kk = p.dim == 2 ? (size_t)p.fno_ksize * p.fno_ksize : (size_t)p.fno_ksize;
    const size_t rm = p.dim == 2 ? 2 * C * C * m * m : C * C * m;
    return 2 * C + (size_t)p.fno_layers * (2 * rm + C * C * kk + C) + C + 1;
}

int fno_level_modes(const Ctx* c, int l) { return std::min(c->p.fno_modes, c->n[(size_t)l] / 2); }

template <typename T>
nmg_status ensure_fno(Ctx* c) {
    Work<T>& w = work_of<T>(c);
    if (w.fno_ready) return NMG_OK;
    if (c->capturing) return fail(NMG_ERR_STATE, "FNO buffers must exist before graph capture");
    const size_t B = (size_t)c->p.max_batch, C = (size_t)c->p.fno_width;
    const size_t per0 = level_elems(c, 0);
    const size_t ny0 = (size_t)c->ny0, n0 = (size_t)c->n[0];
    const size_t m = (size_t)std::max(1, fno_level_modes(c, 0));
    NMG_TRY(falloc(&w.fz0, B * C * per0));
    NMG_TRY(falloc(&w.fz1, B * C * per0));
    NMG_TRY(falloc(&w.fta, B * C * ny0 * 2 * m));
    const size_t modes = c->p.dim == 2 ? 2 * m * m : m;
    NMG_TRY(falloc(&w.fxh, B * C * modes * 2));
    NMG_TRY(falloc(&w.fyh, B * C * modes * 2));
    NMG_TRY(falloc(&w.fcd, B * C * ny0 * m * 2));
    NMG_TRY(falloc(&w.fsp, B * C * per0));
    if (c->p.dim == 2) {
        const size_t kk = (size_t)c->p.fno_ksize * c->p.fno_ksize;
        NMG_TRY(falloc(&w.fwt, (size_t)std::max(1, c->p.n_weight_sets) * C * C * kk));
    }
    (void)n0;
    std::vector<double> tab;
    w.ftab_off.clear();
    for (int l = 0; l < c->L; ++l) {
        const int n = c->n[(size_t)l];
        w.ftab_off.push_back(tab.size());
        for (int q = 0; q < n; ++q) tab.push_back(std::cos(2.0 * M_PI * q / n));
        for (int q = 0; q < n; ++q) tab.push_back(std::sin(2.0 * M_PI * q / n));
    }
    NMG_TRY(falloc(&w.ftab, tab.size()));
    std::vector<T> tabT(tab.begin(), tab.end());
    NMG_HIP(hipMemcpy(w.ftab, tabT.data(), tabT.size() * sizeof(T), hipMemcpyHostToDevice));
    // dense twiddle matrices of the column transforms per level:
    //   forward [n][2k]: cos(2 pi j y / n) | -sin(2 pi j y / n)
    //   inverse [2k][n]: w_j cos(2 pi j y / n) / n ; -w_j sin(2 pi j y / n) / n  (w_0 = 1, w_j = 2)
    std::vector<T> mats;
    w.fmat_off.clear();
    for (int l = 0; l < c->L; ++l) {
        const int n = c->n[(size_t)l];
        const int k = std::max(1, fno_level_modes(c, l));
        w.fmat_off.push_back(mats.size());
        for (int y = 0; y < n; ++y)
            for (int j = 0; j < 2 * k; ++j) {
                const int f = j < k ? j : j - k;
                const double a = 2.0 * M_PI * (double)(((long long)f * y) % n) / n;
                mats.push_back((T)(j < k ? std::cos(a) : -std::sin(a)));
            }
        for (int j = 0; j < 2 * k; ++j)
            for (int y = 0; y < n; ++y) {
                const int f = j < k ? j : j - k;
                const double wgt = (f == 0 ? 1.0 : 2.0) / n;
                const double a = 2.0 * M_PI * (double)(((long long)f * y) % n) / n;
                mats.push_back((T)(j < k ? wgt * std::cos(a) : -wgt * std::sin(a)));
            }
    }
    NMG_TRY(falloc(&w.fmat, mats.size()));
    NMG_HIP(hipMemcpy(w.fmat, mats.data(), mats.size() * sizeof(T), hipMemcpyHostToDevice));
    w.fno_ready = true;
    return NMG_OK;
}
template nmg_status ensure_fno<float>(Ctx*);
template nmg_status ensure_fno<double>(Ctx*);

template <typename T>
nmg_status launch_fno_smoother(const Ctx* c, int l, int batch, const int* ws, const T* b, const double* nrm2, T* dst,
                               int accumulate, Work<T>& w, hipStream_t s) {
    if (!w.fno_ready) return fail(NMG_ERR_STATE, "FNO buffers not allocated");
    const FnoDims d = fno_dims(c);
    const int n = c->n[(size_t)l];
    const int ny = d.dim == 2 ? n : 1;
    const size_t per = (size_t)ny * n;
    const int k = fno_level_modes(c, l);
    if (k < 1) return fail(NMG_ERR_SHAPE, "FNO needs at least one mode on every smoothing level");
    const int nsets = c->p.n_weight_sets;
    const size_t stride = (size_t)c->wcount;
    const T* wl = w.wts + (size_t)l * nsets * stride;
    const T* cs = w.ftab + w.ftab_off[(size_t)l];
    const T* sn = cs + n;
    const int C = d.C;
    hipLaunchKernelGGL(k_fno_lift<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, b, nrm2, w.fz0, wl, stride,
                       ws, nsets, C, per);
    T* z0 = w.fz0;
    T* z1 = w.fz1;
    const size_t modes = d.dim == 2 ? (size_t)2 * k * k : (size_t)k;
    for (int layer = 0; layer < d.NL; ++layer) {
        const size_t base = 2 * (size_t)C + (size_t)layer * d.layer_stride;
        const size_t rows = (size_t)batch * C * ny;
        const T* fwd = w.fmat + w.fmat_off[(size_t)l];
        const T* inv_m = fwd + (size_t)n * 2 * k;
        hipLaunchKernelGGL(k_gemm_rm<T>, dim3((unsigned)((rows + 63) / 64), (unsigned)((2 * k + 63) / 64)), dim3(256),
                           0, s, z0, fwd, w.fta, (int)rows, 2 * k, n);
        const T* xsrc = w.fta;  // 1D: T[img][c][2k] is (re | -im) of X, re-laid out by the mix below
        if (d.dim == 2) {
            const size_t cnt = (size_t)batch * C * 2 * k * k;
            hipLaunchKernelGGL(k_fno_dft_rows<T>, dim3(blocks_for(cnt)), dim3(kBlock), 0, s, w.fta, w.fxh, cs, sn,
                               n, k, cnt);
            xsrc = w.fxh;
        } else {
            // interleave (re, im) per mode: X[v] = T[v] + i T[k + v]
            const size_t cnt = (size_t)batch * C * k;
            hipLaunchKernelGGL(k_fno_interleave<T>, dim3(blocks_for(cnt)), dim3(kBlock), 0, s, w.fta, w.fxh, k, cnt);
            xsrc = w.fxh;
        }
        const size_t mcnt = (size_t)batch * C * modes;
        hipLaunchKernelGGL(k_fno_mix<T>, dim3(blocks_for(mcnt)), dim3(kBlock), 0, s, xsrc, w.fyh, wl, stride, base,
                           d.rm, ws, nsets, C, k, d.m, d.dim == 2 ? 1 : 0, modes, mcnt);
        const T* cdp = w.fyh;
        const bool t2 = d.dim == 2 && C % 16 == 0 && (d.ks == 3 || d.ks == 5 || d.ks == 7);
        if (t2) {
            // inverse rows in split layout, then the inverse columns as one GEMM into the spectral plane
            const size_t cnt = (size_t)batch * C * n * k;
            hipLaunchKernelGGL(k_fno_idft_rows_split<T>, dim3(blocks_for(cnt)), dim3(kBlock), 0, s, w.fyh, w.fcd, cs,
                               sn, n, k, cnt);
            hipLaunchKernelGGL(k_gemm_rm<T>, dim3((unsigned)((rows + 63) / 64), (unsigned)((n + 63) / 64)),
                               dim3(256), 0, s, w.fcd, inv_m, w.fsp, (int)rows, n, 2 * k);
        } else if (d.dim == 2) {
            const size_t cnt = (size_t)batch * C * n * k;
            hipLaunchKernelGGL(k_fno_idft_rows<T>, dim3(blocks_for(cnt)), dim3(kBlock), 0, s, w.fyh, w.fcd, cs, sn,
                               n, k, cnt);
            cdp = w.fcd;
        }
        bool done = false;
        if constexpr (std::is_same<T, float>::value) {
            // FP32 MFMA for 32 or 64 channels and 3 x 3, 5 x 5, 7 x 7 kernels
            if (t2 && w.fwt && (C == 32 || C == 64)) {
                const size_t ww = (size_t)nsets * C * C * d.kk;
                hipLaunchKernelGGL(k_fno_wt<float>, dim3(blocks_for(ww)), dim3(kBlock), 0, s, wl, stride,
                                   base + 2 * d.rm, nsets, C, d.kk, w.fwt);
                const int tiles_x = (n + kMW - 1) / kMW, tiles_y = (n + kMH - 1) / kMH;
                const dim3 grid((unsigned)(tiles_x * tiles_y), (unsigned)batch);
                auto go = [&](auto ks_tag, auto mb_tag) {
                    constexpr int KS = decltype(ks_tag)::value, MB = decltype(mb_tag)::value;
                    hipLaunchKernelGGL((k_fno_layer_out_mfma<KS, MB>), grid, dim3(256), 0, s, z0, z1, w.fsp, wl,
                                       stride, base + 2 * d.rm, w.fwt, ws, nsets, n, tiles_x);
                };
                auto by_ks = [&](auto mb_tag) {
                    if (d.ks == 3) go(std::integral_constant<int, 3>{}, mb_tag);
                    if (d.ks == 5) go(std::integral_constant<int, 5>{}, mb_tag);
                    if (d.ks == 7) go(std::integral_constant<int, 7>{}, mb_tag);
                };
                if (C == 32)
                    by_ks(std::integral_constant<int, 2>{});
                else
                    by_ks(std::integral_constant<int, 4>{});
                done = true;
            }
        }
        if (!done && t2) {
            const int tiles_x = (n + kFT2 - 1) / kFT2;
            constexpr int CI = sizeof(T) == 4 ? 8 : 4;
            auto go = [&](auto ks_tag) {
                constexpr int KS = decltype(ks_tag)::value;
                constexpr int S = kFT2 + 2 * (KS / 2);
                hipLaunchKernelGGL((k_fno_layer_out_t2<T, 16, KS, CI>), dim3(tiles_x * tiles_x, C / 16, batch),
                                   dim3(256), (size_t)CI * S * S * sizeof(T), s, z0, z1, w.fsp, wl, stride,
                                   base + 2 * d.rm, ws, nsets, C, n, tiles_x);
            };
            if (d.ks == 3) go(std::integral_constant<int, 3>{});
            if (d.ks == 5) go(std::integral_constant<int, 5>{});
            if (d.ks == 7) go(std::integral_constant<int, 7>{});
            done = true;
        }
        if (done) {
        } else if (d.dim == 2 && C % 16 == 0) {
            const int tiles_x = (n + kFT - 1) / kFT;
            const int S = kFT + 2 * (d.ks / 2);
            hipLaunchKernelGGL((k_fno_layer_out_tiled<T, 16>), dim3(tiles_x * tiles_x, C / 16, batch),
                               dim3(kFT * kFT), (size_t)kFCI * S * S * sizeof(T), s, z0, z1, cdp, wl, stride,
                               base + 2 * d.rm, ws, nsets, cs, sn, C, d.ks, n, k, tiles_x);
        } else {
            hipLaunchKernelGGL(k_fno_layer_out<T>, dim3(blocks_for(per), C, batch), dim3(kBlock), 0, s, z0, z1, cdp,
                               wl, stride, base + 2 * d.rm, ws, nsets, cs, sn, C, d.ks, ny, n, k);
        }
        std::swap(z0, z1);
    }
    const size_t p_off = 2 * (size_t)C + (size_t)d.NL * d.layer_stride;
    hipLaunchKernelGGL(k_fno_project<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, z0, nrm2, dst, wl, stride,
                       p_off, ws, nsets, C, per, accumulate);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}
template nmg_status launch_fno_smoother<float>(const Ctx*, int, int, const int*, const float*, const double*, float*,
                                               int, Work<float>&, hipStream_t);
template nmg_status launch_fno_smoother<double>(const Ctx*, int, int, const int*, const double*, const double*,
                                                double*, int, Work<double>&, hipStream_t);

template <typename T>
static nmg_status ensure_fno_train(Ctx* c, Work<T>& w) {
    NMG_TRY(ensure_fno<T>(c));
    if (w.ftr_ready) return NMG_OK;
    const size_t B = (size_t)c->p.max_batch, C = (size_t)c->p.fno_width, NL = (size_t)c->p.fno_layers;
    const size_t per0 = level_elems(c, 0), ny0 = (size_t)c->ny0;
    const size_t m = (size_t)std::max(1, fno_level_modes(c, 0));
    const size_t modes = c->p.dim == 2 ? 2 * m * m : m;
    NMG_TRY(falloc(&w.ftz, (NL + 1) * B * C * per0));
    NMG_TRY(falloc(&w.ftp, NL * B * C * per0));
    NMG_TRY(falloc(&w.ftx, NL * B * C * modes * 2));
    NMG_TRY(falloc(&w.ftgz, B * C * per0));
    NMG_TRY(falloc(&w.ftgp, B * C * per0));
    NMG_TRY(falloc(&w.ftgs, B * C * per0));
    NMG_TRY(falloc(&w.ftga, B * C * ny0 * 2 * m));
    NMG_TRY(falloc(&w.ftgx, B * C * modes * 2));
    NMG_TRY(falloc(&w.ftgy, B * C * modes * 2));
    NMG_TRY(falloc(&w.ftgo, B * per0));
    w.ftr_ready = true;
    return NMG_OK;
}

template <typename T>
nmg_status fno_backward(Ctx* c, Work<T>& w, int l, int set, int batch, const T* b, const double* nrm2,
                        const T* upstream, T sign, int accumulate, T* grad, hipStream_t s) {
    if (c->capturing) return fail(NMG_ERR_STATE, "FNO training cannot run inside a graph capture");
    NMG_TRY(ensure_fno_train<T>(c, w));
    const FnoDims d = fno_dims(c);
    const int n = c->n[(size_t)l];
    const int ny = d.dim == 2 ? n : 1;
    const size_t per = (size_t)ny * n, per0 = level_elems(c, 0);
    const int k = fno_level_modes(c, l);
    const int C = d.C;
    const size_t stride = (size_t)c->wcount;
    const int nsets = c->p.n_weight_sets;
    const T* wl = w.wts + (size_t)l * nsets * stride + (size_t)set * stride;  // this set only
    const T* cs = w.ftab + w.ftab_off[(size_t)l];
    const T* sn = cs + n;
    const T* fwd = w.fmat + w.fmat_off[(size_t)l];
    const T* inv_m = fwd + (size_t)n * 2 * k;
    const size_t modes = d.dim == 2 ? (size_t)2 * k * k : (size_t)k;
    const size_t m0 = (size_t)std::max(1, fno_level_modes(c, 0));
    const size_t modes0 = d.dim == 2 ? 2 * m0 * m0 : m0;
    const size_t rows = (size_t)batch * C * ny;
    const size_t plane = (size_t)c->p.max_batch * C * per0;  // stride of the per-layer stores
    auto Z = [&](int i) { return w.ftz + (size_t)i * plane; };
    auto P = [&](int i) { return w.ftp + (size_t)i * plane; };
    auto X = [&](int i) { return w.ftx + (size_t)i * c->p.max_batch * C * modes0 * 2; };
    const int* ws = nullptr;  // one weight set for the whole batch: wl already points at it
    if (!accumulate) hipLaunchKernelGGL(k_fno_zero<T>, dim3(blocks_for(stride)), dim3(kBlock), 0, s, grad, stride);
    // ---- forward with stored activations
    hipLaunchKernelGGL(k_fno_lift<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, b, nrm2, Z(0), wl, stride, ws,
                       1, C, per);
    for (int i = 0; i < d.NL; ++i) {
        const size_t base = 2 * (size_t)C + (size_t)i * d.layer_stride;
        hipLaunchKernelGGL(k_gemm_rm<T>, dim3((unsigned)((rows + 63) / 64), (unsigned)((2 * k + 63) / 64)), dim3(256),
                           0, s, Z(i), fwd, w.fta, (int)rows, 2 * k, n, 0);
        const size_t xc = (size_t)batch * C * modes;
        if (d.dim == 2)
            hipLaunchKernelGGL(k_fno_dft_rows<T>, dim3(blocks_for(xc)), dim3(kBlock), 0, s, w.fta, X(i), cs, sn, n, k,
                               xc);
        else
            hipLaunchKernelGGL(k_fno_interleave<T>, dim3(blocks_for(xc)), dim3(kBlock), 0, s, w.fta, X(i), k, xc);
        hipLaunchKernelGGL(k_fno_mix<T>, dim3(blocks_for(xc)), dim3(kBlock), 0, s, X(i), w.fyh, wl, stride, base, d.rm,
                           ws, 1, C, k, d.m, d.dim == 2 ? 1 : 0, modes, xc);
        if (d.dim == 2) {
            const size_t cnt = (size_t)batch * C * n * k;
            hipLaunchKernelGGL(k_fno_idft_rows_split<T>, dim3(blocks_for(cnt)), dim3(kBlock), 0, s, w.fyh, w.fcd, cs,
                               sn, n, k, cnt);
        } else {
            hipLaunchKernelGGL(k_fno_deinterleave<T>, dim3(blocks_for(xc)), dim3(kBlock), 0, s, w.fyh, w.fcd, k, xc);
        }
        hipLaunchKernelGGL(k_gemm_rm<T>, dim3((unsigned)((rows + 63) / 64), (unsigned)((n + 63) / 64)), dim3(256), 0,
                           s, w.fcd, inv_m, w.fsp, (int)rows, n, 2 * k, 0);
        hipLaunchKernelGGL(k_fno_pre<T>, dim3(blocks_for(per), C, batch), dim3(kBlock), 0, s, Z(i), w.fsp, P(i),
                           Z(i + 1), wl, stride, base + 2 * d.rm, ws, 1, C, d.ks, ny, n);
    }
    // ---- adjoint
    const size_t p_off = 2 * (size_t)C + (size_t)d.NL * d.layer_stride;
    hipLaunchKernelGGL(k_fno_gout<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, upstream, nrm2, w.ftgo, w.ftgz,
                       wl, stride, p_off, ws, 1, C, per, sign);
    hipLaunchKernelGGL(k_fno_sum_prod<T>, dim3(C), dim3(kBlock), 0, s, Z(d.NL), w.ftgo, (const double*)nullptr,
                       grad + p_off, C, per, batch);
    hipLaunchKernelGGL(k_fno_sum_prod<T>, dim3(1), dim3(kBlock), 0, s, w.ftgo, (const T*)nullptr,
                       (const double*)nullptr, grad + p_off + C, 1, per, batch);
    const size_t tot = (size_t)batch * C * per;
    for (int i = d.NL - 1; i >= 0; --i) {
        const size_t base = 2 * (size_t)C + (size_t)i * d.layer_stride;
        hipLaunchKernelGGL(k_fno_gelu_bwd<T>, dim3(blocks_for(tot)), dim3(kBlock), 0, s, w.ftgz, P(i), w.ftgp, tot);
        // bias and convolution weights
        hipLaunchKernelGGL(k_fno_sum_prod<T>, dim3(C), dim3(kBlock), 0, s, w.ftgp, (const T*)nullptr,
                           (const double*)nullptr, grad + base + 2 * d.rm + (size_t)C * C * d.kk, C, per, batch);
        hipLaunchKernelGGL(k_fno_wgrad<T>, dim3(C * C), dim3(kBlock), 0, s, w.ftgp, Z(i), grad + base + 2 * d.rm, C,
                           d.ks, ny, n, batch);
        // spectral path: gCDs = gPre Finv^T, then the adjoint inverse rows
        hipLaunchKernelGGL(k_gemm_rm<T>, dim3((unsigned)((rows + 63) / 64), (unsigned)((2 * k + 63) / 64)), dim3(256),
                           0, s, w.ftgp, inv_m, w.ftga, (int)rows, 2 * k, n, 1);
        const size_t xc = (size_t)batch * C * modes;
        if (d.dim == 2)
            hipLaunchKernelGGL(k_fno_idft_rows_split_adj<T>, dim3(blocks_for(xc)), dim3(kBlock), 0, s, w.ftga, w.ftgy,
                               cs, sn, n, k, xc);
        else
            hipLaunchKernelGGL(k_fno_interleave<T>, dim3(blocks_for(xc)), dim3(kBlock), 0, s, w.ftga, w.ftgy, k, xc);
        const size_t rc = (size_t)C * C * modes;
        hipLaunchKernelGGL(k_fno_mix_adj_r<T>, dim3(blocks_for(rc)), dim3(kBlock), 0, s, X(i), w.ftgy, grad + base,
                           d.rm, C, k, d.m, d.dim == 2 ? 1 : 0, modes, batch, rc);
        hipLaunchKernelGGL(k_fno_mix_adj_x<T>, dim3(blocks_for(xc)), dim3(kBlock), 0, s, w.ftgy, w.ftgx, wl, stride,
                           base, d.rm, ws, 1, C, k, d.m, d.dim == 2 ? 1 : 0, modes, xc);
        if (d.dim == 2) {
            const size_t cnt = (size_t)batch * C * n * k;
            hipLaunchKernelGGL(k_fno_dft_rows_adj<T>, dim3(blocks_for(cnt)), dim3(kBlock), 0, s, w.ftgx, w.ftga, cs,
                               sn, n, k, cnt);
        } else {
            hipLaunchKernelGGL(k_fno_deinterleave<T>, dim3(blocks_for(xc)), dim3(kBlock), 0, s, w.ftgx, w.ftga, k, xc);
        }
        hipLaunchKernelGGL(k_gemm_rm<T>, dim3((unsigned)((rows + 63) / 64), (unsigned)((n + 63) / 64)), dim3(256), 0,
                           s, w.ftga, fwd, w.ftgs, (int)rows, n, 2 * k, 1);
        // gZ of the layer input = spectral part + transposed convolution
        hipLaunchKernelGGL(k_fno_conv_t_add<T>, dim3(blocks_for(per), C, batch), dim3(kBlock), 0, s, w.ftgp, w.ftgs,
                           w.ftgz, wl, stride, base + 2 * d.rm, ws, 1, C, d.ks, ny, n);
    }
    // lift: u = b / ||b||
    hipLaunchKernelGGL(k_fno_sum_prod<T>, dim3(C), dim3(kBlock), 0, s, w.ftgz, b, nrm2, grad, C, per, batch);
    hipLaunchKernelGGL(k_fno_sum_prod<T>, dim3(C), dim3(kBlock), 0, s, w.ftgz, (const T*)nullptr,
                       (const double*)nullptr, grad + C, C, per, batch);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}
template nmg_status fno_backward<float>(Ctx*, Work<float>&, int, int, int, const float*, const double*, const float*,
                                        float, int, float*, hipStream_t);
template nmg_status fno_backward<double>(Ctx*, Work<double>&, int, int, int, const double*, const double*,
                                         const double*, double, int, double*, hipStream_t);


}  // namespace nmg
