// Smoothing steps in FP64 / FP32 (parity and plain-FP32 paths).
//
// Neural smoother (Algorithm 2 and Algorithm 4, pre-smoothing line):
//   h = ||b||_2 N_theta(b / ||b||_2)
// with N_theta a bias-free CNN (conv, ReLU, ..., conv), cross-correlation
// with zero "same" padding.  Weighted Jacobi (Sec. 2.2): h = omega D^{-1} b.
//
// FP64 (and shapes other than 2D 3x3 with 1 or 32 channels) use a direct
// convolution with one output (pixel, channel) per thread; 2D FP32 layers of
// the workloads' networks use a tiled kernel (16 x 16 output pixels per
// workgroup, every output channel of a pixel per thread, input channels and
// weights staged in LDS).  Activations go through global memory between
// layers in both; the fast BF16 path lives in the MFMA smoother.
#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kBlock = 256;

// One conv layer.  in: [B][cin][ny][n]; out: [B][cout][ny][n].
// first: input is the residual (1 channel) scaled by 1/||b||.
// last : output is multiplied by ||b|| and written (or added) to dst [B][ny][n].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_conv(const T* __restrict__ in, T* __restrict__ out,
                                                 const T* __restrict__ wlevel, const int* __restrict__ ws,
                                                 int nsets, int wcount, int layer_off, int cin, int cout, int kh, int kw,
                                                 int ny, int n, int relu, int first, int last, int accumulate,
                                                 const double* __restrict__ nrm2) {
    const size_t per = (size_t)ny * n;
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    const int co = blockIdx.y;
    const int b = blockIdx.z;
    const int y = (int)(e / n), x = (int)(e % n);
    // out-of-range set indices are clamped so that a bad index cannot read past the weights
    const int set = ws ? min(max(ws[b], 0), nsets - 1) : 0;
    const T* w = wlevel + (size_t)set * wcount + layer_off + (size_t)co * cin * kh * kw;
    const double nb = sqrt(nrm2[b]);
    const T inscale = first ? (nb > 0.0 ? (T)(1.0 / nb) : (T)0) : (T)1;
    const T* src = in + (size_t)b * cin * per;
    T acc = 0;
    const int py = kh / 2, px = kw / 2;
    for (int ci = 0; ci < cin; ++ci) {
        const T* plane = src + (size_t)ci * per;
        const T* wc = w + (size_t)ci * kh * kw;
        for (int dy = 0; dy < kh; ++dy) {
            const int yy = y + dy - py;
            if (yy < 0 || yy >= ny) continue;
            for (int dx = 0; dx < kw; ++dx) {
                const int xx = x + dx - px;
                if (xx < 0 || xx >= n) continue;
                acc += wc[dy * kw + dx] * plane[(size_t)yy * n + xx];
            }
        }
    }
    acc *= inscale;
    if (relu && acc < (T)0) acc = (T)0;
    if (last) {
        const T v = acc * (T)nb;
        T* d = out + (size_t)b * per + e;
        *d = accumulate ? *d + v : v;
    } else {
        out[((size_t)b * cout + co) * per + e] = acc;
    }
}

// One 2D 3x3 FP32 layer, CIN -> COUT channels: workgroup = 16 x 16 output
// pixels of one image, thread = one pixel with all COUT accumulators.  The
// input channels are staged CC at a time as 18 x 18 tiles (zero outside the
// image) together with their weights ([ci][tap][co], read as broadcasts).
// The sum runs over input channels in order, taps in row-major order, as the
// direct kernel's; FIRST scales the sum by 1/||b|| afterwards, LAST writes
// ||b|| times the (only) output channel to dst, other layers apply ReLU.
constexpr int kTile = 16;

template <int CIN, int COUT, bool FIRST, bool LAST>
__global__ void __launch_bounds__(kTile * kTile) k_conv3_tiled(const float* __restrict__ in, float* __restrict__ out,
                                                                const float* __restrict__ wlevel,
                                                                const int* __restrict__ ws, int nsets, int wcount,
                                                                int layer_off, int n, int tiles_x, int accumulate,
                                                                const double* __restrict__ nrm2) {
    constexpr int H = kTile + 2, CC = CIN < 8 ? CIN : 8;
    static_assert(CIN % CC == 0 && (!LAST || COUT == 1), "layer shape");
    __shared__ float xs[CC][H][H];
    __shared__ __attribute__((aligned(16))) float wsm[CC][9][COUT];
    const int b = blockIdx.y;
    const int ty0 = (blockIdx.x / tiles_x) * kTile, tx0 = (blockIdx.x % tiles_x) * kTile;
    const int tid = threadIdx.x, ty = tid / kTile, tx = tid % kTile;
    // out-of-range set indices are clamped so that a bad index cannot read past the weights
    const int set = ws ? min(max(ws[b], 0), nsets - 1) : 0;
    const float* w = wlevel + (size_t)set * wcount + layer_off;  // [COUT][CIN][3][3]
    const size_t per = (size_t)n * n;
    const float* src = in + (size_t)b * CIN * per;
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = 0.f;
    for (int c0 = 0; c0 < CIN; c0 += CC) {
        __syncthreads();  // the previous chunk has been read
        for (int e = tid; e < CC * H * H; e += kTile * kTile) {
            const int ci = e / (H * H), rem = e - ci * (H * H), r = rem / H, c = rem - r * H;
            const int gy = ty0 - 1 + r, gx = tx0 - 1 + c;
            xs[ci][r][c] = (gy >= 0 && gy < n && gx >= 0 && gx < n) ? src[(size_t)(c0 + ci) * per + (size_t)gy * n + gx]
                                                                     : 0.f;
        }
        for (int e = tid; e < CC * 9 * COUT; e += kTile * kTile) {
            const int co = e % COUT, t = (e / COUT) % 9, ci = e / (9 * COUT);
            wsm[ci][t][co] = w[((size_t)co * CIN + c0 + ci) * 9 + t];
        }
        __syncthreads();
#pragma unroll 2
        for (int ci = 0; ci < CC; ++ci)
#pragma unroll 3
            for (int t = 0; t < 9; ++t) {
                const float x = xs[ci][ty + t / 3][tx + t % 3];
#pragma unroll
                for (int co = 0; co < COUT; ++co) acc[co] = fmaf(wsm[ci][t][co], x, acc[co]);
            }
    }
    const int gy = ty0 + ty, gx = tx0 + tx;
    if (gy >= n || gx >= n) return;
    const double nb = sqrt(nrm2[b]);
    if (FIRST) {
        const float inscale = nb > 0.0 ? (float)(1.0 / nb) : 0.f;
#pragma unroll
        for (int co = 0; co < COUT; ++co) acc[co] *= inscale;
    }
    const size_t pix = (size_t)gy * n + gx;
    if (LAST) {
        const float v = acc[0] * (float)nb;
        float* d = out + (size_t)b * per + pix;
        *d = accumulate ? *d + v : v;
    } else {
#pragma unroll
        for (int co = 0; co < COUT; ++co) out[((size_t)b * COUT + co) * per + pix] = acc[co] < 0.f ? 0.f : acc[co];
    }
}

// Weighted Jacobi: h = omega b / diag(A_l), diag = alpha m_i m_j + g_i g_j (2D).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_jacobi(const T* __restrict__ bres, T* __restrict__ dst,
                                                   const T* __restrict__ G, int rg, const T* __restrict__ M, int rm,
                                                   const double* __restrict__ alpha, double omega, int n, int two_d,
                                                   int accumulate) {
    const size_t per = (size_t)(two_d ? n : 1) * n;
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    const int b = blockIdx.y;
    const int i = (int)(e / n), j = (int)(e % n);
    const T a = (T)alpha[b];
    const T gj = G[(size_t)j * (2 * rg + 1) + rg], mj = M[(size_t)j * (2 * rm + 1) + rm];
    T d;
    if (two_d) {
        const T gi = G[(size_t)i * (2 * rg + 1) + rg], mi = M[(size_t)i * (2 * rm + 1) + rm];
        d = a * mi * mj + gi * gj;
    } else {
        d = a * mj + gj;
    }
    const T v = (T)omega * bres[(size_t)b * per + e] / d;
    T* o = dst + (size_t)b * per + e;
    *o = accumulate ? *o + v : v;
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

template <typename T>
nmg_status launch_conv_smoother(const Ctx* c, int l, int batch, const int* ws, const T* b, const double* nrm2,
                                T* dst, int accumulate, Work<T>& w, hipStream_t s) {
    const int n = c->n[l];
    const int ny = c->p.dim == 2 ? n : 1;
    const int kh = c->p.dim == 2 ? c->p.ksize : 1, kw = c->p.ksize;
    const size_t per = (size_t)ny * n;
    const T* wl = w.wts + (size_t)l * c->p.n_weight_sets * c->wcount;
    const int nl = c->p.n_layers;
    const T* src = b;
    if (!w.act0 || !w.act1) return fail(NMG_ERR_STATE, "convolution smoother buffers not allocated");
    T* bufs[2] = {w.act0, w.act1};
    for (int i = 0; i < nl; ++i) {
        const int cin = c->p.channels[i], cout = c->p.channels[i + 1];
        const int first = i == 0, last = i == nl - 1;
        T* out = last ? dst : bufs[i & 1];
        if constexpr (sizeof(T) == 4) {
            // tiled FP32 layers for the shapes of the workloads' networks
            if (c->p.dim == 2 && c->p.ksize == 3) {
                const int tiles_x = (n + kTile - 1) / kTile;
                const dim3 tg((unsigned)(tiles_x * tiles_x), (unsigned)batch);
                bool done = true;
                if (cin == 1 && cout == 32 && first && !last)
                    hipLaunchKernelGGL((k_conv3_tiled<1, 32, true, false>), tg, dim3(kTile * kTile), 0, s, src, out,
                                       wl, ws, c->p.n_weight_sets, c->wcount, c->layer_off[i], n, tiles_x, 0, nrm2);
                else if (cin == 32 && cout == 32 && !first && !last)
                    hipLaunchKernelGGL((k_conv3_tiled<32, 32, false, false>), tg, dim3(kTile * kTile), 0, s, src, out,
                                       wl, ws, c->p.n_weight_sets, c->wcount, c->layer_off[i], n, tiles_x, 0, nrm2);
                else if (cin == 32 && cout == 1 && !first && last)
                    hipLaunchKernelGGL((k_conv3_tiled<32, 1, false, true>), tg, dim3(kTile * kTile), 0, s, src, out,
                                       wl, ws, c->p.n_weight_sets, c->wcount, c->layer_off[i], n, tiles_x,
                                       accumulate, nrm2);
                else
                    done = false;
                if (done) {
                    src = out;
                    continue;
                }
            }
        }
        dim3 grid(blocks_for(per), last ? 1 : cout, batch);
        hipLaunchKernelGGL(k_conv<T>, grid, dim3(kBlock), 0, s, src, out, wl, ws, c->p.n_weight_sets, c->wcount,
                           c->layer_off[i], cin,
                           cout, kh, kw, ny, n, last ? 0 : 1, first, last, accumulate, nrm2);
        src = out;
    }
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

template <typename T>
nmg_status launch_jacobi(const Ctx* c, int l, int batch, const double* alpha, double omega, const T* b, T* dst,
                         int accumulate, Work<T>& w, hipStream_t s) {
    const int n = c->n[l];
    const size_t per = level_elems(c, l);
    const HostLevel& hl = c->host[l];
    hipLaunchKernelGGL(k_jacobi<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, b, dst, w.Gd + w.g_off[l],
                       hl.G.r, w.Md + w.m_off[l], hl.M.r, alpha, omega, n, c->p.dim == 2 ? 1 : 0, accumulate);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

#define NMG_INST(T)                                                                                            \
    template nmg_status launch_conv_smoother<T>(const Ctx*, int, int, const int*, const T*, const double*, T*, \
                                                int, Work<T>&, hipStream_t);                                   \
    template nmg_status launch_jacobi<T>(const Ctx*, int, int, const double*, double, const T*, T*, int,       \
                                         Work<T>&, hipStream_t);
NMG_INST(float)
NMG_INST(double)
#undef NMG_INST

}  // namespace nmg
