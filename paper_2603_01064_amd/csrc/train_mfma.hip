// Backward pass of the BF16 smoother network on MFMA (mixed-precision
// training: BF16 activations, BF16 weights, FP32 sums, FP32 master weights;
// Sec. 3.4 training, eq. loss_3 adjoint).
//
// For a CNN 1 -> 32 -> ... -> 32 -> 1 with 3x3 kernels and ReLU between the
// layers, one level's backward is
//   recompute  a_1 = relu(conv(u, W_1)),  a_{i+1} = relu(conv(a_i, W_{i+1}))
//              with u = BF16(b / ||b||) and every activation rounded to BF16
//   delta      D_last = [a_last > 0] conv^T(d_out, W_last)
//              D_i    = [a_i > 0] conv^T(D_{i+1}, W_{i+1})      (hidden layers)
//   gradients  dW_last = sum_p d_out[p] a_last[p + off]
//              dW_{i+1} = sum_p D_{i+1}[p] a_i[p + off],  dW_1 = sum_p D_1[p] u[p + off]
// Activations and deltas are pixel-major BF16 records (32 channels, 64 bytes
// per pixel).  The 32 -> 32 layers (recompute, and the data gradient as the
// same convolution with transposed, tap-flipped weights) are implicit GEMMs
// on v_mfma_f32_16x16x32_bf16: output channels as M, 16 pixels of a row as N,
// input channels of one tap as K.  Their weight gradients are GEMMs over
// pixels (output channel x input channel per tap) with the tiles transposed
// to channel-major in LDS.  The one-channel first and last layers run on the
// VALU.  Weight gradients are per-workgroup partial sums added in a fixed
// order, so the result does not depend on scheduling.
#include <algorithm>

#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kThreads = 256;
constexpr int kC = 32;        // hidden channels
constexpr int kT = 16;        // output tile side of the 32 -> 32 kernels
constexpr int kH = kT + 2;    // staged side (one-pixel halo)
constexpr int kWPk = 9 * 2 * 64 * 8;  // packed BF16 elements of one 32 -> 32 layer (one orientation)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats to packed BF16 (hardware round-to-nearest-even).
__device__ inline uint32_t pack2(float a, float b) {
    const float2v f = {a, b};
    const bf16x2 p = __builtin_convertvector(f, bf16x2);
    uint32_t u;
    __builtin_memcpy(&u, &p, 4);
    return u;
}
__device__ inline float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ inline float round_bf(float v) { return bf2f(pack2(v, 0.f) & 0xFFFFu); }

// Packs W [co][ci][9] (FP32) into per-lane MFMA operand order, two
// orientations: out[0 .. kWPk) for the forward convolution (operand M slot =
// output channel co = nb*16 + lane%16, K slot = input channel 8*(lane/16)+j),
// out[kWPk .. 2 kWPk) for the data gradient (M slot = ci, K slot = co, tap
// flipped: t -> 8 - t).  Element ((t*2 + nb)*64 + lane)*8 + j.
__global__ void __launch_bounds__(kThreads) k_tr_pack32(const float* __restrict__ W, uint16_t* __restrict__ out) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= kWPk) return;
    const int t = e / 1024, nb = (e / 512) & 1, lane = (e / 8) & 63, j = e & 7;
    const int m = nb * 16 + (lane & 15), k = 8 * (lane >> 4) + j;
    out[e] = (uint16_t)(pack2(W[(m * kC + k) * 9 + t], 0.f) & 0xFFFFu);
    out[kWPk + e] = (uint16_t)(pack2(W[(k * kC + m) * 9 + (8 - t)], 0.f) & 0xFFFFu);
}

// a_1 = BF16(relu(conv(u, W_1))) with u = BF16(b * (1 / ||b||)); one thread
// per pixel, the nine taps in the order (dy, dx) of the reference kernels.
__global__ void __launch_bounds__(kThreads) k_tr_first_fwd(const float* __restrict__ b, const double* __restrict__ nrm2,
                                                           const float* __restrict__ W1, uint16_t* __restrict__ a1,
                                                           int n) {
    __shared__ float w[kC * 9];
    for (int e = threadIdx.x; e < kC * 9; e += kThreads) w[e] = round_bf(W1[e]);
    __syncthreads();
    const size_t per = (size_t)n * n;
    const int img = blockIdx.y;
    const size_t p = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= per) return;
    const double nb = sqrt(nrm2[img]);
    const float sc = nb > 0.0 ? (float)(1.0 / nb) : 0.f;
    const int y = (int)(p / n), x = (int)(p % n);
    const float* src = b + (size_t)img * per;
    float u[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
        u[t] = (yy >= 0 && yy < n && xx >= 0 && xx < n) ? round_bf(src[(size_t)yy * n + xx] * sc) : 0.f;
    }
    uint32_t pk[kC / 2];
#pragma unroll
    for (int c2 = 0; c2 < kC / 2; ++c2) {
        float v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int co = 2 * c2 + h;
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) acc += w[co * 9 + t] * u[t];
            v[h] = acc > 0.f ? acc : 0.f;
        }
        pk[c2] = pack2(v[0], v[1]);
    }
    uint4* dst = reinterpret_cast<uint4*>(a1 + ((size_t)img * per + p) * kC);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = make_uint4(pk[4 * q], pk[4 * q + 1], pk[4 * q + 2], pk[4 * q + 3]);
}

// One 32 -> 32 3x3 layer on a 16 x 16 pixel tile of one image.
//   MODE 0 (forward):       out = BF16(relu(conv(in, W)))
//   MODE 1 (data gradient): out = BF16([ref > 0] conv(in, W')), W' the
//                           transposed, tap-flipped weights
// The 18 x 18 input records are staged in LDS with chunk g of pixel column c
// at g ^ ((c >> 1) & 3), so a 16-lane operand read is conflict-free.  Wave w
// computes output rows 4w .. 4w + 3; per row and tap one operand read feeds
// two MFMAs (output channels 0..15 and 16..31).
template <int MODE>
__global__ void __launch_bounds__(kThreads) k_tr_conv32(const uint16_t* __restrict__ in,
                                                        const uint16_t* __restrict__ ref, uint16_t* __restrict__ out,
                                                        const uint16_t* __restrict__ wpk, int n, int tiles_x) {
    __shared__ __attribute__((aligned(16))) char S[kH * kH * 64];
    const int img = blockIdx.y, tile = blockIdx.x;
    const int y0 = (tile / tiles_x) * kT, x0 = (tile % tiles_x) * kT;
    const size_t per = (size_t)n * n;
    const uint16_t* src = in + (size_t)img * per * kC;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ln = lane & 15, lg = lane >> 4;
    bf16x8 w[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) w[t][nb] = *reinterpret_cast<const bf16x8*>(wpk + ((t * 2 + nb) * 64 + lane) * 8);
    for (int e = tid; e < kH * kH * 4; e += kThreads) {
        const int pix = e >> 2, g = e & 3;
        const int r = pix / kH, c = pix % kH;
        const int gy = y0 - 1 + r, gx = x0 - 1 + c;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gy >= 0 && gy < n && gx >= 0 && gx < n)
            v = *reinterpret_cast<const uint4*>(src + ((size_t)gy * n + gx) * kC + g * 8);
        *reinterpret_cast<uint4*>(S + (r * kH + c) * 64 + ((g ^ ((c >> 1) & 3)) << 4)) = v;
    }
    __syncthreads();
#pragma unroll 1
    for (int rr = 0; rr < 4; ++rr) {
        const int ry = wave * 4 + rr;
        floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int r = ry + dy, c = ln + dx;
                const bf16x8 bop = *reinterpret_cast<const bf16x8*>(S + (r * kH + c) * 64 + ((lg ^ ((c >> 1) & 3)) << 4));
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                    acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[dy * 3 + dx][nb], bop, acc[nb], 0, 0, 0);
            }
        const int gy = y0 + ry, gx = x0 + ln;
        if (gy < n && gx < n) {
            const size_t pix = (size_t)img * per + (size_t)gy * n + gx;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int co0 = nb * 16 + lg * 4;
                float v[4];
                if constexpr (MODE == 0) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = acc[nb][q] > 0.f ? acc[nb][q] : 0.f;
                } else {
                    // ReLU mask of the forward activation: a BF16 value is positive
                    // exactly when its 16-bit pattern is positive as a signed integer
                    const uint2 rv = *reinterpret_cast<const uint2*>(ref + pix * kC + co0);
                    const short rs[4] = {(short)(rv.x & 0xFFFFu), (short)(rv.x >> 16), (short)(rv.y & 0xFFFFu),
                                         (short)(rv.y >> 16)};
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = rs[q] > 0 ? acc[nb][q] : 0.f;
                }
                *reinterpret_cast<uint2*>(out + pix * kC + co0) = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
            }
        }
    }
}

// Delta of the last hidden activation: D[q][c] = BF16([a[q][c] > 0]
// sum_t w[c][t] d_out[q - off(t)]) for the 32 -> 1 last layer (w BF16-rounded).
__global__ void __launch_bounds__(kThreads) k_tr_last_bwd(const float* __restrict__ dout,
                                                          const uint16_t* __restrict__ a,
                                                          const float* __restrict__ Wl, uint16_t* __restrict__ D,
                                                          int n) {
    __shared__ float w[kC * 9];
    for (int e = threadIdx.x; e < kC * 9; e += kThreads) w[e] = round_bf(Wl[e]);
    __syncthreads();
    const size_t per = (size_t)n * n;
    const int img = blockIdx.y;
    const size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= per) return;
    const int y = (int)(q / n), x = (int)(q % n);
    const float* g = dout + (size_t)img * per;
    float dv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y - t / 3 + 1, xx = x - t % 3 + 1;
        dv[t] = (yy >= 0 && yy < n && xx >= 0 && xx < n) ? g[(size_t)yy * n + xx] : 0.f;
    }
    const size_t rec = ((size_t)img * per + q) * kC;
    const uint4* ap = reinterpret_cast<const uint4*>(a + rec);
    uint4* dp = reinterpret_cast<uint4*>(D + rec);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const uint4 av = ap[qq];
        const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = qq * 8 + 2 * k + h;
                const short as = (short)(h ? (aw[k] >> 16) : (aw[k] & 0xFFFFu));
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < 9; ++t) acc += w[c * 9 + t] * dv[t];
                v[h] = as > 0 ? acc : 0.f;
            }
            o[k] = pack2(v[0], v[1]);
        }
        dp[qq] = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// Gradient at the network input of the first layer (one input channel):
// din[q] = sum_co sum_t w[co][t] D[q - off(t)][co] (FP32 plane).
__global__ void __launch_bounds__(kThreads) k_tr_first_din(const uint16_t* __restrict__ D,
                                                           const float* __restrict__ W1, float* __restrict__ din,
                                                           int n) {
    __shared__ float w[kC * 9];
    for (int e = threadIdx.x; e < kC * 9; e += kThreads) w[e] = round_bf(W1[e]);
    __syncthreads();
    const size_t per = (size_t)n * n;
    const int img = blockIdx.y;
    const size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= per) return;
    const int y = (int)(q / n), x = (int)(q % n);
    float acc = 0.f;
    for (int co = 0; co < kC; ++co)
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y - t / 3 + 1, xx = x - t % 3 + 1;
            if (yy < 0 || yy >= n || xx < 0 || xx >= n) continue;
            const uint16_t h = D[((size_t)img * per + (size_t)yy * n + xx) * kC + co];
            acc += w[co * 9 + t] * bf2f(h);
        }
    din[(size_t)img * per + q] = acc;
}

// Weight-gradient partials of a one-channel layer over a run of rows of one
// image (workgroup g: image g / wpi, rows [(g % wpi) rpw, + rpw)):
//   FIRST: dW_1[c][t] = sum_p D[p][c] u[p + off(t)],  u = BF16(b / ||b||)
//   else : dW_l[c][t] = sum_q a[q][c] d_out[q - off(t)]  (q = p + off(t))
// Both are sum_p A[p][c] B[p][t] with A the 32-channel BF16 record at p and B
// the one-channel plane shifted by the tap, taken on the FP32 MFMA
// (v_mfma_f32_16x16x4f32: M = 16 channels, N = the 9 taps padded to 16, K =
// four pixels of a row), with the FP32 products of the plain loop.  The four
// waves take every fourth quad of a row, each with two accumulator sets
// (alternate quads), added in a fixed order at the end.
// part[blockIdx.x][c * 9 + t] (the layer's [Cout][Cin][3][3] order).
template <int FIRST>
__global__ void __launch_bounds__(kThreads) k_tr_wgrad_small(const float* __restrict__ plane,
                                                             const double* __restrict__ nrm2,
                                                             const uint16_t* __restrict__ rec,
                                                             float* __restrict__ part, int n, int wpi, int rpw) {
    __shared__ floatx4 red[kThreads / 64][2][64];
    const int img = blockIdx.x / wpi;
    const int y0 = (blockIdx.x % wpi) * rpw, y1 = y0 + rpw < n ? y0 + rpw : n;
    const size_t base = (size_t)img * n * n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;  // A: channel m of pixel kq; B: tap m of pixel kq
    float sc = 0.f;
    if constexpr (FIRST) {
        const double nb = sqrt(nrm2[img]);
        sc = nb > 0.0 ? (float)(1.0 / nb) : 0.f;
    }
    const bool tap_ok = m < 9;
    const int dy = m / 3 - 1, dx = m % 3 - 1;
    const int sy = FIRST ? dy : -dy, sx = FIRST ? dx : -dx;  // B reads the plane at p + (sy, sx)
    const int nq = (n + 3) / 4;
    floatx4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
        for (int cb = 0; cb < 2; ++cb) acc[u][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto quad = [&](int y, int xq, floatx4* ac) {
        const int x = 4 * xq + kq;
        const bool px = x < n;
        const size_t p = base + (size_t)y * n + x;
        const float a0 = px ? bf2f(rec[p * kC + m]) : 0.f;
        const float a1 = px ? bf2f(rec[p * kC + 16 + m]) : 0.f;
        const int yy = y + sy, xx = x + sx;
        float bv = 0.f;
        if (px && tap_ok && yy >= 0 && yy < n && xx >= 0 && xx < n) {
            const float v = plane[base + (size_t)yy * n + xx];
            bv = FIRST ? round_bf(v * sc) : v;
        }
        ac[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bv, ac[0], 0, 0, 0);
        ac[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bv, ac[1], 0, 0, 0);
    };
    for (int y = y0; y < y1; ++y) {
        int xq = wave;
        for (; xq + 4 < nq; xq += 8) {
            quad(y, xq, acc[0]);
            quad(y, xq + 4, acc[1]);
        }
        if (xq < nq) quad(y, xq, acc[0]);
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) red[wave][cb][lane] = acc[0][cb] + acc[1][cb];
    __syncthreads();
    // D lane l: channel 16 cb + 4 (l >> 4) + i, tap l & 15
    for (int e = threadIdx.x; e < 2 * 64 * 4; e += kThreads) {
        const int cb = e >> 8, l = (e >> 2) & 63, i = e & 3;
        float v = 0.f;
        for (int w = 0; w < kThreads / 64; ++w) v += red[w][cb][l][i];
        const int c = cb * 16 + 4 * (l >> 4) + i, t = l & 15;
        if (t < 9) part[(size_t)blockIdx.x * (kC * 9) + c * 9 + t] = v;
    }
}

// Weight-gradient partials of a 32 -> 32 layer:
//   dW[co][ci][t] = sum_p D[p][co] X[p + off(t)][ci]
// Workgroup g takes tiles_per_wg consecutive 16 x 16 tiles of one image.
// Per tile, D (16 x 16 pixels) and X (18 x 18 with the halo) are transposed
// to channel-major BF16 in LDS: Dt[co][pixel] and, for each column shift dx,
// Xs[dx][ci][row][col] = X[row][col + dx], so every operand fragment (8
// consecutive pixels of one channel) is one aligned 16-byte read.  Wave w
// owns output-channel block w >> 1 and input-channel block w & 1 for all nine
// taps: per K step of 32 pixels (two tile rows) one D fragment feeds nine
// MFMAs.  part[g][(co * 32 + ci) * 9 + t].
__global__ void __launch_bounds__(kThreads) k_tr_wgrad32(const uint16_t* __restrict__ D, const uint16_t* __restrict__ X,
                                                         float* __restrict__ part, int n, int tiles_x,
                                                         int tiles_per_wg, int wg_per_img) {
    __shared__ __attribute__((aligned(16))) uint16_t Dt[kC * kT * kT];
    __shared__ __attribute__((aligned(16))) uint16_t Xs[3 * kC * kH * kT];
    const int img = blockIdx.x / wg_per_img, part_i = blockIdx.x % wg_per_img;
    const int ntiles = tiles_x * tiles_x;
    const int t0 = part_i * tiles_per_wg, t1 = t0 + tiles_per_wg < ntiles ? t0 + tiles_per_wg : ntiles;
    const size_t per = (size_t)n * n;
    const uint16_t* Ds = D + (size_t)img * per * kC;
    const uint16_t* Xg = X + (size_t)img * per * kC;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ln = lane & 15, lg = lane >> 4;
    const int mb = wave >> 1, cb = wave & 1;
    floatx4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int tile = t0; tile < t1; ++tile) {
        const int y0 = (tile / tiles_x) * kT, x0 = (tile % tiles_x) * kT;
        __syncthreads();  // the previous tile's operands have been read
        for (int e = tid; e < kT * kT * 4; e += kThreads) {
            const int px = e >> 2, g = e & 3;
            const int gy = y0 + px / kT, gx = x0 + px % kT;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (gy < n && gx < n) v = *reinterpret_cast<const uint4*>(Ds + ((size_t)gy * n + gx) * kC + g * 8);
            const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 8; ++j)
                Dt[(g * 8 + j) * (kT * kT) + px] = (uint16_t)((j & 1) ? (vw[j >> 1] >> 16) : (vw[j >> 1] & 0xFFFFu));
        }
        for (int e = tid; e < kH * kH * 4; e += kThreads) {
            const int pix = e >> 2, g = e & 3;
            const int hr = pix / kH, hc = pix % kH;
            const int gy = y0 - 1 + hr, gx = x0 - 1 + hc;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (gy >= 0 && gy < n && gx >= 0 && gx < n)
                v = *reinterpret_cast<const uint4*>(Xg + ((size_t)gy * n + gx) * kC + g * 8);
            const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int col = hc - dx;
                if (col < 0 || col >= kT) continue;
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    Xs[((dx * kC + g * 8 + j) * kH + hr) * kT + col] =
                        (uint16_t)((j & 1) ? (vw[j >> 1] >> 16) : (vw[j >> 1] & 0xFFFFu));
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < kT / 2; ++k) {
            const int row = 2 * k + (lg >> 1), col = 8 * (lg & 1);
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(Dt + (mb * 16 + ln) * (kT * kT) + row * kT + col);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const bf16x8 bop =
                        *reinterpret_cast<const bf16x8*>(Xs + ((dx * kC + cb * 16 + ln) * kH + row + dy) * kT + col);
                    acc[dy * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bop, acc[dy * 3 + dx], 0, 0, 0);
                }
        }
    }
    // acc[t][q] is (co = 16 mb + 4 lg + q, ci = 16 cb + ln, tap t)
    float* out = part + (size_t)blockIdx.x * (kC * kC * 9);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) out[((mb * 16 + lg * 4 + q) * kC + cb * 16 + ln) * 9 + t] = acc[t][q];
}

// grad (+)= the sum of `chunks` partials of `count` values, in a fixed order:
// stage 1 adds group k's run of consecutive partials into tmp[k] (FP64),
// stage 2 adds the groups in order.
constexpr int kReduceGroups = 64;

__global__ void __launch_bounds__(kThreads) k_tr_reduce1(const float* __restrict__ part, double* __restrict__ tmp,
                                                         int count, int chunks, int per_group) {
    const int w = blockIdx.x * kThreads + threadIdx.x, k = blockIdx.y;
    if (w >= count) return;
    const int c0 = k * per_group, c1 = c0 + per_group < chunks ? c0 + per_group : chunks;
    double acc = 0.0;
    for (int c = c0; c < c1; ++c) acc += (double)part[(size_t)c * count + w];
    tmp[(size_t)k * count + w] = acc;
}

__global__ void __launch_bounds__(kThreads) k_tr_reduce2(const double* __restrict__ tmp, float* __restrict__ grad,
                                                         int count, int groups, int accumulate) {
    const int w = blockIdx.x * kThreads + threadIdx.x;
    if (w >= count) return;
    double acc = 0.0;
    for (int k = 0; k < groups; ++k) acc += tmp[(size_t)k * count + w];
    grad[w] = accumulate ? (float)((double)grad[w] + acc) : (float)acc;
}

}  // namespace

bool mfma_backward_supported(const Ctx* c) {
    const nmg_problem& p = c->p;
    if (p.smoother_arch != NMG_ARCH_CNN || p.dim != 2 || p.ksize != 3 || p.n_layers < 3) return false;
    if (p.channels[0] != 1 || p.channels[p.n_layers] != 1) return false;
    for (int i = 1; i < p.n_layers; ++i)
        if (p.channels[i] != kC) return false;
    return true;
}

size_t mfma_backward_wpk_elems(const Ctx* c) { return (size_t)std::max(1, c->p.n_layers - 2) * 2 * kWPk; }

size_t mfma_backward_reduce_elems() { return (size_t)kReduceGroups * kC * kC * 9; }

nmg_status smoother_backward_mfma(const Ctx* c, const MfmaBackwardArgs& a, hipStream_t s) {
    const int n = a.n, NL = c->p.n_layers, batch = a.batch;
    const size_t per = (size_t)n * n, total = (size_t)batch * per;
    const int tiles_x = (n + kT - 1) / kT;
    const unsigned gpx = (unsigned)((per + kThreads - 1) / kThreads);
    if (NL - 1 > (int)a.acts.size()) return fail(NMG_ERR_STATE, "MFMA backward: too few activation buffers");
    // packed weights of the hidden layers (both orientations)
    for (int i = 1; i + 1 < NL; ++i)
        hipLaunchKernelGGL(k_tr_pack32, dim3((kWPk + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                           a.W + c->layer_off[(size_t)i], a.wpk + (size_t)(i - 1) * 2 * kWPk);
    // recompute a_1 .. a_{NL-1}
    hipLaunchKernelGGL(k_tr_first_fwd, dim3(gpx, batch), dim3(kThreads), 0, s, a.b, a.nrm2, a.W + c->layer_off[0],
                       a.acts[0], n);
    for (int i = 1; i + 1 < NL; ++i)
        hipLaunchKernelGGL((k_tr_conv32<0>), dim3((unsigned)(tiles_x * tiles_x), batch), dim3(kThreads), 0, s,
                           a.acts[(size_t)i - 1], (const uint16_t*)nullptr, a.acts[(size_t)i],
                           a.wpk + (size_t)(i - 1) * 2 * kWPk, n, tiles_x);
    auto reduce = [&](int layer, int cnt, int chunks) {
        const int per_group = (chunks + kReduceGroups - 1) / kReduceGroups;
        const int groups = (chunks + per_group - 1) / per_group;
        const unsigned gx = (unsigned)((cnt + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_tr_reduce1, dim3(gx, (unsigned)groups), dim3(kThreads), 0, s, a.part, a.reduce_tmp, cnt,
                           chunks, per_group);
        hipLaunchKernelGGL(k_tr_reduce2, dim3(gx), dim3(kThreads), 0, s, a.reduce_tmp,
                           a.grad + c->layer_off[(size_t)layer], cnt, groups, a.accumulate);
    };
    // one-channel layers: runs of rpw rows, at most 4096 partials
    // (batch * ceil(n / rpw) can exceed batch * n / rpw by up to batch)
    const size_t cap = a.part_count / (kC * 9);
    const size_t max_small = std::min<size_t>((size_t)4096, cap > (size_t)2 * batch ? cap - batch : 1);
    const int rpw = (int)std::max<size_t>(1, ((size_t)batch * n + max_small - 1) / max_small);
    const int wpi = (n + rpw - 1) / rpw;
    const int small_used = batch * wpi;
    if ((size_t)small_used > cap) return fail(NMG_ERR_STATE, "MFMA backward: one-channel partials exceed the scratch");
    (void)total;
    // last layer: its weight gradient and the delta of a_{NL-1}
    const uint16_t* a_last = a.acts[(size_t)NL - 2];
    hipLaunchKernelGGL((k_tr_wgrad_small<0>), dim3(small_used), dim3(kThreads), 0, s, a.dout, (const double*)nullptr,
                       a_last, a.part, n, wpi, rpw);
    reduce(NL - 1, kC * 9, small_used);
    uint16_t* dcur = a.d0;
    uint16_t* dnext = a.d1;
    hipLaunchKernelGGL(k_tr_last_bwd, dim3(gpx, batch), dim3(kThreads), 0, s, a.dout, a_last,
                       a.W + c->layer_off[(size_t)NL - 1], dcur, n);
    // hidden layers NL-2 .. 1 (weights W_{i+1} map a_i to a_{i+1})
    // about 1024 workgroups in all, within the partials scratch
    const int fit = (int)std::min<size_t>((size_t)1 << 20, a.part_count / ((size_t)kC * kC * 9 * batch));
    const int wg_per_img = std::max(1, std::min({tiles_x * tiles_x, (1024 + batch - 1) / batch, fit}));
    const int tiles_per_wg = (tiles_x * tiles_x + wg_per_img - 1) / wg_per_img;
    const int wg_total = batch * wg_per_img;
    if ((size_t)wg_total * kC * kC * 9 > a.part_count)
        return fail(NMG_ERR_STATE, "MFMA backward: weight-gradient partials exceed the scratch");
    for (int i = NL - 2; i >= 1; --i) {
        const uint16_t* X = a.acts[(size_t)i - 1];
        hipLaunchKernelGGL(k_tr_wgrad32, dim3((unsigned)wg_total), dim3(kThreads), 0, s, dcur, X, a.part, n, tiles_x,
                           tiles_per_wg, wg_per_img);
        reduce(i, kC * kC * 9, wg_total);
        hipLaunchKernelGGL((k_tr_conv32<1>), dim3((unsigned)(tiles_x * tiles_x), batch), dim3(kThreads), 0, s, dcur,
                           X, dnext, a.wpk + (size_t)(i - 1) * 2 * kWPk + kWPk, n, tiles_x);
        std::swap(dcur, dnext);
    }
    // first layer
    hipLaunchKernelGGL((k_tr_wgrad_small<1>), dim3(small_used), dim3(kThreads), 0, s, a.b, a.nrm2,
                       (const uint16_t*)dcur, a.part, n, wpi, rpw);
    reduce(0, kC * 9, small_used);
    if (a.din0)
        hipLaunchKernelGGL(k_tr_first_din, dim3(gpx, batch), dim3(kThreads), 0, s, (const uint16_t*)dcur,
                           a.W + c->layer_off[0], a.din0, n);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

}  // namespace nmg
