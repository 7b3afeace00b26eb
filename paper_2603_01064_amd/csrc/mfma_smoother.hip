// Neural smoother h = ||b|| N(b/||b||) in BF16 on MFMA with FP32 accumulation
// (the smoothing line of Algorithm 4; N = Conv2d 1->32->...->32->1, 3x3,
// ReLU between layers, no bias, zero "same" padding).
//
// One workgroup produces a 16x16 output tile of one image and keeps every
// intermediate activation of that tile in LDS: the input tile carries a
// halo of one pixel per layer, layer i is evaluated on the tile grown by
// (layers - i) pixels per side, and activations that fall outside the image
// are stored as zero so each layer sees exactly the zero padding of a
// separate convolution.  Each layer is an implicit GEMM with the output
// channels as the MFMA M dimension, 16 pixels as N and (input channel, tap)
// as K:
//   first layer   1 -> 32 : K = 9 taps (padded to 16), v_mfma 16x16x16 bf16
//   hidden layers 32 -> 32: per tap K = 32 channels,    v_mfma 16x16x32 bf16
//   last layer    32 -> 1 : Z[p][t] = sum_c act[p][c] w[c][t] with t as M,
//                           then out[p] = sum_t Z[p + off(t)][t]
// Weights are packed once per weight set into the per-lane operand order and
// kept in registers while a workgroup walks the tiles of its image.
#include <vector>

#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kT = 16;        // output tile side
constexpr int kThreads = 256; // 4 waves
constexpr int kC = 32;        // hidden channels

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f2bf(float f) {
    // round to nearest even (inputs are finite)
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Byte offset of channel chunk g (8 channels, 16 B) of pixel p in an
// activation buffer; the XOR spreads consecutive pixels over LDS banks.
__device__ inline int act_off(int p, int g) { return p * 64 + ((g ^ (p & 3)) << 4); }

template <int NL>
struct Geo {
    static constexpr int S0 = kT + 2 * NL;                 // input tile side
    static constexpr int side(int i) { return kT + 2 * (NL - i); }  // output region of layer i (1-based)
    static constexpr int in_bytes = ((S0 * S0 * 2 + 255) / 256) * 256;
    static constexpr int bufA = side(1) * side(1) * 64;
    static constexpr int bufB_act = NL >= 3 ? side(2) * side(2) * 64 : 0;
    static constexpr int z_bytes = side(NL - 1) * side(NL - 1) * 64;
    static constexpr int bufB = bufB_act > z_bytes ? bufB_act : z_bytes;
    static constexpr int lds = in_bytes + bufA + bufB;
};

// Packed weight block (uint16 bf16) per (level, set):
//   first : [nb 2][lane 64][4]          co = nb*16 + lane%16, tap = 4*(lane/16)+j (0 if >= 9)
//   hidden: [layer][tap 9][nb 2][lane 64][8]  co = nb*16 + lane%16, ci = 8*(lane/16)+j
//   last  : [lane 64][8]                t = lane%16 (0 if >= 9), ci = 8*(lane/16)+j
constexpr int kFirstElems = 2 * 64 * 4;
constexpr int kHiddenElems = 9 * 2 * 64 * 8;
constexpr int kLastElems = 64 * 8;

inline size_t packed_elems(int n_hidden) { return (size_t)kFirstElems + (size_t)n_hidden * kHiddenElems + kLastElems; }

template <int NL>
__global__ void __launch_bounds__(kThreads) k_smoother_mfma(const float* __restrict__ bres,
                                                            const double* __restrict__ nrm2, float* __restrict__ dst,
                                                            int accumulate, const uint16_t* __restrict__ wlevel,
                                                            size_t set_stride, const int* __restrict__ ws, int n,
                                                            int tiles_x, int tiles_per_img) {
    constexpr int NH = NL - 2;
    using G = Geo<NL>;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    uint16_t* in_t = reinterpret_cast<uint16_t*>(smem);
    char* bufA = smem + G::in_bytes;
    char* bufB = bufA + G::bufA;

    const int img = blockIdx.y;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int ln = lane & 15;   // N index (pixel within group)
    const int lg = lane >> 4;   // K group / output row group

    const int set = ws ? ws[img] : 0;
    const uint16_t* wp = wlevel + (size_t)set * set_stride;

    // weights into registers (kept for all tiles of this image)
    short4v w1[2];
    for (int nb = 0; nb < 2; ++nb) w1[nb] = *reinterpret_cast<const short4v*>(wp + (nb * 64 + lane) * 4);
    bf16x8 wh[NH > 0 ? NH : 1][9][2];
    for (int h = 0; h < NH; ++h)
        for (int t = 0; t < 9; ++t)
            for (int nb = 0; nb < 2; ++nb)
                wh[h][t][nb] = *reinterpret_cast<const bf16x8*>(wp + kFirstElems + (size_t)h * kHiddenElems +
                                                                ((t * 2 + nb) * 64 + lane) * 8);
    const bf16x8 wl = *reinterpret_cast<const bf16x8*>(wp + kFirstElems + (size_t)NH * kHiddenElems + lane * 8);

    const size_t per = (size_t)n * n;
    const float* src = bres + (size_t)img * per;
    float* out = dst + (size_t)img * per;
    const double nb2 = nrm2[img];
    const float nbf = (float)sqrt(nb2);
    const float inv = nb2 > 0.0 ? (float)(1.0 / sqrt(nb2)) : 0.f;

    for (int tile = blockIdx.x; tile < tiles_per_img; tile += gridDim.x) {
        const int ty0 = (tile / tiles_x) * kT, tx0 = (tile % tiles_x) * kT;
        // ---- input tile (halo NL), scaled by 1/||b||, zero outside the image
        {
            constexpr int S0 = G::S0;
            for (int e = tid; e < S0 * S0; e += kThreads) {
                const int gy = ty0 - NL + e / S0, gx = tx0 - NL + e % S0;
                float v = 0.f;
                if (gy >= 0 && gy < n && gx >= 0 && gx < n) v = src[(size_t)gy * n + gx] * inv;
                in_t[e] = f2bf(v);
            }
        }
        __syncthreads();
        // ---- first layer 1 -> 32 on region side(1)
        {
            constexpr int S = G::side(1), SI = G::S0, H = NL - 1;
            constexpr int npx = S * S, ngr = (npx + 15) / 16;
            for (int gi = wave; gi < ngr; gi += 4) {
                const int q = min(gi * 16 + ln, npx - 1);
                const int ry = q / S, rx = q % S;
                short4v bop;
                for (int j = 0; j < 4; ++j) {
                    const int tap = lg * 4 + j;
                    uint16_t v = 0;
                    if (tap < 9) v = in_t[(ry + tap / 3) * SI + rx + tap % 3];
                    bop[j] = (short)v;
                }
                const int gy = ty0 - H + ry, gx = tx0 - H + rx;
                const bool inside = gy >= 0 && gy < n && gx >= 0 && gx < n && (gi * 16 + ln) < npx;
                for (int nb = 0; nb < 2; ++nb) {
                    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[nb], bop, acc, 0, 0, 0);
                    if ((gi * 16 + ln) < npx) {
                        const int co = nb * 16 + lg * 4;
                        uint32_t lo = 0, hi = 0;
                        if (inside) {
                            lo = (uint32_t)f2bf(fmaxf(acc[0], 0.f)) | ((uint32_t)f2bf(fmaxf(acc[1], 0.f)) << 16);
                            hi = (uint32_t)f2bf(fmaxf(acc[2], 0.f)) | ((uint32_t)f2bf(fmaxf(acc[3], 0.f)) << 16);
                        }
                        uint2* p = reinterpret_cast<uint2*>(bufA + act_off(q, co >> 3) + (co & 7) * 2);
                        *p = make_uint2(lo, hi);
                    }
                }
            }
        }
        __syncthreads();
        // ---- hidden layers 32 -> 32 (ping-pong between bufA and bufB)
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int layer = 2 + h;  // 1-based layer index
            const int S = kT + 2 * (NL - layer), SI = S + 2, H = NL - layer;
            const int npx = S * S, ngr = (npx + 15) / 16;
            const char* ain = (h & 1) ? bufB : bufA;
            char* aout = (h & 1) ? bufA : bufB;
            for (int gi = wave; gi < ngr; gi += 4) {
                const int q = min(gi * 16 + ln, npx - 1);
                const int ry = q / S, rx = q % S;
                floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const int p = (ry + t / 3) * SI + rx + t % 3;
                    const bf16x8 bop = *reinterpret_cast<const bf16x8*>(ain + act_off(p, lg));
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[h][t][0], bop, acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[h][t][1], bop, acc1, 0, 0, 0);
                }
                if ((gi * 16 + ln) < npx) {
                    const int gy = ty0 - H + ry, gx = tx0 - H + rx;
                    const bool inside = gy >= 0 && gy < n && gx >= 0 && gx < n;
                    for (int nb = 0; nb < 2; ++nb) {
                        const floatx4 a = nb ? acc1 : acc0;
                        const int co = nb * 16 + lg * 4;
                        uint32_t lo = 0, hi = 0;
                        if (inside) {
                            lo = (uint32_t)f2bf(fmaxf(a[0], 0.f)) | ((uint32_t)f2bf(fmaxf(a[1], 0.f)) << 16);
                            hi = (uint32_t)f2bf(fmaxf(a[2], 0.f)) | ((uint32_t)f2bf(fmaxf(a[3], 0.f)) << 16);
                        }
                        uint2* pp = reinterpret_cast<uint2*>(aout + act_off(q, co >> 3) + (co & 7) * 2);
                        *pp = make_uint2(lo, hi);
                    }
                }
            }
            __syncthreads();
        }
        // ---- last layer 32 -> 1: Z[p][t] on region side(NL-1), then gather
        {
            constexpr int S = G::side(NL - 1);
            constexpr int npx = S * S, ngr = (npx + 15) / 16;
            const char* ain = (NH & 1) ? bufB : bufA;
            float* Z = reinterpret_cast<float*>((NH & 1) ? bufA : bufB);
            for (int gi = wave; gi < ngr; gi += 4) {
                const int q = min(gi * 16 + ln, npx - 1);
                const bf16x8 bop = *reinterpret_cast<const bf16x8*>(ain + act_off(q, lg));
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, bop, acc, 0, 0, 0);
                if ((gi * 16 + ln) < npx && lg < 3) *reinterpret_cast<floatx4*>(Z + q * 16 + lg * 4) = acc;
            }
            __syncthreads();
            const int oy = tid / kT, ox = tid % kT;
            const int gy = ty0 + oy, gx = tx0 + ox;
            if (gy < n && gx < n) {
                float v = 0.f;
#pragma unroll
                for (int t = 0; t < 9; ++t) v += Z[((oy + t / 3) * S + ox + t % 3) * 16 + t];
                v *= nbf;
                float* o = out + (size_t)gy * n + gx;
                *o = accumulate ? *o + v : v;
            }
        }
        __syncthreads();
    }
}

bool mfma_supported(const Ctx* c, std::string* why) {
    const nmg_problem& p = c->p;
    if (p.dim != 2 || p.ksize != 3) {
        if (why) *why = "BF16 MFMA smoother supports 2D 3x3 networks only";
        return false;
    }
    if (p.n_layers != 3 && p.n_layers != 4) {
        if (why) *why = "BF16 MFMA smoother supports 3 or 4 conv layers";
        return false;
    }
    for (int i = 1; i < p.n_layers; ++i)
        if (p.channels[i] != kC) {
            if (why) *why = "BF16 MFMA smoother needs 32 hidden channels";
            return false;
        }
    return true;
}

}  // namespace

nmg_status repack_bf16(Ctx* c, int level, int weight_set) {
    if (!mfma_supported(c, nullptr)) return NMG_OK;
    const int NH = c->p.n_layers - 2;
    const size_t stride = packed_elems(NH);
    const int nsm = std::max(1, c->L - 1);
    if (!c->wbf) {
        const size_t total = stride * nsm * c->p.n_weight_sets;
        hipError_t e = hipMalloc((void**)&c->wbf, total * sizeof(uint16_t));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            c->wbf = nullptr;
            return fail(NMG_ERR_OOM, "hipMalloc failed for packed weights");
        }
        NMG_HIP(hipMemset(c->wbf, 0, total * sizeof(uint16_t)));
        c->wbf_stride = stride;
    }
    std::vector<float> w((size_t)c->wcount);
    const size_t off = ((size_t)level * c->p.n_weight_sets + weight_set) * c->wcount;
    NMG_HIP(hipMemcpy(w.data(), c->w32 + off, w.size() * sizeof(float), hipMemcpyDeviceToHost));
    std::vector<uint16_t> pk(stride, 0);
    // first layer [32][1][3][3]
    const float* w1 = w.data() + c->layer_off[0];
    for (int nb = 0; nb < 2; ++nb)
        for (int lane = 0; lane < 64; ++lane)
            for (int j = 0; j < 4; ++j) {
                const int co = nb * 16 + lane % 16, tap = 4 * (lane / 16) + j;
                pk[(size_t)(nb * 64 + lane) * 4 + j] = tap < 9 ? f2bf(w1[co * 9 + tap]) : 0;
            }
    for (int h = 0; h < NH; ++h) {
        const float* wh = w.data() + c->layer_off[1 + h];  // [32][32][3][3]
        for (int t = 0; t < 9; ++t)
            for (int nb = 0; nb < 2; ++nb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 8; ++j) {
                        const int co = nb * 16 + lane % 16, ci = 8 * (lane / 16) + j;
                        pk[kFirstElems + (size_t)h * kHiddenElems + (size_t)((t * 2 + nb) * 64 + lane) * 8 + j] =
                            f2bf(wh[(co * kC + ci) * 9 + t]);
                    }
    }
    const float* wl = w.data() + c->layer_off[(size_t)c->p.n_layers - 1];  // [1][32][3][3]
    for (int lane = 0; lane < 64; ++lane)
        for (int j = 0; j < 8; ++j) {
            const int t = lane % 16, ci = 8 * (lane / 16) + j;
            pk[kFirstElems + (size_t)NH * kHiddenElems + (size_t)lane * 8 + j] = t < 9 ? f2bf(wl[ci * 9 + t]) : 0;
        }
    const size_t dst = ((size_t)level * c->p.n_weight_sets + weight_set) * stride;
    NMG_HIP(hipMemcpy(c->wbf + dst, pk.data(), stride * sizeof(uint16_t), hipMemcpyHostToDevice));
    return NMG_OK;
}

nmg_status launch_mfma_smoother(const Ctx* c, int l, int batch, const int* ws, const float* b, const double* nrm2,
                                float* dst, int accumulate, Work<float>& w, hipStream_t s) {
    (void)w;
    std::string why;
    if (!mfma_supported(c, &why)) return fail(NMG_ERR_STATE, why);
    if (!c->wbf) return fail(NMG_ERR_STATE, "no weights loaded for the BF16 smoother");
    const int n = c->n[(size_t)l];
    const int tiles_x = (n + kT - 1) / kT;
    const int tiles = tiles_x * tiles_x;
    const int per_img = std::max(1, std::min(tiles, (2048 + batch - 1) / batch));
    dim3 grid((unsigned)per_img, (unsigned)batch);
    const uint16_t* wl = c->wbf + (size_t)l * c->p.n_weight_sets * c->wbf_stride;
    if (c->p.n_layers == 3) {
        hipLaunchKernelGGL(k_smoother_mfma<3>, grid, dim3(kThreads), Geo<3>::lds, s, b, nrm2, dst, accumulate, wl,
                           c->wbf_stride, ws, n, tiles_x, tiles);
    } else {
        hipLaunchKernelGGL(k_smoother_mfma<4>, grid, dim3(kThreads), Geo<4>::lds, s, b, nrm2, dst, accumulate, wl,
                           c->wbf_stride, ws, n, tiles_x, tiles);
    }
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

size_t mfma_lds_bytes(int n_layers) { return n_layers == 3 ? Geo<3>::lds : Geo<4>::lds; }

}  // namespace nmg
