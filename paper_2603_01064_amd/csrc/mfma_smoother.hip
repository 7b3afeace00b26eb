// Neural smoother h = ||b|| N(b/||b||) in BF16 on MFMA with FP32 accumulation
// (the smoothing line of Algorithm 4; N = Conv2d 1->32->...->32->1, 3x3,
// ReLU between layers, no bias, zero "same" padding).
//
// One workgroup produces a TW x TH output tile of one image and keeps every
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
#include <type_traits>
#include <vector>

#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kThreads = 256; // 4 waves
constexpr int kC = 32;        // hidden channels

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

inline uint16_t f2bf(float f) {
    // round to nearest even (inputs are finite)
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Activation buffers hold 32 BF16 channels per pixel (64 B) in four chunks of
// 8 channels; chunk g of pixel (row r, column c) sits at
//   (r * P + c) * 64 + ((g ^ ((c >> 1) & 3)) << 4),
// so any 8 consecutive pixels put a given chunk in 8 distinct 16-byte bank
// slots and a 16-lane operand read is conflict-free.  The pitch P is a
// multiple of 8, so the swizzle depends on the column only and every tap of
// a lane is its base address plus a constant.
constexpr int kP = 40;

__device__ inline int swz(int c, int g) { return (g ^ ((c >> 1) & 3)) << 4; }
__device__ inline int act_addr(int r, int c, int g) { return (r * kP + c) * 64 + swz(c, g); }

// Packed weight block (uint16 bf16) per (level, set):
//   first : [nb 2][lane 64][4]          co = nb*16 + lane%16, tap (dy, dx) = (lane/16, j), 0 if dy or dx is 3
//   hidden: [layer][tap 9][nb 2][lane 64][8]  co = nb*16 + lane%16, ci = 8*(lane/16)+j
//   last  : [lane 64][8]                t = lane%16 (0 if >= 9), ci = 8*(lane/16)+j
constexpr int kFirstElems = 2 * 64 * 4;
constexpr int kHiddenElems = 9 * 2 * 64 * 8;
constexpr int kLastElems = 64 * 8;

inline size_t packed_elems(int n_hidden) { return (size_t)kFirstElems + (size_t)n_hidden * kHiddenElems + kLastElems; }

// Tile geometry.  The output tile is TW x TH; layer i (1-based) is evaluated
// on the tile grown by NL - i pixels per side.  TW makes the hidden layers'
// output rows whole (or nearly whole) groups of 16 pixels, so one MFMA
// column group is 16 consecutive pixels of one row.
template <int NL>
struct Geo {
    static constexpr int TW = 32 - 2 * (NL - 2);  // 30 (3 layers), 28 (4 layers)
    static constexpr int TH = NL == 3 ? 12 : 10;
    static constexpr int W0 = TW + 2 * NL, H0 = TH + 2 * NL;
    static constexpr int W(int i) { return TW + 2 * (NL - i); }
    static constexpr int H(int i) { return TH + 2 * (NL - i); }
    // first-layer operand records: pixel (r, c) of the input tile holds the
    // BF16 values of columns c, c+1, c+2 (and a zero), one 8-byte record
    static constexpr int RW = W0 - 2;  // = W(1)
    static constexpr int NREC = H0 * RW;
    static constexpr int in_bytes = ((NREC * 8 + 255) / 256) * 256;
    static constexpr int bufA = H(1) * kP * 64;
    static constexpr int bufB = H(2) * kP * 64;
    static constexpr int lds = in_bytes + bufA + bufB;
    static constexpr int RPT = (NREC + 255) / 256;  // records per thread
};

typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Round four channels to BF16 (hardware RNE pack), then ReLU on the packed
// halves: a BF16 value is negative exactly when its 16-bit pattern is
// negative as a signed integer, so max(v, 0) per 16-bit lane is the ReLU
// (and rounding commutes with it: rounding never changes the sign).
typedef short short2v __attribute__((ext_vector_type(2)));
__device__ inline uint2 relu_pack4(floatx4 a) {
    const float2v lo = {a[0], a[1]};
    const float2v hi = {a[2], a[3]};
    const bf16x2 pl = __builtin_convertvector(lo, bf16x2);
    const bf16x2 ph = __builtin_convertvector(hi, bf16x2);
    short2v sl, sh;
    __builtin_memcpy(&sl, &pl, 4);
    __builtin_memcpy(&sh, &ph, 4);
    const short2v z = {0, 0};
    sl = __builtin_elementwise_max(sl, z);
    sh = __builtin_elementwise_max(sh, z);
    uint2 r;
    __builtin_memcpy(&r.x, &sl, 4);
    __builtin_memcpy(&r.y, &sh, 4);
    return r;
}

__device__ inline uint32_t pack2_bf16(float a, float b) {
    const float2v f = {a, b};
    const bf16x2 p = __builtin_convertvector(f, bf16x2);
    uint32_t u;
    __builtin_memcpy(&u, &p, 4);
    return u;
}

// LDS allows two workgroups (8 waves) per CU, so up to 256 VGPRs cost no occupancy.
template <int NL>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NL == 3 ? 1 : 2, 2))) k_smoother_mfma(const float* __restrict__ bres,
                                                            const double* __restrict__ nrm2, float* __restrict__ dst,
                                                            int accumulate, const uint16_t* __restrict__ wlevel,
                                                            size_t set_stride, const int* __restrict__ ws, int nsets,
                                                            int n, int tiles_x, int tiles_per_img) {
    constexpr int NH = NL - 2;
    using G = Geo<NL>;
    constexpr int TW = G::TW, TH = G::TH, RW = G::RW;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char* recs = smem;
    char* bufA = smem + G::in_bytes;
    char* bufB = bufA + G::bufA;

    const int img = blockIdx.y;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int ln = lane & 15;   // N index (pixel within group)
    const int lg = lane >> 4;   // K group / output row group

    // out-of-range set indices are clamped so that a bad index cannot read past the weights
    const int set = ws ? min(max(ws[img], 0), nsets - 1) : 0;
    const uint16_t* wp = wlevel + (size_t)set * set_stride;

    short4v w1[2];
    for (int nb = 0; nb < 2; ++nb) w1[nb] = *reinterpret_cast<const short4v*>(wp + (nb * 64 + lane) * 4);
    bf16x8 wh[NH][9][2];
    for (int h = 0; h < NH; ++h)
        for (int t = 0; t < 9; ++t)
            for (int nb = 0; nb < 2; ++nb)
                wh[h][t][nb] = *reinterpret_cast<const bf16x8*>(wp + kFirstElems + (size_t)h * kHiddenElems +
                                                                ((t * 2 + nb) * 64 + lane) * 8);
    const bf16x8 wl = *reinterpret_cast<const bf16x8*>(wp + kFirstElems + (size_t)NH * kHiddenElems + lane * 8);

    // per-lane constants for 16-aligned pixel groups (column = 16 k + ln): the
    // operand chunk offsets of pixels ln, ln+1, ln+2 and the output chunk
    // offsets of channels nb*16 + 4*lg .. +3
    const int swz0 = swz(ln, lg), swz1 = swz(ln + 1, lg), swz2 = swz(ln + 2, lg);
    int out_off[2];
    for (int nb = 0; nb < 2; ++nb) {
        const int co = nb * 16 + lg * 4;
        out_off[nb] = swz(ln, co >> 3) + (co & 7) * 2;
    }

    const size_t per = (size_t)n * n;
    const float* src = bres + (size_t)img * per;
    float* out = dst + (size_t)img * per;
    const double nb2 = nrm2[img];
    const float nbf = (float)sqrt(nb2);
    const float inv = nb2 > 0.0 ? (float)(1.0 / sqrt(nb2)) : 0.f;

    // input values of this thread's first-layer records (three per record),
    // loaded one tile ahead so the global latency overlaps the layers
    float pv[G::RPT][3];
    auto load_records = [&](int tile) {
        const int ty0 = (tile / tiles_x) * TH, tx0 = (tile % tiles_x) * TW;
#pragma unroll
        for (int k = 0; k < G::RPT; ++k) {
            const int e = tid + k * kThreads;
            const int r = e / RW, c = e - (e / RW) * RW;
            const int gy = ty0 - NL + r, gx = tx0 - NL + c;
            const bool row_ok = e < G::NREC && gy >= 0 && gy < n;
            const float* rp = src + (size_t)(row_ok ? gy : 0) * n;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                pv[k][d] = (tile < tiles_per_img && row_ok && gx + d >= 0 && gx + d < n) ? rp[gx + d] : 0.f;
        }
    };
    load_records(blockIdx.x);

    for (int tile = blockIdx.x; tile < tiles_per_img; tile += gridDim.x) {
        const int ty0 = (tile / tiles_x) * TH, tx0 = (tile % tiles_x) * TW;
        // ---- records of this tile (scaled by 1/||b||, zero outside the image)
#pragma unroll
        for (int k = 0; k < G::RPT; ++k) {
            const int e = tid + k * kThreads;
            if (e < G::NREC)
                *reinterpret_cast<uint2*>(recs + e * 8) =
                    make_uint2(pack2_bf16(pv[k][0] * inv, pv[k][1] * inv), pack2_bf16(pv[k][2] * inv, 0.f));
        }
        load_records(tile + gridDim.x);
        __syncthreads();
        // tiles whose input region lies inside the image need no zero masking
        const bool interior = ty0 >= NL && tx0 >= NL && ty0 + TH + NL <= n && tx0 + TW + NL <= n;
        auto layers = [&](auto edge_tag) {
            constexpr bool EDGE = decltype(edge_tag)::value;
            // ---- first layer 1 -> 32 on region W(1) x H(1) (flattened groups of 16);
            //      operand K slot (lane/16, j) is tap (dy, dx) = (lane/16, j)
            {
                constexpr int S = G::W(1), HH = G::H(1), HALO = NL - 1;
                constexpr int npx = S * HH, ngr = (npx + 15) / 16;
                constexpr int GPW = (ngr + 3) / 4;  // groups per wave
                // all of a wave's groups are independent: operands first, then the
                // MFMAs, then the stores, fully unrolled so their latencies overlap
                short4v bop[GPW];
                int pry[GPW], prx[GPW];
#pragma unroll
                for (int k = 0; k < GPW; ++k) {
                    const int q = (wave + 4 * k) * 16 + ln;
                    const bool live = q < npx;
                    const int qc = live ? q : npx - 1;
                    pry[k] = live ? q / S : -1;
                    prx[k] = qc - (qc / S) * S;
                    const int ryc = qc / S;
                    bop[k] = short4v{0, 0, 0, 0};
                    if (lg < 3 && wave + 4 * k < ngr)
                        bop[k] = *reinterpret_cast<const short4v*>(recs + ((ryc + lg) * RW + prx[k]) * 8);
                }
#pragma unroll
                for (int k = 0; k < GPW; ++k) {
                    if (wave + 4 * k >= ngr) break;
                    floatx4 acc[2];
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) {
                        acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[nb], bop[k], acc[nb], 0, 0, 0);
                    }
                    if (pry[k] >= 0) {
                        const int ry = pry[k], rx = prx[k];
                        bool inside = true;
                        if constexpr (EDGE) {
                            const int gy = ty0 - HALO + ry, gx = tx0 - HALO + rx;
                            inside = gy >= 0 && gy < n && gx >= 0 && gx < n;
                        }
#pragma unroll
                        for (int nb = 0; nb < 2; ++nb) {
                            const int co = nb * 16 + lg * 4;
                            const uint2 v = inside ? relu_pack4(acc[nb]) : make_uint2(0u, 0u);
                            *reinterpret_cast<uint2*>(bufA + act_addr(ry, rx, co >> 3) + (co & 7) * 2) = v;
                        }
                    }
                }
            }
            __syncthreads();
            // ---- hidden layers 32 -> 32: groups are 16 consecutive pixels of a row
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int layer = 2 + h;
                const int S = TW + 2 * (NL - layer), HH = TH + 2 * (NL - layer), HALO = NL - layer;
                const int ngr = HH * 2;  // S <= 32: two groups per row
                const char* ain = (h & 1) ? bufB : bufA;
                char* aout = (h & 1) ? bufA : bufB;
                constexpr int GPWH = (2 * G::H(2) + 3) / 4;  // groups per wave, largest hidden region
#pragma unroll
                for (int k = 0; k < GPWH; ++k) {
                    const int gi = wave + 4 * k;
                    if (gi >= ngr) break;
                    const int ry = gi >> 1, rx0 = (gi & 1) * 16;
                    const int rx = rx0 + ln;
                    // taps dx = 1, 2 read pixels rx+1, rx+2, whose swizzle uses (ln+dx) & 3
                    const char* a0 = ain + (ry * kP + rx) * 64 + swz0;
                    const char* a1 = ain + (ry * kP + rx + 1) * 64 + swz1;
                    const char* a2 = ain + (ry * kP + rx + 2) * 64 + swz2;
                    floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy) {
                        const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(a0 + dy * kP * 64);
                        const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(a1 + dy * kP * 64);
                        const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(a2 + dy * kP * 64);
                        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[h][dy * 3][0], b0, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[h][dy * 3][1], b0, acc1, 0, 0, 0);
                        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[h][dy * 3 + 1][0], b1, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[h][dy * 3 + 1][1], b1, acc1, 0, 0, 0);
                        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[h][dy * 3 + 2][0], b2, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[h][dy * 3 + 2][1], b2, acc1, 0, 0, 0);
                    }
                    if (rx < S) {
                        bool inside = true;
                        if constexpr (EDGE) {
                            const int gy = ty0 - HALO + ry, gx = tx0 - HALO + rx;
                            inside = gy >= 0 && gy < n && gx >= 0 && gx < n;
                        }
                        char* o = aout + (ry * kP + rx) * 64;
                        *reinterpret_cast<uint2*>(o + out_off[0]) = inside ? relu_pack4(acc0) : make_uint2(0u, 0u);
                        *reinterpret_cast<uint2*>(o + out_off[1]) = inside ? relu_pack4(acc1) : make_uint2(0u, 0u);
                    }
                }
                __syncthreads();
            }
            // ---- last layer 32 -> 1: Z[t][p] on region W(NL-1) x H(NL-1) (tap planes,
            //      so both the stores and the 9-tap gather are unit-stride), then gather
            {
                constexpr int S = G::W(NL - 1), HH = G::H(NL - 1);
                constexpr int ngr = HH * 2;
                constexpr int ZP = 32;          // Z pixel pitch
                constexpr int ZN = HH * ZP;     // pixels per tap plane
                const char* ain = (NH & 1) ? bufB : bufA;
                float* Z = reinterpret_cast<float*>((NH & 1) ? bufA : bufB);
                constexpr int GPW = (ngr + 3) / 4;
                bf16x8 bl[GPW];
#pragma unroll
                for (int k = 0; k < GPW; ++k) {
                    const int gi = wave + 4 * k;
                    const int ry = gi >> 1, rx = (gi & 1) * 16 + ln;
                    if (gi < ngr) bl[k] = *reinterpret_cast<const bf16x8*>(ain + (ry * kP + rx) * 64 + swz0);
                }
#pragma unroll
                for (int k = 0; k < GPW; ++k) {
                    const int gi = wave + 4 * k;
                    if (gi >= ngr) break;
                    const int ry = gi >> 1, rx = (gi & 1) * 16 + ln;
                    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, bl[k], acc, 0, 0, 0);
                    if (rx < S && lg < 3) {
                        // lane group lg holds taps 4 lg .. 4 lg + 3; only taps 0..8 exist
                        float* zp = Z + (lg * 4) * ZN + ry * ZP + rx;
                        zp[0] = acc[0];
                        if (lg < 2) {
                            zp[ZN] = acc[1];
                            zp[2 * ZN] = acc[2];
                            zp[3 * ZN] = acc[3];
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < (TH * TW + kThreads - 1) / kThreads; ++k) {
                    const int e = tid + k * kThreads;
                    if (e >= TH * TW) break;
                    const int oy = e / TW, ox = e - (e / TW) * TW;
                    const int gy = ty0 + oy, gx = tx0 + ox;
                    if (!EDGE || (gy < n && gx < n)) {
                        const float* zb = Z + oy * ZP + ox;
                        float v = 0.f;
#pragma unroll
                        for (int t = 0; t < 9; ++t) v += zb[t * ZN + (t / 3) * ZP + t % 3];
                        v *= nbf;
                        float* o = out + (size_t)gy * n + gx;
                        *o = accumulate ? *o + v : v;
                    }
                }
            }
        };
        if (interior)
            layers(std::false_type{});
        else
            layers(std::true_type{});
        __syncthreads();
    }
}

bool mfma_supported(const Ctx* c, std::string* why) {
    const nmg_problem& p = c->p;
    if (p.smoother_arch != NMG_ARCH_CNN) {
        if (why) *why = "BF16 MFMA smoother implements the CNN";
        return false;
    }
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
                const int co = nb * 16 + lane % 16, dy = lane / 16, dx = j;
                pk[(size_t)(nb * 64 + lane) * 4 + j] = (dy < 3 && dx < 3) ? f2bf(w1[co * 9 + dy * 3 + dx]) : 0;
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
    const uint16_t* wl = c->wbf + (size_t)l * c->p.n_weight_sets * c->wbf_stride;
    if (c->p.n_layers == 3) {
        using G = Geo<3>;
        const int tiles_x = (n + G::TW - 1) / G::TW, tiles = tiles_x * ((n + G::TH - 1) / G::TH);
        const int per_img = std::max(1, std::min(tiles, (1024 + batch - 1) / batch));
        hipLaunchKernelGGL((k_smoother_mfma<3>), dim3((unsigned)per_img, (unsigned)batch), dim3(kThreads), G::lds, s, b,
                           nrm2, dst, accumulate, wl, c->wbf_stride, ws, c->p.n_weight_sets, n, tiles_x, tiles);
    } else {
        using G = Geo<4>;
        const int tiles_x = (n + G::TW - 1) / G::TW, tiles = tiles_x * ((n + G::TH - 1) / G::TH);
        const int per_img = std::max(1, std::min(tiles, (1024 + batch - 1) / batch));
        hipLaunchKernelGGL((k_smoother_mfma<4>), dim3((unsigned)per_img, (unsigned)batch), dim3(kThreads), G::lds, s, b,
                           nrm2, dst, accumulate, wl, c->wbf_stride, ws, c->p.n_weight_sets, n, tiles_x, tiles);
    }
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

size_t mfma_lds_bytes(int n_layers) { return n_layers == 3 ? Geo<3>::lds : Geo<4>::lds; }

}  // namespace nmg
