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
//   last layer    32 -> 1 : Z[p][t] = sum_c act[p][c] w[c][t] with t as M, taken
//                           in the epilogue of the last hidden layer with its
//                           accumulators as the operand (no LDS round trip),
//                           then out[p] = sum_t Z[p + off(t)][t]
// Weights are packed once per weight set into the per-lane operand order and
// kept in registers while a workgroup walks the tiles of its image (with two
// hidden layers, the weights of one hidden layer at a time).
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
// 8 channels, chunk g holding channels 4g .. 4g + 3 and 16 + 4g .. 16 + 4g + 3
// (what lane group g of a 16x16 MFMA tile over the 32 channels holds, so a
// lane writes its chunk with one 16-byte store); chunk g of pixel (row r,
// column c) sits at
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
//   hidden: [layer][tap 9][nb 2][lane 64][8]  co = nb*16 + lane%16, ci = 4*(lane/16)+j (j < 4),
//                                       16+4*(lane/16)+j-4 (j >= 4): the accumulator order
//   last  : [lane 64][8]                t = lane%16 (0 if >= 9), ci = 4*(lane/16)+j (j < 4),
//                                       16+4*(lane/16)+j-4 (j >= 4): the accumulator order
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
    // output rows per register block in the hidden layers (accumulators: 8 RB VGPRs)
    static constexpr int RB = NL == 3 ? 7 : 2;
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
                                                            const double* __restrict__ nrm2, int nparts, float* __restrict__ dst,
                                                            int accumulate, const uint16_t* __restrict__ wlevel,
                                                            size_t set_stride, const int* __restrict__ ws, int nsets,
                                                            int n, int tiles_x, int tiles_per_img,
                                                            uint16_t* __restrict__ dstb, int bpitch, int btiled) {
    constexpr int NH = NL - 2;
    using G = Geo<NL>;
    constexpr int TW = G::TW, TH = G::TH, RW = G::RW;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char* recs = smem;
    char* bufA = smem + G::in_bytes;
    char* bufB = bufA + G::bufA;

    // XCD-aware assignment: workgroups are dispatched round-robin over the 8
    // XCDs by linear id, so the (image, workgroup-in-image) pairs are numbered
    // XCD-major (XCD x takes the contiguous range of its G/8 or G/8 + 1
    // workgroups); the workgroups of one image then run on one XCD, or two,
    // and share its L2 (tile halos, and output cache lines split between
    // neighbouring tiles)
    int img, wgi;
    {
        const int G = gridDim.x * gridDim.y, i = blockIdx.x + blockIdx.y * gridDim.x;
        const int x = i % 8, q = G / 8, rem = G % 8;
        const int p = x * q + min(x, rem) + i / 8;
        img = p / gridDim.x;
        wgi = p - img * gridDim.x;
    }
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: kept in an SGPR
    const int ln = lane & 15;   // N index (pixel within group)
    const int lg = lane >> 4;   // K group / output row group

    // out-of-range set indices are clamped so that a bad index cannot read past the weights
    const int set = ws ? min(max(ws[img], 0), nsets - 1) : 0;
    const uint16_t* wp = wlevel + (size_t)set * set_stride;

    // weights through a buffer resource over this set's block: one VGPR
    // offset (the lane's) and a uniform byte offset per load, so no per-lane
    // 64-bit address is kept per weight operand
    const __amdgpu_buffer_rsrc_t wres =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(wp), (short)0, (int)(set_stride * 2), 0x00020000);
    auto wload = [&](int lane_bytes, int elem_off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(wres, lane_bytes, elem_off * 2, 0);
        bf16x8 o;
        __builtin_memcpy(&o, &v, 16);
        return o;
    };
    short4v w1[2];
    for (int nb = 0; nb < 2; ++nb) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(wres, lane * 8, nb * 64 * 4 * 2, 0);
        __builtin_memcpy(&w1[nb], &v, 8);
    }
    // hidden-layer weights: with one hidden layer they stay in registers for
    // the whole kernel; with two, only the layer being evaluated is held (72
    // VGPRs) and the next one is reloaded from the cache, which keeps the
    // kernel within 256 VGPRs
    constexpr bool kResident = NH == 1;
    bf16x8 wh[kResident ? NH : 1][9][2];
    auto load_hidden = [&](int slot, int h) {
        // the opaque copy of the layer offset keeps a per-tile reload inside
        // the tile loop (hoisted, both layers would be held again)
        int base = kFirstElems + h * kHiddenElems;
        if constexpr (!kResident) asm volatile("" : "+s"(base));
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) wh[slot][t][nb] = wload(lane * 16, base + (t * 2 + nb) * 64 * 8);
    };
    if constexpr (kResident)
        for (int h = 0; h < NH; ++h) load_hidden(h, h);
    const bf16x8 wl = wload(lane * 16, kFirstElems + NH * kHiddenElems);
    // per-lane constants for 16-aligned pixel groups (column = 16 k + ln): the
    // operand chunk offsets of pixels ln, ln+1, ln+2; the output chunk of a
    // lane is its operand chunk of pixel ln (chunk lg)
    const int swz0 = swz(ln, lg), swz1 = swz(ln + 1, lg), swz2 = swz(ln + 2, lg);
    // first-layer record offsets of this lane (tap row dy = min(lane/16, 2)):
    // row groups read pixel ln of a row, column groups row ln of a column
    const int rec_row = (min(lg, 2) * G::RW + ln) * 8;
    const int rec_col = ((ln + min(lg, 2)) * G::RW) * 8;
    // first-layer row group k of this wave is group wave + 4 k: row (wave >> 1) + 2 k,
    // pixels (wave & 1) * 16 + ln, so its operand and output addresses are these
    // per-lane bases plus a multiple of k that fits an LDS immediate offset
    const int rec_wave = rec_row + ((wave >> 1) * G::RW + (wave & 1) * 16) * 8;
    const int st_wave = ((wave >> 1) * kP + (wave & 1) * 16 + ln) * 64 + swz0;

    const size_t per = (size_t)n * n;
    const float* src = bres + (size_t)img * per;
    float* out = dst + (size_t)img * per;
    // input values of this thread's first-layer records (three per record),
    // loaded one tile ahead so the global latency overlaps the layers.  The
    // image is read through a buffer resource: a load whose offset lies past
    // the image returns zero, so a tap outside the image takes an out-of-range
    // offset instead of a branch (the launch keeps n*n*4 below 2^31).
    const __amdgpu_buffer_rsrc_t sres =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(src), (short)0, (int)(per * 4), 0x00020000);
    float pv[G::RPT][3];
    auto load_records = [&](int tile, int t_id) {
        const int ty0 = (tile / tiles_x) * TH, tx0 = (tile % tiles_x) * TW;
#pragma unroll
        for (int k = 0; k < G::RPT; ++k) {
            const int e = t_id + k * kThreads;
            const int r = e / RW, c = e - (e / RW) * RW;
            const int gy = ty0 - NL + r, gx = tx0 - NL + c;
            // (bitwise tests: no short-circuit branches)
            const bool row_ok = (tile < tiles_per_img) & (e < G::NREC) & ((unsigned)gy < (unsigned)n);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const bool ok = row_ok & ((unsigned)(gx + d) < (unsigned)n);
                const int off = ok ? (gy * n + gx + d) * 4 : (int)0x80000000;
                pv[k][d] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sres, off, 0, 0));
            }
        }
    };
    // (issued before the norm's loads below, so the two latencies overlap)
    load_records(wgi, tid);

    // ||b||^2: given, or the sum of this image's partial sums in their order
    double nb2;
    if (nparts > 0) {
        nb2 = 0.0;
        // (unrolled: sixteen partials are loaded together; the sum keeps its order)
#pragma unroll 16
        for (int i = 0; i < nparts; ++i) nb2 += nrm2[(size_t)img * nparts + i];
    } else {
        nb2 = nrm2[img];
    }
    const float nbf = (float)sqrt(nb2);
    const float inv = nb2 > 0.0 ? (float)(1.0 / sqrt(nb2)) : 0.f;

    for (int tile = wgi; tile < tiles_per_img; tile += gridDim.x) {
        // per-tile copies of the lane indices: the per-lane index arithmetic of
        // the first and last layers is redone every tile instead of being kept
        // live (or spilled) across the loop
        int tid_t = tid;
        asm volatile("" : "+v"(tid_t));
        const int ln_t = tid_t & 15, lg_t = (tid_t >> 4) & 3;
        const int ty0 = (tile / tiles_x) * TH, tx0 = (tile % tiles_x) * TW;
        // ---- records of this tile (scaled by 1/||b||, zero outside the image)
#pragma unroll
        for (int k = 0; k < G::RPT; ++k) {
            const int e = tid_t + k * kThreads;
            if (e < G::NREC)
                *reinterpret_cast<uint2*>(recs + e * 8) =
                    make_uint2(pack2_bf16(pv[k][0] * inv, pv[k][1] * inv), pack2_bf16(pv[k][2] * inv, 0.f));
        }
        load_records(tile + gridDim.x, tid_t);
        __syncthreads();
        // tiles whose input region lies inside the image need no zero masking
        const bool interior = ty0 >= NL && tx0 >= NL && ty0 + TH + NL <= n && tx0 + TW + NL <= n;
        if constexpr (!kResident) load_hidden(0, 0);
        auto layers = [&](auto edge_tag) {
            constexpr bool EDGE = decltype(edge_tag)::value;
            // ---- first layer 1 -> 32 on region W(1) x H(1) = 34 x 16.  Groups
            //      0 .. 2 H(1) - 1 are the two 16-pixel halves of a row; the last
            //      W(1) - 32 groups are columns 32, 33 (16 rows each), so every
            //      address is a uniform part plus a per-lane constant.  Operand K
            //      slot (lane/16, j) is tap (dy, dx) = (lane/16, j); the slots of
            //      lane group 3 have zero weights and read a (finite) record of
            //      row dy = 2 instead.
            {
                constexpr int S = G::W(1), HH = G::H(1), HALO = NL - 1;
                static_assert(HH == 16 && S > 32 && S <= 48, "first-layer group layout");
                constexpr int NROWG = 2 * HH, ngr = NROWG + (S - 32);
                static_assert(NROWG % 4 == 0, "row groups fill whole rounds of the four waves");
                constexpr int GPW = (ngr + 3) / 4;  // groups per wave
                auto operand = [&](int k) {
                    const int gi = wave + 4 * k;
                    short4v v = short4v{0, 0, 0, 0};
                    if (4 * k < NROWG)  // row group: row gi / 2, pixels (gi & 1) * 16 + ln
                        v = *reinterpret_cast<const short4v*>(recs + rec_wave + k * (2 * RW * 8));
                    else if (gi < ngr)  // column group: column 32 + gi - NROWG, rows ln
                        v = *reinterpret_cast<const short4v*>(recs + (32 + gi - NROWG) * 8 + rec_col);
                    return v;
                };
                auto compute_store = [&](int k, short4v bop) {
                    const int gi = wave + 4 * k;
                    floatx4 acc[2];
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) {
                        acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[nb], bop, acc[nb], 0, 0, 0);
                    }
                    const bool rowg = 4 * k < NROWG;
                    const int ry = rowg ? gi >> 1 : ln_t;
                    const int rx = rowg ? (gi & 1) * 16 + ln_t : 32 + gi - NROWG;
                    bool inside = true;
                    if constexpr (EDGE) {
                        const int gy = ty0 - HALO + ry, gx = tx0 - HALO + rx;
                        inside = gy >= 0 && gy < n && gx >= 0 && gx < n;
                    }
                    // the lane's eight channels (4 lg .. 4 lg + 3, 16 + 4 lg .. 16 + 4 lg + 3)
                    // are chunk lg of the pixel in the order the hidden weights are
                    // packed: one 16-byte store (row groups start at a multiple of 16
                    // pixels, so the swizzle is the lane's)
                    char* o = rowg ? bufA + st_wave + k * (2 * kP * 64) : bufA + (ry * kP + rx) * 64 + swz(rx, lg_t);
                    const uint2 p0 = inside ? relu_pack4(acc[0]) : make_uint2(0u, 0u);
                    const uint2 p1 = inside ? relu_pack4(acc[1]) : make_uint2(0u, 0u);
                    *reinterpret_cast<uint4*>(o) = make_uint4(p0.x, p0.y, p1.x, p1.y);
                };
                if constexpr (NL == 3) {
                    // all of a wave's groups are independent: operands first, then the
                    // MFMAs, then the stores, fully unrolled so their latencies overlap
                    short4v bop[GPW];
#pragma unroll
                    for (int k = 0; k < GPW; ++k) bop[k] = operand(k);
#pragma unroll
                    for (int k = 0; k < GPW; ++k) {
                        if (4 * k >= NROWG && wave + 4 * k >= ngr) break;
                        compute_store(k, bop[k]);
                    }
                } else {
                    // fewer registers: one group's operand in flight ahead of the MFMAs
                    short4v cur = operand(0);
#pragma unroll
                    for (int k = 0; k < GPW; ++k) {
                        if (4 * k >= NROWG && wave + 4 * k >= ngr) break;
                        const short4v nxt = k + 1 < GPW ? operand(k + 1) : cur;
                        compute_store(k, cur);
                        cur = nxt;
                    }
                }
            }
            __syncthreads();
            // ---- hidden layers 32 -> 32.  Wave w computes the 16 pixels of column
            //      half (w & 1) in the output rows [(w >> 1) R, (w >> 1) R + R),
            //      R = HH / 2, in blocks of at most RB rows: it reads each input row
            //      of a block once (taps dx = 0, 1, 2 as three shifted operands) and
            //      applies it to the up to three output rows that use it, so one
            //      LDS operand read feeds up to six MFMAs.
            auto hidden = [&](auto hc) {
                constexpr int H = decltype(hc)::value;
                constexpr int layer = 2 + H;
                constexpr int S = G::W(layer), HH = G::H(layer), HALO = NL - layer;
                constexpr int R = HH / 2;
                static_assert(HH % 2 == 0 && S <= 32 && R <= 4 * G::RB, "hidden-layer wave split");
                const char* ain = (H & 1) ? bufB : bufA;
                char* aout = (H & 1) ? bufA : bufB;
                // the last hidden layer feeds the last layer from registers; its
                // Z planes take the buffer this layer does not read
                constexpr bool LAST = H == NH - 1;
                constexpr int ZP = 32, ZN = HH * ZP;  // Z pixel pitch, pixels per tap plane
                float* Z = reinterpret_cast<float*>(aout);
                const int rx = (wave & 1) * 16 + ln;
                const int rbase = (wave >> 1) * R;
                // taps dx = 1, 2 read pixels rx+1, rx+2, whose swizzle uses (ln+dx) & 3
                const char* a0 = ain + rx * 64 + swz0;
                const char* a1 = ain + (rx + 1) * 64 + swz1;
                const char* a2 = ain + (rx + 2) * 64 + swz2;
                auto block = [&](auto nc, int r0) {
                    constexpr int RBk = decltype(nc)::value;
                    floatx4 acc[RBk][2];
#pragma unroll
                    for (int r = 0; r < RBk; ++r)
                        for (int nb = 0; nb < 2; ++nb) acc[r][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
                    // input rows are software-pipelined one ahead; the scheduling
                    // barriers keep the compiler from hoisting every row's reads
                    // to the top (which would hold all of them in registers)
                    auto read_row = [&](int i, bf16x8* bx) {
                        const int off = (r0 + i) * kP * 64;
                        bx[0] = *reinterpret_cast<const bf16x8*>(a0 + off);
                        bx[1] = *reinterpret_cast<const bf16x8*>(a1 + off);
                        bx[2] = *reinterpret_cast<const bf16x8*>(a2 + off);
                    };
                    bf16x8 bnext[3];
                    read_row(0, bnext);
#pragma unroll
                    for (int i = 0; i < RBk + 2; ++i) {
                        bf16x8 bx[3] = {bnext[0], bnext[1], bnext[2]};
                        if (i + 1 < RBk + 2) read_row(i + 1, bnext);
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                            for (int dy = 0; dy < 3; ++dy) {
                                const int r = i - dy;  // output row of this block fed by tap (dy, dx)
                                if (r < 0 || r >= RBk) continue;
#pragma unroll
                                for (int nb = 0; nb < 2; ++nb)
                                    acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[kResident ? H : 0][dy * 3 + dx][nb], bx[dx],
                                                                                         acc[r][nb], 0, 0, 0);
                            }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if constexpr (LAST) {
                        // last layer 32 -> 1 straight from the accumulators: lane (ln, lg)
                        // holds channels 4 lg .. 4 lg + 3 and 16 + 4 lg .. 16 + 4 lg + 3 of
                        // pixel ln, which are K slots 8 lg .. 8 lg + 7 of the last-layer
                        // weights as packed.  Z[t][p] = sum_c act[p][c] w[c][t] (taps
                        // t = 4 lg + i) goes to tap planes, so these stores and the 9-tap
                        // gather are unit-stride.
#pragma unroll
                        for (int r = 0; r < RBk; ++r) {
                            const int ry = r0 + r;
                            bool inside = true;
                            if constexpr (EDGE) {
                                const int gy = ty0 - HALO + ry, gx = tx0 - HALO + rx;
                                inside = gy >= 0 && gy < n && gx >= 0 && gx < n;
                            }
                            const uint2 p0 = inside ? relu_pack4(acc[r][0]) : make_uint2(0u, 0u);
                            const uint2 p1 = inside ? relu_pack4(acc[r][1]) : make_uint2(0u, 0u);
                            const uint4 pk = make_uint4(p0.x, p0.y, p1.x, p1.y);
                            bf16x8 bl;
                            __builtin_memcpy(&bl, &pk, 16);
                            floatx4 z = {0.f, 0.f, 0.f, 0.f};
                            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, bl, z, 0, 0, 0);
                            if (rx < S && lg_t < 3) {
                                // only taps 0..8 exist
                                float* zp = Z + (lg_t * 4) * ZN + ry * ZP + rx;
                                zp[0] = z[0];
                                if (lg_t < 2) {
                                    zp[ZN] = z[1];
                                    zp[2 * ZN] = z[2];
                                    zp[3 * ZN] = z[3];
                                }
                            }
                        }
                    } else if (rx < S) {
#pragma unroll
                        for (int r = 0; r < RBk; ++r) {
                            const int ry = r0 + r;
                            bool inside = true;
                            if constexpr (EDGE) {
                                const int gy = ty0 - HALO + ry, gx = tx0 - HALO + rx;
                                inside = gy >= 0 && gy < n && gx >= 0 && gx < n;
                            }
                            const uint2 p0 = inside ? relu_pack4(acc[r][0]) : make_uint2(0u, 0u);
                            const uint2 p1 = inside ? relu_pack4(acc[r][1]) : make_uint2(0u, 0u);
                            *reinterpret_cast<uint4*>(aout + (ry * kP + rx) * 64 + swz0) =
                                make_uint4(p0.x, p0.y, p1.x, p1.y);
                        }
                    }
                };
                constexpr int RB = G::RB, NBLK = (R + RB - 1) / RB;
                block(std::integral_constant<int, (R < RB ? R : RB)>{}, rbase);
                if constexpr (NBLK > 1) block(std::integral_constant<int, (R - RB < RB ? R - RB : RB)>{}, rbase + RB);
                if constexpr (NBLK > 2)
                    block(std::integral_constant<int, (R - 2 * RB < RB ? R - 2 * RB : RB)>{}, rbase + 2 * RB);
                if constexpr (NBLK > 3) block(std::integral_constant<int, R - 3 * RB>{}, rbase + 3 * RB);
                if constexpr (!kResident && H + 1 < NH) load_hidden(0, H + 1);
                __syncthreads();
            };
            hidden(std::integral_constant<int, 0>{});
            if constexpr (NH > 1) hidden(std::integral_constant<int, 1>{});
            // ---- out[p] = ||b|| sum_t Z[t][p + off(t)] (the Z planes were written by
            //      the last hidden layer, before its barrier)
            {
                constexpr int HH = G::H(NL - 1);
                constexpr int ZP = 32, ZN = HH * ZP;
                const float* Z = reinterpret_cast<const float*>((NH & 1) ? bufB : bufA);
#pragma unroll
                for (int k = 0; k < (TH * TW + kThreads - 1) / kThreads; ++k) {
                    const int e = tid_t + k * kThreads;
                    if (e >= TH * TW) break;
                    const int oy = e / TW, ox = e - (e / TW) * TW;
                    const int gy = ty0 + oy, gx = tx0 + ox;
                    const bool in_img = !EDGE || (gy < n && gx < n);
                    float v = 0.f;
                    if (in_img) {
                        const float* zb = Z + oy * ZP + ox;
#pragma unroll
                        for (int t = 0; t < 9; ++t) v += zb[t * ZN + (t / 3) * ZP + t % 3];
                        v *= nbf;
                    }
                    if (bpitch > 0) {
                        // zero-padded BF16 plane for the MFMA filter F' (the tiles
                        // cover the padding too; the host checks it), row-major or
                        // in the filter's fragment-tiled layout: 1 KB tiles of
                        // 16 rows x 32 columns, lane (row & 15) + 16 ((col & 31) >> 3)
                        if (gy < bpitch && gx < bpitch) {
                            const size_t o = btiled ? ((size_t)((gy >> 4) * (bpitch >> 5) + (gx >> 5)) << 9) +
                                                          (size_t)(((gy & 15) + 16 * ((gx & 31) >> 3)) * 8 + (gx & 7))
                                                    : (size_t)gy * bpitch + gx;
                            dstb[(size_t)img * bpitch * bpitch + o] = (uint16_t)pack2_bf16(v, 0.f);
                        }
                    } else if (in_img) {
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
        // no barrier here: the next tile writes the records (read only by this
        // tile's first layer, behind its barrier) and then waits at its own
        // first barrier, which every wave reaches only after this gather
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
    // hidden layers: K slot (lane/16, j) is the input channel that the previous
    // layer's accumulators hold there, 4 (lane/16) + j, then 16 + 4 (lane/16) + j - 4
    // (each layer stores them as one 16-byte chunk per pixel)
    for (int h = 0; h < NH; ++h) {
        const float* wh = w.data() + c->layer_off[1 + h];  // [32][32][3][3]
        for (int t = 0; t < 9; ++t)
            for (int nb = 0; nb < 2; ++nb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 8; ++j) {
                        const int g = lane / 16;
                        const int co = nb * 16 + lane % 16, ci = j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
                        pk[kFirstElems + (size_t)h * kHiddenElems + (size_t)((t * 2 + nb) * 64 + lane) * 8 + j] =
                            f2bf(wh[(co * kC + ci) * 9 + t]);
                    }
    }
    const float* wl = w.data() + c->layer_off[(size_t)c->p.n_layers - 1];  // [1][32][3][3]
    // K slot (lane/16, j) of the last layer is the channel that the hidden
    // layer's accumulators put there: 4 (lane/16) + j, then 16 + 4 (lane/16) + j - 4
    for (int lane = 0; lane < 64; ++lane)
        for (int j = 0; j < 8; ++j) {
            const int t = lane % 16, g = lane / 16, ci = j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
            pk[kFirstElems + (size_t)NH * kHiddenElems + (size_t)lane * 8 + j] = t < 9 ? f2bf(wl[ci * 9 + t]) : 0;
        }
    const size_t dst = ((size_t)level * c->p.n_weight_sets + weight_set) * stride;
    NMG_HIP(hipMemcpy(c->wbf + dst, pk.data(), stride * sizeof(uint16_t), hipMemcpyHostToDevice));
    return NMG_OK;
}

nmg_status launch_mfma_smoother(const Ctx* c, int l, int batch, const int* ws, const float* b, const double* nrm2,
                                int nparts, float* dst, int accumulate, Work<float>& w, hipStream_t s, uint16_t* dstb,
                                int bpitch, bool btiled) {
    (void)w;
    std::string why;
    if (!mfma_supported(c, &why)) return fail(NMG_ERR_STATE, why);
    if (!c->wbf) return fail(NMG_ERR_STATE, "no weights loaded for the BF16 smoother");
    const int n = c->n[(size_t)l];
    if ((size_t)n * n * sizeof(float) >= ((size_t)1 << 31))
        return fail(NMG_ERR_SHAPE, "BF16 smoother: one image of this level exceeds 2 GiB");
    if (dstb && !mfma_smoother_covers(c, l, bpitch))
        return fail(NMG_ERR_SHAPE, "BF16 smoother: its tiles do not cover the padded output plane");
    if (!dstb) bpitch = 0;
    const uint16_t* wl = c->wbf + (size_t)l * c->p.n_weight_sets * c->wbf_stride;
    // one resident round of workgroups (two per CU) over the batch: the
    // workgroups have equal work, so a second, partial round would leave
    // most CUs idle at its end
    int dev = 0, cus = 0;
    NMG_HIP(hipGetDevice(&dev));
    NMG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    auto grid_x = [&](int tiles) { return std::max(1, std::min(tiles, std::max(1, 2 * cus) / batch)); };
    if (c->p.n_layers == 3) {
        using G = Geo<3>;
        const int tiles_x = (n + G::TW - 1) / G::TW, tiles = tiles_x * ((n + G::TH - 1) / G::TH);
        const int per_img = grid_x(tiles);
        hipLaunchKernelGGL((k_smoother_mfma<3>), dim3((unsigned)per_img, (unsigned)batch), dim3(kThreads), G::lds, s, b,
                           nrm2, nparts, dst, accumulate, wl, c->wbf_stride, ws, c->p.n_weight_sets, n, tiles_x, tiles,
                           dstb, bpitch, btiled ? 1 : 0);
    } else {
        using G = Geo<4>;
        const int tiles_x = (n + G::TW - 1) / G::TW, tiles = tiles_x * ((n + G::TH - 1) / G::TH);
        const int per_img = grid_x(tiles);
        hipLaunchKernelGGL((k_smoother_mfma<4>), dim3((unsigned)per_img, (unsigned)batch), dim3(kThreads), G::lds, s, b,
                           nrm2, nparts, dst, accumulate, wl, c->wbf_stride, ws, c->p.n_weight_sets, n, tiles_x, tiles,
                           dstb, bpitch, btiled ? 1 : 0);
    }
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

bool mfma_smoother_covers(const Ctx* c, int l, int pitch) {
    const int n = c->n[(size_t)l];
    int tw, th;
    if (c->p.n_layers == 3) {
        tw = Geo<3>::TW;
        th = Geo<3>::TH;
    } else {
        tw = Geo<4>::TW;
        th = Geo<4>::TH;
    }
    return pitch >= n && (n + tw - 1) / tw * tw >= pitch && (n + th - 1) / th * th >= pitch;
}

size_t mfma_lds_bytes(int n_layers) { return n_layers == 3 ? Geo<3>::lds : Geo<4>::lds; }

}  // namespace nmg
