// Filter F'_l of Algorithms 3-4 in BF16 on MFMA (mixed-precision cycle).
//
//   F'(H) = C^T (m' .* (C H C^T)) C,   C = orthonormal DCT-II of the level size
//
// Operands are BF16, products accumulate in FP32, and every product
// contracts along the contiguous index of both operands.  Three forms:
//  * padded sizes NP <= 512 (levels 65..511): two fused launches.  A
//    workgroup owns a column block I of the result; it forms
//    P = A[I,:] H^T into LDS and then A P^T, i.e. the columns I of A H A^T.
//    The first launch (A = C) applies the ramp mask sqrt(max(k1, k2) / n) and
//    stores the masked spectrum as BF16; the second (A = C^T) adds C^T M C
//    into x.
//  * NP >= 1024: four batched "row GEMMs with transposed store"
//      out[b][j][i] = sum_k in[b][i][k] Mat[j][k]
//    (storing each product transposed turns the left multiplication into
//    another right multiplication), mask in the second pass's epilogue.
//  * n <= 64: one workgroup per image with the intermediate in LDS.
// All three accumulate each dot product over the same ascending K steps of
// 32 and round the same intermediates to BF16, so they give the same values
// (and a result does not depend on the batch it is computed in).
// The input is a zero-padded BF16 NP x NP plane per image: the BF16 smoother
// writes it directly; FP32 inputs are rounded into it first.
#include <mutex>
#include <vector>

#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kThreads = 256;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats to packed BF16 (hardware round-to-nearest-even).
__device__ inline uint32_t pack_bf16(float a, float b) {
    const float2v f = {a, b};
    const bf16x2 p = __builtin_convertvector(f, bf16x2);
    uint32_t u;
    __builtin_memcpy(&u, &p, 4);
    return u;
}

inline uint16_t f2bf_h(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One pass out[b][j][i] = sum_k in[b][i][k] Mat[j][k] on a workgroup tile of
// 64 (i) x 128 (j); wave w computes rows 32*(w/2).. and columns 64*(w%2).. as
// 2 x 4 MFMA blocks.  Each k-step of 32 stages the A tile (in) and the B
// tile (Mat) in LDS with the 16-byte chunk of row r stored at chunk ^ (r & 3)
// to spread the fragment reads over banks; four k-steps are staged per
// barrier pair.
// in is a zero-padded BF16 npad x npad plane;
//   OUT 0: BF16 npad x npad intermediate; 1: the same times the ramp mask;
//       2: FP32 n x n result, stored or added (accumulate) into out
// BF16 intermediates are exactly the values the next pass would have rounded
// an FP32 intermediate to, and they halve the traffic between passes.
constexpr int kTI = 64, kTJ = 128, kKS = 32;

__device__ inline int frag_off(int row, int chunk) { return row * 64 + ((chunk ^ (row & 3)) << 4); }

template <int OUT>
__global__ void __launch_bounds__(kThreads) k_rowgemm_t(const void* __restrict__ in_v, void* __restrict__ out_v,
                                                        const uint16_t* __restrict__ mat,
                                                        const float* __restrict__ ramp, int n, int npad,
                                                        int tiles_j, int accumulate) {
    // kKC K steps of 32 are staged per barrier pair: every thread has all of
    // its loads of a 128-wide K chunk in flight at once
    constexpr int kKC = 4;
    __shared__ __attribute__((aligned(16))) char As[kKC][kTI * kKS * 2];
    __shared__ __attribute__((aligned(16))) char Bs[kKC][kTJ * kKS * 2];
    const int b = blockIdx.y;
    const int ti = blockIdx.x / tiles_j, tj = blockIdx.x % tiles_j;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int ln = lane & 15, lg = lane >> 4;
    const int i0 = ti * kTI, j0 = tj * kTJ;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 64;
    floatx4 acc[2][4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 4; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    // staging roles: A: row tid/4, chunk tid%4 (8 values); B: rows tid/4 and 64 + tid/4
    const int sr = tid >> 2, sc = tid & 3;
    for (int k0 = 0; k0 < npad; k0 += kKS * kKC) {  // npad is a multiple of 128
        uint4 areg[kKC], breg[kKC][2];
#pragma unroll
        for (int s = 0; s < kKC; ++s) {
            const int i = i0 + sr, k = k0 + s * kKS + sc * 8;
            const uint16_t* src = reinterpret_cast<const uint16_t*>(in_v) + (size_t)b * npad * npad;
            areg[s] = *reinterpret_cast<const uint4*>(src + (size_t)i * npad + k);
            for (int h = 0; h < 2; ++h) {
                const int j = j0 + sr + 64 * h;  // < npad by construction
                breg[s][h] = *reinterpret_cast<const uint4*>(mat + (size_t)j * npad + k);
            }
        }
#pragma unroll
        for (int s = 0; s < kKC; ++s) {
            *reinterpret_cast<uint4*>(As[s] + frag_off(sr, sc)) = areg[s];
            for (int h = 0; h < 2; ++h) *reinterpret_cast<uint4*>(Bs[s] + frag_off(sr + 64 * h, sc)) = breg[s][h];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kKC; ++s) {
            bf16x8 af[2], bfr[4];
            for (int r = 0; r < 2; ++r)
                af[r] = *reinterpret_cast<const bf16x8*>(As[s] + frag_off(wi + r * 16 + ln, lg));
            for (int c = 0; c < 4; ++c)
                bfr[c] = *reinterpret_cast<const bf16x8*>(Bs[s] + frag_off(wj + c * 16 + ln, lg));
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 4; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r], bfr[c], acc[r][c], 0, 0, 0);
        }
        __syncthreads();
    }
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + wj + c * 16 + ln;
            const int ib = i0 + wi + r * 16 + lg * 4;  // four consecutive i
            if constexpr (OUT == 2) {
                if (j >= n) continue;
                float* dst = reinterpret_cast<float*>(out_v) + (size_t)b * n * n + (size_t)j * n;
                for (int q = 0; q < 4; ++q) {
                    const int i = ib + q;
                    if (i >= n) continue;
                    dst[i] = accumulate ? dst[i] + acc[r][c][q] : acc[r][c][q];
                }
            } else {
                float v[4];
                for (int q = 0; q < 4; ++q) {
                    v[q] = acc[r][c][q];
                    if constexpr (OUT == 1) {
                        const int i = ib + q;
                        v[q] = (i < n && j < n) ? v[q] * ramp[i > j ? i : j] : 0.f;
                    }
                }
                uint16_t* dst = reinterpret_cast<uint16_t*>(out_v) + (size_t)b * npad * npad + (size_t)j * npad;
                *reinterpret_cast<uint2*>(dst + ib) = make_uint2(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]));
            }
        }
}

// Fragment-tiled BF16 layout of an NP x NP plane (NP <= 512): element (r, k)
// sits in the 1 KB tile ((r >> 4) * (NP / 32) + (k >> 5)) at lane
// (r & 15) + 16 ((k & 31) >> 3), element k & 7.  One tile is exactly one
// 16 x 32 MFMA operand fragment (lane = row + 16 * K group of 8), so every
// operand load is 1 KB of contiguous memory and LDS fragment reads need no
// swizzle.  The smoother writes this layout directly.
__device__ __host__ inline size_t tiled_off(int np, int r, int k) {
    return ((size_t)((r >> 4) * (np >> 5) + (k >> 5)) << 9) + (size_t)(((r & 15) + 16 * ((k & 31) >> 3)) * 8 + (k & 7));
}

// One half of F' for padded sizes NP <= 512 on tiled planes.  Workgroup
// (image, column block I = [I0, I0 + CB)):
//   step 1  P[i][k]      = sum_m A[I0 + i][m] in[k][m]     CB x NP, BF16 in LDS
//   step 2  R[j][I0 + i] = sum_k A[j][k] P[i][k]            NP x CB
// STAGE 0 (A = C, in = H): R = C H C^T on columns I; masked by the ramp and
//   stored as BF16 into the tiled spectrum plane (zero outside n x n).
// STAGE 1 (A = C^T, in = that spectrum M): R = C^T M C on columns I, stored
//   or added into the FP32 n x n level array, row by row through LDS so the
//   global accesses are coalesced.
// The MFMA M dimension is i: the CB rows shared by the WAVES waves (rows of
// A staged whole in LDS for step 1, then P in their place).  N is the
// wave's NP / WAVES private rows (image rows in step 1, rows of A in step
// 2), loaded straight into operand registers.  The 2 NP / 32 K steps of
// those rows (step 1's, then step 2's) form one stream read through a ring
// of KCH register slots: the first KCH are issued at the start, and each
// slot is refilled with the step KCH ahead as soon as its products are
// issued.  With KCH = NP / 32 all of step 1 is in flight at once and step 2
// loads while step 1 computes.
template <int NP, int CB, int WAVES, int KCH, int STAGE>
__global__ void __launch_bounds__(64 * WAVES) k_fprime_tiled(const uint16_t* __restrict__ in, void* __restrict__ out,
                                                             const uint16_t* __restrict__ A,
                                                             const float* __restrict__ ramp, int n, int accumulate) {
    constexpr int NTH = 64 * WAVES;
    constexpr int KST = NP / 32;            // K steps of 32
    constexpr int NBLK = NP / CB;
    constexpr int MT = CB / 16;
    constexpr int NWR = NP / WAVES;         // private rows per wave
    constexpr int NT = NWR / 16;
    constexpr int APT = (CB / 16) * KST * 64 / NTH;  // 16-byte pieces of the staged rows of A per thread
    constexpr int PB = CB * NP * 2;                  // bytes of P (and of the staged rows of A)
    constexpr int OPITCH = CB + 4;                   // floats per LDS row of the STAGE 1 output
    constexpr int OB = STAGE == 1 ? NP * OPITCH * 4 : 0;
    constexpr int LB = PB > OB ? PB : OB;
    static_assert((CB / 16) * KST * 64 % NTH == 0 && APT > 0 && NWR % 16 == 0 && NP % CB == 0, "F' tile shape");
    __shared__ __attribute__((aligned(16))) char Ls[LB];

    // XCD-aware numbering (workgroups go round-robin over the 8 XCDs by linear
    // id): the column blocks of one image run on one XCD and share its L2
    int img, blk;
    {
        const int G = gridDim.x, i = blockIdx.x;
        const int x = i % 8, q = G / 8, rem = G % 8;
        const int p = x * q + min(x, rem) + i / 8;
        img = p / NBLK;
        blk = p - img * NBLK;
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ln = lane & 15, lg = lane >> 4;
    const int I0 = blk * CB;
    const int wrow = wave * NWR;
    const uint16_t* src = in + (size_t)img * NP * NP;
    // fragment (rows 16 g .. 16 g + 15, K step st) of a tiled plane
    auto frag = [&](const uint16_t* base, int g, int st) {
        return *reinterpret_cast<const bf16x8*>(base + ((size_t)(g * KST + st) << 9) + lane * 8);
    };

    // rows I of A: CB / 16 row groups of KST contiguous tiles
    const uint16_t* Ab = A + ((size_t)(I0 >> 4) * KST << 9);
    // (two named registers, not an array: an array here was moved to LDS)
    static_assert(APT <= 2, "staging pieces per thread");
    const uint4 ar0 = *reinterpret_cast<const uint4*>(Ab + (size_t)tid * 8);
    uint4 ar1 = ar0;
    if constexpr (APT == 2) ar1 = *reinterpret_cast<const uint4*>(Ab + (size_t)(tid + NTH) * 8);
    static_assert(KCH >= 1 && KCH <= KST, "register ring depth");
    bf16x8 pv[NT][KCH];
    // stream step t: K step t of the image rows (t < KST), else K step t - KST of the rows of A
    auto fetch = [&](int t) {
        if (t >= 2 * KST) return;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            pv[nt][t % KCH] = t < KST ? frag(src, (wrow >> 4) + nt, t) : frag(A, (wrow >> 4) + nt, t - KST);
    };
#pragma unroll
    for (int t = 0; t < KCH; ++t) fetch(t);
    // STAGE 1 adds into x: this thread's values of x are loaded now (behind
    // the first operand steps, ahead of the refills), so their latency
    // overlaps the products.  Element k is row j = tid / CB + k NTH / CB,
    // column I0 + tid % CB; x is read through a buffer resource and an element
    // outside the image takes an out-of-range offset, which reads zero.  With
    // 16 waves (128 registers per lane) the values would not fit beside the
    // operand ring, so that shape reads x in the epilogue instead.
    constexpr bool kPrefetchX = STAGE == 1 && NTH <= 512;
    constexpr int EPT = STAGE == 1 ? NP * CB / NTH : 1;
    static_assert(STAGE == 0 || (NP * CB % NTH == 0 && NTH % CB == 0), "F' output elements per thread");
    float xv[kPrefetchX ? EPT : 1];
    // STAGE 0 scales its outputs by the ramp mask: the ramp values of this
    // thread's outputs are loaded here too (output (mt, nt, q) is row
    // j = wrow + 16 nt + ln, column i = I0 + 16 mt + 4 lg + q, and takes
    // ramp[max(i, j)], zero outside the grid)
    constexpr bool kPrefetchRamp = STAGE == 0 && NTH <= 512;
    float rv[kPrefetchRamp ? MT : 1][kPrefetchRamp ? NT : 1][4];
    if constexpr (kPrefetchRamp) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = I0 + mt * 16 + lg * 4 + q, j = wrow + nt * 16 + ln;
                    rv[mt][nt][q] = (i < n && j < n) ? ramp[i > j ? i : j] : 0.f;
                }
    }
    if constexpr (kPrefetchX) {
        const __amdgpu_buffer_rsrc_t xres = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<float*>(out) + (size_t)img * n * n, (short)0, n * n * 4, 0x00020000);
        const int xi = I0 + tid % CB;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int j = tid / CB + k * (NTH / CB);
            const bool ok = accumulate && j < n && xi < n;
            xv[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                  xres, ok ? (j * n + xi) * 4 : (int)0x80000000, 0, 0));
        }
    }
    *reinterpret_cast<uint4*>(Ls + tid * 16) = ar0;
    if constexpr (APT == 2) *reinterpret_cast<uint4*>(Ls + (tid + NTH) * 16) = ar1;
    __syncthreads();

    floatx4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    // ---- step 1: P = A[I, :] in^T
#pragma unroll
    for (int st = 0; st < KST; ++st) {
        bf16x8 af[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) af[mt] = *reinterpret_cast<const bf16x8*>(Ls + ((mt * KST + st) << 10) + lane * 16);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], pv[nt][st % KCH], acc[mt][nt], 0, 0, 0);
        fetch(st + KCH);
        // keep each refill behind the products that free its registers
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // every wave has read its last rows of A from LDS
    // P[i][k] into LDS in the tiled layout: acc[mt][nt][q] is row i = 16 mt + 4 lg + q,
    // column k = wrow + 16 nt + ln
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int k = wrow + nt * 16 + ln;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int il = lg * 4 + q;
                const int off = ((mt * KST + (k >> 5)) << 10) + ((il + 16 * ((k & 31) >> 3)) << 4) + (k & 7) * 2;
                *reinterpret_cast<uint16_t*>(Ls + off) = (uint16_t)pack_bf16(acc[mt][nt][q], 0.f);
            }
            acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    __syncthreads();
    // ---- step 2: R[j][I0 + i] = sum_k A[j][k] P[i][k]
#pragma unroll
    for (int st = 0; st < KST; ++st) {
        bf16x8 af[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) af[mt] = *reinterpret_cast<const bf16x8*>(Ls + ((mt * KST + st) << 10) + lane * 16);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], pv[nt][(KST + st) % KCH], acc[mt][nt], 0,
                                                                      0, 0);
        if constexpr (KCH < KST) {
            fetch(KST + st + KCH);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // ---- epilogue: acc[mt][nt][q] = R[j][i], j = wrow + 16 nt + ln, i = I0 + 16 mt + 4 lg + q
    if constexpr (STAGE == 0) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int j = wrow + nt * 16 + ln;
                const int ib = I0 + mt * 16 + lg * 4;
                float v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = ib + q;
                    if constexpr (kPrefetchRamp)
                        v[q] = (i < n && j < n) ? acc[mt][nt][q] * rv[mt][nt][q] : 0.f;
                    else
                        v[q] = (i < n && j < n) ? acc[mt][nt][q] * ramp[i > j ? i : j] : 0.f;
                }
                // four consecutive columns share one 16-byte group of the tile
                uint16_t* dst = reinterpret_cast<uint16_t*>(out) + (size_t)img * NP * NP + tiled_off(NP, j, ib);
                *reinterpret_cast<uint2*>(dst) = make_uint2(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]));
            }
    } else {
        __syncthreads();  // every wave has read P
        float* O = reinterpret_cast<float*>(Ls);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                *reinterpret_cast<floatx4*>(O + (wrow + nt * 16 + ln) * OPITCH + mt * 16 + lg * 4) = acc[mt][nt];
        __syncthreads();
        float* xb = reinterpret_cast<float*>(out) + (size_t)img * n * n;
        const int i = tid % CB;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int j = tid / CB + k * (NTH / CB);
            if (j < n && I0 + i < n) {
                const float v = O[j * OPITCH + i];
                float* d = xb + (size_t)j * n + I0 + i;
                if constexpr (kPrefetchX)
                    *d = accumulate ? xv[k] + v : v;
                else
                    *d = accumulate ? *d + v : v;
            }
        }
    }
}

// FP32 n x n images -> zero-padded BF16 NP x NP planes (round to nearest
// even), tiled (NP <= 512) or row-major
__global__ void __launch_bounds__(kThreads) k_bf16_pad(const float* __restrict__ in, uint16_t* __restrict__ out, int n,
                                                       int np, int tiled) {
    const int b = blockIdx.y;
    const size_t e = ((size_t)blockIdx.x * kThreads + threadIdx.x) * 2;  // two columns per thread
    if (e >= (size_t)np * np) return;
    const int i = (int)(e / np), k = (int)(e % np);
    const float* src = in + (size_t)b * n * n + (size_t)i * n;
    const float v0 = (i < n && k < n) ? src[k] : 0.f;
    const float v1 = (i < n && k + 1 < n) ? src[k + 1] : 0.f;
    const size_t o = tiled ? tiled_off(np, i, k) : e;  // k even: both columns in one 16-byte group
    *reinterpret_cast<uint32_t*>(out + (size_t)b * np * np + o) = pack_bf16(v0, v1);
}

// The same four products for a level with NP = n rounded up to 32 <= 64:
// one workgroup per image keeps the whole (BF16) intermediate, the image and
// both DCT matrices in LDS, so the filter is one launch that reads global
// memory once.  Every pass computes out[j][i] = sum_k Mat[j][k] in[i][k]
// tile by tile with the K steps of the larger kernels in the same order, and
// rounds its result to BF16 exactly where they stage their operands, so all
// forms give the same values.  LDS rows keep their 16-byte chunk c at
// c ^ (row & SW), which spreads the 16 rows of a fragment read over the banks.
constexpr int kSmallThreads = 512;

template <int NP>
__global__ void __launch_bounds__(kSmallThreads) k_fprime_small(const float* __restrict__ in, float* __restrict__ dst,
                                                                const uint16_t* __restrict__ C,
                                                                const uint16_t* __restrict__ Ct,
                                                                const float* __restrict__ ramp, int n, int mstride,
                                                                int accumulate) {
    constexpr int NT = NP / 16;             // 16 x 16 output tiles per side
    constexpr int KS = NP / 32;             // K steps
    constexpr int RB = NP * 2;              // bytes per BF16 row
    constexpr int CPR = NP / 8;             // 16-byte chunks per row
    constexpr int SW = CPR < 8 ? CPR - 1 : 7;
    constexpr int WAVES = kSmallThreads / 64;
    __shared__ __attribute__((aligned(16))) char buf[2][NP * RB];
    __shared__ __attribute__((aligned(16))) char mats[2][NP * RB];
    __shared__ float rp[NP];
    const int b = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ln = lane & 15, lg = lane >> 4;
    const float* src = in + (size_t)b * n * n;
    auto off = [](int r, int ch) { return r * RB + ((ch ^ (r & SW)) << 4); };
    // C and C^T (rows of the padded tables), the ramp, and H as BF16 (zero
    // beyond n): every global load of a thread is issued before its first
    // LDS store
    constexpr int MI = (2 * NP * CPR + kSmallThreads - 1) / kSmallThreads;  // table chunks per thread
    constexpr int HI = (NP * NP / 2 + kSmallThreads - 1) / kSmallThreads;   // H pairs per thread
    uint4 mv[MI];
    float hv[HI][2];
#pragma unroll
    for (int u = 0; u < MI; ++u) {
        const int e = tid + u * kSmallThreads;
        const int m = e / (NP * CPR), r = (e / CPR) % NP, ch = e % CPR;
        const uint16_t* M = m == 0 ? C : Ct;
        mv[u] = e < 2 * NP * CPR ? *reinterpret_cast<const uint4*>(M + (size_t)r * mstride + ch * 8) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < HI; ++u) {
        const int e = tid + u * kSmallThreads;
        const int i = e / (NP / 2), k = (e % (NP / 2)) * 2;
        const bool ok = e < NP * NP / 2;
        hv[u][0] = (ok && i < n && k < n) ? src[(size_t)i * n + k] : 0.f;
        hv[u][1] = (ok && i < n && k + 1 < n) ? src[(size_t)i * n + k + 1] : 0.f;
    }
    const float rpv = (tid < NP && tid < n) ? ramp[tid] : 0.f;
    // the values of dst this wave's last-pass outputs add to, loaded with
    // the rest (output tile t of pass 3 is rows 16 (t / NT) + 4 lg .. + 3,
    // column 16 (t % NT) + ln) through a buffer resource over the image: an
    // element outside it takes an out-of-range offset and reads zero, so the
    // loads need no branch and issue together
    constexpr int TPW = (NT * NT + WAVES - 1) / WAVES;  // output tiles per wave
    float* dimg = dst + (size_t)b * n * n;
    const __amdgpu_buffer_rsrc_t dres = __builtin_amdgcn_make_buffer_rsrc(dimg, (short)0, n * n * 4, 0x00020000);
    float dv[TPW][4];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = wave + u * WAVES;
        const int i = (t % NT) * 16 + ln;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = (t / NT) * 16 + lg * 4 + q;
            const bool ok = accumulate && t < NT * NT && i < n && j < n;
            dv[u][q] = __builtin_bit_cast(float,
                                          __builtin_amdgcn_raw_buffer_load_b32(dres, ok ? (j * n + i) * 4 : (int)0x80000000, 0, 0));
        }
    }
#pragma unroll
    for (int u = 0; u < MI; ++u) {
        const int e = tid + u * kSmallThreads;
        const int m = e / (NP * CPR), r = (e / CPR) % NP, ch = e % CPR;
        if (e < 2 * NP * CPR) *reinterpret_cast<uint4*>(mats[m] + off(r, ch)) = mv[u];
    }
    if (tid < NP) rp[tid] = rpv;
#pragma unroll
    for (int u = 0; u < HI; ++u) {
        const int e = tid + u * kSmallThreads;
        const int i = e / (NP / 2), k = (e % (NP / 2)) * 2;
        if (e < NP * NP / 2)
            *reinterpret_cast<uint32_t*>(buf[0] + off(i, k >> 3) + (k & 7) * 2) = pack_bf16(hv[u][0], hv[u][1]);
    }
    __syncthreads();
#pragma unroll 1
    for (int pass = 0; pass < 4; ++pass) {
        const char* M = mats[pass < 2 ? 0 : 1];
        const char* cur = buf[pass & 1];
        char* nxt = buf[(pass + 1) & 1];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int t = wave + u * WAVES;
            if (t >= NT * NT) break;
            const int tj = t / NT, ti = t % NT;  // output rows j (M), columns i (N)
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int ch = ks * 4 + lg;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(M + off(tj * 16 + ln, ch));
                const bf16x8 bb = *reinterpret_cast<const bf16x8*>(cur + off(ti * 16 + ln, ch));
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc, 0, 0, 0);
            }
            const int i = ti * 16 + ln;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = tj * 16 + lg * 4 + q;
                float v = acc[q];
                if (pass == 1) v = (i < n && j < n) ? v * rp[i > j ? i : j] : 0.f;
                if (pass < 3) {
                    // next pass reads row j, column i
                    *reinterpret_cast<uint16_t*>(nxt + off(j, i >> 3) + (i & 7) * 2) = (uint16_t)pack_bf16(v, 0.f);
                } else if (i < n && j < n) {
                    dimg[(size_t)j * n + i] = accumulate ? dv[u][q] + v : v;
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

nmg_status prepare_fprime_bf16(Ctx* c) {
    if (c->dctbf && c->ramp) return NMG_OK;
    if (c->dctbf) (void)hipFree(c->dctbf);
    if (c->ramp) (void)hipFree(c->ramp);
    c->dctbf = nullptr;
    c->ramp = nullptr;
    std::vector<uint16_t> all;
    c->dctbf_off.clear();
    for (int l = 0; l < c->L; ++l) {
        const int n = c->n[(size_t)l];
        const int npad = (n + 127) / 128 * 128;
        std::vector<uint16_t> C((size_t)npad * npad, 0), Ct((size_t)npad * npad, 0);
        for (int k = 0; k < n; ++k) {
            const double ck = k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
            for (int i = 0; i < n; ++i) {
                const float v = (float)(ck * std::cos(M_PI * k * (2.0 * i + 1.0) / (2.0 * n)));
                C[(size_t)k * npad + i] = f2bf_h(v);
                Ct[(size_t)i * npad + k] = f2bf_h(v);
            }
        }
        if (fprime_tiled_layout(n)) {
            // the two-launch kernels read C and C^T in the fragment-tiled layout
            std::vector<uint16_t> Ctl(C.size()), Cttl(Ct.size());
            for (int r = 0; r < npad; ++r)
                for (int k = 0; k < npad; ++k) {
                    Ctl[tiled_off(npad, r, k)] = C[(size_t)r * npad + k];
                    Cttl[tiled_off(npad, r, k)] = Ct[(size_t)r * npad + k];
                }
            C.swap(Ctl);
            Ct.swap(Cttl);
        }
        c->dctbf_off.push_back(all.size());
        all.insert(all.end(), C.begin(), C.end());
        all.insert(all.end(), Ct.begin(), Ct.end());
    }
    // ramp sqrt(k / n) per level for the mask epilogue
    std::vector<float> ramps;
    c->ramp_off.clear();
    for (int l = 0; l < c->L; ++l) {
        const int n = c->n[(size_t)l];
        c->ramp_off.push_back(ramps.size());
        for (int k = 0; k < n; ++k) ramps.push_back((float)std::sqrt((double)k / (double)n));
    }
    hipError_t er = hipMalloc((void**)&c->ramp, ramps.size() * sizeof(float));
    if (er != hipSuccess) {
        (void)hipGetLastError();
        c->ramp = nullptr;
        return fail(NMG_ERR_OOM, "hipMalloc failed for the F' ramp tables");
    }
    NMG_HIP(hipMemcpy(c->ramp, ramps.data(), ramps.size() * sizeof(float), hipMemcpyHostToDevice));
    hipError_t e = hipMalloc((void**)&c->dctbf, all.size() * sizeof(uint16_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->dctbf = nullptr;
        return fail(NMG_ERR_OOM, "hipMalloc failed for BF16 DCT matrices");
    }
    NMG_HIP(hipMemcpy(c->dctbf, all.data(), all.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    return NMG_OK;
}

namespace {

template <int NP, int CB, int WAVES, int KCH>
void launch_tiled_pair(int batch, const uint16_t* hb, uint16_t* spec, float* dst, const uint16_t* C,
                       const uint16_t* Ct, const float* rp, int n, int accumulate, hipStream_t s) {
    const dim3 grid((unsigned)(NP / CB * batch));
    hipLaunchKernelGGL((k_fprime_tiled<NP, CB, WAVES, KCH, 0>), grid, dim3(64 * WAVES), 0, s, hb, (void*)spec, C, rp,
                       n, 0);
    hipLaunchKernelGGL((k_fprime_tiled<NP, CB, WAVES, KCH, 1>), grid, dim3(64 * WAVES), 0, s, spec, (void*)dst, Ct, rp,
                       n, accumulate);
}

}  // namespace

bool fprime_tiled_layout(int n) { return n > 64 && (n + 127) / 128 * 128 <= 512; }

size_t fprime_mfma_scratch_bytes(int n, int batch) {
    if (n <= 64) return 0;
    const size_t np = (size_t)(n + 127) / 128 * 128;
    return 2 * (size_t)batch * np * np * sizeof(uint16_t);
}

// dst (+)= F'(h) on level l for a 2D float cycle.  The input is either the
// FP32 level array h or, when hb is given, its zero-padded BF16 NP x NP plane.
// t1 and t2 are scratch_bytes each and need batch * NP * NP BF16 values each
// (levels above 64^2); hb may be t1.
nmg_status launch_fprime_mfma(const Ctx* c, int l, int batch, const float* h, const uint16_t* hb, float* dst,
                              int accumulate, void* t1, void* t2, size_t scratch_bytes, hipStream_t s) {
    const int n = c->n[(size_t)l];
    const int npad = (n + 127) / 128 * 128;
    if (!c->dctbf || !c->ramp) return fail(NMG_ERR_STATE, "BF16 DCT tables are not built");
    if (n > 64 && 2 * scratch_bytes < fprime_mfma_scratch_bytes(n, batch))
        return fail(NMG_ERR_SHAPE, "F' scratch too small for this level size and batch");
    const uint16_t* C = c->dctbf + c->dctbf_off[(size_t)l];
    const uint16_t* Ct = C + (size_t)npad * npad;
    const float* rp = c->ramp + c->ramp_off[(size_t)l];
    if (n <= 64) {
        if (!h) return fail(NMG_ERR_ARG, "F' on levels up to 64^2 takes the FP32 level array");
        if (n <= 32)
            hipLaunchKernelGGL(k_fprime_small<32>, dim3(batch), dim3(kSmallThreads), 0, s, h, dst, C, Ct, rp, n, npad,
                               accumulate);
        else
            hipLaunchKernelGGL(k_fprime_small<64>, dim3(batch), dim3(kSmallThreads), 0, s, h, dst, C, Ct, rp, n,
                               npad, accumulate);
        NMG_HIP(hipGetLastError());
        return NMG_OK;
    }
    uint16_t* b1 = reinterpret_cast<uint16_t*>(t1);
    uint16_t* b2 = reinterpret_cast<uint16_t*>(t2);
    const bool tiled = fprime_tiled_layout(n);
    if (!hb) {
        const size_t pairs = (size_t)npad * npad / 2;
        hipLaunchKernelGGL(k_bf16_pad, dim3((unsigned)((pairs + kThreads - 1) / kThreads), (unsigned)batch),
                           dim3(kThreads), 0, s, h, b1, n, npad, tiled ? 1 : 0);
        hb = b1;
    }
    if (hb == b2) return fail(NMG_ERR_ARG, "F' input plane overlaps its scratch");
    if (npad == 128) {
        launch_tiled_pair<128, 32, 8, 4>(batch, hb, b2, dst, C, Ct, rp, n, accumulate, s);
    } else if (npad == 256) {
        launch_tiled_pair<256, 32, 8, 8>(batch, hb, b2, dst, C, Ct, rp, n, accumulate, s);
    } else if (npad == 512) {
        launch_tiled_pair<512, 32, 16, 8>(batch, hb, b2, dst, C, Ct, rp, n, accumulate, s);
    } else if (tiled) {
        return fail(NMG_ERR_SHAPE, "F' on MFMA: unsupported padded size " + std::to_string(npad));
    } else {
        const int ti = npad / kTI, tj = npad / kTJ;
        dim3 grid((unsigned)(ti * tj), (unsigned)batch);
        // hb -> b2 -> b1 (masked) -> b2 -> dst; hb is dead after the first pass
        hipLaunchKernelGGL((k_rowgemm_t<0>), grid, dim3(kThreads), 0, s, hb, b2, C, rp, n, npad, tj, 0);
        hipLaunchKernelGGL((k_rowgemm_t<1>), grid, dim3(kThreads), 0, s, b2, b1, C, rp, n, npad, tj, 0);
        hipLaunchKernelGGL((k_rowgemm_t<0>), grid, dim3(kThreads), 0, s, b1, b2, Ct, rp, n, npad, tj, 0);
        hipLaunchKernelGGL((k_rowgemm_t<2>), grid, dim3(kThreads), 0, s, b2, dst, Ct, rp, n, npad, tj, accumulate);
    }
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

// ---------------------------------------------------------------------------
// No-allocation F' (nmg_apply_fprime_noalloc): its two BF16 scratch planes
// live in this file-scope device array, one copy per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel: it
// uses the device address hipGetSymbolAddress returns for each device.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

nmg_status fprime_noalloc_init() {
    int dev = 0;
    NMG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NMG_ERR_STATE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return NMG_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(NMG_ERR_HIP, std::string("hipGetSymbolAddress of the F' scratch failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
    return NMG_OK;
}

}  // namespace nmg

using namespace nmg;

extern "C" nmg_status nmg_apply_fprime_noalloc(nmg_handle h, int level, int batch, const float* in, float* out,
                                               void* stream) {
    if (!h) return fail(NMG_ERR_ARG, "null handle");
    if (batch < 1 || batch > h->p.max_batch) return fail(NMG_ERR_SHAPE, "batch must be in [1, max_batch]");
    if (!in || !out) return fail(NMG_ERR_ARG, "null pointer");
    if (level < 0 || level >= h->L) return fail(NMG_ERR_ARG, "level out of range");
    if (h->p.dim != 2) return fail(NMG_ERR_ARG, "the no-allocation F' is the 2D BF16 filter");
    const int n = h->n[(size_t)level];
    const size_t need = fprime_mfma_scratch_bytes(n, batch);
    if (need > kNoAllocScratchBytes)
        return fail(NMG_ERR_SHAPE, "no-allocation F' needs " + std::to_string(need) + " bytes of scratch for " +
                                       std::to_string(batch) + " images of side " + std::to_string(n) +
                                       "; the limit is " + std::to_string(kNoAllocScratchBytes) +
                                       " (4 * batch * NP^2 bytes, NP = side rounded up to 128)");
    // first call on a device that no handle was set up on
    NMG_TRY(fprime_noalloc_init());
    int dev = 0;
    NMG_HIP(hipGetDevice(&dev));
    char* base;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = static_cast<char*>(g_scratch_ptr[dev]);
    }
    const size_t half = kNoAllocScratchBytes / 2;
    return launch_fprime_mfma(h, level, batch, in, nullptr, out, 0, base, base + half, half, (hipStream_t)stream);
}

