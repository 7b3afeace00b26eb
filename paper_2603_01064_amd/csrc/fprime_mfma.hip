// Filter F'_l of Algorithms 3-4 in BF16 on MFMA (mixed-precision cycle).
//
//   F'(H) = C^T (m' .* (C H C^T)) C,   C = orthonormal DCT-II of the level size
//
// is evaluated as four batched "row GEMMs with transposed store"
//   out[b][j][i] = sum_k in[b][i][k] Mat[j][k]
// (Mat = C for the forward pair, C^T for the inverse pair); storing each
// product transposed turns the left multiplication into another right
// multiplication.  The ramp mask sqrt(max(k1, k2) / n) is applied in the
// epilogue of the second pass and the last pass accumulates into x.
// Inputs are rounded to BF16, products accumulate in FP32.
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
//   IN  0: in is the FP32 n x n level array (rounded to BF16 while staging)
//       1: in is a BF16 npad x npad intermediate (zero padded)
//   OUT 0: BF16 npad x npad intermediate; 1: the same times the ramp mask;
//       2: FP32 n x n result, stored or added (accumulate) into out
// BF16 intermediates are exactly the values the next pass would have rounded
// an FP32 intermediate to, and they halve the traffic between passes.
constexpr int kTI = 64, kTJ = 128, kKS = 32;

__device__ inline int frag_off(int row, int chunk) { return row * 64 + ((chunk ^ (row & 3)) << 4); }

template <int IN, int OUT>
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
            if constexpr (IN == 0) {
                const float* src = reinterpret_cast<const float*>(in_v) + (size_t)b * n * n;
                float v[8];
                for (int q = 0; q < 8; ++q) v[q] = (i < n && k + q < n) ? src[(size_t)i * n + k + q] : 0.f;
                areg[s] = make_uint4(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]), pack_bf16(v[4], v[5]),
                                     pack_bf16(v[6], v[7]));
            } else {
                const uint16_t* src = reinterpret_cast<const uint16_t*>(in_v) + (size_t)b * npad * npad;
                areg[s] = *reinterpret_cast<const uint4*>(src + (size_t)i * npad + k);
            }
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

// The same four products for a level with NP = n rounded up to 32 <= 64:
// one workgroup per image keeps the whole (BF16) intermediate in LDS, so the
// filter is one launch.  Every pass computes out[j][i] = sum_k Mat[j][k]
// in[i][k] tile by tile with the K steps of the four-launch kernel in the
// same order, and rounds its result to BF16 exactly where that kernel
// stages its operand, so both give the same values.
template <int NP>
__global__ void __launch_bounds__(kThreads) k_fprime_small(const float* __restrict__ in, float* __restrict__ dst,
                                                           const uint16_t* __restrict__ C,
                                                           const uint16_t* __restrict__ Ct,
                                                           const float* __restrict__ ramp, int n, int mstride,
                                                           int accumulate) {
    constexpr int NT = NP / 16;             // 16 x 16 output tiles per side
    constexpr int KS = NP / 32;             // K steps
    constexpr int RB = NP * 2;              // bytes per BF16 row
    __shared__ __attribute__((aligned(16))) char buf[2][NP * RB];
    const int b = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ln = lane & 15, lg = lane >> 4;
    const float* src = in + (size_t)b * n * n;
    // stage H (rows i, columns k) as BF16, zero beyond n
    for (int e = tid; e < NP * NP / 2; e += kThreads) {
        const int i = e / (NP / 2), k = (e % (NP / 2)) * 2;
        const float v0 = (i < n && k < n) ? src[(size_t)i * n + k] : 0.f;
        const float v1 = (i < n && k + 1 < n) ? src[(size_t)i * n + k + 1] : 0.f;
        *reinterpret_cast<uint32_t*>(buf[0] + i * RB + k * 2) = pack_bf16(v0, v1);
    }
    __syncthreads();
#pragma unroll 1
    for (int pass = 0; pass < 4; ++pass) {
        const uint16_t* M = pass < 2 ? C : Ct;
        const char* cur = buf[pass & 1];
        char* nxt = buf[(pass + 1) & 1];
        for (int t = wave; t < NT * NT; t += 4) {
            const int tj = t / NT, ti = t % NT;  // output rows j (M), columns i (N)
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k0 = ks * 32 + lg * 8;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(M + (size_t)(tj * 16 + ln) * mstride + k0);
                const bf16x8 bb = *reinterpret_cast<const bf16x8*>(cur + (ti * 16 + ln) * RB + k0 * 2);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc, 0, 0, 0);
            }
            const int i = ti * 16 + ln;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = tj * 16 + lg * 4 + q;
                float v = acc[q];
                if (pass == 1) v = (i < n && j < n) ? v * ramp[i > j ? i : j] : 0.f;
                if (pass < 3) {
                    // next pass reads row j, column i
                    const float2v f = {v, 0.f};
                    const bf16x2 p = __builtin_convertvector(f, bf16x2);
                    uint16_t u;
                    __builtin_memcpy(&u, &p, 2);
                    *reinterpret_cast<uint16_t*>(nxt + j * RB + i * 2) = u;
                } else if (i < n && j < n) {
                    float* o = dst + (size_t)b * n * n + (size_t)j * n + i;
                    *o = accumulate ? *o + v : v;
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

// dst (+)= F'(h) on level l for a 2D float cycle; t1/t2 are level-sized scratch.
nmg_status launch_fprime_mfma(const Ctx* c, int l, int batch, const float* h, float* dst, int accumulate,
                              float* t1, float* t2, hipStream_t s) {
    const int n = c->n[(size_t)l];
    const int npad = (n + 127) / 128 * 128;
    const int ti = npad / kTI, tj = npad / kTJ;
    const uint16_t* C = c->dctbf + c->dctbf_off[(size_t)l];
    const uint16_t* Ct = C + (size_t)npad * npad;
    if (n <= 64) {
        const float* rp = c->ramp + c->ramp_off[(size_t)l];
        if (n <= 32)
            hipLaunchKernelGGL(k_fprime_small<32>, dim3(batch), dim3(kThreads), 0, s, h, dst, C, Ct, rp, n, npad,
                               accumulate);
        else
            hipLaunchKernelGGL(k_fprime_small<64>, dim3(batch), dim3(kThreads), 0, s, h, dst, C, Ct, rp, n, npad,
                               accumulate);
        NMG_HIP(hipGetLastError());
        return NMG_OK;
    }
    if ((size_t)npad * npad * 2 > (size_t)n * n * 4)
        return fail(NMG_ERR_SHAPE, "F' scratch too small for this level size");
    dim3 grid((unsigned)(ti * tj), (unsigned)batch);
    const float* rp = c->ramp + c->ramp_off[(size_t)l];
    // BF16 intermediates (npad x npad per image) live in the level scratch buffers
    hipLaunchKernelGGL((k_rowgemm_t<0, 0>), grid, dim3(kThreads), 0, s, h, t1, C, rp, n, npad, tj, 0);
    hipLaunchKernelGGL((k_rowgemm_t<1, 1>), grid, dim3(kThreads), 0, s, t1, t2, C, rp, n, npad, tj, 0);
    hipLaunchKernelGGL((k_rowgemm_t<1, 0>), grid, dim3(kThreads), 0, s, t2, t1, Ct, rp, n, npad, tj, 0);
    hipLaunchKernelGGL((k_rowgemm_t<1, 2>), grid, dim3(kThreads), 0, s, t1, dst, Ct, rp, n, npad, tj, accumulate);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

}  // namespace nmg
