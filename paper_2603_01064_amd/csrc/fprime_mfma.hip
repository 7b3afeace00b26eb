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

__device__ inline uint16_t f2bf_d(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

inline uint16_t f2bf_h(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// EPI 0: store, 1: store times the ramp mask, 2: add into out.
template <int EPI>
__global__ void __launch_bounds__(kThreads) k_rowgemm_t(const float* __restrict__ in, float* __restrict__ out,
                                                        const uint16_t* __restrict__ mat, int n, int npad,
                                                        int tiles_j) {
    const int b = blockIdx.y;
    const int ti = blockIdx.x / tiles_j, tj = blockIdx.x % tiles_j;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ln = lane & 15, lg = lane >> 4;
    const int ib = ti * 64 + (wave >> 1) * 32, jb = tj * 64 + (wave & 1) * 32;
    const size_t per = (size_t)n * n;
    const float* src = in + (size_t)b * per;
    floatx4 acc[2][2];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < npad; k0 += 32) {
        const int k = k0 + lg * 8;
        bf16x8 af[2], bfr[2];
        for (int r = 0; r < 2; ++r) {
            const int i = ib + r * 16 + ln;
            uint16_t tmp[8];
            for (int q = 0; q < 8; ++q) {
                const float v = (i < n && k + q < n) ? src[(size_t)i * n + k + q] : 0.f;
                tmp[q] = f2bf_d(v);
            }
            __builtin_memcpy(&af[r], tmp, 16);
        }
        for (int c = 0; c < 2; ++c) {
            const int j = jb + c * 16 + ln;  // < npad by construction of the grid
            bfr[c] = *reinterpret_cast<const bf16x8*>(mat + (size_t)j * npad + k);
        }
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c)
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r], bfr[c], acc[r][c], 0, 0, 0);
    }
    float* dst = out + (size_t)b * per;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            const int j = jb + c * 16 + ln;
            if (j >= n) continue;
            for (int q = 0; q < 4; ++q) {
                const int i = ib + r * 16 + lg * 4 + q;
                if (i >= n) continue;
                float v = acc[r][c][q];
                if (EPI == 1) v *= sqrtf((float)(i > j ? i : j) / (float)n);
                float* o = dst + (size_t)j * n + i;
                if (EPI == 2)
                    *o += v;
                else
                    *o = v;
            }
        }
}

}  // namespace

nmg_status prepare_fprime_bf16(Ctx* c) {
    if (c->dctbf) return NMG_OK;
    std::vector<uint16_t> all;
    c->dctbf_off.clear();
    for (int l = 0; l < c->L; ++l) {
        const int n = c->n[(size_t)l];
        const int npad = (n + 63) / 64 * 64;
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
    const int npad = (n + 63) / 64 * 64;
    const int tiles = npad / 64;
    const uint16_t* C = c->dctbf + c->dctbf_off[(size_t)l];
    const uint16_t* Ct = C + (size_t)npad * npad;
    dim3 grid((unsigned)(tiles * tiles), (unsigned)batch);
    hipLaunchKernelGGL(k_rowgemm_t<0>, grid, dim3(kThreads), 0, s, h, t1, C, n, npad, tiles);
    hipLaunchKernelGGL(k_rowgemm_t<1>, grid, dim3(kThreads), 0, s, t1, t2, C, n, npad, tiles);
    hipLaunchKernelGGL(k_rowgemm_t<0>, grid, dim3(kThreads), 0, s, t2, t1, Ct, n, npad, tiles);
    if (accumulate)
        hipLaunchKernelGGL(k_rowgemm_t<2>, grid, dim3(kThreads), 0, s, t1, dst, Ct, n, npad, tiles);
    else
        hipLaunchKernelGGL(k_rowgemm_t<0>, grid, dim3(kThreads), 0, s, t1, dst, Ct, n, npad, tiles);
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

}  // namespace nmg
