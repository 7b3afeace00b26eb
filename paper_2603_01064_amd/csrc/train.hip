// Level-wise spectral training loss and its hand-written adjoint
// (Sec. 3.2 eq. loss_2_modified, 2D eq. loss_3; training step of
// Algorithm 5).
//
// Forward: y = A e; one pre-smoothing-only cycle from zero records the
// smoother input b_l and output h_l on every level l < L-1
// (x* = 0 on every level, so b_l = y_l), the correction
// hc_l = F'_l(h_l) (or h_l) and y_{l+1} = R(b_l - A_l hc_l).  On the finest
// grid E_l = e - sum_{k<l} I_k^1 hc_k - I_l^1 h_l and
// L_l = (1/B) sum_i || mask_l .* DCT2(E_l) ||^2.
//
// Adjoint (theta_l only; earlier levels are constants):
//   dL_l/dE_l = (2/B) C^T (mask_l^2 .* C E_l C^T) C
//   dL_l/dh_l = -(I_l^1)^T dL_l/dE_l,  (I_{k+1}^k)^T = 2^d R
//   dL_l/dN   = ||b_l|| dL_l/dh_l at the network output
// then the standard convolution / ReLU backward with the activations of the
// level recomputed from b_l / ||b_l||.  Weight gradients are reduced over
// pixels and right-hand sides with fixed-order two-stage sums.
#include <algorithm>
#include <cmath>
#include <vector>

#include "nmg_internal.h"

namespace nmg {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxTaps = 25;
constexpr int kChunk = 4096;  // pixels per weight-gradient partial

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Round to the nearest BF16 value (ties to even), returned as float: the
// rounding the mixed-precision smoother applies to its network input,
// weights and hidden activations.  Finite inputs only.
__device__ __forceinline__ float bf16_round(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}
template <typename T>
__device__ __forceinline__ T maybe_bf16(T v, int bf) {
    return bf ? (T)bf16_round((float)v) : v;
}

// One convolution layer for training: out = act(conv(scale_b * in)), stored
// for every channel (no final ||b|| scaling).  scale_b = 1/sqrt(nrm2[b]) when
// `first` (the input is b), else 1.  bf != 0 repeats the mixed-precision
// forward: the network input b/||b|| and the weights are rounded to BF16,
// products are summed in FP32, and a hidden output is rounded to BF16 after
// its ReLU (so the backward pass differentiates the network whose loss the
// forward reported).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_conv_train(const T* __restrict__ in, T* __restrict__ out,
                                                       const T* __restrict__ W, int cin, int cout, int kh, int kw,
                                                       int ny, int n, int relu, int first,
                                                       const double* __restrict__ nrm2, int bf) {
    const size_t per = (size_t)ny * n;
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    const int co = blockIdx.y, b = blockIdx.z;
    const int y = (int)(e / n), x = (int)(e % n);
    const int py = kh / 2, px = kw / 2;
    const T* src = in + (size_t)b * cin * per;
    const T* w = W + (size_t)co * cin * kh * kw;
    T sc = (T)1;
    if (first) {
        const double nb = sqrt(nrm2[b]);
        sc = nb > 0.0 ? (T)(1.0 / nb) : (T)0;
    }
    T acc = 0;
    for (int ci = 0; ci < cin; ++ci)
        for (int dy = 0; dy < kh; ++dy) {
            const int yy = y + dy - py;
            if (yy < 0 || yy >= ny) continue;
            for (int dx = 0; dx < kw; ++dx) {
                const int xx = x + dx - px;
                if (xx < 0 || xx >= n) continue;
                T v = src[(size_t)ci * per + (size_t)yy * n + xx];
                if (first) v = maybe_bf16(v * sc, bf);
                acc += maybe_bf16(w[(ci * kh + dy) * kw + dx], bf) * v;
            }
        }
    if (relu && acc < (T)0) acc = (T)0;
    if (relu) acc = maybe_bf16(acc, bf);
    out[((size_t)b * cout + co) * per + e] = acc;
}

// Data gradient: din[b][ci][p] = [a_in > 0] * sum_co sum_t W[co][ci][t] dout[b][co][p - off(t)]
// (no ReLU mask when a_in is null: the network input).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_conv_bwd_data(const T* __restrict__ dout, const T* __restrict__ a_in,
                                                          T* __restrict__ din, const T* __restrict__ W, int cin,
                                                          int cout, int kh, int kw, int ny, int n, int bf) {
    const size_t per = (size_t)ny * n;
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= per) return;
    const int ci = blockIdx.y, b = blockIdx.z;
    const size_t idx = ((size_t)b * cin + ci) * per + e;
    if (a_in && !(a_in[idx] > (T)0)) {
        din[idx] = 0;
        return;
    }
    const int y = (int)(e / n), x = (int)(e % n);
    const int py = kh / 2, px = kw / 2;
    T acc = 0;
    for (int co = 0; co < cout; ++co) {
        const T* d = dout + ((size_t)b * cout + co) * per;
        const T* w = W + ((size_t)co * cin + ci) * kh * kw;
        for (int dy = 0; dy < kh; ++dy) {
            const int yy = y - dy + py;
            if (yy < 0 || yy >= ny) continue;
            for (int dx = 0; dx < kw; ++dx) {
                const int xx = x - dx + px;
                if (xx < 0 || xx >= n) continue;
                acc += maybe_bf16(w[dy * kw + dx], bf) * d[(size_t)yy * n + xx];
            }
        }
    }
    din[idx] = acc;
}

// Weight-gradient partials: part[chunk][co][ci][t] = sum over the chunk's
// pixels (b, y, x) of dout[b][co][y][x] * in[b][ci][y+dy-py][x+dx-px]
// (times 1/||b|| for the first layer).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_conv_wgrad(const T* __restrict__ dout, const T* __restrict__ in,
                                                       T* __restrict__ part, int cin, int cout, int kh, int kw,
                                                       int ny, int n, int batch, int first,
                                                       const double* __restrict__ nrm2, int bf) {
    __shared__ T red[kBlock];
    const size_t per = (size_t)ny * n;
    const int co = blockIdx.y, ci = blockIdx.z;
    const int taps = kh * kw;
    const size_t total = (size_t)batch * per;
    const size_t p0 = (size_t)blockIdx.x * kChunk;
    const size_t p1 = p0 + kChunk < total ? p0 + kChunk : total;
    T acc[kMaxTaps];
    for (int t = 0; t < taps; ++t) acc[t] = 0;
    const int py = kh / 2, px = kw / 2;
    for (size_t q = p0 + threadIdx.x; q < p1; q += kBlock) {
        const int b = (int)(q / per);
        const size_t e = q % per;
        const int y = (int)(e / n), x = (int)(e % n);
        const T g = dout[((size_t)b * cout + co) * per + e];
        T sc = (T)1;
        if (first) {
            const double nb = sqrt(nrm2[b]);
            sc = nb > 0.0 ? (T)(1.0 / nb) : (T)0;
        }
        const T* src = in + ((size_t)b * cin + ci) * per;
        for (int dy = 0; dy < kh; ++dy) {
            const int yy = y + dy - py;
            if (yy < 0 || yy >= ny) continue;
            for (int dx = 0; dx < kw; ++dx) {
                const int xx = x + dx - px;
                if (xx < 0 || xx >= n) continue;
                T v = src[(size_t)yy * n + xx];
                if (first) v = maybe_bf16(v * sc, bf);
                acc[dy * kw + dx] += g * v;
            }
        }
    }
    const size_t base = ((size_t)blockIdx.x * cout + co) * cin * taps + (size_t)ci * taps;
    for (int t = 0; t < taps; ++t) {
        red[threadIdx.x] = acc[t];
        __syncthreads();
        for (int s = kBlock / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[base + t] = red[0];
        __syncthreads();
    }
}

// grad[w] (+)= sum_chunk part[chunk][w], fixed order.
template <typename T, typename G>
__global__ void __launch_bounds__(kBlock) k_reduce_chunks(const T* __restrict__ part, G* __restrict__ grad, int count,
                                                          int chunks, int accumulate) {
    const int w = blockIdx.x * kBlock + threadIdx.x;
    if (w >= count) return;
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += (double)part[(size_t)c * count + w];
    grad[w] = accumulate ? (G)((double)grad[w] + acc) : (G)acc;
}

// E = e - acc - P   (elementwise on the finest grid)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_error(const T* __restrict__ e, const T* __restrict__ acc,
                                                  const T* __restrict__ P, T* __restrict__ out, size_t count) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) out[i] = e[i] - acc[i] - P[i];
}

// Masked spectral energy per right-hand side and G = coef * mask^2 * X.
// Level lv (0-based) on the finest grid of N points: p = 2^lv,
// visible <=> kmax p <= N; ramp: sqrt(kmax p / N); band: visible && 2 kmax p > N.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mask_loss(const T* __restrict__ X, T* __restrict__ G,
                                                      double* __restrict__ loss, int N, int two_d, int lv, int ramp,
                                                      T coef) {
    __shared__ double red[kBlock];
    const int b = blockIdx.x;
    const size_t per = (size_t)(two_d ? N : 1) * N;
    const long long p = 1LL << lv;
    double acc = 0.0;
    for (size_t e = threadIdx.x; e < per; e += kBlock) {
        const int i = (int)(e / N), j = (int)(e % N);
        const long long km = two_d ? (i > j ? i : j) : j;
        const bool visible = km * p <= N;
        double m = 0.0;
        if (ramp) {
            if (visible) m = sqrt((double)(km * p) / (double)N);
        } else {
            m = (visible && 2 * km * p > N) ? 1.0 : 0.0;
        }
        const double v = (double)X[(size_t)b * per + e];
        acc += m * m * v * v;
        G[(size_t)b * per + e] = coef * (T)(m * m) * (T)v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[b] = red[0];
}

// out[b][.] = scale * sqrt(nrm2[b]) * in[b][.]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scale_by_norm(const T* __restrict__ in, T* __restrict__ out,
                                                          const double* __restrict__ nrm2, T scale, size_t per) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int b = blockIdx.y;
    if (e >= per) return;
    out[(size_t)b * per + e] = scale * (T)sqrt(nrm2[b]) * in[(size_t)b * per + e];
}

// out = a x + c y (elementwise; out may alias x or y)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_axpby(const T* x, const T* y, T* out, T a, T c, size_t total) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < total) out[e] = a * x[e] + c * y[e];
}

// Per right-hand side b: d1[b] = <u_b, v_b>, d2[b] = <w_b, z_b> in FP64, one
// block per right-hand side with a fixed reduction order.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dot2(const T* __restrict__ u, const T* __restrict__ v,
                                                 const T* __restrict__ w, const T* __restrict__ z,
                                                 double* __restrict__ d1, double* __restrict__ d2, size_t per) {
    __shared__ double s1[kBlock], s2[kBlock];
    const int b = blockIdx.x;
    const size_t o = (size_t)b * per;
    double a1 = 0.0, a2 = 0.0;
    for (size_t e = threadIdx.x; e < per; e += kBlock) {
        a1 += (double)u[o + e] * (double)v[o + e];
        a2 += (double)w[o + e] * (double)z[o + e];
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s1[threadIdx.x] += s1[threadIdx.x + k];
            s2[threadIdx.x] += s2[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d1[b] = s1[0];
        d2[b] = s2[0];
    }
}

// Gradient of the loss with respect to the smoother input b of one level,
// plus the restriction adjoint of the coarser level's gradient:
//   h = ||b|| N(b/||b||), gh = dL/dh, dU = J_N^T (||b|| gh) (network input),
//   dL/db = b (<gh,h>/||b||^2 - <b,dU>/||b||^3) + dU/||b||   (0 when b = 0),
//   out = dL/db + rscale * pg   with pg = P gy_{l+1}, rscale = 2^-d (R^T = P / 2^d).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_input_grad(const T* __restrict__ bv, const T* __restrict__ dU,
                                                       const T* __restrict__ pg, const double* __restrict__ gh_h,
                                                       const double* __restrict__ b_dU,
                                                       const double* __restrict__ nrm2, T* __restrict__ out,
                                                       T rscale, size_t per) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int b = blockIdx.y;
    if (e >= per) return;
    const size_t i = (size_t)b * per + e;
    const double q = nrm2[b];
    T g = 0;
    if (q > 0.0) {
        const double nb = sqrt(q);
        const T cb = (T)(gh_h[b] / q - b_dU[b] / (q * nb));
        g = cb * bv[i] + (T)(1.0 / nb) * dU[i];
    }
    out[i] = g + rscale * pg[i];
}

template <typename G>
__global__ void __launch_bounds__(kBlock) k_adam(float* __restrict__ w, const G* __restrict__ g, float* __restrict__ m,
                                                 float* __restrict__ v, int count, float lr, float b1, float b2,
                                                 float eps, float c1, float c2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    const float gi = (float)g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------
template <typename T>
struct TrainWork {
    bool ready = false;
    std::vector<T*> b, h, hc;   // per level
    std::vector<double*> nrm;   // per level [B]
    T *acc = nullptr, *E = nullptr, *F1 = nullptr, *F2 = nullptr;  // finest grid
    std::vector<T*> acts;       // n_layers - 1 activation buffers [B][cmax][per0]
    T *d0 = nullptr, *d1 = nullptr;  // deltas
    T* part = nullptr;          // weight-gradient partials
    size_t part_count = 0;
    double* lossb = nullptr;    // [B]
    double* dots = nullptr;     // [2B] per-RHS dot products of the cycle-loss adjoint
    T* mf_dout = nullptr;       // MFMA backward: delta at the network output [B][per0]
    uint16_t* mf_wpk = nullptr; // MFMA backward: packed hidden-layer weights
    double* mf_red = nullptr;   // MFMA backward: first stage of the weight-gradient sums
};

template <typename T>
nmg_status talloc(T** p, size_t n) {
    *p = nullptr;
    if (!n) return NMG_OK;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(NMG_ERR_OOM, "hipMalloc failed for training buffers");
    }
    return NMG_OK;
}

struct TrainState {
    TrainWork<double> t64;
    TrainWork<float> t32;
};

}  // namespace

// training state lives beside the context (keyed by pointer)
struct TrainHolder {
    const Ctx* owner;
    TrainState st;
};
static std::vector<TrainHolder*> g_train;

static TrainState& train_state(const Ctx* c) {
    for (auto* t : g_train)
        if (t->owner == c) return t->st;
    auto* t = new TrainHolder{c, {}};
    g_train.push_back(t);
    return t->st;
}

template <typename T>
static void free_train_work(TrainWork<T>& w) {
    auto f = [](auto*& p) {
        if (p) (void)hipFree(p);
        p = nullptr;
    };
    for (auto& p : w.b) f(p);
    for (auto& p : w.h) f(p);
    for (auto& p : w.hc) f(p);
    for (auto& p : w.nrm) f(p);
    for (auto& p : w.acts) f(p);
    f(w.acc);
    f(w.E);
    f(w.F1);
    f(w.F2);
    f(w.d0);
    f(w.d1);
    f(w.part);
    f(w.lossb);
    f(w.dots);
    f(w.mf_dout);
    f(w.mf_wpk);
    f(w.mf_red);
    w.ready = false;
}

void release_training(const Ctx* c) {
    for (size_t i = 0; i < g_train.size(); ++i)
        if (g_train[i]->owner == c) {
            free_train_work(g_train[i]->st.t64);
            free_train_work(g_train[i]->st.t32);
            delete g_train[i];
            g_train.erase(g_train.begin() + (long)i);
            return;
        }
}

template <typename T>
static TrainWork<T>& tw_of(TrainState& s);
template <>
TrainWork<double>& tw_of<double>(TrainState& s) {
    return s.t64;
}
template <>
TrainWork<float>& tw_of<float>(TrainState& s) {
    return s.t32;
}

template <typename T>
static nmg_status ensure_train(const Ctx* c, TrainWork<T>& w) {
    if (w.ready) return NMG_OK;
    const int B = c->p.max_batch, L = c->L;
    const int nsm = std::max(1, L - 1);
    w.b.assign((size_t)nsm, nullptr);
    w.h.assign((size_t)nsm, nullptr);
    w.hc.assign((size_t)nsm, nullptr);
    w.nrm.assign((size_t)nsm, nullptr);
    for (int l = 0; l < nsm; ++l) {
        const size_t cnt = (size_t)B * level_elems(c, l);
        NMG_TRY(talloc(&w.b[(size_t)l], cnt));
        NMG_TRY(talloc(&w.h[(size_t)l], cnt));
        NMG_TRY(talloc(&w.hc[(size_t)l], cnt));
        NMG_TRY(talloc(&w.nrm[(size_t)l], (size_t)B));
    }
    const size_t fine = (size_t)B * level_elems(c, 0);
    NMG_TRY(talloc(&w.acc, fine));
    NMG_TRY(talloc(&w.E, fine));
    NMG_TRY(talloc(&w.F1, fine));
    NMG_TRY(talloc(&w.F2, fine));
    const size_t act = (size_t)B * c->cmax * level_elems(c, 0);
    w.acts.assign((size_t)std::max(1, c->p.n_layers - 1), nullptr);
    for (auto& a : w.acts) NMG_TRY(talloc(&a, act));
    NMG_TRY(talloc(&w.d0, act));
    NMG_TRY(talloc(&w.d1, act));
    const size_t chunks = (fine + kChunk - 1) / kChunk;
    size_t maxlayer = 0;
    for (int i = 0; i < c->p.n_layers; ++i) {
        const int kk = c->p.dim == 2 ? c->p.ksize * c->p.ksize : c->p.ksize;
        maxlayer = std::max(maxlayer, (size_t)c->p.channels[i] * c->p.channels[i + 1] * kk);
    }
    w.part_count = chunks * maxlayer;
    // the MFMA backward's 32 -> 32 weight gradient keeps up to four partials
    // of maxlayer values per image
    if (std::is_same<T, float>::value && mfma_backward_supported(c))
        w.part_count = std::max(w.part_count, (size_t)B * 4 * maxlayer);
    NMG_TRY(talloc(&w.part, w.part_count));
    NMG_TRY(talloc(&w.lossb, (size_t)B));
    NMG_TRY(talloc(&w.dots, (size_t)2 * B));
    if (std::is_same<T, float>::value && mfma_backward_supported(c)) {
        NMG_TRY(talloc(&w.mf_dout, fine));
        NMG_TRY(talloc(&w.mf_wpk, mfma_backward_wpk_elems(c)));
        NMG_TRY(talloc(&w.mf_red, mfma_backward_reduce_elems()));
    }
    w.ready = true;
    return NMG_OK;
}

// Prolongation chain I_l^1 v: from level l down to the finest level; the
// result lands in `out` (finest grid).  Uses the level buffers x of `work`.
template <typename T>
static nmg_status prolong_chain(const Ctx* c, Work<T>& work, int l, int batch, const T* v, T* out, hipStream_t s) {
    if (l == 0) return launch_axpy<T>(batch, level_elems(c, 0), v, out, 0, s);
    const T* cur = v;
    for (int k = l - 1; k >= 0; --k) {
        T* dst = k == 0 ? out : work.lv[(size_t)k].x;
        NMG_TRY(launch_zero<T>(dst, (size_t)batch * level_elems(c, k), s));
        NMG_TRY(launch_prolong_add<T>(c, k, batch, cur, dst, s));
        cur = dst;
    }
    return NMG_OK;
}

// (I_l^1)^T g: from the finest level up to level l; result in work.lv[l].y
// (or a copy of g when l == 0).
template <typename T>
static nmg_status prolong_chain_T(const Ctx* c, Work<T>& work, int l, int batch, const T* g, T* out, hipStream_t s) {
    if (l == 0) return launch_axpy<T>(batch, level_elems(c, 0), g, out, 0, s);
    const T* cur = g;
    for (int k = 0; k < l; ++k) {
        T* dst = k == l - 1 ? out : work.lv[(size_t)k + 1].y;
        NMG_TRY(launch_prolong_transpose<T>(c, k, batch, cur, dst, s));
        cur = dst;
    }
    return NMG_OK;
}

template <typename T>
static T* grad_ptr(Ctx* c, int l, int set);
template <>
double* grad_ptr<double>(Ctx* c, int l, int set) {
    return c->g64 + ((size_t)l * c->p.n_weight_sets + set) * c->wcount;
}
template <>
float* grad_ptr<float>(Ctx* c, int l, int set) {
    return c->g32 + ((size_t)l * c->p.n_weight_sets + set) * c->wcount;
}

// bf != 0: the network of the mixed-precision forward (BF16 operands, FP32
// sums; see k_conv_train), differentiated through its roundings as if they
// were the identity.
template <typename T>
static nmg_status smoother_backward(Ctx* c, Work<T>& work, TrainWork<T>& tw, int l, int set, int batch,
                                    const T* upstream, T sign, int accumulate, hipStream_t s, T* din0 = nullptr,
                                    int bf = 0) {
    const int n = c->n[(size_t)l];
    const int ny = c->p.dim == 2 ? n : 1;
    const int kh = c->p.dim == 2 ? c->p.ksize : 1, kw = c->p.ksize;
    const size_t per = (size_t)ny * n;
    const int NL = c->p.n_layers;
    const T* Wbase = work.wts + ((size_t)l * c->p.n_weight_sets + set) * c->wcount;
    T* gbase = grad_ptr<T>(c, l, set);
    const double* nrm2 = tw.nrm[(size_t)l];
    if constexpr (std::is_same<T, float>::value) {
        if (bf && tw.mf_dout && mfma_backward_supported(c)) {
            // BF16 activations and deltas on MFMA
            hipLaunchKernelGGL(k_scale_by_norm<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, upstream,
                               tw.mf_dout, nrm2, sign, per);
            MfmaBackwardArgs a;
            a.n = n;
            a.batch = batch;
            a.accumulate = accumulate;
            a.b = tw.b[(size_t)l];
            a.nrm2 = nrm2;
            a.W = Wbase;
            a.grad = gbase;
            a.dout = tw.mf_dout;
            a.din0 = din0;
            for (auto* p : tw.acts) a.acts.push_back(reinterpret_cast<uint16_t*>(p));
            a.d0 = reinterpret_cast<uint16_t*>(tw.d0);
            a.d1 = reinterpret_cast<uint16_t*>(tw.d1);
            a.wpk = tw.mf_wpk;
            a.part = tw.part;
            a.part_count = tw.part_count;
            a.reduce_tmp = tw.mf_red;
            return smoother_backward_mfma(c, a, s);
        }
    }
    // recompute activations a_1 .. a_{NL-1}
    const T* src = tw.b[(size_t)l];
    for (int i = 0; i + 1 < NL; ++i) {
        const int cin = c->p.channels[i], cout = c->p.channels[i + 1];
        hipLaunchKernelGGL(k_conv_train<T>, dim3(blocks_for(per), cout, batch), dim3(kBlock), 0, s, src,
                           tw.acts[(size_t)i], Wbase + c->layer_off[(size_t)i], cin, cout, kh, kw, ny, n, 1,
                           i == 0 ? 1 : 0, nrm2, bf);
        src = tw.acts[(size_t)i];
    }
    // delta at the network output: sign * ||b|| * upstream
    hipLaunchKernelGGL(k_scale_by_norm<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, upstream, tw.d0, nrm2,
                       sign, per);
    T* dcur = tw.d0;
    T* dnext = tw.d1;
    const size_t total = (size_t)batch * per;
    const int chunks = (int)((total + kChunk - 1) / kChunk);
    for (int i = NL - 1; i >= 0; --i) {
        const int cin = c->p.channels[i], cout = c->p.channels[i + 1];
        const T* in = i == 0 ? tw.b[(size_t)l] : tw.acts[(size_t)i - 1];
        const int cnt = cin * cout * kh * kw;
        hipLaunchKernelGGL(k_conv_wgrad<T>, dim3(chunks, cout, cin), dim3(kBlock), 0, s, dcur, in, tw.part, cin, cout,
                           kh, kw, ny, n, batch, i == 0 ? 1 : 0, nrm2, bf);
        hipLaunchKernelGGL((k_reduce_chunks<T, T>), dim3((cnt + kBlock - 1) / kBlock), dim3(kBlock), 0, s, tw.part,
                           gbase + c->layer_off[(size_t)i], cnt, chunks, accumulate);
        if (i > 0) {
            hipLaunchKernelGGL(k_conv_bwd_data<T>, dim3(blocks_for(per), cin, batch), dim3(kBlock), 0, s, dcur,
                               tw.acts[(size_t)i - 1], dnext, Wbase + c->layer_off[(size_t)i], cin, cout, kh, kw, ny,
                               n, bf);
            std::swap(dcur, dnext);
        } else if (din0) {  // gradient at the network input u = b / ||b||
            hipLaunchKernelGGL(k_conv_bwd_data<T>, dim3(blocks_for(per), cin, batch), dim3(kBlock), 0, s, dcur,
                               (const T*)nullptr, din0, Wbase + c->layer_off[0], cin, cout, kh, kw, ny, n, bf);
        }
    }
    NMG_HIP(hipGetLastError());
    return NMG_OK;
}

// backward = false evaluates the losses only (nmg_loss_forward).
template <typename T>
nmg_status loss_grad_impl(Ctx* c, Work<T>& work, int set, int batch, const double* alpha, const T* e, int mask,
                          int use_fprime, bool mixed, int zero_grad, double* losses_host, hipStream_t s,
                          bool backward = true) {
    TrainState& ts = train_state(c);
    TrainWork<T>& tw = tw_of<T>(ts);
    NMG_TRY(ensure_train<T>(c, tw));
    if (!mixed || c->p.smoother_arch == NMG_ARCH_FNO) NMG_TRY(ensure_acts<T>(c));
    const int L = c->L;
    const int nsm = L - 1;
    const int N = c->n[0];
    const int two_d = c->p.dim == 2 ? 1 : 0;
    const size_t per0 = level_elems(c, 0);
    const size_t fine = (size_t)batch * per0;
    std::vector<int> wsv((size_t)batch, set);
    int* ws_dev = c->active;  // reuse the [max_batch] int scratch for the weight-set index
    NMG_HIP(hipMemcpyAsync(ws_dev, wsv.data(), (size_t)batch * sizeof(int), hipMemcpyHostToDevice, s));
    // ---- forward cycle (pre-smoothing only, from zero)
    NMG_TRY(launch_operator<T>(c, 0, batch, alpha, e, nullptr, tw.b[0], 1, work, s));
    for (int l = 0; l < nsm; ++l) {
        const size_t per = level_elems(c, l);
        NMG_TRY(launch_sumsq<T>(c, batch, per, tw.b[(size_t)l], tw.nrm[(size_t)l], s));
        if (c->p.smoother_arch == NMG_ARCH_FNO) {
            NMG_TRY(launch_fno_smoother<T>(c, l, batch, ws_dev, tw.b[(size_t)l], tw.nrm[(size_t)l], tw.h[(size_t)l], 0,
                                           work, s));
        } else if (mixed) {
            NMG_TRY(launch_mfma_smoother(c, l, batch, ws_dev, reinterpret_cast<const float*>(tw.b[(size_t)l]),
                                         tw.nrm[(size_t)l], 0, reinterpret_cast<float*>(tw.h[(size_t)l]), 0,
                                         *reinterpret_cast<Work<float>*>(&work), s));
        } else {
            NMG_TRY(launch_conv_smoother<T>(c, l, batch, ws_dev, tw.b[(size_t)l], tw.nrm[(size_t)l], tw.h[(size_t)l],
                                            0, work, s));
        }
        const T* hc = tw.h[(size_t)l];
        if (use_fprime) {
            NMG_TRY(launch_fprime<T>(c, l, batch, tw.h[(size_t)l], tw.hc[(size_t)l], 0, work, s));
            hc = tw.hc[(size_t)l];
        }
        if (l + 1 < nsm) {
            NMG_TRY(launch_operator<T>(c, l, batch, alpha, hc, tw.b[(size_t)l], work.lv[(size_t)l].b, 0, work, s));
            NMG_TRY(launch_restrict<T>(c, l, batch, work.lv[(size_t)l].b, tw.b[(size_t)l + 1], s));
        }
    }
    // ---- per-level losses on the finest grid and the adjoint
    const T* C = work.dct + work.dct_off[0];
    NMG_TRY(launch_zero<T>(tw.acc, fine, s));
    std::vector<double> lossb((size_t)batch);
    for (int l = 0; l < nsm; ++l) {
        NMG_TRY(prolong_chain<T>(c, work, l, batch, tw.h[(size_t)l], tw.F1, s));
        hipLaunchKernelGGL(k_error<T>, dim3(blocks_for(fine)), dim3(kBlock), 0, s, e, tw.acc, tw.F1, tw.E, fine);
        // X = C E C^T
        NMG_TRY(launch_dense_axis<T>(tw.E, tw.F1, C, N, two_d ? N : 1, batch, 0, 0, s));
        const T* X = tw.F1;
        if (two_d) {
            NMG_TRY(launch_dense_axis<T>(tw.F1, tw.F2, C, N, N, batch, 1, 0, s));
            X = tw.F2;
        }
        T* G = two_d ? tw.F1 : tw.F2;
        hipLaunchKernelGGL(k_mask_loss<T>, dim3(batch), dim3(kBlock), 0, s, X, G, tw.lossb, N, two_d, l,
                           mask == NMG_MASK_RAMP ? 1 : 0, (T)(2.0 / batch));
        if (backward) {
            // gE = C^T G C
            T* gE = tw.E;
            if (two_d) {
                NMG_TRY(launch_dense_axis<T>(G, tw.F2, C, N, N, batch, 0, 1, s));
                NMG_TRY(launch_dense_axis<T>(tw.F2, gE, C, N, N, batch, 1, 1, s));
            } else {
                NMG_TRY(launch_dense_axis<T>(G, gE, C, N, 1, batch, 0, 1, s));
            }
            // g_h = (I_l^1)^T gE; dL/dh_l = -g_h, so the network-output delta is -||b_l|| g_h
            T* gh = work.lv[(size_t)l].h;
            NMG_TRY(prolong_chain_T<T>(c, work, l, batch, gE, gh, s));
            if (c->p.smoother_arch == NMG_ARCH_FNO)
                NMG_TRY(fno_backward<T>(c, work, l, set, batch, tw.b[(size_t)l], tw.nrm[(size_t)l], gh, (T)(-1),
                                        zero_grad ? 0 : 1, grad_ptr<T>(c, l, set), s));
            else
                NMG_TRY(smoother_backward<T>(c, work, tw, l, set, batch, gh, (T)(-1), zero_grad ? 0 : 1, s, nullptr,
                                             mixed ? 1 : 0));
        }
        // accumulate the correction of this level on the finest grid
        const T* hc = use_fprime ? tw.hc[(size_t)l] : tw.h[(size_t)l];
        NMG_TRY(prolong_chain<T>(c, work, l, batch, hc, tw.F1, s));
        NMG_TRY(launch_axpy<T>(batch, per0, tw.F1, tw.acc, 1, s));
        NMG_HIP(hipMemcpyAsync(lossb.data(), tw.lossb, (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, s));
        NMG_HIP(hipStreamSynchronize(s));
        double tot = 0.0;
        for (int b = 0; b < batch; ++b) tot += lossb[(size_t)b];
        if (losses_host) losses_host[l] = tot / batch;
    }
    return NMG_OK;
}

// losses_host[0] = (1/B) sum_b ||E_b||^2 of the combined loss, the other
// entries 0 (synchronises).
template <typename T>
static nmg_status finish_cycle_loss(const Ctx*, TrainWork<T>& tw, int batch, int nsm, double* losses_host,
                                    hipStream_t s) {
    std::vector<double> lossb((size_t)batch);
    NMG_HIP(hipMemcpyAsync(lossb.data(), tw.lossb, (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, s));
    NMG_HIP(hipStreamSynchronize(s));
    if (losses_host) {
        double total = 0.0;
        for (int b = 0; b < batch; ++b) total += lossb[(size_t)b];
        losses_host[0] = total / batch;
        for (int l = 1; l < nsm; ++l) losses_host[l] = 0.0;
    }
    return NMG_OK;
}

// Combined loss of the whole cycle (Sec. 3.2 eq. loss_1) and its joint
// gradient over every level.  Forward (levels 0-based, L-1 the coarsest):
//   y_0 = A e;  h_l = S_l(y_l), hc_l = F'_l(h_l) or h_l;
//   y_{l+1} = R(y_l - A_l hc_l);  x_c = A_{L-1}^{-1} y_{L-1};
//   x = sum_l I_l^0 hc_l + I_{L-1}^0 x_c;  L = (1/B) sum_i ||e_i - x_i||^2.
// Adjoint: g_0 = -(2/B)(e - x), g_{l+1} = P^T g_l (gradient of each level's
// output), gy_{L-1} = A_{L-1}^{-1} g_{L-1}, then for l = L-2 .. 0:
//   dL/dhc_l = g_l - A_l R^T gy_{l+1}       (hc_l also feeds y_{l+1})
//   dL/dh_l  = F'_l(dL/dhc_l) or the same    (F'_l is symmetric)
//   theta_l gradient from dL/dh_l (network backward)
//   gy_l     = J_{S_l}^T dL/dh_l + R^T gy_{l+1}   (y_l feeds h_l and y_{l+1})
// with R^T = P / 2^d.  A_l and A_{L-1}^{-1} are symmetric.
template <typename T>
nmg_status cycle_loss_impl(Ctx* c, Work<T>& work, int set, int batch, const double* alpha, const T* e,
                           int use_fprime, bool mixed, int zero_grad, double* losses_host, hipStream_t s,
                           bool backward = true) {
    TrainState& ts = train_state(c);
    TrainWork<T>& tw = tw_of<T>(ts);
    NMG_TRY(ensure_train<T>(c, tw));
    if (!mixed || c->p.smoother_arch == NMG_ARCH_FNO) NMG_TRY(ensure_acts<T>(c));
    NMG_TRY(nmg_prepare(static_cast<nmg_handle>(c), batch, alpha, s));  // coarse factors of these alphas
    const int L = c->L;
    const int nsm = L - 1;
    const int two_d = c->p.dim == 2 ? 1 : 0;
    const T rscale = (T)(two_d ? 0.25 : 0.5);
    const size_t per0 = level_elems(c, 0);
    const size_t fine = (size_t)batch * per0;
    std::vector<int> wsv((size_t)batch, set);
    int* ws_dev = c->active;
    NMG_HIP(hipMemcpyAsync(ws_dev, wsv.data(), (size_t)batch * sizeof(int), hipMemcpyHostToDevice, s));
    LevelBuffers<T>& coarse = work.lv[(size_t)nsm];
    auto coarse_solve = [&](const T* y, T* x) -> nmg_status {
        if (c->eig_coarse) return launch_eig_coarse<T>(c, batch, alpha, y, x, s);
        if (std::is_same<T, double>::value) return launch_coarse_solve<T>(c, batch, y, x, s);
        return launch_coarse_apply_inverse<T>(c, batch, y, x, s);
    };
    // ---- forward
    NMG_TRY(launch_operator<T>(c, 0, batch, alpha, e, nullptr, tw.b[0], 1, work, s));
    for (int l = 0; l < nsm; ++l) {
        const size_t per = level_elems(c, l);
        NMG_TRY(launch_sumsq<T>(c, batch, per, tw.b[(size_t)l], tw.nrm[(size_t)l], s));
        if (c->p.smoother_arch == NMG_ARCH_FNO) {
            NMG_TRY(launch_fno_smoother<T>(c, l, batch, ws_dev, tw.b[(size_t)l], tw.nrm[(size_t)l], tw.h[(size_t)l], 0,
                                           work, s));
        } else if (mixed) {
            NMG_TRY(launch_mfma_smoother(c, l, batch, ws_dev, reinterpret_cast<const float*>(tw.b[(size_t)l]),
                                         tw.nrm[(size_t)l], 0, reinterpret_cast<float*>(tw.h[(size_t)l]), 0,
                                         *reinterpret_cast<Work<float>*>(&work), s));
        } else {
            NMG_TRY(launch_conv_smoother<T>(c, l, batch, ws_dev, tw.b[(size_t)l], tw.nrm[(size_t)l], tw.h[(size_t)l],
                                            0, work, s));
        }
        T* hc = tw.h[(size_t)l];
        if (use_fprime) {
            NMG_TRY(launch_fprime<T>(c, l, batch, tw.h[(size_t)l], tw.hc[(size_t)l], 0, work, s));
            hc = tw.hc[(size_t)l];
        }
        T* ynext = l + 1 < nsm ? tw.b[(size_t)l + 1] : coarse.y;
        NMG_TRY(launch_operator<T>(c, l, batch, alpha, hc, tw.b[(size_t)l], work.lv[(size_t)l].b, 0, work, s));
        NMG_TRY(launch_restrict<T>(c, l, batch, work.lv[(size_t)l].b, ynext, s));
    }
    NMG_TRY(coarse_solve(coarse.y, coarse.x));
    NMG_TRY(launch_zero<T>(tw.acc, fine, s));
    for (int l = 0; l < nsm; ++l) {
        NMG_TRY(prolong_chain<T>(c, work, l, batch, use_fprime ? tw.hc[(size_t)l] : tw.h[(size_t)l], tw.F1, s));
        NMG_TRY(launch_axpy<T>(batch, per0, tw.F1, tw.acc, 1, s));
    }
    NMG_TRY(prolong_chain<T>(c, work, nsm, batch, coarse.x, tw.F1, s));
    hipLaunchKernelGGL(k_error<T>, dim3(blocks_for(fine)), dim3(kBlock), 0, s, e, tw.acc, tw.F1, tw.E, fine);
    NMG_TRY(launch_sumsq<T>(c, batch, per0, tw.E, tw.lossb, s));
    if (!backward) return finish_cycle_loss(c, tw, batch, nsm, losses_host, s);
    // ---- adjoint
    auto gbuf = [&](int l) -> T* { return l == 0 ? tw.E : (l < nsm ? tw.hc[(size_t)l] : coarse.y); };
    hipLaunchKernelGGL(k_axpby<T>, dim3(blocks_for(fine)), dim3(kBlock), 0, s, tw.E, tw.E, tw.E,
                       (T)(-2.0 / batch), (T)0, fine);
    for (int l = 0; l < nsm; ++l) NMG_TRY(launch_prolong_transpose<T>(c, l, batch, gbuf(l), gbuf(l + 1), s));
    NMG_TRY(coarse_solve(coarse.y, coarse.x));  // gy_{L-1}
    for (int l = nsm - 1; l >= 0; --l) {
        const size_t per = level_elems(c, l);
        const size_t tot = (size_t)batch * per;
        LevelBuffers<T>& lb = work.lv[(size_t)l];
        const T* gy_next = work.lv[(size_t)l + 1].x;
        NMG_TRY(launch_zero<T>(lb.b, tot, s));
        NMG_TRY(launch_prolong_add<T>(c, l, batch, gy_next, lb.b, s));                  // pg = P gy_{l+1}
        NMG_TRY(launch_operator<T>(c, l, batch, alpha, lb.b, nullptr, lb.h, 1, work, s));  // A_l pg
        T* ghc = gbuf(l);
        hipLaunchKernelGGL(k_axpby<T>, dim3(blocks_for(tot)), dim3(kBlock), 0, s, ghc, lb.h, ghc, (T)1, -rscale,
                           tot);
        const T* gh = ghc;
        if (use_fprime) {
            NMG_TRY(launch_fprime<T>(c, l, batch, ghc, lb.h, 0, work, s));
            gh = lb.h;
        }
        NMG_TRY(smoother_backward<T>(c, work, tw, l, set, batch, gh, (T)1, zero_grad ? 0 : 1, s,
                                     l > 0 ? tw.F1 : nullptr, mixed ? 1 : 0));
        if (l > 0) {
            hipLaunchKernelGGL(k_dot2<T>, dim3(batch), dim3(kBlock), 0, s, gh, tw.h[(size_t)l], tw.b[(size_t)l],
                               tw.F1, tw.dots, tw.dots + batch, per);
            hipLaunchKernelGGL(k_input_grad<T>, dim3(blocks_for(per), batch), dim3(kBlock), 0, s, tw.b[(size_t)l],
                               tw.F1, lb.b, tw.dots, tw.dots + batch, tw.nrm[(size_t)l], lb.x, rscale, per);
        }
    }
    NMG_HIP(hipGetLastError());
    return finish_cycle_loss(c, tw, batch, nsm, losses_host, s);
}

}  // namespace nmg

using namespace nmg;

namespace {

nmg_status check_training(nmg_handle h, int set, int batch, nmg_mask_kind mask, nmg_precision prec) {
    if (!h) return fail(NMG_ERR_ARG, "null handle");
    if (h->L < 2) return fail(NMG_ERR_SHAPE, "training needs at least two levels");
    if (h->p.smoother_arch == NMG_ARCH_FNO) {
        if (mask == NMG_LOSS_CYCLE) return fail(NMG_ERR_STATE, "the combined loss supports the CNN smoother only");
        const int kk = h->p.dim == 2 ? h->p.fno_ksize * h->p.fno_ksize : h->p.fno_ksize;
        if (kk > 49) return fail(NMG_ERR_SHAPE, "FNO training supports convolutions of at most 49 taps");
    }
    if (batch < 1 || batch > h->p.max_batch) return fail(NMG_ERR_SHAPE, "batch must be in [1, max_batch]");
    if (set < 0 || set >= h->p.n_weight_sets) return fail(NMG_ERR_ARG, "weight_set out of range");
    if (mask != NMG_MASK_BAND && mask != NMG_MASK_RAMP && mask != NMG_LOSS_CYCLE)
        return fail(NMG_ERR_ARG, "unknown loss kind");
    if (prec != NMG_FP64 && prec != NMG_FP32 && prec != NMG_MIXED) return fail(NMG_ERR_ARG, "unknown precision");
    const int kk = h->p.dim == 2 ? h->p.ksize * h->p.ksize : h->p.ksize;
    if (kk > kMaxTaps) return fail(NMG_ERR_SHAPE, "training supports at most 25 taps per kernel");
    for (int l = 0; l + 1 < h->L; ++l)
        if (h->kind[(size_t)l] != 0 || !h->loaded[(size_t)l][(size_t)set])
            return fail(NMG_ERR_STATE, "every level needs neural weights of this set before training");
    return NMG_OK;
}

}  // namespace

extern "C" {

nmg_status nmg_loss_grad(nmg_handle h, int set, int batch, const double* alpha, const void* e, nmg_mask_kind mask,
                         int use_fprime, nmg_precision prec, int zero_grad, double* losses_host, void* stream) {
    NMG_TRY(check_training(h, set, batch, mask, prec));
    if (!alpha || !e) return fail(NMG_ERR_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    if (prec == NMG_FP64) {
        NMG_TRY(ensure_work<double>(h));
        if (mask == NMG_LOSS_CYCLE)
            NMG_TRY(cycle_loss_impl<double>(h, h->w64, set, batch, alpha, (const double*)e, use_fprime, false,
                                            zero_grad, losses_host, s));
        else
            NMG_TRY(loss_grad_impl<double>(h, h->w64, set, batch, alpha, (const double*)e, mask, use_fprime, false,
                                           zero_grad, losses_host, s));
        h->grad_is_fp64 = true;
        return NMG_OK;
    }
    NMG_TRY(ensure_work<float>(h));
    if (mask == NMG_LOSS_CYCLE)
        NMG_TRY(cycle_loss_impl<float>(h, h->w32b, set, batch, alpha, (const float*)e, use_fprime,
                                       prec == NMG_MIXED, zero_grad, losses_host, s));
    else
        NMG_TRY(loss_grad_impl<float>(h, h->w32b, set, batch, alpha, (const float*)e, mask, use_fprime,
                                      prec == NMG_MIXED, zero_grad, losses_host, s));
    h->grad_is_fp64 = false;
    return NMG_OK;
}

nmg_status nmg_loss_forward(nmg_handle h, int set, int batch, const double* alpha, const void* e,
                            nmg_mask_kind mask, int use_fprime, nmg_precision prec, double* losses_host,
                            void* stream) {
    NMG_TRY(check_training(h, set, batch, mask, prec));
    if (!alpha || !e) return fail(NMG_ERR_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    if (prec == NMG_FP64) {
        NMG_TRY(ensure_work<double>(h));
        if (mask == NMG_LOSS_CYCLE)
            return cycle_loss_impl<double>(h, h->w64, set, batch, alpha, (const double*)e, use_fprime, false, 0,
                                           losses_host, s, false);
        return loss_grad_impl<double>(h, h->w64, set, batch, alpha, (const double*)e, mask, use_fprime, false, 0,
                                      losses_host, s, false);
    }
    NMG_TRY(ensure_work<float>(h));
    if (mask == NMG_LOSS_CYCLE)
        return cycle_loss_impl<float>(h, h->w32b, set, batch, alpha, (const float*)e, use_fprime, prec == NMG_MIXED,
                                      0, losses_host, s, false);
    return loss_grad_impl<float>(h, h->w32b, set, batch, alpha, (const float*)e, mask, use_fprime, prec == NMG_MIXED,
                                 0, losses_host, s, false);
}

nmg_status nmg_get_gradient(nmg_handle h, int level, int set, double* grad_host, size_t count) {
    if (!h || !grad_host) return fail(NMG_ERR_ARG, "null argument");
    if (level < 0 || level >= h->L - 1) return fail(NMG_ERR_ARG, "level must be in [0, L-2]");
    if (set < 0 || set >= h->p.n_weight_sets) return fail(NMG_ERR_ARG, "weight_set out of range");
    if (count != (size_t)h->wcount) return fail(NMG_ERR_SHAPE, "gradient count mismatch");
    NMG_HIP(hipDeviceSynchronize());
    const size_t off = ((size_t)level * h->p.n_weight_sets + set) * h->wcount;
    if (h->grad_is_fp64) {
        NMG_HIP(hipMemcpy(grad_host, h->g64 + off, count * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(count);
        NMG_HIP(hipMemcpy(tmp.data(), h->g32 + off, count * sizeof(float), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < count; ++i) grad_host[i] = tmp[i];
    }
    return NMG_OK;
}

nmg_status nmg_adam_step(nmg_handle h, int set, double lr, double beta1, double beta2, double eps, void* stream) {
    if (!h) return fail(NMG_ERR_ARG, "null handle");
    if (set < 0 || set >= h->p.n_weight_sets) return fail(NMG_ERR_ARG, "weight_set out of range");
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(NMG_ERR_ARG, "invalid Adam hyper-parameters");
    hipStream_t s = (hipStream_t)stream;
    const int t = ++h->adam_step[(size_t)set];
    const float c1 = (float)(1.0 - std::pow(beta1, t)), c2 = (float)(1.0 - std::pow(beta2, t));
    const int cnt = h->wcount;
    for (int l = 0; l + 1 < h->L; ++l) {
        const size_t off = ((size_t)l * h->p.n_weight_sets + set) * cnt;
        dim3 grid((unsigned)((cnt + kBlock - 1) / kBlock));
        if (h->grad_is_fp64)
            hipLaunchKernelGGL(k_adam<double>, grid, dim3(kBlock), 0, s, h->w32 + off, h->g64 + off, h->adam_m + off,
                               h->adam_v + off, cnt, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
        else
            hipLaunchKernelGGL(k_adam<float>, grid, dim3(kBlock), 0, s, h->w32 + off, h->g32 + off, h->adam_m + off,
                               h->adam_v + off, cnt, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
        NMG_HIP(hipGetLastError());
        if (h->w64.ready) NMG_TRY(launch_convert<float, double>(h->w32 + off, h->w64.wts + off, (size_t)cnt, s));
    }
    NMG_HIP(hipStreamSynchronize(s));
    for (int l = 0; l + 1 < h->L; ++l) NMG_TRY(repack_bf16(h, l, set));
    return NMG_OK;
}

nmg_status nmg_train_step(nmg_handle h, int set, int batch, const double* alpha, const void* e, nmg_mask_kind mask,
                          int use_fprime, nmg_precision prec, double lr, double* losses_host, void* stream) {
    NMG_TRY(nmg_loss_grad(h, set, batch, alpha, e, mask, use_fprime, prec, 1, losses_host, stream));
    return nmg_adam_step(h, set, lr, 0.9, 0.999, 1e-8, stream);
}

}  // extern "C"
