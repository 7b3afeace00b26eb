// C ABI entry points: hierarchy setup, weights, the V-cycle and the solve.
//
// The cycle follows Algorithm 1 with the neural smoothing step of
// Algorithms 2-4: on each level above the coarsest, nu1 times
//   b = y - A x ;  h = ||b|| N(b/||b||) ;  x += F'(h)  (F' optional)
// then restriction of y - A x, a recursive cycle from zero on the next
// level, interpolation and correction, and nu2 post-smoothing steps with
// the same smoother; the coarsest level is solved exactly by Cholesky.
// The recursion is unrolled on the host into a fixed launch sequence.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "nmg_internal.h"

namespace nmg {

namespace {
thread_local std::string g_last_error;

template <typename T>
nmg_status dev_alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return NMG_OK;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(NMG_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return NMG_OK;
}

template <typename T>
void dev_free(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace

nmg_status fail(nmg_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

nmg_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "HIP error %s (%d) in %s at %s:%d", hipGetErrorString(e), (int)e, what, file,
                  line);
    g_last_error = buf;
    return NMG_ERR_HIP;
}

static hipEvent_t prof_event(Ctx* c) {
    if (!c->prof_pool.empty()) {
        hipEvent_t e = c->prof_pool.back();
        c->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

ProfScope::ProfScope(const Ctx* cc, hipStream_t ss, int k, int l) : c(const_cast<Ctx*>(cc)), s(ss), kind(k), level(l) {
    if (!(c->prof_mask & (1 << k)) || !(c->prof_levels & (1 << (l < 0 ? 0 : (l > 15 ? 15 : l))))) return;
    if (c->capturing) {
        // graph node timing: wall-clock stamps (events cannot be timed inside graphs)
        if (!c->stamps || c->stamp_next + 2 > kStampSlots) return;
        stamp = c->stamp_next;
        c->stamp_next += 2;
        launch_stamp(c->stamps + stamp, s);
        return;
    }
    a = prof_event(c);
    b = prof_event(c);
    if (a && b) (void)hipEventRecord(a, s);
}

ProfScope::~ProfScope() {
    if (stamp >= 0) {
        launch_stamp(c->stamps + stamp + 1, s);
        c->capture_stamps.push_back({stamp, kind, level});
        return;
    }
    if (!a || !b) return;
    (void)hipEventRecord(b, s);
    c->prof_pending.push_back({a, b, kind, level});
}

nmg_status prof_resolve(Ctx* c) {
    for (auto& ev : c->prof_pending) {
        NMG_HIP(hipEventSynchronize(ev.b));
        float ms = 0.f;
        NMG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        const int k = ev.kind & 7, l = ev.level < 0 ? 0 : (ev.level > 15 ? 15 : ev.level);
        c->prof_ms[k][l] += ms;
        c->prof_cnt[k][l] += 1;
        c->prof_pool.push_back(ev.a);
        c->prof_pool.push_back(ev.b);
    }
    c->prof_pending.clear();
    if (!c->stamp_pending.empty()) {
        std::vector<long long> st((size_t)c->stamp_next);
        NMG_HIP(hipDeviceSynchronize());
        NMG_HIP(hipMemcpy(st.data(), c->stamps, st.size() * sizeof(long long), hipMemcpyDeviceToHost));
        for (auto& e : c->stamp_pending) {
            const double ms = (double)(st[(size_t)e.first + 1] - st[(size_t)e.first]) / c->wall_khz;
            const int k = e.kind & 7, l = e.level < 0 ? 0 : (e.level > 15 ? 15 : e.level);
            c->prof_ms[k][l] += ms;
            c->prof_cnt[k][l] += 1;
        }
        c->stamp_pending.clear();
    }
    return NMG_OK;
}

void release_graphs(Ctx* c) {
    for (auto& kv : c->graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    c->graphs.clear();
    c->stamp_pending.clear();
    c->stamp_next = 0;
}

namespace {

// Orthonormal DCT-II of size n: C[k][i] = c_k cos(pi k (2 i + 1) / (2 n)).
std::vector<double> dct2(int n) {
    std::vector<double> C((size_t)n * n);
    for (int k = 0; k < n; ++k) {
        const double ck = k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
        for (int i = 0; i < n; ++i) C[(size_t)k * n + i] = ck * std::cos(M_PI * k * (2.0 * i + 1.0) / (2.0 * n));
    }
    return C;
}

template <typename T>
nmg_status upload(T* dst, const std::vector<double>& src) {
    std::vector<T> tmp(src.begin(), src.end());
    NMG_HIP(hipMemcpy(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
    return NMG_OK;
}

}  // namespace

template <>
Work<double>& work_of<double>(Ctx* c) {
    return c->w64;
}
template <>
Work<float>& work_of<float>(Ctx* c) {
    return c->w32b;
}

template <typename T>
nmg_status ensure_work(Ctx* c) {
    Work<T>& w = work_of<T>(c);
    if (w.ready) return NMG_OK;
    const int B = c->p.max_batch;
    w.lv.assign((size_t)c->L, LevelBuffers<T>{});
    for (int l = 0; l < c->L; ++l) {
        const size_t cnt = (size_t)B * level_elems(c, l);
        LevelBuffers<T>& lb = w.lv[(size_t)l];
        NMG_TRY(dev_alloc(&lb.x, cnt));
        NMG_TRY(dev_alloc(&lb.y, cnt));
        NMG_TRY(dev_alloc(&lb.b, cnt));
        NMG_TRY(dev_alloc(&lb.h, cnt));
        NMG_TRY(dev_alloc(&lb.t1, cnt));
        NMG_TRY(dev_alloc(&lb.t2, cnt));
    }
    // band tables and DCT matrices
    std::vector<double> G, M, D;
    w.g_off.clear();
    w.m_off.clear();
    w.dct_off.clear();
    for (int l = 0; l < c->L; ++l) {
        w.g_off.push_back(G.size());
        G.insert(G.end(), c->host[(size_t)l].G.a.begin(), c->host[(size_t)l].G.a.end());
        w.m_off.push_back(M.size());
        M.insert(M.end(), c->host[(size_t)l].M.a.begin(), c->host[(size_t)l].M.a.end());
        w.dct_off.push_back(D.size());
        std::vector<double> C = dct2(c->n[(size_t)l]);
        D.insert(D.end(), C.begin(), C.end());
    }
    NMG_TRY(dev_alloc(&w.Gd, G.size()));
    NMG_TRY(dev_alloc(&w.Md, M.size()));
    NMG_TRY(dev_alloc(&w.dct, D.size()));
    NMG_TRY(upload(w.Gd, G));
    NMG_TRY(upload(w.Md, M));
    NMG_TRY(upload(w.dct, D));
    // tiled-residual tables: Toeplitz taps padded to a multiple of 4, corner blocks
    w.tiled.assign((size_t)c->L, TiledOp<T>{});
    for (int l = 0; l < c->L; ++l) {
        const HostLevel& hl = c->host[(size_t)l];
        TiledOp<T>& op = w.tiled[(size_t)l];
        if (c->p.dim != 2 || !hl.Gs.ok || !hl.Ms.ok || hl.Ms.rc != 0) continue;
        const int rg = hl.Gs.r, rm = hl.Ms.r;
        const int rgp = ((2 * rg + 1) + 3) / 4 * 4, rmp = ((2 * rm + 1) + 3) / 4 * 4;
        // LDS bound (TH = 32): staged tile + row-pass buffers must fit in 160 KB
        const int TW = sizeof(T) == 4 ? 64 : 32;
        const int TH = 64;
        const size_t lds = ((size_t)(TH + 2 * rg) * (TW + rgp) + (size_t)(TH + rgp) * TW +
                            (l == 0 ? 0 : (size_t)(TH + rmp) * TW)) * sizeof(T);
        op.fused_ok = !(lds > 160 * 1024 || TW + rgp > 256);
        std::vector<double> tab;
        std::vector<double> tgv(hl.Gs.t), tmv(hl.Ms.t);
        tgv.resize((size_t)rgp, 0.0);
        tmv.resize((size_t)rmp, 0.0);
        const size_t o_tg = 0, o_tm = o_tg + rgp, o_dtl = o_tm + rmp, o_dbr = o_dtl + hl.Gs.dtl.size();
        tab.insert(tab.end(), tgv.begin(), tgv.end());
        tab.insert(tab.end(), tmv.begin(), tmv.end());
        tab.insert(tab.end(), hl.Gs.dtl.begin(), hl.Gs.dtl.end());
        tab.insert(tab.end(), hl.Gs.dbr.begin(), hl.Gs.dbr.end());
        NMG_TRY(dev_alloc(&op.base, tab.size()));
        NMG_TRY(upload(op.base, tab));
        op.tg = op.base + o_tg;
        op.tm = op.base + o_tm;
        op.dtl = op.base + o_dtl;
        op.dbr = op.base + o_dbr;
        op.rg = rg;
        op.rgp = rgp;
        op.rc = hl.Gs.rc;
        op.rm = rm;
        op.rmp = rmp;
        op.m_ident = (l == 0) ? 1 : 0;
        op.ok = true;
    }
    if (std::is_same<T, double>::value) {
        const size_t wn = (size_t)std::max(1, c->L - 1) * c->p.n_weight_sets * c->wcount;
        NMG_TRY(dev_alloc(&w.wts, wn));
        NMG_TRY(launch_convert<float, T>(c->w32, w.wts, wn, nullptr));
    } else {
        w.wts = reinterpret_cast<T*>(c->w32);
    }
    NMG_HIP(hipDeviceSynchronize());
    w.ready = true;
    return NMG_OK;
}

template nmg_status ensure_work<float>(Ctx*);
template nmg_status ensure_work<double>(Ctx*);

// Activation buffers of the direct-convolution smoother (FP32 and FP64
// cycles, training): cmax channels of the finest level per slot, allocated
// on first use only, since the BF16 MFMA smoother of mixed-precision cycles
// keeps its activations in LDS.  Never called inside a graph capture.
template <typename T>
nmg_status ensure_acts(Ctx* c) {
    NMG_TRY(ensure_work<T>(c));
    if (c->p.smoother_arch == NMG_ARCH_FNO) return ensure_fno<T>(c);
    Work<T>& w = work_of<T>(c);
    if (w.act0) return NMG_OK;
    if (c->capturing) return fail(NMG_ERR_STATE, "smoother buffers must exist before graph capture");
    const size_t act = (size_t)c->p.max_batch * c->cmax * level_elems(c, 0);
    NMG_TRY(dev_alloc(&w.act0, act));
    NMG_TRY(dev_alloc(&w.act1, act));
    return NMG_OK;
}
template nmg_status ensure_acts<float>(Ctx*);
template nmg_status ensure_acts<double>(Ctx*);

size_t request_bytes(const Ctx* c, nmg_precision prec) {
    size_t levels = 0;
    for (int l = 0; l < c->L; ++l) levels += level_elems(c, l);
    const size_t fine = level_elems(c, 0);
    // engine: x, b, r in FP64 and x, b in FP32; FP64 level buffers (6 planes)
    // always (refinement residual), FP32 ones for FP32 / mixed cycles, and the
    // direct-convolution activations for FP32 / FP64 cycles
    size_t bytes = fine * (3 * 8 + 2 * 4) + levels * 6 * 8;
    if (prec != NMG_FP64) bytes += levels * 6 * 4;
    const size_t tsize = prec == NMG_FP64 ? 8 : 4;
    if (c->p.smoother_arch == NMG_ARCH_FNO)
        bytes += fine * 2 * (size_t)c->p.fno_width * tsize;  // activation ping-pong
    else if (prec != NMG_MIXED)
        bytes += fine * 2 * (size_t)c->cmax * tsize;
    return bytes;
}

namespace {

template <typename T>
void free_work(Ctx* c, Work<T>& w) {
    for (auto& lb : w.lv) {
        dev_free(lb.x);
        dev_free(lb.y);
        dev_free(lb.b);
        dev_free(lb.h);
        dev_free(lb.t1);
        dev_free(lb.t2);
    }
    dev_free(w.act0);
    dev_free(w.act1);
    dev_free(w.fz0);
    dev_free(w.fz1);
    dev_free(w.fta);
    dev_free(w.fxh);
    dev_free(w.fyh);
    dev_free(w.fcd);
    dev_free(w.ftab);
    dev_free(w.fsp);
    dev_free(w.fwt);
    dev_free(w.fmat);
    dev_free(w.ftz);
    dev_free(w.ftp);
    dev_free(w.ftx);
    dev_free(w.ftgz);
    dev_free(w.ftgp);
    dev_free(w.ftga);
    dev_free(w.ftgx);
    dev_free(w.ftgy);
    dev_free(w.ftgo);
    dev_free(w.ftgs);
    w.ftr_ready = false;
    w.fno_ready = false;
    dev_free(w.Gd);
    dev_free(w.Md);
    dev_free(w.dct);
    for (auto& op : w.tiled) dev_free(op.base);
    w.tiled.clear();
    if (std::is_same<T, double>::value) dev_free(w.wts);
    w.wts = nullptr;
    w.ready = false;
    (void)c;
}

nmg_status check_handle(nmg_handle h) {
    if (!h) return fail(NMG_ERR_ARG, "null handle");
    return NMG_OK;
}

nmg_status check_batch(const Ctx* c, int batch) {
    if (batch < 1 || batch > c->p.max_batch) return fail(NMG_ERR_SHAPE, "batch must be in [1, max_batch]");
    return NMG_OK;
}

}  // namespace

nmg_status check_opts(const Ctx* c, const nmg_cycle_opts* o) {
    if (!o) return fail(NMG_ERR_ARG, "null cycle options");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 > 16) return fail(NMG_ERR_ARG, "nu1/nu2 out of range");
    if (o->precision != NMG_FP64 && o->precision != NMG_FP32 && o->precision != NMG_MIXED)
        return fail(NMG_ERR_ARG, "unknown precision");
    for (int l = 0; l + 1 < c->L; ++l) {
        if (c->kind[(size_t)l] < 0) return fail(NMG_ERR_STATE, "no smoother set for level " + std::to_string(l));
    }
    return NMG_OK;
}

namespace {

// ---------------------------------------------------------------------------
// The cycle
// ---------------------------------------------------------------------------
template <typename T>
struct CycleArgs {
    Ctx* c;
    Work<T>* w;
    int batch;
    const double* alpha;
    const int* ws;
    nmg_cycle_opts o;
    hipStream_t s;
    int chain_from = -1;     // level whose restriction chain produced every coarser y (-1: none)
    bool chain_eig = false;  // the chain also solved the coarsest level
};

// A cycle without pre-smoothing from x = 0 may restrict from level l down
// in one launch (launch_restrict_chain): 2D, the grids below l small enough
// for its LDS buffers, and sizes that halve.
template <typename T>
bool chain_restrict(const Ctx* c, int l, RestrictChain<T>& ch, Work<T>& w, const T* y) {
    if (c->dbg_separate_restrict || c->p.dim != 2 || l + 1 > c->L - 1 || c->L - l > kChainLevels) return false;
    if (c->n[(size_t)l + 1] > kChainMax) return false;
    for (int k = l; k + 1 < c->L; ++k)
        if (c->n[(size_t)k + 1] != (c->n[(size_t)k] - 1) / 2 || c->n[(size_t)k + 1] < 1) return false;
    ch.levels = c->L - l;
    for (int k = 0; k < ch.levels; ++k) {
        ch.n[k] = c->n[(size_t)(l + k)];
        ch.y[k] = k == 0 ? const_cast<T*>(y) : w.lv[(size_t)(l + k)].y;
    }
    const bool eig = c->eig_coarse && c->n[(size_t)c->L - 1] <= eig_small_max();
    ch.x_coarse = eig ? w.lv[(size_t)c->L - 1].x : nullptr;
    return true;
}

// parts_ready > 0 (with x_zero): c->norm_part already holds that many partial
// sums of ||y||^2 per right-hand side (written by the restriction that
// produced y)
template <typename T>
nmg_status smooth_step(CycleArgs<T>& a, int l, T* x, const T* y, bool x_zero, int parts_ready = 0) {
    Ctx* c = a.c;
    Work<T>& w = *a.w;
    const size_t per = level_elems(c, l);
    const T* bres = y;
    // the BF16 smoother takes ||b||^2 as per-image partial sums, which the
    // FP32 residual writes itself where it can
    const bool mfma = c->kind[(size_t)l] == 0 && c->p.smoother_arch != NMG_ARCH_FNO && a.o.precision == NMG_MIXED;
    if (!x_zero) {
        ProfScope ps(c, a.s, NMG_K_OPERATOR, l);
        NMG_TRY(launch_operator<T>(c, l, a.batch, a.alpha, x, y, w.lv[(size_t)l].b, 0, w, a.s,
                                   mfma ? c->norm_part : nullptr, mfma ? &parts_ready : nullptr));
        bres = w.lv[(size_t)l].b;
    }
    T* target = a.o.use_fprime ? w.lv[(size_t)l].h : x;
    const int acc = a.o.use_fprime ? 0 : (x_zero ? 0 : 1);
    // the BF16 smoother feeds the MFMA filter F' a zero-padded BF16 plane
    // (in the level's first F' scratch buffer) on levels above 64^2
    const int n_l = c->n[(size_t)l], np_l = (n_l + 127) / 128 * 128;
    const bool bf_plane = !c->dbg_fp32_handoff && mfma && a.o.use_fprime && c->p.dim == 2 && n_l > 64 && mfma_smoother_covers(c, l, np_l) &&
                          (size_t)np_l * np_l * 2 <= level_elems(c, l) * sizeof(T);
    if (c->kind[(size_t)l] == 1) {
        ProfScope ps(c, a.s, NMG_K_SMOOTHER, l);
        NMG_TRY(launch_jacobi<T>(c, l, a.batch, a.alpha, c->omega[(size_t)l], bres, target, acc, w, a.s));
    } else {
        // the BF16 kernel adds the per-image partial sums itself
        const bool have_parts = mfma && parts_ready > 0;
        const int nparts = have_parts ? parts_ready : norm_chunks(per);
        if (!have_parts) {
            ProfScope ps(c, a.s, NMG_K_NORM, l);
            if (mfma)
                NMG_TRY(launch_sumsq_part<T>(c, a.batch, per, bres, a.s));
            else
                NMG_TRY(launch_sumsq<T>(c, a.batch, per, bres, c->nrm, a.s));
        }
        ProfScope ps(c, a.s, NMG_K_SMOOTHER, l);
        if (c->p.smoother_arch == NMG_ARCH_FNO) {
            NMG_TRY(launch_fno_smoother<T>(c, l, a.batch, a.ws, bres, c->nrm, target, acc, w, a.s));
        } else if (a.o.precision == NMG_MIXED) {
            NMG_TRY(launch_mfma_smoother(c, l, a.batch, a.ws, reinterpret_cast<const float*>(bres), c->norm_part,
                                         nparts, reinterpret_cast<float*>(target), acc,
                                         *reinterpret_cast<Work<float>*>(&w), a.s,
                                         bf_plane ? reinterpret_cast<uint16_t*>(w.lv[(size_t)l].t1) : nullptr,
                                         bf_plane ? np_l : 0, fprime_tiled_layout(n_l)));
        } else {
            NMG_TRY(launch_conv_smoother<T>(c, l, a.batch, a.ws, bres, c->nrm, target, acc, w, a.s));
        }
    }
    if (a.o.use_fprime) {
        ProfScope ps(c, a.s, NMG_K_FPRIME, l);
        if (a.o.precision == NMG_MIXED && c->p.dim == 2) {
            NMG_TRY(prepare_fprime_bf16(c));
            NMG_TRY(launch_fprime_mfma(c, l, a.batch, reinterpret_cast<const float*>(w.lv[(size_t)l].h),
                                       bf_plane ? reinterpret_cast<const uint16_t*>(w.lv[(size_t)l].t1) : nullptr,
                                       reinterpret_cast<float*>(x), x_zero ? 0 : 1, w.lv[(size_t)l].t1,
                                       w.lv[(size_t)l].t2, (size_t)c->p.max_batch * level_elems(c, l) * sizeof(T),
                                       a.s));
        } else {
            NMG_TRY(launch_fprime<T>(c, l, a.batch, w.lv[(size_t)l].h, x, x_zero ? 0 : 1, w, a.s));
        }
    }
    return NMG_OK;
}

template <typename T>
nmg_status cycle(CycleArgs<T>& a, int l, T* x, const T* y, bool x_zero, int parts_ready = 0) {
    Ctx* c = a.c;
    Work<T>& w = *a.w;
    if (l == c->L - 1) {
        if (a.chain_eig) return NMG_OK;  // solved by the restriction chain
        ProfScope ps(c, a.s, NMG_K_COARSE, l);
        if (c->eig_coarse) return launch_eig_coarse<T>(c, a.batch, a.alpha, y, x, a.s);
        if (a.o.precision == NMG_FP64) return launch_coarse_solve<T>(c, a.batch, y, x, a.s);
        return launch_coarse_apply_inverse<T>(c, a.batch, y, x, a.s);
    }
    // with no pre-smoothing from x = 0, the residual is y itself: y is
    // restricted directly and the coarse correction sets x (no zero fill, no
    // residual launch)
    const bool from_zero = x_zero && a.o.nu1 == 0;
    for (int k = 0; k < a.o.nu1; ++k) {
        NMG_TRY(smooth_step<T>(a, l, x, y, x_zero, k == 0 ? parts_ready : 0));
        x_zero = false;
    }
    LevelBuffers<T>& lb = w.lv[(size_t)l];
    if (!from_zero) {
        ProfScope ps(c, a.s, NMG_K_OPERATOR, l);
        NMG_TRY(launch_operator<T>(c, l, a.batch, a.alpha, x, y, lb.b, 0, w, a.s));
    }
    // the restriction also writes the first stage of ||y_{l+1}||^2 when the next
    // level starts with a BF16 neural smoothing step on it
    const bool fuse_norm = l + 1 < c->L - 1 && a.o.nu1 > 0 && c->kind[(size_t)l + 1] == 0 &&
                           a.o.precision == NMG_MIXED && c->p.smoother_arch != NMG_ARCH_FNO;
    if (!(from_zero && a.chain_from >= 0 && l > a.chain_from)) {  // else the chain restricted this level
        ProfScope ps(c, a.s, NMG_K_RESTRICT, l);
        RestrictChain<T> ch;
        if (from_zero && !fuse_norm && chain_restrict<T>(c, l, ch, w, y)) {
            NMG_TRY(launch_restrict_chain<T>(c, a.batch, a.alpha, ch, a.s));
            a.chain_from = l;
            a.chain_eig = ch.x_coarse != nullptr;
        } else {
            NMG_TRY(launch_restrict<T>(c, l, a.batch, from_zero ? y : lb.b, w.lv[(size_t)l + 1].y, a.s,
                                       fuse_norm ? c->norm_part : nullptr));
        }
    }
    NMG_TRY(cycle<T>(a, l + 1, w.lv[(size_t)l + 1].x, w.lv[(size_t)l + 1].y, true,
                     fuse_norm ? restrict_norm_parts(c, l) : 0));
    {
        ProfScope ps(c, a.s, NMG_K_PROLONG, l);
        NMG_TRY(launch_prolong_add<T>(c, l, a.batch, w.lv[(size_t)l + 1].x, x, a.s, from_zero));
    }
    for (int k = 0; k < a.o.nu2; ++k) NMG_TRY(smooth_step<T>(a, l, x, y, false));
    return NMG_OK;
}

template <typename T>
nmg_status run_cycle(Ctx* c, int batch, const double* alpha, const int* ws, const T* y, T* x, bool x_zero,
                     const nmg_cycle_opts& o, hipStream_t s, int parts_ready = 0) {
    NMG_TRY(ensure_work<T>(c));
    if (o.precision != NMG_MIXED || c->p.smoother_arch == NMG_ARCH_FNO) NMG_TRY(ensure_acts<T>(c));
    CycleArgs<T> a{c, &work_of<T>(c), batch, alpha, ws, o, s};
    return cycle<T>(a, 0, x, y, x_zero, parts_ready);
}

}  // namespace

}  // namespace nmg

using namespace nmg;


namespace nmg {

constexpr int kMaxRollout = 64;  // rollout cycles per training sample

// Coarse factors are cached per alpha value (exact match): U distinct alphas
// need at most U factorizations, and alphas seen before cost nothing.  idx
// receives the cache slot of every alpha.  Slots used by requests the
// serving engine holds are never evicted.
nmg_status check_alpha(const Ctx* h, double a, int slot) {
    if (!std::isfinite(a) || !(a > 0.0))
        return fail(NMG_ERR_ARG, "alpha must be positive and finite (slot " + std::to_string(slot) + ")");
    if (!(a > h->alpha_floor))
        return fail(NMG_ERR_NOT_SPD, "alpha " + std::to_string(a) + " leaves alpha I + K indefinite (needs > " +
                                         std::to_string(h->alpha_floor) + ", slot " + std::to_string(slot) + ")");
    return NMG_OK;
}

nmg_status factor_alphas(Ctx* h, const std::vector<double>& al, std::vector<int>& idx, hipStream_t s) {
    const int n = (int)al.size();
    for (int b = 0; b < n; ++b) NMG_TRY(check_alpha(h, al[(size_t)b], b));
    if (h->eig_coarse) {  // the eigenbasis solve takes alpha directly: nothing to factor
        idx.assign((size_t)n, 0);
        return NMG_OK;
    }
    const long long stamp = ++h->prepare_count;
    const int slots = (int)h->cache_alpha.size();
    for (const auto& sl : h->eng.slot) h->cache_used[(size_t)sl.fidx] = stamp;
    idx.assign((size_t)n, -1);
    std::vector<int> new_slots;
    std::vector<double> new_alphas;
    auto find = [&](double a) {
        for (int k = 0; k < slots; ++k)
            if (h->cache_alpha[(size_t)k] == a) return k;
        return -1;
    };
    for (int b = 0; b < n; ++b) {
        const double a = al[(size_t)b];
        int k = find(a);
        if (k < 0) {
            // least recently used slot not claimed by this call (claimed slots carry `stamp`)
            long long best = stamp;
            for (int j = 0; j < slots; ++j)
                if (h->cache_used[(size_t)j] < best) {
                    best = h->cache_used[(size_t)j];
                    k = j;
                }
            if (k < 0) return fail(NMG_ERR_STATE, "coarse factor cache exhausted");
            h->cache_alpha[(size_t)k] = a;
            new_slots.push_back(k);
            new_alphas.push_back(a);
        }
        h->cache_used[(size_t)k] = stamp;
        idx[(size_t)b] = k;
    }
    const int cnt = (int)new_slots.size();
    if (cnt > 0) {
        NMG_HIP(hipMemcpyAsync(h->alpha_prepared, new_alphas.data(), (size_t)cnt * sizeof(double),
                               hipMemcpyHostToDevice, s));
        NMG_HIP(hipMemcpyAsync(h->slot_dev, new_slots.data(), (size_t)cnt * sizeof(int), hipMemcpyHostToDevice, s));
        NMG_TRY(launch_coarse_factor(h, cnt, h->alpha_prepared, h->slot_dev, s));
        NMG_TRY(launch_coarse_inverse(h, cnt, h->slot_dev, s));
        std::vector<int> flags((size_t)cnt);
        NMG_HIP(hipMemcpyAsync(flags.data(), h->flags, (size_t)cnt * sizeof(int), hipMemcpyDeviceToHost, s));
        NMG_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < cnt; ++k)
            if (flags[(size_t)k]) {
                h->cache_alpha[(size_t)new_slots[(size_t)k]] = std::nan("");
                return fail(NMG_ERR_NOT_SPD, "coarse Cholesky failed for alpha " + std::to_string(new_alphas[(size_t)k]));
            }
    }
    return NMG_OK;
}

namespace {
// Launch sizes for captured iterations: exact up to 32, where a solve's tail
// spends most of its iterations and a padded slot costs as much as a real
// one, then multiples of 4 (at most 40 graphs for a batch of 64).
int graph_batch(int k, int B) {
    int kb = k <= 32 ? k : (k + 3) / 4 * 4;
    return std::min(kb, B);
}

// Captures the work `body` enqueues on the handle's capture stream into an
// executable graph; profiler events recorded during the capture belong to it.
template <typename F>
nmg_status capture_graph(Ctx* h, F&& body, Ctx::GraphEntry& ge) {
    if (!h->cap_stream) NMG_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = h->cap_stream;
    if (h->prof_mask && !h->stamps) {
        int khz = 0;
        NMG_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, 0));
        h->wall_khz = khz > 0 ? (double)khz : 1.0e5;
        NMG_HIP(hipMalloc((void**)&h->stamps, (size_t)kStampSlots * sizeof(long long)));
    }
    h->capture_stamps.clear();
    NMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    h->capturing = true;
    const nmg_status st = body(cs);
    h->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    auto drop_events = [&]() { h->capture_stamps.clear(); };
    if (st != NMG_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        drop_events();
        (void)hipGetLastError();
        return st != NMG_OK ? st : hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        drop_events();
        (void)hipGetLastError();
        return hip_fail(ei, "hipGraphInstantiate", __FILE__, __LINE__);
    }
    ge.exec = ex;
    ge.stamps = h->capture_stamps;
    h->capture_stamps.clear();
    return NMG_OK;
}

}  // namespace

namespace {
// Points the cycle's coarse solve at the engine's per-slot factor indices
// for one step and restores the prepare order on every exit.
struct FidxGuard {
    Ctx* c;
    ~FidxGuard() { c->cycle_fidx = nullptr; }
};
}  // namespace

// One step of the serving engine (see nmg_serve_step).
nmg_status engine_step(Ctx* h, double rtol, int max_cycles, const nmg_cycle_opts* o,
                       std::vector<nmg_request_result>& done, hipStream_t s, hipEvent_t retired,
                       std::vector<double>* submit_ms) {
    Engine& E = h->eng;
    const int B = h->p.max_batch;
    const size_t per = level_elems(h, 0);
    const bool plain32 = o->precision == NMG_FP32;
    int k = (int)E.slot.size();
    if (k > 0 && E.precision != (int)o->precision)
        return fail(NMG_ERR_STATE, "cycle precision changed while requests are active");
    NMG_TRY(ensure_work<double>(h));
    if (o->precision != NMG_FP64) NMG_TRY(ensure_work<float>(h));
    if (o->precision == NMG_FP64) NMG_TRY(ensure_acts<double>(h));
    if (o->precision == NMG_FP32 || (o->precision == NMG_MIXED && h->p.smoother_arch == NMG_ARCH_FNO))
        NMG_TRY(ensure_acts<float>(h));
    if (o->precision == NMG_MIXED && h->p.dim == 2 && o->use_fprime) NMG_TRY(prepare_fprime_bf16(h));
    FidxGuard guard{h};
    double* X64 = h->x64;
    double* B64 = h->b64;
    double* R64 = h->r64;
    float* X32 = h->xs32;
    float* B32 = h->bs32;
    float* R32 = reinterpret_cast<float*>(h->r64);  // r64 has room for max_batch doubles per point
    double* d_alpha = h->slot_d;
    double* d_bn2 = h->slot_d + B;
    double* d_rn2 = h->slot_d + 2 * B;
    int* d_ws = h->slot_i;
    int* d_fidx = h->slot_i + B;
    int* d_pairs = h->slot_i + 2 * B;  // 2B ints: slots of finished requests
    int* d_moves = h->slot_i + 4 * B;  // 2B ints: (destination, source) slot moves
    double* hd = h->pin_d;
    int* hi = h->pin_i;
    // ---- admission: queued requests fill slots [k, k + m)
    const int m = std::min(B - k, (int)E.queue.size());
    if (m > 0) {
        std::vector<double> al((size_t)m);
        for (int i = 0; i < m; ++i) al[(size_t)i] = E.queue[(size_t)i].alpha;
        std::vector<int> fidx;
        NMG_TRY(factor_alphas(h, al, fidx, s));
        // copy runs of contiguous right-hand sides with one transfer each
        for (int i = 0; i < m;) {
            int j = i + 1;
            while (j < m && E.queue[(size_t)j].b == E.queue[(size_t)i].b + (size_t)(j - i) * per) ++j;
            NMG_HIP(hipMemcpyAsync(B64 + (size_t)(k + i) * per, E.queue[(size_t)i].b, (size_t)(j - i) * per *
                                   sizeof(double), hipMemcpyDeviceToDevice, s));
            i = j;
        }
        const size_t off = (size_t)k * per, cnt = (size_t)m * per;
        // x0 = 0, so the first residual is b itself
        if (plain32) {
            NMG_TRY(launch_sumsq<double>(h, m, per, B64 + off, h->nrm + k, s));  // ||b||^2 in FP64
            NMG_TRY(launch_convert<double, float>(B64 + off, B32 + off, cnt, s));
            NMG_HIP(hipMemcpyAsync(R32 + off, B32 + off, cnt * sizeof(float), hipMemcpyDeviceToDevice, s));
            NMG_TRY(launch_zero<float>(X32 + off, cnt, s));
            NMG_TRY(launch_sumsq<float>(h, m, per, R32 + off, h->nrm2 + k, s, h->pin_rd + k));
        } else {
            NMG_TRY(launch_sumsq<double>(h, m, per, B64 + off, h->nrm2 + k, s, h->pin_rd + k));
            NMG_HIP(hipMemcpyAsync(R64 + off, B64 + off, cnt * sizeof(double), hipMemcpyDeviceToDevice, s));
            NMG_TRY(launch_zero<double>(X64 + off, cnt, s));
        }
        for (int i = 0; i < m; ++i) {
            const EngineRequest& r = E.queue[(size_t)i];
            EngineSlot sl;
            sl.id = r.id;
            sl.x = r.x;
            sl.hist = r.hist;
            sl.hist_len = r.hist_len;
            sl.alpha = r.alpha;
            sl.ws = r.ws;
            sl.fidx = fidx[(size_t)i];
            sl.t_submit = r.t_submit;
            E.slot.push_back(sl);
            E.any_ws = E.any_ws || r.ws != 0;
        }
        E.queue.erase(E.queue.begin(), E.queue.begin() + m);
        E.precision = (int)o->precision;
    }
    k = (int)E.slot.size();
    if (k == 0) return NMG_OK;
    // ---- residual norms of every active slot (new ones: ||b||^2).  Every
    // launch that writes h->nrm2 in this engine (the admission above, the
    // residual of each iteration) also writes the sums into pinned host
    // memory at the same index, so they are read there once the stream's
    // work is done
    double* rn2 = h->pin_rd;
    double* bn2n = h->pin_rd + B;
    if (m > 0)
        NMG_HIP(hipMemcpyAsync(bn2n, (plain32 ? h->nrm : h->nrm2) + (k - m), (size_t)m * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    NMG_HIP(hipStreamSynchronize(s));
    if (h->prof_mask) NMG_TRY(prof_resolve(h));
    for (int i = 0; i < m; ++i) E.slot[(size_t)(k - m + i)].bn2 = bn2n[(size_t)i];
    const double now = E.now_ms();
    const double tol2 = rtol * rtol;
    const double kDiverge2 = NMG_DIVERGENCE_FACTOR * NMG_DIVERGENCE_FACTOR;
    // ---- retire finished requests
    std::vector<char> keep((size_t)k, 0);
    int nfin = 0, nkeep = 0;
    for (int i = 0; i < k; ++i) {
        EngineSlot& sl = E.slot[(size_t)i];
        const double q = rn2[(size_t)i], bb = sl.bn2;
        sl.rn2 = q;
        int status = -100;  // still running
        if (!std::isfinite(q) || !std::isfinite(bb)) {
            status = NMG_ERR_NONFINITE;
        } else {
            if (sl.hist && sl.cycles < sl.hist_len) sl.hist[sl.cycles] = bb > 0 ? std::sqrt(q / bb) : 0.0;
            if (!(q > tol2 * bb))
                status = NMG_OK;
            else if (q > kDiverge2 * bb)
                status = NMG_DIVERGED;
            else if (sl.cycles >= max_cycles)
                status = NMG_NOT_CONVERGED;
        }
        if (status == -100) {
            keep[(size_t)i] = 1;
            ++nkeep;
            continue;
        }
        nmg_request_result res;
        res.id = sl.id;
        res.status = status;
        res.cycles = sl.cycles;
        res.rel_residual = (std::isfinite(q) && bb > 0) ? std::sqrt(q / bb) : (bb > 0 ? q : 0.0);
        res.latency_ms = now - sl.t_submit;
        done.push_back(res);
        if (submit_ms) submit_ms->push_back(sl.t_submit);
        hi[(size_t)2 * B + nfin] = i;
        h->pin_ptr[nfin] = sl.x;
        ++nfin;
    }
    // ---- refill the finished slots below nkeep from active slots at or above it
    int nmoves = 0;
    {
        int src = k - 1;
        for (int dst = 0; dst < nkeep; ++dst) {
            if (keep[(size_t)dst]) continue;
            while (!keep[(size_t)src]) --src;  // src >= nkeep holds an active slot
            hi[(size_t)4 * B + 2 * nmoves] = dst;
            hi[(size_t)4 * B + 2 * nmoves + 1] = src;
            ++nmoves;
            E.slot[(size_t)dst] = E.slot[(size_t)src];
            keep[(size_t)src] = 0;
            --src;
        }
    }
    E.slot.resize((size_t)nkeep);
    k = nkeep;
    // ---- the next outer iteration runs on kb >= k slots (a fixed set of
    // launch sizes, so a few captured graphs serve every active count); slots
    // k..kb-1 carry slot 0's parameters with a zero residual norm, which the
    // cycle treats as converged (zero input, no update)
    const int kb = k == 0 ? 0 : (h->use_graphs ? graph_batch(k, B) : k);
    for (int i = 0; i < kb; ++i) {
        const EngineSlot& sl = E.slot[(size_t)(i < k ? i : 0)];
        hd[(size_t)i] = sl.alpha;
        hd[(size_t)B + i] = sl.bn2;
        hd[(size_t)2 * B + i] = i < k ? sl.rn2 : 0.0;
        hi[(size_t)i] = sl.ws;
        hi[(size_t)B + i] = sl.fidx;
    }
    // one transfer for the slot tables, the finished slots and the slot
    // moves (the host block is laid out like the device one); the finished
    // iterates are copied out before the moves overwrite their slots
    if (kb > 0 || nfin > 0 || nmoves > 0)
        NMG_HIP(hipMemcpyAsync(h->slot_d, hd, (size_t)3 * B * sizeof(double) + (size_t)6 * B * sizeof(int),
                               hipMemcpyHostToDevice, s));
    if (nfin > 0) {
        NMG_HIP(hipMemcpyAsync(h->xptr_dev, h->pin_ptr, (size_t)nfin * sizeof(double*),
                               hipMemcpyHostToDevice, s));
        if (plain32)
            NMG_TRY(launch_scatter_ptrs<float>(nfin, per, X32, h->xptr_dev, d_pairs, s));
        else
            NMG_TRY(launch_scatter_ptrs<double>(nfin, per, X64, h->xptr_dev, d_pairs, s));
        if (retired) NMG_HIP(hipEventRecord(retired, s));
    }
    if (nmoves > 0) {
        if (plain32)
            NMG_TRY(launch_move_slots<float>(nmoves, per, X32, B32, R32, d_moves, s));
        else
            NMG_TRY(launch_move_slots<double>(nmoves, per, X64, B64, R64, d_moves, s));
    }
    if (k == 0) {
        E.precision = -1;
        E.any_ws = false;
        NMG_HIP(hipStreamSynchronize(s));
        return NMG_OK;
    }
    h->cycle_fidx = d_fidx;
    const int* wsd = E.any_ws ? d_ws : nullptr;
    auto residual = [&](int kk, hipStream_t st) -> nmg_status {
        ProfScope ps(h, st, NMG_K_REFINE, 0);
        if (plain32) {
            NMG_TRY(launch_operator<float>(h, 0, kk, d_alpha, X32, B32, R32, 0, h->w32b, st));
            NMG_TRY(launch_sumsq<float>(h, kk, per, R32, h->nrm2, st, h->pin_rd));
        } else {
            NMG_TRY(launch_operator<double>(h, 0, kk, d_alpha, X64, B64, R64, 0, h->w64, st));
            NMG_TRY(launch_sumsq<double>(h, kk, per, R64, h->nrm2, st, h->pin_rd));
        }
        return NMG_OK;
    };
    // d = MG(0, r / ||r||), x += ||r|| d, then the residual for the next check
    auto iterate = [&](int kk, hipStream_t st) -> nmg_status {
        if (plain32) {
            Work<float>& w = h->w32b;
            NMG_TRY(launch_refine_scale<float, float>(kk, per, R32, w.lv[0].y, d_rn2, d_bn2, rtol, h->active, st));
            NMG_TRY(run_cycle<float>(h, kk, d_alpha, wsd, w.lv[0].y, w.lv[0].x, true, *o, st));
            NMG_TRY(launch_refine_update<float, float>(kk, per, X32, w.lv[0].x, d_rn2, h->active, st));
        } else if (o->precision == NMG_FP64) {
            Work<double>& w = h->w64;
            NMG_TRY(launch_refine_scale<double, double>(kk, per, R64, w.lv[0].y, d_rn2, d_bn2, rtol, h->active, st));
            NMG_TRY(run_cycle<double>(h, kk, d_alpha, wsd, w.lv[0].y, w.lv[0].x, true, *o, st));
            // the update inside the residual's row pass, the norm inside its column pass
            if (refine_residual_fusable(h, h->w64)) {
                ProfScope ps(h, st, NMG_K_REFINE, 0);
                (void)launch_refine_residual<double>(h, kk, d_alpha, X64, w.lv[0].x, d_rn2, h->active, B64, R64,
                                                  h->nrm2, h->w64, st, h->pin_rd);
                NMG_HIP(hipGetLastError());
                return NMG_OK;
            }
            NMG_TRY(launch_refine_update<double, double>(kk, per, X64, w.lv[0].x, d_rn2, h->active, st));
        } else {
            Work<float>& w = h->w32b;
            // the scaling also writes the first stage of ||y||^2 for the cycle's first smoothing step
            NMG_TRY(launch_refine_scale<double, float>(kk, per, R64, w.lv[0].y, d_rn2, d_bn2, rtol, h->active, st,
                                                       h->norm_part));
            NMG_TRY(run_cycle<float>(h, kk, d_alpha, wsd, w.lv[0].y, w.lv[0].x, true, *o, st, norm_chunks(per)));
            if (refine_residual_fusable(h, h->w64)) {
                ProfScope ps(h, st, NMG_K_REFINE, 0);
                (void)launch_refine_residual<float>(h, kk, d_alpha, X64, w.lv[0].x, d_rn2, h->active, B64, R64,
                                                  h->nrm2, h->w64, st, h->pin_rd);
                NMG_HIP(hipGetLastError());
                return NMG_OK;
            }
            NMG_TRY(launch_refine_update<double, float>(kk, per, X64, w.lv[0].x, d_rn2, h->active, st));
        }
        return residual(kk, st);
    };
    // sampled timing: iterations off the sampling period run without timing
    // nodes (their own graph), so the timing adds no launches to them
    struct MaskGuard {
        Ctx* c;
        int saved;
        ~MaskGuard() { c->prof_mask = saved; }
    } mask_guard{h, h->prof_mask};
    if (h->prof_mask && h->prof_period > 1 && (h->prof_iter++ % h->prof_period) != 0) h->prof_mask = 0;
    if (h->prof_mask) h->prof_rhs += k;
    if (h->use_graphs) {
        std::vector<long long> key = {kb, (long long)o->precision, o->nu1, o->nu2, o->use_fprime, wsd ? 1 : 0,
                                      (long long)h->prof_mask, (long long)h->prof_levels};
        long long rbits;
        __builtin_memcpy(&rbits, &rtol, sizeof(rbits));
        key.push_back(rbits);
        auto found = h->graphs.find(key);
        if (found == h->graphs.end()) {
            Ctx::GraphEntry ge;
            NMG_TRY(capture_graph(h, [&](hipStream_t cs) { return iterate(kb, cs); }, ge));
            found = h->graphs.emplace(key, std::move(ge)).first;
        }
        if (h->prof_mask)
            for (auto& e : found->second.stamps) h->stamp_pending.push_back(e);
        NMG_HIP(hipGraphLaunch(found->second.exec, s));
    } else {
        NMG_TRY(iterate(kb, s));
    }
    for (int i = 0; i < k; ++i) E.slot[(size_t)i].cycles += 1;
    return NMG_OK;
}

}  // namespace nmg

extern "C" {

const char* nmg_last_error(void) { return nmg::g_last_error.c_str(); }

nmg_status nmg_setup_hierarchy(const nmg_problem* p, nmg_handle* out) {
    if (!p || !out) return fail(NMG_ERR_ARG, "null argument");
    *out = nullptr;
    if (p->dim != 1 && p->dim != 2) return fail(NMG_ERR_SHAPE, "dim must be 1 or 2");
    if (p->levels < 1 || p->levels > 16) return fail(NMG_ERR_SHAPE, "levels must be in [1, 16]");
    if (p->max_batch < 1 || p->max_batch > 4096) return fail(NMG_ERR_SHAPE, "max_batch must be in [1, 4096]");
    if (p->n_layers < 1 || p->n_layers > NMG_MAX_LAYERS) return fail(NMG_ERR_SHAPE, "n_layers out of range");
    if (p->channels[0] != 1 || p->channels[p->n_layers] != 1)
        return fail(NMG_ERR_SHAPE, "first and last channel counts must be 1");
    for (int i = 0; i <= p->n_layers; ++i)
        if (p->channels[i] < 1 || p->channels[i] > 256) return fail(NMG_ERR_SHAPE, "channel count out of range");
    if (p->ksize < 1 || (p->ksize & 1) == 0 || p->ksize > 15) return fail(NMG_ERR_SHAPE, "ksize must be odd, <= 15");
    if (p->n_weight_sets < 1 || p->n_weight_sets > 64) return fail(NMG_ERR_SHAPE, "n_weight_sets out of range");
    // the transfer kernels index a level's points with 32-bit integers
    if (p->n < 1 || (p->dim == 2 ? (long long)p->n * p->n : (long long)p->n) >= (1LL << 31))
        return fail(NMG_ERR_SHAPE, "n out of range (a level must hold fewer than 2^31 points)");
    std::unique_ptr<nmg_ctx> c(new nmg_ctx());
    c->p = *p;
    std::string err;
    if (!build_host_hierarchy(p->n, p->s, p->trunc, p->levels, p->dim, p->operator_form, c->host, &c->taps_radius,
                              &c->alpha_floor, err))
        return fail(NMG_ERR_SHAPE, err);
    c->L = p->levels;
    for (auto& hl : c->host) c->n.push_back(hl.n);
    c->ny0 = p->dim == 2 ? p->n : 1;
    const int nl = c->n.back();
    c->nc = p->dim == 2 ? nl * nl : nl;
    // 2D: the coarsest operator alpha M (x) M + G (x) G is solved exactly in the
    // eigenbasis of the pencil (G, M), which does not depend on alpha: no
    // factorization per alpha (a dense Cholesky and inverse of the 225 x 225
    // operator of a 15^2 grid took 6.6 ms per new alpha, which a serving
    // stream with a new alpha per request paid on every admission), and the
    // solve is four n x n products per right-hand side.  1D: dense factors.
    if (c->nc > 1024 && (p->dim != 2 || nl > 511))
        return fail(NMG_ERR_SHAPE, "coarsest grid too large (dense factor up to 1024 unknowns; in 2D the "
                                   "eigenbasis solve up to 511^2)");
    c->eig_coarse = p->dim == 2;
    // smoother layout
    const int kk = p->dim == 2 ? p->ksize * p->ksize : p->ksize;
    c->wcount = 0;
    c->cmax = 1;
    for (int i = 0; i < p->n_layers; ++i) {
        c->layer_off.push_back(c->wcount);
        c->wcount += p->channels[i] * p->channels[i + 1] * kk;
        c->cmax = std::max(c->cmax, p->channels[i + 1]);
    }
    if (p->smoother_arch == NMG_ARCH_FNO) {
        if (p->fno_width < 1 || p->fno_width > 256 || p->fno_layers < 1 || p->fno_layers > 16 || p->fno_modes < 1 ||
            p->fno_modes > 128 ||
            p->fno_ksize < 1 || (p->fno_ksize & 1) == 0 || p->fno_ksize > 15)
            return fail(NMG_ERR_SHAPE, "FNO width (1..256), layers (1..16), modes (1..128) or ksize (odd, <= 15) out of range");
        for (int l = 0; l + 1 < c->L; ++l)
            if (c->n[(size_t)l] / 2 < 1) return fail(NMG_ERR_SHAPE, "FNO needs n >= 2 on every smoothing level");
        c->wcount = (int)fno_weight_count(*p);
        c->cmax = 1;
    } else if (p->smoother_arch != NMG_ARCH_CNN) {
        return fail(NMG_ERR_SHAPE, "unknown smoother architecture");
    }
    const int nsm = std::max(1, c->L - 1);
    c->kind.assign((size_t)nsm, -1);
    c->omega.assign((size_t)nsm, 0.0);
    c->loaded.assign((size_t)nsm, std::vector<char>((size_t)p->n_weight_sets, 0));
    c->adam_step.assign((size_t)p->n_weight_sets, 0);
    const size_t wn = (size_t)nsm * p->n_weight_sets * c->wcount;
    const int B = p->max_batch;
    NMG_TRY(dev_alloc(&c->w32, wn));
    NMG_TRY(dev_alloc(&c->g32, wn));
    NMG_TRY(dev_alloc(&c->g64, wn));
    NMG_TRY(dev_alloc(&c->adam_m, wn));
    NMG_TRY(dev_alloc(&c->adam_v, wn));
    NMG_HIP(hipMemset(c->w32, 0, wn * sizeof(float)));
    NMG_HIP(hipMemset(c->g32, 0, wn * sizeof(float)));
    NMG_HIP(hipMemset(c->g64, 0, wn * sizeof(double)));
    NMG_HIP(hipMemset(c->adam_m, 0, wn * sizeof(float)));
    NMG_HIP(hipMemset(c->adam_v, 0, wn * sizeof(float)));
    // coarse factors
    std::vector<double> Mc((size_t)nl * nl), Gc((size_t)nl * nl);
    const HostLevel& hc = c->host.back();
    for (int i = 0; i < nl; ++i)
        for (int j = 0; j < nl; ++j) {
            Mc[(size_t)i * nl + j] = hc.M.get(i, j);
            Gc[(size_t)i * nl + j] = hc.G.get(i, j);
        }
    NMG_TRY(dev_alloc(&c->Mc, Mc.size()));
    NMG_TRY(dev_alloc(&c->Gc, Gc.size()));
    NMG_TRY(upload(c->Mc, Mc));
    NMG_TRY(upload(c->Gc, Gc));
    if (c->eig_coarse) {
        std::vector<double> V, lam;
        if (!coarse_eigenbasis(hc.M, hc.G, V, lam, err)) return fail(NMG_ERR_NOT_SPD, err);
        NMG_TRY(dev_alloc(&c->eigV, V.size()));
        NMG_TRY(dev_alloc(&c->eigLam, lam.size()));
        NMG_TRY(upload(c->eigV, V));
        NMG_TRY(upload(c->eigLam, lam));
        NMG_TRY(dev_alloc(&c->eigT, (size_t)2 * B * nl * nl));
    } else {
        NMG_TRY(dev_alloc(&c->chol, (size_t)B * c->nc * c->nc));
        NMG_TRY(dev_alloc(&c->cholT, (size_t)B * c->nc * c->nc));
        NMG_TRY(dev_alloc(&c->cinv, (size_t)B * c->nc * c->nc));
        NMG_TRY(dev_alloc(&c->cwork, (size_t)B * c->nc * c->nc));
    }
    NMG_TRY(dev_alloc(&c->flags, (size_t)B));
    NMG_TRY(dev_alloc(&c->alpha_prepared, (size_t)B));
    NMG_TRY(dev_alloc(&c->slot_dev, (size_t)B));
    NMG_TRY(dev_alloc(&c->coarse_idx, (size_t)B));
    c->cache_alpha.assign((size_t)B, std::nan(""));
    c->cache_used.assign((size_t)B, -1);
    NMG_TRY(dev_alloc(&c->nrm, (size_t)B));
    NMG_TRY(dev_alloc(&c->nrm2, (size_t)B));
    NMG_TRY(dev_alloc(&c->norm_part, (size_t)B * std::max(kResidualNormParts, kNormChunksMax)));

    NMG_TRY(dev_alloc(&c->hist_dev, (size_t)B));
    NMG_TRY(dev_alloc(&c->active, (size_t)B));
    NMG_TRY(dev_alloc(&c->x64, (size_t)B * level_elems(c.get(), 0)));
    NMG_TRY(dev_alloc(&c->b64, (size_t)B * level_elems(c.get(), 0)));
    // 3B doubles, then 6B ints (= 3B doubles' bytes)
    NMG_TRY(dev_alloc(&c->slot_d, (size_t)6 * B));
    c->slot_i = reinterpret_cast<int*>(c->slot_d + (size_t)3 * B);
    NMG_HIP(hipMalloc((void**)&c->xptr_dev, (size_t)B * sizeof(double*)));
    NMG_HIP(hipHostMalloc((void**)&c->pin_d, (size_t)8 * B * sizeof(double), hipHostMallocDefault));
    c->pin_i = reinterpret_cast<int*>(c->pin_d + (size_t)3 * B);
    c->pin_rd = c->pin_d + (size_t)6 * B;
    NMG_HIP(hipHostMalloc((void**)&c->pin_ptr, (size_t)B * sizeof(double*), hipHostMallocDefault));
    NMG_TRY(dev_alloc(&c->r64, (size_t)B * level_elems(c.get(), 0)));
    NMG_TRY(dev_alloc(&c->xs32, (size_t)B * level_elems(c.get(), 0)));
    NMG_TRY(dev_alloc(&c->bs32, (size_t)B * level_elems(c.get(), 0)));
    NMG_TRY(dev_alloc(&c->loss_dev, (size_t)nsm));
    if (p->dim == 2) {
        // the BF16 filter's tables, and the device address of the scratch
        // of nmg_apply_fprime_noalloc on this device
        NMG_TRY(prepare_fprime_bf16(c.get()));
        NMG_TRY(fprime_noalloc_init());
    }
    NMG_HIP(hipDeviceSynchronize());
    *out = c.release();
    return NMG_OK;
}

void nmg_destroy(nmg_handle h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    nmg::Ctx* c = h;
    (void)prof_resolve(c);
    for (auto e : c->prof_pool) (void)hipEventDestroy(e);
    c->prof_pool.clear();
    release_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    if (c->serve_retired) (void)hipEventDestroy(c->serve_retired);
    c->serve_retired = nullptr;
    if (c->stamps) (void)hipFree(c->stamps);
    c->stamps = nullptr;
    release_training(c);
    free_work(c, c->w64);
    free_work(c, c->w32b);
    dev_free(c->w32);
    dev_free(c->g32);
    dev_free(c->g64);
    dev_free(c->adam_m);
    dev_free(c->adam_v);
    dev_free(c->wbf);
    dev_free(c->dctbf);
    dev_free(c->ramp);
    dev_free(c->Mc);
    dev_free(c->Gc);
    dev_free(c->chol);
    dev_free(c->cholT);
    dev_free(c->cinv);
    dev_free(c->cwork);
    dev_free(c->eigV);
    dev_free(c->eigLam);
    dev_free(c->eigT);
    dev_free(c->flags);
    dev_free(c->alpha_prepared);
    dev_free(c->slot_dev);
    dev_free(c->coarse_idx);
    dev_free(c->nrm);
    dev_free(c->nrm2);
    dev_free(c->norm_part);
    dev_free(c->hist_dev);
    dev_free(c->active);
    dev_free(c->x64);
    dev_free(c->b64);
    dev_free(c->slot_d);
    c->slot_i = nullptr;
    dev_free(c->xptr_dev);
    if (c->pin_d) (void)hipHostFree(c->pin_d);
    c->pin_i = nullptr;
    c->pin_rd = nullptr;
    if (c->pin_ptr) (void)hipHostFree(c->pin_ptr);
    dev_free(c->r64);
    dev_free(c->xs32);
    dev_free(c->bs32);
    dev_free(c->loss_dev);
    delete h;
}

int nmg_level_size(nmg_handle h, int level) {
    if (!h || level < 0 || level >= h->L) return -1;
    return h->n[(size_t)level];
}

nmg_status nmg_alpha_floor(nmg_handle h, double* floor_out) {
    NMG_TRY(check_handle(h));
    if (!floor_out) return fail(NMG_ERR_ARG, "null pointer");
    *floor_out = h->alpha_floor;
    return NMG_OK;
}

nmg_status nmg_load_smoother_weights(nmg_handle h, int level, int weight_set, const float* w, size_t count) {
    NMG_TRY(check_handle(h));
    if (!w) return fail(NMG_ERR_ARG, "null weights");
    if (level < 0 || level >= h->L - 1) return fail(NMG_ERR_ARG, "level must be in [0, L-2]");
    if (weight_set < 0 || weight_set >= h->p.n_weight_sets) return fail(NMG_ERR_ARG, "weight_set out of range");
    if (count != (size_t)h->wcount)
        return fail(NMG_ERR_SHAPE, "weight count " + std::to_string(count) + " != expected " +
                                       std::to_string(h->wcount));
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(w[i])) return fail(NMG_ERR_NONFINITE, "non-finite weight");
    const size_t off = ((size_t)level * h->p.n_weight_sets + weight_set) * h->wcount;
    NMG_HIP(hipMemcpy(h->w32 + off, w, count * sizeof(float), hipMemcpyHostToDevice));
    if (h->w64.ready) NMG_TRY(launch_convert<float, double>(h->w32 + off, h->w64.wts + off, count, nullptr));
    NMG_HIP(hipDeviceSynchronize());
    h->kind[(size_t)level] = 0;
    h->loaded[(size_t)level][(size_t)weight_set] = 1;
    NMG_TRY(repack_bf16(h, level, weight_set));
    return NMG_OK;
}

nmg_status nmg_get_smoother_weights(nmg_handle h, int level, int weight_set, float* w, size_t count) {
    NMG_TRY(check_handle(h));
    if (!w) return fail(NMG_ERR_ARG, "null weights");
    if (level < 0 || level >= h->L - 1) return fail(NMG_ERR_ARG, "level must be in [0, L-2]");
    if (weight_set < 0 || weight_set >= h->p.n_weight_sets) return fail(NMG_ERR_ARG, "weight_set out of range");
    if (count != (size_t)h->wcount) return fail(NMG_ERR_SHAPE, "weight count mismatch");
    const size_t off = ((size_t)level * h->p.n_weight_sets + weight_set) * h->wcount;
    NMG_HIP(hipDeviceSynchronize());
    NMG_HIP(hipMemcpy(w, h->w32 + off, count * sizeof(float), hipMemcpyDeviceToHost));
    return NMG_OK;
}

nmg_status nmg_set_jacobi_smoother(nmg_handle h, int level, double omega) {
    NMG_TRY(check_handle(h));
    if (level < 0 || level >= h->L - 1) return fail(NMG_ERR_ARG, "level must be in [0, L-2]");
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(NMG_ERR_ARG, "omega must be positive");
    h->kind[(size_t)level] = 1;
    h->omega[(size_t)level] = omega;
    return NMG_OK;
}

nmg_status nmg_prepare(nmg_handle h, int batch, const double* alpha, void* stream) {
    NMG_TRY(check_handle(h));
    NMG_TRY(check_batch(h, batch));
    if (!alpha) return fail(NMG_ERR_ARG, "null alpha");
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> al((size_t)batch);
    NMG_HIP(hipMemcpyAsync(al.data(), alpha, (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, s));
    NMG_HIP(hipStreamSynchronize(s));
    std::vector<int> idx;
    NMG_TRY(factor_alphas(h, al, idx, s));
    h->coarse_idx_host = idx;
    h->alpha_host = al;
    NMG_HIP(hipMemcpyAsync(h->coarse_idx, h->coarse_idx_host.data(), (size_t)batch * sizeof(int),
                           hipMemcpyHostToDevice, s));
    NMG_HIP(hipStreamSynchronize(s));
    return NMG_OK;
}

nmg_status nmg_apply_operator(nmg_handle h, int level, int batch, const double* alpha, const void* x, void* y,
                              nmg_precision prec, void* stream) {
    NMG_TRY(check_handle(h));
    NMG_TRY(check_batch(h, batch));
    if (!alpha || !x || !y) return fail(NMG_ERR_ARG, "null pointer");
    if (level < 0 || level >= h->L) return fail(NMG_ERR_ARG, "level out of range");
    hipStream_t s = (hipStream_t)stream;
    if (prec == NMG_FP64) {
        NMG_TRY(ensure_work<double>(h));
        return launch_operator<double>(h, level, batch, alpha, (const double*)x, nullptr, (double*)y, 1, h->w64, s);
    }
    NMG_TRY(ensure_work<float>(h));
    return launch_operator<float>(h, level, batch, alpha, (const float*)x, nullptr, (float*)y, 1, h->w32b, s);
}

nmg_status nmg_apply_smoother(nmg_handle h, int level, int batch, const double* alpha, const int* ws, const void* b,
                              void* out, nmg_precision prec, void* stream) {
    NMG_TRY(check_handle(h));
    NMG_TRY(check_batch(h, batch));
    if (!b || !out) return fail(NMG_ERR_ARG, "null pointer");
    if (level < 0 || level >= h->L - 1) return fail(NMG_ERR_ARG, "level must be in [0, L-2]");
    if (h->kind[(size_t)level] < 0) return fail(NMG_ERR_STATE, "no smoother set for this level");
    if (h->kind[(size_t)level] == 1 && !alpha) return fail(NMG_ERR_ARG, "Jacobi needs alpha");
    hipStream_t s = (hipStream_t)stream;
    const size_t per = level_elems(h, level);
    if (prec == NMG_FP64) {
        NMG_TRY(ensure_work<double>(h));
        const double* bb = (const double*)b;
        double* oo = (double*)out;
        if (h->kind[(size_t)level] == 1)
            return launch_jacobi<double>(h, level, batch, alpha, h->omega[(size_t)level], bb, oo, 0, h->w64, s);
        NMG_TRY(launch_sumsq<double>(h, batch, per, bb, h->nrm, s));
        NMG_TRY(ensure_acts<double>(h));
        if (h->p.smoother_arch == NMG_ARCH_FNO)
            return launch_fno_smoother<double>(h, level, batch, ws, bb, h->nrm, oo, 0, h->w64, s);
        return launch_conv_smoother<double>(h, level, batch, ws, bb, h->nrm, oo, 0, h->w64, s);
    }
    NMG_TRY(ensure_work<float>(h));
    const float* bb = (const float*)b;
    float* oo = (float*)out;
    if (h->kind[(size_t)level] == 1)
        return launch_jacobi<float>(h, level, batch, alpha, h->omega[(size_t)level], bb, oo, 0, h->w32b, s);
    if (prec == NMG_MIXED && h->p.smoother_arch != NMG_ARCH_FNO) {
        // as in the cycle: the BF16 kernel adds the per-image partial sums itself
        NMG_TRY(launch_sumsq_part<float>(h, batch, per, bb, s));
        return launch_mfma_smoother(h, level, batch, ws, bb, h->norm_part, norm_chunks(per), oo, 0, h->w32b, s);
    }
    NMG_TRY(launch_sumsq<float>(h, batch, per, bb, h->nrm, s));
    if (h->p.smoother_arch == NMG_ARCH_FNO) {
        NMG_TRY(ensure_acts<float>(h));
        return launch_fno_smoother<float>(h, level, batch, ws, bb, h->nrm, oo, 0, h->w32b, s);
    }
    NMG_TRY(ensure_acts<float>(h));
    return launch_conv_smoother<float>(h, level, batch, ws, bb, h->nrm, oo, 0, h->w32b, s);
}

nmg_status nmg_apply_fprime(nmg_handle h, int level, int batch, const void* in, void* out, nmg_precision prec,
                            void* stream) {
    NMG_TRY(check_handle(h));
    NMG_TRY(check_batch(h, batch));
    if (!in || !out) return fail(NMG_ERR_ARG, "null pointer");
    if (level < 0 || level >= h->L) return fail(NMG_ERR_ARG, "level out of range");
    hipStream_t s = (hipStream_t)stream;
    if (prec == NMG_FP64) {
        NMG_TRY(ensure_work<double>(h));
        return launch_fprime<double>(h, level, batch, (const double*)in, (double*)out, 0, h->w64, s);
    }
    NMG_TRY(ensure_work<float>(h));
    if (prec == NMG_MIXED && h->p.dim == 2) {
        NMG_TRY(prepare_fprime_bf16(h));
        return launch_fprime_mfma(h, level, batch, (const float*)in, nullptr, (float*)out, 0,
                                  h->w32b.lv[(size_t)level].t1, h->w32b.lv[(size_t)level].t2,
                                  (size_t)h->p.max_batch * level_elems(h, level) * sizeof(float), s);
    }
    return launch_fprime<float>(h, level, batch, (const float*)in, (float*)out, 0, h->w32b, s);
}

nmg_status nmg_vcycle(nmg_handle h, int batch, const double* alpha, const int* ws, const void* y, void* x,
                      const nmg_cycle_opts* o, void* stream) {
    NMG_TRY(check_handle(h));
    NMG_TRY(check_batch(h, batch));
    NMG_TRY(check_opts(h, o));
    if (!alpha || !y || !x) return fail(NMG_ERR_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    if (o->precision == NMG_FP64)
        return run_cycle<double>(h, batch, alpha, ws, (const double*)y, (double*)x, false, *o, s);
    return run_cycle<float>(h, batch, alpha, ws, (const float*)y, (float*)x, false, *o, s);
}

nmg_status nmg_rollout(nmg_handle h, int batch, const double* alpha, const int* ws, const int* k_host, void* e,
                       void* y, const nmg_cycle_opts* o, void* stream) {
    NMG_TRY(check_handle(h));
    NMG_TRY(check_batch(h, batch));
    NMG_TRY(check_opts(h, o));
    if (!alpha || !k_host || !e) return fail(NMG_ERR_ARG, "null pointer");
    if (!h->eng.queue.empty() || !h->eng.slot.empty())
        return fail(NMG_ERR_STATE, "serving requests are queued or active on this handle");
    int kmax = 0;
    for (int i = 0; i < batch; ++i) {
        if (k_host[i] < 0 || k_host[i] > kMaxRollout)
            return fail(NMG_ERR_ARG, "rollout count out of [0, 64] (sample " + std::to_string(i) + ")");
        kmax = std::max(kmax, k_host[i]);
    }
    hipStream_t s = (hipStream_t)stream;
    NMG_TRY(nmg_prepare(h, batch, alpha, stream));
    // the engine's slot tables are idle (no serving work): per-sample counts
    int* kdev = h->slot_i;
    NMG_HIP(hipMemcpyAsync(kdev, k_host, (size_t)batch * sizeof(int), hipMemcpyHostToDevice, s));
    const size_t per = level_elems(h, 0);
    auto run = [&](auto* ep, auto* yp) -> nmg_status {
        using T = std::remove_pointer_t<decltype(ep)>;
        NMG_TRY(ensure_work<T>(h));
        Work<T>& w = work_of<T>(h);
        for (int j = 0; j < kmax; ++j) {
            // d = MG(0, A e); e -= d where j < k
            NMG_TRY(launch_operator<T>(h, 0, batch, alpha, ep, nullptr, w.lv[0].y, 1, w, s));
            NMG_TRY(run_cycle<T>(h, batch, alpha, ws, w.lv[0].y, w.lv[0].x, true, *o, s));
            NMG_TRY(launch_rollout_sub<T>(batch, per, ep, w.lv[0].x, kdev, j, s));
        }
        if (yp) NMG_TRY(launch_operator<T>(h, 0, batch, alpha, ep, nullptr, yp, 1, w, s));
        return NMG_OK;
    };
    if (o->precision == NMG_FP64)
        NMG_TRY(run((double*)e, (double*)y));
    else
        NMG_TRY(run((float*)e, (float*)y));
    NMG_HIP(hipStreamSynchronize(s));
    return NMG_OK;
}

nmg_status nmg_solve(nmg_handle h, int batch, const double* alpha, const int* ws, const double* b, double* x,
                     double rtol, int max_cycles, const nmg_cycle_opts* o, nmg_solve_stats* stats,
                     double* history_host, void* stream) {
    const double t_entry = h ? h->eng.now_ms() : 0.0;
    if (stats)
        for (int i = 0; i < batch && i < (h ? h->p.max_batch : 0); ++i) stats[i] = {0, NMG_NOT_CONVERGED, -1.0, -1.0};
    NMG_TRY(check_handle(h));
    NMG_TRY(check_batch(h, batch));
    NMG_TRY(check_opts(h, o));
    if (!alpha || !b || !x) return fail(NMG_ERR_ARG, "null pointer");
    if (!(rtol > 0.0) || max_cycles < 0) return fail(NMG_ERR_ARG, "rtol must be > 0 and max_cycles >= 0");
    if (!h->eng.queue.empty() || !h->eng.slot.empty())
        return fail(NMG_ERR_STATE, "serving requests are queued or active on this handle");
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> al((size_t)batch);
    std::vector<int> wsv((size_t)batch, 0);
    NMG_HIP(hipMemcpyAsync(al.data(), alpha, (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, s));
    if (ws) NMG_HIP(hipMemcpyAsync(wsv.data(), ws, (size_t)batch * sizeof(int), hipMemcpyDeviceToHost, s));
    NMG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < batch; ++i) {
        NMG_TRY(check_alpha(h, al[(size_t)i], i));
        if (wsv[(size_t)i] < 0 || wsv[(size_t)i] >= h->p.n_weight_sets)
            return fail(NMG_ERR_ARG, "weight set out of range (right-hand side " + std::to_string(i) + ")");
    }
    if (history_host)
        for (size_t i = 0; i < (size_t)batch * (max_cycles + 1); ++i) history_host[i] = -1.0;
    const size_t per = level_elems(h, 0);
    for (int i = 0; i < batch; ++i)
        h->eng.queue.push_back({(long long)i, al[(size_t)i], wsv[(size_t)i], b + (size_t)i * per,
                                x + (size_t)i * per,
                                history_host ? history_host + (size_t)i * (max_cycles + 1) : nullptr, max_cycles + 1,
                                t_entry});
    std::vector<nmg_request_result> done;
    nmg_status st = NMG_OK;
    while (st == NMG_OK && (!h->eng.queue.empty() || !h->eng.slot.empty()))
        st = engine_step(h, rtol, max_cycles, o, done, s);
    if (st != NMG_OK) {
        h->eng.queue.clear();
        h->eng.slot.clear();
        h->eng.precision = -1;
        h->eng.any_ws = false;
        return st;
    }
    // the last step retired every request and synchronised after their copy-out
    int bad = 0;
    for (const auto& r : done) {
        const int i = (int)r.id;
        if (stats) stats[i] = {r.cycles, r.status, r.rel_residual, r.latency_ms};
        bad += r.status != NMG_OK;
    }
    if (bad) {
        int first = -1, fst = 0;
        for (const auto& r : done)
            if (r.status != NMG_OK && (first < 0 || (int)r.id < first)) {
                first = (int)r.id;
                fst = r.status;
            }
        const char* why = fst == NMG_DIVERGED ? "diverged" : (fst == NMG_ERR_NONFINITE ? "non-finite residual"
                                                                                         : "max_cycles reached");
        return fail(NMG_NOT_CONVERGED, std::to_string(bad) + " right-hand side(s) did not converge (first: " +
                                           std::to_string(first) + ", " + why + ")");
    }
    return NMG_OK;
}

nmg_status nmg_serve_submit(nmg_handle h, long long id, double alpha, int weight_set, const double* b_dev,
                            double* x_dev) {
    NMG_TRY(check_handle(h));
    if (!b_dev || !x_dev) return fail(NMG_ERR_ARG, "null pointer");
    NMG_TRY(check_alpha(h, alpha, 0));
    if (weight_set < 0 || weight_set >= h->p.n_weight_sets) return fail(NMG_ERR_ARG, "weight set out of range");
    h->eng.queue.push_back({id, alpha, weight_set, b_dev, x_dev, nullptr, 0, h->eng.now_ms()});
    return NMG_OK;
}

nmg_status nmg_serve_step(nmg_handle h, double rtol, int max_cycles, const nmg_cycle_opts* o,
                          nmg_request_result* done, int* n_done, void* stream) {
    if (n_done) *n_done = 0;
    NMG_TRY(check_handle(h));
    NMG_TRY(check_opts(h, o));
    if (!done || !n_done) return fail(NMG_ERR_ARG, "null result array");
    if (!(rtol > 0.0) || max_cycles < 0) return fail(NMG_ERR_ARG, "rtol must be > 0 and max_cycles >= 0");
    if (!h->serve_retired) NMG_HIP(hipEventCreateWithFlags(&h->serve_retired, hipEventDisableTiming));
    std::vector<nmg_request_result> out;
    std::vector<double> t_sub;
    NMG_TRY(engine_step(h, rtol, max_cycles, o, out, (hipStream_t)stream, h->serve_retired, &t_sub));
    if (!out.empty()) {
        // wait for the copy-out of the finished solutions only (the next
        // iteration queued behind it keeps running); latency ends here
        NMG_HIP(hipEventSynchronize(h->serve_retired));
        const double now = h->eng.now_ms();
        for (size_t i = 0; i < out.size(); ++i) out[i].latency_ms = now - t_sub[i];
    }
    for (size_t i = 0; i < out.size(); ++i) done[i] = out[i];
    *n_done = (int)out.size();
    return NMG_OK;
}

nmg_status nmg_serve_pending(nmg_handle h, int* queued, int* active) {
    NMG_TRY(check_handle(h));
    if (queued) *queued = (int)h->eng.queue.size();
    if (active) *active = (int)h->eng.slot.size();
    return NMG_OK;
}

nmg_status nmg_serve_reset(nmg_handle h) {
    NMG_TRY(check_handle(h));
    h->eng.queue.clear();
    h->eng.slot.clear();
    h->eng.precision = -1;
    h->eng.any_ws = false;
    return NMG_OK;
}

nmg_status nmg_debug_transfer_map(nmg_handle h, int level, int kind, int32_t* idx, float* w) {
    NMG_TRY(check_handle(h));
    if (level < 0 || level >= h->L - 1) return fail(NMG_ERR_ARG, "level must be in [0, L-2]");
    if (!idx || !w) return fail(NMG_ERR_ARG, "null output");
    if (kind != 0 && kind != 1) return fail(NMG_ERR_ARG, "kind must be 0 or 1");
    const int cnt = kind == 0 ? h->n[(size_t)level + 1] : h->n[(size_t)level];
    const int per = kind == 0 ? 3 : 2;
    int32_t* di = nullptr;
    float* dw = nullptr;
    NMG_TRY(dev_alloc(&di, (size_t)cnt * per));
    nmg_status st = dev_alloc(&dw, (size_t)cnt * per);
    if (st == NMG_OK) st = launch_export_maps(h, level, kind, di, dw, nullptr);
    if (st == NMG_OK) {
        hipError_t e1 = hipMemcpy(idx, di, (size_t)cnt * per * sizeof(int32_t), hipMemcpyDeviceToHost);
        hipError_t e2 = hipMemcpy(w, dw, (size_t)cnt * per * sizeof(float), hipMemcpyDeviceToHost);
        if (e1 != hipSuccess) st = hip_fail(e1, "hipMemcpy", __FILE__, __LINE__);
        else if (e2 != hipSuccess) st = hip_fail(e2, "hipMemcpy", __FILE__, __LINE__);
    }
    dev_free(di);
    dev_free(dw);
    return st;
}

nmg_status nmg_debug_option(nmg_handle h, int option, int value) {
    NMG_TRY(check_handle(h));
    if (option == NMG_DEBUG_FP32_HANDOFF)
        h->dbg_fp32_handoff = value != 0;
    else if (option == NMG_DEBUG_SEPARATE_RESTRICT)
        h->dbg_separate_restrict = value != 0;
    else
        return fail(NMG_ERR_ARG, "unknown debug option");
    NMG_HIP(hipDeviceSynchronize());
    release_graphs(h);
    return NMG_OK;
}

nmg_status nmg_set_graphs(nmg_handle h, int enable) {
    NMG_TRY(check_handle(h));
    h->use_graphs = enable != 0;
    if (!h->use_graphs) {
        NMG_HIP(hipDeviceSynchronize());
        release_graphs(h);
    }
    return NMG_OK;
}

nmg_status nmg_profile_enable(nmg_handle h, int on) {
    NMG_TRY(check_handle(h));
    NMG_TRY(prof_resolve(h));
    h->prof_mask = on;
    for (auto& row : h->prof_ms)
        for (auto& v : row) v = 0.0;
    for (auto& row : h->prof_cnt)
        for (auto& v : row) v = 0;
    h->prof_rhs = 0;
    h->prof_iter = 0;
    return NMG_OK;
}

nmg_status nmg_profile_rhs(nmg_handle h, long long* rhs_iterations) {
    NMG_TRY(check_handle(h));
    if (!rhs_iterations) return fail(NMG_ERR_ARG, "null argument");
    *rhs_iterations = h->prof_rhs;
    return NMG_OK;
}

nmg_status nmg_profile_sample(nmg_handle h, int period) {
    NMG_TRY(check_handle(h));
    if (period < 1) return fail(NMG_ERR_ARG, "period must be >= 1");
    h->prof_period = period;
    h->prof_iter = 0;
    return NMG_OK;
}

nmg_status nmg_profile_levels(nmg_handle h, int level_mask) {
    NMG_TRY(check_handle(h));
    NMG_TRY(prof_resolve(h));
    h->prof_levels = level_mask;
    return NMG_OK;
}

nmg_status nmg_profile_query(nmg_handle h, int kind, int level, double* total_ms, int* launches) {
    NMG_TRY(check_handle(h));
    if (kind < 0 || kind > 7) return fail(NMG_ERR_ARG, "unknown kernel kind");
    if (level < -1 || level >= 16) return fail(NMG_ERR_ARG, "level out of range");
    NMG_TRY(prof_resolve(h));
    double ms = 0.0;
    int cnt = 0;
    for (int l = 0; l < 16; ++l)
        if (level < 0 || l == level) {
            ms += h->prof_ms[kind][l];
            cnt += h->prof_cnt[kind][l];
        }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = cnt;
    return NMG_OK;
}

nmg_status nmg_debug_factor(nmg_handle h, int level, int which, double* out, int* radius) {
    NMG_TRY(check_handle(h));
    if (level < 0 || level >= h->L) return fail(NMG_ERR_ARG, "level out of range");
    if (which != 0 && which != 1) return fail(NMG_ERR_ARG, "which must be 0 or 1");
    const Band& B = which == 0 ? h->host[(size_t)level].M : h->host[(size_t)level].G;
    if (radius) *radius = B.r;
    if (out) std::memcpy(out, B.a.data(), B.a.size() * sizeof(double));
    return NMG_OK;
}

}  // extern "C"
