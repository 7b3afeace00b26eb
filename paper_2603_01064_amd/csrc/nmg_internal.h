// Internal declarations of the neural multigrid library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <string>
#include <deque>
#include <chrono>
#include <map>
#include <vector>

#include "../../include/nmg.h"

namespace nmg {

// ---------------------------------------------------------------------------
// Error plumbing: every internal call returns nmg_status; messages go to a
// thread-local string read by nmg_last_error().
// ---------------------------------------------------------------------------
nmg_status fail(nmg_status code, const std::string& msg);
nmg_status hip_fail(hipError_t e, const char* what, const char* file, int line);

#define NMG_HIP(...)                                                         \
    do {                                                                     \
        hipError_t _e = (__VA_ARGS__);                                       \
        if (_e != hipSuccess) return ::nmg::hip_fail(_e, #__VA_ARGS__, __FILE__, __LINE__); \
    } while (0)

#define NMG_TRY(...)                                                         \
    do {                                                                     \
        nmg_status _s = (__VA_ARGS__);                                       \
        if (_s < 0) return _s;                                               \
    } while (0)

// ---------------------------------------------------------------------------
// Host-side hierarchy (FP64): banded Galerkin factors of
// A_l = alpha M_l (x) M_l + G_l (x) G_l  (1D: alpha M_l + G_l).
// ---------------------------------------------------------------------------
struct Band {
    int n = 0;   // rows
    int r = 0;   // radius
    std::vector<double> a;  // a[i*(2r+1) + (j - i + r)]
    double get(int i, int j) const {
        int d = j - i;
        if (i < 0 || j < 0 || i >= n || j >= n || d < -r || d > r) return 0.0;
        return a[(size_t)i * (2 * r + 1) + (d + r)];
    }
};

// A band matrix written as a Toeplitz part (coefficients t[d + r] of the
// interior rows) plus corrections confined to the top-left and bottom-right
// rc x rc corners: B = T + D_TL + D_BR.  Zero boundary values make the
// Gaussian factor K^T K differ from its Toeplitz interior only there, and
// Galerkin products keep that form.
struct ToeplitzSplit {
    bool ok = false;
    int r = 0, rc = 0;
    std::vector<double> t;        // 2r+1
    std::vector<double> dtl, dbr; // rc x rc, row-major (row = first index)
};
bool split_toeplitz(const Band& B, ToeplitzSplit& out);

struct HostLevel {
    int n = 0;
    Band M, G;
    ToeplitzSplit Ms, Gs;
};

// Builds taps, G_1 = K K, M_1 = I and the Galerkin chain; returns false with
// a message on invalid input.
bool build_host_hierarchy(int n, double s, double trunc, int levels, int dim, int form, std::vector<HostLevel>& out,
                          int* taps_radius, double* alpha_floor, std::string& err);

// ---------------------------------------------------------------------------
// Device-side state
// ---------------------------------------------------------------------------
template <typename T>
struct LevelBuffers {
    T* x = nullptr;   // iterate / correction on this level
    T* y = nullptr;   // right-hand side on this level
    T* b = nullptr;   // residual work
    T* h = nullptr;   // smoother output (for F')
    T* t1 = nullptr;  // axis-pass temporary
    T* t2 = nullptr;  // axis-pass temporary
};

// Device form of a level's operator for the tiled residual kernel.
template <typename T>
struct TiledOp {
    bool ok = false;        // Toeplitz + corner tables exist (2D, exact split)
    bool fused_ok = false;  // the generic one-launch tile kernel fits in LDS
    int rg = 0, rgp = 0, rc = 0, rm = 0, rmp = 0, m_ident = 0;
    T *tg = nullptr, *dtl = nullptr, *dbr = nullptr, *tm = nullptr;  // into one allocation
    T* base = nullptr;
};

template <typename T>
struct Work {
    bool ready = false;
    std::vector<LevelBuffers<T>> lv;
    T* act0 = nullptr;   // conv activations ping
    T* act1 = nullptr;   // conv activations pong
    T* Gd = nullptr;     // per level band tables, concatenated
    T* Md = nullptr;
    std::vector<size_t> g_off, m_off;
    T* dct = nullptr;    // per level DCT-II matrices [n][n], concatenated
    std::vector<size_t> dct_off;
    T* wts = nullptr;    // smoother weights in this precision [L-1][sets][count]
    std::vector<TiledOp<T>> tiled;
    // FNO smoother: activations ping-pong [B][C][per0], truncated-DFT
    // intermediates and per-level cos / sin (2 pi q / n) tables
    bool fno_ready = false;
    T *fz0 = nullptr, *fz1 = nullptr, *fta = nullptr, *fxh = nullptr, *fyh = nullptr, *fcd = nullptr;
    T* ftab = nullptr;
    std::vector<size_t> ftab_off;
    T* fsp = nullptr;             // spectral part of a layer's output [B][C][per0]
    T* fwt = nullptr;             // one layer's convolution weights as [set][ci][tap][co] (2D)
    // FNO training: per-layer activations Z_0..Z_NL, pre-activations, spectra,
    // and the adjoint's work planes
    bool ftr_ready = false;
    T *ftz = nullptr, *ftp = nullptr, *ftx = nullptr, *ftgz = nullptr, *ftgp = nullptr, *ftga = nullptr;
    T *ftgx = nullptr, *ftgy = nullptr, *ftgo = nullptr, *ftgs = nullptr;
    T* fmat = nullptr;            // per level dense column-transform matrices
    std::vector<size_t> fmat_off;
};

// Serving engine: requests wait in a host queue and are admitted into free
// batch slots between outer iterations; slots [0, k) are the active ones.
struct EngineRequest {
    long long id;
    double alpha;
    int ws;
    const double* b;
    double* x;
    double* hist;  // host row of residual history or null
    int hist_len;
    double t_submit;
};
struct EngineSlot {
    long long id = 0;
    double* x = nullptr;
    double* hist = nullptr;
    int hist_len = 0;
    int cycles = 0;
    double alpha = 0.0, bn2 = 0.0, rn2 = 0.0;
    int ws = 0, fidx = 0;
    double t_submit = 0.0;
};
struct Engine {
    std::deque<EngineRequest> queue;
    std::vector<EngineSlot> slot;
    int precision = -1;  // cycle precision of the active slots
    bool any_ws = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

struct Ctx {
    nmg_problem p{};
    int L = 0;
    int ny0 = 0;                       // rows of the finest grid (n or 1)
    std::vector<int> n;                // points per axis per level
    std::vector<HostLevel> host;
    int taps_radius = 0;
    double alpha_floor = 0.0;  // alphas at or below it leave the fine operator indefinite
    // smoother description
    int wcount = 0;                    // weights per (level, set)
    std::vector<int> layer_off;        // offset of each layer in a weight block
    int cmax = 1;                      // widest layer
    std::vector<int> kind;             // per level: 0 neural, 1 jacobi, -1 unset
    std::vector<double> omega;
    std::vector<std::vector<char>> loaded;  // [level][set]
    // FP32 master weights, gradients and Adam moments [L-1][sets][wcount]
    float* w32 = nullptr;
    float* g32 = nullptr;
    double* g64 = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    std::vector<int> adam_step;        // per set
    bool dbg_fp32_handoff = false;     // nmg_debug_option NMG_DEBUG_FP32_HANDOFF
    bool dbg_separate_restrict = false;  // nmg_debug_option NMG_DEBUG_SEPARATE_RESTRICT
    uint16_t* dctbf = nullptr;         // BF16 DCT-II matrices C and C^T per level (padded)
    std::vector<size_t> dctbf_off;
    float* ramp = nullptr;             // sqrt(k / n_l) per level (F' mask)
    std::vector<size_t> ramp_off;
    uint16_t* wbf = nullptr;           // BF16 MFMA-packed weights
    size_t wbf_stride = 0;             // per (level, set)
    // coarse solve
    int nc = 0;                        // coarse unknowns n_L^dim
    double* Mc = nullptr;              // dense n_L x n_L
    double* Gc = nullptr;
    double* chol = nullptr;            // [max_batch][nc][nc] lower factor, row-major
    double* cholT = nullptr;           // [max_batch][nc][nc] its transpose
    double* cinv = nullptr;            // [max_batch][nc][nc] A_L^{-1} (FP32 / mixed cycles)
    double* cwork = nullptr;           // [max_batch][nc][nc] L^{-1} scratch
    int* flags = nullptr;              // [max_batch] non-SPD / non-finite flags per new factor
    // coarsest grids beyond the dense factor (2D, n_L^2 > 1024): exact solve in
    // the simultaneous eigenbasis V of (M_L, G_L), any alpha, no factors
    bool eig_coarse = false;
    double* eigV = nullptr;            // [n_L][n_L] row-major
    double* eigLam = nullptr;          // [n_L]
    double* eigT = nullptr;            // [2][max_batch][n_L][n_L] stage scratch
    double* alpha_prepared = nullptr;  // [max_batch] alphas of the factors being computed
    int* slot_dev = nullptr;           // [max_batch] cache slots of the factors being computed
    int* coarse_idx = nullptr;         // [max_batch] cache slot of each right-hand side
    const int* cycle_fidx = nullptr;   // factor index per batch slot used by the cycle (null: coarse_idx)
    std::vector<int> coarse_idx_host;  // host copy of coarse_idx from the last prepare
    std::vector<double> alpha_host;    // alphas of the last prepare
    // coarse-factor cache: slot k holds the factors of alpha cache_alpha[k]
    std::vector<double> cache_alpha;   // NaN = empty
    std::vector<long long> cache_used; // last use (prepare counter)
    long long prepare_count = 0;
    // norms and scratch
    double* nrm = nullptr;             // [max_batch] per right-hand-side norms
    double* nrm2 = nullptr;            // [max_batch] second norm slot
    double* norm_part = nullptr;       // [max_batch][max(kResidualNormParts, kNormChunksMax)] partial sums
    double* x64 = nullptr;             // [max_batch][ny][n] compacted FP64 iterates (solve)
    double* b64 = nullptr;             // [max_batch][ny][n] compacted FP64 right-hand sides (solve)
    // slot tables, one device block: slot_d [3][max_batch] alpha, ||b||^2,
    // ||r||^2 per compacted slot, then slot_i [2][max_batch] weight set, factor
    // index and [2][max_batch] x 2 move lists (slot_i points into slot_d's block)
    double* slot_d = nullptr;
    int* slot_i = nullptr;
    // pinned host staging of the engine (rewritten only after a stream sync),
    // one block laid out like the device one, so the per-iteration tables go
    // up in one copy: pin_d [3B] slot tables, pin_i [6B] slot tables and move
    // lists, then pin_rd [B] residual norms, [B] right-hand-side norms read
    // back; pin_ptr [B] destinations
    double* pin_d = nullptr;
    int* pin_i = nullptr;
    double* pin_rd = nullptr;
    double** pin_ptr = nullptr;
    double** xptr_dev = nullptr;       // [max_batch] destinations of finished iterates
    Engine eng;
    float* xs32 = nullptr;             // [max_batch][ny][n] plain-FP32 iterate
    float* bs32 = nullptr;             // [max_batch][ny][n] plain-FP32 right-hand side
    double* r64 = nullptr;
    double* hist_dev = nullptr;        // [max_batch] residual snapshot
    int* active = nullptr;             // [max_batch]
    // training scratch
    double* loss_dev = nullptr;        // [L-1]
    Work<double> w64;
    Work<float> w32b;
    bool grad_is_fp64 = false;         // which gradient buffer the last loss_grad filled
    // profiler
    int prof_mask = 0;         // bit k: time kernel family k
    int prof_levels = 0xFFFF;  // bit l: time launches on level l
    int prof_period = 1;       // time every prof_period-th solve iteration
    long long prof_iter = 0;   // solve iterations seen since profiling was enabled
    long long prof_rhs = 0;    // active right-hand sides summed over the timed solve iterations
    struct ProfEv { hipEvent_t a, b; int kind, level; };
    std::vector<ProfEv> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[8][16] = {};
    int prof_cnt[8][16] = {};
    // captured solve iterations (refine scale, cycle, update, next residual)
    // inside graphs the profiler brackets a launch with two tiny kernels that
    // store the device wall clock into stamp slots (first, first + 1)
    struct StampEv { int first, kind, level; };
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        std::vector<StampEv> stamps;
    };
    std::map<std::vector<long long>, GraphEntry> graphs;
    bool use_graphs = true;
    bool capturing = false;
    std::vector<StampEv> capture_stamps;
    std::vector<StampEv> stamp_pending;
    long long* stamps = nullptr;       // [kStampSlots] device wall-clock stamps
    int stamp_next = 0;
    double wall_khz = 0.0;
    hipStream_t cap_stream = nullptr;
    hipEvent_t serve_retired = nullptr;  // copy-out of finished serving requests
};

// Records a start event on construction and a stop event on destruction
// when profiling is on.
constexpr int kStampSlots = 8192;
struct ProfScope {
    Ctx* c;
    hipStream_t s;
    int kind, level;
    hipEvent_t a = nullptr, b = nullptr;
    int stamp = -1;
    ProfScope(const Ctx* cc, hipStream_t ss, int k, int l);
    ~ProfScope();
};
nmg_status prof_resolve(Ctx* c);
void release_graphs(Ctx* c);
void launch_stamp(long long* slot, hipStream_t s);

template <typename T>
Work<T>& work_of(Ctx* c);
template <typename T>
nmg_status ensure_work(Ctx* c);
template <typename T>
nmg_status ensure_acts(Ctx* c);
// FNO smoother (fno.hip)
size_t fno_weight_count(const nmg_problem& p);
int fno_level_modes(const Ctx* c, int l);
template <typename T>
nmg_status ensure_fno(Ctx* c);
template <typename T>
nmg_status launch_fno_smoother(const Ctx* c, int l, int batch, const int* ws, const T* b, const double* nrm2, T* dst,
                               int accumulate, Work<T>& w, hipStream_t s);
// Weight gradient of the FNO smoother of level l (weight set `set`) for the
// upstream gradient dL/dh (scaled by `sign`) of h = ||b|| N(b / ||b||);
// accumulates into grad (the level's block) unless `accumulate` is 0.
template <typename T>
nmg_status fno_backward(Ctx* c, Work<T>& w, int l, int set, int batch, const T* b, const double* nrm2,
                        const T* upstream, T sign, int accumulate, T* grad, hipStream_t s);
void release_training(const Ctx* c);

size_t level_elems(const Ctx* c, int l);  // ny_l * n_l

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
constexpr int kNormChunksPerRhs = 32;
// chunks of the two-stage norm of an image of `per` elements: 32 up to 511^2,
// more on larger images so that the first stage fills the GPU at small
// batches; a function of the image size only, so the partial sums (and the
// norm) do not depend on the batch
constexpr int kNormChunksMax = 256;
inline int norm_chunks(size_t per) {
    return per >= ((size_t)1 << 21) ? 256 : per >= ((size_t)1 << 19) ? 64 : kNormChunksPerRhs;
}
// at most this many partial sums of ||out||^2 per image from launch_operator
constexpr int kResidualNormParts = 64;
// mode 0: out = y - A x ; mode 1: out = A x.  With norm_part and nparts, the
// FP32 one-launch form also writes partial sums of ||out||^2, one per 32 x 32
// block of the image, to norm_part[b][*nparts] (fixed order whatever the
// batch); *nparts = 0 where it does not (other forms, or more blocks than
// kResidualNormParts)
template <typename T>
nmg_status launch_operator(const Ctx* c, int l, int batch, const double* alpha, const T* x, const T* y,
                           T* out, int mode, Work<T>& w, hipStream_t s, double* norm_part = nullptr,
                           int* nparts = nullptr);
// mirror (optional): the sums also into pinned host memory (see k_sumsq_final)
template <typename T>
nmg_status launch_sumsq(const Ctx* c, int batch, size_t elems, const T* v, double* out, hipStream_t s,
                        double* mirror = nullptr);
// first stage only: c->norm_part[b][norm_chunks(elems)]
template <typename T>
nmg_status launch_sumsq_part(const Ctx* c, int batch, size_t elems, const T* v, hipStream_t s);
template <typename T>
nmg_status launch_restrict(const Ctx* c, int l, int batch, const T* r, T* yc, hipStream_t s,
                           double* norm_part = nullptr);
// number of partial sums launch_restrict writes per image for level l -> l + 1
int restrict_norm_parts(const Ctx* c, int l);
template <typename T>
nmg_status launch_prolong_transpose(const Ctx* c, int l, int batch, const T* g, T* out, hipStream_t s);
template <typename T>
nmg_status launch_dense_axis(const T* in, T* out, const T* C, int n, int ny, int batch, int col_axis, int inverse,
                             hipStream_t s);
template <typename T>
// x += P e (set: x = P e)
nmg_status launch_prolong_add(const Ctx* c, int l, int batch, const T* e, T* x, hipStream_t s, bool set = false);
template <typename T>
nmg_status launch_axpy(int batch, size_t elems, const T* src, T* dst, int accumulate, hipStream_t s);
template <typename T>
nmg_status launch_conv_smoother(const Ctx* c, int l, int batch, const int* ws, const T* b, const double* nrm2,
                                T* dst, int accumulate, Work<T>& w, hipStream_t s);
// nparts == 0: nrm2[b] is ||b||^2 of image b; nparts > 0: nrm2 holds the
// [batch][nparts] partial sums of launch_sumsq_part, which the kernel adds in
// the order k_sumsq_final uses (same value, one launch fewer)
// dstb != nullptr: write h as a zero-padded BF16 bpitch x bpitch plane per
// image (the input of the MFMA filter F', fragment-tiled when btiled)
// instead of the FP32 array dst
nmg_status launch_mfma_smoother(const Ctx* c, int l, int batch, const int* ws, const float* b,
                                const double* nrm2, int nparts, float* dst, int accumulate, Work<float>& w,
                                hipStream_t s, uint16_t* dstb = nullptr, int bpitch = 0, bool btiled = false);
// Fused FP64 refinement residual on level 0 (x += ||r|| d for active slots,
// r = y - A x, ||r||^2 into nrm2); false when it does not apply (nothing launched)
bool refine_residual_fusable(const Ctx* c, const Work<double>& w);
template <typename D>
bool launch_refine_residual(const Ctx* c, int batch, const double* alpha, double* x, const D* d,
                            const double* rn2, const int* active, const double* y, double* out, double* nrm2,
                            Work<double>& w, hipStream_t s, double* mirror = nullptr);
// Mixed-precision backward of the CNN smoother on MFMA (train_mfma.hip):
// buffers and weights of one level and weight set.
struct MfmaBackwardArgs {
    int n = 0, batch = 0, accumulate = 0;
    const float* b = nullptr;        // smoother input of the level [B][n][n]
    const double* nrm2 = nullptr;    // ||b||^2 per right-hand side
    const float* W = nullptr;        // FP32 master weights of the level and set (layer_off order)
    float* grad = nullptr;           // weight gradient, same order (stored or added)
    const float* dout = nullptr;     // delta at the network output [B][n][n]
    float* din0 = nullptr;           // optional: gradient at the network input u = b / ||b||
    std::vector<uint16_t*> acts;     // n_layers - 1 activation record buffers [B][n*n][32] BF16
    uint16_t *d0 = nullptr, *d1 = nullptr;  // delta record buffers, same shape
    uint16_t* wpk = nullptr;         // packed hidden-layer weights (mfma_backward_wpk_elems)
    float* part = nullptr;           // weight-gradient partials
    size_t part_count = 0;
    double* reduce_tmp = nullptr;    // mfma_backward_reduce_elems doubles
};
size_t mfma_backward_reduce_elems();
bool mfma_backward_supported(const Ctx* c);
size_t mfma_backward_wpk_elems(const Ctx* c);
nmg_status smoother_backward_mfma(const Ctx* c, const MfmaBackwardArgs& a, hipStream_t s);
// whether the smoother's tiles of level l cover a padded pitch x pitch plane
bool mfma_smoother_covers(const Ctx* c, int l, int pitch);
template <typename T>
nmg_status launch_jacobi(const Ctx* c, int l, int batch, const double* alpha, double omega, const T* b, T* dst,
                         int accumulate, Work<T>& w, hipStream_t s);
template <typename T>
nmg_status launch_fprime(const Ctx* c, int l, int batch, const T* h, T* dst, int accumulate, Work<T>& w,
                         hipStream_t s);
nmg_status prepare_fprime_bf16(Ctx* c);
nmg_status launch_fprime_mfma(const Ctx* c, int l, int batch, const float* h, const uint16_t* hb, float* dst,
                              int accumulate, void* t1, void* t2, size_t scratch_bytes, hipStream_t s);
// scratch bytes launch_fprime_mfma needs (t1 + t2) for `batch` images of side n
size_t fprime_mfma_scratch_bytes(int n, int batch);
// whether the BF16 F' input plane of a level of side n uses the fragment-tiled
// layout (sides 65..511) rather than row-major
bool fprime_tiled_layout(int n);
// resolves the device address of the no-allocation F' scratch on the current
// device (once per device)
nmg_status fprime_noalloc_init();
nmg_status launch_export_maps(const Ctx* c, int l, int kind, int32_t* idx, float* w, hipStream_t s);
nmg_status launch_coarse_factor(Ctx* c, int count, const double* alphas, const int* slots, hipStream_t s);
bool coarse_eigenbasis(const Band& M, const Band& G, std::vector<double>& V, std::vector<double>& lam,
                       std::string& err);
template <typename T>
nmg_status launch_eig_coarse(const Ctx* c, int batch, const double* alpha, const T* y, T* x, hipStream_t s);
// Restriction chain (2D): y[k + 1] = R y[k] for k = 0 .. levels - 2 in one
// launch, one workgroup per right-hand side, and, with x_coarse, the
// eigenbasis solve of the last grid into x_coarse.  n[1] <= kChainMax; with
// x_coarse the last side is at most eig_small_max().
constexpr int kChainLevels = 8;
constexpr int kChainMax = 64;
template <typename T>
struct RestrictChain {
    int levels = 0;                   // grids in the chain: the level read and every level below it
    int n[kChainLevels] = {};         // their sides
    T* y[kChainLevels] = {};          // right-hand sides (y[0] read, the others written)
    T* x_coarse = nullptr;            // coarsest solution when the solve is fused, else null
};
template <typename T>
nmg_status launch_restrict_chain(const Ctx* c, int batch, const double* alpha, const RestrictChain<T>& ch,
                                 hipStream_t s);
int eig_small_max();
nmg_status launch_coarse_inverse(Ctx* c, int count, const int* slots, hipStream_t s);
template <typename T>
nmg_status launch_coarse_apply_inverse(const Ctx* c, int batch, const T* y, T* x, hipStream_t s);
template <typename T>
nmg_status launch_coarse_solve(const Ctx* c, int batch, const T* y, T* x, hipStream_t s);
template <typename T>
nmg_status launch_zero(T* p, size_t count, hipStream_t s);
template <typename A, typename B>
nmg_status launch_convert(const A* src, B* dst, size_t count, hipStream_t s);
template <typename T>
nmg_status launch_move_slots(int count, size_t per, T* a, T* b, T* c, const int* moves, hipStream_t s);
template <typename T>
nmg_status launch_scatter_slots(int count, size_t per, const T* xc, double* x, const int* pairs, hipStream_t s);
template <typename T>
nmg_status launch_scatter_ptrs(int count, size_t per, const T* xc, double* const* dst, const int* slots,
                               hipStream_t s);
nmg_status factor_alphas(Ctx* h, const std::vector<double>& al, std::vector<int>& idx, hipStream_t s);
nmg_status check_opts(const Ctx* c, const nmg_cycle_opts* o);
nmg_status check_alpha(const Ctx* h, double a, int slot);
// One continuous-batching step on stream s; `retired`, when given, is
// recorded on s once the solutions of the requests returned in `done` have
// been written (before the next iteration is launched).  submit_ms, when
// given, receives each returned request's submission time (engine clock).
nmg_status engine_step(Ctx* h, double rtol, int max_cycles, const nmg_cycle_opts* o,
                       std::vector<nmg_request_result>& done, hipStream_t s, hipEvent_t retired = nullptr,
                       std::vector<double>* submit_ms = nullptr);
// Device bytes one request slot of the handle occupies in a solve of the
// given precision (engine planes plus the cycle's level buffers).
size_t request_bytes(const Ctx* c, nmg_precision prec);
template <typename R, typename T>
nmg_status launch_refine_scale(int batch, size_t per, const R* r, T* y, const double* rn2, const double* bn2,
                               double rtol, int* active, hipStream_t s, double* part = nullptr);
template <typename X, typename T>
nmg_status launch_refine_update(int batch, size_t per, X* x, const T* d, const double* rn2, const int* active,
                                hipStream_t s);
template <typename T>
nmg_status launch_rollout_sub(int batch, size_t per, T* e, const T* d, const int* k, int j, hipStream_t s);
nmg_status repack_bf16(Ctx* c, int level, int weight_set);

}  // namespace nmg

struct nmg_ctx : public nmg::Ctx {};
