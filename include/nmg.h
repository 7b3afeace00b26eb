/*
 * nmg.h - C ABI of the MI355X (gfx950) neural multigrid library.
 *
 * The library solves the regularised convolution system
 *     (K^T K + alpha I) u = b
 * arising from a convolution-type integral equation with a truncated
 * Gaussian kernel (paper Sec. 2.1; 2D Kronecker form K2 = K (x) K of Sec. 4.2)
 * by V-cycles whose smoothers are learned per-level CNNs (Algorithms 2-4),
 * with full-weighting restriction, linear interpolation, Galerkin coarse
 * operators (Algorithm 1) and an exact solve on the coarsest grid.
 *
 * Conventions shared by every entry point
 *  - Grids have n = 2^k - 1 interior points per axis, mesh h = 1/(n+1),
 *    zero boundary values.  Level l+1 has (n_l - 1)/2 points per axis.
 *  - Batched device arrays are contiguous [B][n] (dim 1) or [B][n][n]
 *    (dim 2, row-major [row][col]); per right-hand-side scalars are [B].
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller.  The library
 *    owns everything it allocates inside a handle and frees it in
 *    nmg_destroy.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Work is enqueued asynchronously unless an entry point says it
 *    synchronises.
 *  - Errors: every call returns an nmg_status; negative values are errors
 *    and leave outputs unspecified, NMG_NOT_CONVERGED is a warning with the
 *    last iterate written.  All argument and shape checks happen on the host
 *    before any launch.  nmg_last_error() gives a thread-local message.
 *  - A handle is not thread-safe; use one handle per host thread/stream.
 */
#ifndef NMG_H
#define NMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmg_ctx* nmg_handle;

typedef enum {
    NMG_OK = 0,
    NMG_NOT_CONVERGED = 1,
    NMG_DIVERGED = 2,        /* per right-hand side: residual beyond the guard */
    NMG_ERR_ARG = -1,        /* bad argument value or NULL pointer        */
    NMG_ERR_SHAPE = -2,      /* n, levels, batch or layer shapes invalid  */
    NMG_ERR_OOM = -3,        /* device allocation failed                  */
    NMG_ERR_NOT_SPD = -4,    /* alpha leaves an operator indefinite       */
    NMG_ERR_NONFINITE = -5,  /* NaN/Inf in an input or a residual         */
    NMG_ERR_HIP = -6,        /* HIP runtime error                         */
    NMG_ERR_BUDGET = -7,     /* request exceeds the handle's HBM budget   */
    NMG_ERR_STATE = -8       /* call out of order (e.g. no weights yet)   */
} nmg_status;

/* Arithmetic of a cycle.
 *  NMG_FP64  : everything in FP64 (parity path).
 *  NMG_FP32  : plain FP32 cycle and FP32 smoother; FP64 coarse solve.
 *  NMG_MIXED : BF16 smoother on MFMA with FP32 accumulation, FP32 residuals
 *              and transfers, FP64 coarse solve; nmg_solve wraps it in FP64
 *              iterative refinement. */
typedef enum { NMG_FP64 = 0, NMG_FP32 = 1, NMG_MIXED = 2 } nmg_precision;

typedef enum { NMG_MASK_BAND = 0, NMG_MASK_RAMP = 1, NMG_LOSS_CYCLE = 2 } nmg_mask_kind;

#define NMG_MAX_LAYERS 7

/* Problem and smoother architecture fixed for the lifetime of a handle. */
/* Fine-grid operator (Sec. 2.1; 2D Kronecker form of Sec. 4.2).  K is the
 * truncated Gaussian convolution (Toeplitz, zero boundary values).
 *  NMG_OP_NORMAL : A = alpha I + K^T K (2D: alpha I + (K(x)K)^T (K(x)K)),
 *                  the Tikhonov normal equations; SPD for every alpha > 0.
 *  NMG_OP_KERNEL : A = alpha I + K (2D: alpha I(x)I + K(x)K), the form the
 *                  paper writes.
 *  NMG_OP_ANISO  : A = alpha D + K, 1D only (Sec. 4.1, anisotropic case): D
 *                  is the three-point -(a u')' with a(z) = 1 + 0.5 sin 2 pi z
 *                  at cell midpoints, without the 1/h^2 factor.
 * The truncated Gaussian K can be slightly indefinite (lowest eigenvalue
 * about -3e-5 at s/h = 2.56), so the last two forms are SPD only for alpha
 * above a floor, which setup computes to about 1e-16 (host band Cholesky,
 * bisection on alpha in 1D and on the ends of the spectrum of K in 2D).
 * Every entry point that takes alphas for a solve (nmg_prepare, nmg_solve,
 * nmg_serve_submit) rejects one at or below the floor with NMG_ERR_NOT_SPD.
 * The Galerkin levels below the finest inherit definiteness. */
typedef enum { NMG_OP_NORMAL = 0, NMG_OP_KERNEL = 1, NMG_OP_ANISO = 2 } nmg_operator_form;

typedef struct {
    int dim;                         /* 1 or 2                                   */
    int n;                           /* interior points per axis, 2^k - 1        */
    double s;                        /* Gaussian width, unit-interval units      */
    double trunc;                    /* truncation radius in units of s (e.g. 4) */
    int levels;                      /* L >= 1; n_L >= 1                         */
    int max_batch;                   /* right-hand sides per call                */
    int n_layers;                    /* smoother conv layers, 1..NMG_MAX_LAYERS  */
    int channels[NMG_MAX_LAYERS + 1];/* channels[0] = channels[n_layers] = 1     */
    int ksize;                       /* odd convolution kernel size              */
    int n_weight_sets;               /* independent smoother sets per level      */
    int operator_form;               /* nmg_operator_form (0: the default below) */
    int smoother_arch;               /* nmg_smoother_arch (0: the CNN above)     */
    int fno_width;                   /* FNO: channels C                          */
    int fno_layers;                  /* FNO: Fourier layers                      */
    int fno_modes;                   /* FNO: retained modes per axis, k          */
    int fno_ksize;                   /* FNO: odd size of the convolution W       */
} nmg_problem;

/* Smoother network N of h = ||b|| N(b / ||b||).
 *  NMG_ARCH_CNN : bias-free ReLU CNN of n_layers convolutions (channels,
 *                 ksize); BF16 MFMA kernels in mixed precision.
 *  NMG_ARCH_FNO : Fourier neural operator (Sec. 3.1; network description
 *                 of the appendix): pointwise lift 1 -> C with bias, then
 *                 fno_layers Fourier layers
 *                   z <- GELU(DFT^-1 R DFT z + W z + B)
 *                 with the real DFT of the level's grid values, R complex on
 *                 the k_l = min(fno_modes, n_l / 2) lowest modes per axis
 *                 (2D: rows [0, k_l) and [n_l - k_l, n_l) of the half
 *                 spectrum times columns [0, k_l)), W a same-padded
 *                 fno_ksize convolution C -> C and B a bias, then a pointwise
 *                 projection C -> 1 with bias (C <= 256, k <= 128).  Runs in FP32 (also inside
 *                 mixed-precision cycles) or FP64; not trainable here.
 *                 Weight block per (level, set), float, in this order:
 *                   lift_w[C], lift_b[C],
 *                   per layer: R_re[RM], R_im[RM], W[C][C][ks(][ks)], B[C]
 *                     with RM = 2*C*C*k*k in 2D ([corner][ci][co][u][v],
 *                     corner 1 = rows n - k + u) and C*C*k in 1D ([ci][co][v]),
 *                     k = fno_modes (a level uses the leading k_l x k_l),
 *                   proj_w[C], proj_b.
 *                 The CNN fields must still describe a valid CNN (they are
 *                 ignored). */
typedef enum { NMG_ARCH_CNN = 0, NMG_ARCH_FNO = 1 } nmg_smoother_arch;

/* Options of one V(nu1, nu2) cycle (Algorithm 1 with the neural smoothing
 * step of Algorithms 2-4; use_fprime enables the filter F'_l of Algorithms 3
 * and 4 on every smoother output). */
typedef struct {
    int nu1;
    int nu2;
    int use_fprime;
    nmg_precision precision;
} nmg_cycle_opts;

/* ---- setup ------------------------------------------------------------- */

/* Builds the grid hierarchy (Sec. 2.3 / Algorithm 1): Gaussian taps, the
 * banded factor G_1 = K^T K, the Galerkin factors M_l, G_l of
 * A_l = alpha M_l (x) M_l + G_l (x) G_l, device copies and workspaces for
 * max_batch right-hand sides.  Synchronises.  *out receives the handle.
 * The exact coarsest solve of Algorithm 1: in 2D (coarsest n_L up to 511)
 * in the simultaneous eigenbasis V of (M_L, G_L), computed once on the host
 * and independent of alpha: x = V [(V^T y V) / (alpha + lam_i lam_j)] V^T;
 * in 1D a dense FP64 Cholesky factor per alpha (n_L <= 1024),
 * four FP64 products per right-hand side and nothing to factor per alpha.
 * Errors: NMG_ERR_SHAPE (n not 2^k-1, too many levels, coarsest grid too
 * large, bad channels), NMG_ERR_ARG, NMG_ERR_OOM, NMG_ERR_HIP. */
nmg_status nmg_setup_hierarchy(const nmg_problem* problem, nmg_handle* out);

/* Frees every device and host resource of the handle (NULL is ignored). */
void nmg_destroy(nmg_handle h);

/* Thread-local description of the last error returned on this thread. */
const char* nmg_last_error(void);

/* Copies the CNN weights of smoother N_theta_l (level 0-based, l < L-1) of
 * weight set `weight_set` from host memory.  Layout: all layers
 * concatenated, layer i as [C_{i+1}][C_i][k] (dim 1) or [C_{i+1}][C_i][k][k]
 * (dim 2), cross-correlation, no bias (Algorithm 2's smoother, Appendix A's
 * convolution operator W).  `count` must equal the total weight count.
 * Selects the neural smoother for that level.  Synchronises. */
nmg_status nmg_load_smoother_weights(nmg_handle h, int level, int weight_set,
                                     const float* weights_host, size_t count);

/* Copies the current FP32 weights of (level, weight_set) back to the host. */
nmg_status nmg_get_smoother_weights(nmg_handle h, int level, int weight_set,
                                    float* weights_host, size_t count);

/* Selects the weighted Jacobi smoother h = omega D_l^{-1} b of Sec. 2.2 on
 * level `level` (omega > 0), in place of the neural smoother. */
nmg_status nmg_set_jacobi_smoother(nmg_handle h, int level, double omega);

/* Coarse preparation for the right-hand sides b < batch.  1D: for every
 * distinct alpha[b] forms A_L = alpha M_L + G_L and its FP64 Cholesky factor
 * (Algorithm 1, exact coarsest solve), plus the FP64 inverse used by FP32 /
 * mixed cycles; factors are cached per alpha value (up to max_batch of
 * them), so repeated alphas cost nothing.  2D: the eigenbasis solve needs no
 * factor, and this only checks the alphas.  alpha: device
 * double[batch].  Must precede nmg_vcycle for these right-hand sides
 * (nmg_solve calls it itself).  Synchronises; NMG_ERR_ARG for alpha <= 0 or
 * non-finite, NMG_ERR_NOT_SPD if a pivot is not positive (1D) or alpha is
 * at or below the operator's floor. */
nmg_status nmg_prepare(nmg_handle h, int batch, const double* alpha_dev, void* stream);

/* ---- operators ---------------------------------------------------------- */

/* y = A_l x on level `level` for every right-hand side (alpha device
 * double[batch]).  x, y: device [B][n_l]([n_l]) of type double (NMG_FP64)
 * or float (otherwise).  Used to form b = A u* and training pairs. */
nmg_status nmg_apply_operator(nmg_handle h, int level, int batch, const double* alpha_dev,
                              const void* x, void* y, nmg_precision precision, void* stream);

/* h = ||b||_2 N_theta_l(b / ||b||_2) per right-hand side: the neural
 * smoothing step of Algorithm 2 / Algorithm 4 on level `level` (l < L-1),
 * or omega D_l^{-1} b if that level uses weighted Jacobi (Sec. 2.2).  b, h:
 * device [B][n_l]([n_l]); double for NMG_FP64, float otherwise (NMG_MIXED
 * runs the BF16 MFMA network).  alpha_dev is only read by Jacobi.  A zero b
 * gives h = 0. */
nmg_status nmg_apply_smoother(nmg_handle h, int level, int batch, const double* alpha_dev,
                              const int* weight_set_dev, const void* b, void* h_out,
                              nmg_precision precision, void* stream);

/* out = F'_l(in) = C^T (m'_l .* (C in C^T)) C on level `level` (the filter
 * of Algorithm 3 / Algorithm 4 with the DCT-II basis of a zero-boundary
 * grid and m'_l = sqrt(max(k1, k2) / n_l)).  in, out: device, double for
 * NMG_FP64, float otherwise; NMG_MIXED runs the four transforms on BF16
 * MFMA with FP32 accumulation.  in and out must not overlap. */
nmg_status nmg_apply_fprime(nmg_handle h, int level, int batch, const void* in, void* out,
                            nmg_precision precision, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * filter as nmg_apply_fprime with NMG_MIXED on a 2D handle (BF16 MFMA, FP32
 * accumulation, bit-identical results), with its two BF16 intermediate
 * planes in a fixed 16 MiB device array that the library holds on each GPU
 * it runs on until the process ends, instead of handle buffers.  The call
 * allocates nothing: the BF16 DCT tables are built by nmg_setup_hierarchy,
 * which also resolves the array's address on its device (a first call on
 * another device resolves it there).  in, out: device float [batch][n][n]
 * of level `level`, caller-owned, not overlapping; out is overwritten.
 * Levels above 64^2 need 4 * batch * NP^2 bytes, NP = n rounded up to 128
 * (batch <= 64 at 255^2, <= 16 at 511^2, <= 4 at 1023^2, <= 1 at 2047^2);
 * larger requests fail with NMG_ERR_SHAPE and a message naming the limit.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap in
 * time on one GPU, from any handle or stream, race and must be serialised
 * by the caller.  NMG_ERR_ARG for a 1D handle, a bad level or NULL
 * pointers. */
nmg_status nmg_apply_fprime_noalloc(nmg_handle h, int level, int batch, const float* in, float* out,
                                    void* stream);

/* ---- the cycle ---------------------------------------------------------- */

/* x <- MG(x, y): one V(nu1, nu2) cycle on the finest level with initial
 * guess x (Algorithm 1 skeleton with the neural smoothing step
 * b = y - A x, h = ||b|| N(b/||b||), x += F'(h) of Algorithms 2-4, Galerkin
 * coarse levels, exact coarsest solve).  x, y: device, double for
 * NMG_FP64, float otherwise.  weight_set_dev: device int[batch] choosing the
 * smoother set per right-hand side, or NULL for set 0 (indices outside
 * [0, n_weight_sets) are clamped into it).  Requires nmg_prepare for the
 * same alphas. */
nmg_status nmg_vcycle(nmg_handle h, int batch, const double* alpha_dev, const int* weight_set_dev,
                      const void* y, void* x, const nmg_cycle_opts* opts, void* stream);

/* A right-hand side whose relative residual ||b - A x|| / ||b|| exceeds
 * this factor has diverged (a smoother that does not fit its operator): it
 * is retired with status NMG_DIVERGED and leaves the others untouched. */
#define NMG_DIVERGENCE_FACTOR 1.0e6

/* Per right-hand-side outcome of nmg_solve. */
typedef struct {
    int cycles;           /* outer iterations applied                                */
    int status;           /* NMG_OK, NMG_NOT_CONVERGED (max_cycles reached),
                             NMG_DIVERGED or NMG_ERR_NONFINITE (NaN/Inf residual)  */
    double rel_residual;  /* ||b - A x||_2 / ||b||_2 of the returned x in FP64 (the
                             check that retired it; 0 for b = 0)                   */
    double done_ms;       /* host ms from entry to that check                      */
} nmg_solve_stats;

/* Outer iteration x^{t+1} = MG(x^t, b) from x^0 = 0 until
 * ||b - A x||_2 / ||b||_2 <= rtol per right-hand side or max_cycles
 * (Sec. 2.3; stopping rule of Sec. 4).  b, x: device double[B][n]([n]).
 * NMG_FP64 / NMG_MIXED iterate in FP64 with d = MG(0, r/||r||) computed in
 * the cycle precision (residual-driven form of the same iteration);
 * NMG_FP32 iterates in plain FP32 and converts at the end.  Converged
 * right-hand sides are frozen: they leave the batch, so every cycle runs on
 * the active ones only, and each result is the same as when that
 * right-hand side is solved alone.  A right-hand side whose residual turns
 * non-finite or grows beyond NMG_DIVERGENCE_FACTOR ||b|| leaves the batch
 * the same way, with its own status; the others go on.  weight_set_dev
 * entries must lie in [0, n_weight_sets) (NMG_ERR_ARG otherwise).
 * stats_host (nmg_solve_stats[batch], may be NULL) receives each right-hand
 * side's outcome; history_host (double[batch][max_cycles+1], may be NULL)
 * receives the relative residual before each cycle (unused entries -1).
 * x holds the last iterate of every right-hand side, whatever its status.
 * Synchronises once per cycle.  Returns NMG_OK when every right-hand side
 * converged, NMG_NOT_CONVERGED (a warning: see stats_host for which one
 * and why) otherwise, NMG_ERR_STATE while serving requests are queued or
 * active (it runs on the same engine). */
nmg_status nmg_solve(nmg_handle h, int batch, const double* alpha_dev, const int* weight_set_dev,
                     const double* b_dev, double* x_dev, double rtol, int max_cycles,
                     const nmg_cycle_opts* opts, nmg_solve_stats* stats_host, double* history_host,
                     void* stream);

/* ---- serving: continuous batching ----------------------------------------
 *
 * Every right-hand side is an independent solve (Sec. 2.3 outer iteration,
 * Sec. 4 stopping rule), so requests can join and leave the batch between
 * outer iterations: the handle keeps up to max_batch requests in flight,
 * runs one iteration on all of them per step, retires the ones that reached
 * rtol (or max_cycles, or a non-finite residual) and admits queued requests
 * into the freed slots.  A request's result does not depend on which other
 * requests share its iterations.  nmg_solve runs on the same engine. */

typedef struct {
    long long id;         /* the caller's request id */
    int status;           /* NMG_OK, NMG_NOT_CONVERGED, NMG_DIVERGED or NMG_ERR_NONFINITE */
    int cycles;           /* outer iterations applied */
    double rel_residual;  /* ||b - A x||_2 / ||b||_2 when it left (0 for b = 0) */
    double latency_ms;    /* host time from submission to the check that finished it */
} nmg_request_result;

/* Queues one request (host side only, no device work): b_dev is the
 * right-hand side, x_dev receives the solution when the request finishes
 * (device double[ny][n] each, caller-owned; both must stay valid until
 * then).  alpha > 0 finite; weight_set in [0, n_weight_sets). */
nmg_status nmg_serve_submit(nmg_handle h, long long id, double alpha, int weight_set,
                            const double* b_dev, double* x_dev);

/* One engine step on `stream`: admits queued requests into free slots
 * (copies b, factors new alphas), checks every active request against
 * rtol / max_cycles and the divergence guard, writes the iterates of
 * finished requests to their x_dev and reports them in done (host array of
 * at least max_batch entries; *n_done = count), then enqueues one outer
 * iteration on the remaining ones.  Returns once the solutions in done are
 * written (their latency_ms is taken then); the iteration it enqueued may
 * still be running on the stream, and the next step waits for it.
 * opts->precision must stay the same while requests are active. */
nmg_status nmg_serve_step(nmg_handle h, double rtol, int max_cycles, const nmg_cycle_opts* opts,
                          nmg_request_result* done, int* n_done, void* stream);

/* Queued and active request counts. */
nmg_status nmg_serve_pending(nmg_handle h, int* queued, int* active);

/* Drops every queued and active request (their x_dev are left as they are). */
nmg_status nmg_serve_reset(nmg_handle h);

/* ---- serving pool: several handles, one budget ------------------------ */

/* Device bytes one request slot occupies in a solve of `precision` on this
 * handle: the engine's FP64/FP32 planes plus the cycle's level buffers (and
 * the direct-convolution activations for FP32 / FP64 cycles). */
nmg_status nmg_request_bytes(nmg_handle h, nmg_precision precision, size_t* bytes);

/* A pool serves requests of several problems at once (Sec. 2.3: every
 * right-hand side is an independent solve), typically one handle per grid
 * size.  Each member handle keeps its hierarchy, weights and iterates on the
 * device and runs its continuous-batching engine (nmg_serve_*) on a stream
 * the pool creates for it (default priority); one pool step advances every
 * member with work whose previous outer iteration has finished by one more
 * (waiting for the first to finish when none has), so members iterate at
 * their own pace and different members' iterations overlap on the device.  Requests wait in one FIFO and are admitted while the bytes of
 * the admitted requests (nmg_request_bytes at the step's precision) stay
 * within hbm_budget_bytes; the head request is always admitted when nothing
 * is in flight.  The pool does not own its handles: they must outlive it and
 * receive no other solve or serving calls while it holds work.  Not
 * thread-safe. */
typedef struct nmg_pool_ctx* nmg_pool;
nmg_status nmg_pool_create(size_t hbm_budget_bytes, nmg_pool* out);
/* Waits for the members' streams; requests still queued or in flight are
 * abandoned (their members' serving state is reset). */
void nmg_pool_destroy(nmg_pool p);
/* Adds a handle (with no serving work of its own); *member_out = its index. */
nmg_status nmg_pool_add(nmg_pool p, nmg_handle h, int* member_out);
/* Queues request `id` (unique among the pool's queued and running requests)
 * for member `member`: b_dev / x_dev as in nmg_serve_submit, ready on the
 * device before the next nmg_pool_step (the pool's streams do not wait on
 * the caller's).  NMG_ERR_ARG if one request of this size exceeds the budget
 * in mixed precision, NMG_ERR_NOT_SPD / NMG_ERR_ARG for a bad alpha. */
nmg_status nmg_pool_submit(nmg_pool p, int member, long long id, double alpha, int weight_set,
                           const double* b_dev, double* x_dev);
/* Admission, then one outer iteration of every member with work whose
 * previous iteration has finished (at least one: the call waits for the
 * first to finish when none has).  Finished
 * requests are written to done[0..*n_done) with their member index in
 * done_member; latency_ms counts from nmg_pool_submit.  Their solutions are
 * complete in x when the call returns.  capacity must be at least the
 * number of requests in flight (nmg_pool_pending). */
nmg_status nmg_pool_step(nmg_pool p, double rtol, int max_cycles, const nmg_cycle_opts* opts,
                         nmg_request_result* done, int* done_member, int capacity, int* n_done);
nmg_status nmg_pool_pending(nmg_pool p, int* queued, int* active, size_t* bytes_in_flight);

/* ---- training (Sec. 3.2 eq. loss_2_modified / Sec. 3.3 eq. loss_3,
 *      Algorithm 5) ----------------------------------------------------- */

/* Level-wise losses and their gradients for one batch of true solutions
 * e (device, [B][n]([n]), double for NMG_FP64 else float):
 * y = A e, one pre-smoothing-only cycle from zero recording b_l, then
 * L_l = (1/B) sum_i || mask_l (.) DCT2(e - sum_{k<l} I_k^1 F'_k(h_k) - I_l^1 h_l) ||^2
 * and dL_l/dtheta_l (earlier levels held fixed).  alpha_dev: double[batch].
 * losses_host: double[L-1] (may be NULL).  The gradients are accumulated
 * into the handle's gradient buffers of `weight_set` (zeroed first when
 * zero_grad != 0).  Precision NMG_FP64 computes everything in FP64;
 * otherwise FP32 arithmetic with BF16 MFMA smoother forward.  Synchronises.
 *
 * mask = NMG_LOSS_CYCLE selects the combined loss of Sec. 3.2 eq. loss_1
 * instead: L = (1/B) sum_i || e_i - NMG(0, A e_i) ||^2 for the whole
 * pre-smoothing-only cycle with its exact coarsest solve, and dL/dtheta_l
 * for every level jointly (finer corrections change coarser residuals).
 * It factors the batch's alphas itself (as nmg_prepare does, so the coarse
 * indices of a following nmg_vcycle refer to these alphas).  losses_host[0]
 * receives L, the other entries 0. */
nmg_status nmg_loss_grad(nmg_handle h, int weight_set, int batch, const double* alpha_dev,
                         const void* e_dev, nmg_mask_kind mask, int use_fprime,
                         nmg_precision precision, int zero_grad, double* losses_host, void* stream);

/* Training pairs of Algorithm 5 (procedure DataGeneration), in place:
 * sample i of e (device [B][n]([n]), double for NMG_FP64 else float) goes
 * through k_host[i] rollout cycles e_i <- e_i - MG(0, A e_i) with the
 * current smoothers and the cycle of opts (Algorithm 5 uses V(1, 0), with
 * F' in the filtered variant), no gradients.  Afterwards y (same layout, or
 * NULL) receives A e, so (e, y) is a consistent pair again: the reading of
 * the procedure's right-hand-side update.  Algorithm 5 draws k_i uniformly
 * from 1..K; the caller draws them (host int[batch], each in [0, 64]).
 * alpha_dev / weight_set_dev as for nmg_vcycle; the coarse factors are
 * formed as nmg_prepare does.  NMG_ERR_STATE while serving requests are
 * active (it uses the engine's slot tables).  Synchronises. */
nmg_status nmg_rollout(nmg_handle h, int batch, const double* alpha_dev, const int* weight_set_dev,
                       const int* k_host, void* e_dev, void* y_dev, const nmg_cycle_opts* opts, void* stream);

/* The forward half of nmg_loss_grad: the same losses (level-wise, or the
 * combined loss for NMG_LOSS_CYCLE) for the same arguments, without the
 * adjoint; the gradient buffers are left as they are.  For evaluation and
 * for a loss whose gradient is not needed.  Synchronises. */
nmg_status nmg_loss_forward(nmg_handle h, int weight_set, int batch, const double* alpha_dev,
                            const void* e_dev, nmg_mask_kind mask, int use_fprime,
                            nmg_precision precision, double* losses_host, void* stream);

/* Copies the gradient of (level, weight_set) filled by the last
 * nmg_loss_grad to the host as doubles (layout as nmg_load_smoother_weights). */
nmg_status nmg_get_gradient(nmg_handle h, int level, int weight_set, double* grad_host, size_t count);

/* One bias-corrected Adam step (beta1, beta2, eps as given; no weight decay)
 * on every level of `weight_set` from the accumulated gradients; updates the
 * FP32 master weights and the FP64 / BF16 copies. */
nmg_status nmg_adam_step(nmg_handle h, int weight_set, double lr, double beta1, double beta2,
                         double eps, void* stream);

/* nmg_loss_grad followed by nmg_adam_step (Algorithm 5, one training step). */
nmg_status nmg_train_step(nmg_handle h, int weight_set, int batch, const double* alpha_dev,
                          const void* e_dev, nmg_mask_kind mask, int use_fprime,
                          nmg_precision precision, double lr, double* losses_host, void* stream);

/* ---- execution ------------------------------------------------------------ */

/* nmg_solve replays each outer iteration (refinement scaling, cycle, update,
 * next residual) as a captured HIP graph, one graph per launch size, cached
 * in the handle (default on).  enable = 0 frees the graphs and launches every
 * kernel directly; the results are the same either way.  Synchronises the
 * device when turning graphs off. */
nmg_status nmg_set_graphs(nmg_handle h, int enable);

/* ---- profiling ------------------------------------------------------------ */

/* Kernel families timed by the built-in profiler. */
typedef enum {
    NMG_K_SMOOTHER = 0, NMG_K_OPERATOR = 1, NMG_K_RESTRICT = 2, NMG_K_PROLONG = 3,
    NMG_K_COARSE = 4, NMG_K_FPRIME = 5, NMG_K_REFINE = 6, NMG_K_NORM = 7
} nmg_kernel_kind;

/* Turns timing on for the kernel families in kind_mask (bit k =
 * nmg_kernel_kind k; 0 turns it off) and clears the accumulated times.
 * HIP events are recorded on the caller's stream around each timed launch;
 * inside captured solve iterations, where events cannot be timed, two
 * one-wave kernels write the device's real-time counter before and after it. */
nmg_status nmg_profile_enable(nmg_handle h, int kind_mask);

/* Times only every period-th solve iteration of nmg_solve and the serving
 * engine (default 1: all of them); the others run without timing launches.
 * The accumulated launch counts then cover the sampled iterations only.
 * period < 1: NMG_ERR_ARG. */
nmg_status nmg_profile_sample(nmg_handle h, int period);

/* The number of right-hand sides still iterating, summed over the solve
 * iterations that were timed since nmg_profile_enable (each such iteration
 * runs nu1 + nu2 smoothing steps per level on each of them). */
nmg_status nmg_profile_rhs(nmg_handle h, long long* rhs_iterations);

/* Restricts timing to the levels in level_mask (bit l = level l; default
 * all levels).  Fewer timed launches mean less timing overhead. */
nmg_status nmg_profile_levels(nmg_handle h, int level_mask);

/* Accumulated device time (ms) and launch count of one kernel family on one
 * level (level -1 sums all levels).  Synchronises the recorded events. */
nmg_status nmg_profile_query(nmg_handle h, int kind, int level, double* total_ms, int* launches);

/* ---- introspection ------------------------------------------------------ */

/* Grid size of level `level` (0-based). */
int nmg_level_size(nmg_handle h, int level);

/* The alpha floor of the handle's operator form (see nmg_operator_form):
 * alphas at or below it are rejected with NMG_ERR_NOT_SPD; 0 for
 * NMG_OP_NORMAL and for kernels with no negative eigenvalue. */
nmg_status nmg_alpha_floor(nmg_handle h, double* floor_out);

/* Integer index maps of the 1D transfers between level and level+1 as the
 * kernels use them.  kind 0 = restriction: idx int32[n_{l+1}][3], w float
 * same shape (fine indices read by each coarse node).  kind 1 =
 * interpolation: idx int32[n_l][2], w float[n_l][2] (coarse indices read by
 * each fine node, -1 where absent). */
nmg_status nmg_debug_transfer_map(nmg_handle h, int level, int kind, int32_t* idx, float* w);

/* Copies the banded Galerkin factor rows of level `level` to the host:
 * which 0 = M_l, 1 = G_l; out double[n_l][2 r + 1], *radius receives r
 * (call with out == NULL to query the radius). */
nmg_status nmg_debug_factor(nmg_handle h, int level, int which, double* out, int* radius);

/* Test switches that change how results are computed but not their values.
 *   NMG_DEBUG_FP32_HANDOFF, value 1: in mixed-precision cycles with F' the
 *     BF16 smoother writes h as FP32 and F' rounds it to BF16 itself (the
 *     path of nmg_apply_fprime) instead of receiving the zero-padded BF16
 *     plane the smoother writes directly on levels above 64^2.  Both give
 *     bit-identical iterates.  Value 0 (default) restores the direct plane.
 *   NMG_DEBUG_SEPARATE_RESTRICT, value 1: 2D cycles without pre-smoothing
 *     (nu1 = 0, Algorithm 4's restriction of y from x = 0) restrict level by
 *     level, one launch each, and solve the coarsest level in its own
 *     launch, instead of taking the restrictions onto grids of at most
 *     64 x 64 (and the coarsest eigenbasis solve up to 32 x 32) in one
 *     launch.  Both give bit-identical iterates.  Value 0 (default) restores
 *     the single launch.
 * Takes effect for cycles launched afterwards (captured solve graphs are
 * dropped).  NMG_ERR_ARG for an unknown option. */
typedef enum { NMG_DEBUG_FP32_HANDOFF = 1, NMG_DEBUG_SEPARATE_RESTRICT = 2 } nmg_debug_opt;
nmg_status nmg_debug_option(nmg_handle h, int option, int value);

#ifdef __cplusplus
}
#endif

#endif /* NMG_H */
