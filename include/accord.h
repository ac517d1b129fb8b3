/*
 * accord.h -- C ABI of the MI355X (gfx950) ACCORD-FBS library.
 *
 * The library computes the ACCORD estimator (arXiv 2412.11554, eq. 3.2)
 *
 *     Omega_hat = argmin  -sum_j log Omega_jj  +  ||X Omega||_F^2 / (2n)  +  lambda ||Omega||_1
 *
 * with the forward-backward splitting iteration of Alg. 1 (ACCORD-FBS with
 * backtracking).  The penalty covers all p^2 entries, the diagonal included
 * (eq. 3.2; the diagonal update of eq. 3.5 carries the -tau*lambda term).
 *
 * Matrix convention.  The paper writes the smooth part as tr(Omega^T Omega S)/2
 * with gradient Omega S, so row i of the paper's Omega is node-wise problem i
 * (supplement, proof of Theorem 3.2).  This library works on the transpose
 * ("column form"): column j of Omega is node-wise problem j, the smooth part is
 * g(Omega) = ||X Omega||_F^2 / (2n) and its gradient is G = X^T (X Omega) / n.
 * Column-form matrices are stored COLUMN-MAJOR: entry (i, j) at [j*p + i].
 * That buffer is byte-identical to the paper's Omega stored row-major, i.e. a
 * C-contiguous torch [p, p] tensor holding the paper's Omega.
 *
 * Layouts.  X is n x p, row-major (entry (k, i) at [k*p + i]), float32, with
 * centred columns (Sec. 2).  W = X Omega is n x p row-major.  Omega, G and
 * Omega_out are p x p column-major as above.  All pointers marked "device"
 * must be device memory on the current HIP device, 16-byte aligned.
 *
 * Ownership.  The caller owns every buffer, including the workspace `ws`
 * (device, 256-byte aligned, at least accord_workspace_bytes() bytes).  The
 * library allocates no device memory and frees nothing; its only global state
 * is a thread-local last-error string, the pinned host mailbox of the fit loop (one
 * hipHostMalloc of 16 bytes per calling thread, allocated on that thread's first
 * accord_fit and kept until the process ends), (with params.timing) a thread-local
 * cache of HIP events that later calls reuse, and the static partial-sum array of
 * accord_prox_noalloc.  Calls with distinct workspaces are
 * independent; calls sharing a workspace must be stream-ordered.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default stream).
 * accord_grad, accord_prox and accord_objective are asynchronous and
 * stream-ordered; problems found on the device (non-finite values, a
 * non-positive diagonal) show up as NaN / inf in their outputs.  accord_fit,
 * accord_fit_batch and accord_refit are synchronous: they return after their work on
 * `stream` has completed.
 *
 * Errors.  Every entry point returns an accord_status.  Argument, alignment and
 * workspace-size problems are detected on the host and returned before any
 * work is enqueued.  HIP runtime failures return ACCORD_ERR_HIP; the text is in
 * accord_last_error().
 */
#ifndef ACCORD_H
#define ACCORD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ACCORD_OK = 0,
    ACCORD_ERR_INVALID_ARG = 1,  /* null pointer, size < 1 or > 2^20, bad parameter, misalignment */
    ACCORD_ERR_DOMAIN = 2,       /* some Omega_jj <= 0 where a positive diagonal is required */
    ACCORD_ERR_NONFINITE = 3,    /* NaN/inf in X or in an iterate */
    ACCORD_ERR_WORKSPACE = 4,    /* workspace null, misaligned or smaller than required */
    ACCORD_ERR_UNSUPPORTED = 5,  /* precision form not available on this device/build */
    ACCORD_ERR_HIP = 6           /* HIP runtime error (see accord_last_error) */
} accord_status;

/* Arithmetic of the two contractions X Delta and X^T W (the precision form).  The
 * prox, the acceptance test, the objective sums and the diagonal root are the same in
 * every form (FP32 iterate, FP64 sums and root); W = X Omega is carried in FP32. */
typedef enum {
    ACCORD_FP32 = 0,    /* FP32 MFMA (v_mfma_f32_16x16x4f32) */
    ACCORD_BF16X1 = 1,  /* bf16 MFMA on bf16(X), bf16(Delta), bf16(W); FP32 accumulation.
                           About 3 significant digits: use for a first phase, then refine
                           with ACCORD_BF16X3 from its result (Omega in/out). */
    ACCORD_BF16X3 = 2,  /* bf16 MFMA on the split x = hi + lo (hi = bf16(x), lo =
                           bf16(x - hi)) of every operand: hi*hi + hi*lo + lo*hi, FP32
                           accumulation; relative product error about 2^-16 */
    ACCORD_FP8 = 3      /* OCP MX operands on the scaled MFMA (v_mfma_scale_f32_32x32x64_
                           f8f6f4): E4M3 elements with one power-of-two (E8M0) scale per
                           32 consecutive values along the contraction index -- X per row
                           over features for X Delta and per feature over samples for
                           X^T W, Delta per column, W per column over samples.  Scale
                           2^s with s = floor(log2(block max)) - 7; elements rounded to
                           nearest even.  FP32 accumulation.  About 2^-4 relative
                           rounding per operand: use for a first phase, then refine with
                           ACCORD_BF16X3 from its result. */
} accord_precision;

/* Columns of the optional per-iteration trace (device double[(max_iter+1) * 8]).
 * Row 0 describes the starting point, row t+1 the iterate after iteration t. */
enum {
    ACCORD_TRACE_F = 0,         /* f = g + h                                       */
    ACCORD_TRACE_G = 1,         /* g = ||X Omega||_F^2 / (2n)                      */
    ACCORD_TRACE_H = 2,         /* h = -sum log Omega_jj + lambda ||Omega||_1      */
    ACCORD_TRACE_TAU = 3,       /* accepted step tau_t                             */
    ACCORD_TRACE_TRIALS = 4,    /* backtracking trials used                        */
    ACCORD_TRACE_DELTA = 5,     /* ||Omega_{t+1} - Omega_t||_F                     */
    ACCORD_TRACE_FLOOR = 6,     /* 1 if accepted only because tau <= 1/L           */
    ACCORD_TRACE_NNZ = 7,       /* nonzero off-diagonal entries of the iterate     */
    ACCORD_TRACE_COLS = 8
};

/* Parameters of accord_fit (Alg. 1 inputs plus run control). */
typedef struct {
    double lambda;      /* penalty, >= 0 */
    double tau0;        /* initial step of EVERY iteration (Alg. 1), > 0; typical 1 */
    double beta;        /* backtracking factor in (0, 1]; 1 = fixed step tau0, no test */
    double lipschitz;   /* L = sigma_max(X^T X / n) (Sec. 3.2); 0 = estimate on the device
                           by the Lanczos iteration: theta + beta_m |s_m|, the top Ritz value
                           plus its residual bound, so that the estimate errs above sigma_max
                           and the step floor tau <= 1/L stays on the safe side.  The
                           iteration stops once the bound is below 1e-12 theta (checked every
                           8 steps), when the Krylov space stops growing, or at power_iters
                           steps.  The step floor of Alg. 1 is tau <= 1/L. */
    double tol;         /* 0 = run exactly max_iter iterations; > 0 = also stop once
                           ||Delta||_F <= tol * max(1, ||Omega_{t+1}||_F) */
    int32_t max_iter;   /* iterations, >= 0 */
    int32_t precision;  /* accord_precision */
    int32_t power_iters;/* cap on the Lanczos steps of the L estimate when lipschitz == 0
                           (0 = 256; larger values are taken as 256); fewer are run once the
                           residual bound is met or the Krylov space stops growing */
    int32_t timing;     /* 0 = off; k >= 1 = bracket the launch groups of every k-th iteration
                           with HIP events (fills the *_ms fields: sums and counts over those
                           iterations, whose means estimate every launch's).  Each event costs a
                           few microseconds of GPU time, so k = 1 slows the fit measurably */
    int32_t warm_tau;   /* 0 = every iteration's first trial is tau0 (Alg. 1).  1 = a variant
                           that departs from Alg. 1: after the first iteration, the first
                           trial is min(tau0, tau_{t-1} / beta) (one step above the last
                           accepted one).  The acceptance test and the step floor are
                           unchanged, so every accepted step still satisfies Alg. 1's
                           inequality (or tau <= 1/L); the iterates differ, the fixed point
                           does not.  Fewer trials per iteration. */
    int32_t graph;      /* accord_fit_batch only: 1 = capture one sweep of each parity into a
                           HIP graph once and replay the graphs, instead of enqueuing every
                           launch (same kernels, same results; needs a non-default stream,
                           ignored on the default stream).  Ignored by accord_fit. */
    int32_t refresh_every; /* accord_fit / accord_refit: 0 = W = X Omega is carried across
                           iterations (W_{t+1} = W_t + X Delta_t, the trial product); k > 0 =
                           after every k-th accepted iteration W is recomputed as X Omega
                           in FP32 (one extra product), which bounds the drift of the carried
                           W (in the BF16X1 / FP8 forms the carried W sums rounded steps). */
    int32_t probe;      /* accord_fit / accord_refit, BF16X1 / BF16X3 / FP8 forms with at least
                           4 tiles of 256 samples (n > 768): 1 (the default of
                           accord_default_params) = run each trial first on the first 256
                           samples; ||X Delta||^2 over them is a lower bound of the whole
                           sum, so when it alone fails Alg. 1's test the trial is rejected
                           without the rest of the product (the same decision, since every
                           term is a square); otherwise the product is completed and tested
                           as usual.  When one tile of 256 samples fills the GPU (p of about
                           32768 and more, or a split product) the rest also goes one tile
                           at a time, with the same partial test after each.  Once a trial
                           of an iteration has failed the full test, or a partial test
                           over two thirds of the tiles or more, the iteration's later
                           trials (whose test ratio is about half and likely to pass) run
                           without partial tests.  0 = always the whole product.  Same
                           iterates either way, up to FP64 rounding of the sums at a tie. */
    int32_t support_skip; /* accord_refit: 1 (the default of accord_default_params) = the
                           trial products walk only the 32-row K steps of each 128-column
                           block that hold support entries, and the gradient skips its tiles
                           (256 x 256 in the BF16 / FP8 forms, 128 x 128 in FP32) without any
                           (everything off the support stays exactly zero, so the results are
                           the same bits); 0 = every block.  The FP32 form with n > 512 (a
                           separate prox pass) walks every block.  Ignored by accord_fit. */
    int32_t batch_order; /* accord_fit_batch: launch code of the batched gradient (bits 0-7)
                           and trial kernel (bits 8-15), each 0 (default) or a code 1..20
                           from accord_tune_batch: codes 1..10 are tile orders at two
                           workgroups per CU, 11..20 the same orders at one.  Both decide
                           only which workgroup computes which tile and how many share a
                           CU, so every code gives the same bits. */
} accord_params;

/* Results of accord_fit (host memory, filled on return). */
typedef struct {
    int32_t iters;          /* iterations completed */
    int32_t trials;         /* backtracking trials over all iterations */
    int32_t floor_accepts;  /* trials accepted only by the tau <= 1/L rule */
    int32_t converged;      /* tol-based stop reached */
    int64_t nnz_offdiag;    /* nonzero off-diagonal entries of the result */
    double f, g, h;         /* objective pieces at the result */
    double tau_last;        /* accepted step of the last iteration */
    double delta_fro;       /* ||Delta||_F of the last iteration */
    double lipschitz;       /* L used for the step floor */
    /* per-kernel device time (params.timing >= 1; executed launches of the sampled
       iterations only; total_ms covers the whole fit) */
    double grad_gemm_ms;    int32_t grad_gemm_launches;   /* G = X^T W / n          */
    double trial_gemm_ms;   int32_t trial_gemm_launches;  /* W+ = W + X Delta, with the
                                                             prox (eq. 3.5) inside except
                                                             as below                  */
    double prox_ms;         int32_t prox_launches;        /* separate prox pass: only the
                                                             FP32 form with n > 512 (more
                                                             than 4 row tiles of 128
                                                             samples); 0 launches else */
    double total_ms;        /* event time of the whole fit on the stream */
    double log_det_d;       /* sum_j log Omega_jj at the result (log det of the diagonal) */
    double l1;              /* ||Omega||_1 at the result (all entries) */
    int32_t lz_steps;       /* Lanczos steps of the device estimate of L (0 if L was given) */
    int32_t probe_rejects;  /* trials rejected by a partial test over their first tiles of
                               256 samples (params.probe) */
    int32_t unprobed_trials;/* trials of a probed fit run without a probe: once a trial of
                               an iteration fails the full test (or a late partial test), the
                               later ones (at half the step and less) run as one launch over
                               all samples */
    int32_t probe_mtiles;   /* tiles of 256 samples that the trials rejected by a partial
                               test had multiplied (params.probe) */
    int32_t tail_blocks;    /* trial product: 128-column blocks run as a separate launch
                               split along the contraction (the blocks past the last whole
                               round of workgroups; 0: none, and always 0 for the FP32 form
                               up to 512 samples, whose fused trial runs unsplit) */
    int32_t tail_splits;    /* its split count (0: none) */
} accord_stats;

/* Fills `prm` with defaults: lambda 0.1, tau0 1, beta 0.5, lipschitz 0 (estimate),
 * tol 0, max_iter 100, FP32, power_iters 256, timing 0, warm_tau 0, probe 1, support_skip 1,
 * graph 0, refresh_every 0. */
void accord_default_params(accord_params* prm);

/* Workspace bytes needed by accord_fit for an n x p problem with `prm` (NULL =
 * defaults).  The same size (or accord_workspace_bytes(n, p, NULL)) is enough for
 * accord_grad and accord_objective on that problem, and accord_workspace_bytes(1, p,
 * NULL) for accord_prox.  Returns 0 for n < 1 or p < 1. */
size_t accord_workspace_bytes(int64_t n, int64_t p, const accord_params* prm);

/* Gradient of the smooth part (eq. 3.4; Remark 3.1's two-step product):
 *     W = X Omega  (n x p, row-major, optional: W may be NULL)
 *     G = X^T W / n  (p x p, column form, column-major)
 * X: device n x p.  Omega: device p x p column form.  Asynchronous. */
int accord_grad(const float* X, int64_t n, int64_t p, const float* Omega,
                float* W, float* G, void* ws, size_t ws_bytes, void* stream);

/* One proximal (backward) step at a given tau (eq. 3.5), for the whole matrix:
 *     A = Omega - tau*G;  off-diagonal: soft-threshold at tau*lambda;
 *     diagonal: (b + sqrt(b^2 + 4 tau)) / 2 with b = A_jj - tau*lambda (FP64).
 * Omega, G, Omega_out: device p x p column form (Omega_out must not alias).
 * red (device double[6], written): { ||Delta||_F^2, <Delta, G>, ||Omega_out||_1,
 *   sum_j log Omega_out_jj, nnz off-diagonal of Omega_out, ||Omega_out||_F^2 },
 * Delta = Omega_out - Omega, sums in FP64 in a fixed order.  tau > 0, lambda >= 0.
 * Asynchronous. */
int accord_prox(const float* Omega, const float* G, int64_t p, double tau, double lambda,
                float* Omega_out, double* red, void* ws, size_t ws_bytes, void* stream);

/* accord_prox for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same operation,
 * arguments (without the workspace), errors and kernels as accord_prox, so the same
 * results bit for bit.  Its FP64 partial sums go to a library-owned device array of
 * 256 KiB (4096 rows of 8 doubles; every p the library accepts needs at most 4096 rows,
 * and a larger need is rejected with ACCORD_ERR_INVALID_ARG), one per GPU, held until the
 * process ends.  The call allocates nothing: the first call on a device looks up the
 * array's address there.  All calls on one GPU share that array, and each call leaves
 * its partial sums in it: calls that overlap on one GPU (on different streams, or from
 * different threads without ordering) race and must be serialised by the caller.
 * Asynchronous and stream-ordered like accord_prox. */
int accord_prox_noalloc(const float* Omega, const float* G, int64_t p, double tau,
                        double lambda, float* Omega_out, double* red, void* stream);

/* Objective of eq. 3.2 at Omega (column form):
 * out (device double[3], written) = { g, h, f } with g = ||X Omega||_F^2/(2n),
 * h = -sum_j log Omega_jj + lambda ||Omega||_1 (+inf if some Omega_jj <= 0), f = g + h.
 * Asynchronous. */
int accord_objective(const float* X, int64_t n, int64_t p, const float* Omega, double lambda,
                     double* out, void* ws, size_t ws_bytes, void* stream);

/* ACCORD-FBS (Alg. 1).  Omega: device p x p column form; on input the starting
 * point Omega^(0) (diagonal > 0, else ACCORD_ERR_DOMAIN), on output the last iterate.
 * Every iteration computes G = X^T (X Omega_t) / n once, then tries
 * tau = tau0, beta*tau0, ... : Omega+ = prox(Omega_t - tau G) (eq. 3.5),
 * Delta = Omega+ - Omega_t, and accepts the first tau with
 *     ||X Delta||_F^2 / n <= ||Delta||_F^2 / tau      or      tau <= 1/L
 * (the acceptance inequality of Alg. 1, written without subtracting values of g,
 * which is exact because g is quadratic).  stats: host, filled on return (may be
 * NULL).  trace: device double[(max_iter+1) * ACCORD_TRACE_COLS] or NULL.
 * Synchronous.  The device posts each trial's outcome to a small pinned host buffer
 * (allocated once per calling thread and kept), so the host enqueues only the
 * trials an iteration needs plus one. */
int accord_fit(const float* X, int64_t n, int64_t p, float* Omega, const accord_params* prm,
               accord_stats* stats, double* trace, void* ws, size_t ws_bytes, void* stream);

/* ---- Batched form: many independent fits in one call (a lambda path over several
 * data sets, e.g. bootstrap subsamples).  nsub data sets X_b (n[b] x p, row-major
 * FP32, centred) are stacked row-wise in one device array: X_b starts at row
 * n[0] + ... + n[b-1].  nlam penalties lambda[l] (host).  Problem k = b * nlam + l
 * is the fit of (X_b, lambda[l]) by Alg. 1 with its own step, acceptance and stop;
 * every problem advances one iteration per sweep, and the kernels of a sweep cover
 * all problems at once (the gradients and trial products of one data set form a
 * single wide product over its nlam problems).
 *   Omega: device, nsub*nlam matrices of p x p (column form as in accord_fit),
 *          problem k at offset k*p*p; in: starting points (diagonal > 0), out: the
 *          last iterates.
 *   prm: tau0, beta, tol, max_iter, power_iters as in accord_fit; prm->lambda is
 *        not used; precision must be ACCORD_FP32 (else ACCORD_ERR_UNSUPPORTED).
 *   lipschitz: host double[nsub] (L of each data set) or NULL (Lanczos estimate).
 *   stats: host accord_batch_stats[nsub*nlam] or NULL.
 *   trials: device int32[nsub*nlam*max_iter] or NULL: the trials each iteration
 *           used (the accepted step of iteration t of problem k is
 *           tau0 * beta^(trials[k*max_iter + t] - 1); with prm->warm_tau it is
 *           s_t * beta^(trials - 1), s_0 = tau0, s_t = min(tau0, tau_{t-1} / beta));
 *           entries past a problem's last iteration are left unspecified.
 * ws: device, 256-byte aligned, at least accord_batch_workspace_bytes() bytes.
 * Synchronous.  Errors as accord_fit; the first failing problem is named in
 * accord_last_error(). */
typedef struct {
    int32_t iters, trials, floor_accepts, converged;
    int64_t nnz_offdiag;
    double f, g, h, tau_last, delta_fro, lipschitz;
    double log_det_d, l1;   /* as in accord_stats */
} accord_batch_stats;

/* Workspace bytes of accord_fit_batch (0 for invalid sizes). */
size_t accord_batch_workspace_bytes(const int64_t* n, int64_t nsub, int64_t p, int64_t nlam,
                                    const accord_params* prm);

int accord_fit_batch(const float* X, const int64_t* n, int64_t nsub, int64_t p,
                     const double* lambda, int64_t nlam, float* Omega,
                     const accord_params* prm, const double* lipschitz,
                     accord_batch_stats* stats, int32_t* trials, void* ws, size_t ws_bytes,
                     void* stream);

/* Autotuner of the batched form's launches (for callers that repeat fits of one shape,
 * e.g. a lambda path over bootstrap subsamples).  Runs the set-up of accord_fit_batch
 * (same arguments, max_iter ignored), then times the batched gradient and trial kernels
 * under each of 20 launch codes (10 tile orders: bands of 1, 2, 4, 8 or 16 M tiles in
 * plain block order or an XCD-contiguous one; each with the kernel compiled for two or
 * for one workgroup per CU) and writes the fastest as a params.batch_order code to
 * *order (host).  table (host float[40], or NULL) receives the mean ms per launch of each
 * code, gradient first.  No code changes a result.  Omega is left as given; workspace as
 * accord_fit_batch; synchronous. */
int accord_tune_batch(const float* X, const int64_t* n, int64_t nsub, int64_t p,
                      const double* lambda, int64_t nlam, float* Omega,
                      const accord_params* prm, const double* lipschitz, void* ws,
                      size_t ws_bytes, void* stream, int32_t* order, float* table);

/* ---- Differentiation form: gradients of a held-out loss through K unrolled
 * iterations with the step sizes held fixed (recorded from a backtracking fit and
 * replayed).  The forward map of one step is Alg. 1's iteration at a given tau,
 *     Omega_t+1 = prox(Omega_t - tau_t S Omega_t; tau_t, lambda)    (eq. 3.5),
 * with S = X^T X / n computed through X as everywhere else (G = X^T (X Omega) / n,
 * W recomputed from Omega_t at every step).  The held-out loss is the pseudolikelihood
 * part of eq. 3.2 on validation data X_v (n_v rows), without the penalty:
 *     l_val(Omega) = -sum_j log Omega_jj + ||X_v Omega||_F^2 / (2 n_v).
 * All matrices in the column form of accord_fit; all calls FP32, asynchronous and
 * stream-ordered; ws: device, 256-byte aligned, at least
 * accord_adjoint_workspace_bytes(n, p) bytes (enough for all three calls with
 * n = max(n, n_v)). */
size_t accord_adjoint_workspace_bytes(int64_t n, int64_t p);

/* nsteps fixed steps of sizes taus[0..nsteps-1] (host) from Omega (device p x p; in:
 * Omega_start, out: Omega_end).  Omega_seq: device float[nsteps * p * p] receiving
 * Omega_start+1 ... Omega_end, or NULL. */
int accord_fbs_replay(const float* X, int64_t n, int64_t p, float* Omega, const double* taus,
                      int64_t nsteps, double lambda, float* Omega_seq, void* ws, size_t ws_bytes,
                      void* stream);

/* Held-out loss and its gradient at Omega: out (device double[3]) = { ||X_v Omega||^2/(2 n_v),
 * -sum_j log Omega_jj, l_val }; Obar (device p x p) = S_v Omega - diag(1 / Omega_jj). */
int accord_val_loss_grad(const float* Xv, int64_t nv, int64_t p, const float* Omega,
                         double* out, float* Obar, void* ws, size_t ws_bytes, void* stream);

/* Reverse of one step at (Omega_t, tau): given Obar = dl/dOmega_t+1 (device p x p),
 * overwrites Obar with dl/dOmega_t and accumulates lbar[0] += dl/dlambda (device
 * double) and Xbar += dl/dX (device n x p, row-major, FP32).  The prox Jacobian is
 * taken entry by entry: off-diagonal 1{|a| > tau lambda} (0 at the kink), diagonal
 * (1 + b / sqrt(b^2 + 4 tau)) / 2 with b = a - tau lambda; then
 *     Abar = Obar * J,  dl/dlambda += sum(Obar * dOmega+/dlambda),
 *     dl/dOmega_t = Abar - tau S Abar,
 *     dl/dX += -(tau / n) (X Omega_t Abar^T + X Abar Omega_t^T). */
int accord_fbs_adjoint_step(const float* X, int64_t n, int64_t p, const float* Omega_t,
                            double tau, double lambda, float* Obar, double* lbar, float* Xbar,
                            void* ws, size_t ws_bytes, void* stream);

/* ---- Steps around the solver: tuning by epBIC (eq. 3.7), the refit on the estimated
 * support (eq. 3.8) and the reparametrisation of Sec. 2. */

/* Extended pseudo-BIC of eq. 3.7 of one estimate from the statistics of its fit
 * (host arithmetic in FP64):
 *     out = 2n (-log_det_d + g) + nnz_offdiag (log n + 4 gamma log p),
 * log_det_d = sum_j log Omega_jj, g = ||X Omega||_F^2 / (2n) (so the bracket is the
 * loss of eq. 3.2 without the penalty, tr(Omega^T Omega S)/2 in the paper's
 * orientation), nnz_offdiag = number of nonzero off-diagonal entries.
 * gamma in (0, 1] (the extended-BIC weight), 0 <= nnz_offdiag <= p (p - 1). */
int accord_epbic(int64_t n, int64_t p, double g, double log_det_d, int64_t nnz_offdiag,
                 double gamma, double* out);

/* epBIC of every problem of a batched fit (stats: host, nsub * nlam entries as
 * returned by accord_fit_batch; n: host row counts of the nsub data sets) into
 * epbic (host double[nsub * nlam], problem k = b * nlam + l), and for each data set b
 * the penalty index with the smallest value into best[b] (host int64[nsub], may be
 * NULL; the first index on ties). */
int accord_epbic_path(const accord_batch_stats* stats, const int64_t* n, int64_t nsub,
                      int64_t nlam, int64_t p, double gamma, double* epbic, int64_t* best);

/* Workspace bytes of accord_refit (0 for invalid sizes). */
size_t accord_refit_workspace_bytes(int64_t n, int64_t p, const accord_params* prm);

/* Refit of eq. 3.8: minimises -sum_j log Omega_jj + g(Omega) + phi * lambda ||Omega||_1
 * over Omega that vanish off the support of the first-stage estimate, by Alg. 1 with
 * the per-entry penalty phi * lambda on the support and infinity off it.
 *   Omega_hat: device p x p column form, the first-stage estimate; its support is
 *     its nonzero entries plus the diagonal.  Read once, before any iteration (it may
 *     be the same buffer as Omega).
 *   phi in [0, 1]; lambda = prm->lambda (the first-stage penalty).
 *   Omega: device p x p, in: the starting point (its entries off the support are set
 *     to zero first; Omega_hat itself is the natural start), out: the last iterate.
 *     Entries off the support are exactly zero in every iterate.
 * Every precision form of accord_fit runs the refit: the gradient is set to zero off
 * the support as it is stored, so the prox (eq. 3.5, whose soft threshold maps the
 * zero argument Omega_ij - tau G_ij = 0 to 0) keeps those entries at zero, which is
 * exactly what the infinite penalty gives.
 * Everything else (parameters, stats with phi * lambda as the penalty, trace, errors,
 * synchronous behaviour) as accord_fit.
 * ws: device, 256-byte aligned, at least accord_refit_workspace_bytes() bytes (which
 * depends on prm->precision). */
int accord_refit(const float* X, int64_t n, int64_t p, const float* Omega_hat, double phi,
                 float* Omega, const accord_params* prm, accord_stats* stats, double* trace,
                 void* ws, size_t ws_bytes, void* stream);

/* Reparametrisation of Sec. 2 from an estimate Omega (device p x p column form, positive
 * diagonal):
 *   Theta = Omega_D Omega in the paper's orientation, the inverse of the map
 *     T: Theta -> Theta_D^{-1/2} Theta; written in the column form like Omega
 *     (Theta^T column-major: column j of Omega times Omega_jj), or NULL;
 *   Rho: partial correlations rho_ij = -(w_ij / w_jj + w_ji / w_ii) / 2 (w in the paper's
 *     orientation), symmetric, with rho_ii = 1, p x p, or NULL.
 * One of the two may be NULL, not both; neither may overlap Omega or the other.
 * Theta is correctly rounded; Rho is computed with FP64 reciprocals of the diagonal
 * and one final rounding.  Asynchronous, stream-ordered; no workspace. */
int accord_reparam(const float* Omega, int64_t p, float* Theta, float* Rho, void* stream);

/* Static description of a status code. */
const char* accord_status_str(int status);

/* Text of the last error on the calling thread ("" if none). */
const char* accord_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ACCORD_H */
