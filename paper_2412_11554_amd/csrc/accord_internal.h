// Internal declarations shared by the kernel and host translation units of
// libaccord (gfx950).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace accord {

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
constexpr int kPad = 64;            // K-dimension padding of every MFMA operand
constexpr int kBM = 128;            // FP32 GEMM workgroup tile (rows of C)
constexpr int kBN = 128;            // FP32 GEMM workgroup tile (columns of C)
constexpr int kWBM = 256;           // bf16 GEMM workgroup tile (rows of C)
constexpr int kWBN = 256;           // bf16 GEMM workgroup tile (columns of C)
constexpr int kWThreads = 512;      // bf16 GEMM threads per workgroup
constexpr int kFBM = 256;           // fused prox + trial tile (rows of W^T = samples)
constexpr int kFBN = 128;           // fused prox + trial tile (columns of Omega)
constexpr int kFReduceParts = 2;    // workgroups per tile in the fused split-K reduction
constexpr int kBK32 = 32;           // FP32 GEMM K step staged through LDS
constexpr int kThreads = 256;       // threads per workgroup for every kernel
constexpr int kMaxProxBlocks = 4096;
constexpr int kPartCols = 8;        // FP64 partial sums per prox workgroup
constexpr int kNormCols = 2;        // FP64 partial sums per trial-GEMM tile
constexpr int kSlots = 512;         // resident FP32 GEMM workgroups (2 per CU, 256 CUs)
constexpr int kWSlots = 256;        // resident bf16 GEMM workgroups (1 per CU)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// prox partial columns
enum { P_D2 = 0, P_DG = 1, P_L1 = 2, P_LOGD = 3, P_NNZ = 4, P_FRO = 5 };

// ---------------------------------------------------------------------------
// device-resident iteration state of accord_fit (one per workspace)
// ---------------------------------------------------------------------------
struct LsState {
    double tau;        // step of the trial in flight
    double inv_L;      // step floor 1/L
    double L;
    double tau0, beta, lambda, tol, inv_n;
    double g_cur, h_cur, f_cur;  // objective pieces at the current iterate
    double delta_fro;            // ||Delta||_F of the last accepted step
    double tau_acc;              // accepted step of the last iteration
    double logd_cur, l1_cur;     // sum_j log Omega_jj and ||Omega||_1 at the current iterate
    int64_t nnz_off;
    int32_t done;       // current iteration accepted a trial: later trials are skipped
    int32_t converged;  // stop: every later launch is skipped
    int32_t trials;     // trials of the current iteration
    int32_t iter;       // accepted iterations
    int32_t total_trials;
    int32_t floor_accepts;
    int32_t bad;        // bit 0: diagonal <= 0, bit 1: non-finite value
    int32_t max_iter;
    int32_t fixed_step; // beta == 1: the single trial is accepted
    int32_t warm_tau;   // 1: an iteration starts from min(tau0, tau_acc / beta), not tau0
    int32_t lz_steps;   // Lanczos steps of the device estimate of L (0: L was given)
    int32_t probe_rej;  // the trial in flight was rejected by a partial test (its first
                        // M tiles)
    int32_t probe_rejects;  // trials rejected by a partial test, over the fit
    int32_t probe_off;  // this iteration's later trials run unprobed (set when a trial
                        // fails the full test of a probing fit, or a partial test late)
    int32_t unprobed;   // trials of a probing fit that ran unprobed, over the fit
    int32_t probe_mtiles;   // M tiles the trials rejected by partial tests had run
};

// Pinned host mailbox: after every executed acceptance test the device posts the
// trial count, the accepted-iteration count and the stop flag, so the host can
// enqueue only the trials an iteration needs.  The three travel in one 64-bit word
// (one system-scope store, read whole by the host), so no release fence -- which
// would write back the whole L2 -- is needed to keep them consistent.
struct Mailbox {
    uint64_t word;   // bits 0-31 trials, 32-62 accepted iterations, 63 stop
    uint64_t pad;
};

inline __host__ __device__ uint64_t mailbox_word(int32_t trials, int32_t iter, int32_t stop) {
    return (uint64_t)(uint32_t)trials | ((uint64_t)((uint32_t)iter & 0x7fffffffu) << 32) |
           ((uint64_t)(stop ? 1u : 0u) << 63);
}

// ---------------------------------------------------------------------------
// kernel argument blocks
// ---------------------------------------------------------------------------
enum GemmEpi { EPI_GRAD = 0, EPI_TRIAL = 1, EPI_PARTIAL = 2 };
enum Prec { PREC_FP32 = 0, PREC_BF16X1 = 1, PREC_BF16X3 = 2, PREC_FP8 = 3 };

// optional bf16 hi/lo copies of the padded X operands
struct XSplit {
    uint16_t* xp_h;
    uint16_t* xp_l;
    uint16_t* xt_h;
    uint16_t* xt_l;
};

// MX-FP8 copies of the padded X operands (E4M3 bytes + one E8M0 scale byte per 32)
struct XQuant {
    uint8_t* x8;    // n_pad x p_pad, blocks along the features (row-major)
    uint8_t* x8s;   // n_pad x p_pad/32
    uint8_t* xt8;   // p_pad x n_pad, blocks along the samples (row-major)
    uint8_t* xt8s;  // p_pad x n_pad/32
};

struct GemmArgs {
    const float* A;     // FP32: M x K row-major (lda), K a multiple of kPad, zero-padded
    const float* B;     // FP32: N x K row-major (ldb)
    const uint16_t* Ah; // bf16 forms: hi / lo parts of A and B, same layouts
    const uint16_t* Al;
    const uint16_t* Bh;
    const uint16_t* Bl;
    const uint8_t* A8;  // FP8 form: E4M3 A and B (same layouts, lda/ldb in bytes)
    const uint8_t* B8;
    const uint8_t* As;  // FP8 form: E8M0 scales, one per 32 K values, row-major
    const uint8_t* Bs;
    int64_t ldas, ldbs; // scale bytes per row (K / 32)
    int64_t lda, ldb;   // elements
    int M, N, K;        // C is M x N column-major; K = padded contraction length
    int tilesM, tilesN, splits;
    float* C;           // C[m + n*ldc]
    uint16_t* Ch;       // optional bf16 hi/lo split of C (same layout)
    uint16_t* Cl;
    int64_t ldc;
    int vec_store;      // ldc % 4 == 0 and C 16-byte aligned
    float alpha;        // EPI_GRAD scale
    const float* Wprev; // EPI_TRIAL: C += Wprev (same layout), may be null
    float* P;           // EPI_PARTIAL: split partial tiles
    double* norm_part;  // EPI_TRIAL: per tile {||V||^2, ||C||^2}
    LsState* ls;        // predication state (null = always run)
    int pred;           // 1: skip if converged; 2: skip if done or converged; 3: also
                        // skip if the trial's probe rejected it
    int begin_iter;     // reset the line-search state of a new iteration
    int Mvalid, Nvalid; // extent counted in the norms
    const uint8_t* cmask; // EPI_GRAD, optional: C entries whose byte (same layout as C)
                          // is 0 are stored as 0 (the refit's support)
    // fused trial kernels: the launch covers the M tiles m_first .. m_first + m_count - 1
    // (m_count 0: all tilesM); the tile with tile_m == store_m writes Omega+ and the one
    // with tile_m == sums_m writes the prox sums (-1: none).  trial_args sets 0, 0, 0, 0.
    int m_first, m_count, store_m, sums_m;
    // fused trial kernels, optional: the K steps (of the kernel's step length) each column
    // block walks, as CSR lists (kstep_ptr[tilesN + 1] positions into kstep_idx); steps
    // left out must hold Delta = 0 (a refit's blocks off the support).  Null: every step.
    const int32_t* kstep_ptr;
    const int32_t* kstep_idx;
    // gradient kernels, optional: one byte per tile (tile_m + tile_n * tilesM), 0 = the
    // tile of C is zero and is neither computed nor stored
    const uint8_t* tile_occ;
    int order;          // batched kernels: tile order code (batch_tile), 0 = default
    int probe_mode;     // trials of a probing fit: 0 always run; 1 only while the
                        // iteration probes (probe_off == 0); 2 only once it stopped
    // fused trial kernels: the launch covers the column blocks n_first .. n_first +
    // n_count - 1 (n_count 0: all tilesN) and numbers its split-K partial tiles within
    // that range; the prox sums of (column block, split) go to row tile_n * part_stride +
    // split (part_stride 0: splits), and a split-0 workgroup zeroes the rows of its
    // column block that the launch's splits do not reach; zero_part1: the trial epilogue
    // also writes a zero norm row at tiles + tile (the row a second reduce part fills
    // for the split tiles of the same product)
    int n_first, n_count, part_stride, zero_part1;
    // fused trial product as launch_trial_fused splits it: the column blocks from
    // tail_n0 on run as a separate launch split tail_splits ways along K, then reduced
    // (tail_splits 0: one launch over every column block)
    int tail_n0, tail_splits;
};

struct ProxArgs {
    const float* om;
    const float* g;
    float* om_new;      // may be null in reduce-only mode
    float* d;           // Delta output, FP32 (same layout), may be null
    uint16_t* dh;       // Delta output as bf16 hi (and lo), instead of d
    uint16_t* dl;
    int64_t total;      // elements = p * ld
    int64_t ld;         // rows stored per column (>= p)
    int64_t p;
    int64_t step_col, step_row;  // advance of (col,row) per 4*kThreads elements
    double tau, lambda; // used when ls == null
    const LsState* ls;  // if set: tau/lambda from here; skip if done or converged
    double* part;       // [gridDim.x][kPartCols]
    int reduce_only;    // 1: no writes, statistics of om itself
};

// acceptance-test arguments of one problem of the batched form
struct FinArgs {
    LsState* ls;
    const double* prox_part;
    int nprox;
    const double* norm_part;
    int ntiles;
    int32_t* trials_log;
};

// reverse of one prox step (differentiation form)
struct AdjArgs {
    const float* om;    // Omega_t, p columns x ld
    const float* g;     // G_t = S Omega_t, same layout
    const float* obar;  // dl/dOmega_t+1, p columns x ld_obar
    int64_t ld, ld_obar, p;
    double tau, lambda;
    float* abar;        // out: p columns x ld (zero padded rows)
    double* part;       // out: [gridDim.x] FP64 partials of dl/dlambda
};

// ---------------------------------------------------------------------------
// launchers (accord_kernels.hip)
// ---------------------------------------------------------------------------
void launch_init_state(LsState* ls, double tau0, double beta, double lambda, double tol,
                       double inv_n, double L, int max_iter, hipStream_t st, int warm_tau = 0);
void launch_pad_x(const float* X, int64_t n, int64_t p, float* Xp, int64_t p_pad, float* Xt,
                  int64_t n_pad, XSplit sp, LsState* ls, hipStream_t st);
void launch_copy_cols(const float* src, int64_t ld_src, float* dst, int64_t ld_dst, int64_t p,
                      int64_t rows, LsState* check_ls, hipStream_t st);
void launch_quant_x8(const float* X, int64_t n, int64_t p, int64_t p_pad, int64_t n_pad,
                     XQuant q, hipStream_t st);
void launch_quant_w8(const float* Wt, int64_t total, uint8_t* w8, uint8_t* w8s, const LsState* ls,
                     hipStream_t st);
void launch_gemm(const GemmArgs& a, int epi, int prec, hipStream_t st);
void launch_splitk_reduce(const GemmArgs& a, hipStream_t st);
void launch_trial_fused(const GemmArgs& a, const ProxArgs& px, int prec, hipStream_t st);
void launch_trial_fused32(const GemmArgs& a, const ProxArgs& px, hipStream_t st);
int prox_blocks(int64_t total);
void launch_prox(ProxArgs a, int nblocks, hipStream_t st);
// probing: the fit probes its trials; a trial failing the full test then turns the
// probes off for the rest of its iteration (LsState::probe_off)
void launch_finalize(LsState* ls, const double* prox_part, int nprox, const double* norm_part,
                     int ntiles, double* trace, int32_t* trials_log, Mailbox* mbox,
                     int probing, hipStream_t st);
// partial test of a probed trial after its first mt M tiles (1 <= mt < tilesM)
void launch_probe_decide(LsState* ls, const double* prox_part, int nprox,
                         const double* norm_part, int tilesN, int tilesM, int nparts, int mt,
                         Mailbox* mbox, hipStream_t st);
void launch_fit_init(LsState* ls, const double* prox_part, int nprox, const double* norm_part,
                     int ntiles, double* trace, hipStream_t st);
void launch_combine_prox(const double* prox_part, int nprox, double* red, hipStream_t st);
void launch_combine_objective(const double* prox_part, int nprox, const double* norm_part,
                              int ntiles, double lambda, double inv_n, double* out, hipStream_t st);
void launch_transpose_w(const float* Wt, int64_t ldt, int64_t n, int64_t p, float* W,
                        hipStream_t st);
// Lanczos estimate of L (buffers carved by lz_buf from lz_buf_bytes bytes)
constexpr int kBatchOrders = 10;   // tile orders accord_tune_batch tries per kernel
constexpr int kBatchCodes = 2 * kBatchOrders;  // codes per kernel: each order at 2 and at 1
                                               // workgroups per CU
// workgroups per CU a batched kernel is compiled for under an order code
inline int batch_occupancy(int code) { return code > kBatchOrders ? 1 : 2; }
constexpr int kLzMaxSteps = 256;   // cap on the Lanczos steps
constexpr int kLzDefaultSteps = 256;
constexpr int kLzCheck = 8;         // steps between checks of the Ritz residual bound
constexpr double kLzRelTol = 1e-12; // stop once beta_m |s_m| <= kLzRelTol * theta
constexpr int kLzInvariant = 1, kLzConverged = 2;  // why the iteration stopped early
constexpr int kLzMaxBlocks = 1024; // cap on the elementwise kernels' workgroups
struct LzBuf {
    double *q0, *q1, *r, *w, *u;   // q_{k-1}, q_k, residual, S q_k (p_pad), X q_k (n_pad)
    double *pa, *pb;               // partials of alpha and ||r||^2
    double *alpha, *beta;          // the tridiagonal (kLzMaxSteps each)
    int* stop;                     // [0]: 0, or the valid steps of an early stop;
                                   // [1]: kLzInvariant or kLzConverged
};
size_t lz_buf_bytes(int64_t n_pad, int64_t p_pad);
LzBuf lz_buf(void* base, int64_t n_pad, int64_t p_pad);
void launch_lipschitz(const float* Xp, int64_t p_pad, const float* Xt, int64_t n_pad, int64_t n,
                      int64_t p, const LzBuf& buf, int steps, LsState* ls, hipStream_t st);

// steps around the solver: support mask of a refit, reparametrisation
void launch_support_mask(const float* om_hat, int64_t p, int64_t p_pad, uint8_t* mask,
                         float* om0, hipStream_t st);
void launch_support_occupancy(const uint8_t* mask, int64_t p, int64_t p_pad, int tilesN,
                              int ksteps, uint8_t* occ, hipStream_t st);
void launch_reparam(const float* om, int64_t p, float* theta, float* rho, hipStream_t st);

// differentiation form
void launch_prox_adjoint(const AdjArgs& a, int nblocks, hipStream_t st);
void launch_adjoint_combine(const float* abar, const float* sa, int64_t ld, int64_t p, float tau,
                            float* out, int64_t ld_out, hipStream_t st);
void launch_transpose_ld(const float* src, int64_t ld_src, int64_t rows, int64_t cols, float* dst,
                         int64_t ld_dst, hipStream_t st);
void launch_accumulate_scalar(const double* part, int count, double* acc, hipStream_t st);
void launch_sub_inv_diag(float* obar, int64_t ld_obar, const float* om, int64_t ld_om, int64_t p,
                         hipStream_t st);

// batched form (argument blocks in device memory)
// code: the params.batch_order code of the launch (0 = default), which also picks the
// workgroups per CU the kernel is compiled for (batch_occupancy)
void launch_gemm_f32_batch(const GemmArgs* batch, int ngroups, int max_tiles, int tpp, int epi,
                           int code, hipStream_t st);
void launch_prox_batch(const ProxArgs* batch, int nprob, int nblocks, hipStream_t st);
void launch_trial_fused32_batch(const GemmArgs* gb, const ProxArgs* pb, int ngroups,
                                int max_tiles, int tpp, int nprox_rows, int code,
                                hipStream_t st);
void launch_finalize_batch(const FinArgs* batch, int nprob, hipStream_t st);
void launch_fit_init_batch(const FinArgs* batch, int nprob, hipStream_t st);
void launch_init_state_batch(LsState* ls, int nprob, int nlam, const double* lam,
                             const double* inv_n, const double* L, double tau0, double beta,
                             double tol, int max_iter, hipStream_t st, int warm_tau = 0);
void launch_share_L_batch(LsState* ls, int nprob, int nlam, hipStream_t st);

}  // namespace accord
