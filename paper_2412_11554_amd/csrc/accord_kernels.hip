// HIP kernels of the ACCORD-FBS hot path for gfx950 (MI355X).
//
//   k_gemm_f32     FP32 MFMA (v_mfma_f32_16x16x4f32) GEMM, LDS double-buffered
//                  128x128 tiles, XCD-aware tile order
//   k_gemm_bf16pp  256x256 bf16 GEMM (v_mfma_f32_32x32x16_bf16) on bf16 (hi) or
//                  hi+lo split operands, 1 or 3 passes, ping-pong schedule: the bf16
//                  forms' gradient
//   k_gemm_fp8w    the same tile on MX-FP8 operands: the FP8 form's gradient
//   k_trial_fused  bf16 forms: prox (eq. 3.5) fused into the trial product (k_trial_fused8:
//                  FP8, k_trial_fused32: FP32), over an M range so that a trial can be
//                  tested on its first M tiles of 256 samples (k_probe_decide)
//   FP32 uses of k_gemm_f32:
//                    gradient  G  = X^T W / n              (Remark 3.1, two-step product)
//                    trial     W+ = W + X Delta, ||X Delta||^2, ||W+||^2 (Alg. 1 test)
//   k_splitk_reduce fixed-order sum of split-K partial tiles + trial epilogue
//                  (k_splitk_reduce_f for the fused tiles)
//   k_prox         fused closed-form prox (eq. 3.5) + FP64 line-search partial sums
//   k_finalize     FP64 acceptance test of Alg. 1, step update, iteration record
//   k_lz_*         Lanczos estimate of L = sigma_max(X^T X / n) (Sec. 3.2)
//   copies / transposes into the padded operand layouts
//   *_batch        the batched form (many problems per launch, tile orders batch_tile)
//   k_support_*, k_reparam, k_prox_adjoint ...  steps after the fit, differentiation form
//
// All cross-workgroup reductions are two-stage (per-workgroup partials, then one
// workgroup summing them in a fixed order), so results are bit-reproducible.
#include <math.h>

#include "accord_internal.h"

namespace accord {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));  // 16-byte staging word

// Streaming accesses (nontemporal hint) for data touched once per launch: Omega+ from
// the trial kernels (read again only by the next iteration's trials, after the
// gradient has streamed G) and the trial kernels' split-K partial tiles (written once,
// read once by the reduce).  Measured at n = 500, p = 5000: the BF16x3 trial group
// drops from 147 to 136 us.  The same hint on W+, G, the Omega / G loads or the plain
// FP32 GEMM's partials (the differentiation form's) made things slower, so those stay
// ordinary accesses.
__device__ __forceinline__ void st_stream(f4 v, f4* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ f4 ld_stream(const f4* p) { return __builtin_nontemporal_load(p); }

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum of NV doubles over NW waves (blockDim.x == 64 NW) through the LDS
// scratch `sh` (NW * NV doubles); result valid in thread 0.
template <int NV, int NW = kThreads / 64>
__device__ inline void block_sum_in(double (&v)[NV], double* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) sh[wave * NV + q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = sh[q];
            for (int w = 1; w < NW; ++w) s += sh[w * NV + q];
            v[q] = s;
        }
    }
    __syncthreads();
}

template <int NV, int NW = kThreads / 64>
__device__ inline void block_sum(double (&v)[NV]) {
    __shared__ double sh[NW * NV];
    block_sum_in<NV, NW>(v, sh);
}

// Sum of `count` rows of a [count][stride] partial array, columns 0..NV-1,
// in a fixed order (thread t takes rows t, t+256, ...).  Valid in thread 0.
template <int NV>
__device__ inline void sum_partials(const double* part, int count, int stride, double (&v)[NV]) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
    for (int r = threadIdx.x; r < count; r += kThreads) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] += part[(int64_t)r * stride + q];
    }
    block_sum<NV>(v);
}

// FP32 value -> bf16 hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest even)
__device__ inline void split_bf16(float x, uint16_t& h, uint16_t& l) {
    const __bf16 bh = (__bf16)x;
    const __bf16 bl = (__bf16)(x - (float)bh);
    h = __builtin_bit_cast(uint16_t, bh);
    l = __builtin_bit_cast(uint16_t, bl);
}

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------
__global__ void k_init_state(LsState* ls, double tau0, double beta, double lambda, double tol,
                             double inv_n, double L, int max_iter, int warm_tau) {
    if (threadIdx.x != 0) return;
    LsState s = {};
    s.tau = tau0;
    s.tau0 = tau0;
    s.beta = beta;
    s.lambda = lambda;
    s.tol = tol;
    s.inv_n = inv_n;
    s.L = L;
    s.inv_L = L > 0 ? 1.0 / L : 0.0;
    s.max_iter = max_iter;
    s.fixed_step = beta >= 1.0;
    s.warm_tau = warm_tau;
    *ls = s;
}

void launch_init_state(LsState* ls, double tau0, double beta, double lambda, double tol,
                       double inv_n, double L, int max_iter, hipStream_t st, int warm_tau) {
    k_init_state<<<1, 64, 0, st>>>(ls, tau0, beta, lambda, tol, inv_n, L, max_iter, warm_tau);
}

// ---------------------------------------------------------------------------
// operand preparation
// ---------------------------------------------------------------------------
// X (n x p row-major) -> Xp (n_pad x p_pad row-major) and Xt (p_pad x n_pad row-major),
// zero padding, plus (if requested) their bf16 hi/lo splits; flags non-finite input
// (bit 1 of ls->bad).
__global__ void __launch_bounds__(kThreads) k_pad_x(const float* __restrict__ X, int64_t n,
                                                    int64_t p, float* __restrict__ Xp,
                                                    int64_t p_pad, float* __restrict__ Xt,
                                                    int64_t n_pad, XSplit sp, LsState* ls) {
    __shared__ float tile[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32;  // column block of X (variable index)
    const int64_t r0 = (int64_t)blockIdx.y * 32;  // row block of X (sample index)
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    bool bad = false;
    for (int rr = ty; rr < 32; rr += 8) {
        const int64_t r = r0 + rr, c = c0 + tx;
        float v = 0.f;
        if (r < n && c < p) {
            v = X[r * p + c];
            bad |= !isfinite(v);
        }
        tile[rr][tx] = v;
        Xp[r * p_pad + c] = v;
        if (sp.xp_h) {
            uint16_t h, l;
            split_bf16(v, h, l);
            sp.xp_h[r * p_pad + c] = h;
            sp.xp_l[r * p_pad + c] = l;
        }
    }
    __syncthreads();
    for (int cc = ty; cc < 32; cc += 8) {
        const int64_t c = c0 + cc, r = r0 + tx;
        const float v = tile[tx][cc];
        Xt[c * n_pad + r] = v;
        if (sp.xt_h) {
            uint16_t h, l;
            split_bf16(v, h, l);
            sp.xt_h[c * n_pad + r] = h;
            sp.xt_l[c * n_pad + r] = l;
        }
    }
    if (bad) atomicOr(&ls->bad, 2);
}

void launch_pad_x(const float* X, int64_t n, int64_t p, float* Xp, int64_t p_pad, float* Xt,
                  int64_t n_pad, XSplit sp, LsState* ls, hipStream_t st) {
    dim3 grid((unsigned)(p_pad / 32), (unsigned)(n_pad / 32));
    k_pad_x<<<grid, kThreads, 0, st>>>(X, n, p, Xp, p_pad, Xt, n_pad, sp, ls);
}

// Column-by-column copy of p columns: dst[j*ld_dst + i] = src[j*ld_src + i] for i < p,
// zero for p <= i < rows.  With check_ls: flags a non-positive diagonal (bit 0) and
// non-finite entries (bit 1).
__global__ void __launch_bounds__(kThreads) k_copy_cols(const float* __restrict__ src,
                                                        int64_t ld_src, float* __restrict__ dst,
                                                        int64_t ld_dst, int64_t p, int64_t rows,
                                                        LsState* ls) {
    int flags = 0;
    for (int64_t j = blockIdx.x; j < p; j += gridDim.x) {
        const float* s = src + j * ld_src;
        float* d = dst + j * ld_dst;
        for (int64_t i = threadIdx.x; i < rows; i += kThreads) {
            float v = i < p ? s[i] : 0.f;
            d[i] = v;
            if (ls) {
                if (!isfinite(v)) flags |= 2;
                if (i == j && !(v > 0.f)) flags |= 1;
            }
        }
    }
    if (ls && flags) atomicOr(&ls->bad, flags);
}

void launch_copy_cols(const float* src, int64_t ld_src, float* dst, int64_t ld_dst, int64_t p,
                      int64_t rows, LsState* check_ls, hipStream_t st) {
    const int64_t blocks = p < 8192 ? p : 8192;
    k_copy_cols<<<(unsigned)blocks, kThreads, 0, st>>>(src, ld_src, dst, ld_dst, p, rows,
                                                       check_ls);
}

// Wt (p rows x ldt) -> W (n x p row-major): W[k*p + j] = Wt[j*ldt + k].
__global__ void __launch_bounds__(kThreads) k_transpose_w(const float* __restrict__ Wt,
                                                          int64_t ldt, int64_t n, int64_t p,
                                                          float* __restrict__ W) {
    __shared__ float tile[32][33];
    const int64_t j0 = (int64_t)blockIdx.x * 32, k0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t j = j0 + jj, k = k0 + tx;
        tile[jj][tx] = (j < p && k < n) ? Wt[j * ldt + k] : 0.f;
    }
    __syncthreads();
    for (int kk = ty; kk < 32; kk += 8) {
        const int64_t k = k0 + kk, j = j0 + tx;
        if (k < n && j < p) W[k * p + j] = tile[tx][kk];
    }
}

void launch_transpose_w(const float* Wt, int64_t ldt, int64_t n, int64_t p, float* W,
                        hipStream_t st) {
    dim3 grid((unsigned)cdiv(p, 32), (unsigned)cdiv(n, 32));
    k_transpose_w<<<grid, kThreads, 0, st>>>(Wt, ldt, n, p, W);
}

// ---------------------------------------------------------------------------
// GEMMs:  C(m, n) = sum_k A[m, k] * B[n, k]   (both operands K-contiguous)
//
// FP32: workgroup tile 128 x 128, 4 waves in a 2 x 2 arrangement, each wave 64 x 64 =
// 4 x 4 blocks of 16 x 16 MFMA outputs.  One K step is staged in LDS and
// double-buffered: the next step's global loads are in flight while the current
// step's MFMAs run.  LDS rows are padded by 16 bytes, so the 16 lanes that read
// 16 rows at one K offset hit distinct banks.
//
//   FP32:    v_mfma_f32_16x16x4f32, 32-wide K steps.  Lane l supplies A row l % 16
//            and B column l % 16 at MFMA-internal k = l / 16.  Each lane reads 4
//            consecutive K values with one 16-byte LDS read and feeds them to 4
//            successive MFMAs (MFMA-internal k = g of step q is tile column 4g + q;
//            A and B use the same map, so only the summation order changes).
//   BF16xP:  v_mfma_f32_16x16x32_bf16.  Lane l supplies 8 consecutive K values of
//            A row l % 16 / B column l % 16 starting at 8 (l / 16).  Operands are
//            pre-split FP32 values x = hi + lo (hi = bf16(x), lo = bf16(x - hi));
//            P = 1 multiplies hi parts only, P = 3 adds hi*lo and lo*hi (the lo*lo
//            term, relative size 2^-16, is dropped).  FP32 accumulation.
//
// The 16 x 16 accumulator holds C(4 (l / 16) + r, l % 16) in register r of lane l.
// ---------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ inline void decode_tile(const GemmArgs& g, int& tile_m, int& tile_n, int& split) {
    // Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
    // Give every XCD a contiguous range of logical tiles so tiles that share operand
    // panels run on the same XCD and hit in its L2.
    const int nblk = gridDim.x, bid = blockIdx.x;
    const int xcd = bid & 7, local = bid >> 3, q8 = nblk >> 3, r8 = nblk & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + local;
    // over the launch's N tiles n_first .. n_first + n_count - 1 (all with n_count 0)
    const int ncnt = g.n_count > 0 ? g.n_count : g.tilesN;
    if (g.splits > 1) {
        // tile_m fastest: the M tiles of one (split, N tile) share the B panel
        tile_m = logical % g.tilesM;
        const int rest = logical / g.tilesM;
        tile_n = g.n_first + rest % ncnt;
        split = rest / ncnt;
    } else {
        // grouped order: bands of 8 M tiles walk across N
        constexpr int GM = 8;
        const int per_group = GM * ncnt;
        const int group = logical / per_group;
        const int first_m = group * GM;
        const int gsize = (g.tilesM - first_m) < GM ? (g.tilesM - first_m) : GM;
        const int in_group = logical - group * per_group;
        tile_m = first_m + in_group % gsize;
        tile_n = g.n_first + in_group / gsize;
        split = 0;
    }
}

// First position p in [lo, hi) of the ascending list a with a[p] >= v (hi if none).
// Uniform across the workgroup.
__device__ inline int first_at_least(const int32_t* a, int lo, int hi, int v) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First trial step of an iteration: tau0 (Alg. 1), or with the warm-start variant
// min(tau0, tau_{t-1} / beta) once an iteration has been accepted.
__device__ inline double start_tau(const LsState& s) {
    if (s.warm_tau && s.iter > 0) {
        const double t = s.tau_acc / s.beta;
        return t < s.tau0 ? t : s.tau0;
    }
    return s.tau0;
}

// Predication and iteration start; returns true if the launch has nothing to do.
__device__ inline bool gemm_skip(const GemmArgs& g) {
    if (g.ls) {
        if (g.pred >= 1 && g.ls->converged) return true;
        if (g.pred >= 2 && g.ls->done) return true;
        if (g.pred >= 3 && g.ls->probe_rej) return true;
        if (g.probe_mode == 1 && g.ls->probe_off) return true;
        if (g.probe_mode == 2 && !g.ls->probe_off) return true;
    }
    if (g.begin_iter && blockIdx.x == 0 && threadIdx.x == 0) {
        // a new iteration starts from tau0 (Alg. 1); nothing else reads these now
        g.ls->done = 0;
        g.ls->trials = 0;
        g.ls->probe_rej = 0;
        g.ls->probe_off = 0;
        g.ls->tau = start_tau(*g.ls);
    }
    return false;
}

// Stores one 4-row accumulator fragment (rows m..m+3 of column n).
//   EPI_GRAD:  C = alpha * acc
//   EPI_TRIAL: C = Wprev + alpha * acc, with FP64 sums of (alpha acc)^2 and C^2 over the
//              valid extent (alpha = 1 in the trial products)
// With Ch/Cl set, the bf16 hi/lo split of the stored value is written as well.
// NT: the FP32 value goes out with the streaming hint (the bf16 gradient's G, written
// in whole 128-byte lines by its column-walk epilogue and read once by the next trials).
// Support bytes of rows m..m+3 of column n (the refit's G mask; all ones without one).
__device__ inline uint32_t load_mask4(const GemmArgs& g, int m, int n) {
    if (!g.cmask || n >= g.N || m >= g.M) return 0x01010101u;
    const int64_t off = (int64_t)n * g.ldc + m;
    if (g.vec_store && m + 3 < g.M) return *(const uint32_t*)(g.cmask + off);
    uint32_t m4 = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) m4 |= (m + r < g.M ? (uint32_t)g.cmask[off + r] : 0u) << (8 * r);
    return m4;
}

// m4: the support bytes of the quad, when the caller loaded them ahead of its stores
// (kNoMask4: load them here).
constexpr uint64_t kNoMask4 = ~0ull;

template <int EPI, bool NT = false>
__device__ inline void store_frag(const GemmArgs& g, f4 v, int m, int n, double (&nv)[2],
                                  uint64_t m4pre = kNoMask4) {
    if (n >= g.N || m >= g.M) return;
    const int64_t off = (int64_t)n * g.ldc + m;
    const bool vec = g.vec_store && m + 3 < g.M;
    v = v * g.alpha;  // EPI_GRAD: 1/n; EPI_TRIAL: 1 (or the adjoint's -tau/n)
    if (EPI == EPI_GRAD && g.cmask) {  // refit: G is zero off the support
        const uint32_t m4 = m4pre != kNoMask4 ? (uint32_t)m4pre : load_mask4(g, m, n);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = ((m4 >> (8 * r)) & 0xffu) ? v[r] : 0.f;
    }
    if (EPI != EPI_GRAD) {
        f4 w = f4{0.f, 0.f, 0.f, 0.f};
        if (g.Wprev) {
            if (vec) {
                w = *(const f4*)(g.Wprev + off);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) w[r] = (m + r < g.M) ? g.Wprev[off + r] : 0.f;
            }
        }
        const f4 out = w + v;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (m + r < g.Mvalid && n < g.Nvalid) {
                nv[0] += (double)v[r] * (double)v[r];
                nv[1] += (double)out[r] * (double)out[r];
            }
        }
        v = out;
    }
    uint16_t h[4], l[4];
    if (g.Ch) {
#pragma unroll
        for (int r = 0; r < 4; ++r) split_bf16(v[r], h[r], l[r]);
    }
    if (vec) {
        if (NT)
            st_stream(v, (f4*)(g.C + off));
        else
            *(f4*)(g.C + off) = v;
        if (g.Ch) {
            *(uint2*)(g.Ch + off) = make_uint2(h[0] | ((uint32_t)h[1] << 16),
                                               h[2] | ((uint32_t)h[3] << 16));
            *(uint2*)(g.Cl + off) = make_uint2(l[0] | ((uint32_t)l[1] << 16),
                                               l[2] | ((uint32_t)l[3] << 16));
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (m + r < g.M) {
                g.C[off + r] = v[r];
                if (g.Ch) {
                    g.Ch[off + r] = h[r];
                    g.Cl[off + r] = l[r];
                }
            }
        }
    }
}

// Epilogue shared by all GEMM kernels (thread t owns fragments (i, j) of its wave).
// Column-walk epilogues turn a wave's 64-column block through LDS 32 rows at a time:
// kEpiLDR floats per column (32 rows + 4, so that 16 lanes writing a quad of rows each
// cover all 64 banks), one region of 64 columns per wave.
constexpr int kEpiLDR = 32 + 4;
constexpr int kEpiFloats = (kWThreads / 64) * 64 * kEpiLDR;  // the 512-thread GEMMs

// Epilogue of the FP32 tile (4 waves of 64 x 64, 16x16 accumulators).  EPI_GRAD walks
// the tile column by column through LDS (lds: the tile's idle A stages, at least
// 4 x 64 x kEpiLDR floats), so that 8 lanes store 32 consecutive rows of a column (a
// 128-byte line) and G takes the streaming hint.  STREAM: partial tiles
// written with the streaming hint (the fused FP32 trial; the plain GEMM's partials,
// e.g. the differentiation form's, stay ordinary stores).
template <int EPI, bool STREAM = false>
__device__ inline void gemm_epilogue(const GemmArgs& g, f4 (&acc)[4][4], int tile_m, int tile_n,
                                     int split, double* red_lds, double* nrm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (EPI == EPI_PARTIAL) {
        // numbered within the launch's N tiles (split-major), as k_splitk_reduce reads them
        const int ncnt = g.n_count > 0 ? g.n_count : g.tilesN;
        const int64_t ptile = (int64_t)(tile_n - g.n_first) * g.tilesM + tile_m;
        f4* P = (f4*)(g.P + ((int64_t)split * g.tilesM * ncnt + ptile) * (kBM * kBN));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (STREAM)
                    st_stream(acc[i][j], &P[(i * 4 + j) * kThreads + tid]);
                else
                    P[(i * 4 + j) * kThreads + tid] = acc[i][j];
            }
        return;
    }
    double nv[2] = {0.0, 0.0};
    if (EPI == EPI_TRIAL) {
        // the trial products keep the fragment-order stores (the column walk measured no
        // better for them at n = 1000, p = 1e5)
        const int m0 = tile_m * kBM + (wave >> 1) * 64 + (lane >> 4) * 4;
        const int n0 = tile_n * kBN + (wave & 1) * 64 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                store_frag<EPI>(g, acc[i][j], m0 + 16 * i, n0 + 16 * j, nv);
        block_sum_in<2>(nv, red_lds);  // the tile LDS is free after the K loop
        if (tid == 0) {
            nrm[0] = nv[0];
            nrm[1] = nv[1];
        }
        return;
    }
    const int mw = tile_m * kBM + (wave >> 1) * 64, nw = tile_n * kBN + (wave & 1) * 64;
    float* sw = (float*)red_lds + wave * (64 * kEpiLDR);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        // fragment (i, j): rows 16 i + 4 (lane / 16) .. + 3, column 16 j + lane % 16
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                *(f4*)&sw[(16 * j + (lane & 15)) * kEpiLDR + 16 * i + (lane >> 4) * 4] =
                    acc[2 * h + i][j];
        // the refit's support bytes are loaded before any store (a byte load may alias G,
        // so the compiler would not move it above the stores itself)
        uint32_t m4[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = lane + 64 * k;
            m4[k] = load_mask4(g, mw + 32 * h + (e & 7) * 4, nw + (e >> 3));
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = lane + 64 * k;
            const int c = e >> 3, r = (e & 7) * 4;
            store_frag<EPI, true>(g, *(const f4*)&sw[c * kEpiLDR + r], mw + 32 * h + r, nw + c,
                                  nv, m4[k]);
        }
        __syncthreads();
    }
}

constexpr int kLDK32 = kBK32 + 4;  // FP32 LDS row stride (floats)

// One 128 x 128 tile of the FP32 GEMM (tile_m, tile_n, split); nrm receives the
// tile's FP64 norm sums (EPI_TRIAL).
template <int EPI>
__device__ __forceinline__ void gemm_f32_tile(const GemmArgs& g, int tile_m, int tile_n,
                                              int split, double* nrm) {
    __shared__ __attribute__((aligned(16))) float sA[2][kBM * kLDK32];
    __shared__ __attribute__((aligned(16))) float sB[2][kBN * kLDK32];
    const int m0 = tile_m * kBM, n0 = tile_n * kBN;
    const int ksteps = g.K / kBK32;
    const int s_begin = (int)((int64_t)ksteps * split / g.splits);
    const int s_end = (int)((int64_t)ksteps * (split + 1) / g.splits);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lrow = tid >> 3, lcol = (tid & 7) * 4;
    const float* pa[4];
    const float* pb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int ra = m0 + lrow + 32 * i;
        ra = ra < g.M ? ra : g.M - 1;  // rows past the edge load a valid row; never stored
        int rb = n0 + lrow + 32 * i;
        rb = rb < g.N ? rb : g.N - 1;
        pa[i] = g.A + (int64_t)ra * g.lda + lcol;
        pb[i] = g.B + (int64_t)rb * g.ldb + lcol;
    }
    f4 va[4], vb[4];
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int r16 = lane & 15, g4 = (lane >> 4) * 4;

    if (s_begin < s_end) {
        {
            const int64_t ko = (int64_t)s_begin * kBK32;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                va[i] = *(const f4*)(pa[i] + ko);
                vb[i] = *(const f4*)(pb[i] + ko);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                *(f4*)&sA[0][(lrow + 32 * i) * kLDK32 + lcol] = va[i];
                *(f4*)&sB[0][(lrow + 32 * i) * kLDK32 + lcol] = vb[i];
            }
        }
        __syncthreads();
        int cur = 0;
        for (int s = s_begin; s < s_end; ++s) {
            {   // Unconditional prefetch (the last step re-reads its own rows into the idle
                // buffer): a conditional load would be merged at a branch join, which forces
                // a wait on it before the MFMAs below.  The scheduling barriers keep the
                // loads ahead of the MFMAs and their LDS stores after them, so the load
                // latency hides behind the whole MFMA block.
                const int64_t ko = (int64_t)(s + 1 < s_end ? s + 1 : s) * kBK32;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    va[i] = *(const f4*)(pa[i] + ko);
                    vb[i] = *(const f4*)(pb[i] + ko);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            const float* a_base = &sA[cur][(wm + r16) * kLDK32 + g4];
            const float* b_base = &sB[cur][(wn + r16) * kLDK32 + g4];
#pragma unroll
            for (int kk = 0; kk < kBK32; kk += 16) {
                f4 af[4], bf[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) af[i] = *(const f4*)(a_base + i * 16 * kLDK32 + kk);
#pragma unroll
                for (int j = 0; j < 4; ++j) bf[j] = *(const f4*)(b_base + j * 16 * kLDK32 + kk);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][q], bf[j][q],
                                                                             acc[i][j], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                *(f4*)&sA[cur ^ 1][(lrow + 32 * i) * kLDK32 + lcol] = va[i];
                *(f4*)&sB[cur ^ 1][(lrow + 32 * i) * kLDK32 + lcol] = vb[i];
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    __syncthreads();
    static_assert(sizeof(sA) >= (size_t)(kThreads / 64) * 64 * kEpiLDR * sizeof(float),
                  "the epilogue's LDS regions live in sA");
    gemm_epilogue<EPI>(g, acc, tile_m, tile_n, split, (double*)&sA[0][0], nrm);
}

template <int EPI>
__global__ void __launch_bounds__(kThreads, 2) k_gemm_f32(GemmArgs g) {
    if (gemm_skip(g)) return;
    int tile_m, tile_n, split;
    decode_tile(g, tile_m, tile_n, split);
    if (g.tile_occ && !g.tile_occ[tile_m + tile_n * g.tilesM]) return;  // a zero tile of C
    gemm_f32_tile<EPI>(g, tile_m, tile_n, split,
                       g.norm_part + (int64_t)(tile_m + tile_n * g.tilesM) * kNormCols);
}

// ---------------------------------------------------------------------------
// Wide bf16 GEMM: 256 x 256 workgroup tile, 8 waves (2 along M x 4 along N), each
// wave 128 x 64 = 4 x 2 blocks of v_mfma_f32_32x32x16_bf16, the full-rate bf16
// instruction on gfx950 (the 16x16x32 form issues at about two thirds of it).
// Twice the flops per byte of operand traffic of the 128 x 128 tile, which the
// three-pass form needs to stay ahead of L2.  One workgroup per CU (160 KiB LDS for
// the double-buffered hi/lo stages).
//   32x32x16 operands: lane l supplies row / column l % 32, K values 8 (l / 32) .. +7.
//   Accumulator register r of lane l holds C(8 (r / 4) + 4 (l / 32) + r % 4, l % 32).
// ---------------------------------------------------------------------------
typedef float f16v __attribute__((ext_vector_type(16)));

// Gradient epilogue of the wide GEMMs (32x32 accumulators, each wave a 128 x 64 block
// at rows m0w, columns n0w): the block is turned through the wave's own LDS region
// (sT + wave * 64 * 36 floats, idle after the K loop), 32 rows at a time, so that 8
// lanes store 32 consecutive rows of a column (a 128-byte line) instead of 32 columns
// x 32 bytes per instruction.  Whole lines let G go out with the streaming hint:
// measured at n = 500, p = 5000, the BF16x3 trials that read G next drop from 136 to
// 130 us and the gradient from 115 to 114 us (with partial lines the hint cost the
// gradient 50 us).
template <int EPI>
__device__ __forceinline__ void grad_epilogue_cols(const GemmArgs& g, const f16v (&acc)[4][2],
                                                   float* sT, int m0w, int n0w,
                                                   double (&nv)[2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float* sw = sT + wave * (64 * kEpiLDR);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *(f4*)&sw[((lane & 31) + 32 * j) * kEpiLDR + 8 * q + 4 * (lane >> 5)] =
                    f4{acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2],
                       acc[i][j][4 * q + 3]};
        // the refit's support bytes are loaded before any store (see gemm_epilogue)
        uint32_t m4[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = lane + 64 * k;
            m4[k] = load_mask4(g, m0w + 32 * i + (e & 7) * 4, n0w + (e >> 3));
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = lane + 64 * k;
            const int c = e >> 3, r = (e & 7) * 4;
            store_frag<EPI, true>(g, *(const f4*)&sw[c * kEpiLDR + r], m0w + 32 * i + r,
                                  n0w + c, nv, m4[k]);
        }
        __syncthreads();
    }
}

// Gradient of the bf16 forms (G = X^T W / n on bf16 hi or hi + lo operands, 1 or 3
// passes), with a ping-pong schedule.  Wave w computes rows (w / 4) 128 .. + 127 and
// columns (w % 4) 64 .. + 63 of the 256 x 256 tile; the two halves of the workgroup
// (waves 0-3: rows 0..127, waves 4-7: rows 128..255; one wave of each on every SIMD)
// take turns.  Each K step has two phases separated by barriers: in the first, waves 0-3
// run the step's MFMAs from LDS while waves 4-7 store the B operand of the next step
// (loaded a step earlier) into the other stage and issue the loads of the step after; in
// the second the roles swap (waves 4-7 multiply, waves 0-3 stage A).  So on every SIMD
// one wave multiplies while the other moves data.  Every element is summed over K in a
// fixed order (16-deep slices in K order; per slice hi*hi, hi*lo, lo*hi).  Measured at
// n = 1000, p = 1e5 against the same tile with all eight waves staging and multiplying in
// step (one barrier per K step; the same bits on every fit tried): BF16x3 60.6 against
// 66.4 ms, BF16x1 27.4 against 28.6 ms.
template <int PASSES>
__global__ void __launch_bounds__(kWThreads, 1) k_gemm_bf16pp(GemmArgs g) {
    if (gemm_skip(g)) return;
    constexpr int BK = PASSES == 1 ? 64 : 32;
    constexpr int LDK = BK + 8;
    constexpr int H = PASSES == 1 ? 1 : 2;
    constexpr int CPR = BK / 8;
    constexpr int GT = kWThreads / 2;          // threads per half
    constexpr int ROWS = GT / CPR;             // rows one pass of a half's threads covers
    constexpr int RPT = kWBM / ROWS;           // passes per operand half
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][H][kWBM * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][H][kWBN * LDK];

    int tile_m, tile_n, split;
    decode_tile(g, tile_m, tile_n, split);
    if (g.tile_occ && !g.tile_occ[tile_m + tile_n * g.tilesM]) return;  // a zero tile of C
    const int m0 = tile_m * kWBM, n0 = tile_n * kWBN;
    const int ksteps = g.K / BK;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = wave >> 2;                // 0: multiplies first, stages A; 1: stages B
    const int gt = tid & (GT - 1);
    const int lrow = gt / CPR, lcol = (gt % CPR) * 8;
    // this half's operand (A for half 0, B for half 1): tile base and 32-bit byte offsets
    // per row pass (rows past M / N re-read the last row; 2 x 256 rows x ld < 2^31 bytes)
    const int64_t ld = half == 0 ? g.lda : g.ldb;
    const int lim = half == 0 ? g.M - m0 : g.N - n0;
    const char* const oph = (const char*)((half == 0 ? g.Ah + (int64_t)m0 * g.lda
                                                     : g.Bh + (int64_t)n0 * g.ldb));
    const char* const opl = H == 2 ? (const char*)((half == 0 ? g.Al + (int64_t)m0 * g.lda
                                                              : g.Bl + (int64_t)n0 * g.ldb))
                                   : oph;
    uint32_t off[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        int r = lrow + ROWS * i;
        r = r < lim ? r : lim - 1;
        off[i] = (uint32_t)(((int64_t)r * ld + lcol) * 2);
    }
    u4 v[H][RPT];
    auto load_step = [&](int s) {
        const int64_t kb = (int64_t)(s < ksteps ? s : ksteps - 1) * BK * 2;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            v[0][i] = *(const u4*)(oph + kb + off[i]);
            if (H == 2) v[H - 1][i] = *(const u4*)(opl + kb + off[i]);
        }
    };
    auto store_stage = [&](int st) {
        uint16_t* base = half == 0 ? &sA[st][0][0] : &sB[st][0][0];
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                *(u4*)&base[h * (kWBM * LDK) + (lrow + ROWS * i) * LDK + lcol] = v[h][i];
    };

    f16v acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    const int wm = (wave >> 2) * 128, wn = (wave & 3) * 64;
    const int r32 = lane & 31, k8 = (lane >> 5) * 8;
    auto mfma_step = [&](int cur) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            bf8 ah[4], bh[2];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                ah[i] = *(const bf8*)&sA[cur][0][(wm + 32 * i + r32) * LDK + kk + k8];
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bh[j] = *(const bf8*)&sB[cur][0][(wn + 32 * j + r32) * LDK + kk + k8];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j],
                                                                        0, 0, 0);
            if (PASSES == 3) {
                bf8 al[4], bl[2];
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    bl[j] = *(const bf8*)&sB[cur][H - 1][(wn + 32 * j + r32) * LDK + kk + k8];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j],
                                                                            acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    al[i] = *(const bf8*)&sA[cur][H - 1][(wm + 32 * i + r32) * LDK + kk + k8];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j],
                                                                            acc[i][j], 0, 0, 0);
            }
        }
    };

    // prologue: stage 0 from both halves, then each half's loads of step 1
    load_step(0);
    store_stage(0);
    load_step(1);
    __syncthreads();
    int cur = 0;
    for (int s = 0; s < ksteps; ++s) {
        // phase 1: half 0 multiplies stage cur; half 1 stages B of step s + 1 into the
        // other stage (steps past the end re-store the last step: in bounds, unused) and
        // loads B of step s + 2
        // (the multiplying wave runs at raised issue priority, so that on its SIMD its
        // MFMAs go first and the staging wave fills the gaps: same bits, BF16x3 56.4 ->
        // 54.6 ms at n = 1000, p = 1e5)
        if (half == 0) {
            __builtin_amdgcn_s_setprio(1);
            mfma_step(cur);
            __builtin_amdgcn_s_setprio(0);
        } else {
            store_stage(cur ^ 1);
            load_step(s + 2);
        }
        __syncthreads();
        // phase 2: the roles swap
        if (half == 1) {
            __builtin_amdgcn_s_setprio(1);
            mfma_step(cur);
            __builtin_amdgcn_s_setprio(0);
        } else {
            store_stage(cur ^ 1);
            load_step(s + 2);
        }
        __syncthreads();
        cur ^= 1;
    }

    double nv[2] = {0.0, 0.0};
    static_assert(sizeof(sA) >= kEpiFloats * sizeof(float), "epilogue regions live in sA");
    grad_epilogue_cols<EPI_GRAD>(g, acc, (float*)&sA[0][0][0], m0 + wm, n0 + wn, nv);
}

// Fixed-order sum of the split-K partial tiles, then the trial epilogue.  One
// workgroup per tile.  Thread t first sums the 16 fragments it owned in the GEMM
// kernel (coalesced reads of the partials; each sum over s = 0, 1, ... in order), then
// the tile is turned through LDS so that the epilogue walks W column by column: a
// wave covers two columns of 128 samples, so W, W+ (and its bf16 split) move in whole
// lines.  S > 0 is the split count at compile time, so that a thread's loads of one
// split are issued together (S = 0 takes it from g.splits).  STREAM: the partials are
// read with the streaming hint (those of the fused FP32 trial).
template <int S, bool STREAM>
__global__ void __launch_bounds__(kThreads) k_splitk_reduce(GemmArgs g) {
    if (g.ls) {
        if (g.pred >= 1 && g.ls->converged) return;
        if (g.pred >= 2 && g.ls->done) return;
    }
    constexpr int LDR = kBM + 4;  // LDS floats per column (16 lanes of a quad write hit 64 banks)
    __shared__ __attribute__((aligned(16))) float sT[kBN * LDR];
    // one workgroup per tile of the launch's N tiles n_first .. n_first + n_count - 1
    const int ncnt = g.n_count > 0 ? g.n_count : g.tilesN;
    const int ptile = blockIdx.x;
    const int tile_m = ptile % g.tilesM, tile_n = g.n_first + ptile / g.tilesM;
    const int tile = tile_m + tile_n * g.tilesM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tiles = (int64_t)g.tilesM * ncnt;  // partial tiles per split
    f4 v[16];
#pragma unroll
    for (int idx = 0; idx < 16; ++idx) v[idx] = f4{0.f, 0.f, 0.f, 0.f};
    const int nsplit = S > 0 ? S : g.splits;
    constexpr int kUnroll = S > 0 ? S : 1;
#pragma unroll kUnroll
    for (int s = 0; s < nsplit; ++s) {
        const f4* P = (const f4*)(g.P + ((int64_t)s * tiles + ptile) * (kBM * kBN));
#pragma unroll
        for (int idx = 0; idx < 16; ++idx)
            v[idx] += STREAM ? ld_stream(&P[idx * kThreads + tid]) : P[idx * kThreads + tid];
    }
    // fragment (i, j) of this thread: rows (wave / 2) 64 + 4 (lane / 16) + 16 i .. + 3,
    // column (wave & 1) 64 + lane % 16 + 16 j of the tile
#pragma unroll
    for (int idx = 0; idx < 16; ++idx) {
        const int rl = (wave >> 1) * 64 + (lane >> 4) * 4 + 16 * (idx >> 2);
        const int cl = (wave & 1) * 64 + (lane & 15) + 16 * (idx & 3);
        *(f4*)&sT[cl * LDR + rl] = v[idx];
    }
    __syncthreads();
    double nv[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kBN * (kBM / 4) / kThreads; ++k) {
        const int e = tid + kThreads * k;
        const int cl = e / (kBM / 4), rl = (e % (kBM / 4)) * 4;
        store_frag<EPI_TRIAL>(g, *(const f4*)&sT[cl * LDR + rl], tile_m * kBM + rl,
                              tile_n * kBN + cl, nv);
    }
    block_sum<2>(nv);
    if (tid == 0) {
        g.norm_part[(int64_t)tile * kNormCols + 0] = nv[0];
        g.norm_part[(int64_t)tile * kNormCols + 1] = nv[1];
    }
}

void launch_grad_fp8(const GemmArgs& a, hipStream_t st);
void launch_trial_fused8(const GemmArgs& a, const ProxArgs& px, hipStream_t st);

void launch_gemm(const GemmArgs& a, int epi, int prec, hipStream_t st) {
    const int ncnt = a.n_count > 0 ? a.n_count : a.tilesN;
    const unsigned blocks = (unsigned)((int64_t)a.tilesM * ncnt * a.splits);
    if (prec == PREC_FP8) {  // FP8 form: gradient only, like the bf16 forms
        launch_grad_fp8(a, st);
        return;
    }
    if (prec != PREC_FP32) {
        // bf16 forms: gradient only (their trial products run in k_trial_fused)
        if (prec == PREC_BF16X3)
            k_gemm_bf16pp<3><<<blocks, kWThreads, 0, st>>>(a);
        else
            k_gemm_bf16pp<1><<<blocks, kWThreads, 0, st>>>(a);
        return;
    }
    if (epi == EPI_GRAD)
        k_gemm_f32<EPI_GRAD><<<blocks, kThreads, 0, st>>>(a);
    else if (epi == EPI_TRIAL)
        k_gemm_f32<EPI_TRIAL><<<blocks, kThreads, 0, st>>>(a);
    else
        k_gemm_f32<EPI_PARTIAL><<<blocks, kThreads, 0, st>>>(a);
}

template <bool STREAM>
void launch_splitk_reduce_t(const GemmArgs& a, hipStream_t st) {
    const int ncnt = a.n_count > 0 ? a.n_count : a.tilesN;
    const unsigned blocks = (unsigned)((int64_t)a.tilesM * ncnt);
    switch (a.splits) {
        case 2: k_splitk_reduce<2, STREAM><<<blocks, kThreads, 0, st>>>(a); break;
        case 3: k_splitk_reduce<3, STREAM><<<blocks, kThreads, 0, st>>>(a); break;
        case 4: k_splitk_reduce<4, STREAM><<<blocks, kThreads, 0, st>>>(a); break;
        case 5: k_splitk_reduce<5, STREAM><<<blocks, kThreads, 0, st>>>(a); break;
        case 6: k_splitk_reduce<6, STREAM><<<blocks, kThreads, 0, st>>>(a); break;
        case 7: k_splitk_reduce<7, STREAM><<<blocks, kThreads, 0, st>>>(a); break;
        case 8: k_splitk_reduce<8, STREAM><<<blocks, kThreads, 0, st>>>(a); break;
        default: k_splitk_reduce<0, STREAM><<<blocks, kThreads, 0, st>>>(a); break;
    }
}

void launch_splitk_reduce(const GemmArgs& a, hipStream_t st) {
    launch_splitk_reduce_t<false>(a, st);
}

// ---------------------------------------------------------------------------
// Fused prox (eq. 3.5) + line-search partial sums.
//
// Streams Omega and G once (16-byte loads), writes Omega+ and Delta (in the trial
// GEMM's operand format: FP32, bf16 hi, or bf16 hi + lo), and keeps per-thread
// FP64 sums of ||Delta||^2, <Delta, G>, ||Omega+||_1, sum log Omega+_jj, the
// off-diagonal nonzero count and ||Omega+||_F^2.  Off-diagonal entries are
// soft-thresholded in FP32; the diagonal root is evaluated in FP64 in the
// cancellation-free form  b >= 0: (b + r)/2,  b < 0: 2 tau / (r - b),
// r = sqrt(b^2 + 4 tau), which equals (b + r)/2 exactly in real arithmetic.
// The sums use the Delta the GEMM will multiply (the split's hi + lo, or hi).
// ---------------------------------------------------------------------------
struct ProxAcc {
    double d2 = 0, dg = 0, l1 = 0, logd = 0, nnz = 0, fro = 0;
};

__device__ inline float prox_one(float o, float gv, bool diag, double tau, double lam,
                                 float tau_f, float thr_f) {
    if (diag) {
        const double y = (double)o - tau * (double)gv;
        const double b = y - tau * lam;
        const double r = sqrt(b * b + 4.0 * tau);
        const double w = b >= 0.0 ? 0.5 * (b + r) : (2.0 * tau) / (r - b);
        return (float)w;
    }
    const float a = fmaf(-tau_f, gv, o);
    const float s = fabsf(a) - thr_f;
    return s > 0.f ? copysignf(s, a) : 0.f;
}

__device__ inline void prox_account(ProxAcc& acc, float dl, float gv, float nw, bool diag,
                                    bool valid, bool reduce_only) {
    if (!valid) return;
    if (!reduce_only) {
        acc.d2 += (double)dl * (double)dl;
        acc.dg += (double)dl * (double)gv;
    }
    acc.l1 += fabs((double)nw);
    acc.fro += (double)nw * (double)nw;
    if (diag) {
        acc.logd += nw > 0.f ? log((double)nw) : -INFINITY;
    } else if (nw != 0.f) {
        acc.nnz += 1.0;
    }
}

// Delta as the GEMM sees it: DOUT 0 = FP32, 1 = bf16(Delta), 2 = hi + lo
template <int DOUT>
__device__ inline float delta_repr(float dl, uint16_t& h, uint16_t& l) {
    if (DOUT == 0) return dl;
    split_bf16(dl, h, l);
    const float fh = (float)__builtin_bit_cast(__bf16, h);
    if (DOUT == 1) return fh;
    return fh + (float)__builtin_bit_cast(__bf16, l);
}

template <int DOUT>
__device__ __forceinline__ void prox_run(const ProxArgs& a) {
    double tau = a.tau, lam = a.lambda;
    if (a.ls) {
        if (a.ls->done || a.ls->converged) return;
        tau = a.ls->tau;
        lam = a.ls->lambda;
    }
    const float tau_f = (float)tau, thr_f = (float)(tau * lam);
    const int64_t n4 = a.total >> 2;
    const int64_t per = (n4 + gridDim.x - 1) / gridDim.x;
    const int64_t q_begin = (int64_t)blockIdx.x * per;
    const int64_t q_end = (q_begin + per) < n4 ? (q_begin + per) : n4;
    ProxAcc acc;
    const f4* om4 = (const f4*)a.om;
    const f4* g4 = (const f4*)a.g;
    f4* on4 = (f4*)a.om_new;
    f4* d4 = (f4*)a.d;
    uint2* dh2 = (uint2*)a.dh;
    uint2* dl2 = (uint2*)a.dl;

    int64_t q = q_begin + threadIdx.x;
    int64_t e = q << 2;
    int64_t col = e / a.ld, row = e - col * a.ld;
    for (; q < q_end; q += kThreads) {
        const f4 o = om4[q];
        const f4 gv = a.reduce_only ? f4{0.f, 0.f, 0.f, 0.f} : g4[q];
        f4 nw, dv;
        uint16_t h[4], l[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int64_t r = row + u, c = col;
            if (r >= a.ld) {
                r -= a.ld;
                c += 1;
            }
            const bool diag = (r == c);
            nw[u] = a.reduce_only ? o[u] : prox_one(o[u], gv[u], diag, tau, lam, tau_f, thr_f);
            dv[u] = delta_repr<DOUT>(nw[u] - o[u], h[u], l[u]);
            prox_account(acc, dv[u], gv[u], nw[u], diag, r < a.p, a.reduce_only);
        }
        if (!a.reduce_only) {
            on4[q] = nw;
            if (DOUT == 0) {
                if (d4) d4[q] = dv;
            } else {
                dh2[q] = make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
                if (DOUT == 2)
                    dl2[q] = make_uint2(l[0] | ((uint32_t)l[1] << 16), l[2] | ((uint32_t)l[3] << 16));
            }
        }
        row += a.step_row;
        col += a.step_col;
        if (row >= a.ld) {
            row -= a.ld;
            col += 1;
        }
    }
    // scalar tail (total not a multiple of 4), handled by the last workgroup
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x < (int)(a.total - (n4 << 2))) {
        const int64_t ee = (n4 << 2) + threadIdx.x;
        const int64_t c = ee / a.ld, r = ee - c * a.ld;
        const float o = a.om[ee];
        const float gv = a.reduce_only ? 0.f : a.g[ee];
        const bool diag = (r == c);
        float nw = a.reduce_only ? o : prox_one(o, gv, diag, tau, lam, tau_f, thr_f);
        uint16_t h, l;
        const float dv = delta_repr<DOUT>(nw - o, h, l);
        prox_account(acc, dv, gv, nw, diag, r < a.p, a.reduce_only);
        if (!a.reduce_only) {
            a.om_new[ee] = nw;
            if (DOUT == 0) {
                if (a.d) a.d[ee] = dv;
            } else {
                a.dh[ee] = h;
                if (DOUT == 2) a.dl[ee] = l;
            }
        }
    }
    double v[6] = {acc.d2, acc.dg, acc.l1, acc.logd, acc.nnz, acc.fro};
    block_sum<6>(v);
    if (threadIdx.x == 0) {
        double* out = a.part + (int64_t)blockIdx.x * kPartCols;
#pragma unroll
        for (int k = 0; k < 6; ++k) out[k] = v[k];
        out[6] = 0.0;
        out[7] = 0.0;
    }
}

template <int DOUT>
__global__ void __launch_bounds__(kThreads) k_prox(ProxArgs a) {
    prox_run<DOUT>(a);
}

// ---------------------------------------------------------------------------
// Fused trial kernel of the FP32 form: prox (eq. 3.5) + trial product W+ = W + X Delta.
//
// The FP32 GEMM tile (128 x 128, 4 waves of 64 x 64 on v_mfma_f32_16x16x4f32, two
// workgroups per CU) with its B operand produced in place: each K step loads 32 rows
// of the tile's 128 columns of Omega and G, applies the prox in registers and writes
// Delta = Omega+ - Omega (FP32) into the LDS stage.  The workgroup with tile_m 0 owns
// the column block: it stores Omega+ and keeps the line-search sums (FP32 over a
// thread's 16 entries of a step, FP64 beyond; one row per (tile_n, split) of
// px.part).  Delta never goes through HBM and the separate prox pass disappears.
// Off-diagonal entries take the FP32 soft threshold without a branch; the diagonal
// entries a column can hold (in 8 of its K steps) are redone with the FP64 root under
// a wave-uniform branch.  Rows past p are zero in Omega and G, so they produce zeros.
//
// Column j of the tile belongs to the problem whose columns start at jbase; it is a
// column of that problem when j - jbase < p.  Loads read column min(j, ncols - 1) of
// the buffers: in the single fit the buffers hold exactly p columns (ncols = p) and the
// products of the columns past p are never stored; in the batched form every
// problem's columns are padded to a multiple of 128 with zero columns, which produce
// Delta = 0 and W+ = W there.  Only columns of the problem store Omega+ and count.
// ---------------------------------------------------------------------------
// LIST: the K steps come from g.kstep_ptr / kstep_idx (a refit's support).  A compile-time
// choice: with a runtime test on the list pointer the compiler loads list entries inside
// the K loop, and since vector loads retire in order, their waits drain the operand
// prefetch (measured at n = 1000, p = 1e5: the plain fit's BF16x1 trial launches 20-27 %
// slower, BF16x3 7-8 %).
template <int EPI, bool LIST = false>
__device__ __forceinline__ void trial_fused32_tile(const GemmArgs& g, const ProxArgs& px,
                                                   int tile_m, int tile_n, int split, int jbase,
                                                   int ncols, double tau, double lam,
                                                   double* part_row, double* nrm) {
    __shared__ __attribute__((aligned(16))) float sA[2][kBM * kLDK32];
    __shared__ __attribute__((aligned(16))) float sB[2][kBN * kLDK32];
    const bool owner = tile_m == 0;
    const float tau_f = (float)tau, thr_f = (float)(tau * lam);
    const int m0 = tile_m * kBM, n0 = tile_n * kBN;
    // the split's share of the column block's K steps, as positions in a step sequence:
    // every step (kstep_idx null), or the column block's list of steps that can hold a
    // nonzero Delta (a refit's support); the split keeps its K range either way, so the
    // partial sums group the same products as when every step is walked
    const int32_t* kidx = LIST ? g.kstep_idx : nullptr;
    int s_begin, s_end;
    {
        const int ksteps = g.K / kBK32;
        s_begin = (int)((int64_t)ksteps * split / g.splits);
        s_end = (int)((int64_t)ksteps * (split + 1) / g.splits);
        if (kidx) {
            const int c0 = g.kstep_ptr[tile_n], c1 = g.kstep_ptr[tile_n + 1];
            s_begin = first_at_least(kidx, c0, c1, s_begin);
            s_end = first_at_least(kidx, c0, c1, s_end);
        }
    }
#define KS32(pos) (kidx ? kidx[(pos)] : (pos))

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lrow = tid >> 3, lcol = (tid & 7) * 4;
    const float* pa[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int ra = m0 + lrow + 32 * i;
        ra = ra < g.M ? ra : g.M - 1;  // rows past the edge load a valid row; never stored
        pa[i] = g.A + (int64_t)ra * g.lda + lcol;
    }
    // Omega / G / Omega+: per-workgroup base plus 32-bit byte offsets (p <= 2^20, so a
    // 128-column block spans less than 2^31 bytes)
    const char* b_om = (const char*)(px.om + (int64_t)n0 * px.ld);
    const char* b_g = (const char*)(px.g + (int64_t)n0 * px.ld);
    char* b_on = (char*)(px.om_new + (int64_t)n0 * px.ld);
    uint32_t ob[4];
    int jcol[4];
    bool jvalid[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = n0 + lrow + 32 * i;
        jvalid[i] = j - jbase < px.p;
        jcol[i] = j - jbase;  // column within the problem: the diagonal is row jcol
        const int jc = j < ncols ? j : ncols - 1;
        ob[i] = (uint32_t)(((int64_t)(jc - n0) * px.ld + lcol) * 4);
    }
    f4 va[4], vo[4], vg[4];
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    ProxAcc pacc;

    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int r16 = lane & 15, g4 = (lane >> 4) * 4;

#define F32_LOAD(step)                                                                    \
    do {                                                                                  \
        const int64_t ka_ = (int64_t)(step) * kBK32;                                      \
        const uint32_t ko_ = (uint32_t)(step) * (kBK32 * 4);                              \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                   \
            va[i] = *(const f4*)(pa[i] + ka_);                                            \
            vo[i] = *(const f4*)(b_om + (ob[i] + ko_));                                   \
            vg[i] = *(const f4*)(b_g + (ob[i] + ko_));                                    \
        }                                                                                 \
    } while (0)

    // prox of the staged step into LDS stage `buf`; the owner stores Omega+ and counts
#define F32_PRODUCE(buf, step)                                                            \
    do {                                                                                  \
        f4 nw_[4];                                                                        \
        _Pragma("unroll") for (int i = 0; i < 4; ++i)                                     \
            _Pragma("unroll") for (int u = 0; u < 4; ++u) {                               \
                const float a_ = fmaf(-tau_f, vg[i][u], vo[i][u]);                        \
                const float t_ = fabsf(a_) - thr_f;                                       \
                nw_[i][u] = t_ > 0.f ? copysignf(t_, a_) : 0.f;                           \
            }                                                                             \
        const int k0_ = (step) * kBK32 + lcol;                                            \
        bool hd_[4];                                                                      \
        bool any_ = false;                                                                \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                   \
            hd_[i] = jvalid[i] && (unsigned)(jcol[i] - k0_) < 4u;                         \
            any_ = any_ || hd_[i];                                                        \
        }                                                                                 \
        double logd_ = 0.0, nzd_ = 0.0;                                                   \
        if (__builtin_amdgcn_ballot_w64(any_)) {                                          \
            _Pragma("unroll") for (int i = 0; i < 4; ++i) {                               \
                if (hd_[i]) {                                                             \
                    const int du_ = jcol[i] - k0_;                                        \
                    const float od_ = du_ == 0 ? vo[i][0] : du_ == 1 ? vo[i][1]           \
                                    : du_ == 2 ? vo[i][2] : vo[i][3];                     \
                    const float gd_ = du_ == 0 ? vg[i][0] : du_ == 1 ? vg[i][1]           \
                                    : du_ == 2 ? vg[i][2] : vg[i][3];                     \
                    const float wd_ = prox_one(od_, gd_, true, tau, lam, tau_f, thr_f);   \
                    _Pragma("unroll") for (int u = 0; u < 4; ++u)                         \
                        nw_[i][u] = u == du_ ? wd_ : nw_[i][u];                           \
                    logd_ += wd_ > 0.f ? log((double)wd_) : -INFINITY;                    \
                    nzd_ += wd_ != 0.f ? 1.0 : 0.0;                                       \
                }                                                                         \
            }                                                                             \
        }                                                                                 \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                   \
            *(f4*)&sA[(buf)][(lrow + 32 * i) * kLDK32 + lcol] = va[i];                    \
            *(f4*)&sB[(buf)][(lrow + 32 * i) * kLDK32 + lcol] = nw_[i] - vo[i];           \
        }                                                                                 \
        if (owner) {                                                                      \
            const uint32_t ko_ = (uint32_t)(step) * (kBK32 * 4);                          \
            float sd2_ = 0.f, sdg_ = 0.f, sl1_ = 0.f, sfr_ = 0.f, snz_ = 0.f;            \
            _Pragma("unroll") for (int i = 0; i < 4; ++i) {                               \
                if (jvalid[i]) st_stream(nw_[i], (f4*)(b_on + (ob[i] + ko_)));           \
                const float lv_ = jvalid[i] ? 1.f : 0.f;                                  \
                _Pragma("unroll") for (int u = 0; u < 4; ++u) {                           \
                    const float dv_ = (nw_[i][u] - vo[i][u]) * lv_;                       \
                    const float nv_ = nw_[i][u] * lv_;                                    \
                    sd2_ = fmaf(dv_, dv_, sd2_);                                          \
                    sdg_ = fmaf(dv_, vg[i][u], sdg_);                                     \
                    sl1_ += fabsf(nv_);                                                   \
                    sfr_ = fmaf(nv_, nv_, sfr_);                                          \
                    snz_ += nv_ != 0.f ? 1.f : 0.f;                                       \
                }                                                                         \
            }                                                                             \
            pacc.d2 += (double)sd2_;                                                      \
            pacc.dg += (double)sdg_;                                                      \
            pacc.l1 += (double)sl1_;                                                      \
            pacc.fro += (double)sfr_;                                                     \
            pacc.nnz += (double)snz_ - nzd_;                                              \
            pacc.logd += logd_;                                                           \
        }                                                                                 \
    } while (0)

    if (s_begin < s_end) {
        F32_LOAD(KS32(s_begin));
        F32_PRODUCE(0, KS32(s_begin));
        __syncthreads();
        int cur = 0;
        for (int s = s_begin; s < s_end; ++s) {
            const bool more = s + 1 < s_end;
            if (more) F32_LOAD(KS32(s + 1));
            __builtin_amdgcn_sched_barrier(0);
            const float* a_base = &sA[cur][(wm + r16) * kLDK32 + g4];
            const float* b_base = &sB[cur][(wn + r16) * kLDK32 + g4];
#pragma unroll
            for (int kk = 0; kk < kBK32; kk += 16) {
                f4 af[4], bf[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) af[i] = *(const f4*)(a_base + i * 16 * kLDK32 + kk);
#pragma unroll
                for (int j = 0; j < 4; ++j) bf[j] = *(const f4*)(b_base + j * 16 * kLDK32 + kk);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][q], bf[j][q],
                                                                             acc[i][j], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (more) F32_PRODUCE(cur ^ 1, KS32(s + 1));
            __syncthreads();
            cur ^= 1;
        }
    }
#undef F32_LOAD
#undef F32_PRODUCE
#undef KS32
    __syncthreads();
    double* red = (double*)&sA[0][0];  // LDS is free after the K loop
    if (owner) {
        double v[6] = {pacc.d2, pacc.dg, pacc.l1, pacc.logd, pacc.nnz, pacc.fro};
        block_sum_in<6>(v, red);
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < 6; ++k) part_row[k] = v[k];
            part_row[6] = 0.0;
            part_row[7] = 0.0;
        }
        __syncthreads();
    }
    static_assert(sizeof(sA) >= (size_t)(kThreads / 64) * 64 * kEpiLDR * sizeof(float),
                  "the epilogue's LDS regions live in sA");
    gemm_epilogue<EPI, true>(g, acc, tile_m, tile_n, split, red, nrm);
}

template <int EPI, bool LIST>
__global__ void __launch_bounds__(kThreads, 2) k_trial_fused32(GemmArgs g, ProxArgs px) {
    if (gemm_skip(g)) return;
    int tile_m, tile_n, split;
    decode_tile(g, tile_m, tile_n, split);
    trial_fused32_tile<EPI, LIST>(g, px, tile_m, tile_n, split, 0, (int)px.p, px.ls->tau,
                            px.ls->lambda,
                            px.part + ((int64_t)tile_n * g.splits + split) * kPartCols,
                            g.norm_part + (int64_t)(tile_m + tile_n * g.tilesM) * kNormCols);
}

void launch_trial_fused32(const GemmArgs& a, const ProxArgs& px, hipStream_t st) {
    const unsigned blocks = (unsigned)((int64_t)a.tilesM * a.tilesN * a.splits);
    const bool list = a.kstep_idx != nullptr;
    if (a.splits > 1) {
        if (list) k_trial_fused32<EPI_PARTIAL, true><<<blocks, kThreads, 0, st>>>(a, px);
        else k_trial_fused32<EPI_PARTIAL, false><<<blocks, kThreads, 0, st>>>(a, px);
        launch_splitk_reduce_t<true>(a, st);
    } else {
        if (list) k_trial_fused32<EPI_TRIAL, true><<<blocks, kThreads, 0, st>>>(a, px);
        else k_trial_fused32<EPI_TRIAL, false><<<blocks, kThreads, 0, st>>>(a, px);
    }
}

// Prox sums of a fused trial workgroup: row tile_n * stride + split (stride =
// part_stride, or the launch's split count), and, from split 0, zero rows for the splits
// of the column block that this launch does not run (a column block's rows are summed
// whole, whichever launch covered it).
__device__ inline void fused_sums_out(const GemmArgs& g, const ProxArgs& px, int tile_n,
                                      int split, const double (&v)[6]) {
    const int stride = g.part_stride > 0 ? g.part_stride : g.splits;
    double* out = px.part + ((int64_t)tile_n * stride + split) * kPartCols;
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k] = v[k];
    out[6] = 0.0;
    out[7] = 0.0;
    if (split == 0)
        for (int s = g.splits; s < stride; ++s)
#pragma unroll
            for (int k = 0; k < kPartCols; ++k)
                px.part[((int64_t)tile_n * stride + s) * kPartCols + k] = 0.0;
}

// Split-K partial tile of (tile_m, tile_n, split), numbered within the launch's column
// blocks n_first .. n_first + ncnt - 1 (split-major, then the tile in column-major tile
// order); k_splitk_reduce_f reads the same numbering.
__device__ inline int64_t fused_partial_tile(const GemmArgs& g, int ncnt, int tile_m,
                                             int tile_n, int split) {
    return ((int64_t)split * ncnt + (tile_n - g.n_first)) * g.tilesM + tile_m;
}

// B-operand producer of k_trial_fused for stage `buf` holding K step `step`, written
// without branches so that it shares one basic block with the MFMAs of the previous
// stage and the scheduler can interleave the two: prox of the 2 x 4 staged Omega / G
// values with the FP32 soft threshold, Delta -> bf16 hi (/ lo) into LDS, Omega+ kept
// in `onw` for the owner's store, and the line-search sums (FP32 over the 8 entries,
// FP64 beyond; multiplied by `live`, 0 for the clamped copy of the last step).  Also
// stores the staged X rows.  The one diagonal entry a column can have is corrected
// after the block by FUSED_DIAG.  Columns past p read and write the zero padding
// columns of Omega, G and Omega+, so they produce zeros without a test.  (Macros keep
// every staging array in registers.)
#define FUSED_PRODUCE(buf, step, vo, vg, va, live)                                        \
    do {                                                                                  \
        _Pragma("unroll") for (int q = 0; q < H * 2; ++q)                                 \
            *(u4*)&sA[(buf)][q >> 1][(arow + 128 * (q & 1)) * LDK + acol] = va[q];         \
        float sd2_ = 0.f, sdg_ = 0.f, sl1_ = 0.f, sfr_ = 0.f, snz_ = 0.f;                \
        _Pragma("unroll") for (int q = 0; q < 2; ++q) {                                   \
            const f4 o_ = vo[q], g_ = vg[q];                                              \
            uint16_t h_[4], l_[4];                                                        \
            _Pragma("unroll") for (int u = 0; u < 4; ++u) {                               \
                const float a_ = fmaf(-tau_f, g_[u], o_[u]);                              \
                const float t_ = fabsf(a_) - thr_f;                                       \
                const float nw_ = t_ > 0.f ? copysignf(t_, a_) : 0.f;                     \
                const float dv_ = delta_repr<DOUT>(nw_ - o_[u], h_[u], l_[u]);            \
                sd2_ = fmaf(dv_, dv_, sd2_);                                              \
                sdg_ = fmaf(dv_, g_[u], sdg_);                                            \
                sl1_ += fabsf(nw_);                                                       \
                sfr_ = fmaf(nw_, nw_, sfr_);                                              \
                snz_ += nw_ != 0.f ? 1.f : 0.f;                                           \
                onw[q][u] = nw_;                                                          \
            }                                                                             \
            const int lo_ = (bc + 64 * q) * LDK + br;                                     \
            *(uint2*)&sB[(buf)][0][lo_] =                                                 \
                make_uint2(h_[0] | ((uint32_t)h_[1] << 16), h_[2] | ((uint32_t)h_[3] << 16)); \
            if (H == 2)                                                                   \
                *(uint2*)&sB[(buf)][H - 1][lo_] = make_uint2(                             \
                    l_[0] | ((uint32_t)l_[1] << 16), l_[2] | ((uint32_t)l_[3] << 16));    \
        }                                                                                 \
        const float lv_ = (live) ? 1.f : 0.f;                                             \
        pacc.d2 += (double)(sd2_ * lv_);                                                  \
        pacc.dg += (double)(sdg_ * lv_);                                                  \
        pacc.l1 += (double)(sl1_ * lv_);                                                  \
        pacc.fro += (double)(sfr_ * lv_);                                                 \
        pacc.nnz += (double)(snz_ * lv_);                                                 \
    } while (0)

// Diagonal entries of stage `buf` (rows step*BK + br .. + 3 of column jcol[q]): the
// positive root of eq. 3.5 in FP64 replaces the soft-threshold value in LDS, in `onw`
// and in the sums (the diagonal is not an off-diagonal nonzero; it adds log w).  Only
// a few stages of a column block hold diagonal entries, so this is a rarely taken,
// wave-uniform branch after the producer's block.
#define FUSED_DIAG(buf, step, vo, vg, live)                                               \
    do {                                                                                  \
        const int k0_ = (step) * BK + br;                                                 \
        bool hd_[2];                                                                      \
        _Pragma("unroll") for (int q = 0; q < 2; ++q)                                     \
            hd_[q] = (live) && jvalid[q] && (unsigned)(jcol[q] - k0_) < 4u;               \
        if (__builtin_amdgcn_ballot_w64(hd_[0] || hd_[1])) {                              \
            _Pragma("unroll") for (int q = 0; q < 2; ++q) {                               \
                if (hd_[q]) {                                                             \
                    const int du_ = jcol[q] - k0_;                                        \
                    const f4 o_ = vo[q], g_ = vg[q];                                      \
                    const float od_ = du_ == 0 ? o_[0] : du_ == 1 ? o_[1] : du_ == 2 ? o_[2] : o_[3]; \
                    const float gd_ = du_ == 0 ? g_[0] : du_ == 1 ? g_[1] : du_ == 2 ? g_[2] : g_[3]; \
                    const float sv_ = du_ == 0 ? onw[q][0] : du_ == 1 ? onw[q][1]         \
                                    : du_ == 2 ? onw[q][2] : onw[q][3];                   \
                    const float dv_ = prox_one(od_, gd_, true, tau, lam, tau_f, thr_f);   \
                    uint16_t hs_, ls_, hd2_, ld2_;                                        \
                    const double es_ = delta_repr<DOUT>(sv_ - od_, hs_, ls_);             \
                    const double ed_ = delta_repr<DOUT>(dv_ - od_, hd2_, ld2_);           \
                    const int lo_ = (bc + 64 * q) * LDK + br + du_;                       \
                    sB[(buf)][0][lo_] = hd2_;                                             \
                    if (H == 2) sB[(buf)][H - 1][lo_] = ld2_;                             \
                    _Pragma("unroll") for (int u = 0; u < 4; ++u)                         \
                        onw[q][u] = u == du_ ? dv_ : onw[q][u];                           \
                    pacc.d2 += ed_ * ed_ - es_ * es_;                                     \
                    pacc.dg += (ed_ - es_) * (double)gd_;                                 \
                    pacc.l1 += fabs((double)dv_) - fabs((double)sv_);                     \
                    pacc.fro += (double)dv_ * (double)dv_ - (double)sv_ * (double)sv_;    \
                    pacc.nnz -= sv_ != 0.f ? 1.0 : 0.0;                                   \
                    pacc.logd += dv_ > 0.f ? log((double)dv_) : -INFINITY;                \
                }                                                                         \
            }                                                                             \
        }                                                                                 \
    } while (0)

// The owning M tile writes Omega+ of stage `step` (padding columns included: zeros).
#define FUSED_STORE(step, live)                                                           \
    do {                                                                                  \
        if (owner && (live)) {                                                            \
            const uint32_t ko_ = (uint32_t)(step) * (BK * 4);                             \
            _Pragma("unroll") for (int q = 0; q < 2; ++q)                                 \
                st_stream(onw[q], (f4*)(b_on + (ob[q] + ko_)));                           \
        }                                                                                 \
    } while (0)

// ---------------------------------------------------------------------------
// Fused trial kernel of the bf16 forms: prox (eq. 3.5) + trial product.
//
// The B operand of X Delta is produced in place: each step streams 32 rows of 128
// columns of Omega and G (FP32, column-major, so K-contiguous), applies the
// closed-form prox in registers, and writes the bf16 hi (and lo) parts of
// Delta = Omega+ - Omega straight into the LDS stage.  The workgroup with tile_m 0
// owns its column block: it also writes Omega+ and keeps the FP64 line-search sums
// (||Delta||^2, <Delta, G>, ||Omega+||_1, sum log Omega+_jj, nnz, ||Omega+||_F^2);
// the other M tiles recompute Delta for their rows of X only.  Delta never goes
// through HBM, and the separate prox pass disappears.
// Tile 256 x 128, 8 waves (4 along M x 2 along N), each 64 x 64 = 2 x 2 blocks of
// v_mfma_f32_32x32x16_bf16; tile_m is the fastest tile index, so the M tiles of a
// column block run together on one XCD and share Omega / G through its L2.
// ---------------------------------------------------------------------------
// LIST: K steps from a list, as in trial_fused32_tile.
template <int PASSES, int EPI, bool LIST>
__global__ void __launch_bounds__(kWThreads, 1) k_trial_fused(GemmArgs g, ProxArgs px) {
    if (gemm_skip(g)) return;
    constexpr int BK = 32;
    constexpr int LDK = BK + 8;                  // bf16 per LDS row (16-byte pad)
    constexpr int H = PASSES == 1 ? 1 : 2;
    constexpr int DOUT = PASSES == 1 ? 1 : 2;
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][H][kFBM * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][H][kFBN * LDK];

    const double tau = px.ls->tau, lam = px.ls->lambda;
    const float tau_f = (float)tau, thr_f = (float)(tau * lam);

    // tile order: tile_m fastest, then tile_n, then split (XCD-contiguous ranges), over
    // the launch's M tiles m_first .. m_first + m_count - 1 and column blocks n_first ..
    // n_first + n_count - 1
    const int nblk = gridDim.x, bid = blockIdx.x;
    const int xcd = bid & 7, local = bid >> 3, q8 = nblk >> 3, r8 = nblk & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + local;
    const int mcnt = g.m_count > 0 ? g.m_count : g.tilesM;
    const int ncnt = g.n_count > 0 ? g.n_count : g.tilesN;
    const int tile_m = g.m_first + logical % mcnt;
    const int tile_n = g.n_first + (logical / mcnt) % ncnt;
    const int split = logical / (mcnt * ncnt);
    const bool owner = tile_m == g.store_m;         // stores Omega+
    const bool sums_owner = tile_m == g.sums_m;     // writes the prox sums
    const int m0 = tile_m * kFBM, n0 = tile_n * kFBN;
    // The split's share of the column block's K steps, as positions in a step sequence:
    // every step (kstep_idx null), or the column block's list of steps that can hold a
    // nonzero Delta (a refit's support)
    // (the split keeps its K range either way, so the FP32 partial sums group the same
    // products as when every step is walked)
    const int32_t* kidx = LIST ? g.kstep_idx : nullptr;
    int s_begin, s_end;
    {
        const int ksteps = g.K / BK;
        s_begin = (int)((int64_t)ksteps * split / g.splits);
        s_end = (int)((int64_t)ksteps * (split + 1) / g.splits);
        if (kidx) {
            const int c0 = g.kstep_ptr[tile_n], c1 = g.kstep_ptr[tile_n + 1];
            s_begin = first_at_least(kidx, c0, c1, s_begin);
            s_end = first_at_least(kidx, c0, c1, s_end);
        }
    }
#define KS(pos) (kidx ? kidx[(pos)] : (pos))

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // A loader: 256 rows x 64 bytes per half, 2 row passes of 128 rows
    const int arow = tid >> 2, acol = (tid & 3) * 8;
    // Per-workgroup (scalar) base addresses plus 32-bit per-thread byte offsets: the
    // loads use scalar-base addressing and the offsets take one VGPR each.  A tile
    // spans at most 256 rows (or 128 columns) of a matrix whose leading dimension is
    // below 2^20 + 64 elements, so every offset stays below 2^31.
    const char* a_h = (const char*)(g.Ah + (int64_t)m0 * g.lda);
    const char* a_l = H == 2 ? (const char*)(g.Al + (int64_t)m0 * g.lda) : a_h;
    uint32_t oa[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        int ra = m0 + arow + 128 * i;
        ra = ra < g.M ? ra : g.M - 1;
        oa[i] = (uint32_t)(((int64_t)(ra - m0) * g.lda + acol) * 2);
    }
    // B producer: columns bc + 64 q (q = 0, 1), rows br .. br + 3 of the step
    const int bc = tid >> 3, br = (tid & 7) * 4;
    const char* b_om = (const char*)(px.om + (int64_t)n0 * px.ld);
    const char* b_g = (const char*)(px.g + (int64_t)n0 * px.ld);
    char* b_on = (char*)(px.om_new + (int64_t)n0 * px.ld);
    int jcol[2];  // p < 2^20 + 64
    bool jvalid[2];
    uint32_t ob[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        // columns past p are the zero padding columns (Omega, G and Omega+ hold
        // tilesN * 128 columns)
        const int j = n0 + bc + 64 * q;
        jvalid[q] = j < px.p;
        jcol[q] = j;
        ob[q] = (uint32_t)(((int64_t)(j - n0) * px.ld + br) * 4);
    }
    // X rows and the Omega / G columns (the HBM stream) are staged two steps ahead in
    // two register sets, so each load has a whole step (MFMAs + prox) to arrive
    u4 va0[H * 2], va1[H * 2];
    f4 vo0[2], vg0[2], vo1[2], vg1[2];
    f4 onw[2];
    f16v acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    ProxAcc pacc;

    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int r32 = lane & 31, k8 = (lane >> 5) * 8;

#define FUSED_LOAD_A(VA, step)                                                            \
    do {                                                                                  \
        const uint32_t ko_ = (uint32_t)(step) * (BK * 2);                                 \
        _Pragma("unroll") for (int q = 0; q < H * 2; ++q)                                 \
            VA[q] = *(const u4*)(((q >> 1) ? a_l : a_h) + (oa[q & 1] + ko_));             \
    } while (0)

#define FUSED_LOAD_OG(VO, VG, step)                                                       \
    do {                                                                                  \
        const uint32_t ko_ = (uint32_t)(step) * (BK * 4);                                 \
        _Pragma("unroll") for (int q = 0; q < 2; ++q) {                                   \
            VO[q] = *(const f4*)(b_om + (ob[q] + ko_));                                   \
            VG[q] = *(const f4*)(b_g + (ob[q] + ko_));                                    \
        }                                                                                 \
    } while (0)

#define FUSED_MMA(buf)                                                                    \
    do {                                                                                  \
        _Pragma("unroll") for (int kk = 0; kk < BK; kk += 16) {                           \
            bf8 ah[2], bh[2];                                                             \
            _Pragma("unroll") for (int i = 0; i < 2; ++i)                                 \
                ah[i] = *(const bf8*)&sA[(buf)][0][(wm + 32 * i + r32) * LDK + kk + k8];  \
            _Pragma("unroll") for (int j = 0; j < 2; ++j)                                 \
                bh[j] = *(const bf8*)&sB[(buf)][0][(wn + 32 * j + r32) * LDK + kk + k8];  \
            _Pragma("unroll") for (int i = 0; i < 2; ++i)                                 \
                _Pragma("unroll") for (int j = 0; j < 2; ++j)                             \
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j],     \
                                                                        acc[i][j], 0, 0, 0); \
            if (PASSES == 3) {                                                            \
                bf8 al[2], bl[2];                                                         \
                _Pragma("unroll") for (int j = 0; j < 2; ++j)                             \
                    bl[j] = *(const bf8*)&sB[(buf)][H - 1][(wn + 32 * j + r32) * LDK + kk + k8]; \
                _Pragma("unroll") for (int i = 0; i < 2; ++i)                             \
                    al[i] = *(const bf8*)&sA[(buf)][H - 1][(wm + 32 * i + r32) * LDK + kk + k8]; \
                /* one pass at a time: dependent MFMAs on an accumulator stay four  */    \
                /* instructions apart                                                */    \
                _Pragma("unroll") for (int i = 0; i < 2; ++i)                             \
                    _Pragma("unroll") for (int j = 0; j < 2; ++j)                         \
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(              \
                            ah[i], bl[j], acc[i][j], 0, 0, 0);                            \
                _Pragma("unroll") for (int i = 0; i < 2; ++i)                             \
                    _Pragma("unroll") for (int j = 0; j < 2; ++j)                         \
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(              \
                            al[i], bh[j], acc[i][j], 0, 0, 0);                            \
            }                                                                             \
        }                                                                                 \
    } while (0)

    if (s_begin < s_end) {
        const int last = s_end - 1;
        // Loads past the range re-read the last step (unconditional prefetch, see
        // gemm_f32_tile).  The producer always runs (no branch between it and the
        // MFMAs); past the range it fills the idle stage and neither counts nor stores.
        FUSED_LOAD_A(va0, KS(s_begin));
        FUSED_LOAD_OG(vo0, vg0, KS(s_begin));
        FUSED_LOAD_A(va1, KS(s_begin + 1 < last ? s_begin + 1 : last));
        FUSED_LOAD_OG(vo1, vg1, KS(s_begin + 1 < last ? s_begin + 1 : last));
        FUSED_PRODUCE(0, s_begin, vo0, vg0, va0, true);
        FUSED_DIAG(0, KS(s_begin), vo0, vg0, true);
        FUSED_STORE(KS(s_begin), true);
        __syncthreads();
        int cur = 0;
        for (int s = s_begin; s < s_end; s += 2) {
            // step s is in LDS[cur]; set 1 holds step s + 1
            const int s1 = s + 1 < last ? s + 1 : last;
            const bool live1 = s + 1 < s_end;
            FUSED_LOAD_A(va0, KS(s + 2 < last ? s + 2 : last));
            FUSED_LOAD_OG(vo0, vg0, KS(s + 2 < last ? s + 2 : last));
            FUSED_MMA(cur);
            FUSED_PRODUCE(cur ^ 1, s1, vo1, vg1, va1, live1);
            FUSED_DIAG(cur ^ 1, KS(s1), vo1, vg1, live1);
            FUSED_STORE(KS(s1), live1);
            __syncthreads();
            cur ^= 1;
            if (!live1) break;
            // step s + 1 is in LDS[cur]; set 0 holds step s + 2
            const int s2 = s + 2 < last ? s + 2 : last;
            const bool live2 = s + 2 < s_end;
            FUSED_LOAD_A(va1, KS(s + 3 < last ? s + 3 : last));
            FUSED_LOAD_OG(vo1, vg1, KS(s + 3 < last ? s + 3 : last));
            FUSED_MMA(cur);
            FUSED_PRODUCE(cur ^ 1, s2, vo0, vg0, va0, live2);
            FUSED_DIAG(cur ^ 1, KS(s2), vo0, vg0, live2);
            FUSED_STORE(KS(s2), live2);
            __syncthreads();
            cur ^= 1;
        }
    }
#undef FUSED_LOAD_A
#undef FUSED_LOAD_OG
#undef FUSED_MMA
#undef KS
    __syncthreads();

    const int tile = tile_m + tile_n * g.tilesM;
    double* red = (double*)&sA[0][0][0];  // LDS is free after the K loop
    if (sums_owner) {
        double v[6] = {pacc.d2, pacc.dg, pacc.l1, pacc.logd, pacc.nnz, pacc.fro};
        block_sum_in<6, kWThreads / 64>(v, red);
        if (tid == 0) fused_sums_out(g, px, tile_n, split, v);
    }
    if (EPI == EPI_PARTIAL) {
        f4* P = (f4*)(g.P + fused_partial_tile(g, ncnt, tile_m, tile_n, split) * (kFBM * kFBN));
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    st_stream(f4{acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2],
                                 acc[i][j][4 * q + 3]},
                              &P[((i * 2 + j) * 4 + q) * kWThreads + tid]);
        return;
    }
    const int mw = m0 + wm + 4 * (lane >> 5), nw = n0 + wn + (lane & 31);
    double nv[2] = {0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                store_frag<EPI_TRIAL>(g,
                                      f4{acc[i][j][4 * q], acc[i][j][4 * q + 1],
                                         acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]},
                                      mw + 32 * i + 8 * q, nw + 32 * j, nv);
    block_sum_in<2, kWThreads / 64>(nv, red);
    if (tid == 0) {
        g.norm_part[(int64_t)tile * kNormCols + 0] = nv[0];
        g.norm_part[(int64_t)tile * kNormCols + 1] = nv[1];
        if (g.zero_part1) {
            const int64_t row = (int64_t)g.tilesM * g.tilesN + tile;
            g.norm_part[row * kNormCols + 0] = 0.0;
            g.norm_part[row * kNormCols + 1] = 0.0;
        }
    }
}

// Split-K reduction for the fused tiles; kFReduceParts (2) workgroups per tile, part
// p owning the rows 64 c + 32 p .. + 31 (c = 0..3) of the tile, norm row =
// part * tiles + tile.  S > 0: the split count at compile time, so that a thread's
// loads of one split are issued together (S = 0 takes it from g.splits).  Like the
// trial launch it follows, it covers the M tiles m_first .. m_first + m_count - 1 and the
// column blocks n_first .. n_first + n_count - 1 (all with a count of 0), and pred 3
// skips it after a probe rejected the trial.
// The partial fragments are summed in the GEMM's thread -> fragment map (coalesced
// reads, each sum over s = 0, 1, ... in order), then turned through LDS so that the
// epilogue (store_frag) walks W column by column: 8 lanes cover 32 consecutive samples
// of a column, so W, W+ and its bf16 split move in whole 128-byte lines.
template <int S>
__global__ void __launch_bounds__(kWThreads) k_splitk_reduce_f(GemmArgs g) {
    static_assert(kFReduceParts == 2, "part p owns fragment row block i = p");
    if (g.ls) {
        if (g.pred >= 1 && g.ls->converged) return;
        if (g.pred >= 2 && g.ls->done) return;
        if (g.pred >= 3 && g.ls->probe_rej) return;
        if (g.probe_mode == 1 && g.ls->probe_off) return;
        if (g.probe_mode == 2 && !g.ls->probe_off) return;
    }
    constexpr int LDR = 132;  // LDS floats per column (128 rows + 4: 16 lanes hit 64 banks)
    __shared__ __attribute__((aligned(16))) float sT[kFBN * LDR];
    const int tiles = g.tilesM * g.tilesN;
    const int mcnt = g.m_count > 0 ? g.m_count : g.tilesM;
    const int ncnt = g.n_count > 0 ? g.n_count : g.tilesN;
    const int in_launch = mcnt * ncnt;
    const int local = blockIdx.x % in_launch, part = blockIdx.x / in_launch;
    const int tile_m = g.m_first + local % mcnt, tile_n = g.n_first + local / mcnt;
    const int tile = tile_m + tile_n * g.tilesM;
    // partial tiles of split s: s * in_split + ptile (fused_partial_tile's numbering)
    const int64_t in_split = (int64_t)g.tilesM * ncnt;
    const int64_t ptile = (int64_t)(tile_n - g.n_first) * g.tilesM + tile_m;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int PER = 16 / kFReduceParts;
    f4 v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) v[u] = f4{0.f, 0.f, 0.f, 0.f};
    if (S > 0) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const f4* P = (const f4*)(g.P + (s * in_split + ptile) * (kFBM * kFBN));
#pragma unroll
            for (int u = 0; u < PER; ++u) v[u] += ld_stream(&P[(part * PER + u) * kWThreads + tid]);
        }
    } else {
        for (int s = 0; s < g.splits; ++s) {
            const f4* P = (const f4*)(g.P + (s * in_split + ptile) * (kFBM * kFBN));
#pragma unroll
            for (int u = 0; u < PER; ++u) v[u] += ld_stream(&P[(part * PER + u) * kWThreads + tid]);
        }
    }
    // fragment (i = part, j, q) of this thread: rows 32 part + 8 q + 4 (lane / 32) .. + 3 of
    // the wave's 64-row block, column (wave & 1) 64 + lane % 32 + 32 j
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int j = (u >> 2) & 1, q = u & 3;
        const int rl = (wave >> 1) * 32 + 8 * q + 4 * (lane >> 5);
        const int cl = (wave & 1) * 64 + (lane & 31) + 32 * j;
        *(f4*)&sT[cl * LDR + rl] = v[u];
    }
    __syncthreads();
    double nv[2] = {0.0, 0.0};
    constexpr int ITEMS = kFBN * 32 / kWThreads;  // f4 per thread: 128 columns x 32 quads
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int e = tid + kWThreads * k;
        const int cl = e >> 5, rl = (e & 31) * 4;
        const int m = tile_m * kFBM + (rl >> 5) * 64 + 32 * part + (rl & 31);
        const int n = tile_n * kFBN + cl;
        store_frag<EPI_TRIAL>(g, *(const f4*)&sT[cl * LDR + rl], m, n, nv);
    }
    block_sum<2, kWThreads / 64>(nv);
    if (tid == 0) {
        const int64_t row = (int64_t)part * tiles + tile;
        g.norm_part[row * kNormCols + 0] = nv[0];
        g.norm_part[row * kNormCols + 1] = nv[1];
    }
}

void launch_splitk_reduce_f(const GemmArgs& a, hipStream_t st) {
    const int mcnt = a.m_count > 0 ? a.m_count : a.tilesM;
    const int ncnt = a.n_count > 0 ? a.n_count : a.tilesN;
    const unsigned blocks = (unsigned)(mcnt * ncnt * kFReduceParts);
    switch (a.splits) {
        case 2: k_splitk_reduce_f<2><<<blocks, kWThreads, 0, st>>>(a); break;
        case 3: k_splitk_reduce_f<3><<<blocks, kWThreads, 0, st>>>(a); break;
        case 4: k_splitk_reduce_f<4><<<blocks, kWThreads, 0, st>>>(a); break;
        default: k_splitk_reduce_f<0><<<blocks, kWThreads, 0, st>>>(a); break;
    }
}

void launch_trial_fused(const GemmArgs& a, const ProxArgs& px, int prec, hipStream_t st) {
    if (a.splits == 1 && a.tail_splits > 1 && a.tail_n0 > 0 && a.tail_n0 < a.tilesN) {
        // the column blocks before tail_n0 unsplit, then the tail split along K (and its
        // reduce); each column block keeps its split count in every launch of the product
        GemmArgs f = a, t = a;
        f.tail_splits = t.tail_splits = 0;
        f.n_first = 0;
        f.n_count = a.tail_n0;
        f.part_stride = a.tail_splits;
        f.zero_part1 = 1;
        t.n_first = a.tail_n0;
        t.n_count = a.tilesN - a.tail_n0;
        t.splits = a.tail_splits;
        t.part_stride = a.tail_splits;
        t.zero_part1 = 0;
        launch_trial_fused(f, px, prec, st);
        launch_trial_fused(t, px, prec, st);
        return;
    }
    if (prec == PREC_FP8) {
        launch_trial_fused8(a, px, st);
        return;
    }
    const int mcnt = a.m_count > 0 ? a.m_count : a.tilesM;
    const int ncnt = a.n_count > 0 ? a.n_count : a.tilesN;
    const unsigned blocks = (unsigned)((int64_t)mcnt * ncnt * a.splits);
    const bool list = a.kstep_idx != nullptr;
    const bool x3 = prec == PREC_BF16X3;
    if (a.splits > 1) {
        if (list && x3) k_trial_fused<3, EPI_PARTIAL, true><<<blocks, kWThreads, 0, st>>>(a, px);
        else if (list) k_trial_fused<1, EPI_PARTIAL, true><<<blocks, kWThreads, 0, st>>>(a, px);
        else if (x3) k_trial_fused<3, EPI_PARTIAL, false><<<blocks, kWThreads, 0, st>>>(a, px);
        else k_trial_fused<1, EPI_PARTIAL, false><<<blocks, kWThreads, 0, st>>>(a, px);
        launch_splitk_reduce_f(a, st);
    } else {
        if (list && x3) k_trial_fused<3, EPI_TRIAL, true><<<blocks, kWThreads, 0, st>>>(a, px);
        else if (list) k_trial_fused<1, EPI_TRIAL, true><<<blocks, kWThreads, 0, st>>>(a, px);
        else if (x3) k_trial_fused<3, EPI_TRIAL, false><<<blocks, kWThreads, 0, st>>>(a, px);
        else k_trial_fused<1, EPI_TRIAL, false><<<blocks, kWThreads, 0, st>>>(a, px);
    }
}

// ---------------------------------------------------------------------------
// FP8 form: OCP MX operands (E4M3 elements, one E8M0 power-of-two scale per 32
// consecutive values along the contraction index) on the gfx950 scaled MFMA
// v_mfma_scale_f32_32x32x64_f8f6f4, FP32 accumulation.
//
// Block scale: 2^s with s = floor(log2(block max)) - 7, so the block maximum maps
// into [128, 256) and no element needs clamping; s >= -126; an all-zero block
// takes s = 0.  Elements are rounded to nearest, ties to even (v_cvt_pk_fp8_f32),
// after multiplying by 2^-s (exact).  The conversion turns magnitudes >= 480 into
// NaN, so the scaled values are clamped to +-448 first (a no-op for finite input
// under this scale rule).
//
// 32x32x64 operand layout (A rows / B columns alike): lane l supplies row l % 32;
// with g = l / 32 its bytes 0..15 are K = 16 g .. 16 g + 15 and bytes 16..31 are
// K = 32 + 16 g .. 32 + 16 g + 15.  Lane l's scale byte (op_sel 0) applies to
// MX block g of its row: K 0..31 for g = 0, K 32..63 for g = 1.  The accumulator
// layout is that of the bf16 32x32 instructions.
// ---------------------------------------------------------------------------
typedef int i8v __attribute__((ext_vector_type(8)));

__device__ inline uint32_t mx_scale_byte(float amax) {
    if (!(amax > 0.f)) return 127u;                      // zero block: 2^0
    const int e = (int)(__float_as_uint(amax) >> 23);    // biased exponent (sign is 0)
    const int b = e - 7;
    return (uint32_t)(b < 1 ? 1 : b);
}

__device__ inline float mx_inv_scale(uint32_t sb) { return __uint_as_float((254u - sb) << 23); }
__device__ inline float mx_scale(uint32_t sb) { return __uint_as_float(sb << 23); }

__device__ inline float clamp448(float v) { return fminf(fmaxf(v, -448.f), 448.f); }

// four values -> four E4M3 bytes (value u in byte u)
__device__ inline uint32_t mx_pack4(f4 v, float inv) {
    uint32_t w = __builtin_amdgcn_cvt_pk_fp8_f32(clamp448(v[0] * inv), clamp448(v[1] * inv), 0,
                                                 false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(clamp448(v[2] * inv), clamp448(v[3] * inv), w, true);
}

__device__ inline f4 mx_unpack4(uint32_t w, float sc) {
    return f4{__builtin_amdgcn_cvt_f32_fp8((int)w, 0) * sc, __builtin_amdgcn_cvt_f32_fp8((int)w, 1) * sc,
              __builtin_amdgcn_cvt_f32_fp8((int)w, 2) * sc, __builtin_amdgcn_cvt_f32_fp8((int)w, 3) * sc};
}

__device__ inline float fmax4(f4 v) {
    return fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
}

// X (n x p row-major) -> MX copies of both GEMM operands:
//   x8  (n_pad x p_pad, blocks of 32 features per row: the A operand of X Delta)
//   xt8 (p_pad x n_pad, blocks of 32 samples per feature: the A operand of X^T W)
// with scale bytes x8s [n_pad][p_pad/32] and xt8s [p_pad][n_pad/32].  One 32 x 32
// tile of X per workgroup; padding is zero.
__global__ void __launch_bounds__(kThreads) k_quant_x8(const float* __restrict__ X, int64_t n,
                                                       int64_t p, int64_t p_pad, int64_t n_pad,
                                                       XQuant q) {
    __shared__ float t[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int rr = ty; rr < 32; rr += kThreads / 32) {
        const int64_t r = r0 + rr, c = c0 + tx;
        t[rr][tx] = (r < n && c < p) ? X[r * p + c] : 0.f;
    }
    __syncthreads();
    const int line = threadIdx.x >> 3, part = threadIdx.x & 7;  // 8 lanes per block
    {   // row `line` of the tile: features c0 .. c0+31 of sample r0 + line
        f4 v;
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = t[line][4 * part + u];
        float m = fmax4(v);
        m = fmaxf(m, __shfl_xor(m, 1, 64));
        m = fmaxf(m, __shfl_xor(m, 2, 64));
        m = fmaxf(m, __shfl_xor(m, 4, 64));
        const uint32_t sb = mx_scale_byte(m);
        *(uint32_t*)(q.x8 + (r0 + line) * p_pad + c0 + 4 * part) = mx_pack4(v, mx_inv_scale(sb));
        if (part == 0) q.x8s[(r0 + line) * (p_pad / 32) + blockIdx.x] = (uint8_t)sb;
    }
    {   // column `line` of the tile: samples r0 .. r0+31 of feature c0 + line
        f4 v;
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = t[4 * part + u][line];
        float m = fmax4(v);
        m = fmaxf(m, __shfl_xor(m, 1, 64));
        m = fmaxf(m, __shfl_xor(m, 2, 64));
        m = fmaxf(m, __shfl_xor(m, 4, 64));
        const uint32_t sb = mx_scale_byte(m);
        *(uint32_t*)(q.xt8 + (c0 + line) * n_pad + r0 + 4 * part) = mx_pack4(v, mx_inv_scale(sb));
        if (part == 0) q.xt8s[(c0 + line) * (n_pad / 32) + blockIdx.y] = (uint8_t)sb;
    }
}

void launch_quant_x8(const float* X, int64_t n, int64_t p, int64_t p_pad, int64_t n_pad,
                     XQuant q, hipStream_t st) {
    dim3 grid((unsigned)(p_pad / 32), (unsigned)(n_pad / 32));
    k_quant_x8<<<grid, kThreads, 0, st>>>(X, n, p, p_pad, n_pad, q);
}

// W^T (rows x n_pad FP32, row-major) -> MX (blocks of 32 samples per row): the B
// operand of the FP8 gradient.  Eight lanes per block, four values per lane.
// Skipped once the fit has stopped.
__global__ void __launch_bounds__(kThreads) k_quant_w8(const float* __restrict__ Wt, int64_t total,
                                                       uint8_t* __restrict__ w8,
                                                       uint8_t* __restrict__ w8s,
                                                       const LsState* ls) {
    if (ls && ls->converged) return;
    const int64_t n4 = total >> 2;  // total is a multiple of 32: blocks never straddle
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < n4;
         base += (int64_t)gridDim.x * kThreads) {
        const int64_t i4 = base + threadIdx.x;
        const bool ok = i4 < n4;    // uniform over each aligned group of 8 lanes
        const f4 v = ok ? ((const f4*)Wt)[i4] : f4{0.f, 0.f, 0.f, 0.f};
        float m = fmax4(v);
        m = fmaxf(m, __shfl_xor(m, 1, 64));
        m = fmaxf(m, __shfl_xor(m, 2, 64));
        m = fmaxf(m, __shfl_xor(m, 4, 64));
        const uint32_t sb = mx_scale_byte(m);
        if (ok) {
            ((uint32_t*)w8)[i4] = mx_pack4(v, mx_inv_scale(sb));
            if ((threadIdx.x & 7) == 0) w8s[i4 >> 3] = (uint8_t)sb;
        }
    }
}

void launch_quant_w8(const float* Wt, int64_t total, uint8_t* w8, uint8_t* w8s, const LsState* ls,
                     hipStream_t st) {
    const int64_t n4 = total >> 2;
    int64_t blocks = cdiv(n4, (int64_t)kThreads);
    if (blocks > 8192) blocks = 8192;
    k_quant_w8<<<(unsigned)blocks, kThreads, 0, st>>>(Wt, total, w8, w8s, ls);
}

// operand fragment of the 32x32x64 instruction from an LDS row of 64 bytes
__device__ inline i8v frag8(const uint8_t* row, int g) {
    const u4 lo = *(const u4*)(row + 16 * g);
    const u4 hi = *(const u4*)(row + 32 + 16 * g);
    return i8v{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
               (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
}

// FP8 gradient GEMM G = X^T W / n: 256 x 256 tile, 8 waves (2 along M x 4 along N),
// each 128 x 64 = 4 x 2 blocks of the 32x32x64 instruction; one 64-deep K step
// (two MX blocks) per LDS stage, double-buffered; same tile order and epilogue as
// the bf16 gradient.
constexpr int kLDK8 = 64 + 16;  // bytes per LDS row (16-byte pad: conflict-free reads)

template <int EPI>
__global__ void __launch_bounds__(kWThreads, 1) k_gemm_fp8w(GemmArgs g) {
    if (gemm_skip(g)) return;
    __shared__ __attribute__((aligned(16))) uint8_t sA[2][kWBM * kLDK8];
    __shared__ __attribute__((aligned(16))) uint8_t sB[2][kWBN * kLDK8];
    __shared__ __attribute__((aligned(16))) uint8_t sAs[2][kWBM * 2];
    __shared__ __attribute__((aligned(16))) uint8_t sBs[2][kWBN * 2];

    int tile_m, tile_n, split;
    decode_tile(g, tile_m, tile_n, split);
    if (g.tile_occ && !g.tile_occ[tile_m + tile_n * g.tilesM]) return;  // a zero tile of C
    const int m0 = tile_m * kWBM, n0 = tile_n * kWBN;
    const int ksteps = g.K / 64;
    const int s_begin = (int)((int64_t)ksteps * split / g.splits);
    const int s_end = (int)((int64_t)ksteps * (split + 1) / g.splits);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // data loader: row tid / 2, bytes 32 (tid & 1) .. +31 of the step
    const int lrow = tid >> 1, lcol = (tid & 1) * 32;
    int ra = m0 + lrow;
    ra = ra < g.M ? ra : g.M - 1;
    int rb = n0 + lrow;
    rb = rb < g.N ? rb : g.N - 1;
    const uint8_t* pa = g.A8 + (int64_t)ra * g.lda + lcol;
    const uint8_t* pb = g.B8 + (int64_t)rb * g.ldb + lcol;
    // scale loader: threads 0..255 take A rows, 256..511 B rows (2 bytes per step)
    const int srow = tid & 255;
    const bool sa_side = tid < 256;
    int rs = (sa_side ? m0 : n0) + srow;
    const int rlim = sa_side ? g.M : g.N;
    rs = rs < rlim ? rs : rlim - 1;
    const uint8_t* ps = sa_side ? g.As + (int64_t)rs * g.ldas : g.Bs + (int64_t)rs * g.ldbs;
    uint8_t* sdst0 = sa_side ? &sAs[0][srow * 2] : &sBs[0][srow * 2];
    uint8_t* sdst1 = sa_side ? &sAs[1][srow * 2] : &sBs[1][srow * 2];

    u4 va[2], vb[2];
    uint16_t vs;
    f16v acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int wm = (wave >> 2) * 128, wn = (wave & 3) * 64;
    const int r32 = lane & 31, gk = lane >> 5;

    if (s_begin < s_end) {
        {
            const int64_t ko = (int64_t)s_begin * 64;
            va[0] = *(const u4*)(pa + ko);
            va[1] = *(const u4*)(pa + ko + 16);
            vb[0] = *(const u4*)(pb + ko);
            vb[1] = *(const u4*)(pb + ko + 16);
            vs = *(const uint16_t*)(ps + 2 * (int64_t)s_begin);
        }
        *(u4*)&sA[0][lrow * kLDK8 + lcol] = va[0];
        *(u4*)&sA[0][lrow * kLDK8 + lcol + 16] = va[1];
        *(u4*)&sB[0][lrow * kLDK8 + lcol] = vb[0];
        *(u4*)&sB[0][lrow * kLDK8 + lcol + 16] = vb[1];
        *(uint16_t*)sdst0 = vs;
        __syncthreads();
        int cur = 0;
        for (int s = s_begin; s < s_end; ++s) {
            {   // unconditional prefetch (see gemm_f32_tile)
                const int sn = s + 1 < s_end ? s + 1 : s;
                const int64_t ko = (int64_t)sn * 64;
                va[0] = *(const u4*)(pa + ko);
                va[1] = *(const u4*)(pa + ko + 16);
                vb[0] = *(const u4*)(pb + ko);
                vb[1] = *(const u4*)(pb + ko + 16);
                vs = *(const uint16_t*)(ps + 2 * (int64_t)sn);
            }
            __builtin_amdgcn_sched_barrier(0);
            i8v af[4], bf[2];
            int sa[4], sbv[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = wm + 32 * i + r32;
                af[i] = frag8(&sA[cur][row * kLDK8], gk);
                sa[i] = sAs[cur][row * 2 + gk];
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int row = wn + 32 * j + r32;
                bf[j] = frag8(&sB[cur][row * kLDK8], gk);
                sbv[j] = sBs[cur][row * 2 + gk];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        af[i], bf[j], acc[i][j], 0, 0, 0, sa[i], 0, sbv[j]);
            __builtin_amdgcn_sched_barrier(0);
            *(u4*)&sA[cur ^ 1][lrow * kLDK8 + lcol] = va[0];
            *(u4*)&sA[cur ^ 1][lrow * kLDK8 + lcol + 16] = va[1];
            *(u4*)&sB[cur ^ 1][lrow * kLDK8 + lcol] = vb[0];
            *(u4*)&sB[cur ^ 1][lrow * kLDK8 + lcol + 16] = vb[1];
            *(uint16_t*)(cur ? sdst0 : sdst1) = vs;
            __syncthreads();
            cur ^= 1;
        }
    }
    __syncthreads();

    static_assert(EPI == EPI_GRAD, "the FP8 GEMM computes the gradient only");
    __shared__ __attribute__((aligned(16))) float sT[kEpiFloats];
    double nv[2] = {0.0, 0.0};
    grad_epilogue_cols<EPI>(g, acc, sT, m0 + wm, n0 + wn, nv);
}

// Fused prox + trial product of the FP8 form.  Same structure as k_trial_fused
// (256 x 128 tile, 8 waves of 64 x 64, tile_m fastest, the tile_m == 0 workgroup
// owns its column block), with a 64-deep K step: each thread produces rows
// br .. br + 7 of columns bc and bc + 64, the four lanes covering one 32-row MX
// block agree on its scale through lane shuffles, and Delta reaches LDS as E4M3
// bytes plus scale bytes.  The line-search sums take Delta as represented.
#define FUSED_PRODUCE8(buf, step)                                                         \
    do {                                                                                  \
        const int64_t k0_ = (int64_t)(step) * 64;                                         \
        *(u4*)&sA8[(buf)][arow * kLDK8 + acol] = va[0];                                   \
        *(u4*)&sA8[(buf)][arow * kLDK8 + acol + 16] = va[1];                              \
        if (tid < kFBM) *(uint16_t*)&sAs8[(buf)][tid * 2] = vsa;                          \
        _Pragma("unroll") for (int q = 0; q < 2; ++q) {                                   \
            f4 nw_[2];                                                                    \
            _Pragma("unroll") for (int h = 0; h < 2; ++h) {                               \
                const f4 o_ = vo[q][h], g_ = vg[q][h];                                    \
                _Pragma("unroll") for (int u = 0; u < 4; ++u) {                           \
                    const float a_ = fmaf(-tau_f, g_[u], o_[u]);                          \
                    const float t_ = fabsf(a_) - thr_f;                                   \
                    nw_[h][u] = t_ > 0.f ? copysignf(t_, a_) : 0.f;                       \
                }                                                                         \
            }                                                                             \
            const int64_t dpos_ = jcol[q] - (k0_ + br);                                   \
            const bool has_diag_ = dpos_ >= 0 && dpos_ < 8;                               \
            float dval_ = 0.f;                                                            \
            if (has_diag_) {                                                              \
                const int du_ = (int)dpos_;                                               \
                const f4 od4_ = du_ < 4 ? vo[q][0] : vo[q][1];                            \
                const f4 gd4_ = du_ < 4 ? vg[q][0] : vg[q][1];                            \
                const int uu_ = du_ & 3;                                                  \
                const float od_ = uu_ == 0 ? od4_[0] : uu_ == 1 ? od4_[1] : uu_ == 2 ? od4_[2] : od4_[3]; \
                const float gd_ = uu_ == 0 ? gd4_[0] : uu_ == 1 ? gd4_[1] : uu_ == 2 ? gd4_[2] : gd4_[3]; \
                dval_ = prox_one(od_, gd_, true, tau, lam, tau_f, thr_f);                 \
                _Pragma("unroll") for (int h = 0; h < 2; ++h)                             \
                    _Pragma("unroll") for (int u = 0; u < 4; ++u)                         \
                        nw_[h][u] = (4 * h + u == du_) ? dval_ : nw_[h][u];               \
            }                                                                             \
            f4 d_[2];                                                                     \
            _Pragma("unroll") for (int h = 0; h < 2; ++h) d_[h] = nw_[h] - vo[q][h];      \
            if (!jvalid[q]) d_[0] = d_[1] = f4{0.f, 0.f, 0.f, 0.f};                       \
            float m_ = fmaxf(fmax4(d_[0]), fmax4(d_[1]));                                 \
            m_ = fmaxf(m_, __shfl_xor(m_, 1, 64));                                        \
            m_ = fmaxf(m_, __shfl_xor(m_, 2, 64));                                        \
            const uint32_t sb_ = mx_scale_byte(m_);                                       \
            const float inv_ = mx_inv_scale(sb_), sc_ = mx_scale(sb_);                    \
            const uint32_t w0_ = mx_pack4(d_[0], inv_), w1_ = mx_pack4(d_[1], inv_);      \
            const int col_ = bc + 64 * q;                                                 \
            *(uint2*)&sB8[(buf)][col_ * kLDK8 + br] = make_uint2(w0_, w1_);               \
            if ((tid & 3) == 0) sBs8[(buf)][col_ * 2 + ((tid >> 2) & 1)] = (uint8_t)sb_;  \
            if (owner && jvalid[q]) {                                                     \
                if (store_owner) {                                                        \
                    st_stream(nw_[0], (f4*)(pn[q] + k0_));                                \
                    st_stream(nw_[1], (f4*)(pn[q] + k0_ + 4));                            \
                }                                                                         \
                float sd2_ = 0.f, sdg_ = 0.f, sl1_ = 0.f, sfr_ = 0.f;                     \
                int nz_ = 0;                                                              \
                _Pragma("unroll") for (int h = 0; h < 2; ++h) {                           \
                    const f4 dq_ = mx_unpack4(h ? w1_ : w0_, sc_);                        \
                    _Pragma("unroll") for (int u = 0; u < 4; ++u) {                       \
                        const float dv_ = dq_[u];                                         \
                        sd2_ = fmaf(dv_, dv_, sd2_);                                      \
                        sdg_ = fmaf(dv_, vg[q][h][u], sdg_);                              \
                        sl1_ += fabsf(nw_[h][u]);                                         \
                        sfr_ = fmaf(nw_[h][u], nw_[h][u], sfr_);                          \
                        nz_ += (nw_[h][u] != 0.f && !(has_diag_ && 4 * h + u == (int)dpos_)) ? 1 : 0; \
                    }                                                                     \
                }                                                                         \
                pacc.d2 += (double)sd2_;                                                  \
                pacc.dg += (double)sdg_;                                                  \
                pacc.l1 += (double)sl1_;                                                  \
                pacc.fro += (double)sfr_;                                                 \
                pacc.nnz += (double)nz_;                                                  \
                if (has_diag_) pacc.logd += dval_ > 0.f ? log((double)dval_) : -INFINITY; \
            }                                                                             \
        }                                                                                 \
    } while (0)

// LIST: K steps from a list, as in trial_fused32_tile.
template <int EPI, bool LIST>
__global__ void __launch_bounds__(kWThreads, 1) k_trial_fused8(GemmArgs g, ProxArgs px) {
    if (gemm_skip(g)) return;
    __shared__ __attribute__((aligned(16))) uint8_t sA8[2][kFBM * kLDK8];
    __shared__ __attribute__((aligned(16))) uint8_t sB8[2][kFBN * kLDK8];
    __shared__ __attribute__((aligned(16))) uint8_t sAs8[2][kFBM * 2];
    __shared__ __attribute__((aligned(16))) uint8_t sBs8[2][kFBN * 2];

    const double tau = px.ls->tau, lam = px.ls->lambda;
    const float tau_f = (float)tau, thr_f = (float)(tau * lam);

    const int nblk = gridDim.x, bid = blockIdx.x;
    const int xcd = bid & 7, local = bid >> 3, q8 = nblk >> 3, r8 = nblk & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + local;
    const int mcnt = g.m_count > 0 ? g.m_count : g.tilesM;
    const int ncnt = g.n_count > 0 ? g.n_count : g.tilesN;
    const int tile_m = g.m_first + logical % mcnt;
    const int tile_n = g.n_first + (logical / mcnt) % ncnt;
    const int split = logical / (mcnt * ncnt);
    const bool store_owner = tile_m == g.store_m;   // stores Omega+
    const bool sums_owner = tile_m == g.sums_m;     // writes the prox sums
    const bool owner = store_owner || sums_owner;   // computes them
    const int m0 = tile_m * kFBM, n0 = tile_n * kFBN;
    // positions over the column block's K steps of 64 (all, or its list: see k_trial_fused)
    const int32_t* kidx = LIST ? g.kstep_idx : nullptr;
    int s_begin, s_end;
    {
        const int ksteps = g.K / 64;
        s_begin = (int)((int64_t)ksteps * split / g.splits);
        s_end = (int)((int64_t)ksteps * (split + 1) / g.splits);
        if (kidx) {
            const int c0 = g.kstep_ptr[tile_n], c1 = g.kstep_ptr[tile_n + 1];
            s_begin = first_at_least(kidx, c0, c1, s_begin);
            s_end = first_at_least(kidx, c0, c1, s_end);
        }
    }

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // A loader: row tid / 2 of the tile, 32 bytes; scale bytes by threads 0..255
    const int arow = tid >> 1, acol = (tid & 1) * 32;
    int ra = m0 + arow;
    ra = ra < g.M ? ra : g.M - 1;
    const uint8_t* pa = g.A8 + (int64_t)ra * g.lda + acol;
    int rsa = m0 + (tid & (kFBM - 1));
    rsa = rsa < g.M ? rsa : g.M - 1;
    const uint8_t* psa = g.As + (int64_t)rsa * g.ldas;
    // B producer: columns bc + 64 q (q = 0, 1), rows br .. br + 7 of the step
    const int bc = tid >> 3, br = (tid & 7) * 8;
    int64_t jcol[2];
    bool jvalid[2];
    const float* po[2];
    const float* pg[2];
    float* pn[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int64_t j = (int64_t)n0 + bc + 64 * q;
        jvalid[q] = j < px.p;
        jcol[q] = j;
        const int64_t jc = jvalid[q] ? j : px.p - 1;
        po[q] = px.om + jc * px.ld + br;
        pg[q] = px.g + jc * px.ld + br;
        pn[q] = px.om_new + jc * px.ld + br;
    }
    u4 va[2];
    uint16_t vsa = 0;
    f4 vo[2][2], vg[2][2];
    f16v acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    ProxAcc pacc;

    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int r32 = lane & 31, gk = lane >> 5;

    if (s_begin < s_end) {
        {
            const int64_t sk = kidx ? kidx[s_begin] : s_begin;
            const int64_t ko = sk * 64;
            va[0] = *(const u4*)(pa + ko);
            va[1] = *(const u4*)(pa + ko + 16);
            vsa = *(const uint16_t*)(psa + 2 * sk);
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    vo[q][h] = *(const f4*)(po[q] + ko + 4 * h);
                    vg[q][h] = *(const f4*)(pg[q] + ko + 4 * h);
                }
        }
        FUSED_PRODUCE8(0, kidx ? kidx[s_begin] : s_begin);
        __syncthreads();
        int cur = 0;
        for (int s = s_begin; s < s_end; ++s) {
            const bool more = s + 1 < s_end;
            const int64_t sn = kidx ? kidx[more ? s + 1 : s] : (more ? s + 1 : s);
            {   // unconditional prefetch (see gemm_f32_tile)
                const int64_t ko = sn * 64;
                va[0] = *(const u4*)(pa + ko);
                va[1] = *(const u4*)(pa + ko + 16);
                vsa = *(const uint16_t*)(psa + 2 * sn);
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        vo[q][h] = *(const f4*)(po[q] + ko + 4 * h);
                        vg[q][h] = *(const f4*)(pg[q] + ko + 4 * h);
                    }
            }
            __builtin_amdgcn_sched_barrier(0);
            i8v af[2], bf[2];
            int sa[2], sbv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = wm + 32 * i + r32;
                af[i] = frag8(&sA8[cur][row * kLDK8], gk);
                sa[i] = sAs8[cur][row * 2 + gk];
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int row = wn + 32 * j + r32;
                bf[j] = frag8(&sB8[cur][row * kLDK8], gk);
                sbv[j] = sBs8[cur][row * 2 + gk];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        af[i], bf[j], acc[i][j], 0, 0, 0, sa[i], 0, sbv[j]);
            __builtin_amdgcn_sched_barrier(0);
            if (more) FUSED_PRODUCE8(cur ^ 1, sn);
            __syncthreads();
            cur ^= 1;
        }
    }
    __syncthreads();

    const int tile = tile_m + tile_n * g.tilesM;
    double* red = (double*)&sA8[0][0];  // LDS is free after the K loop
    if (sums_owner) {
        double v[6] = {pacc.d2, pacc.dg, pacc.l1, pacc.logd, pacc.nnz, pacc.fro};
        block_sum_in<6, kWThreads / 64>(v, red);
        if (tid == 0) fused_sums_out(g, px, tile_n, split, v);
    }
    if (EPI == EPI_PARTIAL) {
        f4* P = (f4*)(g.P + fused_partial_tile(g, ncnt, tile_m, tile_n, split) * (kFBM * kFBN));
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    st_stream(f4{acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2],
                                 acc[i][j][4 * q + 3]},
                              &P[((i * 2 + j) * 4 + q) * kWThreads + tid]);
        return;
    }
    const int mw = m0 + wm + 4 * (lane >> 5), nw = n0 + wn + (lane & 31);
    double nv[2] = {0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                store_frag<EPI_TRIAL>(g,
                                      f4{acc[i][j][4 * q], acc[i][j][4 * q + 1],
                                         acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]},
                                      mw + 32 * i + 8 * q, nw + 32 * j, nv);
    block_sum_in<2, kWThreads / 64>(nv, red);
    if (tid == 0) {
        g.norm_part[(int64_t)tile * kNormCols + 0] = nv[0];
        g.norm_part[(int64_t)tile * kNormCols + 1] = nv[1];
        if (g.zero_part1) {
            const int64_t row = (int64_t)g.tilesM * g.tilesN + tile;
            g.norm_part[row * kNormCols + 0] = 0.0;
            g.norm_part[row * kNormCols + 1] = 0.0;
        }
    }
}

void launch_grad_fp8(const GemmArgs& a, hipStream_t st) {
    const unsigned blocks = (unsigned)((int64_t)a.tilesM * a.tilesN * a.splits);
    k_gemm_fp8w<EPI_GRAD><<<blocks, kWThreads, 0, st>>>(a);
}

void launch_trial_fused8(const GemmArgs& a, const ProxArgs& px, hipStream_t st) {
    const int mcnt = a.m_count > 0 ? a.m_count : a.tilesM;
    const int ncnt = a.n_count > 0 ? a.n_count : a.tilesN;
    const unsigned blocks = (unsigned)((int64_t)mcnt * ncnt * a.splits);
    const bool list = a.kstep_idx != nullptr;
    if (a.splits > 1) {
        if (list) k_trial_fused8<EPI_PARTIAL, true><<<blocks, kWThreads, 0, st>>>(a, px);
        else k_trial_fused8<EPI_PARTIAL, false><<<blocks, kWThreads, 0, st>>>(a, px);
        launch_splitk_reduce_f(a, st);
    } else {
        if (list) k_trial_fused8<EPI_TRIAL, true><<<blocks, kWThreads, 0, st>>>(a, px);
        else k_trial_fused8<EPI_TRIAL, false><<<blocks, kWThreads, 0, st>>>(a, px);
    }
}

int prox_blocks(int64_t total) {
    const int64_t n4 = total >> 2;
    int64_t b = cdiv(n4 > 0 ? n4 : 1, (int64_t)kThreads * 4);
    if (b > kMaxProxBlocks) b = kMaxProxBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

void launch_prox(ProxArgs a, int nblocks, hipStream_t st) {
    const int64_t step = 4 * (int64_t)kThreads;
    a.step_col = step / a.ld;
    a.step_row = step - a.step_col * a.ld;
    if (a.dh && a.dl)
        k_prox<2><<<nblocks, kThreads, 0, st>>>(a);
    else if (a.dh)
        k_prox<1><<<nblocks, kThreads, 0, st>>>(a);
    else
        k_prox<0><<<nblocks, kThreads, 0, st>>>(a);
}

// ---------------------------------------------------------------------------
// Acceptance test of Alg. 1 (one workgroup, FP64, fixed summation order).
//
//   accept  <=>  ||X Delta||^2 / n <= ||Delta||^2 / tau   or   tau <= 1/L
//
// g is quadratic, so g(Omega + Delta) = g(Omega) + <G, Delta> + ||X Delta||^2/(2n)
// exactly and this is the printed inequality without subtracting values of g.
// On acceptance the iterate's objective pieces come from the same sums:
// g = ||W+||^2/(2n), h = -sum log Omega+_jj + lambda ||Omega+||_1.
// ---------------------------------------------------------------------------
// Posts the line-search state to the host mailbox (system scope; the trial count
// is released last, after the fields it vouches for).
__device__ inline void post_mailbox(Mailbox* mb, const LsState* ls) {
    if (!mb) return;
    // relaxed: the host acts on this word alone; everything it then enqueues on the
    // stream is ordered after this kernel anyway
    __hip_atomic_store(&mb->word, mailbox_word(ls->total_trials, ls->iter, ls->converged),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// probing: the fit probes its trials (see k_probe_decide).  Once a trial that no partial
// test rejected fails the full test, its ratio ||X Delta||^2 tau / (n ||Delta||^2) was
// below the inverse of the last partial test's share of the samples, and the next
// trial's, at half the step, is about half of it: a partial test could reject it only if
// the ratio did not fall, so the rest of the iteration runs each trial as one launch over
// all samples (the same tiles and sums, so the same bits, without the extra launches).
__device__ __forceinline__ void finalize_run(LsState* ls, const double* prox_part, int nprox,
                                             const double* norm_part, int ntiles, double* trace,
                                             int32_t* trials_log, Mailbox* mbox, int probing) {
    if (ls->done || ls->converged) return;
    // a trial its probe has rejected is complete: clear the flag for the next trial
    const int probe_rej = ls->probe_rej;
    __syncthreads();
    if (probe_rej) {
        if (threadIdx.x == 0) ls->probe_rej = 0;
        return;
    }
    double pv[6];
    sum_partials<6>(prox_part, nprox, kPartCols, pv);
    double nv[2];
    sum_partials<2>(norm_part, ntiles, kNormCols, nv);
    if (threadIdx.x != 0) return;
    const double d2 = pv[P_D2], l1 = pv[P_L1], logd = pv[P_LOGD], fro = pv[P_FRO];
    const double v2 = nv[0], w2 = nv[1];
    const double tau = ls->tau;
    const bool canonical = v2 * ls->inv_n <= d2 / tau;
    const bool at_floor = tau <= ls->inv_L;
    const bool finite = isfinite(d2) && isfinite(v2) && isfinite(w2) && isfinite(l1) &&
                        isfinite(logd) && isfinite(fro);
    ls->trials += 1;
    ls->total_trials += 1;
    if (probing && ls->probe_off) ls->unprobed += 1;
    if (!finite) {
        ls->bad |= 2;
        ls->converged = 1;  // stop: every later launch is skipped
        post_mailbox(mbox, ls);
        return;
    }
    if (canonical || at_floor || ls->fixed_step) {
        ls->done = 1;
        if (!canonical && !ls->fixed_step) ls->floor_accepts += 1;
        const int it = ls->iter;
        ls->iter = it + 1;
        ls->tau_acc = tau;
        ls->g_cur = 0.5 * w2 * ls->inv_n;
        ls->h_cur = -logd + ls->lambda * l1;
        ls->f_cur = ls->g_cur + ls->h_cur;
        ls->logd_cur = logd;
        ls->l1_cur = l1;
        ls->delta_fro = sqrt(d2);
        ls->nnz_off = (int64_t)pv[P_NNZ];
        if (trials_log) trials_log[it] = ls->trials;
        if (trace) {
            double* row = trace + (int64_t)(it + 1) * 8;
            row[0] = ls->f_cur;
            row[1] = ls->g_cur;
            row[2] = ls->h_cur;
            row[3] = tau;
            row[4] = (double)ls->trials;
            row[5] = ls->delta_fro;
            row[6] = (!canonical && !ls->fixed_step) ? 1.0 : 0.0;
            row[7] = pv[P_NNZ];
        }
        if (ls->tol > 0.0) {
            const double ref = sqrt(fro) > 1.0 ? sqrt(fro) : 1.0;
            if (sqrt(d2) <= ls->tol * ref) ls->converged = 1;
        }
        if (ls->iter >= ls->max_iter) ls->converged = 1;
    } else {
        ls->tau = tau * ls->beta;
        if (probing) ls->probe_off = 1;
    }
    post_mailbox(mbox, ls);
}

__global__ void __launch_bounds__(kThreads) k_finalize(LsState* ls, const double* prox_part,
                                                       int nprox, const double* norm_part,
                                                       int ntiles, double* trace,
                                                       int32_t* trials_log, Mailbox* mbox,
                                                       int probing) {
    finalize_run(ls, prox_part, nprox, norm_part, ntiles, trace, trials_log, mbox, probing);
}

void launch_finalize(LsState* ls, const double* prox_part, int nprox, const double* norm_part,
                     int ntiles, double* trace, int32_t* trials_log, Mailbox* mbox,
                     int probing, hipStream_t st) {
    k_finalize<<<1, kThreads, 0, st>>>(ls, prox_part, nprox, norm_part, ntiles, trace,
                                       trials_log, mbox, probing);
}

// Partial test of a probed trial after the fused trial kernel ran on its first mt M
// tiles (samples 0 .. 256 mt - 1; M tile 0 also wrote the prox sums over every column).
// Every term of ||X Delta||^2 is a square, so the sum over those samples is a lower bound
// of the whole: when it alone exceeds n ||Delta||^2 / tau, the trial fails Alg. 1's test
// exactly as the full product would.  It is then rejected here (counted, tau <- beta tau,
// posted to the mailbox) and flagged, so that the later M tiles, the unprobed launch and
// the acceptance test of this trial do nothing.  A trial at the floor tau <= 1/L, a fixed
// step and non-finite sums always go on to the full test.  A trial rejected this late
// (3 mt >= 2 tilesM: its ratio is only known to exceed tilesM / mt) leaves a next trial,
// at half the step, that most likely passes, so the iteration's later trials run
// unprobed, as after a failed full test.  Norm rows: part * tiles + tile_n * tilesM +
// tile_m, part < nparts (kFReduceParts after a split-K reduce, else 1).  Nothing runs once
// the iteration has stopped probing.
__global__ void __launch_bounds__(kThreads) k_probe_decide(LsState* ls, const double* prox_part,
                                                           int nprox, const double* norm_part,
                                                           int tilesN, int tilesM, int nparts,
                                                           int mt, Mailbox* mbox) {
    if (ls->done || ls->converged || ls->probe_off) return;  // (no probe ran)
    if (mt > 1 && ls->probe_rej) return;                      // rejected at an earlier test
    double pv[6];
    sum_partials<6>(prox_part, nprox, kPartCols, pv);
    double nv[1] = {0.0};
    const int64_t tiles = (int64_t)tilesM * tilesN;
    // norm rows of M tiles 0 .. mt - 1 of every column block, for each reduce part
    const int per = tilesN * mt;
    for (int r = threadIdx.x; r < per * nparts; r += kThreads) {
        const int part = r / per, q = r % per;
        nv[0] += norm_part[(part * tiles + (int64_t)(q / mt) * tilesM + q % mt) * kNormCols];
    }
    block_sum<1>(nv);
    if (threadIdx.x != 0) return;
    const double d2 = pv[P_D2], v2 = nv[0], tau = ls->tau;
    const bool reject = isfinite(d2) && isfinite(v2) && !(tau <= ls->inv_L) &&
                        !ls->fixed_step && v2 * ls->inv_n > d2 / tau;
    if (reject) {
        ls->trials += 1;
        ls->total_trials += 1;
        ls->tau = tau * ls->beta;
        ls->probe_rej = 1;
        ls->probe_rejects += 1;
        ls->probe_mtiles += mt;
        if (3 * mt >= 2 * tilesM) ls->probe_off = 1;
        post_mailbox(mbox, ls);
    } else if (mt == 1) {
        ls->probe_rej = 0;
    }
}

void launch_probe_decide(LsState* ls, const double* prox_part, int nprox,
                         const double* norm_part, int tilesN, int tilesM, int nparts, int mt,
                         Mailbox* mbox, hipStream_t st) {
    k_probe_decide<<<1, kThreads, 0, st>>>(ls, prox_part, nprox, norm_part, tilesN, tilesM,
                                           nparts, mt, mbox);
}

// Starting point: objective pieces of Omega^(0) (reduce-only prox sums of Omega^(0)
// and the norm sums of W0 = X Omega^(0)).
__device__ __forceinline__ void fit_init_run(LsState* ls, const double* prox_part, int nprox,
                                             const double* norm_part, int ntiles,
                                             double* trace) {
    double pv[6];
    sum_partials<6>(prox_part, nprox, kPartCols, pv);
    double nv[2];
    sum_partials<2>(norm_part, ntiles, kNormCols, nv);
    if (threadIdx.x != 0) return;
    ls->g_cur = 0.5 * nv[1] * ls->inv_n;
    ls->h_cur = -pv[P_LOGD] + ls->lambda * pv[P_L1];
    ls->f_cur = ls->g_cur + ls->h_cur;
    ls->logd_cur = pv[P_LOGD];
    ls->l1_cur = pv[P_L1];
    ls->nnz_off = (int64_t)pv[P_NNZ];
    if (!isfinite(nv[1]) || !isfinite(pv[P_L1])) ls->bad |= 2;
    if (!isfinite(ls->f_cur)) ls->bad |= 1;
    if (ls->bad || ls->max_iter <= 0) ls->converged = 1;
    if (trace) {
        trace[0] = ls->f_cur;
        trace[1] = ls->g_cur;
        trace[2] = ls->h_cur;
        trace[3] = 0.0;
        trace[4] = 0.0;
        trace[5] = 0.0;
        trace[6] = 0.0;
        trace[7] = pv[P_NNZ];
    }
}

__global__ void __launch_bounds__(kThreads) k_fit_init(LsState* ls, const double* prox_part,
                                                       int nprox, const double* norm_part,
                                                       int ntiles, double* trace) {
    fit_init_run(ls, prox_part, nprox, norm_part, ntiles, trace);
}

void launch_fit_init(LsState* ls, const double* prox_part, int nprox, const double* norm_part,
                     int ntiles, double* trace, hipStream_t st) {
    k_fit_init<<<1, kThreads, 0, st>>>(ls, prox_part, nprox, norm_part, ntiles, trace);
}

__global__ void __launch_bounds__(kThreads) k_combine_prox(const double* prox_part, int nprox,
                                                           double* red) {
    double pv[6];
    sum_partials<6>(prox_part, nprox, kPartCols, pv);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 6; ++k) red[k] = pv[k];
    }
}

void launch_combine_prox(const double* prox_part, int nprox, double* red, hipStream_t st) {
    k_combine_prox<<<1, kThreads, 0, st>>>(prox_part, nprox, red);
}

__global__ void __launch_bounds__(kThreads) k_combine_objective(const double* prox_part,
                                                                int nprox,
                                                                const double* norm_part,
                                                                int ntiles, double lambda,
                                                                double inv_n, double* out) {
    double pv[6];
    sum_partials<6>(prox_part, nprox, kPartCols, pv);
    double nv[2];
    sum_partials<2>(norm_part, ntiles, kNormCols, nv);
    if (threadIdx.x == 0) {
        const double g = 0.5 * nv[1] * inv_n;
        const double h = -pv[P_LOGD] + lambda * pv[P_L1];
        out[0] = g;
        out[1] = h;
        out[2] = g + h;
    }
}

void launch_combine_objective(const double* prox_part, int nprox, const double* norm_part,
                              int ntiles, double lambda, double inv_n, double* out,
                              hipStream_t st) {
    k_combine_objective<<<1, kThreads, 0, st>>>(prox_part, nprox, norm_part, ntiles, lambda,
                                                inv_n, out);
}

// ---------------------------------------------------------------------------
// L = sigma_max(S), S = X^T X / n (Sec. 3.2), by the Lanczos iteration on S:
//   q_1 = fixed sign vector / sqrt(p),  w = S q_k,  alpha_k = q_k^T w,
//   r = w - alpha_k q_k - beta_{k-1} q_{k-1},  beta_k = ||r||,  q_{k+1} = r / beta_k.
// After m steps the tridiagonal T_m (diagonal alpha, off-diagonal beta) has a largest
// eigenvalue theta (its top Ritz value) with unit eigenvector s, and the Ritz pair
// (theta, Q_m s) has the residual norm ||S Q_m s - theta Q_m s|| = beta_m |s_m|.  theta
// approaches sigma_max from below; the estimate is theta + beta_m |s_m|, so that the
// step floor tau <= 1/L of Alg. 1 errs on the safe side.  Every kLzCheck steps the
// residual bound is evaluated and the iteration stops once it is below kLzRelTol * theta
// (at n = 500, p = 5000 after 64 steps; at n = 1000, p = 1e5, where the top of the
// spectrum is crowded, after about 110).  It also stops when beta_k vanishes (the
// Krylov space is invariant, e.g. p = 1 or rank-one X: theta is then exact) and at the
// step cap.  theta comes from Sturm-count multisection on 64 lanes, s from inverse
// iteration on the positive definite sigma I - T_m with sigma just above theta.
// FP64 vectors, FP32 data; one step is four launches: u = X q (one workgroup per
// sample), w = X^T u / n with the partials of alpha (one wave per variable), r with the
// partials of ||r||^2, and q <- r / beta.  Every workgroup sums a set of partials
// itself, in the same fixed order, so all see the same alpha / beta.
// ---------------------------------------------------------------------------
struct LzArgs {
    const float* Xp;   // n x p_pad, row-major (padded X)
    int64_t ldp;
    const float* Xt;   // p x n_pad, row-major (padded X^T)
    int64_t ldt;
    int64_t n, p;
    LzBuf b;
    int nbw;           // workgroups of the w kernel (kThreads / 64 variables each)
    int nbr;           // workgroups of the elementwise kernels
};

__global__ void __launch_bounds__(kThreads) k_lz_start(LzArgs a) {
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < a.p;
         k += (int64_t)gridDim.x * kThreads) {
        // fixed pseudo-random signs (integer hash), scaled to a unit vector
        uint32_t h = (uint32_t)k * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        a.b.q1[k] = ((h & 1u) ? 1.0 : -1.0) / sqrt((double)a.p);
        a.b.q0[k] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.b.stop[0] = 0;
        a.b.stop[1] = 0;
    }
}

// u = X q_k: one workgroup per sample row
__global__ void __launch_bounds__(kThreads) k_lz_xq(LzArgs a) {
    if (*a.b.stop) return;
    const int64_t i = blockIdx.x;
    const float* row = a.Xp + i * a.ldp;
    double v[1] = {0.0};
    for (int64_t k = threadIdx.x; k < a.p; k += kThreads) v[0] += (double)row[k] * a.b.q1[k];
    block_sum<1>(v);
    if (threadIdx.x == 0) a.b.u[i] = v[0];
}

// w = X^T u / n (one wave per variable) and the partials of alpha_k = q_k^T w
__global__ void __launch_bounds__(kThreads) k_lz_xtu(LzArgs a) {
    if (*a.b.stop) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * (kThreads / 64) + wave;
    double s = 0.0;
    if (j < a.p) {
        const float* row = a.Xt + j * a.ldt;
        for (int64_t k = lane; k < a.n; k += 64) s += (double)row[k] * a.b.u[k];
        s = wave_sum(s) / (double)a.n;
        if (lane == 0) a.b.w[j] = s;
    }
    double v[1] = {(j < a.p && lane == 0) ? s * a.b.q1[j] : 0.0};
    block_sum<1>(v);
    if (threadIdx.x == 0) a.b.pa[blockIdx.x] = v[0];
}

// alpha_k, r = w - alpha_k q_k - beta_{k-1} q_{k-1} and the partials of ||r||^2
__global__ void __launch_bounds__(kThreads) k_lz_resid(LzArgs a, int k) {
    if (*a.b.stop) return;
    double al[1];
    sum_partials<1>(a.b.pa, a.nbw, 1, al);
    __shared__ double s_al;
    if (threadIdx.x == 0) s_al = al[0];
    __syncthreads();
    const double alpha = s_al, beta = k > 0 ? a.b.beta[k - 1] : 0.0;
    double v[1] = {0.0};
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < a.p;
         j += (int64_t)gridDim.x * kThreads) {
        const double r = a.b.w[j] - alpha * a.b.q1[j] - beta * a.b.q0[j];
        a.b.r[j] = r;
        v[0] += r * r;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) {
        a.b.pb[blockIdx.x] = v[0];
        if (blockIdx.x == 0) a.b.alpha[k] = alpha;
    }
}

// beta_k = ||r||; q_{k-1} <- q_k, q_k <- r / beta_k; stop (k + 1 valid steps) when beta_k
// vanishes against alpha_k + beta_{k-1}
__global__ void __launch_bounds__(kThreads) k_lz_next(LzArgs a, int k) {
    if (*a.b.stop) return;
    double bb[1];
    sum_partials<1>(a.b.pb, a.nbr, 1, bb);
    __shared__ double s_b;
    if (threadIdx.x == 0) s_b = sqrt(bb[0]);
    __syncthreads();
    const double beta = s_b;
    const double scale = fabs(a.b.alpha[k]) + (k > 0 ? a.b.beta[k - 1] : 0.0);
    if (!(beta > 1e-13 * scale)) {  // also for beta = 0 and non-finite values
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *a.b.stop = k + 1;
            a.b.stop[1] = kLzInvariant;
        }
        return;
    }
    const double inv = 1.0 / beta;
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < a.p;
         j += (int64_t)gridDim.x * kThreads) {
        a.b.q0[j] = a.b.q1[j];
        a.b.q1[j] = a.b.r[j] * inv;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.b.beta[k] = beta;
}

// Number of eigenvalues of the tridiagonal (alpha, beta) below x (Sturm sequence).
__device__ inline int sturm_below(const double* al, const double* be, int m, double x) {
    int cnt = 0;
    double d = al[0] - x;
    for (int i = 0;; ++i) {
        if (d == 0.0) d = -1e-300;  // x on an eigenvalue of the leading block: count it below
        cnt += d < 0.0 ? 1 : 0;
        if (i + 1 == m) break;
        d = al[i + 1] - x - be[i] * be[i] / d;
    }
    return cnt;
}

// Largest eigenvalue theta of T_m (one wave): the Gershgorin interval is cut into 65
// parts per round by the Sturm counts of 64 lanes; [lo, hi] keeps the top eigenvalue.
// Returns hi (>= theta up to the count's rounding) and writes lo.
__device__ double lz_top_ritz(const double* al, const double* be, int m, double* lo_out) {
    const int lane = threadIdx.x & 63;
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < m; ++i) {
        const double rad = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < m ? fabs(be[i]) : 0.0);
        lo = i == 0 ? al[i] - rad : fmin(lo, al[i] - rad);
        hi = i == 0 ? al[i] + rad : fmax(hi, al[i] + rad);
    }
    for (int round = 0; round < 12 && hi > lo; ++round) {
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        // lanes whose point lies above every eigenvalue
        const uint64_t above = __ballot(sturm_below(al, be, m, x) == m);
        const int first = above ? __ffsll((unsigned long long)above) - 1 : 64;
        const double nhi = first < 64 ? __shfl(x, first, 64) : hi;
        const double nlo = first > 0 ? __shfl(x, first - 1, 64) : lo;
        if (!(nhi < hi || nlo > lo)) break;  // the points no longer split the interval
        lo = nlo;
        hi = nhi;
    }
    *lo_out = lo;
    return hi;
}

// |s_m| of the unit eigenvector s of T_m for its top eigenvalue: three steps of inverse
// iteration with sigma I - T_m (sigma above every eigenvalue, so the LDL^T pivots are
// positive and the tridiagonal solve needs no pivoting).  One thread.
__device__ double lz_last_component(const double* al, const double* be, int m, double hi) {
    if (m == 1) return 1.0;
    const double sigma = hi + 1e-13 * fabs(hi) + 1e-300;
    double d[kLzMaxSteps], y[kLzMaxSteps];
    d[0] = sigma - al[0];
    for (int i = 1; i < m; ++i) d[i] = sigma - al[i] - be[i - 1] * be[i - 1] / d[i - 1];
    for (int i = 0; i < m; ++i) y[i] = 1.0;
    double last = 0.0;
    for (int it = 0; it < 3; ++it) {
        // (sigma I - T) z = y: forward with L (sub-diagonal -be[i] / d[i]), back with D L^T
        for (int i = 1; i < m; ++i) y[i] += be[i - 1] / d[i - 1] * y[i - 1];
        y[m - 1] /= d[m - 1];
        for (int i = m - 2; i >= 0; --i) y[i] = (y[i] + be[i] * y[i + 1]) / d[i];
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm = fmax(nrm, fabs(y[i]));
        double ss = 0.0;
        for (int i = 0; i < m; ++i) {
            y[i] /= nrm;
            ss += y[i] * y[i];
        }
        last = fabs(y[m - 1]) / sqrt(ss);
    }
    return last;
}

// Every kLzCheck steps: stop once the Ritz residual bound is below kLzRelTol * theta.
__global__ void k_lz_check(LzArgs a, int k) {
    if (*a.b.stop) return;
    const int m = k + 1;
    double lo;
    const double hi = lz_top_ritz(a.b.alpha, a.b.beta, m, &lo);
    if (threadIdx.x != 0) return;
    const double bound = a.b.beta[k] * lz_last_component(a.b.alpha, a.b.beta, m, hi);
    if (bound <= kLzRelTol * hi) {
        *a.b.stop = m;
        a.b.stop[1] = kLzConverged;
    }
}

// L = theta + beta_m |s_m| after m valid steps (theta alone when the space is invariant)
__global__ void k_lz_finish(LzArgs a, int steps, LsState* ls) {
    if (blockIdx.x != 0) return;
    const int m = *a.b.stop > 0 ? *a.b.stop : steps;
    double lo;
    const double hi = lz_top_ritz(a.b.alpha, a.b.beta, m, &lo);
    if (threadIdx.x != 0) return;
    const double theta = 0.5 * (lo + hi);
    const bool invariant = *a.b.stop > 0 && a.b.stop[1] == kLzInvariant;
    const double bound = invariant ? 0.0
                                   : a.b.beta[m - 1] * lz_last_component(a.b.alpha, a.b.beta, m, hi);
    const double L = isfinite(theta) ? theta + bound : theta;
    ls->L = L;
    ls->inv_L = L > 0.0 ? 1.0 / L : 0.0;
    ls->lz_steps = m;
}

size_t lz_buf_bytes(int64_t n_pad, int64_t p_pad) {
    const int64_t nbw = cdiv(p_pad, kThreads / 64);
    return (size_t)(4 * p_pad + n_pad + nbw + kLzMaxBlocks + 2 * kLzMaxSteps + 2) * sizeof(double);
}

LzBuf lz_buf(void* base, int64_t n_pad, int64_t p_pad) {
    double* d = (double*)base;
    const int64_t nbw = cdiv(p_pad, kThreads / 64);
    LzBuf b;
    b.q0 = d;
    b.q1 = b.q0 + p_pad;
    b.r = b.q1 + p_pad;
    b.w = b.r + p_pad;
    b.u = b.w + p_pad;
    b.pa = b.u + n_pad;
    b.pb = b.pa + nbw;
    b.alpha = b.pb + kLzMaxBlocks;
    b.beta = b.alpha + kLzMaxSteps;
    b.stop = (int*)(b.beta + kLzMaxSteps);
    return b;
}

void launch_lipschitz(const float* Xp, int64_t p_pad, const float* Xt, int64_t n_pad, int64_t n,
                      int64_t p, const LzBuf& buf, int steps, LsState* ls, hipStream_t st) {
    if (steps > kLzMaxSteps) steps = kLzMaxSteps;
    LzArgs a;
    a.Xp = Xp;
    a.ldp = p_pad;
    a.Xt = Xt;
    a.ldt = n_pad;
    a.n = n;
    a.p = p;
    a.b = buf;
    a.nbw = (int)cdiv(p, kThreads / 64);
    const int64_t nr = cdiv(p, kThreads);
    a.nbr = (int)(nr < kLzMaxBlocks ? nr : kLzMaxBlocks);
    k_lz_start<<<(unsigned)a.nbr, kThreads, 0, st>>>(a);
    for (int k = 0; k < steps; ++k) {
        k_lz_xq<<<(unsigned)n, kThreads, 0, st>>>(a);
        k_lz_xtu<<<(unsigned)a.nbw, kThreads, 0, st>>>(a);
        k_lz_resid<<<(unsigned)a.nbr, kThreads, 0, st>>>(a, k);
        k_lz_next<<<(unsigned)a.nbr, kThreads, 0, st>>>(a, k);
        if ((k + 1) % kLzCheck == 0 && k + 1 < steps) k_lz_check<<<1, 64, 0, st>>>(a, k);
    }
    k_lz_finish<<<1, 64, 0, st>>>(a, steps, ls);
}

}  // namespace accord

// ---------------------------------------------------------------------------
// Batched form: many independent fits advanced in lockstep, one iteration per
// sweep.  A group (one data set X_b) holds nlam problems whose column blocks are
// concatenated along N, each padded to a whole number of 128-column tiles, so a
// tile belongs to exactly one problem: problem = tile_n / tpp.  Every problem
// keeps its own line-search state; a tile, prox block or acceptance workgroup of a
// problem that has accepted (or stopped) returns at once.  Argument blocks live in
// device memory, one per group (GEMM) or per problem (prox, acceptance).
// ---------------------------------------------------------------------------
namespace accord {

// Tile order of the batched kernels: which tile of group blockIdx.y workgroup blockIdx.x
// computes.  Every order is a permutation of the tiles, and a tile's arithmetic and the
// rows its partial sums go to do not depend on which workgroup computes it, so the order
// changes the run time only, never a result.  code 0: the default (plain block order,
// bands of 8 M tiles walking across N); code 1 + c and 1 + kBatchOrders + c (the same
// order at one workgroup per CU, batch_occupancy), c < kBatchOrders: bands of
// GM = 2^(c % 5) M tiles, in plain block order (c < 5) or with every XCD given a
// contiguous range of the tiles (c >= 5; blocks are dispatched round-robin over the 8
// XCDs).  Returns false for the workgroups beyond the group's tiles.
__device__ inline bool batch_tile(int code, int tilesM, int tilesN, int& tile_m, int& tile_n) {
    const int tiles = tilesM * tilesN;
    const int c = code > 0 ? (code - 1) % kBatchOrders : 3;
    const int GM = 1 << (c % 5);
    int logical = blockIdx.x;
    if (c >= 5) {
        const int nblk = gridDim.x, bid = blockIdx.x;
        const int xcd = bid & 7, local = bid >> 3, q8 = nblk >> 3, r8 = nblk & 7;
        logical = xcd * q8 + (xcd < r8 ? xcd : r8) + local;
    }
    if (logical >= tiles) return false;
    const int per_group = GM * tilesN;
    const int group = logical / per_group;
    const int first_m = group * GM;
    const int gsize = (tilesM - first_m) < GM ? (tilesM - first_m) : GM;
    const int in_group = logical - group * per_group;
    tile_m = first_m + in_group % gsize;
    tile_n = in_group / gsize;
    return true;
}

// OCC: workgroups per CU the code is compiled for (2: at most 128 registers per lane;
// 1: up to 512, which the compiler spends on accumulators in AGPRs and deeper operand
// staging).  The arithmetic of a tile is the same instruction sequence either way.
template <int EPI, int OCC>
__global__ void __launch_bounds__(kThreads, OCC) k_gemm_f32_batch(const GemmArgs* __restrict__ batch,
                                                                 int tpp) {
    const GemmArgs g = batch[blockIdx.y];
    // Default order (code 0): plain block order, so consecutive tiles land on different
    // XCDs and the tiles of every problem spread over all of them.  Problems finish
    // their line searches at different trials; an XCD-contiguous order can leave the
    // XCDs of finished problems idle while the others carry the problems still
    // searching.  The operand shared by a group's tiles (its X) is a few MB and stays
    // in every XCD's L2.  Other orders: batch_tile (chosen by accord_tune_batch).
    int tile_m, tile_n;
    if (!batch_tile(g.order, g.tilesM, g.tilesN, tile_m, tile_n)) return;
    const int prob = tile_n / tpp;
    LsState* ls = g.ls + prob;
    if (g.pred >= 1 && ls->converged) return;
    if (g.pred >= 2 && ls->done) return;
    if (g.begin_iter && tile_m == 0 && tile_n == prob * tpp && threadIdx.x == 0) {
        // a new iteration of this problem starts from tau0 (Alg. 1)
        ls->done = 0;
        ls->trials = 0;
        ls->tau = start_tau(*ls);
    }
    double* nrm = g.norm_part +
                  ((int64_t)prob * g.tilesM * tpp + tile_m + (int64_t)(tile_n - prob * tpp) * g.tilesM) *
                      kNormCols;
    gemm_f32_tile<EPI>(g, tile_m, tile_n, 0, nrm);
}

// Batched fused prox + trial product (FP32 tile of k_trial_fused32): group blockIdx.y,
// whose problems' columns are packed along N (tpp tiles each, no split), same tile
// order as k_gemm_f32_batch.  Each tile reads its problem's state (skipped once that
// problem accepted or stopped), step and penalty, and leaves its prox sums in row
// tile_n - prob * tpp of the problem's block of nprox_rows rows.
template <int OCC>
__global__ void __launch_bounds__(kThreads, OCC) k_trial_fused32_batch(
    const GemmArgs* __restrict__ gb, const ProxArgs* __restrict__ pb, int tpp, int nprox_rows) {
    const GemmArgs g = gb[blockIdx.y];
    const ProxArgs px = pb[blockIdx.y];
    int tile_m, tile_n;
    if (!batch_tile(g.order, g.tilesM, g.tilesN, tile_m, tile_n)) return;
    const int prob = tile_n / tpp;
    const LsState* ls = px.ls + prob;
    if (g.pred >= 1 && ls->converged) return;
    if (g.pred >= 2 && ls->done) return;
    const int tn = tile_n - prob * tpp;
    double* nrm = g.norm_part +
                  ((int64_t)prob * g.tilesM * tpp + tile_m + (int64_t)tn * g.tilesM) * kNormCols;
    double* part_row = px.part + ((int64_t)prob * nprox_rows + tn) * kPartCols;
    trial_fused32_tile<EPI_TRIAL>(g, px, tile_m, tile_n, 0, prob * tpp * kBN, g.N, ls->tau,
                                  ls->lambda, part_row, nrm);
}

template <int DOUT>
__global__ void __launch_bounds__(kThreads) k_prox_batch(const ProxArgs* __restrict__ batch) {
    const ProxArgs a = batch[blockIdx.y];
    prox_run<DOUT>(a);
}

__global__ void __launch_bounds__(kThreads) k_finalize_batch(const FinArgs* __restrict__ batch) {
    const FinArgs f = batch[blockIdx.x];
    finalize_run(f.ls, f.prox_part, f.nprox, f.norm_part, f.ntiles, nullptr, f.trials_log,
                 nullptr, 0);
}

__global__ void __launch_bounds__(kThreads) k_fit_init_batch(const FinArgs* __restrict__ batch) {
    const FinArgs f = batch[blockIdx.x];
    fit_init_run(f.ls, f.prox_part, f.nprox, f.norm_part, f.ntiles, nullptr);
}

// Line-search state of every problem k = b * nlam + l: lambda[l], 1/n_b, and L_b
// (0 = taken later from the Lanczos estimate of group b).
__global__ void k_init_state_batch(LsState* ls, int nprob, int nlam, const double* lam,
                                   const double* inv_n, const double* L, double tau0,
                                   double beta, double tol, int max_iter, int warm_tau) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nprob) return;
    const int b = k / nlam;
    LsState s = {};
    s.tau = tau0;
    s.tau0 = tau0;
    s.beta = beta;
    s.lambda = lam[k - b * nlam];
    s.tol = tol;
    s.inv_n = inv_n[b];
    s.L = L[b];
    s.inv_L = L[b] > 0 ? 1.0 / L[b] : 0.0;
    s.max_iter = max_iter;
    s.fixed_step = beta >= 1.0;
    s.warm_tau = warm_tau;
    ls[k] = s;
}

// L of group b (estimated into its first problem's state) -> every problem of b
__global__ void k_share_L_batch(LsState* ls, int nprob, int nlam) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nprob) return;
    const int first = (k / nlam) * nlam;
    if (k == first) return;
    ls[k].L = ls[first].L;
    ls[k].inv_L = ls[first].inv_L;
}

void launch_gemm_f32_batch(const GemmArgs* batch, int ngroups, int max_tiles, int tpp, int epi,
                           int code, hipStream_t st) {
    dim3 grid((unsigned)max_tiles, (unsigned)ngroups);
    const bool one = batch_occupancy(code) == 1;
    if (epi == EPI_GRAD) {
        if (one) k_gemm_f32_batch<EPI_GRAD, 1><<<grid, kThreads, 0, st>>>(batch, tpp);
        else k_gemm_f32_batch<EPI_GRAD, 2><<<grid, kThreads, 0, st>>>(batch, tpp);
    } else {
        if (one) k_gemm_f32_batch<EPI_TRIAL, 1><<<grid, kThreads, 0, st>>>(batch, tpp);
        else k_gemm_f32_batch<EPI_TRIAL, 2><<<grid, kThreads, 0, st>>>(batch, tpp);
    }
}

void launch_trial_fused32_batch(const GemmArgs* gb, const ProxArgs* pb, int ngroups,
                                int max_tiles, int tpp, int nprox_rows, int code,
                                hipStream_t st) {
    dim3 grid((unsigned)max_tiles, (unsigned)ngroups);
    if (batch_occupancy(code) == 1)
        k_trial_fused32_batch<1><<<grid, kThreads, 0, st>>>(gb, pb, tpp, nprox_rows);
    else
        k_trial_fused32_batch<2><<<grid, kThreads, 0, st>>>(gb, pb, tpp, nprox_rows);
}

void launch_prox_batch(const ProxArgs* batch, int nprob, int nblocks, hipStream_t st) {
    dim3 grid((unsigned)nblocks, (unsigned)nprob);
    k_prox_batch<0><<<grid, kThreads, 0, st>>>(batch);
}

void launch_finalize_batch(const FinArgs* batch, int nprob, hipStream_t st) {
    k_finalize_batch<<<(unsigned)nprob, kThreads, 0, st>>>(batch);
}

void launch_fit_init_batch(const FinArgs* batch, int nprob, hipStream_t st) {
    k_fit_init_batch<<<(unsigned)nprob, kThreads, 0, st>>>(batch);
}

void launch_init_state_batch(LsState* ls, int nprob, int nlam, const double* lam,
                             const double* inv_n, const double* L, double tau0, double beta,
                             double tol, int max_iter, hipStream_t st, int warm_tau) {
    k_init_state_batch<<<(unsigned)cdiv(nprob, 256), 256, 0, st>>>(ls, nprob, nlam, lam, inv_n, L,
                                                                   tau0, beta, tol, max_iter,
                                                                   warm_tau);
}

void launch_share_L_batch(LsState* ls, int nprob, int nlam, hipStream_t st) {
    k_share_L_batch<<<(unsigned)cdiv(nprob, 256), 256, 0, st>>>(ls, nprob, nlam);
}

// ---------------------------------------------------------------------------
// Steps around the solver.
//
// Support mask of the refit (eq. 3.8): byte (r, c) of the padded p x p_pad layout is
// 1 where the first-stage estimate is nonzero or r == c (the diagonal is positive on
// the domain), 0 elsewhere and on the padded rows.  The refit's starting iterate (already
// copied into the padded layout) is projected onto the support in the same pass.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_support_mask(const float* __restrict__ om_hat,
                                                           int64_t p, int64_t p_pad,
                                                           uint8_t* __restrict__ mask,
                                                           float* __restrict__ om0) {
    const int64_t n4 = p * p_pad / 4;  // p_pad is a multiple of 4: quads never cross columns
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n4;
         q += (int64_t)gridDim.x * kThreads) {
        const int64_t e = q * 4;
        const int64_t c = e / p_pad, r0 = e - c * p_pad;
        f4 o = ((const f4*)om0)[q];
        uint32_t m4 = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t r = r0 + u;
            const bool in = r < p && (r == c || om_hat[r + c * p] != 0.f);
            m4 |= (in ? 1u : 0u) << (8 * u);
            if (!in) o[u] = 0.f;
        }
        ((uint32_t*)mask)[q] = m4;
        ((f4*)om0)[q] = o;
    }
}

void launch_support_mask(const float* om_hat, int64_t p, int64_t p_pad, uint8_t* mask,
                         float* om0, hipStream_t st) {
    int64_t b = cdiv(p * p_pad / 4, kThreads);
    if (b > 16384) b = 16384;
    k_support_mask<<<(unsigned)b, kThreads, 0, st>>>(om_hat, p, p_pad, mask, om0);
}

// Blocks of a refit that can hold a nonzero entry: occ[tn * ksteps + s] = 1 if the support
// mask has a nonzero byte in rows 32 s .. 32 s + 31 of the columns 128 tn .. 128 tn + 127
// (those below p).  Everywhere else the iterate, its gradient and every trial step are
// zero in every iteration (the start is projected onto the support, and the gradient is
// stored as zero off it).  One thread per (tn, s), 32 bytes per column.
__global__ void __launch_bounds__(kThreads) k_support_occupancy(const uint8_t* __restrict__ mask,
                                                                int64_t p, int64_t p_pad,
                                                                int tilesN, int ksteps,
                                                                uint8_t* __restrict__ occ) {
    const int64_t total = (int64_t)tilesN * ksteps;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t tn = e / ksteps, s = e - tn * ksteps;
        const int64_t c0 = tn * kFBN;
        const int64_t c1 = c0 + kFBN < p ? c0 + kFBN : p;
        unsigned int any = 0;
        for (int64_t c = c0; c < c1; ++c) {
            const u4* q = (const u4*)(mask + c * p_pad + 32 * s);
            const u4 a = q[0], b = q[1];
            any |= a[0] | a[1] | a[2] | a[3] | b[0] | b[1] | b[2] | b[3];
        }
        occ[e] = any ? 1 : 0;
    }
}

void launch_support_occupancy(const uint8_t* mask, int64_t p, int64_t p_pad, int tilesN,
                              int ksteps, uint8_t* occ, hipStream_t st) {
    int64_t b = cdiv((int64_t)tilesN * ksteps, kThreads);
    if (b > 16384) b = 16384;
    k_support_occupancy<<<(unsigned)b, kThreads, 0, st>>>(mask, p, p_pad, tilesN, ksteps, occ);
}

// ---------------------------------------------------------------------------
// Reparametrisation (Sec. 2): Theta = Omega_D Omega (the inverse of the map T) and the
// partial correlations rho_ij = -(w_ij / w_jj + w_ji / w_ii) / 2, w in the paper's
// orientation.  In the column form (Om = Omega^T, column-major) that is
//     Theta^T(i, j) = Om(j, j) Om(i, j)            (column j scaled by its diagonal)
//     rho(i, j)     = -(Om(j, i) / Om(j, j) + Om(i, j) / Om(i, i)) / 2,   rho(i, i) = 1.
// rho needs Om and Om^T, so one workgroup owns a pair of 64 x 64 tiles (I, J), (J, I)
// with I <= J: both are staged through LDS once (padded rows, no bank conflicts), and
// all four output tiles are written with columns along the lanes.  Omega is read once
// and each output written once: HBM-bound.  The ratios use FP64 reciprocals of the
// diagonal and one rounding to FP32; the Theta product of two FP32 values is exact in
// FP64, so Theta is correctly rounded.
// ---------------------------------------------------------------------------
constexpr int kRT = 64;

__global__ void __launch_bounds__(kThreads) k_reparam(const float* __restrict__ om, int64_t p,
                                                      float* __restrict__ theta,
                                                      float* __restrict__ rho) {
    __shared__ float sa[kRT][kRT + 1];   // sa[c][r] = Om(I0 + r, J0 + c)
    __shared__ float sb[kRT][kRT + 1];   // sb[c][r] = Om(J0 + r, I0 + c)
    __shared__ float dI[kRT], dJ[kRT];
    __shared__ double iI[kRT], iJ[kRT];
    // pair k = J (J + 1) / 2 + I, 0 <= I <= J
    const int64_t k = blockIdx.x;
    int64_t J = (int64_t)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
    while ((J + 1) * (J + 2) / 2 <= k) ++J;
    while (J * (J + 1) / 2 > k) --J;
    const int64_t I = k - J * (J + 1) / 2;
    const int64_t I0 = I * kRT, J0 = J * kRT;
    const int r = threadIdx.x & (kRT - 1);
    const int c4 = threadIdx.x >> 6;   // 0..3
    const bool rI = I0 + r < p, rJ = J0 + r < p;
    for (int c = c4; c < kRT; c += kThreads / kRT) {
        const bool cJ = J0 + c < p, cI = I0 + c < p;
        sa[c][r] = (rI && cJ) ? om[(I0 + r) + (J0 + c) * p] : 0.f;
        sb[c][r] = (rJ && cI) ? om[(J0 + r) + (I0 + c) * p] : 0.f;
    }
    if (threadIdx.x < kRT) {
        const float di = rI ? om[(I0 + r) * (p + 1)] : 1.f;
        const float dj = rJ ? om[(J0 + r) * (p + 1)] : 1.f;
        dI[r] = di;
        dJ[r] = dj;
        iI[r] = 1.0 / (double)di;
        iJ[r] = 1.0 / (double)dj;
    }
    __syncthreads();
    // tile (I, J): row I0 + r, column J0 + c
    if (rI) {
        for (int c = c4; c < kRT; c += kThreads / kRT) {
            if (J0 + c >= p) break;
            const int64_t o = (I0 + r) + (J0 + c) * p;
            if (theta) theta[o] = (float)((double)dJ[c] * (double)sa[c][r]);
            if (rho) {
                const double v = -0.5 * ((double)sb[r][c] * iJ[c] + (double)sa[c][r] * iI[r]);
                rho[o] = (I0 + r == J0 + c) ? 1.f : (float)v;
            }
        }
    }
    if (I == J) return;
    // tile (J, I): row J0 + r, column I0 + c
    if (rJ) {
        for (int c = c4; c < kRT; c += kThreads / kRT) {
            if (I0 + c >= p) break;
            const int64_t o = (J0 + r) + (I0 + c) * p;
            if (theta) theta[o] = (float)((double)dI[c] * (double)sb[c][r]);
            if (rho) {
                const double v = -0.5 * ((double)sb[c][r] * iJ[r] + (double)sa[r][c] * iI[c]);
                rho[o] = (float)v;
            }
        }
    }
}

void launch_reparam(const float* om, int64_t p, float* theta, float* rho, hipStream_t st) {
    const int64_t nt = cdiv(p, kRT);
    k_reparam<<<(unsigned)(nt * (nt + 1) / 2), kThreads, 0, st>>>(om, p, theta, rho);
}

}  // namespace accord

// ---------------------------------------------------------------------------
// Differentiation form: reverse pass of the fixed-step iteration (the adjoint of
// one prox-gradient step) and the held-out loss gradient.
// ---------------------------------------------------------------------------
namespace accord {

// Reverse of eq. 3.5 at a = Omega - tau G (same FP32 arithmetic as the forward
// prox, so the active set matches it):
//   off-diagonal  abar = obar 1{|a| > tau lambda},  dl = -tau sign(a) 1{...}
//   diagonal      b = a - tau lambda, r = sqrt(b^2 + 4 tau), d = (1 + b/r)/2 (FP64):
//                 abar = obar d,  dl = -tau d
// abar -> p x ld (zero in padded rows); per-workgroup FP64 partials of sum(obar dl).
__global__ void __launch_bounds__(kThreads) k_prox_adjoint(AdjArgs a) {
    const float tau_f = (float)a.tau, thr_f = (float)(a.tau * a.lambda);
    double s = 0.0;
    const int64_t total = a.p * a.ld;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t j = e / a.ld, i = e - j * a.ld;
        float out = 0.f;
        if (i < a.p) {
            const float o = a.om[e], gv = a.g[e];
            const float ob = a.obar[j * a.ld_obar + i];
            if (i == j) {
                const double y = (double)o - a.tau * (double)gv;
                const double b = y - a.tau * a.lambda;
                const double r = sqrt(b * b + 4.0 * a.tau);
                const double d = 0.5 * (1.0 + b / r);
                out = (float)((double)ob * d);
                s += (double)ob * (-a.tau * d);
            } else {
                const float av = fmaf(-tau_f, gv, o);
                if (fabsf(av) - thr_f > 0.f) {
                    out = ob;
                    s += (double)ob * (av > 0.f ? -a.tau : a.tau);
                }
            }
        }
        a.abar[e] = out;
    }
    double v[1] = {s};
    block_sum<1>(v);
    if (threadIdx.x == 0) a.part[blockIdx.x] = v[0];
}

// obar_t = abar - tau * SA  (p x p, ld_out) from the padded abar / SA (ld)
__global__ void __launch_bounds__(kThreads) k_adjoint_combine(const float* __restrict__ abar,
                                                              const float* __restrict__ sa,
                                                              int64_t ld, int64_t p, float tau,
                                                              float* __restrict__ out,
                                                              int64_t ld_out) {
    const int64_t total = p * p;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t j = e / p, i = e - j * p;
        out[j * ld_out + i] = fmaf(-tau, sa[j * ld + i], abar[j * ld + i]);
    }
}

// dst[c * ld_dst + r] = src[r * ld_src + c]  for r < rows, c < cols (32 x 32 LDS tiles)
__global__ void __launch_bounds__(kThreads) k_transpose_ld(const float* __restrict__ src,
                                                           int64_t ld_src, int64_t rows,
                                                           int64_t cols, float* __restrict__ dst,
                                                           int64_t ld_dst) {
    __shared__ float tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int rr = ty; rr < 32; rr += kThreads / 32) {
        const int64_t r = r0 + rr, c = c0 + tx;
        tile[rr][tx] = (r < rows && c < cols) ? src[r * ld_src + c] : 0.f;
    }
    __syncthreads();
    for (int cc = ty; cc < 32; cc += kThreads / 32) {
        const int64_t c = c0 + cc, r = r0 + tx;
        if (c < cols && r < rows) dst[c * ld_dst + r] = tile[tx][cc];
    }
}

// acc[0] += sum of the partials (fixed order)
__global__ void __launch_bounds__(kThreads) k_accumulate_scalar(const double* part, int count,
                                                                double* acc) {
    double v[1];
    sum_partials<1>(part, count, 1, v);
    if (threadIdx.x == 0) acc[0] += v[0];
}

// obar_jj -= 1 / Omega_jj  (the -sum log Omega_jj term of the held-out loss)
__global__ void k_sub_inv_diag(float* obar, int64_t ld_obar, const float* om, int64_t ld_om,
                               int64_t p) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p) return;
    obar[j * ld_obar + j] -= (float)(1.0 / (double)om[j * ld_om + j]);
}

void launch_prox_adjoint(const AdjArgs& a, int nblocks, hipStream_t st) {
    k_prox_adjoint<<<(unsigned)nblocks, kThreads, 0, st>>>(a);
}

void launch_adjoint_combine(const float* abar, const float* sa, int64_t ld, int64_t p, float tau,
                            float* out, int64_t ld_out, hipStream_t st) {
    int64_t b = cdiv(p * p, (int64_t)kThreads * 8);
    if (b > 16384) b = 16384;
    k_adjoint_combine<<<(unsigned)b, kThreads, 0, st>>>(abar, sa, ld, p, tau, out, ld_out);
}

void launch_transpose_ld(const float* src, int64_t ld_src, int64_t rows, int64_t cols, float* dst,
                         int64_t ld_dst, hipStream_t st) {
    dim3 grid((unsigned)cdiv(cols, 32), (unsigned)cdiv(rows, 32));
    k_transpose_ld<<<grid, kThreads, 0, st>>>(src, ld_src, rows, cols, dst, ld_dst);
}

void launch_accumulate_scalar(const double* part, int count, double* acc, hipStream_t st) {
    k_accumulate_scalar<<<1, kThreads, 0, st>>>(part, count, acc);
}

void launch_sub_inv_diag(float* obar, int64_t ld_obar, const float* om, int64_t ld_om, int64_t p,
                         hipStream_t st) {
    k_sub_inv_diag<<<(unsigned)cdiv(p, 256), 256, 0, st>>>(obar, ld_obar, om, ld_om, p);
}

}  // namespace accord
