// HIP kernels of the ACCORD-FBS hot path for gfx950 (MI355X).
//
//   k_gemm_f32     FP32 MFMA (v_mfma_f32_16x16x4f32) GEMM, LDS double-buffered
//                  128x128x32 tiles, XCD-aware tile order.  Two uses:
//                    gradient  G  = X^T W / n              (Remark 3.1, two-step product)
//                    trial     W+ = W + X Delta, ||X Delta||^2, ||W+||^2 (Alg. 1 test)
//   k_splitk_reduce fixed-order sum of split-K partial tiles + trial epilogue
//   k_prox         fused closed-form prox (eq. 3.5) + FP64 line-search partial sums
//   k_finalize     FP64 acceptance test of Alg. 1, step update, iteration record
//   k_pow_*        power iteration for L = sigma_max(X^T X / n) (Sec. 3.2)
//   copies / transposes into the padded operand layouts
//
// All cross-workgroup reductions are two-stage (per-workgroup partials, then one
// workgroup summing them in a fixed order), so results are bit-reproducible.
#include <math.h>

#include "accord_internal.h"

namespace accord {

typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum of NV doubles (blockDim.x == kThreads); result valid in thread 0.
template <int NV>
__device__ inline void block_sum(double (&v)[NV]) {
    __shared__ double sh[kThreads / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) sh[wave][q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = sh[0][q];
            for (int w = 1; w < kThreads / 64; ++w) s += sh[w][q];
            v[q] = s;
        }
    }
    __syncthreads();
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

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------
__global__ void k_init_state(LsState* ls, double tau0, double beta, double lambda, double tol,
                             double inv_n, double L, int max_iter) {
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
    *ls = s;
}

void launch_init_state(LsState* ls, double tau0, double beta, double lambda, double tol,
                       double inv_n, double L, int max_iter, hipStream_t st) {
    k_init_state<<<1, 64, 0, st>>>(ls, tau0, beta, lambda, tol, inv_n, L, max_iter);
}

// ---------------------------------------------------------------------------
// operand preparation
// ---------------------------------------------------------------------------
// X (n x p row-major) -> Xp (n_pad x p_pad row-major) and Xt (p_pad x n_pad row-major),
// zero padding; flags non-finite input (bit 1 of ls->bad).
__global__ void __launch_bounds__(kThreads) k_pad_x(const float* __restrict__ X, int64_t n,
                                                    int64_t p, float* __restrict__ Xp,
                                                    int64_t p_pad, float* __restrict__ Xt,
                                                    int64_t n_pad, LsState* ls) {
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
    }
    __syncthreads();
    for (int cc = ty; cc < 32; cc += 8) {
        const int64_t c = c0 + cc, r = r0 + tx;
        Xt[c * n_pad + r] = tile[tx][cc];
    }
    if (bad) atomicOr(&ls->bad, 2);
}

void launch_pad_x(const float* X, int64_t n, int64_t p, float* Xp, int64_t p_pad, float* Xt,
                  int64_t n_pad, LsState* ls, hipStream_t st) {
    dim3 grid((unsigned)(p_pad / 32), (unsigned)(n_pad / 32));
    k_pad_x<<<grid, kThreads, 0, st>>>(X, n, p, Xp, p_pad, Xt, n_pad, ls);
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
// FP32 MFMA GEMM:  C(m, n) = sum_k A[m, k] * B[n, k]   (both operands K-contiguous)
//
// Workgroup tile 128 x 128, 4 waves in a 2 x 2 arrangement, each wave 64 x 64 =
// 4 x 4 blocks of v_mfma_f32_16x16x4f32.  A 32-wide K step is staged in LDS
// (row stride 36 floats, so 16 lanes reading 16 rows at one K offset hit distinct
// banks) and double-buffered: the next step's global loads are in flight while
// the current step's MFMAs run.
//
// Lane l of a wave supplies, for one MFMA, A row (l % 16) and B column (l % 16)
// at MFMA-internal k = l / 16.  Each lane reads 4 consecutive K values with one
// 16-byte LDS read and feeds them to 4 successive MFMAs, i.e. MFMA-internal k = g
// of step q maps to tile column 4g + q.  A and B use the same map, so every
// product pairs matching K indices; only the summation order changes.
// The 16x16 accumulator holds C(4*(l/16) + r, l % 16) in register r of lane l.
// ---------------------------------------------------------------------------
constexpr int kLDK = kBK + 4;

__device__ inline void decode_tile(const GemmArgs& g, int& tile_m, int& tile_n, int& split) {
    // Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
    // Give every XCD a contiguous range of logical tiles so tiles that share operand
    // panels run on the same XCD and hit in its L2.
    const int nblk = gridDim.x, bid = blockIdx.x;
    const int xcd = bid & 7, local = bid >> 3, q8 = nblk >> 3, r8 = nblk & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + local;
    if (g.splits > 1) {
        // tile_m fastest: the M tiles of one (split, N tile) share the B panel
        tile_m = logical % g.tilesM;
        const int rest = logical / g.tilesM;
        tile_n = rest % g.tilesN;
        split = rest / g.tilesN;
    } else {
        // grouped order: bands of 8 M tiles walk across N
        constexpr int GM = 8;
        const int per_group = GM * g.tilesN;
        const int group = logical / per_group;
        const int first_m = group * GM;
        const int gsize = (g.tilesM - first_m) < GM ? (g.tilesM - first_m) : GM;
        const int in_group = logical - group * per_group;
        tile_m = first_m + in_group % gsize;
        tile_n = in_group / gsize;
        split = 0;
    }
}

template <int EPI>
__global__ void __launch_bounds__(kThreads, 2) k_gemm_f32(GemmArgs g) {
    if (g.ls) {
        if (g.pred >= 1 && g.ls->converged) return;
        if (g.pred >= 2 && g.ls->done) return;
    }
    if (g.begin_iter && blockIdx.x == 0 && threadIdx.x == 0) {
        // a new iteration starts from tau0 (Alg. 1); nothing else reads these now
        g.ls->done = 0;
        g.ls->trials = 0;
        g.ls->tau = g.ls->tau0;
    }
    __shared__ __attribute__((aligned(16))) float sA[2][kBM * kLDK];
    __shared__ __attribute__((aligned(16))) float sB[2][kBN * kLDK];

    int tile_m, tile_n, split;
    decode_tile(g, tile_m, tile_n, split);
    const int m0 = tile_m * kBM, n0 = tile_n * kBN;
    const int s_begin = (int)((int64_t)g.ksteps * split / g.splits);
    const int s_end = (int)((int64_t)g.ksteps * (split + 1) / g.splits);

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
            const int64_t ko = (int64_t)s_begin * kBK;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                va[i] = *(const f4*)(pa[i] + ko);
                vb[i] = *(const f4*)(pb[i] + ko);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                *(f4*)&sA[0][(lrow + 32 * i) * kLDK + lcol] = va[i];
                *(f4*)&sB[0][(lrow + 32 * i) * kLDK + lcol] = vb[i];
            }
        }
        __syncthreads();
        int cur = 0;
        for (int s = s_begin; s < s_end; ++s) {
            const bool more = s + 1 < s_end;
            if (more) {
                const int64_t ko = (int64_t)(s + 1) * kBK;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    va[i] = *(const f4*)(pa[i] + ko);
                    vb[i] = *(const f4*)(pb[i] + ko);
                }
            }
            const float* a_base = &sA[cur][(wm + r16) * kLDK + g4];
            const float* b_base = &sB[cur][(wn + r16) * kLDK + g4];
#pragma unroll
            for (int kk = 0; kk < kBK; kk += 16) {
                f4 af[4], bf[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) af[i] = *(const f4*)(a_base + i * 16 * kLDK + kk);
#pragma unroll
                for (int j = 0; j < 4; ++j) bf[j] = *(const f4*)(b_base + j * 16 * kLDK + kk);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][q], bf[j][q],
                                                                             acc[i][j], 0, 0, 0);
            }
            if (more) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    *(f4*)&sA[cur ^ 1][(lrow + 32 * i) * kLDK + lcol] = va[i];
                    *(f4*)&sB[cur ^ 1][(lrow + 32 * i) * kLDK + lcol] = vb[i];
                }
            }
            __syncthreads();
            cur ^= 1;
        }
    }

    const int tile = tile_m + tile_n * g.tilesM;
    if (EPI == EPI_PARTIAL) {
        f4* P = (f4*)(g.P + ((int64_t)split * g.tilesM * g.tilesN + tile) * (kBM * kBN));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) P[(i * 4 + j) * kThreads + tid] = acc[i][j];
        return;
    }

    double nv[2] = {0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + wm + 16 * i + g4;
            const int n = n0 + wn + 16 * j + r16;
            if (n >= g.N || m >= g.M) continue;
            f4 v = acc[i][j];
            float* c = g.C + (int64_t)n * g.ldc + m;
            if (EPI == EPI_GRAD) {
                v = v * g.alpha;
            } else {
                f4 w = f4{0.f, 0.f, 0.f, 0.f};
                if (g.Wprev) {
                    const float* wp = g.Wprev + (int64_t)n * g.ldc + m;
                    if (g.vec_store && m + 3 < g.M) {
                        w = *(const f4*)wp;
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r) w[r] = (m + r < g.M) ? wp[r] : 0.f;
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
            if (g.vec_store && m + 3 < g.M) {
                *(f4*)c = v;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (m + r < g.M) c[r] = v[r];
            }
        }
    }
    if (EPI == EPI_TRIAL) {
        block_sum<2>(nv);
        if (tid == 0) {
            g.norm_part[(int64_t)tile * kNormCols + 0] = nv[0];
            g.norm_part[(int64_t)tile * kNormCols + 1] = nv[1];
        }
    }
}

// Fixed-order sum of the split-K partial tiles, then the trial epilogue.
// One workgroup per tile; thread t owns the same accumulator slots it had in
// k_gemm_f32, so (m, n) follow from (t, i, j) exactly as there.
__global__ void __launch_bounds__(kThreads) k_splitk_reduce(GemmArgs g) {
    if (g.ls) {
        if (g.pred >= 1 && g.ls->converged) return;
        if (g.pred >= 2 && g.ls->done) return;
    }
    const int tile = blockIdx.x;
    const int tile_m = tile % g.tilesM, tile_n = tile / g.tilesM;
    const int m0 = tile_m * kBM, n0 = tile_n * kBN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int r16 = lane & 15, g4 = (lane >> 4) * 4;
    const int64_t tiles = (int64_t)g.tilesM * g.tilesN;
    double nv[2] = {0.0, 0.0};
#pragma unroll 1
    for (int idx = 0; idx < 16; ++idx) {
        const int i = idx >> 2, j = idx & 3;
        const int m = m0 + wm + 16 * i + g4;
        const int n = n0 + wn + 16 * j + r16;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        for (int s = 0; s < g.splits; ++s) {
            const f4* P = (const f4*)(g.P + ((int64_t)s * tiles + tile) * (kBM * kBN));
            v += P[idx * kThreads + tid];
        }
        if (n >= g.N || m >= g.M) continue;
        float* c = g.C + (int64_t)n * g.ldc + m;
        f4 w = f4{0.f, 0.f, 0.f, 0.f};
        if (g.Wprev) {
            const float* wp = g.Wprev + (int64_t)n * g.ldc + m;
            if (g.vec_store && m + 3 < g.M) {
                w = *(const f4*)wp;
            } else {
                for (int r = 0; r < 4; ++r) w[r] = (m + r < g.M) ? wp[r] : 0.f;
            }
        }
        const f4 out = w + v;
        for (int r = 0; r < 4; ++r) {
            if (m + r < g.Mvalid && n < g.Nvalid) {
                nv[0] += (double)v[r] * (double)v[r];
                nv[1] += (double)out[r] * (double)out[r];
            }
        }
        if (g.vec_store && m + 3 < g.M) {
            *(f4*)c = out;
        } else {
            for (int r = 0; r < 4; ++r)
                if (m + r < g.M) c[r] = out[r];
        }
    }
    block_sum<2>(nv);
    if (tid == 0) {
        g.norm_part[(int64_t)tile * kNormCols + 0] = nv[0];
        g.norm_part[(int64_t)tile * kNormCols + 1] = nv[1];
    }
}

void launch_gemm(const GemmArgs& a, int epi, hipStream_t st) {
    const unsigned blocks = (unsigned)((int64_t)a.tilesM * a.tilesN * a.splits);
    if (epi == EPI_GRAD)
        k_gemm_f32<EPI_GRAD><<<blocks, kThreads, 0, st>>>(a);
    else if (epi == EPI_TRIAL)
        k_gemm_f32<EPI_TRIAL><<<blocks, kThreads, 0, st>>>(a);
    else
        k_gemm_f32<EPI_PARTIAL><<<blocks, kThreads, 0, st>>>(a);
}

void launch_splitk_reduce(const GemmArgs& a, hipStream_t st) {
    const unsigned blocks = (unsigned)((int64_t)a.tilesM * a.tilesN);
    k_splitk_reduce<<<blocks, kThreads, 0, st>>>(a);
}

// ---------------------------------------------------------------------------
// Fused prox (eq. 3.5) + line-search partial sums.
//
// Streams Omega and G once (16-byte loads), writes Omega+ and Delta, and keeps
// per-thread FP64 sums of ||Delta||^2, <Delta, G>, ||Omega+||_1, sum log Omega+_jj,
// the off-diagonal nonzero count and ||Omega+||_F^2.  Off-diagonal entries are
// soft-thresholded in FP32; the diagonal root is evaluated in FP64 in the
// cancellation-free form  b >= 0: (b + r)/2,  b < 0: 2 tau / (r - b),
// r = sqrt(b^2 + 4 tau), which equals (b + r)/2 exactly in real arithmetic.
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

__device__ inline void prox_account(ProxAcc& acc, float o, float gv, float nw, bool diag,
                                    bool valid, bool reduce_only) {
    if (!valid) return;
    if (!reduce_only) {
        const float dl = nw - o;
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

__global__ void __launch_bounds__(kThreads) k_prox(ProxArgs a) {
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

    int64_t q = q_begin + threadIdx.x;
    int64_t e = q << 2;
    int64_t col = e / a.ld, row = e - col * a.ld;
    for (; q < q_end; q += kThreads) {
        const f4 o = om4[q];
        const f4 gv = a.reduce_only ? f4{0.f, 0.f, 0.f, 0.f} : g4[q];
        f4 nw;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int64_t r = row + u, c = col;
            if (r >= a.ld) {
                r -= a.ld;
                c += 1;
            }
            const bool diag = (r == c);
            const bool valid = r < a.p;
            nw[u] = a.reduce_only ? o[u] : prox_one(o[u], gv[u], diag, tau, lam, tau_f, thr_f);
            prox_account(acc, o[u], gv[u], nw[u], diag, valid, a.reduce_only);
        }
        if (!a.reduce_only) {
            on4[q] = nw;
            if (d4) d4[q] = nw - o;
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
        const float nw = a.reduce_only ? o : prox_one(o, gv, diag, tau, lam, tau_f, thr_f);
        prox_account(acc, o, gv, nw, diag, r < a.p, a.reduce_only);
        if (!a.reduce_only) {
            a.om_new[ee] = nw;
            if (a.d) a.d[ee] = nw - o;
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
    k_prox<<<nblocks, kThreads, 0, st>>>(a);
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
__global__ void __launch_bounds__(kThreads) k_finalize(LsState* ls, const double* prox_part,
                                                       int nprox, const double* norm_part,
                                                       int ntiles, double* trace,
                                                       int32_t* trials_log) {
    if (ls->done || ls->converged) return;
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
    if (!finite) {
        ls->bad |= 2;
        ls->converged = 1;  // stop: every later launch is skipped
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
    }
}

void launch_finalize(LsState* ls, const double* prox_part, int nprox, const double* norm_part,
                     int ntiles, double* trace, int32_t* trials_log, hipStream_t st) {
    k_finalize<<<1, kThreads, 0, st>>>(ls, prox_part, nprox, norm_part, ntiles, trace,
                                       trials_log);
}

// Starting point: objective pieces of Omega^(0) (reduce-only prox sums of Omega^(0)
// and the norm sums of W0 = X Omega^(0)).
__global__ void __launch_bounds__(kThreads) k_fit_init(LsState* ls, const double* prox_part,
                                                       int nprox, const double* norm_part,
                                                       int ntiles, double* trace) {
    double pv[6];
    sum_partials<6>(prox_part, nprox, kPartCols, pv);
    double nv[2];
    sum_partials<2>(norm_part, ntiles, kNormCols, nv);
    if (threadIdx.x != 0) return;
    ls->g_cur = 0.5 * nv[1] * ls->inv_n;
    ls->h_cur = -pv[P_LOGD] + ls->lambda * pv[P_L1];
    ls->f_cur = ls->g_cur + ls->h_cur;
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
// Power iteration for L = sigma_max(X^T X / n):  v <- X^T (X v) / ||X^T (X v)||.
// The Rayleigh quotient ||X v||^2 / n of the last unit vector is L's estimate
// (it approaches sigma_max from below).  FP64 vectors, FP32 data.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_pow_start(double* w, int64_t p, LsState* ls) {
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < p;
         k += (int64_t)gridDim.x * kThreads) {
        // fixed pseudo-random signs (integer hash), unit-norm after scaling
        uint32_t h = (uint32_t)k * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        w[k] = (h & 1u) ? 1.0 : -1.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ls->pow_scale = 1.0 / sqrt((double)p);
}

// u = X (scale * w): one wave per sample row
__global__ void __launch_bounds__(kThreads) k_pow_xv(const float* __restrict__ Xp,
                                                     int64_t ldx, int64_t n, int64_t p,
                                                     const double* __restrict__ w,
                                                     double* __restrict__ u,
                                                     double* __restrict__ part_u,
                                                     const LsState* ls) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + wave;
    const double scale = ls->pow_scale;
    double s = 0.0;
    if (i < n) {
        const float* row = Xp + i * ldx;
        for (int64_t k = lane; k < p; k += 64) s += (double)row[k] * w[k];
        s = wave_sum(s) * scale;
        if (lane == 0) u[i] = s;
    }
    double v[1] = {(i < n && lane == 0) ? s * s : 0.0};
    block_sum<1>(v);
    if (threadIdx.x == 0) part_u[blockIdx.x] = v[0];
}

// w = X^T u: one wave per variable row of Xt
__global__ void __launch_bounds__(kThreads) k_pow_xtu(const float* __restrict__ Xt,
                                                      int64_t ldt, int64_t p, int64_t n,
                                                      const double* __restrict__ u,
                                                      double* __restrict__ w,
                                                      double* __restrict__ part_w) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * (kThreads / 64) + wave;
    double s = 0.0;
    if (j < p) {
        const float* row = Xt + j * ldt;
        for (int64_t k = lane; k < n; k += 64) s += (double)row[k] * u[k];
        s = wave_sum(s);
        if (lane == 0) w[j] = s;
    }
    double v[1] = {(j < p && lane == 0) ? s * s : 0.0};
    block_sum<1>(v);
    if (threadIdx.x == 0) part_w[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(kThreads) k_pow_norm(const double* part_w, int nbw,
                                                       const double* part_u, int nbu,
                                                       LsState* ls, int last) {
    double vw[1], vu[1];
    sum_partials<1>(part_w, nbw, 1, vw);
    sum_partials<1>(part_u, nbu, 1, vu);
    if (threadIdx.x != 0) return;
    ls->pow_rayleigh = vu[0] * ls->inv_n;
    ls->pow_scale = vw[0] > 0.0 ? 1.0 / sqrt(vw[0]) : 0.0;
    if (last) {
        ls->L = ls->pow_rayleigh;
        ls->inv_L = ls->L > 0.0 ? 1.0 / ls->L : 0.0;
    }
}

void launch_power_iteration(const float* Xp, int64_t p_pad, const float* Xt, int64_t n_pad,
                            int64_t n, int64_t p, double* w, double* u, double* part_u,
                            double* part_w, int steps, LsState* ls, hipStream_t st) {
    const int nbu = (int)cdiv(n, kThreads / 64);
    const int nbw = (int)cdiv(p, kThreads / 64);
    k_pow_start<<<(unsigned)(cdiv(p, kThreads) < 1024 ? cdiv(p, kThreads) : 1024), kThreads, 0,
                  st>>>(w, p, ls);
    for (int s = 0; s < steps; ++s) {
        k_pow_xv<<<nbu, kThreads, 0, st>>>(Xp, p_pad, n, p, w, u, part_u, ls);
        k_pow_xtu<<<nbw, kThreads, 0, st>>>(Xt, n_pad, p, n, u, w, part_w);
        k_pow_norm<<<1, kThreads, 0, st>>>(part_w, nbw, part_u, nbu, ls, s == steps - 1);
    }
}

}  // namespace accord
