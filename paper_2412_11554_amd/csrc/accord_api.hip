// Host side of the libaccord C ABI (declared in include/accord.h).
//
// Every entry point validates its arguments on the host before enqueuing work,
// carves the caller's workspace into the padded operand buffers, and enqueues
// the kernels of accord_kernels.hip on the caller's stream.
//
// accord_fit runs Alg. 1 with the backtracking loop predicated on the device:
// per iteration the host enqueues the gradient GEMM and the trials of tau0,
// beta tau0, ... (prox / trial product / acceptance) one trial ahead of the
// device, reading each trial's outcome from a pinned host mailbox; every kernel
// checks the device state first, so a trial enqueued after an acceptance does no
// work.  accord_fit_batch advances many independent fits in lockstep with the
// same kernels in batched form.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "accord.h"
#include "accord_internal.h"

using namespace accord;

namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ACCORD_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                               \
    } while (0)

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ---------------------------------------------------------------------------
// workspace layout (byte offsets, each region 256-byte aligned).  Regions are
// ordered so each entry point needs a prefix: prox < grad/objective < fit.
// ---------------------------------------------------------------------------
// tile grid of one GEMM launch
struct Geo {
    int tilesM, tilesN, splits;
    int tail_n0, tail_splits;  // fused trial product: split-K tail (choose_tail_splits)
    int tiles() const { return tilesM * tilesN; }
};

// rows of FP64 norm partials a trial product leaves (one per tile, or one per
// reduction workgroup when the bf16 split-K reduction runs)
bool is_bf16(int prec) { return prec == PREC_BF16X1 || prec == PREC_BF16X3; }

int norm_rows(const Geo& g, int prec) {
    return ((g.splits > 1 || g.tail_splits > 1) && prec != PREC_FP32) ? g.tiles() * kFReduceParts
                                                                       : g.tiles();
}

struct Plan {
    int64_t n, p, n_pad, p_pad;
    int64_t p_cols;  // columns allocated for Omega, G and Omega+ (>= p)
    int prec;
    // trial GEMM  (C = W^T:  M = n_pad, N = p, K = p_pad): FP32 geometry (setup
    // products and the FP32 form) and, for the bf16 forms, the fused prox + trial
    // kernel's geometry
    Geo t32, tp;
    int fused;      // bf16 and FP8 forms: the fused trial kernel's 256 x 128 geometry
    int fused32;    // FP32 form: prox fused into the 128 x 128 FP32 trial tile (else a
                    // separate prox pass writes Delta for the plain FP32 GEMM)
    int probe;      // fused forms with >= 4 M tiles: a trial can be rejected from its
                    // first M tile (params.probe)
    int staged;     // probing, and one M tile's launch fills the CUs: the other M tiles
                    // run one launch each, with a partial test after each
    int prox_rows;  // FP64 prox partial rows left per trial
    int nprox;
    size_t off_ls, off_prox_part, off_norm_part, off_lz,
        off_trials, off_xp, off_xt, off_xsplit[4], off_x8, off_x8s, off_xt8, off_xt8s, off_wt0,
        off_wt1, off_wsplit[4], off_w8, off_w8s, off_split,
        off_om0, end_grad, off_g, off_d, off_om1, end_fit;
    size_t off_mask, end_refit;  // refit: support bytes in the padded layout of Omega
    // refit, fused forms: which blocks hold support entries (32-row K steps of each
    // 128-column block), the K-step lists of the trial kernels (CSR) and the occupied
    // 256 x 256 tiles of the gradient
    size_t off_occ, off_kptr, off_kidx, off_gocc;
    int ks32, gbm, gbn, tilesMg, tilesNg;
    size_t end_prox;
};

size_t bump(size_t& cur, size_t bytes) {
    size_t at = cur;
    cur = (size_t)round_up((int64_t)(cur + bytes), 256);
    return at;
}

int choose_splits(int tiles, int ksteps64, int slots) {
    // pick S minimising (rounds of resident workgroups) / S; keep >= 2 steps of 64
    int best = 1;
    double best_cost = (double)cdiv(tiles, slots);
    for (int s = 2; s <= 8; ++s) {
        if (ksteps64 / s < 2) break;
        const double cost = (double)cdiv((int64_t)tiles * s, slots) / s;
        if (cost < best_cost * 0.9) {
            best = s;
            best_cost = cost;
        }
    }
    return best;
}

// Split count of the fused trial product when its trials are probed (>= 4 M tiles): a
// trial is one launch over M tile 0 (tilesN workgroups per split), then, for about every
// other trial, one over the other M tiles.  When the probe launch alone fills the CUs
// (tilesN >= slots) the product is not split: measured at n = 1000, p = 1e5 (782 column
// blocks), two splits moved the BF16x3 probe from 24.9 to 24.2 ms and left the rest at
// 60.1 ms, while the BF16x1 launches took 15% longer (a split's K steps ran slower).
// Otherwise, with every workgroup of a launch doing the same work, a launch takes
// ceil(workgroups / slots) rounds of 1 / S of the unsplit time, and weighting the probe
// launch twice (it runs for every trial) S minimises
//   (2 ceil(tilesN S / slots) + ceil((tilesM - 1) tilesN S / slots)) / S  (1 + 0.03 (S - 1)),
// the last factor a charge for the split-K reduce and the shorter K loops; S = 1 .. 4,
// at least 2 K steps of 64 per split, a larger S only for a 1% lower cost (n = 800,
// p = 8192: 64 column blocks, S = 4).
int choose_probe_splits(int tilesM, int tilesN, int ksteps64, int slots) {
    if (tilesN >= slots) return 1;
    int best = 1;
    double best_cost = 0.0;
    for (int s = 1; s <= 4; ++s) {
        if (s > 1 && ksteps64 / s < 2) break;
        const double rounds = 2.0 * (double)cdiv((int64_t)tilesN * s, slots) +
                              (double)cdiv((int64_t)(tilesM - 1) * tilesN * s, slots);
        const double cost = rounds / s * (1.0 + 0.03 * (s - 1));
        if (s == 1 || cost < 0.99 * best_cost) {  // near ties keep the smaller S
            best = s;
            best_cost = cost;
        }
    }
    return best;
}

// Split-K tail of a trial product.  Its workgroups all run the same K loop (one per CU in
// the fused bf16 / fp8 kernels, two in the FP32 GEMM), so a launch takes whole rounds of
// slots workgroups.  With tilesN = F + T column blocks, F the largest multiple of `unit`
// (the blocks for which every launch of the product is a whole number of rounds: slots
// when trials are probed, since the launches then cover one M tile, else
// slots / gcd(slots, tilesM)), the last T blocks add a round in which most CUs idle.
// Measured at n = 1000, p = 1e5 (782 blocks) in BF16x3: over 768 blocks instead of 782
// the probe took 19.1 instead of 25.2 ms, the rest of a trial 57.5 instead of 60.6 ms
// and the whole product 68.9 instead of 75.2 ms.  So the last T blocks run as a launch
// of their own, split S ways along K and reduced, in every launch of the product (the
// same S, so a column block sums its products in the same order whichever launch covers
// it).  S in {2, 4, 8, 16} minimises the tail's rounds, ceil(m T S / slots) / S
// (1 + 0.03 (S - 1)), over the launches that cover m = 1 (three times: the probe and the
// partial-test stages) and tilesM M tiles when trials are probed, else tilesM, with at
// least 8 K steps of 64 per split; 0 (no tail launch) unless that beats the unsplit tail
// by 10%.  *tail_n0 = F.
int choose_tail_splits(int tilesM, int tilesN, int ksteps64, int slots, bool probe,
                       int* tail_n0) {
    *tail_n0 = 0;
    const int unit = probe ? slots : slots / std::gcd(slots, tilesM);
    const int F = tilesN / unit * unit, T = tilesN - F;
    if (F == 0 || T == 0) return 0;
    auto cost = [&](int S) {
        auto part = [&](int m) {
            return (double)cdiv((int64_t)m * T * S, slots) / S * (1.0 + 0.03 * (S - 1));
        };
        return probe ? 3.0 * part(1) + part(tilesM) : part(tilesM);
    };
    int best = 0;
    double best_cost = 0.9 * cost(1);
    for (int S = 2; S <= 16; S *= 2) {
        if (ksteps64 / S < 8) break;
        const double c = cost(S);
        if (c < best_cost) {
            best = S;
            best_cost = c;
        }
    }
    if (best > 1) *tail_n0 = F;
    return best;
}

Plan make_plan(int64_t n, int64_t p, int32_t max_iter, int prec) {
    Plan P = {};
    P.n = n;
    P.p = p;
    P.prec = prec;
    P.n_pad = round_up(n, kPad);
    P.p_pad = round_up(p, kPad);
    P.t32.tilesM = (int)cdiv(P.n_pad, kBM);
    P.t32.tilesN = (int)cdiv(p, kBN);
    P.t32.splits = choose_splits(P.t32.tiles(), (int)(P.p_pad / kPad), kSlots);
    P.fused = prec != PREC_FP32;
    if (!P.fused) {
        P.tp = P.t32;
    } else {
        P.tp.tilesM = (int)cdiv(P.n_pad, kFBM);
        P.tp.tilesN = (int)cdiv(p, kFBN);
        P.tp.splits = P.tp.tilesM >= 4
                          ? choose_probe_splits(P.tp.tilesM, P.tp.tilesN, (int)(P.p_pad / kPad),
                                                kWSlots)
                          : choose_splits(P.tp.tiles(), (int)(P.p_pad / kPad), kWSlots);
        if (P.tp.splits == 1)
            P.tp.tail_splits = choose_tail_splits(P.tp.tilesM, P.tp.tilesN, (int)(P.p_pad / kPad),
                                                  kWSlots, P.tp.tilesM >= 4, &P.tp.tail_n0);
    }
    P.nprox = prox_blocks(p * P.p_pad);
    // every form's fit runs the prox inside its trial kernel: one row of prox sums per
    // (column block, split)
    // The FP32 fused kernel recomputes the prox in each of the tilesM row tiles of a
    // column block, while it saves one 16 B-per-entry prox pass.  Measured: faster at
    // n = 500 (4 row tiles: 300 us against 287 + 77 us at p = 5000), slower at n = 1000
    // (8 row tiles: 218 ms against 152 + 33 ms at p = 1e5).  So it runs up to 4 row tiles.
    P.fused32 = !P.fused && P.t32.tilesM <= 4;
    // the plain FP32 trial GEMM (and the FP32 set-up product W0 = X Omega0 of every form)
    if (!P.fused32 && P.t32.splits == 1)
        P.t32.tail_splits = choose_tail_splits(P.t32.tilesM, P.t32.tilesN, (int)(P.p_pad / kPad),
                                               kSlots, false, &P.t32.tail_n0);
    // A probe (M tile 0, a quarter of the samples or less) rejects a trial whose test
    // fails by more than the inverse of its share of the rows; with fewer M tiles the
    // probe is a large share of the product and cannot reject the near misses.
    P.probe = P.fused && P.tp.tilesM >= 4;
    // Staged partial tests: after M tile 0 the trial goes on one M tile at a time, with the
    // test of the lower bound after each, while one M tile's launch fills the CUs (at
    // n = 1000, p = 1e5 a launch over one M tile took 19.3 ms and one over three 58.2 ms:
    // the same time per M tile).  A trial whose ratio lies between 2 and 4 is then rejected
    // after two M tiles instead of after the whole product.
    P.staged = P.probe && ((int64_t)P.tp.tilesN * P.tp.splits >= kWSlots);
    P.prox_rows = P.fused ? P.tp.tilesN * (P.tp.tail_splits > 1 ? P.tp.tail_splits : P.tp.splits)
                          : (P.fused32 ? P.t32.tilesN * P.t32.splits : P.nprox);
    const bool bf = is_bf16(prec);
    const bool f8 = prec == PREC_FP8;
    const int ttiles = std::max(norm_rows(P.t32, PREC_FP32), norm_rows(P.tp, prec));
    const size_t split_floats =
        std::max((size_t)(P.t32.splits > 1 ? P.t32.splits : 0) * P.t32.tiles() * kBM * kBN,
                 (size_t)(P.tp.splits > 1 ? P.tp.splits : 0) * P.tp.tiles() * kFBM * kFBN *
                     (P.fused ? 1 : 0));
    const size_t tail_floats = std::max(
        (size_t)(P.tp.tail_splits > 1 ? P.tp.tail_splits : 0) * P.tp.tilesM *
            (P.tp.tilesN - P.tp.tail_n0) * kFBM * kFBN,
        (size_t)(P.t32.tail_splits > 1 ? P.t32.tail_splits : 0) * P.t32.tilesM *
            (P.t32.tilesN - P.t32.tail_n0) * kBM * kBN);
    const size_t xn = (size_t)(P.n_pad * P.p_pad);   // padded X elements
    const size_t wn = (size_t)(p * P.n_pad);         // W^T elements
    const size_t on = (size_t)(p * P.p_pad);         // p x p_pad elements
    // the fused trial kernels read and write whole 128-column blocks of Omega, G and
    // Omega+: their buffers carry zero padding columns up to tilesN * 128
    P.p_cols = P.fused ? round_up(p, kFBN) : p;
    const size_t onc = (size_t)(P.p_cols * P.p_pad);
    size_t cur = 0;
    P.off_ls = bump(cur, sizeof(LsState));
    P.off_prox_part = bump(cur, (size_t)std::max(kMaxProxBlocks, P.prox_rows) * kPartCols *
                                    sizeof(double));
    P.end_prox = cur;
    P.off_norm_part = bump(cur, (size_t)ttiles * kNormCols * sizeof(double));
    P.off_lz = bump(cur, lz_buf_bytes(P.n_pad, P.p_pad));
    P.off_trials = bump(cur, (size_t)(max_iter > 0 ? max_iter : 1) * sizeof(int32_t));
    P.off_xp = bump(cur, xn * sizeof(float));
    P.off_xt = bump(cur, xn * sizeof(float));
    for (int k = 0; k < 4; ++k) P.off_xsplit[k] = bump(cur, bf ? xn * sizeof(uint16_t) : 0);
    P.off_x8 = bump(cur, f8 ? xn : 0);
    P.off_x8s = bump(cur, f8 ? xn / 32 : 0);
    P.off_xt8 = bump(cur, f8 ? xn : 0);
    P.off_xt8s = bump(cur, f8 ? xn / 32 : 0);
    P.off_wt0 = bump(cur, wn * sizeof(float));
    P.off_wt1 = bump(cur, wn * sizeof(float));
    for (int k = 0; k < 4; ++k) P.off_wsplit[k] = bump(cur, bf ? wn * sizeof(uint16_t) : 0);
    P.off_w8 = bump(cur, f8 ? wn : 0);
    P.off_w8s = bump(cur, f8 ? wn / 32 : 0);
    P.off_split = bump(cur, std::max(split_floats, tail_floats) * sizeof(float));
    P.off_om0 = bump(cur, onc * sizeof(float));
    P.end_grad = cur;
    P.off_g = bump(cur, onc * sizeof(float));
    P.off_d = bump(cur, P.fused ? 0 : on * sizeof(float));  // fused forms never store Delta
    P.off_om1 = bump(cur, onc * sizeof(float));
    P.end_fit = cur;
    P.off_mask = bump(cur, on);
    P.ks32 = (int)(P.p_pad / 32);
    P.gbm = prec == PREC_FP32 ? kBM : kWBM;  // gradient tile (G rows x columns)
    P.gbn = prec == PREC_FP32 ? kBN : kWBN;
    P.tilesMg = (int)cdiv(P.p_pad, P.gbm);
    P.tilesNg = (int)cdiv(p, P.gbn);
    P.off_occ = bump(cur, (size_t)P.tp.tilesN * P.ks32);
    P.off_kptr = bump(cur, (size_t)(P.tp.tilesN + 1) * sizeof(int32_t));
    P.off_kidx = bump(cur, (size_t)P.tp.tilesN * P.ks32 * sizeof(int32_t));
    P.off_gocc = bump(cur, (size_t)P.tilesMg * P.tilesNg);
    P.end_refit = cur;
    return P;
}

template <typename T>
T* at(void* ws, size_t off) {
    return (T*)((char*)ws + off);
}

// trial GEMM: Wt_out = Wt_prev + (X B)^T, W^T layout p x n_pad.  prec selects the
// operands: FP32 (Xp, B32) or bf16 splits (Xp hi/lo, Bh/Bl).  wslot >= 0 also writes
// the bf16 split of the result into W split slot wslot.
GemmArgs trial_args(const Plan& P, void* ws, int prec, const float* B32, const uint16_t* Bh,
                    const uint16_t* Bl, const float* Wprev, float* Wout, int wslot, LsState* ls,
                    int pred) {
    GemmArgs a = {};
    a.A = at<float>(ws, P.off_xp);
    a.B = B32;
    if (is_bf16(prec)) {
        a.Ah = at<uint16_t>(ws, P.off_xsplit[0]);
        a.Al = at<uint16_t>(ws, P.off_xsplit[1]);
        a.Bh = Bh;
        a.Bl = Bl;
    } else if (prec == PREC_FP8) {
        a.A8 = at<uint8_t>(ws, P.off_x8);
        a.As = at<uint8_t>(ws, P.off_x8s);
        a.ldas = P.p_pad / 32;
    }
    a.lda = P.p_pad;
    a.ldb = P.p_pad;
    a.M = (int)P.n_pad;
    a.N = (int)P.p;
    a.K = (int)P.p_pad;
    const Geo& geo = prec == PREC_FP32 ? P.t32 : P.tp;
    a.tilesM = geo.tilesM;
    a.tilesN = geo.tilesN;
    a.splits = geo.splits;
    a.C = Wout;
    if (wslot >= 0) {
        a.Ch = at<uint16_t>(ws, P.off_wsplit[2 * wslot]);
        a.Cl = at<uint16_t>(ws, P.off_wsplit[2 * wslot + 1]);
    }
    a.ldc = P.n_pad;
    a.vec_store = 1;
    a.alpha = 1.f;
    a.Wprev = Wprev;
    a.tail_n0 = geo.tail_n0;
    a.tail_splits = geo.tail_splits;
    a.P = (geo.splits > 1 || geo.tail_splits > 1) ? at<float>(ws, P.off_split) : nullptr;
    a.norm_part = at<double>(ws, P.off_norm_part);
    a.ls = ls;
    a.pred = pred;
    a.Mvalid = (int)P.n;
    a.Nvalid = (int)P.p;
    return a;
}

void enqueue_trial(const GemmArgs& a, int prec, hipStream_t st) {
    if (a.splits == 1 && a.tail_splits > 1 && a.tail_n0 > 0 && a.tail_n0 < a.tilesN) {
        // the column blocks before tail_n0 unsplit, then the split-K tail and its reduce
        // (see choose_tail_splits)
        GemmArgs f = a, t = a;
        f.tail_splits = t.tail_splits = 0;
        f.n_count = a.tail_n0;
        t.n_first = a.tail_n0;
        t.n_count = a.tilesN - a.tail_n0;
        t.splits = a.tail_splits;
        enqueue_trial(f, prec, st);
        enqueue_trial(t, prec, st);
        return;
    }
    if (a.splits > 1) {
        launch_gemm(a, EPI_PARTIAL, prec, st);
        launch_splitk_reduce(a, st);
    } else {
        launch_gemm(a, EPI_TRIAL, prec, st);
    }
}

// gradient GEMM: C = Xt * Wt^T / n  (M = p_pad or p rows of C, N = p); bf16 forms
// read the split of W^T from slot wslot
GemmArgs grad_args(const Plan& P, void* ws, int prec, const float* Wt, int wslot, float* C,
                   int64_t ldc, int M, LsState* ls) {
    GemmArgs a = {};
    a.A = at<float>(ws, P.off_xt);
    a.B = Wt;
    if (is_bf16(prec)) {
        a.Ah = at<uint16_t>(ws, P.off_xsplit[2]);
        a.Al = at<uint16_t>(ws, P.off_xsplit[3]);
        a.Bh = at<uint16_t>(ws, P.off_wsplit[2 * wslot]);
        a.Bl = at<uint16_t>(ws, P.off_wsplit[2 * wslot + 1]);
    } else if (prec == PREC_FP8) {
        a.A8 = at<uint8_t>(ws, P.off_xt8);
        a.As = at<uint8_t>(ws, P.off_xt8s);
        a.B8 = at<uint8_t>(ws, P.off_w8);
        a.Bs = at<uint8_t>(ws, P.off_w8s);
        a.ldas = P.n_pad / 32;
        a.ldbs = P.n_pad / 32;
    }
    a.lda = P.n_pad;
    a.ldb = P.n_pad;
    a.M = M;
    a.N = (int)P.p;
    a.K = (int)P.n_pad;
    const int bm = prec == PREC_FP32 ? kBM : kWBM, bn = prec == PREC_FP32 ? kBN : kWBN;
    a.tilesM = (int)cdiv(M, bm);
    a.tilesN = (int)cdiv(P.p, bn);
    a.splits = 1;
    a.C = C;
    a.ldc = ldc;
    a.vec_store = (ldc % 4 == 0) && aligned(C, 16);
    a.alpha = (float)(1.0 / (double)P.n);
    a.ls = ls;
    a.pred = ls ? 1 : 0;
    a.begin_iter = ls ? 1 : 0;
    return a;
}

XSplit x_split(const Plan& P, void* ws) {
    XSplit sp = {};
    if (is_bf16(P.prec)) {
        sp.xp_h = at<uint16_t>(ws, P.off_xsplit[0]);
        sp.xp_l = at<uint16_t>(ws, P.off_xsplit[1]);
        sp.xt_h = at<uint16_t>(ws, P.off_xsplit[2]);
        sp.xt_l = at<uint16_t>(ws, P.off_xsplit[3]);
    }
    return sp;
}

int check_dims(int64_t n, int64_t p) {
    if (n < 1 || p < 1) return fail(ACCORD_ERR_INVALID_ARG, "n and p must be >= 1 (n=%lld p=%lld)",
                                    (long long)n, (long long)p);
    // GEMM tile counts (x split-K factor) are 32-bit; 2^20 keeps them below 2^31
    if (n > (1LL << 20) || p > (1LL << 20))
        return fail(ACCORD_ERR_INVALID_ARG, "n or p too large (n=%lld p=%lld)", (long long)n,
                    (long long)p);
    return ACCORD_OK;
}

int check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (!ws) return fail(ACCORD_ERR_WORKSPACE, "workspace pointer is null");
    if (!aligned(ws, 256)) return fail(ACCORD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(ACCORD_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    return ACCORD_OK;
}

int check_ptr(const void* p, const char* name) {
    if (!p) return fail(ACCORD_ERR_INVALID_ARG, "%s is null", name);
    if (!aligned(p, 16)) return fail(ACCORD_ERR_INVALID_ARG, "%s must be 16-byte aligned", name);
    return ACCORD_OK;
}

#define TRY(expr)                    \
    do {                             \
        int s_ = (expr);             \
        if (s_ != ACCORD_OK) return s_; \
    } while (0)

int check_params(const accord_params* prm) {
    if (!prm) return fail(ACCORD_ERR_INVALID_ARG, "params is null");
    if (!(prm->lambda >= 0.0) || !isfinite(prm->lambda))
        return fail(ACCORD_ERR_INVALID_ARG, "lambda must be finite and >= 0");
    if (!(prm->tau0 > 0.0) || !isfinite(prm->tau0))
        return fail(ACCORD_ERR_INVALID_ARG, "tau0 must be finite and > 0");
    if (!(prm->beta > 0.0 && prm->beta <= 1.0))
        return fail(ACCORD_ERR_INVALID_ARG, "beta must lie in (0, 1]");
    if (!(prm->lipschitz >= 0.0) || !isfinite(prm->lipschitz))
        return fail(ACCORD_ERR_INVALID_ARG, "lipschitz must be finite and >= 0");
    if (!(prm->tol >= 0.0) || !isfinite(prm->tol))
        return fail(ACCORD_ERR_INVALID_ARG, "tol must be finite and >= 0");
    if (prm->max_iter < 0) return fail(ACCORD_ERR_INVALID_ARG, "max_iter must be >= 0");
    if (prm->precision != ACCORD_FP32 && prm->precision != ACCORD_BF16X1 &&
        prm->precision != ACCORD_BF16X3 && prm->precision != ACCORD_FP8)
        return fail(ACCORD_ERR_UNSUPPORTED, "precision form %d is not available", prm->precision);
    if (prm->power_iters < 0) return fail(ACCORD_ERR_INVALID_ARG, "power_iters must be >= 0");
    if (prm->timing < 0) return fail(ACCORD_ERR_INVALID_ARG, "timing must be >= 0");
    if (prm->warm_tau != 0 && prm->warm_tau != 1)
        return fail(ACCORD_ERR_INVALID_ARG, "warm_tau must be 0 or 1");
    if (prm->graph != 0 && prm->graph != 1)
        return fail(ACCORD_ERR_INVALID_ARG, "graph must be 0 or 1");
    if (prm->refresh_every < 0) return fail(ACCORD_ERR_INVALID_ARG, "refresh_every must be >= 0");
    if (prm->probe != 0 && prm->probe != 1)
        return fail(ACCORD_ERR_INVALID_ARG, "probe must be 0 or 1");
    if (prm->support_skip != 0 && prm->support_skip != 1)
        return fail(ACCORD_ERR_INVALID_ARG, "support_skip must be 0 or 1");
    if (prm->batch_order < 0) return fail(ACCORD_ERR_INVALID_ARG, "batch_order must be >= 0");
    return ACCORD_OK;
}

// number of trials Alg. 1 can need: tau0, beta*tau0, ... up to the first tau <= 1/L,
// evaluated with the same double arithmetic as the device (tau *= beta).
int max_trials(double tau0, double beta, double inv_L) {
    if (beta >= 1.0) return 1;
    int k = 1;
    double tau = tau0;
    while (!(tau <= inv_L) && k < 200) {
        tau *= beta;
        ++k;
    }
    return k;
}

// Pinned host mailbox of the calling thread (allocated once per thread and kept:
// accord_fit is synchronous, so one thread never runs two fits at once).
Mailbox* host_mailbox(Mailbox** dev) {
    thread_local Mailbox* host = nullptr;
    thread_local Mailbox* device = nullptr;
    if (!host) {
        void* h = nullptr;
        if (hipHostMalloc(&h, sizeof(Mailbox), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess)
            return nullptr;
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) return nullptr;
        host = (Mailbox*)h;
        device = (Mailbox*)d;
    }
    *dev = device;
    return host;
}

// one snapshot of the device's mailbox word
struct Posted {
    int32_t trials, iter;
    bool stop;
};
Posted read_mailbox(const Mailbox* mb) {
    const uint64_t w = __atomic_load_n(&mb->word, __ATOMIC_ACQUIRE);
    return {(int32_t)(uint32_t)(w & 0xffffffffu), (int32_t)((w >> 32) & 0x7fffffffu),
            (w >> 63) != 0};
}

// HIP events for params.timing.  A fit records two per sampled launch group (thousands
// per fit with timing = 1); rather than creating and destroying them in every call,
// they are kept per thread and device and reused by later calls (a call is
// synchronous: its events have completed and been read before it returns).
struct EventPool {
    std::vector<hipEvent_t>* ev = nullptr;
    size_t used = 0;
    EventPool() {
        static thread_local std::map<int, std::vector<hipEvent_t>> cache;
        int dev = 0;
        (void)hipGetDevice(&dev);
        ev = &cache[dev];
    }
    hipEvent_t get() {
        if (used == ev->size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev->push_back(e);
        }
        return (*ev)[used++];
    }
};

}  // namespace

extern "C" {

void accord_default_params(accord_params* prm) {
    if (!prm) return;
    memset(prm, 0, sizeof *prm);
    prm->lambda = 0.1;
    prm->tau0 = 1.0;
    prm->beta = 0.5;
    prm->lipschitz = 0.0;
    prm->tol = 0.0;
    prm->max_iter = 100;
    prm->precision = ACCORD_FP32;
    prm->power_iters = kLzDefaultSteps;
    prm->timing = 0;
    prm->probe = 1;
    prm->support_skip = 1;
}

size_t accord_workspace_bytes(int64_t n, int64_t p, const accord_params* prm) {
    if (n < 1 || p < 1 || n > (1LL << 24) || p > (1LL << 24)) return 0;
    accord_params d;
    if (!prm) {
        accord_default_params(&d);
        prm = &d;
    }
    return make_plan(n, p, prm->max_iter, prm->precision).end_fit;
}

const char* accord_status_str(int s) {
    switch (s) {
        case ACCORD_OK: return "ok";
        case ACCORD_ERR_INVALID_ARG: return "invalid argument";
        case ACCORD_ERR_DOMAIN: return "diagonal of Omega must be positive";
        case ACCORD_ERR_NONFINITE: return "non-finite value";
        case ACCORD_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case ACCORD_ERR_UNSUPPORTED: return "unsupported";
        case ACCORD_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* accord_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

// arguments of accord_prox and accord_prox_noalloc (everything but the workspace)
int check_prox_args(const float* Omega, const float* G, int64_t p, double tau, double lambda,
                    const float* Omega_out, const double* red) {
    TRY(check_dims(1, p));
    TRY(check_ptr(Omega, "Omega"));
    TRY(check_ptr(G, "G"));
    TRY(check_ptr(Omega_out, "Omega_out"));
    if (!red || !aligned(red, 8)) return fail(ACCORD_ERR_INVALID_ARG, "red must be non-null, 8-byte aligned");
    if (Omega_out == Omega || Omega_out == G)
        return fail(ACCORD_ERR_INVALID_ARG, "Omega_out must not alias Omega or G");
    if (!(tau > 0.0) || !isfinite(tau)) return fail(ACCORD_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (!(lambda >= 0.0) || !isfinite(lambda))
        return fail(ACCORD_ERR_INVALID_ARG, "lambda must be finite and >= 0");
    return ACCORD_OK;
}

// the prox pass and the fixed-order combine of its FP64 partial sums (one row of
// kPartCols per workgroup) into red
int enqueue_prox(const float* Omega, const float* G, int64_t p, double tau, double lambda,
                 float* Omega_out, double* red, double* part, hipStream_t st) {
    ProxArgs a = {};
    a.om = Omega;
    a.g = G;
    a.om_new = Omega_out;
    a.d = nullptr;
    a.total = p * p;
    a.ld = p;
    a.p = p;
    a.tau = tau;
    a.lambda = lambda;
    a.part = part;
    const int nb = prox_blocks(a.total);
    launch_prox(a, nb, st);
    launch_combine_prox(a.part, nb, red, st);
    HIP_TRY(hipGetLastError());
    return ACCORD_OK;
}

}  // namespace

extern "C" {

int accord_prox(const float* Omega, const float* G, int64_t p, double tau, double lambda,
                float* Omega_out, double* red, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    TRY(check_prox_args(Omega, G, p, tau, lambda, Omega_out, red));
    const Plan P = make_plan(1, p, 1, PREC_FP32);
    TRY(check_ws(ws, ws_bytes, P.end_prox));
    return enqueue_prox(Omega, G, p, tau, lambda, Omega_out, red,
                        at<double>(ws, P.off_prox_part), (hipStream_t)stream);
}

// shared by accord_grad and accord_objective: X -> padded copies, Omega -> Om0,
// Wt0 = (X Omega)^T with norm partials
static int enqueue_w(const Plan& P, const float* X, const float* Omega, void* ws, hipStream_t st) {
    LsState* ls = at<LsState>(ws, P.off_ls);
    launch_init_state(ls, 1.0, 0.5, 0.0, 0.0, 1.0 / (double)P.n, 0.0, 0, st);
    launch_pad_x(X, P.n, P.p, at<float>(ws, P.off_xp), P.p_pad, at<float>(ws, P.off_xt), P.n_pad,
                 x_split(P, ws), ls, st);
    float* om0 = at<float>(ws, P.off_om0);
    launch_copy_cols(Omega, P.p, om0, P.p_pad, P.p, P.p_pad, nullptr, st);
    GemmArgs t = trial_args(P, ws, PREC_FP32, om0, nullptr, nullptr, nullptr,
                            at<float>(ws, P.off_wt0), -1, nullptr, 0);
    enqueue_trial(t, PREC_FP32, st);
    return ACCORD_OK;
}

int accord_grad(const float* X, int64_t n, int64_t p, const float* Omega, float* W, float* G,
                void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    TRY(check_dims(n, p));
    TRY(check_ptr(X, "X"));
    TRY(check_ptr(Omega, "Omega"));
    TRY(check_ptr(G, "G"));
    if (W) TRY(check_ptr(W, "W"));
    const Plan P = make_plan(n, p, 1, PREC_FP32);
    TRY(check_ws(ws, ws_bytes, P.end_grad));
    hipStream_t st = (hipStream_t)stream;
    TRY(enqueue_w(P, X, Omega, ws, st));
    const float* wt = at<float>(ws, P.off_wt0);
    if (W) launch_transpose_w(wt, P.n_pad, n, p, W, st);
    GemmArgs g = grad_args(P, ws, PREC_FP32, wt, 0, G, p, (int)p, nullptr);
    launch_gemm(g, EPI_GRAD, PREC_FP32, st);
    HIP_TRY(hipGetLastError());
    return ACCORD_OK;
}

int accord_objective(const float* X, int64_t n, int64_t p, const float* Omega, double lambda,
                     double* out, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    TRY(check_dims(n, p));
    TRY(check_ptr(X, "X"));
    TRY(check_ptr(Omega, "Omega"));
    if (!out || !aligned(out, 8)) return fail(ACCORD_ERR_INVALID_ARG, "out must be non-null, 8-byte aligned");
    if (!(lambda >= 0.0) || !isfinite(lambda))
        return fail(ACCORD_ERR_INVALID_ARG, "lambda must be finite and >= 0");
    const Plan P = make_plan(n, p, 1, PREC_FP32);
    TRY(check_ws(ws, ws_bytes, P.end_grad));
    hipStream_t st = (hipStream_t)stream;
    TRY(enqueue_w(P, X, Omega, ws, st));
    ProxArgs a = {};
    a.om = at<float>(ws, P.off_om0);
    a.total = p * P.p_pad;
    a.ld = P.p_pad;
    a.p = p;
    a.part = at<double>(ws, P.off_prox_part);
    a.reduce_only = 1;
    const int nb = prox_blocks(a.total);
    launch_prox(a, nb, st);
    launch_combine_objective(a.part, nb, at<double>(ws, P.off_norm_part),
                             P.t32.tiles(), lambda, 1.0 / (double)n, out, st);
    HIP_TRY(hipGetLastError());
    return ACCORD_OK;
}

// Refit in a fused form: find the blocks that can hold support entries (on the device),
// then build on the host the K-step list of every 128-column block at the trial kernel's
// step length (units32 32-row units per step) and the occupied 256 x 256 tiles of the
// gradient, and upload them.  Synchronous (set-up of a synchronous call).
static int plan_support_skip(const Plan& P, void* ws, const uint8_t* mask, int units32,
                             hipStream_t st) {
    const int tn = P.tp.tilesN, ks32 = P.ks32;
    uint8_t* occ = at<uint8_t>(ws, P.off_occ);
    launch_support_occupancy(mask, P.p, P.p_pad, tn, ks32, occ, st);
    std::vector<uint8_t> h((size_t)tn * ks32);
    HIP_TRY(hipMemcpyAsync(h.data(), occ, h.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int ks = ks32 / units32;
    std::vector<int32_t> ptr((size_t)tn + 1, 0), idx;
    idx.reserve((size_t)tn * 8);
    for (int c = 0; c < tn; ++c) {
        for (int s = 0; s < ks; ++s) {
            bool any = false;
            for (int u = 0; u < units32; ++u) any = any || h[(size_t)c * ks32 + s * units32 + u];
            if (any) idx.push_back(s);
        }
        ptr[c + 1] = (int32_t)idx.size();
    }
    // a gradient tile covers gbm / 32 steps of 32 rows and gbn / 128 column blocks
    const int spt = P.gbm / 32, cpt = P.gbn / 128;
    std::vector<uint8_t> gocc((size_t)P.tilesMg * P.tilesNg, 0);
    for (int tm = 0; tm < P.tilesMg; ++tm)
        for (int tg = 0; tg < P.tilesNg; ++tg) {
            bool any = false;
            for (int c = cpt * tg; c < cpt * tg + cpt && c < tn; ++c)
                for (int s = spt * tm; s < spt * tm + spt && s < ks32; ++s)
                    any = any || h[(size_t)c * ks32 + s];
            gocc[tm + (size_t)tg * P.tilesMg] = any ? 1 : 0;
        }
    HIP_TRY(hipMemcpyAsync(at<int32_t>(ws, P.off_kptr), ptr.data(), ptr.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, st));
    if (!idx.empty())
        HIP_TRY(hipMemcpyAsync(at<int32_t>(ws, P.off_kidx), idx.data(),
                               idx.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(at<uint8_t>(ws, P.off_gocc), gocc.data(), gocc.size(),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return ACCORD_OK;
}

// Alg. 1; with support_src set, the refit of eq. 3.8: penalty phi * lambda on the
// support of support_src (its nonzero entries and the diagonal), infinite off it.
static int fit_impl(const float* X, int64_t n, int64_t p, float* Omega, const accord_params* prm,
                    accord_stats* stats, double* trace, void* ws, size_t ws_bytes, void* stream,
                    const float* support_src, double phi) {
    TRY(check_dims(n, p));
    TRY(check_ptr(X, "X"));
    TRY(check_ptr(Omega, "Omega"));
    TRY(check_params(prm));
    if (trace && !aligned(trace, 8)) return fail(ACCORD_ERR_INVALID_ARG, "trace must be 8-byte aligned");
    const Plan P = make_plan(n, p, prm->max_iter, prm->precision);
    TRY(check_ws(ws, ws_bytes, support_src ? P.end_refit : P.end_fit));
    if (stats) memset(stats, 0, sizeof *stats);
    const double lambda = support_src ? phi * prm->lambda : prm->lambda;
    hipStream_t st = (hipStream_t)stream;
    const bool timing = prm->timing != 0;
    // every timing-th iteration's launch groups are bracketed by events: an event in the
    // stream costs a few microseconds of GPU time, so sparse sampling keeps the timed fit
    // close to an untimed one
    const int tstride = prm->timing > 0 ? prm->timing : 1;
    EventPool pool;
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    if (timing) {
        ev_begin = pool.get();
        ev_end = pool.get();
        HIP_TRY(hipEventRecord(ev_begin, st));
    }

    LsState* ls = at<LsState>(ws, P.off_ls);
    float* xp = at<float>(ws, P.off_xp);
    float* xt = at<float>(ws, P.off_xt);
    float* om[2] = {at<float>(ws, P.off_om0), at<float>(ws, P.off_om1)};
    float* wt[2] = {at<float>(ws, P.off_wt0), at<float>(ws, P.off_wt1)};
    float* G = at<float>(ws, P.off_g);
    const int prec = prm->precision;
    const bool bf = is_bf16(prec);
    const bool f8 = prec == PREC_FP8;
    const bool fused = P.fused != 0;
    float* D = (fused || P.fused32) ? nullptr : at<float>(ws, P.off_d);
    double* prox_part = at<double>(ws, P.off_prox_part);
    double* norm_part = at<double>(ws, P.off_norm_part);
    int32_t* trials_log = at<int32_t>(ws, P.off_trials);
    const int ttiles32 = norm_rows(P.t32, PREC_FP32);  // setup product W0 = X Omega0 (FP32)
    const int ttiles = norm_rows(P.tp, prec);          // trial products of the form
    const int64_t total = p * P.p_pad;

    // ---- setup: operands, L, W0 = X Omega0, f(Omega0)
    launch_init_state(ls, prm->tau0, prm->beta, lambda, prm->tol, 1.0 / (double)n,
                      prm->lipschitz, prm->max_iter, st, prm->warm_tau);
    launch_pad_x(X, n, p, xp, P.p_pad, xt, P.n_pad, x_split(P, ws), ls, st);
    launch_copy_cols(Omega, p, om[0], P.p_pad, p, P.p_pad, ls, st);
    uint8_t* mask = support_src ? at<uint8_t>(ws, P.off_mask) : nullptr;
    if (mask) launch_support_mask(support_src, p, P.p_pad, mask, om[0], st);
    // refit: walk only the blocks that can hold support entries
    const int32_t* kptr = nullptr;
    const int32_t* kidx = nullptr;
    const uint8_t* gocc = nullptr;
    // (the FP32 form with a separate prox pass, n > 512, walks every block)
    if (mask && (P.fused || P.fused32) && prm->support_skip) {
        TRY(plan_support_skip(P, ws, mask, f8 ? 2 : 1, st));
        kptr = at<int32_t>(ws, P.off_kptr);
        kidx = at<int32_t>(ws, P.off_kidx);
        gocc = at<uint8_t>(ws, P.off_gocc);
        // skipped blocks are never written: the second iterate buffer and G start at zero
        HIP_TRY(hipMemsetAsync(om[1], 0, (size_t)(P.p_cols * P.p_pad) * sizeof(float), st));
        HIP_TRY(hipMemsetAsync(G, 0, (size_t)(P.p_cols * P.p_pad) * sizeof(float), st));
    }
    if (P.p_cols > p) {  // zero padding columns (the fused kernels keep them zero)
        const size_t pad = (size_t)((P.p_cols - p) * P.p_pad) * sizeof(float);
        for (float* b : {om[0], om[1], G}) HIP_TRY(hipMemsetAsync(b + p * P.p_pad, 0, pad, st));
    }
    if (f8) {
        XQuant q = {at<uint8_t>(ws, P.off_x8), at<uint8_t>(ws, P.off_x8s),
                    at<uint8_t>(ws, P.off_xt8), at<uint8_t>(ws, P.off_xt8s)};
        launch_quant_x8(X, n, p, P.p_pad, P.n_pad, q, st);
    }
    if (prm->lipschitz <= 0.0) {
        launch_lipschitz(xp, P.p_pad, xt, P.n_pad, n, p,
                         lz_buf(at<char>(ws, P.off_lz), P.n_pad, P.p_pad),
                         prm->power_iters > 0 ? prm->power_iters : kLzDefaultSteps, ls, st);
    }
    // W0 = X Omega0 in FP32 (once), plus its bf16 split for the first gradient
    enqueue_trial(trial_args(P, ws, PREC_FP32, om[0], nullptr, nullptr, nullptr, wt[0],
                             bf ? 0 : -1, nullptr, 0),
                  PREC_FP32, st);
    {
        ProxArgs a = {};
        a.om = om[0];
        a.total = total;
        a.ld = P.p_pad;
        a.p = p;
        a.part = prox_part;
        a.reduce_only = 1;
        launch_prox(a, P.nprox, st);
    }
    launch_fit_init(ls, prox_part, P.nprox, norm_part, ttiles32, trace, st);
    HIP_TRY(hipGetLastError());
    LsState host = {};
    HIP_TRY(hipMemcpyAsync(&host, ls, sizeof host, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (host.bad & 2) return fail(ACCORD_ERR_NONFINITE, "non-finite value in X or Omega0");
    if (host.bad & 1) return fail(ACCORD_ERR_DOMAIN, "Omega0 has a non-positive diagonal entry");
    if (!(host.L > 0.0) || !isfinite(host.L))
        return fail(ACCORD_ERR_NONFINITE, "Lipschitz estimate is not positive (L=%g)", host.L);
    const int ntr = max_trials(prm->tau0, prm->beta, host.inv_L);

    // ---- Alg. 1
    // Trials are enqueued with one trial of look-ahead: the host enqueues trial k+1
    // and then waits (on the pinned mailbox) for trial k's outcome; it enqueues
    // trial k+2 only if trial k was rejected.  Every kernel still checks the device
    // state first, so the one speculative trial after an acceptance does no work.
    Mailbox* mbox_dev = nullptr;
    Mailbox* mbox = host_mailbox(&mbox_dev);
    if (!mbox) return fail(ACCORD_ERR_HIP, "could not allocate the pinned host mailbox");
    __atomic_store_n(&mbox->word, mailbox_word(0, 0, 0), __ATOMIC_RELEASE);
    struct Launch { hipEvent_t a, b; int iter, trial; };
    std::vector<Launch> ev_grad, ev_trial, ev_prox;
    int cur = 0;
    int base = 0;  // trials finalised before the current iteration
    for (int t = 0; t < prm->max_iter; ++t) {
        const int nxt = cur ^ 1;
        const bool tim = timing && t % tstride == 0;
        GemmArgs ga = grad_args(P, ws, prec, wt[cur], cur, G, P.p_pad, (int)P.p_pad, ls);
        ga.cmask = mask;  // refit: G = 0 off the support, so the prox keeps those entries 0
        ga.tile_occ = gocc;
        Launch lg = {nullptr, nullptr, t, 0};
        if (tim) { lg.a = pool.get(); lg.b = pool.get(); HIP_TRY(hipEventRecord(lg.a, st)); }
        if (f8)  // MX copy of the current W (blocks along the samples) for the gradient
            launch_quant_w8(wt[cur], p * P.n_pad, at<uint8_t>(ws, P.off_w8),
                            at<uint8_t>(ws, P.off_w8s), ls, st);
        launch_gemm(ga, EPI_GRAD, prec, st);
        if (tim) { HIP_TRY(hipEventRecord(lg.b, st)); ev_grad.push_back(lg); }
        const bool probing = fused && P.probe && prm->probe;
        auto enqueue_trial_k = [&](int k) -> int {
            ProxArgs a = {};
            a.om = om[cur];
            a.g = G;
            a.om_new = om[nxt];
            a.d = D;
            a.total = total;
            a.ld = P.p_pad;
            a.p = p;
            a.ls = ls;
            a.part = prox_part;
            GemmArgs ta = trial_args(P, ws, prec, D, nullptr, nullptr, wt[cur], wt[nxt],
                                     bf ? nxt : -1, ls, 2);
            ta.kstep_ptr = kptr;
            ta.kstep_idx = kidx;
            if (D) {  // FP32 form with many row tiles: prox pass, then the plain product
                Launch lp = {nullptr, nullptr, t, k};
                if (tim) { lp.a = pool.get(); lp.b = pool.get(); HIP_TRY(hipEventRecord(lp.a, st)); }
                launch_prox(a, P.nprox, st);
                if (tim) { HIP_TRY(hipEventRecord(lp.b, st)); ev_prox.push_back(lp); }
            }
            Launch lt = {nullptr, nullptr, t, k};
            if (tim) { lt.a = pool.get(); lt.b = pool.get(); HIP_TRY(hipEventRecord(lt.a, st)); }
            if (probing) {
                // probe: M tile 0 with the prox sums, no Omega+ store; then the test of
                // its lower bound; then (unless rejected) the other M tiles: staged, one
                // launch each with the test of the lower bound after each but the last
                // (whose launch stores Omega+), else one launch whose first M tile stores
                // Omega+.  Once the iteration has stopped probing (see k_probe_decide and
                // finalize_run) these are skipped and the last launch runs the whole
                // product instead; a trial rejected by a partial test skips that too.
                const int nparts = (P.tp.splits > 1 || P.tp.tail_splits > 1) ? kFReduceParts : 1;
                const int tm = P.tp.tilesM;
                GemmArgs tpb = ta;
                tpb.m_first = 0;
                tpb.m_count = 1;
                tpb.store_m = -1;
                tpb.sums_m = 0;
                tpb.probe_mode = 1;
                launch_trial_fused(tpb, a, prec, st);
                launch_probe_decide(ls, prox_part, P.prox_rows, norm_part, P.tp.tilesN, tm,
                                    nparts, 1, mbox_dev, st);
                if (P.staged) {
                    for (int m = 1; m < tm; ++m) {
                        GemmArgs ts = ta;
                        ts.m_first = m;
                        ts.m_count = 1;
                        ts.store_m = tm - 1;
                        ts.sums_m = -1;
                        ts.pred = 3;
                        ts.probe_mode = 1;
                        launch_trial_fused(ts, a, prec, st);
                        if (m + 1 < tm)
                            launch_probe_decide(ls, prox_part, P.prox_rows, norm_part,
                                                P.tp.tilesN, tm, nparts, m + 1, mbox_dev, st);
                    }
                } else {
                    GemmArgs tcp = ta;
                    tcp.m_first = 1;
                    tcp.m_count = tm - 1;
                    tcp.store_m = 1;
                    tcp.sums_m = -1;
                    tcp.pred = 3;
                    tcp.probe_mode = 1;
                    launch_trial_fused(tcp, a, prec, st);
                }
                GemmArgs tfl = ta;
                tfl.pred = 3;
                tfl.probe_mode = 2;
                launch_trial_fused(tfl, a, prec, st);
            } else if (fused)
                launch_trial_fused(ta, a, prec, st);
            else if (P.fused32)
                launch_trial_fused32(ta, a, st);
            else
                enqueue_trial(ta, prec, st);
            if (tim) { HIP_TRY(hipEventRecord(lt.b, st)); ev_trial.push_back(lt); }
            launch_finalize(ls, prox_part, P.prox_rows, norm_part, ttiles, trace, trials_log,
                            mbox_dev, probing ? 1 : 0, st);
            HIP_TRY(hipGetLastError());
            return ACCORD_OK;
        };
        int launched = 0;
        TRY(enqueue_trial_k(launched++));
        if (launched < ntr) TRY(enqueue_trial_k(launched++));
        bool stop = false;
        for (int k = 0;; ++k) {
            // wait for trial k of this iteration to be finalised
            const int target = base + k + 1;
            Posted m = read_mailbox(mbox);
            for (long spins = 1; !(m.trials >= target || m.stop); ++spins, m = read_mailbox(mbox)) {
                if ((spins & 4095) == 0) {
                    const hipError_t e = hipStreamQuery(st);
                    if (e == hipSuccess) {  // stream drained: the outcome must be posted now
                        m = read_mailbox(mbox);
                        if (m.trials >= target || m.stop) break;
                        return fail(ACCORD_ERR_HIP, "device stopped posting trial outcomes");
                    }
                    if (e != hipErrorNotReady)
                        return fail(ACCORD_ERR_HIP, "stream error: %s", hipGetErrorString(e));
                }
            }
            if (m.stop) {
                stop = true;
                break;
            }
            if (m.iter > t) {  // accepted at trial k
                base = m.trials;
                break;
            }
            if (launched < ntr) TRY(enqueue_trial_k(launched++));
        }
        cur = nxt;
        if (stop) break;
        if (prm->refresh_every > 0 && (t + 1) % prm->refresh_every == 0) {
            // W = X Omega afresh (FP32), with the bf16 split the next gradient reads; the
            // next trial's sums then describe the refreshed W
            enqueue_trial(trial_args(P, ws, PREC_FP32, om[cur], nullptr, nullptr, nullptr,
                                     wt[cur], bf ? cur : -1, nullptr, 0),
                          PREC_FP32, st);
            HIP_TRY(hipGetLastError());
        }
    }
    if (timing) HIP_TRY(hipEventRecord(ev_end, st));
    HIP_TRY(hipMemcpyAsync(&host, ls, sizeof host, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));

    // the current iterate sits in om[iter % 2]: buffers alternate once per accepted
    // iteration, and iterations after a stop did no work
    const int res = host.iter & 1;
    launch_copy_cols(om[res], P.p_pad, Omega, p, p, p, nullptr, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));

    if (stats) {
        stats->iters = host.iter;
        stats->trials = host.total_trials;
        stats->floor_accepts = host.floor_accepts;
        stats->converged = (prm->tol > 0.0 && host.iter < prm->max_iter && host.converged &&
                            !host.bad) ? 1 : 0;
        stats->nnz_offdiag = host.nnz_off;
        stats->f = host.f_cur;
        stats->g = host.g_cur;
        stats->h = host.h_cur;
        stats->tau_last = host.tau_acc;
        stats->delta_fro = host.delta_fro;
        stats->lipschitz = host.L;
        stats->log_det_d = host.logd_cur;
        stats->l1 = host.l1_cur;
        stats->lz_steps = host.lz_steps;
        stats->probe_rejects = host.probe_rejects;
        stats->unprobed_trials = host.unprobed;
        stats->probe_mtiles = host.probe_mtiles;
        {
            const Geo& tg = fused ? P.tp : P.t32;
            const bool used = fused || !P.fused32;  // the fused FP32 trial runs unsplit
            stats->tail_blocks = used && tg.tail_splits > 1 ? tg.tilesN - tg.tail_n0 : 0;
            stats->tail_splits = used ? tg.tail_splits : 0;
        }
        if (timing) {
            std::vector<int32_t> tl((size_t)(host.iter > 0 ? host.iter : 1), 0);
            if (host.iter > 0)
                HIP_TRY(hipMemcpy(tl.data(), trials_log, sizeof(int32_t) * host.iter,
                                  hipMemcpyDeviceToHost));
            float ms = 0.f;
            for (const Launch& l : ev_grad) {
                if (l.iter >= host.iter) continue;
                HIP_TRY(hipEventElapsedTime(&ms, l.a, l.b));
                stats->grad_gemm_ms += ms;
                stats->grad_gemm_launches += 1;
            }
            for (const Launch& l : ev_trial) {
                if (l.iter >= host.iter || l.trial >= tl[l.iter]) continue;
                HIP_TRY(hipEventElapsedTime(&ms, l.a, l.b));
                stats->trial_gemm_ms += ms;
                stats->trial_gemm_launches += 1;
            }
            for (const Launch& l : ev_prox) {
                if (l.iter >= host.iter || l.trial >= tl[l.iter]) continue;
                HIP_TRY(hipEventElapsedTime(&ms, l.a, l.b));
                stats->prox_ms += ms;
                stats->prox_launches += 1;
            }
            HIP_TRY(hipEventElapsedTime(&ms, ev_begin, ev_end));
            stats->total_ms = ms;
        }
    }
    if (host.bad & 2) return fail(ACCORD_ERR_NONFINITE, "non-finite value in an iterate");
    if (host.bad & 1) return fail(ACCORD_ERR_DOMAIN, "non-positive diagonal in an iterate");
    return ACCORD_OK;
}

int accord_fit(const float* X, int64_t n, int64_t p, float* Omega, const accord_params* prm,
               accord_stats* stats, double* trace, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return fit_impl(X, n, p, Omega, prm, stats, trace, ws, ws_bytes, stream, nullptr, 1.0);
}

// ---------------------------------------------------------------------------
// Steps around the solver: refit (eq. 3.8), epBIC (eq. 3.7), reparametrisation
// ---------------------------------------------------------------------------
size_t accord_refit_workspace_bytes(int64_t n, int64_t p, const accord_params* prm) {
    if (n < 1 || p < 1 || n > (1LL << 24) || p > (1LL << 24)) return 0;
    accord_params d;
    if (!prm) {
        accord_default_params(&d);
        prm = &d;
    }
    return make_plan(n, p, prm->max_iter, prm->precision).end_refit;
}

int accord_refit(const float* X, int64_t n, int64_t p, const float* Omega_hat, double phi,
                 float* Omega, const accord_params* prm, accord_stats* stats, double* trace,
                 void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    TRY(check_ptr(Omega_hat, "Omega_hat"));
    if (!(phi >= 0.0 && phi <= 1.0)) return fail(ACCORD_ERR_INVALID_ARG, "phi must lie in [0, 1]");
    return fit_impl(X, n, p, Omega, prm, stats, trace, ws, ws_bytes, stream, Omega_hat, phi);
}

int accord_epbic(int64_t n, int64_t p, double g, double log_det_d, int64_t nnz_offdiag,
                 double gamma, double* out) {
    g_last_error.clear();
    TRY(check_dims(n, p));
    if (!out) return fail(ACCORD_ERR_INVALID_ARG, "out is null");
    if (!(gamma > 0.0 && gamma <= 1.0)) return fail(ACCORD_ERR_INVALID_ARG, "gamma must lie in (0, 1]");
    if (nnz_offdiag < 0 || nnz_offdiag > p * (p - 1))
        return fail(ACCORD_ERR_INVALID_ARG, "nnz_offdiag must lie in [0, p(p-1)]");
    const double k = (double)nnz_offdiag;
    *out = 2.0 * (double)n * (-log_det_d + g) + k * log((double)n) +
           4.0 * gamma * k * log((double)p);
    return ACCORD_OK;
}

int accord_epbic_path(const accord_batch_stats* stats, const int64_t* n, int64_t nsub,
                      int64_t nlam, int64_t p, double gamma, double* epbic, int64_t* best) {
    g_last_error.clear();
    if (!stats || !n || !epbic) return fail(ACCORD_ERR_INVALID_ARG, "stats, n and epbic must be non-null");
    if (nsub < 1 || nlam < 1) return fail(ACCORD_ERR_INVALID_ARG, "nsub and nlam must be >= 1");
    for (int64_t b = 0; b < nsub; ++b) {
        int64_t arg = 0;
        for (int64_t l = 0; l < nlam; ++l) {
            const int64_t k = b * nlam + l;
            const accord_batch_stats& s = stats[k];
            TRY(accord_epbic(n[b], p, s.g, s.log_det_d, s.nnz_offdiag, gamma, &epbic[k]));
            if (epbic[k] < epbic[b * nlam + arg]) arg = l;
        }
        if (best) best[b] = arg;
    }
    return ACCORD_OK;
}

int accord_reparam(const float* Omega, int64_t p, float* Theta, float* Rho, void* stream) {
    g_last_error.clear();
    TRY(check_dims(1, p));
    TRY(check_ptr(Omega, "Omega"));
    if (!Theta && !Rho) return fail(ACCORD_ERR_INVALID_ARG, "Theta and Rho are both null");
    if (Theta) TRY(check_ptr(Theta, "Theta"));
    if (Rho) TRY(check_ptr(Rho, "Rho"));
    if ((const void*)Theta == (const void*)Omega || (const void*)Rho == (const void*)Omega ||
        (Theta && Theta == Rho))
        return fail(ACCORD_ERR_INVALID_ARG, "outputs must not alias Omega or each other");
    launch_reparam(Omega, p, Theta, Rho, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ACCORD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------
namespace {

struct BatchPlan {
    int64_t p, p_pad, p_c, nsub, nlam, nprob;
    int max_iter, tpp, nprox, part_rows, max_tiles_trial, tiles_grad;
    std::vector<int64_t> n, n_pad, row_off, norm_off;
    std::vector<int> tilesM;
    size_t off_ls, off_lam, off_inv_n, off_L, off_args_w0, off_args_grad, off_args_trial,
        off_prox_init, off_px_trial, off_fin_init, off_fin, off_prox_part, off_norm_part,
        off_trials, off_lz, off_om[2], off_g, end;
    int64_t lz_npad;  // sample extent of the Lanczos buffers (the largest n_pad)
    std::vector<size_t> off_xp, off_xt, off_wt[2];
};

constexpr int kBatchProxBlocks = 64;  // prox workgroups per problem

int make_batch_plan(const int64_t* n, int64_t nsub, int64_t p, int64_t nlam, int max_iter,
                    BatchPlan& B) {
    B = BatchPlan{};
    B.p = p;
    B.p_pad = round_up(p, kPad);
    B.p_c = round_up(p, kBN);  // columns per problem in the concatenated layout
    B.nsub = nsub;
    B.nlam = nlam;
    B.nprob = nsub * nlam;
    B.max_iter = max_iter;
    B.tpp = (int)(B.p_c / kBN);
    B.nprox = kBatchProxBlocks;
    // prox sum rows per problem: the set-up statistics pass leaves nprox, every trial one
    // per column tile
    B.part_rows = std::max(B.nprox, B.tpp);
    B.tiles_grad = (int)(cdiv(B.p_pad, kBM) * nlam * B.tpp);
    B.max_tiles_trial = 0;
    int64_t rows = 0, nmax = 0, norm_rows_total = 0;
    for (int64_t b = 0; b < nsub; ++b) {
        B.n.push_back(n[b]);
        B.n_pad.push_back(round_up(n[b], kPad));
        B.row_off.push_back(rows);
        rows += n[b];
        nmax = std::max(nmax, n[b]);
        const int tm = (int)cdiv(B.n_pad[b], kBM);
        B.tilesM.push_back(tm);
        B.norm_off.push_back(norm_rows_total);
        norm_rows_total += (int64_t)nlam * tm * B.tpp;
        B.max_tiles_trial = std::max(B.max_tiles_trial, (int)(tm * nlam * B.tpp));
    }
    size_t cur = 0;
    const int64_t np = B.nprob;
    B.off_ls = bump(cur, (size_t)np * sizeof(LsState));
    B.off_lam = bump(cur, (size_t)nlam * sizeof(double));
    B.off_inv_n = bump(cur, (size_t)nsub * sizeof(double));
    B.off_L = bump(cur, (size_t)nsub * sizeof(double));
    B.off_args_w0 = bump(cur, (size_t)nsub * sizeof(GemmArgs));
    B.off_args_grad = bump(cur, (size_t)2 * nsub * sizeof(GemmArgs));
    B.off_args_trial = bump(cur, (size_t)2 * nsub * sizeof(GemmArgs));
    B.off_prox_init = bump(cur, (size_t)np * sizeof(ProxArgs));
    B.off_px_trial = bump(cur, (size_t)2 * nsub * sizeof(ProxArgs));
    B.off_fin_init = bump(cur, (size_t)np * sizeof(FinArgs));
    B.off_fin = bump(cur, (size_t)np * sizeof(FinArgs));
    B.off_prox_part = bump(cur, (size_t)np * B.part_rows * kPartCols * sizeof(double));
    B.off_norm_part = bump(cur, (size_t)norm_rows_total * kNormCols * sizeof(double));
    B.off_trials = bump(cur, (size_t)np * std::max(max_iter, 1) * sizeof(int32_t));
    const int64_t nmax_pad = round_up(nmax, kPad);
    B.lz_npad = nmax_pad;
    B.off_lz = bump(cur, lz_buf_bytes(nmax_pad, B.p_pad));
    for (int64_t b = 0; b < nsub; ++b) {
        const size_t xn = (size_t)(B.n_pad[b] * B.p_pad);
        B.off_xp.push_back(bump(cur, xn * sizeof(float)));
        B.off_xt.push_back(bump(cur, xn * sizeof(float)));
        for (int par = 0; par < 2; ++par)
            B.off_wt[par].push_back(bump(cur, (size_t)(nlam * B.p_c * B.n_pad[b]) * sizeof(float)));
    }
    const size_t mat = (size_t)(np * B.p_c * B.p_pad) * sizeof(float);
    B.off_om[0] = bump(cur, mat);
    B.off_om[1] = bump(cur, mat);
    B.off_g = bump(cur, mat);  // Delta never reaches HBM: the trial fuses the prox
    B.end = cur;
    return ACCORD_OK;
}

int check_batch_dims(const int64_t* n, int64_t nsub, int64_t p, int64_t nlam) {
    if (!n) return fail(ACCORD_ERR_INVALID_ARG, "n is null");
    if (nsub < 1 || nlam < 1 || nsub > 65535)
        return fail(ACCORD_ERR_INVALID_ARG, "need 1 <= nsub <= 65535 and nlam >= 1 (nsub=%lld nlam=%lld)",
                    (long long)nsub, (long long)nlam);
    for (int64_t b = 0; b < nsub; ++b) TRY(check_dims(n[b], p));
    // column and tile counts of one group (nlam problems of p_c columns) stay 32-bit
    const double cols = (double)nlam * (double)round_up(p, kBN);
    if (cols > 2147483647.0 ||
        (double)cdiv(round_up(p, kPad), kBM) * nlam * cdiv(p, kBN) > 2147483647.0)
        return fail(ACCORD_ERR_INVALID_ARG, "nlam * p too large for one batched launch");
    return ACCORD_OK;
}

}  // namespace

extern "C" {

size_t accord_batch_workspace_bytes(const int64_t* n, int64_t nsub, int64_t p, int64_t nlam,
                                    const accord_params* prm) {
    if (check_batch_dims(n, nsub, p, nlam) != ACCORD_OK) return 0;
    accord_params d;
    if (!prm) {
        accord_default_params(&d);
        prm = &d;
    }
    BatchPlan B;
    make_batch_plan(n, nsub, p, nlam, prm->max_iter, B);
    return B.end;
}

}  // extern "C"

// The batched fit; with tune_order set, the set-up is followed by timing every order code
// (tile order x workgroups per CU) of the gradient and of the trial kernel (tune_table:
// mean ms per launch), and the fastest of each is written to tune_order.
static int fit_batch_impl(const float* X, const int64_t* n, int64_t nsub, int64_t p,
                          const double* lambda, int64_t nlam, float* Omega,
                          const accord_params* prm, const double* lipschitz,
                          accord_batch_stats* stats, int32_t* trials, void* ws, size_t ws_bytes,
                          void* stream, int32_t* tune_order, float* tune_table) {
    TRY(check_batch_dims(n, nsub, p, nlam));
    TRY(check_ptr(X, "X"));
    TRY(check_ptr(Omega, "Omega"));
    TRY(check_params(prm));
    if (prm->precision != ACCORD_FP32)
        return fail(ACCORD_ERR_UNSUPPORTED, "the batched form runs in FP32 only");
    if (!lambda) return fail(ACCORD_ERR_INVALID_ARG, "lambda is null");
    for (int64_t l = 0; l < nlam; ++l)
        if (!(lambda[l] >= 0.0) || !isfinite(lambda[l]))
            return fail(ACCORD_ERR_INVALID_ARG, "lambda[%lld] must be finite and >= 0", (long long)l);
    if (lipschitz)
        for (int64_t b = 0; b < nsub; ++b)
            if (!(lipschitz[b] > 0.0) || !isfinite(lipschitz[b]))
                return fail(ACCORD_ERR_INVALID_ARG, "lipschitz[%lld] must be finite and > 0",
                            (long long)b);
    if (trials && !aligned(trials, 4)) return fail(ACCORD_ERR_INVALID_ARG, "trials must be 4-byte aligned");
    const int order_grad = prm->batch_order & 0xff, order_trial = (prm->batch_order >> 8) & 0xff;
    int code_grad = order_grad, code_trial = order_trial;  // launch codes (tuning may change)
    if (prm->batch_order < 0 || (prm->batch_order >> 16) != 0 || order_grad > kBatchCodes ||
        order_trial > kBatchCodes)
        return fail(ACCORD_ERR_INVALID_ARG, "batch_order %d is not a tile order code",
                    prm->batch_order);
    BatchPlan B;
    TRY(make_batch_plan(n, nsub, p, nlam, prm->max_iter, B));
    TRY(check_ws(ws, ws_bytes, B.end));
    hipStream_t st = (hipStream_t)stream;
    const int64_t np = B.nprob, mat = B.p_c * B.p_pad;

    LsState* ls = at<LsState>(ws, B.off_ls);
    float* om[2] = {at<float>(ws, B.off_om[0]), at<float>(ws, B.off_om[1])};
    float* G = at<float>(ws, B.off_g);
    double* prox_part = at<double>(ws, B.off_prox_part);
    double* norm_part = at<double>(ws, B.off_norm_part);
    int32_t* trials_log = at<int32_t>(ws, B.off_trials);

    // ---- host-built argument blocks, copied once
    std::vector<double> h_inv_n(nsub), h_L(nsub, 0.0);
    for (int64_t b = 0; b < nsub; ++b) {
        h_inv_n[b] = 1.0 / (double)B.n[b];
        if (lipschitz) h_L[b] = lipschitz[b];
    }
    std::vector<GemmArgs> a_w0(nsub), a_grad(2 * nsub), a_trial(2 * nsub);
    std::vector<ProxArgs> a_prox_init(np), a_px(2 * nsub);
    std::vector<FinArgs> a_fin_init(np), a_fin(np);
    const int64_t pstep = 4 * (int64_t)kThreads;
    for (int64_t b = 0; b < nsub; ++b) {
        const int64_t k0 = b * nlam;
        const float* xp = at<float>(ws, B.off_xp[b]);
        const float* xt = at<float>(ws, B.off_xt[b]);
        for (int par = 0; par < 3; ++par) {
            // par 0, 1: the trial of an iteration with the current buffers in `par`;
            // par 2: the setup product W0 = X Omega0
            GemmArgs t = {};
            const int cur = par == 2 ? 0 : par, nxt = par == 2 ? 0 : par ^ 1;
            t.A = xp;
            t.lda = B.p_pad;
            t.B = par == 2 ? om[0] + k0 * mat : nullptr;  // trials produce Delta in place
            t.ldb = B.p_pad;
            t.M = (int)B.n_pad[b];
            t.N = (int)(nlam * B.p_c);
            t.K = (int)B.p_pad;
            t.tilesM = B.tilesM[b];
            t.tilesN = (int)(nlam * B.tpp);
            t.splits = 1;
            t.C = at<float>(ws, B.off_wt[nxt][b]);
            t.ldc = B.n_pad[b];
            t.vec_store = 1;
            t.alpha = 1.f;
            t.Wprev = par == 2 ? nullptr : at<float>(ws, B.off_wt[cur][b]);
            t.norm_part = norm_part + B.norm_off[b] * kNormCols;
            t.ls = ls + k0;
            t.pred = par == 2 ? 0 : 2;
            t.Mvalid = (int)B.n[b];
            t.Nvalid = t.N;  // padding columns of Delta and Omega are zero
            if (par == 2) {
                a_w0[b] = t;
            } else {
                t.order = order_trial;
                a_trial[par * nsub + b] = t;
            }
        }
        for (int par = 0; par < 2; ++par) {
            // the prox of the fused trial: the group's Omega, G and Omega+ (its problems'
            // columns packed like the trial product's N), per-problem state from ls + k0
            ProxArgs q = {};
            q.om = om[par] + k0 * mat;
            q.g = G + k0 * mat;
            q.om_new = om[par ^ 1] + k0 * mat;
            q.ld = B.p_pad;
            q.p = p;
            q.ls = ls + k0;
            q.part = prox_part + k0 * B.part_rows * kPartCols;
            a_px[par * nsub + b] = q;
        }
        for (int par = 0; par < 2; ++par) {
            GemmArgs g = {};
            g.A = xt;
            g.lda = B.n_pad[b];
            g.B = at<float>(ws, B.off_wt[par][b]);
            g.ldb = B.n_pad[b];
            g.M = (int)B.p_pad;
            g.N = (int)(nlam * B.p_c);
            g.K = (int)B.n_pad[b];
            g.tilesM = (int)cdiv(B.p_pad, kBM);
            g.tilesN = (int)(nlam * B.tpp);
            g.splits = 1;
            g.C = G + k0 * mat;
            g.ldc = B.p_pad;
            g.vec_store = 1;
            g.alpha = (float)(1.0 / (double)B.n[b]);
            g.norm_part = norm_part + B.norm_off[b] * kNormCols;  // unused by the gradient
            g.ls = ls + k0;
            g.pred = 1;
            g.begin_iter = 1;
            g.order = order_grad;
            a_grad[par * nsub + b] = g;
        }
        for (int64_t l = 0; l < nlam; ++l) {
            const int64_t k = k0 + l;
            ProxArgs a = {};
            a.total = p * B.p_pad;
            a.ld = B.p_pad;
            a.p = p;
            a.step_col = pstep / a.ld;
            a.step_row = pstep - a.step_col * a.ld;
            a.part = prox_part + k * B.part_rows * kPartCols;
            ProxArgs r = a;
            r.om = om[0] + k * mat;
            r.reduce_only = 1;
            a_prox_init[k] = r;
            FinArgs f = {};
            f.ls = ls + k;
            f.prox_part = prox_part + k * B.part_rows * kPartCols;
            f.nprox = B.nprox;  // the set-up statistics pass
            f.ntiles = B.tilesM[b] * B.tpp;
            f.norm_part = norm_part + (B.norm_off[b] + l * (int64_t)f.ntiles) * kNormCols;
            f.trials_log = trials_log + k * std::max(B.max_iter, 1);
            a_fin_init[k] = f;
            f.nprox = B.tpp;    // a trial: one row per column tile of the problem
            a_fin[k] = f;
        }
    }
    GemmArgs* d_w0 = at<GemmArgs>(ws, B.off_args_w0);
    GemmArgs* d_grad = at<GemmArgs>(ws, B.off_args_grad);
    GemmArgs* d_trial = at<GemmArgs>(ws, B.off_args_trial);
    ProxArgs* d_prox_init = at<ProxArgs>(ws, B.off_prox_init);
    ProxArgs* d_px = at<ProxArgs>(ws, B.off_px_trial);
    FinArgs* d_fin_init = at<FinArgs>(ws, B.off_fin_init);
    FinArgs* d_fin = at<FinArgs>(ws, B.off_fin);
    HIP_TRY(hipMemcpyAsync(d_w0, a_w0.data(), a_w0.size() * sizeof(GemmArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_grad, a_grad.data(), a_grad.size() * sizeof(GemmArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_trial, a_trial.data(), a_trial.size() * sizeof(GemmArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_prox_init, a_prox_init.data(), a_prox_init.size() * sizeof(ProxArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_px, a_px.data(), a_px.size() * sizeof(ProxArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_fin_init, a_fin_init.data(), a_fin_init.size() * sizeof(FinArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_fin, a_fin.data(), a_fin.size() * sizeof(FinArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(at<double>(ws, B.off_lam), lambda, nlam * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(at<double>(ws, B.off_inv_n), h_inv_n.data(), nsub * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(at<double>(ws, B.off_L), h_L.data(), nsub * sizeof(double), hipMemcpyHostToDevice, st));

    // ---- setup: state, operands, L, W0 = X_b Omega0, f(Omega0)
    launch_init_state_batch(ls, (int)np, (int)nlam, at<double>(ws, B.off_lam),
                            at<double>(ws, B.off_inv_n), at<double>(ws, B.off_L), prm->tau0,
                            prm->beta, prm->tol, prm->max_iter, st, prm->warm_tau);
    // padding columns of every problem's Omega must read as zero (the trials never write
    // them, and the gradient leaves zeros in those of G)
    HIP_TRY(hipMemsetAsync(om[0], 0, (size_t)(np * mat) * sizeof(float), st));
    HIP_TRY(hipMemsetAsync(om[1], 0, (size_t)(np * mat) * sizeof(float), st));
    for (int64_t b = 0; b < nsub; ++b) {
        const int64_t k0 = b * nlam;
        launch_pad_x(X + B.row_off[b] * p, B.n[b], p, at<float>(ws, B.off_xp[b]), B.p_pad,
                     at<float>(ws, B.off_xt[b]), B.n_pad[b], XSplit{}, ls + k0, st);
        if (!lipschitz)
            launch_lipschitz(at<float>(ws, B.off_xp[b]), B.p_pad, at<float>(ws, B.off_xt[b]),
                             B.n_pad[b], B.n[b], p, lz_buf(at<char>(ws, B.off_lz), B.lz_npad, B.p_pad),
                             prm->power_iters > 0 ? prm->power_iters : kLzDefaultSteps, ls + k0,
                             st);
    }
    if (!lipschitz) launch_share_L_batch(ls, (int)np, (int)nlam, st);
    for (int64_t k = 0; k < np; ++k)
        launch_copy_cols(Omega + k * p * p, p, om[0] + k * mat, B.p_pad, p, B.p_pad, ls + k, st);
    launch_gemm_f32_batch(d_w0, (int)nsub, B.max_tiles_trial, B.tpp, EPI_TRIAL, 0, st);
    launch_prox_batch(d_prox_init, (int)np, B.nprox, st);
    launch_fit_init_batch(d_fin_init, (int)np, st);
    HIP_TRY(hipGetLastError());
    std::vector<LsState> host((size_t)np);
    HIP_TRY(hipMemcpyAsync(host.data(), ls, np * sizeof(LsState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int ntr = 1;
    for (int64_t k = 0; k < np; ++k) {
        const int b = (int)(k / nlam);
        if (host[k].bad & 2)
            return fail(ACCORD_ERR_NONFINITE, "non-finite value in X (subsample %d) or Omega0 (problem %lld)",
                        b, (long long)k);
        if (host[k].bad & 1)
            return fail(ACCORD_ERR_DOMAIN, "Omega0 of problem %lld has a non-positive diagonal entry",
                        (long long)k);
        if (!(host[k].L > 0.0) || !isfinite(host[k].L))
            return fail(ACCORD_ERR_NONFINITE, "Lipschitz estimate of subsample %d is not positive", b);
        ntr = std::max(ntr, max_trials(prm->tau0, prm->beta, host[k].inv_L));
    }

    if (tune_order) {
        // Time every order code (tile order x workgroups per CU) of the gradient, then of
        // the trial kernel (three launches each, the first to warm up).  Nothing here disturbs the fit: the gradient resets
        // each problem's line search to the start of an iteration, as the first sweep's
        // does; the trial launches (without an acceptance test) only write buffers the
        // first sweep overwrites.
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        int best[2] = {0, 0};
        int err = ACCORD_OK;
        for (int kind = 0; kind < 2 && err == ACCORD_OK; ++kind) {
            std::vector<GemmArgs>& args = kind == 0 ? a_grad : a_trial;
            GemmArgs* dev = kind == 0 ? d_grad : d_trial;
            float best_ms = 0.f;
            for (int code = 1; code <= kBatchCodes && err == ACCORD_OK; ++code) {
                for (GemmArgs& g : args) g.order = code;
                HIP_TRY(hipMemcpyAsync(dev, args.data(), args.size() * sizeof(GemmArgs),
                                       hipMemcpyHostToDevice, st));
                for (int rep = 0; rep < 3; ++rep) {
                    if (rep == 1) HIP_TRY(hipEventRecord(e0, st));
                    if (kind == 0)
                        launch_gemm_f32_batch(d_grad, (int)nsub, B.tiles_grad, B.tpp, EPI_GRAD,
                                              code, st);
                    else
                        launch_trial_fused32_batch(d_trial, d_px, (int)nsub, B.max_tiles_trial,
                                                   B.tpp, B.part_rows, code, st);
                }
                HIP_TRY(hipEventRecord(e1, st));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                ms *= 0.5f;
                if (tune_table) tune_table[kind * kBatchCodes + code - 1] = ms;
                if (best[kind] == 0 || ms < best_ms) {
                    best[kind] = code;
                    best_ms = ms;
                }
            }
            for (GemmArgs& g : args) g.order = best[kind];
            HIP_TRY(hipMemcpyAsync(dev, args.data(), args.size() * sizeof(GemmArgs),
                                   hipMemcpyHostToDevice, st));
        }
        HIP_TRY(hipStreamSynchronize(st));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *tune_order = best[0] | (best[1] << 8);
        code_grad = best[0];
        code_trial = best[1];
    }

    // ---- Alg. 1 for every problem, one iteration per sweep.  Each sweep enqueues the
    // gradient and ntr trials (enough for the problem whose floor is lowest); a
    // problem that accepted, or stopped, skips the rest of the sweep.
    // Sweep t uses the argument blocks of parity t & 1 (ping-pong buffers); nothing in a
    // sweep depends on the host, so with prm->graph the two sweeps are captured once and
    // replayed.
    auto enqueue_sweep = [&](int par) {
        launch_gemm_f32_batch(d_grad + par * nsub, (int)nsub, B.tiles_grad, B.tpp, EPI_GRAD,
                              code_grad, st);
        for (int k = 0; k < ntr; ++k) {
            launch_trial_fused32_batch(d_trial + par * nsub, d_px + par * nsub, (int)nsub,
                                       B.max_tiles_trial, B.tpp, B.part_rows, code_trial, st);
            launch_finalize_batch(d_fin, (int)np, st);
        }
    };
    const int nsweeps = tune_order ? 0 : prm->max_iter;  // tuning: no sweeps
    if (prm->graph && st != nullptr && nsweeps > 0) {
        struct Graphs {
            hipGraph_t g[2] = {nullptr, nullptr};
            hipGraphExec_t e[2] = {nullptr, nullptr};
            ~Graphs() {
                for (int i = 0; i < 2; ++i) {
                    if (e[i]) (void)hipGraphExecDestroy(e[i]);
                    if (g[i]) (void)hipGraphDestroy(g[i]);
                }
            }
        } G;
        const int nsweep = nsweeps < 2 ? nsweeps : 2;
        for (int par = 0; par < nsweep; ++par) {
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            enqueue_sweep(par);
            const hipError_t cap = hipGetLastError();
            const hipError_t end = hipStreamEndCapture(st, &G.g[par]);
            if (cap != hipSuccess) return fail(ACCORD_ERR_HIP, "sweep capture: %s", hipGetErrorString(cap));
            if (end != hipSuccess) return fail(ACCORD_ERR_HIP, "sweep capture: %s", hipGetErrorString(end));
            HIP_TRY(hipGraphInstantiate(&G.e[par], G.g[par], nullptr, nullptr, 0));
        }
        for (int t = 0; t < nsweeps; ++t) HIP_TRY(hipGraphLaunch(G.e[t & 1], st));
        HIP_TRY(hipStreamSynchronize(st));  // before the graphs are destroyed
    } else {
        for (int t = 0; t < nsweeps; ++t) {
            enqueue_sweep(t & 1);
            HIP_TRY(hipGetLastError());
        }
    }
    HIP_TRY(hipMemcpyAsync(host.data(), ls, np * sizeof(LsState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t k = 0; k < np; ++k)
        launch_copy_cols(om[host[k].iter & 1] + k * mat, B.p_pad, Omega + k * p * p, p, p, p,
                         nullptr, st);
    if (trials && nsweeps > 0)
        HIP_TRY(hipMemcpyAsync(trials, trials_log, (size_t)np * prm->max_iter * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    int status = ACCORD_OK;
    for (int64_t k = 0; k < np; ++k) {
        const LsState& h = host[k];
        if (stats) {
            accord_batch_stats& s = stats[k];
            s.iters = h.iter;
            s.trials = h.total_trials;
            s.floor_accepts = h.floor_accepts;
            s.converged = (prm->tol > 0.0 && h.iter < prm->max_iter && h.converged && !h.bad) ? 1 : 0;
            s.nnz_offdiag = h.nnz_off;
            s.f = h.f_cur;
            s.g = h.g_cur;
            s.h = h.h_cur;
            s.tau_last = h.tau_acc;
            s.delta_fro = h.delta_fro;
            s.lipschitz = h.L;
            s.log_det_d = h.logd_cur;
            s.l1 = h.l1_cur;
        }
        if (status == ACCORD_OK && (h.bad & 2))
            status = fail(ACCORD_ERR_NONFINITE, "non-finite value in an iterate of problem %lld", (long long)k);
        if (status == ACCORD_OK && (h.bad & 1))
            status = fail(ACCORD_ERR_DOMAIN, "non-positive diagonal in an iterate of problem %lld", (long long)k);
    }
    return status;
}

extern "C" {

int accord_fit_batch(const float* X, const int64_t* n, int64_t nsub, int64_t p,
                     const double* lambda, int64_t nlam, float* Omega, const accord_params* prm,
                     const double* lipschitz, accord_batch_stats* stats, int32_t* trials,
                     void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return fit_batch_impl(X, n, nsub, p, lambda, nlam, Omega, prm, lipschitz, stats, trials, ws,
                          ws_bytes, stream, nullptr, nullptr);
}

int accord_tune_batch(const float* X, const int64_t* n, int64_t nsub, int64_t p,
                      const double* lambda, int64_t nlam, float* Omega, const accord_params* prm,
                      const double* lipschitz, void* ws, size_t ws_bytes, void* stream,
                      int32_t* order, float* table) {
    g_last_error.clear();
    if (!order) return fail(ACCORD_ERR_INVALID_ARG, "order is null");
    if (!prm) return fail(ACCORD_ERR_INVALID_ARG, "params is null");
    accord_params q = *prm;
    // the set-up of a fit (which must leave the problems running: max_iter >= 1), then the
    // timing instead of the sweeps
    q.max_iter = q.max_iter > 0 ? q.max_iter : 1;
    q.tol = 0.0;
    q.batch_order = 0;
    return fit_batch_impl(X, n, nsub, p, lambda, nlam, Omega, &q, lipschitz, nullptr, nullptr,
                          ws, ws_bytes, stream, order, table);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Differentiation form
// ---------------------------------------------------------------------------
namespace {

constexpr int kAdjBlocks = 1024;  // workgroups of the prox adjoint (FP64 partial rows)

struct AdjPlan {
    Plan P;
    Geo gx;  // X bar product: M = p, N = n, K = 2 p_pad
    size_t off_at, off_bw, off_xsplit, off_xnorm, off_adjpart, end;
};

AdjPlan make_adj_plan(int64_t n, int64_t p) {
    AdjPlan A;
    A.P = make_plan(n, p, 1, PREC_FP32);
    const int64_t k2 = 2 * A.P.p_pad;
    A.gx.tilesM = (int)cdiv(p, kBM);
    A.gx.tilesN = (int)cdiv(n, kBN);
    A.gx.splits = choose_splits(A.gx.tiles(), (int)(k2 / kPad), kSlots);
    size_t cur = A.P.end_fit;
    A.off_at = bump(cur, (size_t)(A.P.p_pad * k2) * sizeof(float));
    A.off_bw = bump(cur, (size_t)(A.P.n_pad * k2) * sizeof(float));
    A.off_xsplit = bump(cur, (size_t)(A.gx.splits > 1 ? A.gx.splits : 0) * A.gx.tiles() * kBM *
                                 kBN * sizeof(float));
    A.off_xnorm = bump(cur, (size_t)A.gx.tiles() * kNormCols * sizeof(double));
    A.off_adjpart = bump(cur, (size_t)kAdjBlocks * sizeof(double));
    A.end = cur;
    return A;
}

int check_taus(const double* taus, int64_t nsteps) {
    if (nsteps < 0) return fail(ACCORD_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (nsteps > 0 && !taus) return fail(ACCORD_ERR_INVALID_ARG, "taus is null");
    for (int64_t t = 0; t < nsteps; ++t)
        if (!(taus[t] > 0.0) || !isfinite(taus[t]))
            return fail(ACCORD_ERR_INVALID_ARG, "taus[%lld] must be finite and > 0", (long long)t);
    return ACCORD_OK;
}

}  // namespace

extern "C" {

size_t accord_adjoint_workspace_bytes(int64_t n, int64_t p) {
    if (n < 1 || p < 1 || n > (1LL << 20) || p > (1LL << 20)) return 0;
    return make_adj_plan(n, p).end;
}

int accord_fbs_replay(const float* X, int64_t n, int64_t p, float* Omega, const double* taus,
                      int64_t nsteps, double lambda, float* Omega_seq, void* ws, size_t ws_bytes,
                      void* stream) {
    g_last_error.clear();
    TRY(check_dims(n, p));
    TRY(check_ptr(X, "X"));
    TRY(check_ptr(Omega, "Omega"));
    TRY(check_taus(taus, nsteps));
    if (!(lambda >= 0.0) || !isfinite(lambda))
        return fail(ACCORD_ERR_INVALID_ARG, "lambda must be finite and >= 0");
    if (Omega_seq) TRY(check_ptr(Omega_seq, "Omega_seq"));
    const Plan P = make_plan(n, p, 1, PREC_FP32);
    TRY(check_ws(ws, ws_bytes, P.end_fit));
    hipStream_t st = (hipStream_t)stream;
    LsState* ls = at<LsState>(ws, P.off_ls);
    launch_init_state(ls, 1.0, 1.0, lambda, 0.0, 1.0 / (double)n, 1.0, 0, st);
    launch_pad_x(X, n, p, at<float>(ws, P.off_xp), P.p_pad, at<float>(ws, P.off_xt), P.n_pad,
                 XSplit{}, ls, st);
    float* om[2] = {at<float>(ws, P.off_om0), at<float>(ws, P.off_om1)};
    float* wt = at<float>(ws, P.off_wt0);
    float* G = at<float>(ws, P.off_g);
    launch_copy_cols(Omega, p, om[0], P.p_pad, p, P.p_pad, nullptr, st);
    int cur = 0;
    for (int64_t t = 0; t < nsteps; ++t) {
        // fresh W = X Omega_t and G = X^T W / n, then the prox at tau_t (eq. 3.5)
        enqueue_trial(trial_args(P, ws, PREC_FP32, om[cur], nullptr, nullptr, nullptr, wt, -1,
                                 nullptr, 0),
                      PREC_FP32, st);
        launch_gemm(grad_args(P, ws, PREC_FP32, wt, 0, G, P.p_pad, (int)P.p_pad, nullptr),
                    EPI_GRAD, PREC_FP32, st);
        ProxArgs a = {};
        a.om = om[cur];
        a.g = G;
        a.om_new = om[cur ^ 1];
        a.total = p * P.p_pad;
        a.ld = P.p_pad;
        a.p = p;
        a.tau = taus[t];
        a.lambda = lambda;
        a.part = at<double>(ws, P.off_prox_part);
        launch_prox(a, P.nprox, st);
        cur ^= 1;
        if (Omega_seq) launch_copy_cols(om[cur], P.p_pad, Omega_seq + t * p * p, p, p, p, nullptr, st);
    }
    launch_copy_cols(om[cur], P.p_pad, Omega, p, p, p, nullptr, st);
    HIP_TRY(hipGetLastError());
    return ACCORD_OK;
}

int accord_val_loss_grad(const float* Xv, int64_t nv, int64_t p, const float* Omega, double* out,
                         float* Obar, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    TRY(check_dims(nv, p));
    TRY(check_ptr(Xv, "Xv"));
    TRY(check_ptr(Omega, "Omega"));
    TRY(check_ptr(Obar, "Obar"));
    if (!out || !aligned(out, 8)) return fail(ACCORD_ERR_INVALID_ARG, "out must be non-null, 8-byte aligned");
    const Plan P = make_plan(nv, p, 1, PREC_FP32);
    TRY(check_ws(ws, ws_bytes, P.end_grad));
    hipStream_t st = (hipStream_t)stream;
    TRY(enqueue_w(P, Xv, Omega, ws, st));
    const float* wt = at<float>(ws, P.off_wt0);
    launch_gemm(grad_args(P, ws, PREC_FP32, wt, 0, Obar, p, (int)p, nullptr), EPI_GRAD, PREC_FP32, st);
    launch_sub_inv_diag(Obar, p, at<float>(ws, P.off_om0), P.p_pad, p, st);
    ProxArgs a = {};
    a.om = at<float>(ws, P.off_om0);
    a.total = p * P.p_pad;
    a.ld = P.p_pad;
    a.p = p;
    a.part = at<double>(ws, P.off_prox_part);
    a.reduce_only = 1;
    launch_prox(a, P.nprox, st);
    launch_combine_objective(a.part, P.nprox, at<double>(ws, P.off_norm_part), P.t32.tiles(), 0.0,
                             1.0 / (double)nv, out, st);
    HIP_TRY(hipGetLastError());
    return ACCORD_OK;
}

int accord_fbs_adjoint_step(const float* X, int64_t n, int64_t p, const float* Omega_t, double tau,
                            double lambda, float* Obar, double* lbar, float* Xbar, void* ws,
                            size_t ws_bytes, void* stream) {
    g_last_error.clear();
    TRY(check_dims(n, p));
    TRY(check_ptr(X, "X"));
    TRY(check_ptr(Omega_t, "Omega_t"));
    TRY(check_ptr(Obar, "Obar"));
    TRY(check_ptr(Xbar, "Xbar"));
    if (!lbar || !aligned(lbar, 8)) return fail(ACCORD_ERR_INVALID_ARG, "lbar must be non-null, 8-byte aligned");
    if (!(tau > 0.0) || !isfinite(tau)) return fail(ACCORD_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (!(lambda >= 0.0) || !isfinite(lambda))
        return fail(ACCORD_ERR_INVALID_ARG, "lambda must be finite and >= 0");
    const AdjPlan A = make_adj_plan(n, p);
    const Plan& P = A.P;
    TRY(check_ws(ws, ws_bytes, A.end));
    hipStream_t st = (hipStream_t)stream;
    const int64_t k2 = 2 * P.p_pad;
    float* om = at<float>(ws, P.off_om0);
    float* wt0 = at<float>(ws, P.off_wt0);
    float* wt1 = at<float>(ws, P.off_wt1);
    float* G = at<float>(ws, P.off_g);
    float* abar = at<float>(ws, P.off_d);
    float* AT = at<float>(ws, A.off_at);
    float* BW = at<float>(ws, A.off_bw);
    double* part = at<double>(ws, A.off_adjpart);
    // forward quantities of step t: W = X Omega_t, G = S Omega_t (the same kernels and
    // inputs as the replay, so the same bits)
    TRY(enqueue_w(P, X, Omega_t, ws, st));
    launch_gemm(grad_args(P, ws, PREC_FP32, wt0, 0, G, P.p_pad, (int)P.p_pad, nullptr), EPI_GRAD,
                PREC_FP32, st);
    // through the prox: Abar and the lambda derivative
    AdjArgs a = {};
    a.om = om;
    a.g = G;
    a.obar = Obar;
    a.ld = P.p_pad;
    a.ld_obar = p;
    a.p = p;
    a.tau = tau;
    a.lambda = lambda;
    a.abar = abar;
    a.part = part;
    launch_prox_adjoint(a, kAdjBlocks, st);
    launch_accumulate_scalar(part, kAdjBlocks, lbar, st);
    // V = X Abar (W^T layout), then S Abar = X^T V / n into G
    enqueue_trial(trial_args(P, ws, PREC_FP32, abar, nullptr, nullptr, nullptr, wt1, -1, nullptr, 0),
                  PREC_FP32, st);
    launch_gemm(grad_args(P, ws, PREC_FP32, wt1, 0, G, P.p_pad, (int)P.p_pad, nullptr), EPI_GRAD,
                PREC_FP32, st);
    // Omega_t bar = Abar - tau S Abar  (written over Obar)
    launch_adjoint_combine(abar, G, P.p_pad, p, (float)tau, Obar, p, st);
    // X bar += -(tau/n) (W Abar^T + V Omega_t^T) as one product with K = 2 p_pad:
    // rows i of [Abar | Omega_t] against rows m of [W | V]
    HIP_TRY(hipMemsetAsync(AT, 0, (size_t)(P.p_pad * k2) * sizeof(float), st));
    HIP_TRY(hipMemsetAsync(BW, 0, (size_t)(P.n_pad * k2) * sizeof(float), st));
    launch_transpose_ld(abar, P.p_pad, p, p, AT, k2, st);
    launch_transpose_ld(om, P.p_pad, p, p, AT + P.p_pad, k2, st);
    launch_transpose_ld(wt0, P.n_pad, p, n, BW, k2, st);
    launch_transpose_ld(wt1, P.n_pad, p, n, BW + P.p_pad, k2, st);
    GemmArgs x = {};
    x.A = AT;
    x.lda = k2;
    x.B = BW;
    x.ldb = k2;
    x.M = (int)p;
    x.N = (int)n;
    x.K = (int)k2;
    x.tilesM = A.gx.tilesM;
    x.tilesN = A.gx.tilesN;
    x.splits = A.gx.splits;
    x.C = Xbar;
    x.ldc = p;
    x.vec_store = (p % 4 == 0) && aligned(Xbar, 16);
    x.alpha = (float)(-tau / (double)n);
    x.Wprev = Xbar;
    x.P = A.gx.splits > 1 ? at<float>(ws, A.off_xsplit) : nullptr;
    x.norm_part = at<double>(ws, A.off_xnorm);
    x.Mvalid = (int)p;
    x.Nvalid = (int)n;
    enqueue_trial(x, PREC_FP32, st);
    HIP_TRY(hipGetLastError());
    return ACCORD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free prox: the FP64 partial sums of accord_prox go to a file-scope
// device array instead of the caller's workspace.  Each GPU holds its own copy of
// the array; its address on a device comes from hipGetSymbolAddress (the array's
// name in host code is only a host-side stand-in) and is looked up once per device.
// ---------------------------------------------------------------------------
namespace {
constexpr int kScratchRows = kMaxProxBlocks;             // prox workgroups of one call, at most
constexpr int kScratchDoubles = kScratchRows * kPartCols;  // 256 KiB
constexpr int kMaxScratchDevices = 64;
}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxScratchDevices];  // device address of `scratch` on each GPU

int scratch_on_current_device(double** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(ACCORD_ERR_UNSUPPORTED, "device index %d beyond the %d devices supported",
                    dev, kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(ACCORD_ERR_HIP, "no device address for the prox scratch array");
        g_scratch_dev[dev] = (double*)ptr;
    }
    *out = g_scratch_dev[dev];
    return ACCORD_OK;
}

}  // namespace

extern "C" {

int accord_prox_noalloc(const float* Omega, const float* G, int64_t p, double tau,
                        double lambda, float* Omega_out, double* red, void* stream) {
    g_last_error.clear();
    TRY(check_prox_args(Omega, G, p, tau, lambda, Omega_out, red));
    const int nb = prox_blocks(p * p);
    if (nb > kScratchRows)
        return fail(ACCORD_ERR_INVALID_ARG, "p=%lld needs %d partial rows; the scratch array "
                    "holds %d", (long long)p, nb, kScratchRows);
    double* part = nullptr;
    TRY(scratch_on_current_device(&part));
    return enqueue_prox(Omega, G, p, tau, lambda, Omega_out, red, part, (hipStream_t)stream);
}

}  // extern "C"
