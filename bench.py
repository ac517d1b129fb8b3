"""Benchmark of the ACCORD-FBS hot path on one MI355X.

One step = one complete accord_fit (Alg. 1) on the block power-law workload
n = 500, p = 5000 (10 Barabasi-Albert(m=1) blocks of 500, lambda = 0.05,
500 iterations, FP32 contractions, L estimated on the device by power iteration).
X is resident in HBM before the timed region.  `value` = prox-grad iterations per
second over the K timed steps.

Also reported:
  roofline      the dominant kernel's achieved FLOP rate (algorithmic 2 n p^2 flops
                per launch / its mean HIP-event duration over the timed region, on the
                stream the kernels are launched on) against the FP32 matrix peak
  kernels       the same for every hot-path kernel
  error_vs_oracle  relative Frobenius error of sampled columns of the final iterate
                against the FP64 oracle replaying the GPU's step sizes (untimed)
  cpu_baseline  the FP64 oracle timed on this host on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 matrix/vector peak
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
METRIC = "prox-grad iters/sec + X^T(XΩ) MFMA TFLOP/s, mixed vs FP32 at matched error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, iters_budget_s: float = 15.0):
    """The FP64 oracle (numpy/OpenBLAS) on the same workload, first few iterations."""
    import oracle

    x = w.X.astype(np.float64)
    L = oracle.lipschitz(x)
    t0 = time.perf_counter()
    r = oracle.fit_fbs(x, w.lam, 1, L=L)
    one = time.perf_counter() - t0
    k = max(1, min(20, int(iters_budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    r = oracle.fit_fbs(x, w.lam, k, L=L)
    dt = time.perf_counter() - t0
    threads = os.cpu_count()
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        if info:
            threads = max(i.get("num_threads", 0) for i in info) or threads
    except Exception:
        pass
    return {"value": k / dt, "unit": "iters/s", "cores": threads, "kind": "oracle",
            "sample": f"first {k} iterations of the same n={w.n}, p={w.p} fit "
                      f"({sum(r.trials)} backtracking trials, {dt:.1f} s, FP64 numpy)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the estimator's columns shard across GPUs, but no multi-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import datagen
    from paper_2412_11554_amd import accord

    dev = torch.device("cuda:0")
    w = datagen.workload("ba5000")
    n, p, iters = w.n, w.p, w.iters
    X = torch.from_numpy(w.X).to(dev)
    ws = torch.empty(accord.accord_workspace_bytes(n, p, accord.default_params(max_iter=iters)),
                     dtype=torch.uint8, device=dev)
    om = torch.empty((p, p), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    def step(timing: bool):
        return accord.accord_fit(X, w.lam, iters, ws=ws, omega_out=om, timing=timing,
                                 trace=True)

    for i in range(args.warmup):
        step(False)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    all_stats = []
    last_trace = None
    for i in range(args.steps):
        _, st, last_trace = step(True)
        all_stats.append(st)
        log(f"step {i + 1}/{args.steps}: {st['iters']} iters, {st['trials']} trials, "
            f"{st['total_ms']:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    total_iters = sum(s["iters"] for s in all_stats)
    value = total_iters / elapsed
    flops = 2.0 * n * p * p          # per GEMM launch, both contractions

    def agg(key_ms, key_n):
        ms = sum(s[key_ms] for s in all_stats)
        cnt = sum(s[key_n] for s in all_stats)
        return ms, cnt

    g_ms, g_n = agg("grad_gemm_ms", "grad_gemm_launches")
    t_ms, t_n = agg("trial_gemm_ms", "trial_gemm_launches")
    p_ms, p_n = agg("prox_ms", "prox_launches")
    kernels = {}
    if g_n:
        a = flops / (g_ms / g_n * 1e-3) / 1e12
        kernels["grad_gemm"] = {"what": "G = X^T W / n", "launches": g_n, "avg_ms": g_ms / g_n,
                                "achieved": a, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                "frac": a / PEAK_FP32_TFLOPS, "bound": "mfma",
                                "total_ms": g_ms}
    if t_n:
        a = flops / (t_ms / t_n * 1e-3) / 1e12
        kernels["trial_gemm"] = {"what": "W+ = W + X Delta (+ norms)", "launches": t_n,
                                 "avg_ms": t_ms / t_n, "achieved": a, "peak": PEAK_FP32_TFLOPS,
                                 "unit": "TFLOP/s", "frac": a / PEAK_FP32_TFLOPS, "bound": "mfma",
                                 "total_ms": t_ms}
    if p_n:
        bytes_per = 16.0 * p * (p + (-p) % 32)  # read Omega, G; write Omega+, Delta (FP32)
        a = bytes_per / (p_ms / p_n * 1e-3) / 1e9
        kernels["prox"] = {"what": "fused prox + reductions", "launches": p_n,
                           "avg_ms": p_ms / p_n, "achieved": a, "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": a / PEAK_HBM_GBS, "bound": "hbm",
                           "total_ms": p_ms}
    dom_name = max(kernels, key=lambda k: kernels[k]["total_ms"]) if kernels else None
    roofline = None
    if dom_name:
        d = kernels[dom_name]
        roofline = {"kernel": dom_name, "bound": d["bound"], "achieved": d["achieved"],
                    "peak": d["peak"], "unit": d["unit"], "frac": d["frac"], "traffic": None}
    xtw = kernels.get("grad_gemm", {}).get("achieved")

    err = None
    if not args.no_check:
        import oracle
        cols = np.array([0, 1, 499, 2500, 4998, 4999])
        taus = last_trace.cpu().numpy()[1:, 3]
        ref = oracle.fit_fbs(w.X.astype(np.float64), w.lam, len(taus),
                             L=all_stats[-1]["lipschitz"], tau_replay=taus, columns=cols)
        got = om.cpu().numpy()[cols, :].astype(np.float64).T
        err = {"rel_fro_sampled_cols": float(np.linalg.norm(got - ref.omega) /
                                             np.linalg.norm(ref.omega)),
               "cols": cols.tolist(), "reference": "FP64 oracle replaying the GPU step sizes"}

    cpu = None if args.no_cpu_baseline else cpu_baseline(w)

    st = all_stats[-1]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"block power-law ACCORD-FBS fit: n={n}, p={p}, "
                               f"10 BA(m=1) blocks of 500, lambda={w.lam}, {iters} iterations",
                   "n": n, "p": p, "lambda": w.lam, "iters_per_step": iters,
                   "precision": "fp32 (FP64 reductions, FP64 diagonal root)",
                   "lipschitz": "device power iteration, 200 steps"},
        "xtw_tflops": xtw,
        "trials_per_iter": st["trials"] / max(1, st["iters"]),
        "roofline": roofline,
        "kernels": kernels,
        "error_vs_oracle": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
