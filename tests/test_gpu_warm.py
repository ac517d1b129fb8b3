"""GPU parity of the warm-started step variant (params.warm_tau = 1): each iteration's
first trial is min(tau0, tau_{t-1} / beta) instead of tau0.  It departs from Alg. 1,
so it is never the parity path of the plain fit; here it is checked on its own terms
against the oracle's variant (fit_fbs(warm_tau=True), pinned in P13).

Bars as the plain fit: the oracle replays the device's accepted steps, relative
Frobenius error <= 1e-4 (FP32, BF16x3); the trace obeys the variant's step rule
exactly; the oracle's own decisions agree with the device's until a near-tie.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _warm_rule_holds(taus, trials, tau0=1.0, beta=0.5):
    start = tau0
    for t, (tau, k) in enumerate(zip(taus, trials)):
        if t > 0:
            start = min(tau0, taus[t - 1] / beta)
        if tau != start * beta ** (int(k) - 1):
            return False
    return True


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_warm_small_workload(gpu_lib, prec):
    w = datagen.workload("er200")
    x = w.X.astype(np.float64)
    L = oracle.lipschitz(x)
    om, st, tr = gpu_lib.accord_fit(_dev(w.X), w.lam, w.iters, lipschitz=L, trace=True,
                                    precision=prec, warm_tau=True)
    tr = tr.cpu().numpy()
    taus, trials = tr[1:, 3], tr[1:, 4]
    assert st["iters"] == w.iters
    assert _warm_rule_holds(taus, trials)
    ref = oracle.fit_fbs(x, w.lam, len(taus), L=L, tau_replay=taus)
    got = om.cpu().numpy().astype(np.float64).T
    rel = np.linalg.norm(got - ref.omega) / np.linalg.norm(ref.omega)
    own = oracle.fit_fbs(x, w.lam, w.iters, L=L, warm_tau=True)
    agree = int(np.argmax(~np.isclose(taus, own.tau))) if not np.allclose(taus, own.tau) else len(taus)
    plain = gpu_lib.accord_fit(_dev(w.X), w.lam, w.iters, lipschitz=L, precision=prec)[1]
    print(f"{prec}: rel {rel:.2e}; trials {st['trials']} (plain {plain['trials']}); "
          f"oracle's own steps agree for {agree} of {len(taus)} iterations", flush=True)
    assert rel <= 1e-4
    assert np.all(np.diff(tr[:, 0]) <= 1e-6 * np.abs(tr[1:, 0]))
    assert agree >= 20
    assert st["trials"] < plain["trials"]


def test_warm_benchmark_shape_sampled(gpu_lib):
    """n = 500, p = 5000, 500 iterations, BF16x3 (the benchmarked form)."""
    w = datagen.workload("ba5000")
    om, st, tr = gpu_lib.accord_fit(_dev(w.X), w.lam, w.iters, trace=True, precision="bf16x3",
                                    warm_tau=True)
    tr = tr.cpu().numpy()
    taus = tr[1:, 3]
    assert _warm_rule_holds(taus, tr[1:, 4])
    cols = np.array([0, 1, 499, 2500, 4998, 4999])
    ref = oracle.fit_fbs(w.X.astype(np.float64), w.lam, len(taus), L=st["lipschitz"],
                         tau_replay=taus, columns=cols)
    got = om.cpu().numpy()[cols, :].astype(np.float64).T
    rel = np.linalg.norm(got - ref.omega) / np.linalg.norm(ref.omega)
    print(f"ba5000 bf16x3 warm: {st['trials'] / st['iters']:.3f} trials per iteration, "
          f"rel {rel:.2e}", flush=True)
    assert rel <= 1e-4


def test_warm_batched(gpu_lib):
    """Batched form with the variant: each problem's steps follow the rule and replay."""
    import torch
    w = datagen.batch_workload(p=150, nsub=2, nlam=3, n_base=100, lo=50, hi=100, prob=0.03,
                               lam_lo=0.05, lam_hi=0.4, iters=40, key=51)
    Ls = [oracle.lipschitz(x.astype(np.float64)) for x in w.xs]
    X = torch.from_numpy(w.stacked()).cuda()
    om, stats, tr = gpu_lib.accord_fit_batch(X, w.n, w.lams, w.iters, trials=True, lipschitz=Ls,
                                             warm_tau=True)
    tr = tr.cpu().numpy()
    om = om.cpu().numpy().astype(np.float64)
    nlam = len(w.lams)
    for k, s in enumerate(stats):
        b, l = divmod(k, nlam)
        taus, start = [], 1.0
        for t in range(s["iters"]):
            if t > 0:
                start = min(1.0, taus[-1] / 0.5)
            taus.append(start * 0.5 ** (int(tr[k, t]) - 1))
        ref = oracle.fit_fbs(w.xs[b].astype(np.float64), w.lams[l], len(taus), L=Ls[b],
                             tau_replay=taus)
        rel = np.linalg.norm(om[k].T - ref.omega) / np.linalg.norm(ref.omega)
        assert rel <= 1e-4, (k, rel)
        assert s["tau_last"] == taus[-1]
