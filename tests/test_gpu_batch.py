"""GPU parity of the batched form (accord_fit_batch): many independent fits, each
checked against the FP64 oracle replaying that problem's accepted steps.

Every problem runs Alg. 1 on its own (own step, acceptance and stop), so the bar is
the FP32 one of the single fit: relative Frobenius error <= 1e-4 per problem.  The
steps come back as per-iteration trial counts (tau_t = tau0 beta^(trials_t - 1)).
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def _taus(trials_row, iters, tau0=1.0, beta=0.5):
    return tau0 * beta ** (np.asarray(trials_row[:iters], dtype=np.float64) - 1)


def _run(gpu_lib, w, iters, **kw):
    import torch
    X = torch.from_numpy(w.stacked()).cuda()
    om, stats, tr = gpu_lib.accord_fit_batch(X, w.n, w.lams, iters, trials=True, **kw)
    torch.cuda.synchronize()
    return om, stats, tr.cpu().numpy()


def _check_problem(w, k, om_k, stats_k, trials_k, L, cols=None, tol=0.0):
    nlam = len(w.lams)
    b, l = divmod(k, nlam)
    x = w.xs[b].astype(np.float64)
    taus = _taus(trials_k, stats_k["iters"])
    ref = oracle.fit_fbs(x, w.lams[l], len(taus), L=L, tau_replay=taus, columns=cols)
    got = om_k.T if cols is None else om_k[cols, :].T
    return np.linalg.norm(got - ref.omega) / np.linalg.norm(ref.omega)


def test_batch_small_all_problems(gpu_lib):
    """3 data sets (n = 40..130 rows of one p = 200 base sample) x 4 penalties,
    40 iterations, exact L per data set."""
    w = datagen.batch_workload(p=200, nsub=3, nlam=4, n_base=150, lo=40, hi=130, prob=0.02,
                               lam_lo=0.05, lam_hi=0.3, iters=40, key=31)
    Ls = [oracle.lipschitz(x.astype(np.float64)) for x in w.xs]
    om, stats, tr = _run(gpu_lib, w, w.iters, lipschitz=Ls)
    om = om.cpu().numpy().astype(np.float64)
    for k in range(len(stats)):
        assert stats[k]["iters"] == w.iters
        assert stats[k]["lipschitz"] == pytest.approx(Ls[k // len(w.lams)], rel=1e-12)
        rel = _check_problem(w, k, om[k], stats[k], tr[k], Ls[k // len(w.lams)])
        assert rel <= 1e-4, (k, rel)
        # each problem's own line search: tau = tau0 beta^(k-1), at or above the floor
        assert np.all(tr[k, :w.iters] >= 1)
        assert np.all(_taus(tr[k], w.iters) >= 0.5 / Ls[k // len(w.lams)] * (1 - 1e-12))
    # problems differ (the batch really holds distinct fits)
    assert len({round(s["f"], 6) for s in stats}) == len(stats)


@pytest.mark.parametrize("p,ns", [(150, [1, 33, 65]), (130, [64, 65])])
def test_batch_ragged(gpu_lib, p, ns):
    """p not a multiple of the 128-column tile, tiny and ragged n (n = 1: rank one), L by
    the device's Lanczos estimate (the step count asked for is capped at 256)."""
    rng = np.random.default_rng(p)
    xs = [rng.normal(size=(n, p)).astype(np.float32) for n in ns]
    w = datagen.BatchWorkload("ragged", p, xs, np.array([0.08, 0.2, 0.5]), 12)
    om, stats, tr = _run(gpu_lib, w, w.iters, power_iters=2000)
    om = om.cpu().numpy().astype(np.float64)
    for k in range(len(stats)):
        b = k // len(w.lams)
        L = oracle.lipschitz(xs[b].astype(np.float64))
        assert abs(stats[k]["lipschitz"] - L) <= 1e-6 * L
        rel = _check_problem(w, k, om[k], stats[k], tr[k], stats[k]["lipschitz"])
        assert rel <= 1e-4, (k, rel)


def test_batch_stop_rule_per_problem(gpu_lib):
    """With a tolerance, problems stop at different iterations; each result is the
    iterate at its own stop."""
    w = datagen.batch_workload(p=120, nsub=2, nlam=3, n_base=100, lo=60, hi=100, prob=0.03,
                               lam_lo=0.1, lam_hi=0.6, iters=400, key=32)
    Ls = [oracle.lipschitz(x.astype(np.float64)) for x in w.xs]
    om, stats, tr = _run(gpu_lib, w, w.iters, lipschitz=Ls, tol=1e-5)
    om = om.cpu().numpy().astype(np.float64)
    iters = [s["iters"] for s in stats]
    assert all(s["converged"] == 1 for s in stats)
    assert len(set(iters)) > 1 and max(iters) < w.iters
    for k in range(len(stats)):
        rel = _check_problem(w, k, om[k], stats[k], tr[k], Ls[k // len(w.lams)])
        assert rel <= 1e-4, (k, rel)


def test_batch_full_size_sampled(gpu_lib):
    """16 bootstrap subsamples (n in 100..400) x 32 penalties in [0.02, 0.5] at
    p = 2000, 300 iterations, L by the Lanczos estimate: 34 problems (every subsample at
    the smallest and the largest penalty, and two more) on 24 columns each against the
    oracle replaying their steps."""
    w = datagen.workload("batch")
    print(f"batch: {len(w.xs)} x {len(w.lams)} problems, p={w.p}, {w.iters} iterations",
          flush=True)
    om, stats, tr = _run(gpu_lib, w, w.iters)
    assert all(s["iters"] == w.iters for s in stats)
    cols = np.r_[np.arange(0, 2000, 100), [1, 999, 1998, 1999]]
    nlam = len(w.lams)
    probs = [b * nlam for b in range(len(w.xs))] + [b * nlam + nlam - 1 for b in range(len(w.xs))]
    for k in probs + [5 * nlam + 13, 9 * nlam + 2]:
        b = k // nlam
        L = oracle.lipschitz(w.xs[b].astype(np.float64))
        assert L * (1 - 1e-3) <= stats[k]["lipschitz"] <= L * (1 + 1e-9)
        rel = _check_problem(w, k, om[k].cpu().numpy().astype(np.float64), stats[k], tr[k],
                             stats[k]["lipschitz"], cols=cols)
        print(f"problem {k}: lambda {w.lams[k % nlam]:.4f} n {w.n[b]} rel {rel:.2e}", flush=True)
        assert rel <= 1e-4, (k, rel)
    # larger penalties give sparser estimates along each path
    nnz = np.array([s["nnz_offdiag"] for s in stats]).reshape(len(w.xs), nlam)
    assert np.all(nnz[:, 0] > nnz[:, -1])


def test_batch_full_size_deterministic(gpu_lib):
    """The benchmark's 16 x 32 problems at p = 2000, 10 iterations, twice (the second
    through the captured graphs): the same bits."""
    import torch
    w = datagen.workload("batch")
    X = torch.from_numpy(w.stacked()).cuda()
    print(f"[determinism] batch {len(w.xs)} x {len(w.lams)} problems, p={w.p}, 10 iterations "
          "twice", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a, sa, ta = gpu_lib.accord_fit_batch(X, w.n, w.lams, 10, trials=True)
        a, ta = a.clone(), ta.clone()
        b, sb, tb = gpu_lib.accord_fit_batch(X, w.n, w.lams, 10, trials=True, graph=True)
        s.synchronize()
    assert torch.equal(a, b) and torch.equal(ta, tb)
    assert [d["f"] for d in sa] == [d["f"] for d in sb]


def test_batch_tile_orders_are_bit_identical(gpu_lib):
    """Every launch code of the batched kernels (params.batch_order, codes 1..20 for the
    gradient and the trial kernel: 10 tile orders at two and at one workgroups per CU)
    gives the default's bits: a code decides only which workgroup computes which tile and
    the register budget the kernel is compiled for."""
    import torch
    w = datagen.batch_workload(p=300, nsub=3, nlam=4, n_base=120, lo=40, hi=120, prob=0.02,
                               iters=20, key=35)
    X = torch.from_numpy(w.stacked()).cuda()
    ref, st_ref, tr_ref = gpu_lib.accord_fit_batch(X, w.n, w.lams, w.iters, trials=True)
    ref, tr_ref = ref.clone(), tr_ref.clone()
    for c in range(1, gpu_lib.BATCH_ORDERS + 1):
        code = c | ((gpu_lib.BATCH_ORDERS + 1 - c) << 8)
        om, st, tr = gpu_lib.accord_fit_batch(X, w.n, w.lams, w.iters, trials=True,
                                              batch_order=code)
        torch.cuda.synchronize()
        assert torch.equal(om, ref) and torch.equal(tr, tr_ref), code
        assert [d["f"] for d in st] == [d["f"] for d in st_ref]


def test_batch_autotune_full_size(gpu_lib):
    """The autotuner on the benchmark's 16 x 32 problems at p = 2000: a valid order code
    from timings of all 40 candidates, and a fit in that order equal to the default."""
    import torch
    w = datagen.workload("batch")
    X = torch.from_numpy(w.stacked()).cuda()
    print(f"[tune] batch {len(w.xs)} x {len(w.lams)} problems, p={w.p}", flush=True)
    code, table = gpu_lib.accord_tune_batch(X, w.n, w.lams)
    g, t = code & 0xff, code >> 8
    print(f"[tune] order code {code}: gradient {g} ({min(table['grad']):.2f} ms), trial {t} "
          f"({min(table['trial']):.2f} ms); default {table['grad'][3]:.2f} / "
          f"{table['trial'][3]:.2f} ms", flush=True)
    assert 1 <= g <= gpu_lib.BATCH_ORDERS and 1 <= t <= gpu_lib.BATCH_ORDERS
    # every candidate did the work: a gradient over 512 problems at p = 2000 is about
    # 1e12 flops, a trial (all problems searching) as much
    assert all(v > 1.0 for v in table["grad"] + table["trial"]), table
    assert table["grad"][g - 1] == min(table["grad"]) and table["trial"][t - 1] == min(table["trial"])
    a, sa, ta = gpu_lib.accord_fit_batch(X, w.n, w.lams, 8, trials=True)
    a, ta = a.clone(), ta.clone()
    b, sb, tb = gpu_lib.accord_fit_batch(X, w.n, w.lams, 8, trials=True, batch_order=code)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ta, tb)


def test_batch_errors(gpu_lib):
    import torch
    from paper_2412_11554_amd import accord
    w = datagen.batch_workload(p=64, nsub=2, nlam=2, n_base=50, lo=20, hi=40, prob=0.05,
                               iters=5, key=33)
    X = torch.from_numpy(w.stacked()).cuda()
    om0 = torch.eye(64).repeat(4, 1, 1).cuda()
    om0[3, 5, 5] = -1.0
    with pytest.raises(accord.AccordError) as e:
        gpu_lib.accord_fit_batch(X, w.n, w.lams, 5, omega0=om0)
    assert e.value.status == 2 and "problem 3" in str(e.value)
    Xbad = X.clone()
    Xbad[w.n[0] + 2, 7] = float("nan")
    with pytest.raises(accord.AccordError) as e:
        gpu_lib.accord_fit_batch(Xbad, w.n, w.lams, 5)
    assert e.value.status == 3


def test_batch_graph_replay_matches_eager(gpu_lib):
    """The captured sweeps (params.graph) replay the same kernels on the same device
    state: results equal the eagerly enqueued run bit for bit, on two calls in a row
    (fresh capture each call) with eager work and synchronisation in between."""
    import torch
    w = datagen.batch_workload(p=130, nsub=2, nlam=3, n_base=90, lo=40, hi=90, prob=0.03,
                               iters=25, key=34)
    X = torch.from_numpy(w.stacked()).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ref, st_ref, tr_ref = gpu_lib.accord_fit_batch(X, w.n, w.lams, w.iters, trials=True)
        ref, tr_ref = ref.clone(), tr_ref.clone()
        for rep in range(2):
            om, st, tr = gpu_lib.accord_fit_batch(X, w.n, w.lams, w.iters, trials=True, graph=True)
            s.synchronize()
            assert torch.equal(om, ref), rep
            assert torch.equal(tr, tr_ref), rep
            assert [d["f"] for d in st] == [d["f"] for d in st_ref]
            assert [d["iters"] for d in st] == [d["iters"] for d in st_ref]
            # eager work on the same stream between the graph calls
            _ = (X * 2.0).sum().item()
    s.synchronize()
