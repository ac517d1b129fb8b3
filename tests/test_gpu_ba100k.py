"""Parity at the largest single-GPU size: n = 1000, p = 100000 (200 power-law blocks
of 500, lambda = 0.03), through accord_fit in the configuration a full fit uses
(split-K choice, tile geometry and workspace layout all come from n and p).

The oracle replays the device's step sizes on a sample of columns: once the steps
are fixed, each column of the iterate evolves on its own (the objective separates
over columns), so the FP64 reference costs |J| columns of the p = 1e5 problem.
A few iterations keep the oracle and the device run within seconds; every kernel
of the iteration runs at its full size in each of them.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

COLS = np.array([0, 1, 2, 499, 500, 31337, 50000, 77777, 99998, 99999])
ITERS = {"bf16x3": 6, "fp32": 3, "bf16x1": 3, "fp8": 1}
# relative Frobenius error of the sampled columns: the FP32 bar for fp32 and the
# split-precision form; bf16 unit roundoff (2^-8 relative) for the single-pass form
TOL = {"bf16x3": 1e-4, "fp32": 1e-4, "bf16x1": 5e-2}
# fp8: one fixed step, compared with the MX oracle (same operand rounding) at the
# one-step bar derived in tests/test_gpu_fp8.py
TOL_MX = 1e-4


@pytest.fixture(scope="module")
def big(gpu_lib, ba100k):
    import torch

    from paper_2412_11554_amd import accord

    _, total = torch.cuda.mem_get_info()
    w = ba100k["w"]
    need = max(accord.accord_workspace_bytes(
        w.n, w.p, accord.default_params(max_iter=max(ITERS.values()), precision=f))
        for f in ITERS)
    if need + 4 * w.p * w.p + (8 << 30) > total:
        pytest.skip(f"device holds {total / 1e9:.0f} GB; n=1000, p=1e5 needs "
                    f"{(need + 4 * w.p * w.p) / 1e9:.0f} GB")
    X = torch.from_numpy(w.X).cuda()
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    om = torch.empty((w.p, w.p), dtype=torch.float32, device="cuda")
    yield {"w": w, "X": X, "ws": ws, "om": om, "x64": ba100k["x64"], "L": ba100k["L"]}
    del X, ws, om
    torch.cuda.empty_cache()


@pytest.mark.parametrize("form", ["bf16x3", "fp32", "bf16x1"])
def test_ba100k_sampled_columns(big, form):
    from paper_2412_11554_amd import accord

    w = big["w"]
    T = ITERS[form]
    print(f"[big] {form}: accord_fit n={w.n} p={w.p} iters={T}", flush=True)
    om, st, tr = accord.accord_fit(big["X"], w.lam, T, precision=form, trace=True,
                                   ws=big["ws"], omega_out=big["om"])
    # 782 column blocks: the trial products run the last 14 (the fused forms: past three
    # whole rounds of 256 workgroups; FP32: past 768 x 8 tiles, 12 rounds of 512) as a
    # split-K tail launch, and COLS samples columns 99998, 99999 of it
    assert st["tail_blocks"] == 14 and st["tail_splits"] == (4 if form == "fp32" else 16), (
        st["tail_blocks"], st["tail_splits"])
    _check_sampled(big, form, om, st, tr)


def test_ba100k_fp8_fixed_step(big):
    """FP8: one fixed step (beta = 1, tau = 1/64) from the identity."""
    from paper_2412_11554_amd import accord
    w = big["w"]
    print(f"[big] fp8: accord_fit n={w.n} p={w.p} one fixed step", flush=True)
    om, st, tr = accord.accord_fit(big["X"], w.lam, 1, precision="fp8", trace=True,
                                   tau0=1.0 / 64, beta=1.0, ws=big["ws"], omega_out=big["om"])
    _check_sampled(big, "fp8", om, st, tr)


def test_ba100k_bf16x3_deterministic(big):
    """Two 2-iteration BF16x3 fits at n = 1000, p = 1e5 give the same bits."""
    import torch
    from paper_2412_11554_amd import accord
    w = big["w"]
    print(f"[big] bf16x3 twice, 2 iterations, n={w.n} p={w.p}", flush=True)
    _, sa, ta = accord.accord_fit(big["X"], w.lam, 2, precision="bf16x3", trace=True,
                                  ws=big["ws"], omega_out=big["om"])
    def bit_sums(om):
        # int64 sums of the FP32 bit patterns, 5000 columns at a time (any changed bit
        # changes its chunk's sum unless differences cancel exactly)
        return [int(om[r:r + 5000].view(torch.int32).to(torch.int64).sum())
                for r in range(0, om.shape[0], 5000)]

    cols = np.array([0, 777, 50000, 99999])
    first = big["om"][cols, :].clone()
    h1 = bit_sums(big["om"])
    _, sb, tb = accord.accord_fit(big["X"], w.lam, 2, precision="bf16x3", trace=True,
                                  ws=big["ws"], omega_out=big["om"])
    h2 = bit_sums(big["om"])
    assert torch.equal(first, big["om"][cols, :]) and torch.equal(ta, tb)
    assert h1 == h2 and sa["f"] == sb["f"]


def test_ba100k_probe_is_the_full_trial(big):
    """Three BF16x3 iterations with trials tested on their first 256 samples and then
    after each further tile of 256 (and, after a trial of an iteration fails the full
    test or a late partial test, the later ones unprobed) equal those that always run the
    whole product, bit for bit (checked by column-chunk sums of the FP32 bit patterns and
    on sampled columns), with the same trial counts."""
    import torch
    from paper_2412_11554_amd import accord
    w = big["w"]

    def bit_sums(om):
        return [int(om[r:r + 5000].view(torch.int32).to(torch.int64).sum())
                for r in range(0, om.shape[0], 5000)]

    cols = np.array([0, 777, 50000, 99999])
    runs = []
    for probe in (True, False):
        print(f"[big] bf16x3 3 iterations, probe {probe}", flush=True)
        _, st, tr = accord.accord_fit(big["X"], w.lam, 3, precision="bf16x3", trace=True,
                                      ws=big["ws"], omega_out=big["om"], probe=probe)
        runs.append((st, tr.clone(), big["om"][cols, :].clone(), bit_sums(big["om"])))
    (sa, ta, ca, ha), (sb, tb, cb, hb) = runs
    print(f"[big] trials {sa['trials']} (probe: {sa['probe_rejects']} rejected by partial "
          f"tests after {sa['probe_mtiles']} M tiles, {sa['unprobed_trials']} unprobed) "
          f"vs {sb['trials']}", flush=True)
    assert sb["probe_rejects"] == 0 and sb["unprobed_trials"] == 0
    assert sa["trials"] == sb["trials"] and torch.equal(ta, tb)
    assert torch.equal(ca, cb) and ha == hb


def _check_sampled(big, form, om, st, tr):
    import oracle
    from oracle import mx_oracle
    w = big["w"]
    T = ITERS[form]
    assert st["iters"] == T
    trace = tr.cpu().numpy()
    taus = trace[1:, 3]
    # steps are tau0 * beta^k
    k = np.log2(taus)
    assert np.allclose(k, np.round(k)) and np.all(taus <= 1.0)
    # device Lanczos estimate: top Ritz value plus its residual bound, so never below
    # sigma_max beyond rounding, and within 1e-10 once the bound is met
    assert st["lipschitz"] >= big["L"] * (1 - 1e-13)
    assert abs(st["lipschitz"] - big["L"]) <= 1e-10 * big["L"]
    f = trace[:, 0]
    assert np.all(np.isfinite(f))
    if form == "fp8":
        # (the FP8 form carries W + X q(Delta), not X Omega+, so its traced g is not
        # that of the iterate and need not decrease)
        assert np.all(taus == 1.0 / 64)
        ref = mx_oracle.fit_fbs_mx(big["x64"], w.lam, taus, columns=COLS)
    else:
        # the objective does not increase (sufficient decrease of the accepted steps),
        # up to the FP32 rounding of sums over 1e10 entries
        assert np.all(np.diff(f) <= 1e-5 * np.abs(f[:-1])), f
        ref = oracle.fit_fbs(big["x64"], w.lam, T, L=st["lipschitz"], tau_replay=taus,
                             columns=COLS)
    got = om[COLS, :].cpu().numpy().astype(np.float64).T
    err = np.linalg.norm(got - ref.omega) / np.linalg.norm(ref.omega)
    print(f"[big] {form}: rel err {err:.3e}, trials {st['trials']}, "
          f"floor accepts {st['floor_accepts']}, L {st['lipschitz']:.6f} vs {big['L']:.6f}",
          flush=True)
    assert err <= (TOL_MX if form == "fp8" else TOL[form]), err
