"""Host-side tests of the C ABI (no GPU needed): the library loads, exports every
function include/accord.h declares, its structs match the ctypes mirrors, and
argument validation returns the documented status before touching the device."""
import ctypes
import os
import subprocess

import pytest

from paper_2412_11554_amd import accord

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(accord.LIB_PATH):
        pytest.skip("libaccord.so not built")
    return accord.lib()


def test_exports_every_declared_symbol(L):
    names = accord.header_functions()
    assert {"accord_fit", "accord_grad", "accord_prox", "accord_objective",
            "accord_workspace_bytes", "accord_status_str", "accord_last_error"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", accord.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "accord.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(accord_params), sizeof(accord_stats),"
        " offsetof(accord_stats, grad_gemm_ms), offsetof(accord_stats, total_ms),"
        " offsetof(accord_params, timing)); printf(\"%zu %zu\\n\", sizeof(accord_batch_stats),"
        " offsetof(accord_batch_stats, lipschitz)); printf(\"%zu %zu\\n\","
        " offsetof(accord_stats, log_det_d), offsetof(accord_batch_stats, log_det_d));"
        " printf(\"%zu\\n\", offsetof(accord_stats, lz_steps));"
        " return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(accord.accord_params)
    assert vals[1] == ctypes.sizeof(accord.accord_stats)
    assert vals[2] == accord.accord_stats.grad_gemm_ms.offset
    assert vals[3] == accord.accord_stats.total_ms.offset
    assert vals[4] == accord.accord_params.timing.offset
    assert vals[5] == ctypes.sizeof(accord.accord_batch_stats)
    assert vals[6] == accord.accord_batch_stats.lipschitz.offset
    assert vals[7] == accord.accord_stats.log_det_d.offset
    assert vals[8] == accord.accord_batch_stats.log_det_d.offset
    assert vals[9] == accord.accord_stats.lz_steps.offset


def test_default_params(L):
    prm = accord.default_params()
    assert prm.lambda_ == 0.1 and prm.tau0 == 1.0 and prm.beta == 0.5
    assert prm.lipschitz == 0.0 and prm.max_iter == 100
    assert prm.warm_tau == 0 and prm.graph == 0 and prm.refresh_every == 0
    assert prm.power_iters == 256  # cap on the Lanczos steps of the L estimate
    assert prm.probe == 1


def test_status_strings(L):
    for s in range(7):
        assert L.accord_status_str(s)
    assert L.accord_status_str(99) == b"unknown status"


def test_workspace_bytes(L):
    assert accord.accord_workspace_bytes(0, 10) == 0
    assert accord.accord_workspace_bytes(10, 0) == 0
    small = accord.accord_workspace_bytes(100, 200)
    big = accord.accord_workspace_bytes(500, 5000)
    assert 0 < small < big
    # at least the four p x p_pad FP32 matrices of the iteration
    p_pad = 5024
    assert big >= 4 * 5000 * p_pad * 4
    # fits one 288 GB device at the largest single-GPU problem (n=1000, p=100000)
    assert accord.accord_workspace_bytes(1000, 100000) < 200e9


FAKE = 1 << 20  # a 16-byte aligned non-null address; validation fails before any use


@pytest.mark.parametrize("kw,status", [
    (dict(X=None), 1), (dict(n=0), 1), (dict(p=0), 1), (dict(Omega=None), 1),
    (dict(X=FAKE + 4), 1), (dict(ws=None), 4), (dict(ws=FAKE + 16), 4), (dict(ws_bytes=10), 4),
    (dict(lam=-1.0), 1), (dict(tau0=0.0), 1), (dict(beta=0.0), 1), (dict(beta=1.5), 1),
    (dict(max_iter=-1), 1), (dict(precision=7), 5), (dict(tol=-1e-6), 1),
    (dict(lipschitz=-2.0), 1), (dict(lam=float("nan")), 1),
    (dict(p=(1 << 20) + 1), 1), (dict(n=(1 << 20) + 1), 1),
    (dict(timing=-1), 1), (dict(power_iters=-1), 1), (dict(probe=2), 1),
])
def test_fit_validation(L, kw, status):
    args = dict(X=FAKE, n=10, p=12, Omega=FAKE, ws=FAKE, ws_bytes=1 << 40, lam=0.1, tau0=1.0,
                beta=0.5, max_iter=3, precision=0, tol=0.0, lipschitz=0.0,
                timing=0, power_iters=0, probe=1)
    args.update(kw)
    prm = accord.default_params(lam=args["lam"], tau0=args["tau0"], beta=args["beta"],
                                max_iter=args["max_iter"], precision=args["precision"],
                                tol=args["tol"],
                                lipschitz=args["lipschitz"], timing=args["timing"],
                                power_iters=args["power_iters"], probe=args["probe"])
    st = accord.accord_stats()
    r = L.accord_fit(args["X"], args["n"], args["p"], args["Omega"], ctypes.byref(prm),
                     ctypes.byref(st), None, args["ws"], args["ws_bytes"], None)
    assert r == status, L.accord_last_error()
    assert L.accord_last_error()


def test_prox_validation(L):
    r = L.accord_prox(FAKE, FAKE, 10, 0.0, 0.1, FAKE + 256, FAKE + 512, FAKE, 1 << 30, None)
    assert r == 1  # tau must be > 0
    r = L.accord_prox(FAKE, FAKE, 10, 0.5, 0.1, FAKE, FAKE + 512, FAKE, 1 << 30, None)
    assert r == 1  # output aliases input
    r = L.accord_prox(FAKE, FAKE, 10, 0.5, 0.1, FAKE + 256, FAKE + 512, FAKE, 16, None)
    assert r == 4  # workspace too small


def test_grad_objective_validation(L):
    assert L.accord_grad(FAKE, 0, 5, FAKE, None, FAKE, FAKE, 1 << 30, None) == 1
    assert L.accord_grad(FAKE, 5, 5, FAKE, None, None, FAKE, 1 << 30, None) == 1
    assert L.accord_objective(FAKE, 5, 5, FAKE, -0.1, FAKE, FAKE, 1 << 30, None) == 1
    assert L.accord_objective(FAKE, 5, 5, FAKE, 0.1, None, FAKE, 1 << 30, None) == 1
    assert L.accord_objective(FAKE, 5, 5, FAKE, 0.1, FAKE, FAKE, 8, None) == 4


def test_binding_rejects_host_tensors(L):
    import torch
    with pytest.raises(TypeError):
        accord.accord_fit(torch.zeros(4, 5), 0.1, 2)


def test_batch_workspace_bytes(L):
    assert accord.accord_batch_workspace_bytes([100, 200], 0, 4) == 0
    assert accord.accord_batch_workspace_bytes([0, 200], 50, 4) == 0
    small = accord.accord_batch_workspace_bytes([60, 90], 100, 3)
    assert small > 0
    # at least the four per-problem matrices (Omega x2, G, Delta) of every problem
    assert small >= 4 * 6 * 128 * 128 * 4
    # 16 data sets x 32 penalties at p = 2000 fit one device
    assert accord.accord_batch_workspace_bytes([400] * 16, 2000, 32) < 60e9


def test_fit_batch_validation(L):
    prm = accord.default_params(max_iter=3)
    n = (ctypes.c_int64 * 2)(10, 12)
    lam = (ctypes.c_double * 2)(0.1, 0.2)
    st = (accord.accord_batch_stats * 4)()

    def call(X=FAKE, nn=n, nsub=2, p=7, la=lam, nlam=2, Om=FAKE, pr=prm, lip=None, ws=FAKE,
             ws_bytes=1 << 40):
        return L.accord_fit_batch(X, nn, nsub, p, la, nlam, Om, ctypes.byref(pr), lip, st, None,
                                  ws, ws_bytes, None)
    assert call(X=None) == 1
    assert call(nn=None) == 1
    assert call(nsub=0) == 1
    assert call(nlam=0) == 1
    assert call(la=None) == 1
    assert call(la=(ctypes.c_double * 2)(0.1, -1.0)) == 1
    assert call(lip=(ctypes.c_double * 2)(1.0, 0.0)) == 1
    assert call(nn=(ctypes.c_int64 * 2)(10, 0)) == 1
    assert call(ws=None) == 4
    assert call(ws_bytes=16) == 4
    assert call(pr=accord.default_params(max_iter=3, precision=2)) == 5
    assert call(pr=accord.default_params(beta=0.0)) == 1
    assert call(pr=accord.default_params(max_iter=3, batch_order=21)) == 1      # code > 20
    assert call(pr=accord.default_params(max_iter=3, batch_order=1 << 16)) == 1
    order = ctypes.c_int32()
    assert L.accord_tune_batch(None, n, 2, 7, lam, 2, FAKE, ctypes.byref(prm), None, FAKE,
                               1 << 40, None, ctypes.byref(order), None) == 1
    assert L.accord_tune_batch(FAKE, n, 2, 7, lam, 2, FAKE, ctypes.byref(prm), None, FAKE,
                               1 << 40, None, None, None) == 1
    assert L.accord_last_error()


def test_differentiation_validation(L):
    taus = (ctypes.c_double * 2)(0.5, -0.1)
    ws_ok = 1 << 40
    assert accord.accord_adjoint_workspace_bytes(0, 5) == 0
    assert accord.accord_adjoint_workspace_bytes(10, 20) > 0
    assert L.accord_fbs_replay(FAKE, 10, 5, FAKE, taus, 2, 0.1, None, FAKE, ws_ok, None) == 1
    assert L.accord_fbs_replay(FAKE, 10, 5, FAKE, None, 2, 0.1, None, FAKE, ws_ok, None) == 1
    assert L.accord_fbs_replay(FAKE, 10, 5, FAKE, taus, 1, -0.1, None, FAKE, ws_ok, None) == 1
    assert L.accord_fbs_replay(FAKE, 10, 5, FAKE, taus, 1, 0.1, None, FAKE, 16, None) == 4
    assert L.accord_val_loss_grad(FAKE, 10, 5, FAKE, None, FAKE, FAKE, ws_ok, None) == 1
    assert L.accord_val_loss_grad(FAKE, 10, 5, FAKE, FAKE, None, FAKE, ws_ok, None) == 1
    assert L.accord_fbs_adjoint_step(FAKE, 10, 5, FAKE, 0.0, 0.1, FAKE, FAKE, FAKE, FAKE, ws_ok,
                                     None) == 1
    assert L.accord_fbs_adjoint_step(FAKE, 10, 5, FAKE, 0.5, 0.1, FAKE, None, FAKE, FAKE, ws_ok,
                                     None) == 1
    assert L.accord_fbs_adjoint_step(FAKE, 10, 5, FAKE, 0.5, 0.1, FAKE, FAKE, FAKE, FAKE, 64,
                                     None) == 4
    assert L.accord_last_error()


# ---- steps around the solver ---------------------------------------------------
def test_refit_validation(L):
    prm = accord.default_params(lam=0.1, max_iter=3)
    st = accord.accord_stats()
    need = accord.accord_refit_workspace_bytes(10, 12, prm)
    assert need > accord.accord_workspace_bytes(10, 12, prm) > 0
    assert accord.accord_refit_workspace_bytes(0, 12, prm) == 0

    def call(X=FAKE, om_hat=FAKE, phi=0.5, prm=prm, ws_bytes=1 << 40):
        return L.accord_refit(X, 10, 12, om_hat, phi, FAKE, ctypes.byref(prm), ctypes.byref(st),
                              None, FAKE, ws_bytes, None)
    assert call(om_hat=None) == 1
    assert call(om_hat=FAKE + 4) == 1
    assert call(phi=-0.1) == 1 and call(phi=1.5) == 1 and call(phi=float("nan")) == 1
    assert call(X=None) == 1
    assert call(ws_bytes=accord.accord_workspace_bytes(10, 12, prm)) == 4  # fit size: too small
    # every precision form runs the refit; its workspace follows the form's layout
    for prec in ("bf16x1", "bf16x3", "fp8"):
        q = accord.default_params(lam=0.1, max_iter=3, precision=prec)
        need_q = accord.accord_refit_workspace_bytes(10, 12, q)
        assert need_q > accord.accord_workspace_bytes(10, 12, q) > 0
        assert call(prm=q, ws_bytes=need_q - 1) == 4
    assert L.accord_last_error()


def test_epbic_matches_oracle(L):
    """The library's epBIC from (g, log det, nnz) equals the oracle's eq. 3.7 value."""
    import numpy as np
    import datagen
    import oracle
    from oracle import tuning_oracle as tu
    x = datagen.small_random_problem(50, 15, 3).X.astype(np.float64)
    for lam in (0.05, 0.2):
        om = oracle.fit_fbs(x, lam, 300).omega
        g = oracle.smooth(x, om)
        logd = float(np.sum(np.log(np.diagonal(om))))
        for gamma in (0.5, 1.0):
            v = accord.accord_epbic(50, 15, g, logd, tu.nnz_offdiag(om), gamma)
            assert v == pytest.approx(tu.epbic(x, om, gamma), rel=1e-13)
    out = ctypes.c_double()
    assert L.accord_epbic(50, 15, 1.0, 0.0, 3, 0.0, ctypes.byref(out)) == 1   # gamma in (0, 1]
    assert L.accord_epbic(50, 15, 1.0, 0.0, 3, 1.5, ctypes.byref(out)) == 1
    assert L.accord_epbic(50, 15, 1.0, 0.0, 15 * 14 + 1, 0.5, ctypes.byref(out)) == 1
    assert L.accord_epbic(0, 15, 1.0, 0.0, 3, 0.5, ctypes.byref(out)) == 1
    assert L.accord_epbic(50, 15, 1.0, 0.0, 3, 0.5, None) == 1


def test_epbic_path_matches_oracle(L):
    import numpy as np
    import datagen
    import oracle
    from oracle import tuning_oracle as tu
    lams = [0.02, 0.08, 0.2, 0.5]
    xs = [datagen.small_random_problem(n, 12, 10 + n).X.astype(np.float64) for n in (30, 70)]
    stats, want, best = [], [], []
    for x in xs:
        oms = [oracle.fit_fbs(x, l, 300).omega for l in lams]
        v, b = tu.epbic_path(x, oms, 0.5)
        want.append(list(v))
        best.append(b)
        for om in oms:
            d = {name: 0 for name, _ in accord.accord_batch_stats._fields_}
            d.update(g=oracle.smooth(x, om), log_det_d=float(np.sum(np.log(np.diagonal(om)))),
                     nnz_offdiag=tu.nnz_offdiag(om))
            stats.append(d)
    got, gbest = accord.accord_epbic_path(stats, [30, 70], len(lams), 12, 0.5)
    assert gbest == best
    assert np.allclose(got, want, rtol=1e-13)


def test_reparam_validation(L):
    assert L.accord_reparam(FAKE, 10, None, None, None) == 1
    assert L.accord_reparam(FAKE, 10, FAKE, None, None) == 1        # Theta aliases Omega
    assert L.accord_reparam(FAKE, 10, None, FAKE, None) == 1        # Rho aliases Omega
    assert L.accord_reparam(FAKE, 10, FAKE + 256, FAKE + 256, None) == 1
    assert L.accord_reparam(FAKE, 0, FAKE + 256, None, None) == 1
    assert L.accord_reparam(FAKE, 10, FAKE + 4, None, None) == 1    # misaligned
    assert L.accord_reparam(None, 10, FAKE + 256, None, None) == 1


@pytest.mark.parametrize("field,value", [("warm_tau", 2), ("warm_tau", -1), ("graph", 3),
                                         ("refresh_every", -1), ("batch_order", -1),
                                         ("support_skip", 2)])
def test_variant_params_validation(L, field, value):
    prm = accord.default_params(lam=0.1, max_iter=3)
    setattr(prm, field, value)
    st = accord.accord_stats()
    r = L.accord_fit(FAKE, 10, 12, FAKE, ctypes.byref(prm), ctypes.byref(st), None, FAKE, 1 << 40,
                     None)
    assert r == 1 and field.encode() in L.accord_last_error()


def test_bench_timing_stride():
    """The benchmark samples about 64 iterations of a timed fit (every k-th one)."""
    import bench
    assert bench.timing_stride(500) == 7 and bench.timing_stride(200) == 3
    assert bench.timing_stride(10) == 1 and bench.timing_stride(0) == 1
