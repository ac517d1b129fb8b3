"""Python binding of libaccord (ctypes), with the entry-point names of include/accord.h.

Argument marshalling only: every step runs in the library's HIP kernels.  torch
supplies device memory and the stream; tensors must be float32/float64 CUDA
(HIP) tensors, C-contiguous.  There is no CPU path: a missing library or a
non-device tensor raises.

Matrix convention: Omega / G are torch [p, p] tensors holding the paper's Omega
(row j = node-wise problem j).  Their memory is the column form used by the
library (column j of the column-form matrix = node-wise problem j), so
``tensor.T`` is the column-form matrix g(Omega) = ||X Omega||^2/(2n) refers to.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # noqa: F401  -- load torch's HIP runtime first; libaccord binds to it

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaccord.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "accord.h")

ACCORD_OK = 0
STATUS_NAMES = {0: "ACCORD_OK", 1: "ACCORD_ERR_INVALID_ARG", 2: "ACCORD_ERR_DOMAIN",
                3: "ACCORD_ERR_NONFINITE", 4: "ACCORD_ERR_WORKSPACE",
                5: "ACCORD_ERR_UNSUPPORTED", 6: "ACCORD_ERR_HIP"}
PRECISIONS = {"fp32": 0, "bf16x1": 1, "bf16x3": 2, "fp8": 3}
TRACE_COLS = 8
TRACE_FIELDS = ("f", "g", "h", "tau", "trials", "delta_fro", "floor", "nnz")


class accord_params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("tau0", ctypes.c_double),
                ("beta", ctypes.c_double), ("lipschitz", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32),
                ("power_iters", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("warm_tau", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("refresh_every", ctypes.c_int32), ("probe", ctypes.c_int32),
                ("support_skip", ctypes.c_int32), ("batch_order", ctypes.c_int32)]


class accord_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("floor_accepts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("nnz_offdiag", ctypes.c_int64), ("f", ctypes.c_double),
                ("g", ctypes.c_double), ("h", ctypes.c_double), ("tau_last", ctypes.c_double),
                ("delta_fro", ctypes.c_double), ("lipschitz", ctypes.c_double),
                ("grad_gemm_ms", ctypes.c_double), ("grad_gemm_launches", ctypes.c_int32),
                ("trial_gemm_ms", ctypes.c_double), ("trial_gemm_launches", ctypes.c_int32),
                ("prox_ms", ctypes.c_double), ("prox_launches", ctypes.c_int32),
                ("total_ms", ctypes.c_double), ("log_det_d", ctypes.c_double),
                ("l1", ctypes.c_double), ("lz_steps", ctypes.c_int32),
                ("probe_rejects", ctypes.c_int32), ("unprobed_trials", ctypes.c_int32),
                ("probe_mtiles", ctypes.c_int32), ("tail_blocks", ctypes.c_int32),
                ("tail_splits", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class accord_batch_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("floor_accepts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("nnz_offdiag", ctypes.c_int64), ("f", ctypes.c_double),
                ("g", ctypes.c_double), ("h", ctypes.c_double), ("tau_last", ctypes.c_double),
                ("delta_fro", ctypes.c_double), ("lipschitz", ctypes.c_double),
                ("log_det_d", ctypes.c_double), ("l1", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class AccordError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_d = ctypes.c_double
_sz = ctypes.c_size_t


def lib() -> ctypes.CDLL:
    """The loaded libaccord.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.accord_default_params.argtypes = [ctypes.POINTER(accord_params)]
        L.accord_default_params.restype = None
        L.accord_workspace_bytes.argtypes = [_i64, _i64, ctypes.POINTER(accord_params)]
        L.accord_workspace_bytes.restype = _sz
        L.accord_grad.argtypes = [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp]
        L.accord_prox.argtypes = [_vp, _vp, _i64, _d, _d, _vp, _vp, _vp, _sz, _vp]
        L.accord_prox_noalloc.argtypes = [_vp, _vp, _i64, _d, _d, _vp, _vp, _vp]
        L.accord_prox_noalloc.restype = ctypes.c_int
        L.accord_objective.argtypes = [_vp, _i64, _i64, _vp, _d, _vp, _vp, _sz, _vp]
        L.accord_fit.argtypes = [_vp, _i64, _i64, _vp, ctypes.POINTER(accord_params),
                                 ctypes.POINTER(accord_stats), _vp, _vp, _sz, _vp]
        for f in ("accord_grad", "accord_prox", "accord_objective", "accord_fit"):
            getattr(L, f).restype = ctypes.c_int
        _pi64 = ctypes.POINTER(ctypes.c_int64)
        _pd = ctypes.POINTER(ctypes.c_double)
        L.accord_batch_workspace_bytes.argtypes = [_pi64, _i64, _i64, _i64,
                                                   ctypes.POINTER(accord_params)]
        L.accord_batch_workspace_bytes.restype = _sz
        L.accord_fit_batch.argtypes = [_vp, _pi64, _i64, _i64, _pd, _i64, _vp,
                                       ctypes.POINTER(accord_params), _pd,
                                       ctypes.POINTER(accord_batch_stats), _vp, _vp, _sz, _vp]
        L.accord_fit_batch.restype = ctypes.c_int
        L.accord_tune_batch.argtypes = [_vp, _pi64, _i64, _i64, _pd, _i64, _vp,
                                        ctypes.POINTER(accord_params), _pd, _vp, _sz, _vp,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_float)]
        L.accord_tune_batch.restype = ctypes.c_int
        L.accord_adjoint_workspace_bytes.argtypes = [_i64, _i64]
        L.accord_adjoint_workspace_bytes.restype = _sz
        L.accord_fbs_replay.argtypes = [_vp, _i64, _i64, _vp, _pd, _i64, _d, _vp, _vp, _sz, _vp]
        L.accord_val_loss_grad.argtypes = [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp]
        L.accord_fbs_adjoint_step.argtypes = [_vp, _i64, _i64, _vp, _d, _d, _vp, _vp, _vp, _vp,
                                              _sz, _vp]
        for f in ("accord_fbs_replay", "accord_val_loss_grad", "accord_fbs_adjoint_step"):
            getattr(L, f).restype = ctypes.c_int
        L.accord_epbic.argtypes = [_i64, _i64, _d, _d, _i64, _d, _pd]
        L.accord_epbic_path.argtypes = [ctypes.POINTER(accord_batch_stats), _pi64, _i64, _i64,
                                        _i64, _d, _pd, _pi64]
        L.accord_refit_workspace_bytes.argtypes = [_i64, _i64, ctypes.POINTER(accord_params)]
        L.accord_refit_workspace_bytes.restype = _sz
        L.accord_refit.argtypes = [_vp, _i64, _i64, _vp, _d, _vp, ctypes.POINTER(accord_params),
                                   ctypes.POINTER(accord_stats), _vp, _vp, _sz, _vp]
        L.accord_reparam.argtypes = [_vp, _i64, _vp, _vp, _vp]
        for f in ("accord_epbic", "accord_epbic_path", "accord_refit", "accord_reparam"):
            getattr(L, f).restype = ctypes.c_int
        L.accord_status_str.argtypes = [ctypes.c_int]
        L.accord_status_str.restype = ctypes.c_char_p
        L.accord_last_error.argtypes = []
        L.accord_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/accord.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w ]+?\*?\s*)\b(accord_\w+)\s*\(", text, re.M)))


def _check(status: int) -> None:
    if status != ACCORD_OK:
        msg = lib().accord_last_error().decode()
        raise AccordError(status, msg)


def _dev(t: torch.Tensor, name: str, dtype=torch.float32) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def default_params(**kw) -> accord_params:
    prm = accord_params()
    lib().accord_default_params(ctypes.byref(prm))
    for k, v in kw.items():
        if k == "lam":
            k = "lambda_"
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if not hasattr(prm, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(prm, k, v)
    return prm


def accord_workspace_bytes(n: int, p: int, params: accord_params | None = None) -> int:
    return int(lib().accord_workspace_bytes(n, p, ctypes.byref(params) if params else None))


def _workspace(n: int, p: int, params, device, ws):
    need = accord_workspace_bytes(n, p, params)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
    return ws


def accord_grad(X: torch.Tensor, Omega: torch.Tensor, *, want_W: bool = False,
                G: torch.Tensor | None = None, W: torch.Tensor | None = None, ws=None):
    """G = X^T (X Omega_col) / n (returned as the paper-form [p, p] tensor) and
    optionally W = X Omega_col ([n, p])."""
    n, p = X.shape
    dev = X.device
    if G is None:
        G = torch.empty((p, p), dtype=torch.float32, device=dev)
    if want_W and W is None:
        W = torch.empty((n, p), dtype=torch.float32, device=dev)
    ws = _workspace(n, p, None, dev, ws)
    _check(lib().accord_grad(_dev(X, "X"), n, p, _dev(Omega, "Omega"),
                             _dev(W, "W") if W is not None else None, _dev(G, "G"),
                             ws.data_ptr(), ws.numel(), _stream(dev)))
    return G, W


def accord_prox(Omega: torch.Tensor, G: torch.Tensor, tau: float, lam: float, *,
                out: torch.Tensor | None = None, red: torch.Tensor | None = None, ws=None):
    """One eq.-3.5 step; returns (Omega_out, red[6] float64 device tensor)."""
    p = Omega.shape[0]
    dev = Omega.device
    if out is None:
        out = torch.empty_like(Omega)
    if red is None:
        red = torch.empty(6, dtype=torch.float64, device=dev)
    ws = _workspace(1, p, None, dev, ws)
    _check(lib().accord_prox(_dev(Omega, "Omega"), _dev(G, "G"), p, float(tau), float(lam),
                             _dev(out, "Omega_out"), _dev(red, "red", torch.float64),
                             ws.data_ptr(), ws.numel(), _stream(dev)))
    return out, red


def accord_prox_noalloc(Omega: torch.Tensor, G: torch.Tensor, tau: float, lam: float,
                        out: torch.Tensor, red: torch.Tensor):
    """accord_prox without a workspace (the library's own scratch array); the caller
    passes the outputs: out [p, p] float32 and red [6] float64 device tensors."""
    p = Omega.shape[0]
    _check(lib().accord_prox_noalloc(_dev(Omega, "Omega"), _dev(G, "G"), p, float(tau),
                                     float(lam), _dev(out, "Omega_out"),
                                     _dev(red, "red", torch.float64), _stream(Omega.device)))
    return out, red


def accord_objective(X: torch.Tensor, Omega: torch.Tensor, lam: float, *, out=None, ws=None):
    """(g, h, f) at Omega as a float64 device tensor of length 3."""
    n, p = X.shape
    dev = X.device
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=dev)
    ws = _workspace(n, p, None, dev, ws)
    _check(lib().accord_objective(_dev(X, "X"), n, p, _dev(Omega, "Omega"), float(lam),
                                  _dev(out, "out", torch.float64), ws.data_ptr(), ws.numel(),
                                  _stream(dev)))
    return out


def accord_fit(X: torch.Tensor, lam: float, max_iter: int, *, omega0: torch.Tensor | None = None,
               tau0: float = 1.0, beta: float = 0.5, lipschitz: float = 0.0, tol: float = 0.0,
               power_iters: int = 0, precision: str = "fp32",
               trace: bool = False, timing: int = 0, warm_tau: bool = False,
               refresh_every: int = 0, probe: bool = True, ws=None, omega_out=None):
    """ACCORD-FBS (Alg. 1).  Returns (Omega [p, p] paper form, stats dict, trace or None).
    omega0 defaults to the identity.  warm_tau selects the warm-started step variant;
    probe=False always runs the whole trial product (no rejection from the first 256
    samples)."""
    n, p = X.shape
    dev = X.device
    prm = default_params(lam=lam, max_iter=max_iter, tau0=tau0, beta=beta, lipschitz=lipschitz,
                         tol=tol, power_iters=power_iters,
                         precision=precision, timing=int(timing),
                         warm_tau=1 if warm_tau else 0, refresh_every=refresh_every,
                         probe=1 if probe else 0)
    if omega_out is None:
        omega_out = torch.empty((p, p), dtype=torch.float32, device=dev)
    if omega0 is None:
        omega_out.zero_()
        omega_out.diagonal().fill_(1.0)
    else:
        omega_out.copy_(omega0)
    tr = torch.zeros(((max_iter + 1) * TRACE_COLS,), dtype=torch.float64, device=dev) if trace else None
    ws = _workspace(n, p, prm, dev, ws)
    st = accord_stats()
    _check(lib().accord_fit(_dev(X, "X"), n, p, _dev(omega_out, "Omega"), ctypes.byref(prm),
                            ctypes.byref(st), _dev(tr, "trace", torch.float64) if tr is not None else None,
                            ws.data_ptr(), ws.numel(), _stream(dev)))
    stats = st.as_dict()
    if tr is not None:
        tr = tr.view(max_iter + 1, TRACE_COLS)[: stats["iters"] + 1]
    return omega_out, stats, tr


def accord_batch_workspace_bytes(n, p: int, nlam: int, params: accord_params | None = None) -> int:
    na = (ctypes.c_int64 * len(n))(*[int(v) for v in n])
    return int(lib().accord_batch_workspace_bytes(na, len(n), p, nlam,
                                                  ctypes.byref(params) if params else None))


def accord_fit_batch(X: torch.Tensor, n, lambdas, max_iter: int, *,
                     omega0: torch.Tensor | None = None, tau0: float = 1.0, beta: float = 0.5,
                     tol: float = 0.0, power_iters: int = 0, lipschitz=None, trials: bool = False,
                     warm_tau: bool = False, graph: bool = False, batch_order: int = 0, ws=None,
                     omega_out=None):
    """Batched ACCORD-FBS: X is the row-wise stack of the data sets (sum(n) x p),
    n their row counts, lambdas the penalties.  Problem k = b * len(lambdas) + l.
    Returns (Omega [nprob, p, p] paper form, list of stats dicts, trials
    [nprob, max_iter] int32 device tensor or None).  omega0 defaults to identities.
    batch_order: a tile order code from accord_tune_batch (0 = default)."""
    n = [int(v) for v in n]
    nsub, p = len(n), X.shape[1]
    if X.shape[0] != sum(n):
        raise ValueError(f"X has {X.shape[0]} rows, n sums to {sum(n)}")
    lam = [float(v) for v in lambdas]
    nlam = len(lam)
    nprob = nsub * nlam
    dev = X.device
    prm = default_params(max_iter=max_iter, tau0=tau0, beta=beta, tol=tol,
                         power_iters=power_iters, warm_tau=1 if warm_tau else 0,
                         graph=1 if graph else 0, batch_order=batch_order)
    if omega_out is None:
        omega_out = torch.empty((nprob, p, p), dtype=torch.float32, device=dev)
    if omega0 is None:
        omega_out.zero_()
        omega_out.diagonal(dim1=1, dim2=2).fill_(1.0)
    else:
        omega_out.copy_(omega0)
    need = accord_batch_workspace_bytes(n, p, nlam, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    tr = (torch.zeros((nprob, max(max_iter, 1)), dtype=torch.int32, device=dev)
          if trials else None)
    na = (ctypes.c_int64 * nsub)(*n)
    la = (ctypes.c_double * nlam)(*lam)
    lp = (ctypes.c_double * nsub)(*[float(v) for v in lipschitz]) if lipschitz is not None else None
    st = (accord_batch_stats * nprob)()
    _check(lib().accord_fit_batch(_dev(X, "X"), na, nsub, p, la, nlam, _dev(omega_out, "Omega"),
                                  ctypes.byref(prm), lp, st,
                                  tr.data_ptr() if tr is not None else None,
                                  ws.data_ptr(), ws.numel(), _stream(dev)))
    return omega_out, [s.as_dict() for s in st], tr


BATCH_ORDERS = 20  # launch codes per kernel that accord_tune_batch times (10 tile orders
                   # at two workgroups per CU, then at one)


def accord_tune_batch(X: torch.Tensor, n, lambdas, *, max_iter: int = 1, tau0: float = 1.0,
                      beta: float = 0.5, power_iters: int = 0, lipschitz=None, ws=None):
    """Times the batched kernels under every launch code (tile order x workgroups per CU)
    on this problem set (after the fit's set-up) and returns (batch_order code,
    {"grad": [ms per code], "trial": [...]})."""
    n = [int(v) for v in n]
    nsub, p = len(n), X.shape[1]
    lam = [float(v) for v in lambdas]
    nlam = len(lam)
    dev = X.device
    prm = default_params(max_iter=max_iter, tau0=tau0, beta=beta, power_iters=power_iters)
    om = torch.zeros((nsub * nlam, p, p), dtype=torch.float32, device=dev)
    om.diagonal(dim1=1, dim2=2).fill_(1.0)
    need = accord_batch_workspace_bytes(n, p, nlam, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    na = (ctypes.c_int64 * nsub)(*n)
    la = (ctypes.c_double * nlam)(*lam)
    lp = (ctypes.c_double * nsub)(*[float(v) for v in lipschitz]) if lipschitz is not None else None
    order = ctypes.c_int32(0)
    table = (ctypes.c_float * (2 * BATCH_ORDERS))()
    _check(lib().accord_tune_batch(_dev(X, "X"), na, nsub, p, la, nlam, _dev(om, "Omega"),
                                   ctypes.byref(prm), lp, ws.data_ptr(), ws.numel(), _stream(dev),
                                   ctypes.byref(order), table))
    t = list(table)
    return int(order.value), {"grad": t[:BATCH_ORDERS], "trial": t[BATCH_ORDERS:]}


def accord_adjoint_workspace_bytes(n: int, p: int) -> int:
    return int(lib().accord_adjoint_workspace_bytes(n, p))


def _adj_ws(n, p, device, ws):
    need = accord_adjoint_workspace_bytes(n, p)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
    return ws


def accord_fbs_replay(X: torch.Tensor, omega: torch.Tensor, taus, lam: float, *,
                      seq: torch.Tensor | None = None, ws=None):
    """Fixed steps taus from omega (paper-form [p, p], updated in place); seq
    ([len(taus), p, p] or None) receives every iterate.  Returns omega."""
    n, p = X.shape
    taus = [float(t) for t in taus]
    ta = (ctypes.c_double * max(len(taus), 1))(*taus)
    ws = _adj_ws(n, p, X.device, ws)
    _check(lib().accord_fbs_replay(_dev(X, "X"), n, p, _dev(omega, "Omega"), ta, len(taus),
                                   float(lam), _dev(seq, "seq") if seq is not None else None,
                                   ws.data_ptr(), ws.numel(), _stream(X.device)))
    return omega


def accord_val_loss_grad(Xv: torch.Tensor, omega: torch.Tensor, *, obar=None, out=None, ws=None):
    """(out = [g_v, -sum log diag, loss] float64 device tensor, obar = dloss/dOmega)."""
    nv, p = Xv.shape
    if obar is None:
        obar = torch.empty((p, p), dtype=torch.float32, device=Xv.device)
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=Xv.device)
    ws = _adj_ws(nv, p, Xv.device, ws)
    _check(lib().accord_val_loss_grad(_dev(Xv, "Xv"), nv, p, _dev(omega, "Omega"),
                                      _dev(out, "out", torch.float64), _dev(obar, "Obar"),
                                      ws.data_ptr(), ws.numel(), _stream(Xv.device)))
    return out, obar


def accord_fbs_adjoint_step(X: torch.Tensor, omega_t: torch.Tensor, tau: float, lam: float,
                            obar: torch.Tensor, lbar: torch.Tensor, xbar: torch.Tensor, *, ws=None):
    """One reverse step: obar <- dl/dOmega_t (in place), lbar += dl/dlambda,
    xbar += dl/dX."""
    n, p = X.shape
    ws = _adj_ws(n, p, X.device, ws)
    _check(lib().accord_fbs_adjoint_step(_dev(X, "X"), n, p, _dev(omega_t, "Omega_t"), float(tau),
                                         float(lam), _dev(obar, "Obar"),
                                         _dev(lbar, "lbar", torch.float64), _dev(xbar, "Xbar"),
                                         ws.data_ptr(), ws.numel(), _stream(X.device)))


# ---------------------------------------------------------------------------
# steps around the solver: epBIC (eq. 3.7), refit (eq. 3.8), reparametrisation
# ---------------------------------------------------------------------------
def accord_epbic(n: int, p: int, g: float, log_det_d: float, nnz_offdiag: int,
                 gamma: float) -> float:
    """Extended pseudo-BIC of one estimate from its fit statistics."""
    out = ctypes.c_double()
    _check(lib().accord_epbic(n, p, g, log_det_d, nnz_offdiag, gamma, ctypes.byref(out)))
    return out.value


def accord_epbic_path(stats, n, nlam: int, p: int, gamma: float):
    """epBIC of every problem of a batched fit (stats: the list of dicts
    accord_fit_batch returns) and, per data set, the index of the best penalty.
    Returns (epbic [nsub, nlam] list of lists, best list)."""
    n = [int(v) for v in n]
    nsub = len(n)
    if len(stats) != nsub * nlam:
        raise ValueError(f"{len(stats)} stats for {nsub} x {nlam} problems")
    st = (accord_batch_stats * len(stats))()
    for k, d in enumerate(stats):
        for name, _ in accord_batch_stats._fields_:
            setattr(st[k], name, d[name])
    na = (ctypes.c_int64 * nsub)(*n)
    out = (ctypes.c_double * len(stats))()
    best = (ctypes.c_int64 * nsub)()
    _check(lib().accord_epbic_path(st, na, nsub, nlam, p, gamma, out, best))
    return [[out[b * nlam + l] for l in range(nlam)] for b in range(nsub)], list(best)


def accord_refit_workspace_bytes(n: int, p: int, params: accord_params | None = None) -> int:
    return int(lib().accord_refit_workspace_bytes(n, p, ctypes.byref(params) if params else None))


def accord_refit(X: torch.Tensor, omega_hat: torch.Tensor, lam: float, phi: float, max_iter: int,
                 *, omega0: torch.Tensor | None = None, tau0: float = 1.0, beta: float = 0.5,
                 lipschitz: float = 0.0, tol: float = 0.0, power_iters: int = 0,
                 precision: str = "fp32", trace: bool = False, timing: int = 0, ws=None,
                 omega_out=None, support_skip: bool = True, probe: bool = True):
    """Refit on the support of omega_hat with penalty phi * lam there (eq. 3.8), in any
    precision form.  Returns (Omega [p, p] paper form, stats dict, trace or None); the
    start defaults to omega_hat.  support_skip=False makes the fused forms walk every
    block (same results)."""
    n, p = X.shape
    dev = X.device
    prm = default_params(lam=lam, max_iter=max_iter, tau0=tau0, beta=beta, lipschitz=lipschitz,
                         tol=tol, power_iters=power_iters, timing=int(timing),
                         precision=precision, support_skip=1 if support_skip else 0,
                         probe=1 if probe else 0)
    if omega_out is None:
        omega_out = torch.empty((p, p), dtype=torch.float32, device=dev)
    omega_out.copy_(omega_hat if omega0 is None else omega0)
    tr = torch.zeros(((max_iter + 1) * TRACE_COLS,), dtype=torch.float64, device=dev) if trace else None
    need = accord_refit_workspace_bytes(n, p, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    st = accord_stats()
    _check(lib().accord_refit(_dev(X, "X"), n, p, _dev(omega_hat, "Omega_hat"), phi,
                              _dev(omega_out, "Omega"), ctypes.byref(prm), ctypes.byref(st),
                              _dev(tr, "trace", torch.float64) if tr is not None else None,
                              ws.data_ptr(), ws.numel(), _stream(dev)))
    stats = st.as_dict()
    if tr is not None:
        tr = tr.view(max_iter + 1, TRACE_COLS)[: stats["iters"] + 1]
    return omega_out, stats, tr


def accord_reparam(omega: torch.Tensor, *, theta: bool = True, rho: bool = True,
                   theta_out=None, rho_out=None):
    """Theta = Omega_D Omega and the partial correlations of an estimate (paper form
    [p, p] tensors, like Omega).  Returns (Theta or None, Rho or None)."""
    p = omega.shape[0]
    dev = omega.device
    if theta and theta_out is None:
        theta_out = torch.empty((p, p), dtype=torch.float32, device=dev)
    if rho and rho_out is None:
        rho_out = torch.empty((p, p), dtype=torch.float32, device=dev)
    t = theta_out if theta else None
    r = rho_out if rho else None
    _check(lib().accord_reparam(_dev(omega, "Omega"), p,
                                _dev(t, "Theta") if t is not None else None,
                                _dev(r, "Rho") if r is not None else None, _stream(dev)))
    return t, r
