"""FP64 CPU oracle for the ACCORD-FBS estimator (arXiv 2412.11554).

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the
GPU library is checked against.  Only the test suite, the package smoke check
and the benchmark's CPU-baseline leg may import it; the GPU path never does, and
this module imports nothing from the GPU package.

Everything here is plain numpy/scipy in float64, written for readability, not
speed.  Inputs are the exact float32 values the GPU receives, promoted to float64.

Convention.  The paper (Sec. 3.2, eq. 3.4) writes the smooth part as
g(Omega) = tr(Omega^T Omega S)/2 with gradient Omega S, i.e. it works on the rows
of Omega.  The supplement's proof of Theorem 3.2 rewrites the objective column by
column of Omega^T.  This oracle stores that column form directly:

    Om = Omega_paper^T,   g(Om) = ||X Om||_F^2 / (2n),   grad g(Om) = X^T (X Om) / n = S Om,

so column j of ``Om`` is node-wise problem j.  The diagonal is the same in both
forms; a paper-convention result is ``Om.T``.  The penalty lambda*||Om||_1 covers
all p^2 entries, diagonal included (eq. 3.2; the diagonal root of eq. 3.5 carries
the -tau*lambda term).

Functions and the passages they follow:
  soft_threshold, diag_root, prox   eq. 3.5 (closed-form backward step)
  smooth, grad, objective           eq. 3.2 / eq. 3.4
  lipschitz                         Sec. 3.2: L = sigma_max(S)
  line_search_test                  Alg. 1 acceptance inequality (both forms)
  fit_fbs                           Alg. 1 (ACCORD-FBS with backtracking)
  kkt_residual                      eq. 3.3 (and its column form in the supplement)
  fit_cd                            independent solver: cyclic coordinate descent
                                    on the separable column objective (supplement,
                                    proof of Theorem 3.2)
  brute_column                      independent solver: generic bound-constrained
                                    quasi-Newton on one column (tiny p only)
Pins for each function are listed in the test module ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _f64(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# eq. 3.5: the proximal (backward) step, element by element
# ---------------------------------------------------------------------------

def soft_threshold(x, a):
    """S_a(x) = (|x| - a)_+ sign(x)  (eq. 3.5).  At |x| == a the result is 0."""
    x = _f64(x)
    return np.sign(x) * np.maximum(np.abs(x) - a, 0.0)


def diag_root(y, tau, lam):
    """Diagonal update of eq. 3.5: (y - tau*lam + sqrt((y - tau*lam)^2 + 4 tau)) / 2.

    It is the positive root of w^2 - (y - tau*lam) w - tau = 0, i.e. the minimiser of
    -log w + lam*w + (w - y)^2 / (2 tau) over w > 0."""
    y = _f64(y)
    b = y - tau * lam
    return (b + np.sqrt(b * b + 4.0 * tau)) / 2.0


def prox(om, g, tau, lam):
    """One forward-backward update (eq. 3.5) of the whole matrix:
    off-diagonal entries are soft-thresholded at tau*lam, diagonal entries take the
    positive root above, both applied to  om - tau * g."""
    om = _f64(om)
    a = om - tau * _f64(g)
    out = soft_threshold(a, tau * lam)
    d = np.arange(om.shape[0])
    out[d, d] = diag_root(a[d, d], tau, lam)
    return out


# ---------------------------------------------------------------------------
# eq. 3.2 / 3.4: objective pieces
# ---------------------------------------------------------------------------

def smooth(x, om):
    """g(Om) = ||X Om||_F^2 / (2n)   (eq. 3.4 in column form)."""
    x = _f64(x)
    w = x @ _f64(om)
    return float(np.sum(w * w) / (2.0 * x.shape[0]))


def grad(x, om):
    """grad g(Om) = X^T (X Om) / n = S Om   (the two-step product of Remark 3.1)."""
    x = _f64(x)
    return x.T @ (x @ _f64(om)) / x.shape[0]


def objective(x, om, lam):
    """(g, h, f) with h = -sum_j log om_jj + lam * sum_ij |om_ij| (eq. 3.2, 3.4).
    h and f are +inf outside the domain (some om_jj <= 0)."""
    om = _f64(om)
    g = smooth(x, om)
    d = np.diagonal(om)
    if np.any(d <= 0):
        return g, np.inf, np.inf
    h = float(-np.sum(np.log(d)) + lam * np.sum(np.abs(om)))
    return g, h, g + h


def lipschitz(x):
    """L = sigma_max(S) = sigma_max(X)^2 / n  (Sec. 3.2), by a dense SVD."""
    x = _f64(x)
    return float(np.linalg.norm(x, 2) ** 2 / x.shape[0])


# ---------------------------------------------------------------------------
# Alg. 1: ACCORD-FBS
# ---------------------------------------------------------------------------

def line_search_test(x, om, om_new, g_at_om, g_cur, tau):
    """Alg. 1's acceptance inequality, evaluated two ways.

    literal:   g(Om+) <= g(Om) + <Delta, grad g(Om)> + ||Delta||_F^2 / (2 tau)
    canonical: ||X Delta||_F^2 / n <= ||Delta||_F^2 / tau

    Because g is quadratic, g(Om + D) = g(Om) + <grad g(Om), D> + ||X D||^2/(2n)
    exactly, so the two are the same inequality; the canonical form avoids
    subtracting two large values of g.  (The printed inequality has the inner
    product with g(Omega^(t)); the proof of Theorem 3.3 uses grad g, which is the
    reading taken here.)  Returns (canonical, literal, ||X D||^2/n, ||D||^2)."""
    x = _f64(x)
    n = x.shape[0]
    d = _f64(om_new) - _f64(om)
    v = x @ d
    xd2_over_n = float(np.sum(v * v) / n)
    d2 = float(np.sum(d * d))
    canonical = xd2_over_n <= d2 / tau
    g_new = smooth(x, om_new)
    literal = g_new <= g_cur + float(np.sum(d * _f64(g_at_om))) + d2 / (2.0 * tau)
    return canonical, literal, xd2_over_n, d2


def identity_columns(p, cols):
    """Columns ``cols`` of the p x p identity, built without forming the identity."""
    cols = np.asarray(cols)
    out = np.zeros((p, len(cols)))
    out[cols, np.arange(len(cols))] = 1.0
    return out


def x_times(x, om, nnz=None):
    """X @ om.  When om is almost all zeros (the iterates of a penalised fit late in the
    run), the product runs over its nonzero entries only (scipy.sparse, one thread); the
    value is the same product.  The dense product is many times faster per entry, so the
    sparse one is taken below 0.3% density only.  nnz: om's nonzero count, if known."""
    if om.size >= 1 << 20 and (np.count_nonzero(om) if nnz is None else nnz) < 0.003 * om.size:
        from scipy import sparse
        return np.asarray(x @ sparse.csc_matrix(om))
    return x @ om


@dataclass
class FitResult:
    omega: np.ndarray                   # final iterate (column form)
    iters: int
    f: list = field(default_factory=list)        # f(Om_t), t = 0..iters
    g: list = field(default_factory=list)        # g(Om_t)
    tau: list = field(default_factory=list)      # accepted step of iteration t
    trials: list = field(default_factory=list)   # trials used in iteration t
    floor: list = field(default_factory=list)    # accepted by the tau <= 1/L rule only
    literal_agree: list = field(default_factory=list)  # literal == canonical at every trial
    delta_fro: list = field(default_factory=list)
    converged: bool = False
    lipschitz: float = 0.0


def _prox_by_column_chunks(prox_cols, om, G, tau):
    """prox_cols(om, G, tau), ||result - om||_F^2 and the result's nonzero count for a
    wide column block, with the columns split into chunks handled by threads (numpy's
    elementwise loops release the interpreter lock).  Each entry gets exactly the
    arithmetic of prox_cols; only the FP64 sum of squares is added up chunk by chunk."""
    J = om.shape[1]
    if om.size < 1 << 22:
        out = prox_cols(om, G, tau, slice(0, J))
        return out, float(np.sum((out - om) ** 2)), int(np.count_nonzero(out))
    from concurrent.futures import ThreadPoolExecutor
    import os
    nthreads = max(1, min(16, os.cpu_count() or 1))
    bounds = np.linspace(0, J, nthreads + 1).astype(int)
    out = np.empty_like(om)

    def work(k):
        c = slice(bounds[k], bounds[k + 1])
        out[:, c] = prox_cols(om[:, c], G[:, c], tau, c)
        return float(np.sum((out[:, c] - om[:, c]) ** 2)), int(np.count_nonzero(out[:, c]))

    with ThreadPoolExecutor(nthreads) as pool:
        parts = list(pool.map(work, range(nthreads)))
    return out, sum(d for d, _ in parts), sum(z for _, z in parts)


def fit_fbs(x, lam, iters, omega0=None, tau0=1.0, beta=0.5, L=None, tol=0.0,
            tau_replay=None, columns=None, warm_tau=False, record=True, progress=None):
    """ACCORD-FBS (Alg. 1) in float64.

    For t = 0, 1, ...: compute G = grad g(Om_t) once (it does not depend on tau);
    try tau = tau0, beta*tau0, beta^2*tau0, ...; for each, form Om+ by eq. 3.5 and
    Delta = Om+ - Om_t, and stop at the first tau that passes the acceptance test
    or satisfies tau <= 1/L.  Om_{t+1} = Om+.  beta == 1 means a fixed step
    (the single trial is accepted).

    tau_replay: if given, iteration t uses exactly tau_replay[t] (one trial,
      accepted) -- used to follow another run's step sequence.
    columns: if given (with tau_replay), only these columns of Om are evolved.
      With the steps fixed, column j of the iterate depends only on column j of
      Om and on X (the objective separates over columns; supplement, proof of
      Theorem 3.2), so this reproduces those columns of the full run.
    tol > 0: stop once ||Delta||_F <= tol * max(1, ||Om+||_F).
    warm_tau: a variant that departs from Alg. 1 (which restarts every iteration at
      tau0): after the first iteration the trials start at min(tau0, tau_{t-1} / beta).
      The acceptance test and the floor are unchanged.
    record: with tau_replay, False skips what a replay does not need -- the objective
      values and the acceptance test of each (already decided) step -- so a long replay
      on many columns costs the two products of the gradient per iteration; the
      iterates are the same (f, g and literal_agree stay empty).
    progress: optional callable, called with the iteration count after each iteration.
    """
    if not record and tau_replay is None:
        raise ValueError("record=False needs tau_replay (the line search needs the sums)")
    x = _f64(x)
    n, p = x.shape
    if L is None:
        L = lipschitz(x)
    if columns is not None:
        if tau_replay is None:
            raise ValueError("columns= needs tau_replay (the shared step couples columns)")
        cols = np.asarray(columns)
        om = identity_columns(p, cols) if omega0 is None else _f64(omega0)[:, cols].copy()
        # diagonal positions of the selected columns inside the p x |J| block
        diag_rows = cols
    else:
        om = np.eye(p) if omega0 is None else _f64(omega0).copy()
        diag_rows = None

    def _prox_cols(o, g, tau, c=None):
        # columns c (a slice of the selected columns) of the update, eq. 3.5
        if diag_rows is None and c is None:
            return prox(o, g, tau, lam)
        rows = diag_rows if diag_rows is not None else np.arange(p)
        rows = rows if c is None else rows[c]
        a = o - tau * g
        out = soft_threshold(a, tau * lam)
        jj = np.arange(len(rows))
        out[rows, jj] = diag_root(a[rows, jj], tau, lam)
        return out

    def _obj(o):
        w = x @ o
        g = float(np.sum(w * w) / (2 * n))
        d = o[diag_rows, np.arange(len(diag_rows))] if diag_rows is not None else np.diagonal(o)
        h = float(-np.sum(np.log(d)) + lam * np.sum(np.abs(o))) if np.all(d > 0) else np.inf
        return g, g + h

    res = FitResult(omega=om, iters=0, lipschitz=L)
    if not record:
        xt = np.ascontiguousarray(x.T)
        nnz = None
        for t in range(iters):
            tau = float(tau_replay[t])
            G = xt @ x_times(x, om, nnz)
            G /= n
            om_new, d2, nnz = _prox_by_column_chunks(_prox_cols, om, G, tau)
            res.tau.append(tau)
            res.trials.append(1)
            res.delta_fro.append(np.sqrt(d2))
            om = om_new
            res.iters = t + 1
            if progress is not None:
                progress(t + 1)
            if tol > 0 and np.sqrt(d2) <= tol * max(1.0, float(np.linalg.norm(om))):
                res.converged = True
                break
        res.omega = om
        return res
    g_cur, f_cur = _obj(om)
    res.g.append(g_cur)
    res.f.append(f_cur)
    for t in range(iters):
        G = x.T @ (x @ om) / n
        if tau_replay is not None:
            tau = float(tau_replay[t])
        elif warm_tau and t > 0:
            tau = min(tau0, res.tau[-1] / beta)
        else:
            tau = tau0
        k = 0
        while True:
            k += 1
            om_new = _prox_cols(om, G, tau)
            can, lit, _, d2 = line_search_test(x, om, om_new, G, g_cur, tau)
            at_floor = tau <= 1.0 / L
            res.literal_agree.append(can == lit)
            if tau_replay is not None or beta == 1.0 or can or at_floor:
                res.floor.append(bool(at_floor and not can))
                break
            tau *= beta
        res.tau.append(tau)
        res.trials.append(k)
        res.delta_fro.append(np.sqrt(d2))
        om = om_new
        g_cur, f_cur = _obj(om)
        res.g.append(g_cur)
        res.f.append(f_cur)
        res.iters = t + 1
        if tol > 0 and np.sqrt(d2) <= tol * max(1.0, float(np.linalg.norm(om))):
            res.converged = True
            break
    res.omega = om
    return res


# ---------------------------------------------------------------------------
# eq. 3.3: optimality
# ---------------------------------------------------------------------------

def kkt_residual(x, om, lam):
    """Largest violation of the KKT condition (eq. 3.3, column form):
      diagonal:           -1/om_jj + G_jj + lam = 0
      off-diagonal != 0:  G_ij + lam * sign(om_ij) = 0
      off-diagonal == 0:  |G_ij| <= lam
    with G = S Om.  Returns (max residual, dict of the three parts)."""
    om = _f64(om)
    G = grad(x, om)
    p = om.shape[0]
    diag = np.arange(p)
    off = ~np.eye(p, dtype=bool)
    r_diag = np.abs(-1.0 / om[diag, diag] + G[diag, diag] + lam)
    nz = off & (om != 0)
    z = off & (om == 0)
    r_nz = np.abs(G[nz] + lam * np.sign(om[nz]))
    r_z = np.maximum(np.abs(G[z]) - lam, 0.0)
    parts = {"diag": float(r_diag.max(initial=0.0)), "nonzero": float(r_nz.max(initial=0.0)),
             "zero": float(r_z.max(initial=0.0))}
    return max(parts.values()), parts


# ---------------------------------------------------------------------------
# independent solvers (for "at convergence" checks)
# ---------------------------------------------------------------------------

def fit_cd(x, lam, omega0=None, tol=1e-12, max_sweeps=20000):
    """Cyclic coordinate descent on the separable objective
        phi_j(w) = -log w_j + w^T S w / 2 + lam ||w||_1      (column j of Om)
    (supplement, proof of Theorem 3.2).  Every coordinate update is exact:
      k != j:  w_k = S_{lam}(-c_k) / S_kk,          c_k = sum_{l != k} S_kl w_l
      k == j:  w_j = (-(c_j + lam) + sqrt((c_j + lam)^2 + 4 S_jj)) / (2 S_jj)
    All columns are updated together, coordinate by coordinate (columns do not
    interact).  Stops when the KKT residual is below ``tol``."""
    x = _f64(x)
    n, p = x.shape
    S = x.T @ x / n
    om = np.eye(p) if omega0 is None else _f64(omega0).copy()
    SW = S @ om
    cols = np.arange(p)
    for sweep in range(max_sweeps):
        for k in range(p):
            skk = S[k, k]
            row_old = om[k, :].copy()
            c = SW[k, :] - skk * row_old
            new = soft_threshold(-c, lam) / skk
            cj = c[k] + lam
            new[k] = (-cj + np.sqrt(cj * cj + 4.0 * skk)) / (2.0 * skk)
            delta = new - row_old
            if np.any(delta):
                om[k, :] = new
                SW += np.outer(S[:, k], delta)
        if sweep % 10 == 9 or sweep == max_sweeps - 1:
            SW = S @ om  # refresh the running product
            r, _ = kkt_residual(x, om, lam)
            if r <= tol:
                break
    del cols
    return om


def brute_column(x, lam, j, ftol=1e-15, gtol=1e-12):
    """Column j by a generic solver (scipy L-BFGS-B), for tiny p only.

    Smooth reformulation of phi_j: variables w_j in [1e-12, inf) and, for k != j,
    w_k = u_k - v_k with u_k, v_k >= 0, minimising
        -log w_j + ||X w||^2 / (2n) + lam * (w_j + sum_k (u_k + v_k))."""
    from scipy.optimize import minimize

    x = _f64(x)
    n, p = x.shape
    S = x.T @ x / n
    others = np.array([k for k in range(p) if k != j])

    def unpack(z):
        w = np.zeros(p)
        w[j] = z[0]
        w[others] = z[1:p] - z[p:]
        return w

    def fun(z):
        w = unpack(z)
        Sw = S @ w
        val = -np.log(z[0]) + 0.5 * w @ Sw + lam * (z[0] + np.sum(z[1:]))
        gw = Sw
        gz = np.empty_like(z)
        gz[0] = -1.0 / z[0] + gw[j] + lam
        gz[1:p] = gw[others] + lam
        gz[p:] = -gw[others] + lam
        return val, gz

    z0 = np.concatenate([[1.0], np.zeros(2 * (p - 1))])
    bounds = [(1e-12, None)] + [(0.0, None)] * (2 * (p - 1))
    r = minimize(fun, z0, jac=True, method="L-BFGS-B", bounds=bounds,
                 options={"ftol": ftol, "gtol": gtol, "maxiter": 100000, "maxfun": 200000})
    return unpack(r.x)
