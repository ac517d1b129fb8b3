"""FP64 oracle of the steps either side of the solver: the extended pseudo-BIC over a
lambda path (eq. 3.7), the debiasing refit on the estimated support (eq. 3.8), and
the reparametrisation back to the precision matrix and to partial correlations
(Sec. 2, the map T and its inverse).

TEST INFRASTRUCTURE ONLY (same rules as ``accord_oracle``).

Column form as everywhere in the oracle: Om = Omega_paper^T, column j is node-wise
problem j, and the smooth part is g(Om) = ||X Om||_F^2 / (2n) = tr(Omega^T Omega S)/2
in the paper's orientation.

  loss_part            the loss of eq. 3.2 without the penalty:
                       -sum_j log om_jj + g(Om)
  epbic                eq. 3.7: 2n * loss_part + ||Om||_0 (log n + 4 gamma log p),
                       ||Om||_0 = nonzero off-diagonal entries
  support              the estimated support S_lambda: nonzero entries, diagonal always in
  fit_fbs_weighted     Alg. 1 with one penalty per entry (lam_ij in [0, inf]); an
                       infinite penalty holds its entry at zero
  refit                eq. 3.8 solved as the paper says, by Alg. 1 with phi*lambda on
                       S_lambda and an infinite penalty off it
  theta_hat            Sec. 2: Theta = T^{-1}(Omega) = Omega_D Omega (paper orientation)
  partial_correlations Sec. 2: rho_ij = -(w_ij / w_jj + w_ji / w_ii) / 2 (paper
                       orientation), diagonal set to 1

Pins: tests/test_oracle_tuning_pins.py (a hand-worked 2 x 2 epBIC, the refit at
phi = 0 against its closed form per column, the refit with full support against
the plain fit, the restricted optimality conditions of eq. 3.8, the column-subset
replay, and T^{-1}(T(Theta)) = Theta with the partial correlations of Theta itself).
"""
from __future__ import annotations

import numpy as np

from .accord_oracle import FitResult, diag_root, lipschitz, line_search_test, soft_threshold


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# eq. 3.7: extended pseudo-BIC
# ---------------------------------------------------------------------------

def loss_part(x, om):
    """-log det Om_D + tr(Omega^T Omega S) / 2 = -sum_j log om_jj + ||X Om||_F^2 / (2n).
    +inf outside the domain (some om_jj <= 0)."""
    x, om = _f64(x), _f64(om)
    d = np.diagonal(om)
    if np.any(d <= 0):
        return np.inf
    w = x @ om
    return float(-np.sum(np.log(d)) + np.sum(w * w) / (2.0 * x.shape[0]))


def nnz_offdiag(om):
    """||Om||_0 of eq. 3.7: the number of nonzero off-diagonal entries."""
    om = _f64(om)
    return int(np.count_nonzero(om) - np.count_nonzero(np.diagonal(om)))


def epbic(x, om, gamma):
    """eq. 3.7 for one estimate: (2n) loss_part + ||Om||_0 log n + 4 gamma ||Om||_0 log p."""
    x = _f64(x)
    n, p = x.shape
    k = nnz_offdiag(om)
    return 2.0 * n * loss_part(x, om) + k * np.log(n) + 4.0 * gamma * k * np.log(p)


def epbic_path(x, omegas, gamma):
    """epBIC of every estimate along a lambda path and the index of the smallest
    (the first one on ties)."""
    vals = np.array([epbic(x, om, gamma) for om in omegas])
    return vals, int(np.argmin(vals))


# ---------------------------------------------------------------------------
# eq. 3.8: refit on the estimated support
# ---------------------------------------------------------------------------

def support(om):
    """S_lambda: entries of the estimate that are nonzero; the diagonal (positive on
    the domain) always belongs to it."""
    s = _f64(om) != 0
    np.fill_diagonal(s, True)
    return s


def fit_fbs_weighted(x, lam_mat, iters, omega0=None, tau0=1.0, beta=0.5, L=None, tol=0.0,
                     tau_replay=None, columns=None):
    """Alg. 1 for the objective -sum_j log om_jj + g(Om) + sum_ij lam_ij |om_ij|.

    The prox of eq. 3.5 is elementwise, so a per-entry penalty changes only each
    entry's threshold: off-diagonal S_{tau lam_ij}(a_ij), diagonal the positive root
    with lam_jj.  lam_ij = inf gives threshold inf and the entry 0.  The acceptance
    test involves g only and is unchanged.  The objective's penalty sums over entries
    with a finite penalty (the others are zero from the first iterate on).

    omega0: start (default I); entries with an infinite penalty are set to zero
    first (the start is projected onto the constraint set).  tau_replay, tol and
    columns: as in ``fit_fbs`` (with the steps fixed, column j depends only on
    column j of the start, of the penalty and on X)."""
    x = _f64(x)
    n, p = x.shape
    lam_mat = _f64(lam_mat)
    if np.any(~np.isfinite(lam_mat[np.diag_indices(p)])):
        raise ValueError("the diagonal needs a finite penalty (it is positive on the domain)")
    if L is None:
        L = lipschitz(x)
    om = np.eye(p) if omega0 is None else _f64(omega0).copy()
    if columns is not None:
        if tau_replay is None:
            raise ValueError("columns= needs tau_replay (the shared step couples columns)")
        cols = np.asarray(columns)
        om, lam_mat = om[:, cols].copy(), lam_mat[:, cols]
    else:
        cols = np.arange(p)
    finite = np.isfinite(lam_mat)
    om[~finite] = 0.0
    jj = np.arange(len(cols))
    lam_d = lam_mat[cols, jj]

    def _prox(o, g, tau):
        a = o - tau * g
        out = soft_threshold(a, tau * lam_mat)
        out[cols, jj] = diag_root(a[cols, jj], tau, lam_d)
        return out

    def _obj(o):
        w = x @ o
        g = float(np.sum(w * w) / (2 * n))
        d = o[cols, jj]
        if np.any(d <= 0):
            return g, np.inf
        pen = float(np.sum(lam_mat[finite] * np.abs(o[finite])))
        return g, g + float(-np.sum(np.log(d))) + pen

    res = FitResult(omega=om, iters=0, lipschitz=L)
    g_cur, f_cur = _obj(om)
    res.g.append(g_cur)
    res.f.append(f_cur)
    for t in range(iters):
        G = x.T @ (x @ om) / n
        tau = tau0 if tau_replay is None else float(tau_replay[t])
        k = 0
        while True:
            k += 1
            om_new = _prox(om, G, tau)
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


def refit_penalty(om_hat, lam, phi):
    """The per-entry penalty of eq. 3.8 as Alg. 1 takes it: phi * lambda on the
    support of om_hat, inf off it."""
    s = support(om_hat)
    out = np.full(s.shape, np.inf)
    out[s] = phi * lam
    return out


def refit(x, om_hat, lam, phi, iters, omega0=None, **kw):
    """eq. 3.8 by Alg. 1 with the penalty of ``refit_penalty``.  The start defaults to
    the first-stage estimate om_hat (it satisfies the support constraint)."""
    if not 0.0 <= phi <= 1.0:
        raise ValueError("phi must lie in [0, 1]")
    start = _f64(om_hat) if omega0 is None else omega0
    return fit_fbs_weighted(x, refit_penalty(om_hat, lam, phi), iters, omega0=start, **kw)


def refit_kkt_residual(x, om, lam_mat):
    """Optimality of eq. 3.8 restricted to the support (column form, G = S Om):
      diagonal:                  -1/om_jj + G_jj + lam_jj = 0
      support, om_ij != 0:       G_ij + lam_ij sign(om_ij) = 0
      support, om_ij == 0:       |G_ij| <= lam_ij
      off the support:           om_ij = 0 (no condition on G)
    Returns the largest violation."""
    x, om, lam_mat = _f64(x), _f64(om), _f64(lam_mat)
    G = x.T @ (x @ om) / x.shape[0]
    p = om.shape[0]
    jj = np.arange(p)
    fin = np.isfinite(lam_mat)
    off = ~np.eye(p, dtype=bool)
    r = [np.abs(-1.0 / om[jj, jj] + G[jj, jj] + lam_mat[jj, jj]).max(initial=0.0)]
    nz = fin & off & (om != 0)
    z = fin & off & (om == 0)
    r.append(np.abs(G[nz] + lam_mat[nz] * np.sign(om[nz])).max(initial=0.0))
    r.append(np.maximum(np.abs(G[z]) - lam_mat[z], 0.0).max(initial=0.0))
    r.append(np.abs(om[~fin]).max(initial=0.0))
    return float(max(r))


# ---------------------------------------------------------------------------
# Sec. 2: Theta = T^{-1}(Omega) and partial correlations
# ---------------------------------------------------------------------------

def theta_hat(om):
    """Theta = Omega_D Omega in the paper's orientation (row i of Omega scaled by
    omega_ii), returned in column form like every matrix here: Theta^T, whose column
    j is column j of Om scaled by om_jj."""
    om = _f64(om)
    return om * np.diagonal(om)[None, :]


def partial_correlations(om):
    """rho_ij = -(omega_ij / omega_jj + omega_ji / omega_ii) / 2 with omega in the
    paper's orientation (omega_ij = om_ji); symmetric, so the orientation of the result
    does not matter.  The diagonal is set to 1."""
    P = _f64(om).T           # paper orientation
    d = np.diagonal(P)
    rho = -0.5 * (P / d[None, :] + P.T / d[:, None])
    np.fill_diagonal(rho, 1.0)
    return rho


__all__ = ["loss_part", "nnz_offdiag", "epbic", "epbic_path", "support", "fit_fbs_weighted",
           "refit_penalty", "refit", "refit_kkt_residual", "theta_hat", "partial_correlations"]
