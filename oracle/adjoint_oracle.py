"""FP64 oracle of the differentiation form: gradients of a held-out loss through K
unrolled ACCORD-FBS iterations.

TEST INFRASTRUCTURE ONLY (same rules as ``accord_oracle``).

Forward (column form, as everywhere in the oracle): with the step sizes tau_t held
fixed (recorded from a backtracking run and replayed), Alg. 1's iteration is
    G_t   = S Om_t,            S = X^T X / n          (grad of g, eq. 3.4)
    A_t   = Om_t - tau_t G_t                           (forward step)
    Om_t+1 = prox(A_t; tau_t, lambda)                  (eq. 3.5)
from Om_0 = I.  The held-out loss is the pseudolikelihood part of eq. 3.2 on
validation data X_v (n_v rows), without the penalty:
    l_val(Om) = -sum_j log Om_jj + ||X_v Om||_F^2 / (2 n_v).

Backward (reverse-mode, written out from the chain rule): with Ob = dl/dOm_t+1,
  * prox Jacobian, entry by entry (eq. 3.5 is elementwise):
      off-diagonal  w = S_{tau lambda}(a):   dw/da = 1{|a| > tau lambda},
                                             dw/dlambda = -tau sign(a) 1{|a| > tau lambda}
                    (derivative 0 at the kink |a| = tau lambda);
      diagonal      w = (b + sqrt(b^2 + 4 tau)) / 2, b = a - tau lambda:
                    dw/da = (1 + b / sqrt(b^2 + 4 tau)) / 2,  dw/dlambda = -tau dw/da;
  * Ab = Ob * dw/da,  lambda_bar += sum(Ob * dw/dlambda);
  * A = Om - (tau/n) X^T X Om, so
      Om_t bar = Ab - tau S Ab                          (S symmetric),
      X bar   += -(tau/n) (X Om Ab^T + X Ab Om^T).
The kink decision |a| > tau lambda is a discrete outcome decided by floating point.
``adjoint(..., active=...)`` takes it from the caller for every off-diagonal entry
(one boolean mask per step), so that a comparison with a run whose iterates are
rounded differently can use that run's decisions: an entry whose |a| lies within
that run's rounding of tau lambda may sit on the other side of the kink there, and
its derivative jumps between 0 and 1.  A caller must first check that the two sets of
decisions differ only inside that rounding band.

Pins: tests/test_oracle_adjoint_pins.py (central finite differences in FP64 on
lambda and on entries of X, a directional-derivative (dot-product) test, and the
loss gradient against finite differences).
"""
from __future__ import annotations

import numpy as np

from .accord_oracle import diag_root, soft_threshold


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def replay_iterates(x, lam, taus, omega0=None, active=None, round_fp32=False):
    """[Om_0, ..., Om_K] of the fixed-step iteration (fresh G = S Om each step).

    For perturbation studies: active (one p x p boolean mask per step) fixes the
    off-diagonal kink decisions (an active entry takes a - tau lambda sign(a), an
    inactive one 0), and round_fp32 rounds every iterate to float32, as a run that
    keeps its iterates in FP32 does."""
    x = _f64(x)
    n, p = x.shape
    om = np.eye(p) if omega0 is None else _f64(omega0).copy()
    out = [om]
    jj = np.arange(p)
    for t, tau in enumerate(taus):
        g = x.T @ (x @ om) / n
        a = om - tau * g
        if active is None:
            nw = soft_threshold(a, tau * lam)
        else:
            nw = np.where(active[t], np.sign(a) * (np.abs(a) - tau * lam), 0.0)
        nw[jj, jj] = diag_root(a[jj, jj], tau, lam)
        om = nw.astype(np.float32).astype(np.float64) if round_fp32 else nw
        out.append(om)
    return out


def val_loss(xv, om):
    """l_val(Om) = -sum_j log Om_jj + ||X_v Om||_F^2 / (2 n_v)."""
    xv = _f64(xv)
    d = np.diagonal(om)
    if np.any(d <= 0):
        return np.inf
    w = xv @ om
    return float(-np.sum(np.log(d)) + np.sum(w * w) / (2 * xv.shape[0]))


def val_loss_grad(xv, om):
    """d l_val / d Om = S_v Om - diag(1 / Om_jj)."""
    xv = _f64(xv)
    g = xv.T @ (xv @ om) / xv.shape[0]
    g[np.diag_indices_from(g)] -= 1.0 / np.diagonal(om)
    return g


def adjoint(x, lam, taus, obar_final, omega0=None, iterates=None, active=None):
    """Reverse pass: returns (Om_0 bar, lambda bar, X bar) for the loss whose
    gradient at Om_K is ``obar_final``.  active: None, or one p x p boolean mask per
    step giving the off-diagonal kink decisions |a_t| > tau_t lambda to use instead of
    this function's own (the diagonal has no kink and ignores it)."""
    x = _f64(x)
    n, p = x.shape
    its = replay_iterates(x, lam, taus, omega0) if iterates is None else iterates
    ob = _f64(obar_final).copy()
    lbar = 0.0
    xbar = np.zeros_like(x)
    jj = np.arange(p)
    for t in range(len(taus) - 1, -1, -1):
        tau = float(taus[t])
        om = its[t]
        g = x.T @ (x @ om) / n
        a = om - tau * g
        thr = tau * lam
        act = np.abs(a) > thr if active is None else np.asarray(active[t], dtype=bool)
        dwda = act.astype(np.float64)
        dwdl = -tau * np.sign(a) * act
        b = a[jj, jj] - thr
        r = np.sqrt(b * b + 4.0 * tau)
        dd = 0.5 * (1.0 + b / r)
        dwda[jj, jj] = dd
        dwdl[jj, jj] = -tau * dd
        ab = ob * dwda
        lbar += float(np.sum(ob * dwdl))
        xab = x @ ab
        xom = x @ om
        xbar += -(tau / n) * (xom @ ab.T + xab @ om.T)
        ob = ab - tau * (x.T @ xab) / n
    return ob, lbar, xbar


def unrolled_loss(x, xv, lam, taus, omega0=None):
    """l_val(Om_K) of the fixed-step iteration from Om_0 (for finite differences)."""
    return val_loss(xv, replay_iterates(x, lam, taus, omega0)[-1])


def kink_margins(x, lam, taus, iterates=None):
    """Per step, the signed distance |a_t| - tau_t lambda of every entry from the kink
    of the soft threshold (positive: active), with a_t = Om_t - tau_t S Om_t."""
    x = _f64(x)
    n = x.shape[0]
    its = replay_iterates(x, lam, taus) if iterates is None else iterates
    out = []
    for t, tau in enumerate(taus):
        om = its[t]
        a = om - tau * (x.T @ (x @ om)) / n
        out.append(np.abs(a) - tau * lam)
    return out


__all__ = ["replay_iterates", "val_loss", "val_loss_grad", "adjoint", "kink_margins",
           "unrolled_loss"]
