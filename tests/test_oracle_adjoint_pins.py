"""Pins of the differentiation oracle (oracle/adjoint_oracle.py): the reverse pass
against central finite differences of the unrolled fixed-step iteration, in FP64.

Finite differences see the soft threshold's kink only if a perturbation moves an
entry across |a| = tau lambda; every check below first asserts that the +-h runs
have the same zero pattern at every iteration, so the loss is smooth on the
segment and the central difference is accurate to O(h^2)."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import adjoint_oracle as ad


def _setup(n=40, p=14, nv=25, K=12, lam=0.12, seed=3):
    w = datagen.small_random_problem(n + nv, p, seed=seed)
    x = w.X[:n].astype(np.float64)
    xv = w.X[n:].astype(np.float64)
    taus = oracle.fit_fbs(x, lam, K).tau        # a backtracking run's steps, then replayed
    return x, xv, lam, np.array(taus)


def _pattern(x, lam, taus):
    return [it != 0 for it in ad.replay_iterates(x, lam, taus)]


def _same_pattern(a, b):
    return all(np.array_equal(u, v) for u, v in zip(a, b))


def test_val_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = 9
    xv = rng.normal(size=(30, p))
    om = rng.normal(0, 0.2, size=(p, p))
    om[np.diag_indices(p)] = rng.uniform(0.5, 2.0, size=p)
    g = ad.val_loss_grad(xv, om)
    h = 1e-6
    for (i, j) in [(0, 0), (3, 5), (8, 1), (4, 4)]:
        e = np.zeros_like(om)
        e[i, j] = h
        fd = (ad.val_loss(xv, om + e) - ad.val_loss(xv, om - e)) / (2 * h)
        assert fd == pytest.approx(g[i, j], rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("seed", [3, 4])
def test_adjoint_lambda_matches_finite_differences(seed):
    x, xv, lam, taus = _setup(seed=seed)
    obar = ad.val_loss_grad(xv, ad.replay_iterates(x, lam, taus)[-1])
    _, lbar, _ = ad.adjoint(x, lam, taus, obar)
    h = 1e-6
    assert _same_pattern(_pattern(x, lam + h, taus), _pattern(x, lam - h, taus))
    fd = (ad.unrolled_loss(x, xv, lam + h, taus) - ad.unrolled_loss(x, xv, lam - h, taus)) / (2 * h)
    assert lbar == pytest.approx(fd, rel=1e-6, abs=1e-9)
    assert abs(lbar) > 1e-3      # a non-trivial derivative


def test_adjoint_x_matches_finite_differences():
    x, xv, lam, taus = _setup()
    obar = ad.val_loss_grad(xv, ad.replay_iterates(x, lam, taus)[-1])
    _, _, xbar = ad.adjoint(x, lam, taus, obar)
    rng = np.random.default_rng(1)
    h = 1e-6
    scale = np.max(np.abs(xbar))
    for _ in range(12):
        i, j = rng.integers(0, x.shape[0]), rng.integers(0, x.shape[1])
        e = np.zeros_like(x)
        e[i, j] = h
        assert _same_pattern(_pattern(x + e, lam, taus), _pattern(x - e, lam, taus))
        fd = (ad.unrolled_loss(x + e, xv, lam, taus) - ad.unrolled_loss(x - e, xv, lam, taus)) / (2 * h)
        assert abs(xbar[i, j] - fd) <= 1e-6 * scale, (i, j, xbar[i, j], fd)


def test_adjoint_directional_derivative():
    """<X bar, D> + lambda_bar * dl equals the derivative of the loss along (D, dl)."""
    x, xv, lam, taus = _setup(seed=5)
    obar = ad.val_loss_grad(xv, ad.replay_iterates(x, lam, taus)[-1])
    _, lbar, xbar = ad.adjoint(x, lam, taus, obar)
    rng = np.random.default_rng(2)
    D = rng.normal(size=x.shape)
    dl = 0.3
    h = 1e-7
    assert _same_pattern(_pattern(x + h * D, lam + h * dl, taus), _pattern(x - h * D, lam - h * dl, taus))
    fd = (ad.unrolled_loss(x + h * D, xv, lam + h * dl, taus)
          - ad.unrolled_loss(x - h * D, xv, lam - h * dl, taus)) / (2 * h)
    assert np.sum(xbar * D) + lbar * dl == pytest.approx(fd, rel=1e-6)


def test_adjoint_omega0_matches_finite_differences():
    """The reverse pass also returns d l / d Om_0 (a start point off the identity)."""
    x, xv, lam, taus = _setup(K=6)
    p = x.shape[1]
    rng = np.random.default_rng(7)
    om0 = np.eye(p) * 1.3 + rng.normal(0, 0.05, size=(p, p)) * (rng.random((p, p)) < 0.3)
    its = ad.replay_iterates(x, lam, taus, om0)
    ob0, _, _ = ad.adjoint(x, lam, taus, ad.val_loss_grad(xv, its[-1]), omega0=om0)
    h = 1e-6
    for (i, j) in [(0, 0), (2, 5), (7, 7)]:
        e = np.zeros_like(om0)
        e[i, j] = h
        pp = [it != 0 for it in ad.replay_iterates(x, lam, taus, om0 + e)]
        pm = [it != 0 for it in ad.replay_iterates(x, lam, taus, om0 - e)]
        assert _same_pattern(pp, pm)
        fd = (ad.unrolled_loss(x, xv, lam, taus, om0 + e)
              - ad.unrolled_loss(x, xv, lam, taus, om0 - e)) / (2 * h)
        # rounding of the loss (about 10) over 2h limits the difference to ~1e-9
        assert ob0[i, j] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_adjoint_with_given_decisions():
    """adjoint(active=...) with the oracle's own kink decisions (the signs of
    kink_margins) is the plain reverse pass, bit for bit; a decision flipped at one
    entry of the last step changes lambda bar by that entry's term there, since at
    the last step Ob is the loss gradient itself and the flip touches only that term
    and what propagates to the earlier steps through Ab."""
    x, xv, lam, taus = _setup(K=6)
    its = ad.replay_iterates(x, lam, taus)
    ob = ad.val_loss_grad(xv, its[-1])
    ref = ad.adjoint(x, lam, taus, ob, iterates=its)
    own = [m > 0 for m in ad.kink_margins(x, lam, taus, its)]
    got = ad.adjoint(x, lam, taus, ob, iterates=its, active=own)
    assert np.array_equal(got[0], ref[0]) and got[1] == ref[1]
    assert np.array_equal(got[2], ref[2])
    # the margins are the distances of a_t from the kink, signed by the decision
    n = x.shape[0]
    a0 = its[0] - taus[0] * (x.T @ (x @ its[0])) / n
    assert np.allclose(ad.kink_margins(x, lam, taus, its)[0], np.abs(a0) - taus[0] * lam)
    # one flipped decision at the last step: with a one-step reverse pass (K = 1) the
    # change of lambda bar is exactly that entry's term -tau sign(a) Ob_ij
    t1 = taus[:1]
    its1 = its[:2]
    ob1 = ad.val_loss_grad(xv, its1[-1])
    m = ad.kink_margins(x, lam, t1, its1)[0]
    act = m > 0
    off = ~np.eye(x.shape[1], dtype=bool)
    i, j = np.argwhere(act & off)[0]
    flipped = act.copy()
    flipped[i, j] = False
    base = ad.adjoint(x, lam, t1, ob1, iterates=its1, active=[act])[1]
    fl = ad.adjoint(x, lam, t1, ob1, iterates=its1, active=[flipped])[1]
    a = its1[0] - t1[0] * (x.T @ (x @ its1[0])) / n
    assert fl - base == pytest.approx(t1[0] * np.sign(a[i, j]) * ob1[i, j], rel=1e-12, abs=1e-15)


def test_replay_with_given_decisions_and_rounding():
    """replay_iterates with the run's own kink decisions is the plain replay; with
    round_fp32 every iterate is the float32 rounding of a step from the previous one."""
    x, xv, lam, taus = _setup(K=5)
    its = ad.replay_iterates(x, lam, taus)
    own = [m > 0 for m in ad.kink_margins(x, lam, taus, its)]
    again = ad.replay_iterates(x, lam, taus, active=own)
    assert all(np.array_equal(a, b) for a, b in zip(its, again))
    r32 = ad.replay_iterates(x, lam, taus, active=own, round_fp32=True)
    one = ad.replay_iterates(x, lam, taus[2:3], omega0=r32[2], active=own[2:3])[1]
    assert np.array_equal(r32[3], one.astype(np.float32).astype(np.float64))
    assert 0 < np.abs(r32[-1] - its[-1]).max() < 1e-5
