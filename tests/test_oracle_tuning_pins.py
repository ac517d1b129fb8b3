"""Pins for the oracle of the steps around the solver (epBIC, refit, reparametrisation),
each against something fixed outside the oracle's own formulas.

  T1  epBIC (eq. 3.7) of a 2 x 2 estimate worked by hand, in both orientations
  T2  refit at phi = 0 (eq. 3.8): per column the problem is smooth on the support and
      has the closed form  w_A = S_AA^{-1} e_j / sqrt((S_AA^{-1})_jj)
  T3  refit at phi > 0: each column equals the plain column problem on the reduced
      data X_A, solved by a generic quasi-Newton method (p <= 8)
  T4  refit with full support and phi = 1 is the plain fit
  T5  refit at convergence meets the restricted optimality conditions; off-support
      entries stay exactly zero; the objective never increases
  T6  T^{-1}(T(Theta)) = Theta, and the partial correlations of T(Theta) are the
      textbook ones (conditional correlation from the covariance blocks)
  T7  a hand-worked non-symmetric 3 x 3 estimate (fixes the orientation)
plus mutation tests: a planted mistake makes a pin fail.
"""
import numpy as np
import pytest

import datagen
import oracle
from oracle import tuning_oracle as tu


def _x(n, p, seed):
    return datagen.small_random_problem(n, p, seed).X.astype(np.float64)


# ---------------------------------------------------------------- T1
# X = [[1,0],[0,1],[1,1]] (n = 3), column form Om = [[2, 0.5], [0, 1]].
# X Om = [[2, .5], [0, 1], [2, 1.5]], ||X Om||^2 = 4 + .25 + 0 + 1 + 4 + 2.25 = 11.5,
# so g = 11.5 / 6 and loss = -log 2 - log 1 + 11.5/6.  One nonzero off-diagonal entry.
# epBIC = 6 loss + log 3 + 4 gamma log 2 = 11.5 - 6 log 2 + log 3 + 4 gamma log 2.
# Paper orientation: Omega = Om^T = [[2, 0], [.5, 1]], Omega^T Omega = [[4.25, .5], [.5, 1]],
# S = [[2, 1], [1, 2]] / 3, tr(Omega^T Omega S) = (8.5 + .5 + .5 + 2) / 3 = 11.5 / 3.
_X1 = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
_OM1 = np.array([[2.0, 0.5], [0.0, 1.0]])


def _check_t1(epbic):
    for gamma in (0.25, 0.5, 1.0):
        want = 11.5 - 6 * np.log(2) + np.log(3) + 4 * gamma * np.log(2)
        assert epbic(_X1, _OM1, gamma) == pytest.approx(want, rel=1e-14)
    # a diagonal estimate pays no complexity term: epBIC = 2n (tr(S)/2 - sum log d)...
    d = np.diag([2.0, 0.5])
    # X d = [[2, 0], [0, .5], [2, .5]]: ||.||^2 = 8.5; loss = -log 1 + 8.5 / 6
    assert epbic(_X1, d, 1.0) == pytest.approx(8.5, rel=1e-14)


def test_t1_epbic_hand_worked():
    _check_t1(tu.epbic)
    omp = _OM1.T
    S = _X1.T @ _X1 / 3
    assert 0.5 * np.trace(omp.T @ omp @ S) == pytest.approx(11.5 / 6, rel=1e-15)
    assert tu.nnz_offdiag(_OM1) == 1


def test_t1_epbic_path_picks_minimum():
    x = _x(60, 12, 5)
    lams = [0.02, 0.1, 0.3, 0.8]
    oms = [oracle.fit_fbs(x, l, 400, tol=1e-12).omega for l in lams]
    vals, best = tu.epbic_path(x, oms, 0.5)
    assert best == int(np.argmin(vals))
    # larger penalties: sparser estimates, larger loss part (the loss is what the
    # penalty trades against)
    nnz = [tu.nnz_offdiag(o) for o in oms]
    loss = [tu.loss_part(x, o) for o in oms]
    assert nnz == sorted(nnz, reverse=True) and loss == sorted(loss)


# ---------------------------------------------------------------- T2
def _closed_form_phi0(x, sup):
    n, p = x.shape
    S = x.T @ x / n
    out = np.zeros((p, p))
    for j in range(p):
        A = np.flatnonzero(sup[:, j])
        Sinv = np.linalg.inv(S[np.ix_(A, A)])
        e = (A == j).astype(float)
        jj = int(np.flatnonzero(A == j)[0])
        out[A, j] = Sinv @ e / np.sqrt(Sinv[jj, jj])
    return out


def _random_support(p, prob, seed):
    rng = np.random.default_rng(seed)
    s = rng.random((p, p)) < prob
    np.fill_diagonal(s, True)
    om = np.where(s, rng.uniform(0.1, 1.0, (p, p)) * rng.choice([-1, 1], (p, p)), 0.0)
    np.fill_diagonal(om, rng.uniform(1.0, 2.0, p))
    return om


@pytest.mark.parametrize("n,p,prob,seed", [(40, 8, 0.3, 1), (25, 15, 0.2, 2), (80, 10, 0.6, 3)])
def test_t2_refit_phi0_closed_form(n, p, prob, seed):
    x = _x(n, p, seed)
    om_hat = _random_support(p, prob, seed)
    res = tu.refit(x, om_hat, lam=0.3, phi=0.0, iters=20000, tol=1e-14)
    want = _closed_form_phi0(x, tu.support(om_hat))
    assert np.max(np.abs(res.omega - want)) <= 1e-9 * np.max(np.abs(want))


# ---------------------------------------------------------------- T3
@pytest.mark.parametrize("p,phi,seed", [(6, 0.5, 4), (8, 1.0, 5), (7, 0.25, 6)])
def test_t3_refit_columns_vs_generic_solver(p, phi, seed):
    x = _x(30, p, seed)
    lam = 0.15
    om_hat = _random_support(p, 0.4, seed)
    res = tu.refit(x, om_hat, lam, phi, iters=20000, tol=1e-14)
    sup = tu.support(om_hat)
    for j in range(p):
        A = np.flatnonzero(sup[:, j])
        jj = int(np.flatnonzero(A == j)[0])
        if len(A) == 1:   # -1/w + S_jj w + phi lambda = 0, the positive root
            s_jj, c = x[:, j] @ x[:, j] / x.shape[0], phi * lam
            w = np.array([(-c + np.sqrt(c * c + 4 * s_jj)) / (2 * s_jj)])
        else:
            w = oracle.brute_column(x[:, A], phi * lam, jj)
        assert np.max(np.abs(res.omega[A, j] - w)) <= 2e-6
        assert np.all(res.omega[~sup[:, j], j] == 0.0)


# ---------------------------------------------------------------- T4
def test_t4_full_support_phi1_is_plain_fit():
    x = _x(50, 10, 7)
    rng = np.random.default_rng(7)
    om_hat = rng.uniform(0.1, 0.5, (10, 10))
    np.fill_diagonal(om_hat, 1.5)
    a = tu.refit(x, om_hat, 0.2, 1.0, iters=60)
    b = oracle.fit_fbs(x, 0.2, 60, omega0=om_hat)
    assert a.tau == b.tau and a.trials == b.trials
    assert np.array_equal(a.omega, b.omega)
    assert a.f == pytest.approx(b.f, rel=1e-14)


# ---------------------------------------------------------------- T5
def test_t5_refit_kkt_support_and_descent():
    x = _x(60, 20, 8)
    lam = 0.12
    om_hat = oracle.fit_fbs(x, lam, 3000, tol=1e-13).omega
    sup = tu.support(om_hat)
    assert 0 < tu.nnz_offdiag(om_hat) < 20 * 19
    pen = tu.refit_penalty(om_hat, lam, 0.5)
    res = tu.refit(x, om_hat, lam, 0.5, iters=5000, tol=1e-13)
    assert tu.refit_kkt_residual(x, res.omega, pen) <= 1e-8
    assert np.all(res.omega[~sup] == 0.0)
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(res.f, res.f[1:]))
    # debiasing: a smaller penalty on the same support moves the estimate towards the
    # unpenalised fit on that support: the loss part is lower than the first stage's
    assert tu.loss_part(x, res.omega) < tu.loss_part(x, om_hat)


# ---------------------------------------------------------------- T6
def _spd(p, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(p, p))
    return a @ a.T / p + 0.5 * np.eye(p)


def _textbook_partial_corr(theta):
    sigma = np.linalg.inv(theta)
    p = theta.shape[0]
    out = np.eye(p)
    for i in range(p):
        for j in range(p):
            if i == j:
                continue
            ab = [i, j]
            r = [k for k in range(p) if k not in ab]
            c = sigma[np.ix_(ab, ab)] - sigma[np.ix_(ab, r)] @ np.linalg.solve(
                sigma[np.ix_(r, r)], sigma[np.ix_(r, ab)])
            out[i, j] = c[0, 1] / np.sqrt(c[0, 0] * c[1, 1])
    return out


@pytest.mark.parametrize("p,seed", [(5, 1), (9, 2)])
def test_t6_reparametrisation_round_trip(p, seed):
    theta = _spd(p, seed)
    omega_paper = theta / np.sqrt(np.diagonal(theta))[:, None]     # T(Theta)
    om = omega_paper.T                                             # column form
    assert np.allclose(tu.theta_hat(om).T, theta, rtol=1e-13, atol=1e-14)
    assert np.allclose(tu.partial_correlations(om), _textbook_partial_corr(theta),
                       rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------- T7
# Paper orientation P = [[2, 2, 0], [.5, 4, 0], [0, 0, 1]]:
# rho_01 = -(P01 / P11 + P10 / P00) / 2 = -(2/4 + .5/2) / 2 = -0.375; rho_02 = rho_12 = 0.
# Theta = diag(P) P = [[4, 4, 0], [2, 16, 0], [0, 0, 1]].
_P7 = np.array([[2.0, 2.0, 0.0], [0.5, 4.0, 0.0], [0.0, 0.0, 1.0]])


def _check_t7(theta_hat, partial_correlations):
    om = _P7.T
    rho = partial_correlations(om)
    want = np.array([[1.0, -0.375, 0.0], [-0.375, 1.0, 0.0], [0.0, 0.0, 1.0]])
    assert np.array_equal(rho, want)
    th = theta_hat(om)
    assert np.array_equal(th.T, np.array([[4.0, 4.0, 0.0], [2.0, 16.0, 0.0], [0.0, 0.0, 1.0]]))


def test_t7_hand_worked_orientation():
    _check_t7(tu.theta_hat, tu.partial_correlations)


# ---------------------------------------------------------------- mutations
def test_mutation_dropped_log_n_breaks_t1():
    def bad(x, om, gamma):
        n, p = x.shape
        k = tu.nnz_offdiag(om)
        return 2.0 * n * tu.loss_part(x, om) + 4.0 * gamma * k * np.log(p)
    with pytest.raises(AssertionError):
        _check_t1(bad)


def test_mutation_counted_diagonal_breaks_t1():
    def bad(x, om, gamma):
        n, p = x.shape
        k = int(np.count_nonzero(om))
        return 2.0 * n * tu.loss_part(x, om) + k * np.log(n) + 4.0 * gamma * k * np.log(p)
    with pytest.raises(AssertionError):
        _check_t1(bad)


def test_mutation_transposed_orientation_breaks_t7():
    with pytest.raises(AssertionError):
        _check_t7(tu.theta_hat, lambda om: tu.partial_correlations(np.asarray(om).T))
    with pytest.raises(AssertionError):
        _check_t7(lambda om: tu.theta_hat(np.asarray(om).T).T, tu.partial_correlations)


def test_mutation_unmasked_refit_breaks_t2(monkeypatch):
    """A refit that forgets the support (penalty phi * lambda everywhere) misses the
    closed form."""
    monkeypatch.setattr(tu, "refit_penalty",
                        lambda om_hat, lam, phi: np.full(np.shape(om_hat), phi * lam))
    with pytest.raises(AssertionError):
        test_t2_refit_phi0_closed_form(40, 8, 0.3, 1)


def test_t8_refit_column_subset_replay():
    """With the steps fixed, a column subset of the refit reproduces those columns of
    the full run (the objective separates over columns)."""
    x = _x(45, 30, 9)
    om_hat = _random_support(30, 0.2, 9)
    full = tu.refit(x, om_hat, 0.1, 0.5, iters=40)
    cols = [0, 7, 29]
    sub = tu.refit(x, om_hat, 0.1, 0.5, iters=40, tau_replay=full.tau, columns=cols)
    assert np.allclose(sub.omega, full.omega[:, cols], rtol=1e-12, atol=1e-14)
