"""Pins for the FP64 oracle: each test checks it against something the paper or
the mathematics fixes independently of the oracle's own formulas.

  P1  prox: eq. 3.5 entries are the 1-D minimisers they claim to be
  P2  objective at the identity: f(I) = tr(S)/2 + lambda p (Theorem 3.3)
  P3  gradient: central finite differences of g; paper form Omega S transposed
  P4  lambda = 0, n > p: closed form T(S^{-1}) (Sec. 3.1), column form
  P5  population case S = Sigma*: Omega* = T(Theta*) (Theorem 3.1)
  P6  large lambda: diagonal estimate, closed-form diagonal and lambda_max
  P7  every accepted step: sufficient decrease, monotone f, step floor, and the
      accepted step is the first of tau0, beta tau0, ... that passes
  P8  KKT (eq. 3.3) at convergence
  P9  FBS and an independent coordinate-descent solver agree (uniqueness, Thm 3.2)
  P10 brute force (generic quasi-Newton) for p <= 20
  P11 linear convergence, backtracking faster than the fixed step 1/L (Sec. 5.1)
  P12 column-subset replay reproduces the full run's columns (separability)
  P13 the warm-started step variant: each accepted step is the first passing one from
      min(tau0, tau_{t-1}/beta), f decreases, fewer trials, and the same fixed point
      (KKT, coordinate descent)
plus mutation tests: a planted mistake in the oracle makes a pin fail.
"""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st
from scipy.optimize import minimize_scalar

import datagen
import oracle
from oracle import accord_oracle as ao


def _problem(n, p, seed):
    return datagen.small_random_problem(n, p, seed).X.astype(np.float64)


# ---------------------------------------------------------------- P1
@settings(max_examples=200, deadline=None)
@given(y=st.floats(-20, 20), tau=st.floats(1e-3, 5), lam=st.floats(0, 2))
def test_p1_diag_root_is_1d_minimiser(y, tau, lam):
    w = float(oracle.diag_root(y, tau, lam))
    assert w > 0
    # it is the minimiser of -log w + lam w + (w - y)^2/(2 tau) over w > 0
    phi = lambda v: -np.log(v) + lam * v + (v - y) ** 2 / (2 * tau)
    r = minimize_scalar(phi, bounds=(1e-12, max(1.0, abs(y) + 10 * tau + 10)), method="bounded",
                        options={"xatol": 1e-12})
    assert phi(w) <= phi(r.x) + 1e-10 * max(1.0, abs(phi(w)))
    # first-order condition
    assert abs(-1 / w + lam + (w - y) / tau) <= 1e-8 * (1 / w + abs(lam) + abs(w - y) / tau + 1)


@settings(max_examples=200, deadline=None)
@given(x=st.floats(-10, 10), a=st.floats(0, 5))
def test_p1_soft_threshold_is_1d_minimiser(x, a):
    s = float(oracle.soft_threshold(x, a))
    # argmin_w  a|w| + (w - x)^2 / 2, checked on a dense grid around the answer
    grid = np.linspace(-12, 12, 240001)
    psi = a * np.abs(grid) + (grid - x) ** 2 / 2
    w_grid = grid[np.argmin(psi)]
    assert abs(s - w_grid) <= 2e-4
    assert a * abs(s) + (s - x) ** 2 / 2 <= psi.min() + 1e-12


def test_p1_soft_threshold_tie_is_zero():
    assert oracle.soft_threshold(0.3, 0.3) == 0.0
    assert oracle.soft_threshold(-0.3, 0.3) == 0.0
    assert oracle.soft_threshold(0.0, 0.0) == 0.0


def test_p1_prox_matrix_entries_minimise_their_own_term():
    rng = np.random.default_rng(7)
    p, tau, lam = 4, 0.37, 0.6
    om = rng.normal(size=(p, p)) + 2 * np.eye(p)
    g = rng.normal(size=(p, p))
    out = oracle.prox(om, g, tau, lam)
    a = om - tau * g
    for i in range(p):
        for j in range(p):
            if i == j:
                f = lambda v: -np.log(v) + lam * v + (v - a[i, j]) ** 2 / (2 * tau)
                r = minimize_scalar(f, bounds=(1e-12, 50), method="bounded", options={"xatol": 1e-12})
            else:
                f = lambda v: lam * abs(v) + (v - a[i, j]) ** 2 / (2 * tau)
                r = minimize_scalar(f, bounds=(-50, 50), method="bounded", options={"xatol": 1e-12})
            assert f(out[i, j]) <= f(r.x) + 1e-10


# ---------------------------------------------------------------- P2
def test_p2_objective_at_identity():
    w = datagen.workload("er200")
    x = w.X.astype(np.float64)
    p = w.p
    g, h, f = oracle.objective(x, np.eye(p), w.lam)
    # standardised columns: tr(S) = p up to float32 rounding of X
    assert abs(f - (p / 2 + w.lam * p)) < 1e-4
    assert abs(h - w.lam * p) < 1e-12


def test_p2_smooth_equals_paper_trace_form():
    x = _problem(15, 6, 1)
    rng = np.random.default_rng(0)
    om = rng.normal(size=(6, 6))
    S = x.T @ x / x.shape[0]
    om_paper = om.T
    assert np.isclose(oracle.smooth(x, om), 0.5 * np.trace(om_paper.T @ om_paper @ S), rtol=1e-12)


def test_p2_objective_domain():
    x = _problem(10, 3, 2)
    om = np.eye(3)
    om[1, 1] = -0.5
    assert oracle.objective(x, om, 0.1)[2] == np.inf


# ---------------------------------------------------------------- P3
def test_p3_gradient_matches_finite_differences():
    x = _problem(12, 5, 3)
    rng = np.random.default_rng(1)
    om = rng.normal(size=(5, 5))
    G = oracle.grad(x, om)
    h = 1e-6
    fd = np.zeros_like(om)
    for i in range(5):
        for j in range(5):
            e = np.zeros_like(om)
            e[i, j] = h
            fd[i, j] = (oracle.smooth(x, om + e) - oracle.smooth(x, om - e)) / (2 * h)
    assert np.allclose(G, fd, atol=1e-7)
    # the paper's gradient Omega S (row form) is the transpose
    S = x.T @ x / x.shape[0]
    assert np.allclose((om.T @ S).T, G, atol=1e-12)


def test_p3_lipschitz_is_largest_curvature():
    x = _problem(20, 8, 4)
    L = oracle.lipschitz(x)
    S = x.T @ x / x.shape[0]
    assert np.isclose(L, np.linalg.eigvalsh(S)[-1], rtol=1e-12)


# ---------------------------------------------------------------- P4
def test_p4_lambda_zero_closed_form():
    x = _problem(80, 8, 5)
    S = x.T @ x / x.shape[0]
    Si = np.linalg.inv(S)
    expect = Si / np.sqrt(np.diag(Si))[None, :]        # columns scaled: (T(S^-1))^T
    r = oracle.fit_fbs(x, 0.0, 5000, tol=1e-15)
    assert np.allclose(r.omega, expect, atol=1e-9)
    # the row-scaled matrix is NOT the answer in the column convention
    wrong = Si / np.sqrt(np.diag(Si))[:, None]
    assert np.abs(r.omega - wrong).max() > 1e-3


# ---------------------------------------------------------------- P5
def test_p5_population_case():
    w = datagen.er_workload(n=50, p=12, prob=0.3, lam=0.0, iters=0, key=5)
    theta = w.meta["theta"]
    sigma = np.linalg.inv(theta)
    n = 40
    rng = np.random.default_rng(3)
    q, _ = np.linalg.qr(rng.normal(size=(n, 12)))
    R = np.linalg.cholesky(sigma).T                      # sigma = R^T R
    x = np.sqrt(n) * q @ R                               # X^T X / n = sigma exactly
    r = oracle.fit_fbs(x, 0.0, 20000, tol=1e-15)
    omega_star_paper = theta / np.sqrt(np.diag(theta))[:, None]   # Theta_D^{-1/2} Theta
    assert np.allclose(r.omega, omega_star_paper.T, atol=1e-8)


# ---------------------------------------------------------------- P6
def _lambda_max(S):
    # smallest lambda at which the diagonal estimate satisfies |G_ij| <= lambda
    def viol(lam):
        d = (-lam + np.sqrt(lam ** 2 + 4 * np.diag(S))) / (2 * np.diag(S))
        G = S * d[None, :]
        off = G - np.diag(np.diag(G))
        return np.abs(off).max() - lam
    lo, hi = 0.0, 10.0
    for _ in range(200):
        mid = (lo + hi) / 2
        if viol(mid) > 0:
            lo = mid
        else:
            hi = mid
    return hi


def test_p6_large_lambda_is_diagonal_closed_form():
    x = _problem(30, 10, 6)
    S = x.T @ x / x.shape[0]
    lmax = _lambda_max(S)
    lam = 1.05 * lmax
    r = oracle.fit_fbs(x, lam, 3000, tol=1e-14)
    off = r.omega - np.diag(np.diag(r.omega))
    assert np.count_nonzero(off) == 0
    d = (-lam + np.sqrt(lam ** 2 + 4 * np.diag(S))) / (2 * np.diag(S))
    assert np.allclose(np.diag(r.omega), d, atol=1e-10)
    r2 = oracle.fit_fbs(x, 0.9 * lmax, 3000, tol=1e-14)
    off2 = r2.omega - np.diag(np.diag(r2.omega))
    assert np.count_nonzero(off2) > 0


# ---------------------------------------------------------------- P7
@pytest.mark.parametrize("seed,n,p,lam", [(0, 40, 60, 0.1), (1, 100, 30, 0.05), (2, 20, 50, 0.2)])
def test_p7_line_search_invariants(seed, n, p, lam):
    x = _problem(n, p, seed)
    L = oracle.lipschitz(x)
    tau0, beta = 1.0, 0.5
    r = oracle.fit_fbs(x, lam, 60, L=L, tau0=tau0, beta=beta)
    om = np.eye(p)
    for t in range(r.iters):
        G = oracle.grad(x, om)
        tau = r.tau[t]
        om_next = oracle.prox(om, G, tau, lam)
        f_t = oracle.objective(x, om, lam)[2]
        f_n = oracle.objective(x, om_next, lam)[2]
        d2 = np.sum((om_next - om) ** 2)
        # sufficient decrease (proof of Theorem 3.3) and monotone f
        assert f_n + d2 / (2 * tau) <= f_t + 1e-9 * max(1, abs(f_t))
        assert np.isclose(r.f[t + 1], f_n, rtol=1e-12)
        # step floor tau_t >= min(tau0, beta/L)
        assert tau >= min(tau0, beta / L) * (1 - 1e-12)
        # the accepted step is tau0 beta^(k-1), and the previous trial failed the
        # sufficient-decrease inequality.  It is evaluated here as
        # ||X D||^2/(2n) > ||D||^2/(2 tau): g is quadratic, so this is the same
        # inequality without subtracting two nearly equal values of g; where the
        # margin is large the form written with g values must agree.
        k = r.trials[t]
        assert np.isclose(tau, tau0 * beta ** (k - 1), rtol=1e-14)
        if k > 1:
            tb = tau / beta
            om_b = oracle.prox(om, G, tb, lam)
            db = om_b - om
            xd = x @ db
            lhs, rhs = np.sum(xd * xd) / (2 * n), np.sum(db * db) / (2 * tb)
            assert lhs > rhs
            g0 = oracle.smooth(x, om)
            if lhs - rhs > 1e-10 * max(1.0, g0):
                assert oracle.smooth(x, om_b) > g0 + np.sum(db * G) + rhs
        om = om_next
    assert np.allclose(om, r.omega)


# ---------------------------------------------------------------- P8, P9, P10
@pytest.mark.parametrize("seed,n,p,lam", [(3, 15, 25, 0.15), (4, 60, 20, 0.08)])
def test_p8_p9_fbs_and_cd_agree_at_convergence(seed, n, p, lam):
    x = _problem(n, p, seed)
    r = oracle.fit_fbs(x, lam, 50000, tol=1e-15)
    res, _ = oracle.kkt_residual(x, r.omega, lam)
    assert res < 1e-9
    cd = oracle.fit_cd(x, lam, tol=1e-12)
    assert oracle.kkt_residual(x, cd, lam)[0] < 1e-11
    assert np.allclose(r.omega, cd, atol=1e-8)
    # identical support away from near-ties
    sup_a = (np.abs(r.omega) > 1e-7)
    sup_b = (np.abs(cd) > 1e-7)
    assert np.array_equal(sup_a, sup_b)


def test_p10_brute_force_small():
    x = _problem(12, 8, 8)
    lam = 0.12
    r = oracle.fit_fbs(x, lam, 50000, tol=1e-15)
    for j in range(8):
        wj = oracle.brute_column(x, lam, j)
        assert np.allclose(r.omega[:, j], wj, atol=2e-5), j


# ---------------------------------------------------------------- P11
def test_p11_linear_convergence_and_backtracking_faster():
    w = datagen.er_workload(n=100, p=60, prob=0.1, lam=0.1, iters=0, key=11)
    x = w.X.astype(np.float64)
    L = oracle.lipschitz(x)
    ref = oracle.fit_fbs(x, 0.1, 20000, L=L, tol=1e-15)
    fstar = ref.f[-1]
    bt = oracle.fit_fbs(x, 0.1, 400, L=L)
    fx = oracle.fit_fbs(x, 0.1, 400, L=L, tau0=1.0 / L, beta=1.0)
    gap_bt = np.array(bt.f) - fstar
    gap_fx = np.array(fx.f) - fstar
    # geometric decrease: every 20 iterations the gap shrinks by a fixed factor
    idx = [t for t in range(0, 200, 20) if gap_bt[t + 20] > 1e-11]
    assert idx
    ratios = [gap_bt[t + 20] / gap_bt[t] for t in idx]
    assert max(ratios) < 0.9
    first = lambda gap: int(np.argmax(gap < 1e-8))
    assert first(gap_bt) < first(gap_fx)


# ---------------------------------------------------------------- P12
def test_p12_column_subset_replay():
    x = _problem(30, 40, 12)
    r = oracle.fit_fbs(x, 0.1, 40)
    cols = [0, 7, 19, 39]
    sub = oracle.fit_fbs(x, 0.1, 40, tau_replay=r.tau, columns=cols)
    assert np.allclose(sub.omega, r.omega[:, cols], atol=1e-13)



def test_p12_lean_replay_is_the_same_replay():
    """record=False (no objective or test bookkeeping, products over the nonzeros of
    the iterate, the prox by column chunks on threads) follows the same iterates as the
    recorded replay: on the full matrix, on a column subset sparse enough for the sparse
    product, and on a block large enough for the chunked prox."""
    x = _problem(30, 40, 12)
    r = oracle.fit_fbs(x, 0.1, 40)
    lean = oracle.fit_fbs(x, 0.1, 40, tau_replay=r.tau, record=False)
    assert np.allclose(lean.omega, r.omega, atol=1e-13)
    assert np.allclose(lean.delta_fro, r.delta_fro, rtol=1e-12, atol=1e-15)
    # p = 2048, 512 columns: 2^20 entries, so the left product runs on the nonzeros
    xb = _problem(64, 2048, 13)
    taus = [0.02, 0.04, 0.02, 0.01, 0.02]
    cols = np.r_[0:256, 1792:2048]
    full = oracle.fit_fbs(xb, 0.5, 5, tau_replay=taus, columns=cols)
    lean = oracle.fit_fbs(xb, 0.5, 5, tau_replay=taus, columns=cols, record=False)
    assert np.count_nonzero(lean.omega) < 0.003 * lean.omega.size
    assert np.allclose(lean.omega, full.omega, atol=1e-13)
    # p = 4096, 1024 columns (2^22 entries, a dense iterate): the chunked prox
    xc = _problem(32, 4096, 14)
    cols = np.arange(0, 4096, 4)
    taus = [0.05, 0.1, 0.05]
    full = oracle.fit_fbs(xc, 0.2, 3, tau_replay=taus, columns=cols)
    lean = oracle.fit_fbs(xc, 0.2, 3, tau_replay=taus, columns=cols, record=False)
    assert np.count_nonzero(lean.omega) > 0.2 * lean.omega.size
    assert np.array_equal(lean.omega, full.omega)
    assert np.allclose(lean.delta_fro, full.delta_fro, rtol=1e-12)
    with pytest.raises(ValueError):
        oracle.fit_fbs(xb, 0.2, 5, record=False)


def test_x_times_is_the_product():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(20, 1024))
    om = np.where(rng.random((1024, 1024)) < 0.01, rng.normal(size=(1024, 1024)), 0.0)
    assert np.allclose(ao.x_times(x, om), x @ om, rtol=1e-13, atol=1e-13)
    assert np.array_equal(ao.identity_columns(7, [0, 6, 3]), np.eye(7)[:, [0, 6, 3]])

# ---------------------------------------------------------------- mutations
def test_mutation_transposed_gradient_breaks_p4(monkeypatch):
    """A transposed operand in the smooth part (row form gradient on the column
    iterate) converges to the row-scaled matrix and fails P4."""
    x = _problem(80, 6, 5)
    S = x.T @ x / x.shape[0]
    Si = np.linalg.inv(S)
    expect = Si / np.sqrt(np.diag(Si))[None, :]
    orig = ao.fit_fbs

    def bad_fit(xx, lam, iters, **kw):
        xx = np.asarray(xx, dtype=np.float64)
        om = np.eye(xx.shape[1])
        Sx = xx.T @ xx / xx.shape[0]
        for _ in range(iters):
            G = om @ Sx                       # planted mistake
            om = ao.prox(om, G, 0.05, lam)
        return om

    om = bad_fit(x, 0.0, 3000)
    assert not np.allclose(om, expect, atol=1e-6)
    assert np.allclose(orig(x, 0.0, 5000, tol=1e-15).omega, expect, atol=1e-9)


def test_mutation_dropped_diag_penalty_breaks_p6(monkeypatch):
    """Dropping the -tau*lambda term from the diagonal root changes the large-lambda
    diagonal and fails P6."""
    x = _problem(30, 10, 6)
    S = x.T @ x / x.shape[0]
    lam = 1.05 * _lambda_max(S)
    monkeypatch.setattr(ao, "diag_root",
                        lambda y, tau, lam_: (np.asarray(y) + np.sqrt(np.asarray(y) ** 2 + 4 * tau)) / 2)
    r = ao.fit_fbs(x, lam, 3000, tol=1e-14)
    d = (-lam + np.sqrt(lam ** 2 + 4 * np.diag(S))) / (2 * np.diag(S))
    assert not np.allclose(np.diag(r.omega), d, atol=1e-6)


def test_mutation_sign_flip_breaks_p1():
    bad = lambda x, a: -np.sign(x) * np.maximum(np.abs(x) - a, 0.0)
    x, a = 2.0, 0.5
    psi = lambda w: a * abs(w) + (w - x) ** 2 / 2
    assert psi(bad(x, a)) > psi(oracle.soft_threshold(x, a)) + 1.0


# ---------------------------------------------------------------- P13
@pytest.mark.parametrize("seed,n,p,lam", [(1, 40, 15, 0.1), (2, 25, 30, 0.2)])
def test_p13_warm_started_steps(seed, n, p, lam):
    x = _problem(n, p, seed)
    L = oracle.lipschitz(x)
    tau0, beta = 1.0, 0.5
    r = oracle.fit_fbs(x, lam, 80, L=L, tau0=tau0, beta=beta, warm_tau=True)
    om = np.eye(p)
    for t in range(r.iters):
        G = oracle.grad(x, om)
        start = tau0 if t == 0 else min(tau0, r.tau[t - 1] / beta)
        # the accepted step is start beta^(k-1); every earlier candidate failed the
        # inequality and the accepted one passes it (or sits at the floor)
        k = r.trials[t]
        assert np.isclose(r.tau[t], start * beta ** (k - 1), rtol=1e-14)
        for j in range(k):
            tau = start * beta ** j
            nxt = oracle.prox(om, G, tau, lam)
            v = x @ (nxt - om)
            ok = np.sum(v * v) / n <= np.sum((nxt - om) ** 2) / tau
            assert ok == (j == k - 1) or (j == k - 1 and tau <= 1 / L)
        om_next = oracle.prox(om, G, r.tau[t], lam)
        assert oracle.objective(x, om_next, lam)[2] <= oracle.objective(x, om, lam)[2] + 1e-12
        om = om_next
    # with tau0 well above the accepted steps, the plain rule pays the same backtracking
    # every iteration and the warm start does not (a property of these inputs)
    plain = oracle.fit_fbs(x, lam, 80, L=L, tau0=8.0, beta=beta)
    warm = oracle.fit_fbs(x, lam, 80, L=L, tau0=8.0, beta=beta, warm_tau=True)
    assert sum(warm.trials) < 0.7 * sum(plain.trials)
    conv = oracle.fit_fbs(x, lam, 50000, L=L, tol=1e-15, warm_tau=True)
    assert oracle.kkt_residual(x, conv.omega, lam)[0] < 1e-9
    assert np.allclose(conv.omega, oracle.fit_cd(x, lam, tol=1e-12), atol=1e-8)
