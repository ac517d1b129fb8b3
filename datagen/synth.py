"""Seeded synthetic inputs for the ACCORD workloads.

This module only builds test and benchmark *inputs*: sparse precision matrices
Theta, Gaussian samples X ~ N(0, Theta^{-1}), column standardisation, bootstrap
row draws, and the lambda grid.  It contains none of the estimator's arithmetic
(no objective, gradient, proximal map or line search), so both the FP64 oracle
and the GPU path can consume what it produces without sharing method code.

Sampling follows the paper's recipe for Gaussian data with a prescribed sparse
precision (Sec. 5.2): factor Theta = L L^T and set x = L^{-T} z with
z ~ N(0, I_p), so that x ~ N(0, (L L^T)^{-1}).  Data are centred (Sec. 2, the
sample covariance S = X^T X / n assumes centred columns) and, as the workloads
ask, every column is scaled to unit mean square (so diag(S) = 1).

Random streams: workload k uses np.random.SeedSequence([2412, 11554, k]) spawned
into three independent generators (graph/weights, samples, auxiliary draws).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

SEED_ROOT = (2412, 11554)


def rngs(key: int, extra: int | None = None):
    """Three independent generators (theta, data, aux) for workload ``key``."""
    entropy = [SEED_ROOT[0], SEED_ROOT[1], int(key)]
    if extra is not None:
        entropy.append(int(extra))
    ss = np.random.SeedSequence(entropy)
    return [np.random.default_rng(s) for s in ss.spawn(3)]


# ---------------------------------------------------------------------------
# sparse precision matrices
# ---------------------------------------------------------------------------

def er_precision(p: int, prob: float, wlo: float, whi: float, min_eig: float,
                 rng: np.random.Generator) -> np.ndarray:
    """Erdos-Renyi precision: each upper-triangle edge present with prob ``prob``,
    weight U[wlo, whi] with a random sign, mirrored; the diagonal is then set to
    a constant shift so that the smallest eigenvalue equals ``min_eig``."""
    theta = np.zeros((p, p))
    iu, ju = np.triu_indices(p, k=1)
    keep = rng.random(iu.size) < prob
    iu, ju = iu[keep], ju[keep]
    w = rng.uniform(wlo, whi, size=iu.size) * rng.choice([-1.0, 1.0], size=iu.size)
    theta[iu, ju] = w
    theta[ju, iu] = w
    lam_min = np.linalg.eigvalsh(theta)[0] if p > 0 else 0.0
    theta[np.diag_indices(p)] = min_eig - lam_min
    return theta


def ba_tree_edges(b: int, rng: np.random.Generator) -> np.ndarray:
    """Barabasi-Albert graph with m = 1 on ``b`` nodes (a random tree): node v >= 2
    attaches to one earlier node drawn with probability proportional to degree.
    Written here (not taken from a graph library) so the edge list is stable."""
    if b < 2:
        return np.zeros((0, 2), dtype=np.int64)
    edges = [(1, 0)]
    # list of edge endpoints: sampling uniformly from it = sampling by degree
    ends = [0, 1]
    for v in range(2, b):
        u = ends[int(rng.integers(len(ends)))]
        edges.append((v, u))
        ends.extend((u, v))
    return np.asarray(edges, dtype=np.int64)


def ba_block_precision(b: int, wlo: float, whi: float, shift: float,
                       rng: np.random.Generator) -> np.ndarray:
    """One power-law block: BA(m=1) tree, weights +-U[wlo, whi], diagonal equal to
    the row's absolute off-diagonal sum plus ``shift`` (Gershgorin: lambda_min >= shift)."""
    e = ba_tree_edges(b, rng)
    theta = np.zeros((b, b))
    if e.size:
        w = rng.uniform(wlo, whi, size=len(e)) * rng.choice([-1.0, 1.0], size=len(e))
        theta[e[:, 0], e[:, 1]] = w
        theta[e[:, 1], e[:, 0]] = w
    theta[np.diag_indices(b)] = np.abs(theta).sum(axis=1) + shift
    return theta


# ---------------------------------------------------------------------------
# Gaussian samples
# ---------------------------------------------------------------------------

def sample_gaussian(theta: np.ndarray, n: int, rng: np.random.Generator) -> np.ndarray:
    """n rows i.i.d. N(0, theta^{-1}): theta = L L^T, x = L^{-T} z (float64, n x p)."""
    p = theta.shape[0]
    lower = np.linalg.cholesky(theta)
    z = rng.standard_normal((p, n))
    y = sla.solve_triangular(lower, z, trans="T", lower=True)
    return np.ascontiguousarray(y.T)


def standardise(x: np.ndarray) -> np.ndarray:
    """Centre each column, then divide it by the root of its mean square (1/n
    convention), so the sample covariance has unit diagonal."""
    x = x - x.mean(axis=0, keepdims=True)
    scale = np.sqrt((x * x).mean(axis=0, keepdims=True))
    scale[scale == 0] = 1.0
    return x / scale


def block_diag_sample(nblocks: int, b: int, n: int, wlo: float, whi: float, shift: float,
                      rng_theta: np.random.Generator, rng_data: np.random.Generator,
                      return_theta: bool = False):
    """Block-diagonal power-law Theta of ``nblocks`` blocks of size ``b``; samples are
    drawn blockwise (blocks are independent).  Returns X (n x nblocks*b, float64)."""
    cols = []
    thetas = []
    for _ in range(nblocks):
        th = ba_block_precision(b, wlo, whi, shift, rng_theta)
        cols.append(sample_gaussian(th, n, rng_data))
        if return_theta:
            thetas.append(th)
    x = np.concatenate(cols, axis=1)
    if return_theta:
        return x, thetas
    return x


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    p: int
    lam: float
    iters: int
    X: np.ndarray                 # float32, n x p, C-contiguous, standardised
    meta: dict = field(default_factory=dict)


def _f32(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float32)


def er_workload(n: int = 100, p: int = 200, prob: float = 0.02, lam: float = 0.1,
                iters: int = 200, key: int = 0) -> Workload:
    """Erdos-Renyi workload: edge prob ``prob``, weights +-U[0.2, 0.4],
    lambda_min(Theta) = 0.1, standardised columns (defaults: n=100, p=200)."""
    r_theta, r_data, _ = rngs(key)
    theta = er_precision(p, prob, 0.2, 0.4, 0.1, r_theta)
    x = standardise(sample_gaussian(theta, n, r_data))
    return Workload(f"er_n{n}_p{p}", n, p, lam, iters, _f32(x),
                    {"graph": "erdos-renyi", "edge_prob": prob, "theta": theta})


def ba_block_workload(n: int = 500, nblocks: int = 10, b: int = 500, lam: float = 0.05,
                      iters: int = 500, key: int = 1, keep_theta: bool = False) -> Workload:
    """Block-diagonal power-law workload: ``nblocks`` BA(m=1) blocks of ``b`` nodes,
    weights +-U[0.2, 0.5], diagonal = abs row sum + 0.1, standardised columns
    (defaults: n=500, p=5000)."""
    r_theta, r_data, _ = rngs(key)
    out = block_diag_sample(nblocks, b, n, 0.2, 0.5, 0.1, r_theta, r_data,
                            return_theta=keep_theta)
    x, thetas = (out if keep_theta else (out, None))
    meta = {"graph": "block-diagonal Barabasi-Albert(m=1)", "blocks": nblocks, "block": b}
    if keep_theta:
        meta["thetas"] = thetas
    return Workload(f"ba_n{n}_p{nblocks * b}", n, nblocks * b, lam, iters,
                    _f32(standardise(x)), meta)


def small_random_problem(n: int, p: int, seed: int, lam: float = 0.1) -> Workload:
    """Unstructured standardised Gaussian data for small-case tests."""
    _, r_data, _ = rngs(99, seed)
    x = standardise(r_data.standard_normal((n, p)))
    return Workload(f"rand_n{n}_p{p}_s{seed}", n, p, lam, 0, _f32(x), {})


def lambda_grid(lo: float = 0.02, hi: float = 0.5, count: int = 32) -> np.ndarray:
    """Log-spaced lambda grid."""
    return np.geomspace(lo, hi, count)


def bootstrap_rows(n_base: int, count: int, lo: int, hi: int, rng: np.random.Generator):
    """``count`` bootstrap subsamples: size U{lo..hi}, rows drawn with replacement."""
    sizes = rng.integers(lo, hi + 1, size=count)
    return [rng.integers(0, n_base, size=int(s)) for s in sizes]


@dataclass
class BatchWorkload:
    """Several data sets sharing p, and a lambda grid: problem k = b * len(lams) + l
    fits data set b at lams[l]."""
    name: str
    p: int
    xs: list            # float32 [n_b, p] per data set (centred, unit mean square)
    lams: np.ndarray    # float64 [nlam]
    iters: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return [x.shape[0] for x in self.xs]

    def stacked(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate(self.xs, axis=0), dtype=np.float32)


def batch_workload(p: int = 2000, nsub: int = 16, nlam: int = 32, n_base: int = 400,
                   lo: int = 100, hi: int = 400, prob: float = 0.005, lam_lo: float = 0.02,
                   lam_hi: float = 0.5, iters: int = 300, key: int = 3) -> BatchWorkload:
    """Bootstrap lambda-path workload: one Erdos-Renyi Theta (edge prob ``prob``,
    weights +-U[0.2, 0.4], lambda_min = 0.1), one base sample of ``n_base`` rows,
    ``nsub`` subsamples of U{lo..hi} rows drawn with replacement, each re-centred
    and re-standardised, and ``nlam`` log-spaced penalties in [lam_lo, lam_hi]."""
    r_theta, r_data, r_aux = rngs(key)
    theta = er_precision(p, prob, 0.2, 0.4, 0.1, r_theta)
    base = sample_gaussian(theta, n_base, r_data)
    rows = bootstrap_rows(n_base, nsub, lo, hi, r_aux)
    xs = [_f32(standardise(base[r])) for r in rows]
    return BatchWorkload(f"batch_p{p}_{nsub}x{nlam}", p, xs, lambda_grid(lam_lo, lam_hi, nlam),
                         iters, {"graph": "erdos-renyi", "edge_prob": prob, "n_base": n_base})


def diff_workload(n_train: int = 300, n_val: int = 150, nblocks: int = 6, b: int = 500,
                  lam: float = 0.05, iters: int = 50, every: int = 10, key: int = 4):
    """Held-out workload: one block power-law Theta (``nblocks`` BA(m=1) blocks of
    ``b``), n_train + n_val samples; training and validation rows are centred and
    scaled separately."""
    r_theta, r_data, _ = rngs(key)
    x = block_diag_sample(nblocks, b, n_train + n_val, 0.2, 0.5, 0.1, r_theta, r_data)
    return {"x_train": _f32(standardise(x[:n_train])), "x_val": _f32(standardise(x[n_train:])),
            "lam": lam, "iters": iters, "every": every, "p": nblocks * b}


def refit_workload(lam: float = 0.05, phi: float = 0.5, iters: int = 200, key: int = 1):
    """The n = 500, p = 5000 power-law data (the same X as the "ba5000" workload) with a
    synthetic first-stage estimate whose support is the true graph's: diagonal 1,
    off-diagonal entries on the edges +-U[0.01, 0.05] (column form, float32)."""
    w = ba_block_workload(500, 10, 500, lam, iters, key=key, keep_theta=True)
    _, _, r_aux = rngs(key)
    om = np.zeros((w.p, w.p), dtype=np.float32)
    for k, th in enumerate(w.meta["thetas"]):
        b = th.shape[0]
        blk = np.where(th != 0, r_aux.uniform(0.01, 0.05, (b, b)) * r_aux.choice([-1.0, 1.0], (b, b)),
                       0.0)
        np.fill_diagonal(blk, 1.0)
        om[k * b:(k + 1) * b, k * b:(k + 1) * b] = blk
    return {"x": w.X, "omega_hat": om, "lam": lam, "phi": phi, "iters": iters, "n": w.n,
            "p": w.p}


# the named workloads (sizes as used by tests and the benchmark)
def workload(name: str) -> Workload:
    if name == "er200":
        return er_workload(100, 200, 0.02, 0.1, 200, key=0)
    if name == "ba5000":
        return ba_block_workload(500, 10, 500, 0.05, 500, key=1)
    if name == "ba100k":
        return ba_block_workload(1000, 200, 500, 0.03, 300, key=2)
    if name == "batch":
        return batch_workload()
    raise KeyError(name)
