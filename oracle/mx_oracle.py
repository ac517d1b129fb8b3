"""FP64 oracle of the FP8 (MX) precision form of ACCORD-FBS.

TEST INFRASTRUCTURE ONLY (same rules as ``accord_oracle``): imported by tests,
never by the GPU path, and it imports nothing from the GPU package.

The paper fixes no arithmetic precision.  The FP8 form is this project's reading
of a low-precision variant of the two contractions of Alg. 1: every operand of
G = X^T W / n and of V = X Delta is rounded to the OCP Microscaling (MX) format
before the product, and the products themselves are exact (FP64 here, FP32
accumulation on the device).  Everything else -- the prox of eq. 3.5, the
acceptance test, the objective -- is the same as in ``accord_oracle``.

MX format used (OCP Microscaling v1.0, element type E4M3):
  * a block is 32 consecutive values along the CONTRACTION index of a product;
  * the block shares one power-of-two scale 2^s (an E8M0 byte, s + 127);
  * each element is the E4M3 value nearest to x / 2^s, ties to even
    (1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits; subnormals down
    to 2^-9; largest finite value 448; no infinities);
  * scale rule: s = floor(log2(max |x| over the block)) - 7, so the block maximum
    lands in [128, 256) and never needs clamping (the spec's example rule uses
    -8 and clamps at 448; this choice trades one binade at the bottom of the
    range for no clamping error at the top).  s is kept >= -126; an all-zero
    block has s = 0.

Blocks along each contraction (the index summed over):
  trial  V = X Delta        X: rows of X, blocks of 32 features;  Delta: each column,
                            blocks of 32 rows
  grad   G = X^T W / n      X^T: each feature (column of X), blocks of 32 samples;
                            W: each column, blocks of 32 samples

The device keeps W = X Omega in FP32 and updates it with the accepted trial
(W+ = W + V), so W is the running sum of quantised products, not a fresh X Omega;
``fit_fbs_mx`` follows the same recurrence.  Padding to whole blocks is with zeros.

Functions:
  e4m3_value      decode one E4M3 code (definition of the format)
  e4m3_round      nearest E4M3 value, ties to even
  mx_scale_exp    the block scale exponent s
  mx_quantize     round a matrix to MX blocks along one axis (returns the values)
  fit_fbs_mx      Alg. 1 with MX-rounded contraction operands, replaying a given
                  step-size sequence (optionally on a subset of columns)
Pins: tests/test_oracle_mx_pins.py (exhaustive code enumeration, nearest-value brute
force, block locality and scale invariants, and reduction to ``fit_fbs`` when the
rounding is the identity).
"""
from __future__ import annotations

import numpy as np

from .accord_oracle import FitResult, diag_root, identity_columns, soft_threshold

E4M3_MAX = 448.0
MX_BLOCK = 32


def e4m3_value(code: int) -> float:
    """Value of one E4M3 (OCP 'fn' variant) byte; NaN for the two NaN codes."""
    code = int(code) & 0xFF
    sign = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return sign * (m / 8.0) * 2.0 ** -6
    return sign * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def e4m3_round(v) -> np.ndarray:
    """Nearest E4M3 value to each entry of v (|v| <= 448 expected), ties to even."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    # binade exponent; values below 2^-6 share the subnormal spacing 2^-9
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)
    ulp = 2.0 ** (e - 3.0)
    q = np.round(a / ulp) * ulp  # numpy rounds halves to even: even mantissa wins
    q = np.minimum(q, E4M3_MAX)
    return np.copysign(q, v)


def mx_scale_exp(amax) -> np.ndarray:
    """Scale exponent s of blocks with maximum magnitude amax."""
    amax = np.asarray(amax, dtype=np.float64)
    s = np.floor(np.log2(np.where(amax > 0, amax, 1.0))) - 7.0
    s = np.maximum(s, -126.0)
    return np.where(amax > 0, s, 0.0)


def mx_quantize(v, axis: int) -> np.ndarray:
    """Round v to MX-E4M3 with blocks of 32 consecutive entries along `axis`
    (block k covers indices 32k .. 32k+31, counted from index 0)."""
    v = np.asarray(v, dtype=np.float64)
    moved = np.moveaxis(v, axis, 0)
    k = moved.shape[0]
    kb = -(-k // MX_BLOCK) * MX_BLOCK
    pad = np.zeros((kb,) + moved.shape[1:])
    pad[:k] = moved
    blocks = pad.reshape((kb // MX_BLOCK, MX_BLOCK) + moved.shape[1:])
    amax = np.max(np.abs(blocks), axis=1, keepdims=True)
    scale = 2.0 ** mx_scale_exp(amax)
    q = e4m3_round(blocks / scale) * scale
    out = q.reshape(pad.shape)[:k]
    return np.moveaxis(out, 0, axis)


def _identity(v, axis):
    return np.asarray(v, dtype=np.float64)


def fit_fbs_mx(x, lam, tau_replay, omega0=None, columns=None, quant=mx_quantize):
    """ACCORD-FBS (Alg. 1) with the contraction operands rounded by `quant`, on the
    step sizes ``tau_replay`` (one accepted trial per iteration, as in
    ``fit_fbs(..., tau_replay=...)``).

    Per iteration t:
        G   = q(X^T) q(W) / n          (blocks along the samples)
        Om+ = prox(Om - tau_t G)        eq. 3.5
        D   = Om+ - Om
        W   = W + q(X) q(D)             (blocks along the features)
    with W starting at X Om0 (exact).  ``columns`` restricts Om to those columns
    (the diagonal entry of column j is row j); with the steps fixed the columns
    evolve independently, so this reproduces those columns of the full run.
    quant(v, axis) must return v's rounded values; the identity gives plain FBS.
    """
    x = np.asarray(x, dtype=np.float64)
    n, p = x.shape
    if columns is not None:
        cols = np.asarray(columns)
        om = identity_columns(p, cols) if omega0 is None else np.asarray(omega0, np.float64)[:, cols].copy()
        diag_rows = cols
    else:
        om = np.eye(p) if omega0 is None else np.asarray(omega0, np.float64).copy()
        diag_rows = np.arange(p)
    jj = np.arange(om.shape[1])
    xq_trial = quant(x, 1)   # rows of X: blocks of 32 features (contraction of X D)
    xq_grad = quant(x, 0)    # columns of X: blocks of 32 samples (contraction of X^T W)
    w = x @ om
    res = FitResult(omega=om, iters=0, lipschitz=float("nan"))
    dq_fro = []
    for t in range(len(tau_replay)):
        tau = float(tau_replay[t])
        g = xq_grad.T @ quant(w, 0) / n
        a = om - tau * g
        om_new = soft_threshold(a, tau * lam)
        om_new[diag_rows, jj] = diag_root(a[diag_rows, jj], tau, lam)
        d = om_new - om
        dq = quant(d, 0)
        w = w + xq_trial @ dq
        om = om_new
        res.tau.append(tau)
        res.trials.append(1)
        res.delta_fro.append(float(np.linalg.norm(d)))
        dq_fro.append(float(np.linalg.norm(dq)))
        res.iters = t + 1
    res.omega = om
    # w: the running W; delta_q_fro: ||q(Delta)||_F per iteration (the step the
    # product and the acceptance sums see)
    res.extra = {"w": w, "delta_q_fro": dq_fro}
    return res


__all__ = ["E4M3_MAX", "MX_BLOCK", "e4m3_value", "e4m3_round", "mx_scale_exp",
           "mx_quantize", "fit_fbs_mx"]
