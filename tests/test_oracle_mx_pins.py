"""Pins of the MX-FP8 oracle (oracle/mx_oracle.py) against the format's definition
and against the plain FBS oracle; CPU only."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import mx_oracle as mx


def _codes():
    vals = np.array([mx.e4m3_value(c) for c in range(256)])
    return vals


def test_e4m3_code_table():
    v = _codes()
    nan = np.isnan(v)
    assert list(np.flatnonzero(nan)) == [0x7F, 0xFF]
    fin = v[~nan]
    assert fin.max() == 448.0 and fin.min() == -448.0
    pos = np.unique(fin[fin > 0])
    assert pos[0] == 2.0 ** -9 and len(pos) == 126     # 7 subnormals + 15 binades x 8 - 1
    assert np.all(v[:0x80][~nan[:0x80]] == -v[0x80:][~nan[0x80:]])
    assert mx.e4m3_value(0x38) == 1.0 and mx.e4m3_value(0x7E) == 448.0


def test_e4m3_round_is_nearest_ties_even():
    v = _codes()
    finite = sorted(set(v[~np.isnan(v)].tolist()))
    codes = {val: c for c, val in enumerate(v) if not np.isnan(val) and not (val == 0 and c)}
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-448, 448, 4000), rng.normal(0, 0.05, 2000),
                         rng.normal(0, 1e-3, 500)])
    got = mx.e4m3_round(xs)
    grid = np.array(finite)
    for x, g in zip(xs, got):
        d = np.abs(grid - x)
        assert abs(g - x) == d.min(), (x, g)
    # exact midpoints between neighbours go to the code with even mantissa
    mids = (grid[1:] + grid[:-1]) / 2
    for m, g in zip(mids, mx.e4m3_round(mids)):
        assert codes[float(g)] & 1 == 0, (m, g)


def test_mx_scale_puts_block_max_in_128_256():
    rng = np.random.default_rng(1)
    a = np.exp(rng.uniform(-60, 60, 1000))
    s = mx.mx_scale_exp(a)
    r = a / 2.0 ** s
    assert np.all((r >= 128) & (r < 256))
    assert mx.mx_scale_exp(0.0) == 0.0
    assert mx.mx_scale_exp(1e-45) == -126.0


def test_mx_quantize_error_and_grid():
    rng = np.random.default_rng(2)
    v = rng.normal(size=(96, 7)) * np.exp(rng.uniform(-8, 8, size=(96, 7)))
    q = mx.mx_quantize(v, axis=0)
    for b in range(3):
        blk, qb = v[32 * b:32 * b + 32], q[32 * b:32 * b + 32]
        for j in range(7):
            s = 2.0 ** mx.mx_scale_exp(np.abs(blk[:, j]).max())
            # every value is an E4M3 value times the block scale
            assert np.all(mx.e4m3_round(qb[:, j] / s) == qb[:, j] / s)
            normal = np.abs(blk[:, j]) / s >= 2.0 ** -6
            rel = np.abs(qb[:, j] - blk[:, j]) / np.abs(blk[:, j])
            assert np.all(rel[normal] <= 2.0 ** -4)
            assert np.all(np.abs(qb[:, j] - blk[:, j])[~normal] <= 2.0 ** -10 * s)


def test_mx_quantize_blocks_follow_the_axis():
    rng = np.random.default_rng(3)
    v = rng.normal(size=(70, 40))
    base0, base1 = mx.mx_quantize(v, 0), mx.mx_quantize(v, 1)
    v2 = v.copy()
    v2[37, 5] *= 1000.0
    d0 = mx.mx_quantize(v2, 0) != base0
    d1 = mx.mx_quantize(v2, 1) != base1
    rows, cols = np.nonzero(d0)
    assert set(cols) == {5} and rows.min() >= 32 and rows.max() < 64 and len(rows) > 1
    rows, cols = np.nonzero(d1)
    assert set(rows) == {37} and cols.min() >= 0 and cols.max() < 32 and len(cols) > 1
    # a ragged last block is padded with zeros: its scale follows its own entries
    tail = np.zeros((70, 1))
    tail[64:, 0] = 3.0
    assert np.all(mx.mx_quantize(tail, 0)[64:, 0] == 3.0)


def test_mx_quantize_fixes_representable_blocks():
    rng = np.random.default_rng(4)
    v = np.array([mx.e4m3_value(c) for c in rng.integers(0, 0x78, size=64)])  # |v| <= 240
    v *= rng.choice([-1.0, 1.0], size=64)
    v[0], v[32] = 192.0, -240.0          # block maxima in [128, 256): scale 1
    v = v * 2.0 ** 5
    assert np.all(mx.mx_quantize(v.reshape(64, 1), 0)[:, 0] == v)


def test_fit_fbs_mx_identity_rounding_is_fbs():
    x = datagen.small_random_problem(40, 24, seed=5).X
    lam = 0.15
    ref = oracle.fit_fbs(x, lam, 12)
    got = mx.fit_fbs_mx(x, lam, ref.tau, quant=mx._identity)
    assert np.max(np.abs(got.omega - ref.omega)) < 1e-12
    # W is the running sum of the accepted products: equals X Omega exactly here
    assert np.max(np.abs(got.extra["w"] - x.astype(np.float64) @ ref.omega)) < 1e-10


def test_fit_fbs_mx_column_subset_replay():
    x = datagen.small_random_problem(50, 70, seed=6).X
    lam = 0.1
    taus = oracle.fit_fbs(x, lam, 8).tau
    full = mx.fit_fbs_mx(x, lam, taus)
    cols = np.array([0, 3, 33, 69])
    sub = mx.fit_fbs_mx(x, lam, taus, columns=cols)
    assert np.max(np.abs(sub.omega - full.omega[:, cols])) < 1e-13
    # MX rounding moves the iterate, by about the E4M3 resolution
    plain = oracle.fit_fbs(x, lam, 8, tau_replay=taus)
    rel = np.linalg.norm(full.omega - plain.omega) / np.linalg.norm(plain.omega)
    assert 1e-5 < rel < 0.1
