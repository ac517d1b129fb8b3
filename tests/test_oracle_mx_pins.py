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


def _mx_loops(v, blocks_along_rows):
    """MX rounding written out block by block: for every column (blocks_along_rows) or
    every row, each run of 32 consecutive entries gets the scale 2^s of its own
    maximum and its entries are rounded to E4M3 times that scale."""
    v = np.asarray(v, dtype=np.float64)
    out = np.empty_like(v)
    rows, cols = v.shape
    if blocks_along_rows:
        for j in range(cols):
            for b0 in range(0, rows, 32):
                blk = v[b0:b0 + 32, j]
                s = 2.0 ** mx.mx_scale_exp(np.max(np.abs(blk)))
                out[b0:b0 + 32, j] = mx.e4m3_round(blk / s) * s
    else:
        for i in range(rows):
            for b0 in range(0, cols, 32):
                blk = v[i, b0:b0 + 32]
                s = 2.0 ** mx.mx_scale_exp(np.max(np.abs(blk)))
                out[i, b0:b0 + 32] = mx.e4m3_round(blk / s) * s
    return out


def _one_mx_step_by_hand(x, lam, tau, cols):
    """One MX step from the identity, with every operand blocked along the index its
    product sums over: X^T W sums over samples (X per feature, W per column, runs of
    32 samples); X Delta sums over features (X per sample row, Delta per column, runs
    of 32 features)."""
    n, p = x.shape
    om = np.zeros((p, len(cols)))
    om[cols, np.arange(len(cols))] = 1.0
    w = x @ om
    g = _mx_loops(x, True).T @ _mx_loops(w, True) / n
    a = om - tau * g
    new = np.sign(a) * np.maximum(np.abs(a) - tau * lam, 0.0)
    jj = np.arange(len(cols))
    b = a[cols, jj] - tau * lam
    new[cols, jj] = (b + np.sqrt(b * b + 4 * tau)) / 2
    w_new = w + _mx_loops(x, False) @ _mx_loops(new - om, True)
    return new, w_new


def _axis_probe_data():
    """64 samples x 96 features with a few outliers 2^12 - 2^14 times the other
    entries.  E4M3 keeps 3 mantissa bits in every normal binade, so a block's scale
    matters only for entries that fall below the normal range relative to the block
    maximum: here the ordinary entries of an outlier's 32-run become subnormal or zero,
    and that run is a different set of entries along the row than along the column."""
    rng = np.random.default_rng(11)
    x = rng.normal(size=(64, 96))
    x[3, 40] = 3.0e4
    x[50, 5] = -1.2e4
    x[20, 70] = 6.0e4
    return x


def test_fit_fbs_mx_x_blocks_follow_each_contraction():
    """X enters X^T W blocked along the samples and X Delta blocked along the
    features; the oracle's one MX step equals the step written out block by block."""
    x = _axis_probe_data()
    cols = np.array([5, 33, 40, 70, 90])
    lam, tau = 0.05, 0.02
    want_om, want_w = _one_mx_step_by_hand(x, lam, tau, cols)
    got = mx.fit_fbs_mx(x, lam, [tau], columns=cols)
    assert np.max(np.abs(got.omega - want_om)) <= 1e-13 * np.max(np.abs(want_om))
    assert np.max(np.abs(got.extra["w"] - want_w)) <= 1e-13 * np.max(np.abs(want_w))


@pytest.mark.parametrize("which", ["grad", "trial", "both"])
def test_mutation_swapped_x_axis_breaks_the_block_pin(which):
    """Planting the wrong blocking axis for X (in the gradient's X^T, the trial's X, or
    both) changes the step away from the block-by-block computation."""
    x = _axis_probe_data()
    n, p = x.shape
    cols = np.array([5, 33, 40, 70, 90])
    lam, tau = 0.05, 0.02
    want_om, want_w = _one_mx_step_by_hand(x, lam, tau, cols)

    def swapped(v, axis):
        v = np.asarray(v)
        if v.shape == (n, p) and (which == "both" or (which == "grad") == (axis == 0)):
            axis = 1 - axis
        return mx.mx_quantize(v, axis)

    got = mx.fit_fbs_mx(x, lam, [tau], columns=cols, quant=swapped)
    bad_om = np.max(np.abs(got.omega - want_om)) > 1e-6 * np.max(np.abs(want_om))
    bad_w = np.max(np.abs(got.extra["w"] - want_w)) > 1e-6 * np.max(np.abs(want_w))
    if which == "trial":
        assert bad_w           # the trial's X only enters W
    else:
        assert bad_om and bad_w
