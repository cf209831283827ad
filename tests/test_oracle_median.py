"""Pins for the oracle's lower median (Section 4.3) and Torben's method (Appendix A)."""
import itertools
import math
import os
import struct

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_torben_trace.txt")


def _tot_key(v):
    (u,) = struct.unpack("<I", struct.pack("<f", v))
    return -(u & 0x7FFFFFFF) - 1 if u >> 31 else u


def _bits(v):
    return struct.pack("<f", v)


def _brute(vals):
    valid = [float(v) for v in vals if not math.isnan(v)]
    if not valid:
        return None
    s = sorted(valid, key=_tot_key)
    return s[(len(s) - 1) // 2]


def test_exhaustive_small_multisets():
    pool = [np.float32(v) for v in (-1.0, -0.0, 0.0, 1.0, 2.0, np.nan)]
    for n in range(1, 6):
        for combo in itertools.product(range(len(pool)), repeat=n):
            x = np.array([pool[i] for i in combo], dtype=np.float32)
            want = _brute(x)
            got, cnt = oracle.median(x)
            got2, cnt2 = oracle.median_sort(x)
            if want is None:
                assert math.isnan(got) and math.isnan(got2) and cnt == cnt2 == 0
            else:
                assert _bits(got) == _bits(want) and _bits(got2) == _bits(want), (x, got, got2, want)


@pytest.mark.parametrize("seed", range(6))
def test_random_vs_brute(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3000))
    x = rng.choice(np.float32([-2.5, -1.0, 0.0, 0.5, 1e-40, np.inf, -np.inf, 7.0]), n)
    x = np.where(rng.random(n) < 0.5, rng.standard_normal(n).astype(np.float32), x).astype(np.float32)
    x[rng.random(n) < 0.05] = np.nan
    want = _brute(x)
    got, _ = oracle.median(x)
    if want is None:
        assert math.isnan(got)
    else:
        assert _bits(got) == _bits(want)


def test_odd_n_equals_numpy_median():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(10001).astype(np.float32)
    assert oracle.median(x)[0] == float(np.median(x))


def test_even_n_is_lower_median():
    x = np.float32([4.0, 1.0, 3.0, 2.0])
    assert oracle.median(x)[0] == 2.0  # not 2.5, not 3
    assert oracle.median(np.float32([5.0]))[0] == 5.0


def test_region_and_int16():
    rng = np.random.default_rng(12)
    a = rng.integers(-3000, 3000, (8, 9, 10)).astype(np.int16)
    reg = (1, 0, 2, 9, 7, 6)
    m, n = oracle.median(a, reg)
    sub = a[2:6, 0:7, 1:9].reshape(-1)
    assert n == sub.size and m == float(np.sort(sub)[(sub.size - 1) // 2])
    assert oracle.median_sort(a, reg) == (m, n)


# ---- Torben's method ------------------------------------------------------

def _table1():
    rows = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            it, g, mn, mx, lt, gt, eq = line.split()
            rows.append((int(it), g, mn, mx, int(lt), int(gt), int(eq)))
    return rows


def test_table1_guess_is_single_precision_midpoint():
    for it, g, mn, mx, *_ in _table1():
        got = oracle.torben_guess(float(np.float32(mn)), float(np.float32(mx)))
        assert "%.10f" % got == g, (it, got, g)


def test_table1_rows_consistent_with_algorithm():
    n = 534397200
    half = (n + 1) // 2
    rows = _table1()
    for it, g, mn, mx, lt, gt, eq in rows:
        assert lt + gt + eq == n
    # rows 1..5 are consecutive: the bracket moves as Algorithm 1 says
    by_it = {r[0]: r for r in rows}
    for i in range(1, 5):
        _, g, mn, mx, lt, gt, eq = by_it[i]
        _, g2, mn2, mx2, *_ = by_it[i + 1]
        if lt > gt:
            assert mn2 == mn and float(mx2) < float(g)
        else:
            assert mx2 == mx and float(mn2) > float(g)
    # the last row stops: both counts within the (integer) half, and less+equal reaches it
    _, g, mn, mx, lt, gt, eq = by_it[31]
    assert lt <= half and gt <= half and lt < half <= lt + eq


def _canon(v):
    return 0.0 if v == 0 else v


@pytest.mark.parametrize("seed", range(8))
def test_torben_equals_lower_median(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 4000))
    if seed % 2:
        x = rng.integers(-5, 6, n).astype(np.float32)  # heavy ties
    else:
        x = (rng.standard_normal(n) * 10).astype(np.float32)
    x[rng.random(n) < 0.03] = np.nan
    med, it, _ = oracle.torben(x)
    want, cnt = oracle.median(x)
    if cnt == 0:
        assert math.isnan(med)
    else:
        assert _canon(med) == _canon(want)
        assert it >= 1


def test_torben_real_division_would_be_upper_median():
    # With (n+1)/2 read as integer division the method returns the lower
    # median; the brute-force answer for even n confirms it.
    x = np.float32([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    med, it, trace = oracle.torben(x, trace_cap=64)
    assert med == 3.0
    assert trace.shape[0] == it


def test_torben_trace_shape_follows_table_columns():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(5001).astype(np.float32)
    med, it, tr = oracle.torben(x, trace_cap=100)
    assert tr.shape == (it, 6)
    n = x.size
    assert np.all(tr[:, 3] + tr[:, 4] + tr[:, 5] == n)
    # the first guess is the single-precision midpoint of the data extremes
    assert tr[0, 0] == oracle.torben_guess(float(x.min()), float(x.max()))
    assert med == oracle.median(x)[0]
