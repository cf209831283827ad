"""Pins for the oracle's moments (Section 4.2) against closed forms and exact rationals."""
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _frac_moments(vals):
    fs = [Fraction(float(v)) for v in vals]
    n = len(fs)
    mean = sum(fs) / n
    m2 = sum((f - mean) ** 2 for f in fs)
    return n, mean, m2


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("c", [0.0, 1.0, -3.25, 1e-30, 3.0e38, 7.0])
@pytest.mark.parametrize("n", [1, 2, 17, 1000])
def test_constant(c, n):
    a = np.full(n, c, dtype=np.float32)
    m = oracle.moments(a)
    assert m["count"] == n and m["nan_count"] == 0
    assert m["mean"] == float(np.float32(c))
    assert m["m2"] == 0.0 and m["std"] == 0.0
    assert m["min"] == m["max"] == float(np.float32(c))


@pytest.mark.parametrize("a0,d,n", [(0.0, 1.0, 1001), (-5.5, 0.25, 4096), (1024.0, -0.125, 777), (3.0, 2.0, 2)])
def test_arithmetic_ramp_closed_form(a0, d, n):
    # exactly representable ramp a0 + i*d: mean = a0 + d(n-1)/2, var = d^2 (n^2-1)/12
    x = (a0 + d * np.arange(n, dtype=np.float64)).astype(np.float32)
    assert np.all(x.astype(np.float64) == a0 + d * np.arange(n))
    m = oracle.moments(x)
    mean = a0 + d * (n - 1) / 2
    var = d * d * (n * n - 1) / 12
    assert m["count"] == n
    assert _rel(m["mean"], mean) <= 1e-15 or abs(m["mean"] - mean) <= 1e-15 * abs(d) * n
    assert _rel(m["m2"] / n, var) <= 1e-14
    assert _rel(m["std"], math.sqrt(var)) <= 1e-14
    assert m["min"] == min(x[0], x[-1]) and m["max"] == max(x[0], x[-1])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_rational(seed):
    rng = np.random.default_rng(seed)
    n = 20000
    x = (rng.standard_normal(n) * 3 + 0.7).astype(np.float32)
    x[rng.integers(0, n, 50)] = np.nan
    x[:5] = np.float32(500.0)  # a bright "source"
    valid = x[~np.isnan(x)]
    cnt, mean, m2 = _frac_moments(valid)
    m = oracle.moments(x)
    assert m["count"] == cnt and m["nan_count"] == n - cnt
    assert _rel(m["mean"], float(mean)) <= 1e-15
    assert _rel(m["m2"], float(m2)) <= 1e-14
    assert _rel(m["std"], math.sqrt(float(m2) / cnt)) <= 1e-14


def test_large_mean_small_spread():
    # cancellation case: mean/std ~ 1e4; the exact rational answer still holds
    rng = np.random.default_rng(5)
    x = (1.0e4 + rng.standard_normal(5000)).astype(np.float32)
    cnt, mean, m2 = _frac_moments(x)
    m = oracle.moments(x)
    assert _rel(m["mean"], float(mean)) <= 1e-15
    assert _rel(m["m2"], float(m2)) <= 1e-10


def test_all_nan_and_empty_count():
    a = np.full(64, np.nan, dtype=np.float32)
    m = oracle.moments(a)
    assert m["count"] == 0 and m["nan_count"] == 64
    for k in ("mean", "m2", "std", "min", "max"):
        assert math.isnan(m[k])


def _tot_key(v):
    # IEEE-754 totalOrder for float32 via the sign-magnitude integer
    (u,) = struct.unpack("<I", struct.pack("<f", v))
    return -(u & 0x7FFFFFFF) - 1 if u >> 31 else u


def test_min_max_total_order_brute_force():
    rng = np.random.default_rng(3)
    pool = np.array([0.0, -0.0, 1e-45, -1e-45, -1.0, 1.0, np.inf, -np.inf, 2.5, np.nan], dtype=np.float32)
    for _ in range(400):
        x = pool[rng.integers(0, len(pool), rng.integers(1, 9))]
        valid = [float(v) for v in x if not np.isnan(v)]
        m = oracle.moments(x)
        if not valid:
            assert m["count"] == 0
            continue
        mn = min(valid, key=_tot_key)
        mx = max(valid, key=_tot_key)
        assert struct.pack("<d", m["min"]) == struct.pack("<d", mn)
        assert struct.pack("<d", m["max"]) == struct.pack("<d", mx)


def test_signed_zero_min_max():
    m = oracle.moments(np.array([0.0, -0.0, 0.0], dtype=np.float32))
    assert math.copysign(1.0, m["min"]) == -1.0 and math.copysign(1.0, m["max"]) == 1.0


def test_region_equals_extracted_subcube():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((9, 11, 13)).astype(np.float32)
    a[2, 3, 4] = np.nan
    reg = (2, 1, 1, 12, 7, 8)  # x0,y0,z0,x1,y1,z1
    sub = np.ascontiguousarray(a[1:8, 1:7, 2:12])
    m1 = oracle.moments(a, reg)
    m2 = oracle.moments(sub)
    assert m1 == m2


@pytest.mark.parametrize("reg", [(0, 0, 0, 0, 1, 1), (0, 0, 0, 14, 1, 1), (-1, 0, 0, 2, 2, 2), (3, 0, 0, 2, 1, 1)])
def test_region_rejected(reg):
    a = np.zeros((4, 5, 13), dtype=np.float32)
    with pytest.raises(ValueError):
        oracle.moments(a, reg)


def test_int16():
    rng = np.random.default_rng(9)
    x = rng.integers(-32768, 32768, 30000).astype(np.int16)
    cnt, mean, m2 = _frac_moments(x)
    m = oracle.moments(x)
    assert m["count"] == cnt and m["nan_count"] == 0
    assert _rel(m["mean"], float(mean)) <= 1e-15
    assert _rel(m["m2"], float(m2)) <= 1e-14
    assert m["min"] == int(x.min()) and m["max"] == int(x.max())


def test_mistakes_are_caught():
    # a plausible mistake (sample instead of population spread, or M2 without
    # the mean term) would break the closed form of a ramp
    x = np.arange(10, dtype=np.float32)
    m = oracle.moments(x)
    assert m["std"] == pytest.approx(math.sqrt(99 / 12), rel=1e-15)
    assert m["std"] != pytest.approx(math.sqrt(99 / 12 * 10 / 9), rel=1e-6)
    assert m["m2"] == pytest.approx(82.5, rel=1e-15)


def test_moments_with_infinities():
    """The sum of values holding +inf is +inf (-inf: -inf, both: undefined), so
    the mean is +inf, -inf or NaN and the spread undefined; a set holding one
    value only has that value as its mean and no spread."""
    def mo(v):
        return oracle.moments(np.array(v, dtype=np.float32))
    r = mo([1.0, 2.0, np.inf, np.nan])
    assert r["mean"] == math.inf and math.isnan(r["std"]) and math.isnan(r["m2"]) and r["count"] == 3
    r = mo([-np.inf, 1.0, -np.inf])
    assert r["mean"] == -math.inf and math.isnan(r["std"])
    r = mo([np.inf, -np.inf, 3.0])
    assert math.isnan(r["mean"]) and math.isnan(r["std"])
    r = mo([np.inf, np.inf, np.nan])
    assert r["mean"] == math.inf and r["std"] == 0.0 and r["m2"] == 0.0 and r["count"] == 2
    r = mo([-0.0, 0.0])  # two values under totalOrder, no spread either way
    assert r["mean"] == 0.0 and r["std"] == 0.0 and r["min"] == 0.0 and math.copysign(1, r["min"]) < 0
    r = mo([0.1] * 7)
    assert r["mean"] == float(np.float32(0.1)) and r["std"] == 0.0
