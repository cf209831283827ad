"""Pins for the oracle's quantile (general rank) and median absolute deviation."""
import itertools
import math
import struct

import numpy as np
import pytest

import oracle


def _tot_key(v):
    (u,) = struct.unpack("<I", struct.pack("<f", v))
    return -(u & 0x7FFFFFFF) - 1 if u >> 31 else u


def _bits(v):
    return struct.pack("<f", v)


@pytest.mark.parametrize("q", [0.0, 0.1, 0.25, 0.5, 0.75, 0.9, 0.999, 1.0])
def test_quantile_brute_force(q):
    rng = np.random.default_rng(int(q * 1000) + 1)
    for n in (1, 2, 3, 10, 257, 1000):
        x = (rng.standard_normal(n) * 3).astype(np.float32)
        x[rng.random(n) < 0.1] = np.nan
        valid = sorted((float(v) for v in x if not math.isnan(v)), key=_tot_key)
        got, cnt = oracle.quantile(x, q)
        if not valid:
            assert math.isnan(got) and cnt == 0
            continue
        k = math.floor(q * (len(valid) - 1))
        assert _bits(got) == _bits(valid[k])


def test_quantile_special_ranks():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(999).astype(np.float32)
    assert oracle.quantile(x, 0.0)[0] == float(x.min())
    assert oracle.quantile(x, 1.0)[0] == float(x.max())
    assert oracle.quantile(x, 0.5)[0] == oracle.median(x)[0]
    y = np.concatenate([x, [np.float32(1.5)]])  # even count: 0.5 is still the lower median
    assert oracle.quantile(y, 0.5)[0] == oracle.median(y)[0]
    with pytest.raises(ValueError):
        oracle.quantile(x, 1.5)


def test_quantile_rank_is_double_product():
    # floor(q (n-1)) with the product rounded to double precision
    assert oracle.quantile_rank(0.1, 11) == 1
    assert oracle.quantile_rank(0.3, 11) == 3
    assert oracle.quantile_rank(0.29, 101) == 28  # 0.29*100 = 28.999999999999996 in double
    assert oracle.quantile_rank(0.57, 101) == 56  # 56.99999999999999
    assert oracle.quantile_rank(1.0, 5) == 4 and oracle.quantile_rank(0.0, 5) == 0


def test_mad_closed_forms():
    # symmetric 1..5: median 3, deviations 2,1,0,1,2 -> MAD 1
    assert oracle.mad(np.float32([1, 2, 3, 4, 5]))[1] == 1.0
    # ramp 0..n-1 (n odd = 2r+1): median r, deviations 0,1,1,2,2,..,r,r -> MAD ceil(r/2)... brute check below
    for n in (1, 2, 3, 4, 7, 10, 101):
        x = np.arange(n, dtype=np.float32)
        m = (n - 1) // 2
        dev = sorted(abs(v - m) for v in range(n))
        assert oracle.mad(x)[:2] == (float(m), float(dev[(n - 1) // 2]))
    # constant data: MAD 0
    assert oracle.mad(np.full(17, 2.5, np.float32))[1] == 0.0


def test_mad_brute_force_single_precision():
    rng = np.random.default_rng(8)
    for _ in range(50):
        n = int(rng.integers(1, 200))
        x = (rng.standard_normal(n) * 10 + 3).astype(np.float32)
        x[rng.random(n) < 0.05] = np.nan
        valid = sorted((float(v) for v in x if not math.isnan(v)), key=_tot_key)
        med, mad, cnt = oracle.mad(x)
        if not valid:
            assert cnt == 0 and math.isnan(mad)
            continue
        m = valid[(len(valid) - 1) // 2]
        devs = sorted(abs(float(np.float32(np.float32(v) - np.float32(m)))) for v in valid)
        assert med == m and mad == devs[(len(devs) - 1) // 2]


def test_mad_int16_exact():
    x = np.int16([-32768, 32767, 0, 5, -5, 100])
    med, mad, n = oracle.mad(x)
    # sorted: -32768 -5 0 5 100 32767 -> lower median 0; |x-0|: 32768 32767 0 5 5 100 -> sorted 0 5 5 100 32767 32768
    assert (med, mad, n) == (0.0, 5.0, 6)


def test_mad_exhaustive_small():
    pool = [np.float32(v) for v in (-2.0, -0.5, 0.0, 1.0, 3.0)]
    for n in range(1, 5):
        for combo in itertools.product(range(len(pool)), repeat=n):
            x = np.array([pool[i] for i in combo], dtype=np.float32)
            s = sorted(float(v) for v in x)
            m = s[(n - 1) // 2]
            d = sorted(abs(v - m) for v in s)  # exact here: values on a 2^-1 grid
            assert oracle.mad(x)[1] == d[(n - 1) // 2]


def test_mad_infinite_median():
    """A value equal to the median deviates by zero, also when the median is
    infinite (the IEEE difference inf - inf would be NaN); the rank is taken
    over all valid values."""
    # sorted 1, inf, inf, inf: lower median (rank 1) = inf; deviations inf, 0, 0, 0 -> rank 1 = 0
    assert oracle.mad(np.float32([np.inf, np.inf, np.inf, 1]))[:3] == (math.inf, 0.0, 4)
    # sorted -inf, -inf, 0: median -inf; deviations 0, 0, inf -> 0
    assert oracle.mad(np.float32([-np.inf, -np.inf, 0]))[:3] == (-math.inf, 0.0, 3)
    # median inf with a minority at inf: deviations inf (finite values) and 0 (the infinities)
    m, mad, n = oracle.mad(np.float32([1, 2, np.inf, np.inf, np.inf, np.nan]))
    assert (m, mad, n) == (math.inf, 0.0, 5)
    # median finite, infinities present: their deviation is inf
    m, mad, n = oracle.mad(np.float32([1, 2, 3, np.inf, -np.inf]))
    assert (m, mad, n) == (2.0, 1.0, 5)  # deviations 1, 0, 1, inf, inf -> sorted 0 1 1 inf inf -> rank 2 = 1
    m, mad, n = oracle.mad(np.float32([1, np.inf, np.inf, -np.inf, -np.inf]))
    assert (m, mad, n) == (1.0, math.inf, 5)


def test_mad_brute_force_with_infinities():
    """Brute force by the definition on multisets drawn from values that
    include both infinities and signed zeros."""
    pool = np.float32([-np.inf, -1.0, -0.0, 0.0, 2.0, np.inf])
    for n in range(1, 6):
        for combo in itertools.product(range(len(pool)), repeat=n):
            x = pool[list(combo)]
            s = sorted((float(v) for v in x), key=_tot_key)
            m = s[(n - 1) // 2]
            d = sorted(0.0 if v == m else abs(v - m) for v in s)
            assert oracle.mad(x)[:2] == (m, d[(n - 1) // 2]), x
