"""Pins for the oracle's histogram (Section 4.1) and its single-precision bin formula."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hist_small.txt")


def _bin_of(v, lo, hi, nbins):
    c, o = oracle.histogram(np.array([v], dtype=np.float32), lo, hi, nbins)
    if o[0]:
        return -1
    if o[1]:
        return nbins
    nz = np.nonzero(c)[0]
    return int(nz[0]) if nz.size else None


def test_golden_small():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    for v, b in rows:
        got = _bin_of(np.float32(float(v)), 0.0, 1.0, 10)
        if b == "skip":
            assert got is None
        else:
            assert got == int(b), (v, got, b)


@pytest.mark.parametrize("nbins", [1, 7, 256, 1024, 4096, 65536])
def test_integer_data_reduces_to_bincount(nbins):
    # lo = 0, hi = nbins: scale = 1 and the bin is the value itself; hi itself
    # falls into the last bin
    rng = np.random.default_rng(nbins)
    x = rng.integers(0, nbins, 50000).astype(np.float32)
    x = np.concatenate([x, np.float32([nbins, -1, nbins + 1, np.nan])])
    c, o = oracle.histogram(x, 0.0, float(nbins), nbins)
    ref = np.bincount(x[:50000].astype(np.int64), minlength=nbins).astype(np.uint64)
    ref[nbins - 1] += 1  # the value hi
    assert np.array_equal(c, ref)
    assert list(o) == [1, 1]


def test_totals_equal_non_nan_count():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(100000) * 4).astype(np.float32)
    x[::97] = np.nan
    x[::1013] = np.inf
    x[::1019] = -np.inf
    c, o = oracle.histogram(x, -3.0, 5.0, 333)
    n = np.count_nonzero(~np.isnan(x))
    assert int(c.sum()) + int(o.sum()) == n
    assert o[0] == np.count_nonzero(x < -3.0) and o[1] == np.count_nonzero(x > 5.0)


def test_bins_match_exact_arithmetic_away_from_edges():
    # The single-precision bin is floor((v-lo) * nbins / (hi-lo)) evaluated
    # exactly, except within a few ulps of a bin edge; it is monotone in v and
    # never off by more than one.
    rng = np.random.default_rng(2)
    lo, hi, nb = np.float32(-2.75), np.float32(13.3), 1000
    vals = np.sort(rng.uniform(-2.75, 13.3, 1500).astype(np.float32))
    vals = np.concatenate([[lo], vals, [hi]])
    flo, fhi = Fraction(float(lo)), Fraction(float(hi))
    prev = -1
    for v in vals:
        b = _bin_of(v, float(lo), float(hi), nb)
        exact = min(int((Fraction(float(v)) - flo) * nb / (fhi - flo)), nb - 1)
        assert abs(b - exact) <= 1
        pos = (Fraction(float(v)) - flo) * nb / (fhi - flo)
        dist = abs(pos - round(pos))
        if dist > Fraction(1, 10000):
            assert b == exact, (v, b, exact)
        assert b >= prev
        prev = b
    assert _bin_of(lo, float(lo), float(hi), nb) == 0
    assert _bin_of(hi, float(lo), float(hi), nb) == nb - 1


def test_lo_equals_hi():
    x = np.float32([2.0, 2.0, 1.0, 3.0, np.nan, 2.0])
    c, o = oracle.histogram(x, 2.0, 2.0, 16)
    assert c[0] == 3 and c[1:].sum() == 0 and list(o) == [1, 1]


@pytest.mark.parametrize("lo,hi,nb", [(0.0, 1.0, 0), (0.0, 1.0, 65537), (1.0, 0.0, 8), (float("nan"), 1.0, 8),
                                      (0.0, float("inf"), 8), (-3.0e38, 3.0e38, 8), (0.0, 1e-45, 65536)])
def test_rejected(lo, hi, nb):
    with pytest.raises(ValueError):
        oracle.histogram(np.zeros(4, np.float32), lo, hi, nb)


def test_region_and_int16():
    rng = np.random.default_rng(4)
    a = rng.integers(-100, 100, (6, 7, 9)).astype(np.int16)
    reg = (1, 2, 0, 8, 6, 5)
    c1, o1 = oracle.histogram(a, -50.0, 60.0, 110, reg)
    sub = np.ascontiguousarray(a[0:5, 2:6, 1:8]).astype(np.float32)
    c2, o2 = oracle.histogram(sub, -50.0, 60.0, 110)
    assert np.array_equal(c1, c2) and np.array_equal(o1, o2)
    # integer values on a unit grid: bin = v - lo
    ref = np.bincount((sub[(sub >= -50) & (sub <= 60)] + 50).astype(np.int64), minlength=111)
    ref[109] += ref[110]
    assert np.array_equal(c1, ref[:110].astype(np.uint64))


def test_scale_is_single_precision():
    # (float)nbins / (hi - lo) rounded once in single precision
    s = oracle.hist_scale(0.0, 3.0, 10)
    assert s == float(np.float32(10) / np.float32(3))
    assert s != 10 / 3
