"""Pins of the large-input oracle (exact sums, two-level key counts, slab
streaming) against definitions it does not share code with: exact rational
arithmetic, sorting by totalOrder, and the in-memory oracle."""
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def _bits(v: float) -> bytes:
    return struct.pack("<d", v)


def _same(a: float, b: float) -> bool:
    return (math.isnan(a) and math.isnan(b)) or _bits(a) == _bits(b)


def _tot_key(v: float):
    return (v, math.copysign(1.0, v) > 0)


def _exact_by_fractions(vals):
    """mean, M2 and std of float32 values by exact rational arithmetic, each
    rounded once (std: sqrt of the once-rounded M2 / n)."""
    fr = [Fraction(float(v)) for v in vals]
    n = len(fr)
    mean = sum(fr) / n
    m2 = sum((x - mean) ** 2 for x in fr)
    return float(mean), float(m2), math.sqrt(float(m2 / n))


@pytest.mark.parametrize("seed", range(6))
def test_exact_moments_equal_rational_arithmetic(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3000))
    kind = seed % 3
    if kind == 0:  # noise far from zero: mean/std ~ 1e5
        x = (1e5 + rng.standard_normal(n)).astype(np.float32)
    elif kind == 1:  # every exponent, both signs, denormals
        x = (rng.standard_normal(n) * np.exp2(rng.integers(-150, 120, n))).astype(np.float32)
    else:
        x = rng.integers(-1000, 1000, n).astype(np.float32) * np.float32(0.125)
    x[rng.random(n) < 0.05] = np.nan
    got = oracle.stats_exact(x, 16)
    vals = [v for v in x if not math.isnan(v)]
    if not vals:
        assert got["count"] == 0
        return
    mean, m2, std = _exact_by_fractions(vals)
    assert got["count"] == len(vals)
    if len(set(vals)) == 1:
        assert got["mean"] == vals[0] and got["m2"] == 0.0
        return
    assert _same(got["mean"], mean), (got["mean"], mean)
    assert _same(got["m2"], m2), (got["m2"], m2)
    assert _same(got["std"], std), (got["std"], std)


def _adversarial():
    rng = np.random.default_rng(42)
    n = 4096
    return {
        "noise": rng.standard_normal(n).astype(np.float32),
        "constant": np.full(n, 3.25, np.float32),
        "all_nan": np.full(n, np.nan, np.float32),
        "single": np.float32([7.5]),
        "signed_zeros": rng.choice(np.float32([0.0, -0.0]), n).astype(np.float32),
        "zeros_around_median": np.concatenate([np.full(100, -1.0), np.full(50, -0.0), np.full(50, 0.0),
                                               np.full(100, 1.0)]).astype(np.float32),
        "denormals": (rng.integers(-50, 50, n) * np.float32(1e-45)).astype(np.float32),
        "with_inf": np.concatenate([rng.standard_normal(n - 3), [np.inf, -np.inf, np.nan]]).astype(np.float32),
        "pos_inf": np.concatenate([rng.standard_normal(n - 3), [np.inf, np.inf, np.nan]]).astype(np.float32),
        "all_inf": np.full(n, -np.inf, np.float32),
        "heavy_ties": rng.integers(-3, 4, n).astype(np.float32),
        "huge_range": np.float32([-3.0e38, 3.0e38, 0.0, 1.0, -1.0]),
        "large_mean": (1000.0 + rng.standard_normal(n)).astype(np.float32),
        "int16": rng.integers(-32768, 32768, n).astype(np.int16),
    }


@pytest.mark.parametrize("name", list(_adversarial().keys()))
def test_exact_agrees_with_in_memory_oracle(name):
    x = _adversarial()[name]
    want = oracle.stats(x, 64)
    got = oracle.stats_exact(x, 64, threads=3)
    for k in ("count", "nan_count", "hist_skipped"):
        assert got[k] == want[k], (k, got[k], want[k])
    for k in ("min", "max", "median"):
        assert _same(got[k], want[k]) or (got[k] == want[k] and k != "median"), (k, got[k], want[k])
    # the median is a stored value: bit-exact, sign of zero included
    assert _same(got["median"], want["median"]), (got["median"], want["median"])
    assert np.array_equal(got["counts"], want["counts"]) and np.array_equal(got["outliers"], want["outliers"])
    for k in ("mean", "m2", "std"):
        w, g = want[k], got[k]
        if math.isnan(w) or math.isinf(w) or w == 0.0:
            assert _same(g, w) or (g == w), (k, g, w)
        else:
            assert abs(g - w) <= 4e-16 * abs(w), (k, g, w)  # both within an ulp or two of the exact value


def test_median_by_brute_force_sort():
    rng = np.random.default_rng(7)
    pool = np.float32([-np.inf, -3.4e38, -1.0, -1e-45, -0.0, 0.0, 1e-45, 0.5, 1.0, 3.4e38, np.inf, np.nan])
    for _ in range(300):
        n = int(rng.integers(1, 40))
        x = pool[rng.integers(0, len(pool), n)]
        vals = sorted((float(v) for v in x if not math.isnan(v)), key=_tot_key)
        got = oracle.stats_exact(x, 8, threads=2)
        if not vals:
            assert got["count"] == 0 and math.isnan(got["median"])
            continue
        assert _same(got["median"], vals[(len(vals) - 1) // 2]), (x, got["median"])
        assert _same(got["min"], vals[0]) and _same(got["max"], vals[-1])


def test_thread_count_does_not_change_bits():
    spec = synth.scaled(synth.SPECS["c1"], 96, 80, 40)
    a, _ = synth.generate(spec)
    ref = oracle.stats_exact(a, 1000, threads=1)
    for t in (2, 5, 8):
        got = oracle.stats_exact(a, 1000, threads=t)
        for k in ("count", "nan_count", "mean", "m2", "std", "min", "max", "median"):
            assert _same(got[k], ref[k]) or got[k] == ref[k], (t, k)
        assert np.array_equal(got["counts"], ref["counts"])


@pytest.mark.parametrize("dtype", ["f32", "i16"])
def test_streaming_equals_in_memory(dtype):
    base = synth.SPECS["c1"] if dtype == "f32" else synth.SPECS["c5c"]
    spec = synth.scaled(base, 72, 40, 37)
    whole, nan = synth.generate(spec)
    seen = []
    got = oracle.stats_streaming(spec, 300, threads=3, slab_voxels=72 * 40 * 5,
                                 on_slab=lambda z0, z1, arr: seen.append((z0, z1, arr.copy())))
    # every plane exactly once, in order, with the generator's bytes
    assert [s[0] for s in seen] == list(range(0, 37, 5)) and seen[-1][1] == 37
    assert np.concatenate([s[2] for s in seen]).tobytes() == whole.tobytes()
    want = oracle.stats_exact(whole, 300, threads=2)
    for k in ("count", "nan_count", "mean", "m2", "std", "min", "max", "median", "hist_skipped"):
        assert _same(got[k], want[k]) or got[k] == want[k], k
    assert np.array_equal(got["counts"], want["counts"]) and np.array_equal(got["outliers"], want["outliers"])
    assert got["generator_nan"] == nan == got["nan_count"]
    # and the in-memory oracle agrees on everything it defines exactly
    ref = oracle.stats(whole, 300)
    assert ref["count"] == got["count"] and np.array_equal(ref["counts"], got["counts"])
    assert _same(ref["median"], got["median"])
    assert abs(ref["mean"] - got["mean"]) <= 1e-15 * abs(ref["mean"]) + 1e-16
    assert abs(ref["std"] - got["std"]) <= 1e-15 * ref["std"]


def test_boxes_equal_single_regions():
    spec = synth.scaled(synth.SPECS["c1"], 60, 50, 40)
    a, _ = synth.generate(spec)
    rng = np.random.default_rng(11)
    boxes = synth.regions(40, (60, 50, 40), seed=5, edge_lo=1, edge_hi=40).tolist()
    boxes += [[0, 0, 0, 60, 50, 40], [7, 7, 7, 8, 8, 8], [3, 3, 3, 3, 9, 9], [0, 0, 0, 61, 1, 1]]
    res, counts = oracle.stats_boxes(a, np.array(boxes), 32, threads=4, chunk=7)
    assert res[-1]["status"] == -1 and res[-2]["status"] == -1  # empty and out-of-range boxes
    for i, b in enumerate(boxes[:-2]):
        want = oracle.stats_exact(a, 32, region=b)
        got = res[i]
        assert got["status"] == 0
        for k in ("count", "nan_count", "mean", "m2", "std", "min", "max", "median", "hist_skipped"):
            assert _same(got[k], want[k]) or got[k] == want[k], (i, b, k)
        assert np.array_equal(counts[i], want["counts"]), (i, b)
        ref = oracle.stats(a, 32, b)
        assert _same(ref["median"], got["median"]) and np.array_equal(ref["counts"], counts[i])
    _ = rng
