"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances:
* counts, nan_count, histogram bins, outliers, min, max, median: bit-exact;
* mean: |gpu - oracle| <= 1e-12 |oracle| + 1e-14 rms(x)   (rms = hypot(mean, std));
  the second term only matters when the mean is ~0 relative to the spread,
  where a relative bound on the mean is meaningless.  The kernels sum each
  lane's values in double (one 2^-53 rounding per addition) and merge lanes
  and blocks in double, so for data of either sign the rounding errors
  cancel to far below 1e-14 rms;
* std and m2: relative 1e-12 (exactly 0 when the oracle's is 0).
"""
import math
import struct

import numpy as np

MEAN_REL = 1e-12
MEAN_RMS = 1e-14
STD_REL = 1e-12


def f32_bits(v: float) -> bytes:
    return struct.pack("<f", v)


def same_value(a: float, b: float, dtype: str = "f32") -> bool:
    """Bit-exact equality of two stored values (NaN == NaN)."""
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    if dtype == "f32":
        return f32_bits(a) == f32_bits(b)
    return a == b


def check_moments(got: dict, want: dict, dtype: str = "f32", what: str = ""):
    assert got["status"] == 0, (what, got)
    assert got["count"] == want["count"], (what, got["count"], want["count"])
    assert got["nan_count"] == want["nan_count"], (what, got["nan_count"], want["nan_count"])
    if want["count"] == 0:
        for k in ("mean", "m2", "std", "min", "max"):
            assert math.isnan(got[k]), (what, k, got[k])
        return
    assert same_value(got["min"], want["min"], dtype), (what, "min", got["min"], want["min"])
    assert same_value(got["max"], want["max"], dtype), (what, "max", got["max"], want["max"])
    if not math.isfinite(want["mean"]):
        # infinities in the data: the mean is +inf, -inf or NaN (both signs)
        # and, unless every value is the same (std 0), the spread is NaN
        assert same_value(got["mean"], want["mean"], "f64"), (what, "mean", got["mean"], want["mean"])
        if want["std"] == 0.0:
            assert got["std"] == 0.0 and got["m2"] == 0.0, (what, "std", got["std"])
        else:
            assert math.isnan(want["std"]), (what, want)
            assert math.isnan(got["std"]) and math.isnan(got["m2"]), (what, "std", got["std"])
        return
    rms = math.hypot(want["mean"], want["std"])
    assert abs(got["mean"] - want["mean"]) <= MEAN_REL * abs(want["mean"]) + MEAN_RMS * rms, \
        (what, "mean", got["mean"], want["mean"])
    if want["std"] == 0.0:
        assert got["std"] == 0.0 and got["m2"] == 0.0, (what, got["std"])
    else:
        assert abs(got["std"] - want["std"]) <= STD_REL * want["std"], (what, "std", got["std"], want["std"])
        assert abs(got["m2"] - want["m2"]) <= STD_REL * want["m2"] * 2, (what, "m2", got["m2"], want["m2"])


def check_median(got_median: float, want_median: float, dtype: str = "f32", what: str = ""):
    assert same_value(got_median, want_median, dtype), (what, "median", got_median, want_median)


def as_u64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64) if hasattr(t, "cpu") else np.asarray(t).view(np.uint64)


def check_hist(got_counts, got_outl, want_counts, want_outl, what: str = ""):
    gc = as_u64(got_counts)
    assert np.array_equal(gc, want_counts), (what, "counts differ at", np.nonzero(gc != want_counts)[0][:10])
    if got_outl is not None:
        assert np.array_equal(as_u64(got_outl), want_outl), (what, as_u64(got_outl), want_outl)


def check_sigma_counts(host, got, cell, k, what="", cells=None):
    """Local k-sigma counts against the oracle.  The GPU's cell moments differ
    from the oracle's within the tolerances above, so its threshold may move
    by that much: each count must lie between the oracle's counts at the
    threshold pushed up and down by the tolerance (equal unless a voxel sits
    that close to it).  cells: indices to check (default all).  Returns how
    many counts equal the oracle's exactly."""
    import oracle
    nz, ny, nx = host.shape
    boxes = oracle.minimap_cells((nx, ny, nz), cell)
    idx = range(len(boxes)) if cells is None else cells
    n_equal = 0
    for i in idx:
        x0, y0, z0, x1, y1, z1 = (int(v) for v in boxes[i])
        mo = oracle.moments(host, (x0, y0, z0, x1, y1, z1))
        if mo["count"] == 0:
            assert got[i] == 0, (what, i)
            n_equal += 1
            continue
        thr = mo["mean"] + k * mo["std"]
        rms = math.hypot(mo["mean"], mo["std"])
        slack = MEAN_REL * abs(mo["mean"]) + MEAN_RMS * rms + abs(k) * STD_REL * mo["std"] + 4e-16 * abs(thr)
        v = host[z0:z1, y0:y1, x0:x1].astype(np.float64)
        exact = np.count_nonzero(v > thr)
        lo = np.count_nonzero(v > thr + slack)
        hi = np.count_nonzero(v > thr - slack)
        assert lo <= got[i] <= hi, (what, k, i, (x0, y0, z0, x1, y1, z1), int(got[i]), lo, hi, exact)
        n_equal += int(got[i] == exact)
    return n_equal
