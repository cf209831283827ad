"""CPU oracle for the cube statistics -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does, and this package never
imports the GPU library: the two share no code.  Everything here is a plain,
slow restatement of what the paper (arXiv 1211.4896) defines:

* moments      -- Section 4.2: count, mean and standard deviation of the
                  non-NULL voxels, plus min/max (known at load, Section 4.1);
* histogram    -- Section 4.1: a fixed-range N-bin histogram, one visit per
                  voxel, with the single-precision bin formula
                  b = min((int)((v - lo) * scale), nbins - 1),
                  scale = (float)nbins / (hi - lo);
* median       -- Section 4.3: the exact median, read here as the lower
                  median (0-based rank floor((n-1)/2) under totalOrder), found
                  with a library selection (numpy.partition) on a copy;
* median_sort  -- the same value by qsort, for small inputs;
* torben       -- Appendix A, Algorithm 1 (Torben Mogensen's method), a second
                  and independent algorithm for the same value;
* quantile     -- the lower q-quantile, value of rank floor(q (n-1)); q = 0.5
                  is the lower median (an arbitrary rank is the general form of
                  the selection Section 4.3 performs);
* mad          -- the median absolute deviation Section 4.3 names: the lower
                  median of |x - m| with m the lower median and x - m rounded
                  to single precision (int16: exact);
* minimap_cells, sigma_counts
               -- Section 4.5's statistical mini-map: the cube cut into cells
                  of cx*cy*cz voxels (the last cell along an axis keeps the
                  remainder), each summarised by its statistics, and the local
                  threshold: per cell, the voxels above mean + k * std;
* spectrum     -- Section 4.4's 3-D spectrum tool: the cube sampled along
                  arbitrary rays at a constant step, each sample a trilinear
                  interpolation of its eight neighbouring voxels (Fig. 8).

NaN is the NULL value and is excluded everywhere.  The C parts live in
tsa_oracle.c and are built with gcc by ``build()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

F32, I16 = 0, 1


class _Moments(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("nan_count", ctypes.c_uint64), ("mean", ctypes.c_double),
                ("m2", ctypes.c_double), ("std", ctypes.c_double), ("min", ctypes.c_double),
                ("max", ctypes.c_double)]


def build(force: bool = True) -> str:
    """Compile liboracle.so (gcc, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_moments.argtypes = [P, ctypes.c_int, I64, I64, I64, P, ctypes.POINTER(_Moments)]
        lib.oracle_moments.restype = ctypes.c_int
        lib.oracle_hist_scale.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_float)]
        lib.oracle_hist_scale.restype = ctypes.c_int
        lib.oracle_histogram.argtypes = [P, ctypes.c_int, I64, I64, I64, P, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_int32, P, P]
        lib.oracle_histogram.restype = ctypes.c_int
        lib.oracle_torben_guess.argtypes = [ctypes.c_float, ctypes.c_float]
        lib.oracle_torben_guess.restype = ctypes.c_float
        lib.oracle_torben.argtypes = [P, ctypes.c_int, I64, ctypes.POINTER(ctypes.c_float), P, ctypes.c_int]
        lib.oracle_torben.restype = ctypes.c_int
        lib.oracle_median_sort.argtypes = [P, ctypes.c_int, I64, I64, I64, P, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_median_sort.restype = ctypes.c_int
        _lib = lib
    return _lib


def _cube(a: np.ndarray):
    if a.ndim == 1:
        a = a.reshape(1, 1, -1)
    if a.ndim != 3:
        raise ValueError("cube must be 1-D or (nz, ny, nx)")
    a = np.ascontiguousarray(a)
    if a.dtype == np.float32:
        dt = F32
    elif a.dtype == np.int16:
        dt = I16
    else:
        raise TypeError("cube dtype must be float32 or int16")
    nz, ny, nx = a.shape
    return a, dt, nx, ny, nz


def _box(region):
    if region is None:
        return None, None
    b = np.ascontiguousarray(np.asarray(region, dtype=np.int64).reshape(6))
    return b, b.ctypes.data


def moments(a: np.ndarray, region=None) -> dict:
    """Section 4.2 moments of the non-NaN voxels (plus min/max), in double."""
    lib = _load()
    a, dt, nx, ny, nz = _cube(a)
    b, bp = _box(region)
    out = _Moments()
    if lib.oracle_moments(a.ctypes.data, dt, nx, ny, nz, bp, ctypes.byref(out)) != 0:
        raise ValueError("invalid region or dtype")
    return {k: getattr(out, k) for k, _ in _Moments._fields_}


def hist_scale(lo: float, hi: float, nbins: int) -> float:
    lib = _load()
    s = ctypes.c_float()
    if lib.oracle_hist_scale(lo, hi, nbins, ctypes.byref(s)) != 0:
        raise ValueError("invalid histogram range or bin count")
    return s.value


def histogram(a: np.ndarray, lo: float, hi: float, nbins: int, region=None):
    """Section 4.1 histogram: returns (counts uint64[nbins], outliers uint64[2] = below, above)."""
    lib = _load()
    a, dt, nx, ny, nz = _cube(a)
    b, bp = _box(region)
    counts = np.zeros(nbins, dtype=np.uint64)
    outl = np.zeros(2, dtype=np.uint64)
    if lib.oracle_histogram(a.ctypes.data, dt, nx, ny, nz, bp, lo, hi, nbins, counts.ctypes.data,
                            outl.ctypes.data) != 0:
        raise ValueError("invalid histogram arguments")
    return counts, outl


def torben_guess(mn: float, mx: float) -> float:
    return _load().oracle_torben_guess(mn, mx)


def torben(a: np.ndarray, trace_cap: int = 0):
    """Algorithm 1 on the non-NaN values; returns (median float, iterations, trace rows)."""
    lib = _load()
    a = np.ascontiguousarray(a).reshape(-1)
    dt = F32 if a.dtype == np.float32 else I16
    med = ctypes.c_float()
    tr = np.zeros((max(trace_cap, 1), 6), dtype=np.float64)
    it = lib.oracle_torben(a.ctypes.data, dt, a.size, ctypes.byref(med), tr.ctypes.data, trace_cap)
    if it < 0:
        raise RuntimeError("Torben iteration cap reached")
    return med.value, it, tr[:min(it, trace_cap)]


def median_sort(a: np.ndarray, region=None):
    """Lower median by qsort (small inputs): returns (value, count)."""
    lib = _load()
    a, dt, nx, ny, nz = _cube(a)
    b, bp = _box(region)
    med = ctypes.c_double()
    cnt = ctypes.c_uint64()
    if lib.oracle_median_sort(a.ctypes.data, dt, nx, ny, nz, bp, ctypes.byref(med), ctypes.byref(cnt)) != 0:
        raise ValueError("invalid region or dtype")
    return med.value, int(cnt.value)


def _region_view(a: np.ndarray, region):
    if a.ndim == 1:
        a = a.reshape(1, 1, -1)
    if region is None:
        return a
    x0, y0, z0, x1, y1, z1 = (int(v) for v in region)
    nz, ny, nx = a.shape
    if not (0 <= x0 < x1 <= nx and 0 <= y0 < y1 <= ny and 0 <= z0 < z1 <= nz):
        raise ValueError("invalid region")
    return a[z0:z1, y0:y1, x0:x1]


def median(a: np.ndarray, region=None):
    """Lower median (rank floor((n-1)/2) by totalOrder) of the non-NaN voxels.

    Returns (value, count); value is NaN when count == 0.  Selection is
    numpy.partition on a copy; numpy orders -0 and +0 as equal, so a zero
    result takes the sign that totalOrder gives rank k: -0 when more than k
    values are negative or -0.
    """
    v = _region_view(a, region)
    if v.dtype == np.float32:
        flat = v.reshape(-1)
        vals = flat[~np.isnan(flat)]
    else:
        vals = v.reshape(-1)
    n = vals.size
    if n == 0:
        return float("nan"), 0
    k = (n - 1) // 2
    m = np.partition(vals, k)[k]
    if vals.dtype == np.float32 and m == 0:
        n_before = int(np.count_nonzero(vals < 0)) + int(np.count_nonzero((vals == 0) & np.signbit(vals)))
        m = np.float32(-0.0) if k < n_before else np.float32(0.0)
    return float(m), n


def stats(a: np.ndarray, nbins: int, region=None) -> dict:
    """The full trio on one cube or region: moments, histogram over the
    region's own [min, max] (skipped, all zero, when there is no valid value
    or the range is not representable), and the lower median."""
    mo = moments(a, region)
    out = dict(mo)
    if mo["count"] == 0:
        out["counts"] = np.zeros(nbins, dtype=np.uint64)
        out["outliers"] = np.zeros(2, dtype=np.uint64)
        out["median"] = float("nan")
        out["hist_skipped"] = True
        return out
    lo, hi = np.float32(mo["min"]), np.float32(mo["max"])
    try:
        hist_scale(float(lo), float(hi), nbins)
        out["counts"], out["outliers"] = histogram(a, float(lo), float(hi), nbins, region)
        out["hist_skipped"] = False
    except ValueError:  # infinite extremes or a range wider than single precision
        out["counts"] = np.zeros(nbins, dtype=np.uint64)
        out["outliers"] = np.zeros(2, dtype=np.uint64)
        out["hist_skipped"] = True
    out["median"], _ = median(a, region)
    return out


def _valid_values(a: np.ndarray, region=None) -> np.ndarray:
    v = _region_view(a, region)
    flat = v.reshape(-1)
    return flat[~np.isnan(flat)] if flat.dtype == np.float32 else flat


def _select(vals: np.ndarray, k: int):
    """Value of 0-based rank k by totalOrder (numpy.partition; signed zero as in median())."""
    m = np.partition(vals, k)[k]
    if vals.dtype == np.float32 and m == 0:
        n_before = int(np.count_nonzero(vals < 0)) + int(np.count_nonzero((vals == 0) & np.signbit(vals)))
        m = np.float32(-0.0) if k < n_before else np.float32(0.0)
    return m


def quantile_rank(q: float, n: int) -> int:
    """0-based rank floor(q (n-1)), the product taken in double precision."""
    if not (0.0 <= q <= 1.0) or n < 1:
        raise ValueError("q must lie in [0, 1] and n >= 1")
    k = int(np.floor(np.float64(q) * np.float64(n - 1)))
    return min(max(k, 0), n - 1)


def quantile(a: np.ndarray, q: float, region=None):
    """Lower q-quantile of the non-NaN voxels: returns (value, count); NaN when empty."""
    vals = _valid_values(a, region)
    n = vals.size
    if n == 0:
        return float("nan"), 0
    return float(_select(vals, quantile_rank(q, n))), n


def mad(a: np.ndarray, region=None):
    """Median absolute deviation: returns (median, mad, count).

    m is the lower median; deviations |x - m| are rounded to single precision
    for float32 cubes (numpy float32 arithmetic: one IEEE subtraction, then an
    exact absolute value) and exact integers for int16 cubes; the MAD is their
    lower median."""
    vals = _valid_values(a, region)
    n = vals.size
    if n == 0:
        return float("nan"), float("nan"), 0
    k = (n - 1) // 2
    m = _select(vals, k)
    if vals.dtype == np.float32:
        d = np.abs(vals - np.float32(m))
    else:
        d = np.abs(vals.astype(np.int32) - np.int32(m))
    return float(m), float(np.partition(d, k)[k]), n


def minimap_cells(dims, cell):
    """Boxes (x0,y0,z0,x1,y1,z1) of the mini-map cells, x-fastest cell order."""
    nx, ny, nz = dims
    cx, cy, cz = cell
    if min(cx, cy, cz) < 1:
        raise ValueError("cell edges must be >= 1")
    out = []
    for z0 in range(0, nz, cz):
        for y0 in range(0, ny, cy):
            for x0 in range(0, nx, cx):
                out.append((x0, y0, z0, min(x0 + cx, nx), min(y0 + cy, ny), min(z0 + cz, nz)))
    return np.array(out, dtype=np.int64).reshape(-1, 6)


def sigma_counts(a: np.ndarray, cell, k: float) -> np.ndarray:
    """Per mini-map cell: the number of non-NaN voxels x with x > mean + k*std
    (the cell's own moments, double precision; the comparison is made in double
    on the exactly converted value).  Cells without a valid voxel count 0."""
    nz, ny, nx = a.shape
    boxes = minimap_cells((nx, ny, nz), cell)
    out = np.zeros(len(boxes), dtype=np.uint64)
    for i, b in enumerate(boxes):
        mo = moments(a, b)
        if mo["count"] == 0:
            continue
        thr = mo["mean"] + k * mo["std"]
        v = _region_view(a, b).astype(np.float64)
        out[i] = np.count_nonzero(v > thr)  # NaN compares false
    return out


def _axis_cell(p: np.ndarray, n: int):
    """Lower corner index, fraction and upper corner index of coordinates p
    (all inside [0, n-1]) along an axis of n voxels."""
    i0 = np.floor(p).astype(np.int64)
    if n >= 2:
        i0 = np.minimum(i0, n - 2)
    else:
        i0 = np.zeros_like(i0)
    f = p - i0
    i1 = np.minimum(i0 + 1, n - 1)
    return i0, f, i1


def spectrum(a: np.ndarray, origins, steps, nsamples: int) -> np.ndarray:
    """Section 4.4 (with Fig. 8): a data profile along a ray through the cube,
    sampled at a constant step and trilinearly interpolated.

    Voxel (x, y, z) = a[z, y, x] sits at the integer point (x, y, z).  Ray r's
    sample i is at p = origin[r] + i * step[r], per coordinate: i * step
    rounded to double, then added to the origin and rounded.  A sample outside
    [0, nx-1] x [0, ny-1] x [0, nz-1] is NaN.  Inside, per axis
    x0 = min(floor(x), nx - 2) (0 when nx == 1), fx = x - x0,
    x1 = min(x0 + 1, nx - 1), and the same for y and z.  Corner c = bx + 2 by
    + 4 bz takes (x_bx, y_by, z_bz) with weight (wx * wy) * wz, where w is
    1 - f for bit 0 and f for bit 1.  The sample is 0.0 plus weight * value
    for c = 0, 1, ..., 7 in that order, corners of weight 0 skipped, all in
    double; a NaN corner of non-zero weight makes it NaN.
    Returns float64 [nrays, nsamples]."""
    a = np.asarray(a)
    nz, ny, nx = a.shape
    o = np.asarray(origins, dtype=np.float64).reshape(-1, 3)
    s = np.asarray(steps, dtype=np.float64).reshape(-1, 3)
    if nsamples < 0 or len(o) != len(s):
        raise ValueError("bad rays")
    out = np.full((len(o), nsamples), np.nan)
    ii = np.arange(nsamples, dtype=np.float64)
    for r in range(len(o)):
        px = o[r, 0] + ii * s[r, 0]
        py = o[r, 1] + ii * s[r, 1]
        pz = o[r, 2] + ii * s[r, 2]
        inside = (px >= 0) & (px <= nx - 1) & (py >= 0) & (py <= ny - 1) & (pz >= 0) & (pz <= nz - 1)
        if not inside.any():
            continue
        x0, fx, x1 = _axis_cell(px[inside], nx)
        y0, fy, y1 = _axis_cell(py[inside], ny)
        z0, fz, z1 = _axis_cell(pz[inside], nz)
        xs, ys, zs = (x0, x1), (y0, y1), (z0, z1)
        wx, wy, wz = (1.0 - fx, fx), (1.0 - fy, fy), (1.0 - fz, fz)
        acc = np.zeros(len(x0))
        for c in range(8):
            bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            w = (wx[bx] * wy[by]) * wz[bz]
            v = a[zs[bz], ys[by], xs[bx]].astype(np.float64)
            used = w != 0.0
            acc[used] = acc[used] + w[used] * v[used]
        out[r, inside] = acc
    return out
