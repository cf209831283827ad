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
* stats_exact, stats_boxes, stats_streaming
               -- the same trio as ``stats`` for inputs too large to sort or
                  to hold in memory (tsa_oracle_stream.c): exact sums of the
                  values and of their squares (one rounding of the mean and of
                  M2 at the end), the histogram with the same bin formula, and
                  the lower median by counting keys on their top 16 bits, then
                  on their low 16 bits inside the bucket holding the rank.
                  ``stats_streaming`` regenerates a synthetic cube slab by slab
                  (the 206 GB cube), ``stats_boxes`` takes a batch of boxes.
                  Host threads split the values; they merge by integer
                  addition, so the results do not depend on the thread count.

NaN is the NULL value and is excluded everywhere.  The C parts live in
tsa_oracle.c and tsa_oracle_stream.c and are built with gcc by ``build()``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsa_oracle.c")
_SRC_STREAM = os.path.join(_HERE, "tsa_oracle_stream.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

F32, I16 = 0, 1


class _Moments(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("nan_count", ctypes.c_uint64), ("mean", ctypes.c_double),
                ("m2", ctypes.c_double), ("std", ctypes.c_double), ("min", ctypes.c_double),
                ("max", ctypes.c_double)]


class _Acc1(ctypes.Structure):  # oracle_acc1 (tsa_oracle_stream.c)
    _fields_ = [("n", ctypes.c_uint64), ("nan", ctypes.c_uint64), ("pinf", ctypes.c_uint64),
                ("minf", ctypes.c_uint64), ("kmin", ctypes.c_uint32), ("kmax", ctypes.c_uint32),
                ("s", ctypes.c_int64 * 256), ("qh", ctypes.c_uint64 * 256), ("ql", ctypes.c_uint64 * 256),
                ("top", ctypes.c_uint64 * 65536)]


class _Pass2(ctypes.Structure):  # oracle_pass2_args
    _fields_ = [("lo", ctypes.c_float), ("hi", ctypes.c_float), ("scale", ctypes.c_float), ("nbins", ctypes.c_int32),
                ("hist_on", ctypes.c_int32), ("sel", ctypes.c_uint32), ("sel_on", ctypes.c_int32)]


class _Acc2(ctypes.Structure):  # oracle_acc2
    _fields_ = [("below", ctypes.c_uint64), ("above", ctypes.c_uint64), ("low", ctypes.c_uint64 * 65536)]


BOX_OUT_DTYPE = np.dtype([("n", "<u8"), ("nan", "<u8"), ("pinf", "<u8"), ("minf", "<u8"), ("kmin", "<u4"),
                          ("kmax", "<u4"), ("median_key", "<u4"), ("hist_on", "<i4"), ("status", "<i4"),
                          ("pad", "<i4")])


def build(force: bool = True) -> str:
    """Compile liboracle.so (gcc, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC, _SRC_STREAM, "-lm"])
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
        lib.oracle_acc1_size.restype = ctypes.c_size_t
        lib.oracle_acc2_size.restype = ctypes.c_size_t
        assert lib.oracle_acc1_size() == ctypes.sizeof(_Acc1) and lib.oracle_acc2_size() == ctypes.sizeof(_Acc2)
        lib.oracle_acc1_init.argtypes = [ctypes.POINTER(_Acc1)]
        lib.oracle_acc1_init.restype = None
        lib.oracle_acc1_box.argtypes = [P, ctypes.c_int, I64, I64, I64, P, ctypes.POINTER(_Acc1)]
        lib.oracle_acc1_box.restype = ctypes.c_int
        lib.oracle_acc2_box.argtypes = [P, ctypes.c_int, I64, I64, I64, P, ctypes.POINTER(_Pass2), ctypes.POINTER(_Acc2),
                                        P]
        lib.oracle_acc2_box.restype = ctypes.c_int
        lib.oracle_pass1_array.argtypes = [P, ctypes.c_int, I64, ctypes.c_int, ctypes.POINTER(_Acc1)]
        lib.oracle_pass1_array.restype = ctypes.c_int
        lib.oracle_pass2_array.argtypes = [P, ctypes.c_int, I64, ctypes.c_int, ctypes.POINTER(_Pass2),
                                           ctypes.POINTER(_Acc2), P]
        lib.oracle_pass2_array.restype = ctypes.c_int
        lib.oracle_rank_bin.argtypes = [P, I64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_rank_bin.restype = I64
        lib.oracle_boxes.argtypes = [P, ctypes.c_int, I64, I64, I64, P, I64, ctypes.c_int32, ctypes.c_int, P, P, P, P,
                                     P]
        lib.oracle_boxes.restype = ctypes.c_int
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
    lower median over all n valid values.  A value equal to m deviates by +0,
    written out so that it also holds when m is infinite (the IEEE difference
    inf - inf would be NaN)."""
    vals = _valid_values(a, region)
    n = vals.size
    if n == 0:
        return float("nan"), float("nan"), 0
    k = (n - 1) // 2
    m = _select(vals, k)
    if vals.dtype == np.float32:
        m32 = np.float32(m)
        with np.errstate(invalid="ignore"):
            diff = np.abs(vals - m32)
        d = np.where(vals == m32, np.float32(0.0), diff).astype(np.float32)
        assert not np.isnan(d).any()
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


# ---------------------------------------------------------------------------
# large inputs: exact sums, two-level key counts (tsa_oracle_stream.c)
# ---------------------------------------------------------------------------

def _threads(threads=None) -> int:
    if threads:
        return int(threads)
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def value_of_key(k: int) -> float:
    """The float32 value of an order key (the inverse of the key map)."""
    k = int(k) & 0xFFFFFFFF
    u = (k & 0x7FFFFFFF) if (k & 0x80000000) else (~k & 0xFFFFFFFF)
    return float(np.array([u], dtype=np.uint32).view(np.float32)[0])


def exact_moments(n, nan, pinf, minf, kmin, kmax, s, qh, ql) -> dict:
    """Moments from exact per-exponent bins: the value with biased float32
    exponent E (E = 1 for denormals) and signed significand M is M * 2^(E-150),
    so S = sum of s[E] * 2^(E-1) and Q = sum of (qh[E] * 2^24 + ql[E]) * 2^(2E-2)
    are the exact sum and sum of squares in units of 2^-149 and 2^-298.  Then
    mean = S / n and M2 = (n Q - S^2) / n are each rounded once (Python's
    integer division is correctly rounded); std = sqrt(M2 / n) with M2 / n
    rounded once.  Infinities, one repeated value and n = 0 as in moments()."""
    n, nan = int(n), int(nan)
    out = {"count": n, "nan_count": nan}
    qn = float("nan")
    if n == 0:
        out.update(mean=qn, m2=qn, std=qn, min=qn, max=qn)
        return out
    out["min"], out["max"] = value_of_key(kmin), value_of_key(kmax)
    if int(kmin) == int(kmax):
        out.update(mean=out["min"], m2=0.0, std=0.0)
        return out
    if pinf or minf:
        mean = qn if (pinf and minf) else (math.inf if pinf else -math.inf)
        out.update(mean=mean, m2=qn, std=qn)
        return out
    s = np.asarray(s, dtype=np.int64)
    qh = np.asarray(qh, dtype=np.uint64)
    ql = np.asarray(ql, dtype=np.uint64)
    S = 0
    for e in np.nonzero(s)[0]:
        S += int(s[e]) << (int(e) - 1)
    Q = 0
    for e in np.nonzero(qh | ql)[0]:
        Q += ((int(qh[e]) << 24) + int(ql[e])) << (2 * int(e) - 2)
    num = n * Q - S * S  # n^2 * 2^298 * var, exact
    assert num >= 0
    out["mean"] = S / (n << 149)
    out["m2"] = num / (n << 298)
    out["std"] = math.sqrt(num / ((n * n) << 298))
    return out


def _acc1_moments(a: "_Acc1") -> dict:
    return exact_moments(a.n, a.nan, a.pinf, a.minf, a.kmin, a.kmax, np.ctypeslib.as_array(a.s),
                         np.ctypeslib.as_array(a.qh), np.ctypeslib.as_array(a.ql))


def _pass2_args(mo: dict, nbins: int, a1: "_Acc1"):
    """Histogram range (the values' own [min, max]) and the median's top-16 bucket."""
    lib = _load()
    p = _Pass2()
    p.nbins = nbins
    p.hist_on = 0
    if mo["count"] > 0:
        lo, hi = np.float32(mo["min"]), np.float32(mo["max"])
        sc = ctypes.c_float()
        if lib.oracle_hist_scale(float(lo), float(hi), nbins, ctypes.byref(sc)) == 0:
            p.lo, p.hi, p.scale, p.hist_on = float(lo), float(hi), sc.value, 1
        k = (mo["count"] - 1) // 2
        cum = ctypes.c_uint64()
        top = lib.oracle_rank_bin(ctypes.addressof(a1.top), 65536, k, ctypes.byref(cum))
        assert top >= 0
        p.sel, p.sel_on = top, 1
        return p, k - cum.value
    return p, 0


def _finish(mo: dict, p: "_Pass2", k_low: int, a2: "_Acc2", counts: np.ndarray) -> dict:
    lib = _load()
    out = dict(mo)
    nb = len(counts)
    if p.hist_on:
        out["counts"] = counts
        out["outliers"] = np.array([a2.below, a2.above], dtype=np.uint64)
        out["hist_skipped"] = False
    else:
        out["counts"] = np.zeros(nb, dtype=np.uint64)
        out["outliers"] = np.zeros(2, dtype=np.uint64)
        out["hist_skipped"] = True
    if mo["count"] == 0:
        out["median"] = float("nan")
    else:
        cum = ctypes.c_uint64()
        low = lib.oracle_rank_bin(ctypes.addressof(a2.low), 65536, k_low, ctypes.byref(cum))
        assert low >= 0
        out["median"] = value_of_key((p.sel << 16) | low)
    return out


def stats_exact(a: np.ndarray, nbins: int, region=None, threads=None) -> dict:
    """``stats`` of one array or region by the large-input method (threaded
    over the values when region is None).  Same keys as ``stats``."""
    lib = _load()
    a, dt, nx, ny, nz = _cube(a)
    b, bp = _box(region)
    T = _threads(threads)
    a1 = _Acc1()
    lib.oracle_acc1_init(ctypes.byref(a1))
    if bp is None:
        if lib.oracle_pass1_array(a.ctypes.data, dt, a.size, T, ctypes.byref(a1)) != 0:
            raise ValueError("bad arguments")
    elif lib.oracle_acc1_box(a.ctypes.data, dt, nx, ny, nz, bp, ctypes.byref(a1)) != 0:
        raise ValueError("invalid region or dtype")
    mo = _acc1_moments(a1)
    p, k_low = _pass2_args(mo, nbins, a1)
    a2 = _Acc2()
    counts = np.zeros(nbins, dtype=np.uint64)
    if mo["count"] > 0:
        if bp is None:
            lib.oracle_pass2_array(a.ctypes.data, dt, a.size, T, ctypes.byref(p), ctypes.byref(a2), counts.ctypes.data)
        else:
            lib.oracle_acc2_box(a.ctypes.data, dt, nx, ny, nz, bp, ctypes.byref(p), ctypes.byref(a2),
                                counts.ctypes.data)
    return _finish(mo, p, k_low, a2, counts)


def stats_boxes(a: np.ndarray, boxes, nbins: int, threads=None, chunk: int = 8192):
    """``stats`` of every box of a batch (boxes int64[nq, 6], half-open), boxes
    spread over host threads.  Returns (list of dicts without the histogram,
    counts uint64[nq, nbins]); a bad box has status -1 in its dict."""
    lib = _load()
    a, dt, nx, ny, nz = _cube(a)
    boxes = np.ascontiguousarray(np.asarray(boxes, dtype=np.int64).reshape(-1, 6))
    nq = len(boxes)
    T = _threads(threads)
    counts = np.zeros((nq, nbins), dtype=np.uint64)
    res = []
    for q0 in range(0, nq, chunk):
        q1 = min(nq, q0 + chunk)
        m = q1 - q0
        out = np.zeros(m, dtype=BOX_OUT_DTYPE)
        s = np.zeros((m, 256), dtype=np.int64)
        qh = np.zeros((m, 256), dtype=np.uint64)
        ql = np.zeros((m, 256), dtype=np.uint64)
        cview = counts[q0:q1]
        if lib.oracle_boxes(a.ctypes.data, dt, nx, ny, nz, boxes[q0:q1].ctypes.data, m, nbins, T, out.ctypes.data,
                            s.ctypes.data, qh.ctypes.data, ql.ctypes.data, cview.ctypes.data) != 0:
            raise ValueError("bad arguments")
        for i in range(m):
            o = out[i]
            if o["status"] != 0:
                res.append({"status": int(o["status"])})
                continue
            d = exact_moments(o["n"], o["nan"], o["pinf"], o["minf"], o["kmin"], o["kmax"], s[i], qh[i], ql[i])
            d["status"] = 0
            d["hist_skipped"] = not bool(o["hist_on"])
            d["median"] = value_of_key(o["median_key"]) if o["n"] > 0 else float("nan")
            res.append(d)
    return res, counts


def stats_streaming(spec, nbins: int, threads=None, slab_voxels: int = 1 << 28, on_slab=None, log=None) -> dict:
    """``stats`` of a whole synthetic cube (synth.CubeSpec) that need not fit
    in memory: pass 1 regenerates it in z-slabs of about slab_voxels voxels
    and counts, pass 2 regenerates it again for the histogram and the
    median's low key bits.  on_slab(z0, z1, array) sees every slab of pass 1
    (the same bytes the generator gives any caller); log(str) reports
    progress.  Also returns the generator's NaN count as "generator_nan"."""
    import synth

    lib = _load()
    T = _threads(threads)
    dt = F32 if spec.dtype == "f32" else I16
    planes = max(1, slab_voxels // (spec.nx * spec.ny))
    a1 = _Acc1()
    lib.oracle_acc1_init(ctypes.byref(a1))
    gen_nan = 0
    slabs = list(range(0, spec.nz, planes))
    for i, z0 in enumerate(slabs):
        z1 = min(spec.nz, z0 + planes)
        arr, nn = synth.generate(spec, z0, z1, threads=T)
        gen_nan += nn
        if on_slab is not None:
            on_slab(z0, z1, arr)
        lib.oracle_pass1_array(arr.ctypes.data, dt, arr.size, T, ctypes.byref(a1))
        if log and (i % 8 == 7 or i == len(slabs) - 1):
            log(f"oracle pass 1: slab {i + 1}/{len(slabs)}")
        del arr
    mo = _acc1_moments(a1)
    p, k_low = _pass2_args(mo, nbins, a1)
    a2 = _Acc2()
    counts = np.zeros(nbins, dtype=np.uint64)
    if mo["count"] > 0:
        for i, z0 in enumerate(slabs):
            z1 = min(spec.nz, z0 + planes)
            arr, _ = synth.generate(spec, z0, z1, threads=T)
            lib.oracle_pass2_array(arr.ctypes.data, dt, arr.size, T, ctypes.byref(p), ctypes.byref(a2),
                                   counts.ctypes.data)
            if log and (i % 8 == 7 or i == len(slabs) - 1):
                log(f"oracle pass 2: slab {i + 1}/{len(slabs)}")
            del arr
    out = _finish(mo, p, k_low, a2, counts)
    out["generator_nan"] = gen_nan
    return out
