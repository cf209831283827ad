"""Pins for the oracle's 3-D spectrum tool (Section 4.4): trilinear samples
along rays at a constant step."""
import math

import numpy as np
import pytest

import oracle


def _field(shape, f):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return f(x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))


def test_linear_field_is_reproduced():
    """Trilinear interpolation is exact on a linear field: a swapped weight,
    axis or corner fails here."""
    a = _field((9, 7, 11), lambda x, y, z: 0.5 + 2 * x - 3 * y + 0.25 * z).astype(np.float32)
    origins = np.array([[0.3, 0.1, 0.7], [10.0, 6.0, 8.0], [5.5, 0.0, 0.0], [0.0, 3.2, 1.1]])
    steps = np.array([[0.37, 0.21, 0.33], [-0.5, -0.25, -0.4], [0.0, 0.3, 0.41], [0.9, 0.0, 0.35]])
    got = oracle.spectrum(a, origins, steps, 40)
    for r in range(len(origins)):
        for i in range(40):
            x, y, z = (origins[r] + i * steps[r])
            inside = 0 <= x <= 10 and 0 <= y <= 6 and 0 <= z <= 8
            if not inside:
                assert math.isnan(got[r, i])
            else:
                assert abs(got[r, i] - (0.5 + 2 * x - 3 * y + 0.25 * z)) < 1e-12, (r, i)


def test_multilinear_field_is_reproduced():
    """x*y*z is trilinear inside every cell, so the interpolation reproduces
    it: this catches a weight paired with the wrong corner on any axis."""
    a = _field((6, 5, 7), lambda x, y, z: x * y * z + x * y - 2 * y * z + 3).astype(np.float32)
    rng = np.random.default_rng(1)
    origins = rng.uniform([0, 0, 0], [6, 4, 5], (20, 3))
    got = oracle.spectrum(a, origins, np.zeros((20, 3)), 1)[:, 0]
    x, y, z = origins.T
    assert np.allclose(got, x * y * z + x * y - 2 * y * z + 3, rtol=0, atol=1e-12)


def test_matches_scipy_linear_map_coordinates():
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(2)
    a = rng.standard_normal((8, 9, 10)).astype(np.float32)
    pts = rng.uniform([0, 0, 0], [9, 8, 7], (300, 3))
    got = oracle.spectrum(a, pts, np.zeros_like(pts), 1)[:, 0]
    want = map_coordinates(a.astype(np.float64), [pts[:, 2], pts[:, 1], pts[:, 0]], order=1, mode="nearest")
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_voxel_points_faces_and_outside():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((4, 5, 6)).astype(np.float32)
    # integer points give the voxel exactly, including the upper faces
    got = oracle.spectrum(a, [[0, 0, 0]], [[1, 1, 1]], 6)[0]
    assert [got[i] for i in range(4)] == [float(a[i, i, i]) for i in range(4)]
    assert math.isnan(got[4]) and math.isnan(got[5])
    face = oracle.spectrum(a, [[5.0, 4.0, 3.0]], [[0, 0, 0]], 1)[0, 0]
    assert face == float(a[3, 4, 5])
    # just outside along each axis
    for p in ([-1e-9, 1, 1], [5 + 1e-9, 1, 1], [1, -1e-9, 1], [1, 4.0000001, 1], [1, 1, 3.0000001]):
        assert math.isnan(oracle.spectrum(a, [p], [[0, 0, 0]], 1)[0, 0])
    # an axis of one voxel: only coordinate 0 is inside
    b = rng.standard_normal((1, 3, 4)).astype(np.float32)
    assert oracle.spectrum(b, [[1.5, 2.0, 0.0]], [[0, 0, 0]], 1)[0, 0] == pytest.approx(
        0.5 * float(b[0, 2, 1]) + 0.5 * float(b[0, 2, 2]), abs=1e-15)
    assert math.isnan(oracle.spectrum(b, [[1.5, 2.0, 0.5]], [[0, 0, 0]], 1)[0, 0])
    # zero samples and no rays
    assert oracle.spectrum(a, [[0, 0, 0]], [[1, 0, 0]], 0).shape == (1, 0)
    assert oracle.spectrum(a, np.zeros((0, 3)), np.zeros((0, 3)), 5).shape == (0, 5)


def test_nan_corners():
    a = np.ones((5, 5, 5), np.float32)
    a[2, 2, 2] = np.nan
    got = oracle.spectrum(a, [[2.5, 2, 2], [3, 2, 2], [1, 2, 2], [2, 2, 2], [1.5, 1.5, 1.5], [0.5, 2.5, 3.5]],
                          np.zeros((6, 3)), 1)[:, 0]
    assert math.isnan(got[0])          # NaN corner with weight 1/2
    assert got[1] == 1.0               # a cell starting past it
    assert got[2] == 1.0               # the NaN voxel is a corner of weight 0
    assert math.isnan(got[3])          # the NaN voxel itself
    assert math.isnan(got[4])          # corner (2,2,2) of the cell [1,2]^3, weight 1/8
    assert got[5] == 1.0               # a cell that does not touch it


def test_int16_is_converted_exactly():
    a = np.array([[[-32768, 32767]]], dtype=np.int16)
    got = oracle.spectrum(a, [[0, 0, 0]], [[0.25, 0, 0]], 5)[0]
    assert list(got) == [-32768.0, -32768 + 0.25 * 65535, -0.5, -32768 + 0.75 * 65535, 32767.0]
