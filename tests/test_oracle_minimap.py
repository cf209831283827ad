"""Pins for the oracle's mini-map cells and local k-sigma counts (Section 4.5)."""
import numpy as np

import oracle


def test_cells_tile_the_cube_exactly_once():
    dims = (17, 9, 13)
    boxes = oracle.minimap_cells(dims, (5, 4, 13))
    cover = np.zeros(dims[::-1], dtype=np.int32)
    for x0, y0, z0, x1, y1, z1 in boxes:
        cover[z0:z1, y0:y1, x0:x1] += 1
    assert np.all(cover == 1)
    assert len(boxes) == 4 * 3 * 1
    assert tuple(boxes[0]) == (0, 0, 0, 5, 4, 13) and tuple(boxes[-1]) == (15, 8, 0, 17, 9, 13)


def test_sigma_counts_brute_force():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((6, 7, 8)).astype(np.float32)
    a[1, 2, 3] = np.nan
    a[4, 4, 4] = 50.0
    for k in (-1.0, 0.0, 1.5, 3.0):
        got = oracle.sigma_counts(a, (3, 4, 5), k)
        boxes = oracle.minimap_cells((8, 7, 6), (3, 4, 5))
        for i, (x0, y0, z0, x1, y1, z1) in enumerate(boxes):
            vals = [float(a[z, y, x]) for z in range(z0, z1) for y in range(y0, y1) for x in range(x0, x1)
                    if a[z, y, x] == a[z, y, x]]
            n = len(vals)
            mean = sum(vals) / n
            std = (sum((v - mean) ** 2 for v in vals) / n) ** 0.5
            want = sum(1 for v in vals if v > mean + k * std)
            assert got[i] == want, (k, i)


def test_sigma_counts_limits():
    a = np.arange(64, dtype=np.float32).reshape(4, 4, 4)
    assert oracle.sigma_counts(a, (4, 4, 4), 1e9).sum() == 0
    assert oracle.sigma_counts(a, (4, 4, 4), -1e9).sum() == 64
    # a constant cell: std 0, nothing strictly above its mean
    assert oracle.sigma_counts(np.ones((2, 2, 2), np.float32), (2, 2, 2), 0.0).sum() == 0
    allnan = np.full((2, 2, 2), np.nan, np.float32)
    assert oracle.sigma_counts(allnan, (1, 1, 1), 0.0).sum() == 0
