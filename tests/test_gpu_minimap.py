"""Statistical mini-map and local k-sigma counts (Section 4.5) against the oracle, per cell."""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_hist, check_median, check_moments, check_sigma_counts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1211_4896_amd as tsa  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _dtype(host):
    return "f32" if host.dtype == np.float32 else "i16"


def _check_cells(host, res, hists, cell, nbins, what):
    nz, ny, nx = host.shape
    boxes = oracle.minimap_cells((nx, ny, nz), cell)
    assert len(res) == len(boxes)
    h = hists.cpu().numpy().view(np.uint64)
    for i, b in enumerate(boxes):
        box = tuple(int(v) for v in b)
        want = oracle.stats(host, nbins, box)
        r = {k: res[i][k].item() for k in res.dtype.names}
        tag = f"{what} cell {i} {box}"
        check_moments(r, want, _dtype(host), tag)
        check_median(r["median"], want["median"], _dtype(host), tag)
        assert bool(r["flags"] & tsa.FLAG_HIST_SKIPPED) == want["hist_skipped"], tag
        if not want["hist_skipped"]:
            check_hist(h[i], None, want["counts"], None, tag)


def _check_sigma(host, got, cell, k, what):
    n_equal = check_sigma_counts(host, got, cell, k, what)
    # the bracket's centre is the oracle's own count
    assert n_equal == int(np.count_nonzero(got == oracle.sigma_counts(host, cell, k))), what
    return n_equal


def _run(host, cell, nbins, ks, what):
    dev = _dev(host)
    _say("case minimap", what, host.shape, cell, nbins)
    res, hists, cells_dev = tsa.minimap(dev, cell, nbins)
    _check_cells(host, res, hists, cell, nbins, what)
    for k in ks:
        _say("case sigma", what, k)
        got = tsa.sigma_count(dev, cell, cells_dev, k)
        _check_sigma(host, got, cell, k, what)
    return res, hists, cells_dev, dev


def test_minimap_f32_survey_cube():
    spec = synth.scaled(synth.SPECS["c3"], 128, 96, 70)  # sources + NaN slabs
    host, _ = synth.generate(spec)
    _run(host, (30, 30, 30), 64, (2.0, 3.0, 4.0, 7.0, 0.0, -1.5), "c3 30^3")


def test_minimap_ragged_cells_and_chunks():
    rng = np.random.default_rng(8)
    host = rng.standard_normal((9, 6, 4100)).astype(np.float32)  # two column chunks
    host[2, :, 100:300] = np.nan
    host[5, 3, 4097] = 40.0
    _run(host, (513, 4, 5), 32, (3.0, -0.5), "wide rows")
    _run(host, (4100, 6, 9), 16, (1.0,), "one cell")


def test_minimap_register_sizes():
    """Cells filling each register layout of the 768-lane workgroup: up to 16, 32, 36,
    40, 48 and 64 values per lane (16^3, 32x16x30, 30^3, 32x16x60, 32^3, 32x32x48),
    plus a one-plane cell and a 40x25x20 cell."""
    rng = np.random.default_rng(13)
    host = (rng.standard_normal((64, 60, 100)) * 3 + 1).astype(np.float32)
    host[10, 5:9, :] = np.nan
    for cell in ((16, 16, 16), (32, 16, 30), (30, 30, 30), (32, 16, 60), (32, 32, 32), (32, 32, 48), (100, 60, 1),
                 (40, 25, 20)):
        _run(host, cell, 16, (2.0,), f"cells {cell}")


def test_minimap_scalar_path_unaligned_rows():
    rng = np.random.default_rng(9)
    host = (rng.standard_normal((11, 13, 203)) * 5 + 2).astype(np.float32)  # nx % 4 != 0
    host[4:6] = np.nan
    _run(host, (7, 5, 3), 8, (2.0, 0.0), "scalar")


def test_minimap_int16():
    spec = synth.scaled(synth.SPECS["c5c"], 160, 48, 40)
    host, _ = synth.generate(spec)
    _run(host, (32, 16, 10), 128, (3.0, 1.0, -2.0), "i16 vec")
    _run(np.ascontiguousarray(host[:, :, :157]), (30, 7, 11), 16, (2.5,), "i16 scalar")


def test_minimap_degenerate_cells_and_ties():
    rng = np.random.default_rng(10)
    host = rng.integers(-2, 3, (8, 10, 12)).astype(np.float32)
    host[0] = 5.0          # constant plane: std 0
    host[1, :5, :] = np.nan  # cells that are all NaN
    host[2, :5, :] = np.inf  # constant +inf cells: no histogram
    host[3, 5:, :] = -np.inf
    # signed zeros and denormals: the first-digit bucket's float bounds meet at
    # zero, where the key (-0 < +0) decides; small buckets are ranked by counting
    host[4] = rng.choice(np.array([-0.0, 0.0, 1e-40, -1e-40, 3e-39], dtype=np.float32), (10, 12))
    _run(host, (12, 5, 1), 8, (0.0, 1.0, -1.0), "planes")
    _run(host, (1, 1, 8), 4, (0.5,), "columns")


def test_minimap_deterministic_and_bad_arguments():
    spec = synth.scaled(synth.SPECS["c1"], 96, 64, 48)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    _say("case minimap determinism")
    r1, h1, c1 = tsa.minimap(dev, (16, 16, 16), 32)
    r2, h2, _ = tsa.minimap(dev, (16, 16, 16), 32)
    assert r1.tobytes() == r2.tobytes() and torch.equal(h1, h2)
    a1 = tsa.sigma_count(dev, (16, 16, 16), c1, 3.0)
    a2 = tsa.sigma_count(dev, (16, 16, 16), c1, 3.0)
    assert np.array_equal(a1, a2)
    with pytest.raises(tsa.TsaError):
        tsa.minimap(dev, (1, 1, 1), 32)  # 294912 cells
    with pytest.raises(tsa.TsaError):
        tsa.minimap(dev, (0, 16, 16), 32)
    with pytest.raises(tsa.TsaError):
        tsa.sigma_count(dev, (16, 16, 16), c1, float("inf"))
