"""Full-size workloads in the launch configuration the benchmark times, checked
on sampled outputs the oracle computes one by one."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_hist, check_median, check_moments, check_sigma_counts

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
import paper_1211_4896_amd as tsa  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_c4_region_batch_sampled():
    """4096 boxes on the resident 2048^3 cube (the benchmark's batch, default
    tuning): a spread of queries (largest, smallest, random) against the oracle."""
    spec = synth.SPECS["c4"]
    _say("case c4: generating 2048^3")
    host, _ = synth.generate(spec)
    dev = torch.from_numpy(host).to("cuda:0")
    boxes = synth.regions(4096, (spec.nx, spec.ny, spec.nz), seed=2024, edge_lo=8, edge_hi=512)
    _say("case c4: batch")
    res, hists = tsa.region_batch(dev, boxes, 256)
    hists = hists.cpu().numpy().view(np.uint64)
    vol = np.prod(boxes[:, 3:] - boxes[:, :3], axis=1)
    rng = np.random.default_rng(3)
    pick = sorted(set([int(np.argmax(vol)), int(np.argmin(vol))] + list(rng.choice(4096, 10, replace=False))))
    assert np.all(res["status"] == 0)
    for i in pick:
        b = tuple(int(v) for v in boxes[i])
        _say("case c4 query", i, b, int(vol[i]))
        want = oracle.stats(host, 256, b)
        r = {k: res[i][k].item() for k in res.dtype.names}
        check_moments(r, want, "f32", f"c4 q{i}")
        check_median(r["median"], want["median"], "f32", f"c4 q{i}")
        assert not want["hist_skipped"]
        check_hist(hists[i], None, want["counts"], None, f"c4 q{i}")


def test_c2_minimap_spectrum_rank_sampled():
    """The benchmark's other workloads on the resident 1024x1024x1280 cube, in
    the configuration it times: the 30^3 mini-map (52675 cells, 64 bins) and
    its 3-sigma counts, the spectrum tool's 16384 sight lines x 2560 samples,
    and the 0.9-quantile and MAD, checked on sampled outputs the oracle
    computes one by one (quantile and MAD in full)."""
    import bench
    spec = synth.SPECS["c2"]
    _say("case c2 (minimap/spectrum/rank): generating")
    host, _ = synth.generate(spec)
    dev = torch.from_numpy(host).to("cuda:0")
    dims = (spec.nx, spec.ny, spec.nz)
    cell, nbins, k = bench.MINIMAP_CELL, bench.MINIMAP_NBINS, bench.MINIMAP_K
    _say("case c2: minimap")
    res, hists, cells_dev = tsa.minimap(dev, cell, nbins)
    boxes = oracle.minimap_cells(dims, cell)
    assert len(res) == len(boxes) == 52675 and np.all(res["status"] == 0)
    rng = np.random.default_rng(5)
    pick = sorted(set([0, len(boxes) - 1, 34, 35 * 35 - 1] + list(rng.choice(len(boxes), 12, replace=False))))
    h = hists.cpu().numpy().view(np.uint64)
    for i in pick:
        b = tuple(int(v) for v in boxes[i])
        want = oracle.stats(host, nbins, b)
        r = {kk: res[i][kk].item() for kk in res.dtype.names}
        check_moments(r, want, "f32", f"c2 cell {i}")
        check_median(r["median"], want["median"], "f32", f"c2 cell {i}")
        if not want["hist_skipped"]:
            check_hist(h[i], None, want["counts"], None, f"c2 cell {i}")
    _say("case c2: 3-sigma counts")
    above = tsa.sigma_count(dev, cell, cells_dev, k)
    check_sigma_counts(host, above, cell, k, "c2 sigma", cells=pick)
    _say("case c2: spectrum")
    rays = synth.sight_lines(bench.SPECTRUM_RAYS, dims, bench.SPECTRUM_SEED)
    got = tsa.spectrum(dev, rays, bench.SPECTRUM_SAMPLES).cpu().numpy()
    rsel = sorted(set([0, len(rays) - 1] + list(rng.choice(len(rays), 14, replace=False))))
    want = oracle.spectrum(host, rays[rsel, :3], rays[rsel, 3:], bench.SPECTRUM_SAMPLES)
    g = got[rsel]
    assert np.array_equal(g, want, equal_nan=True), np.argwhere(~((g == want) | (np.isnan(g) & np.isnan(want))))[:5]
    _say("case c2: quantile and MAD")
    wq, n = oracle.quantile(host, 0.9)
    v, w, cnt = tsa.quantile(dev, 0.9)
    assert cnt == n and w == 0.0
    check_median(v, wq, "f32", "c2 q0.9")
    v2, w2, _ = tsa.quantile(dev, 0.9, digits=2)
    assert v2 <= wq <= v2 + w2
    m, mad, cnt = tsa.mad(dev)
    wm, wmad, wn = oracle.mad(host)
    assert cnt == wn
    check_median(m, wm, "f32", "c2 MAD median")
    check_median(mad, wmad, "f32", "c2 MAD")


@pytest.mark.skipif(os.environ.get("TSA_TEST_C3") != "1",
                    reason="206 GB cube, about a minute to generate: set TSA_TEST_C3=1 to run")
def test_c3_full_size_206gb():
    """The 4096x4096x3072 float32 cube (206 GB) resident on one GPU, 65536
    bins: whole-cube results checked by invariants that hold at any size
    (count + nan_count = N, the generator's NaN count, histogram total =
    count, extremes bound every slab's), and two z-slabs checked against the
    oracle on every output."""
    import bench
    spec = synth.SPECS["c3"]
    _say("case c3: generating on the device")
    dev, nan = bench.generate_on_device(synth, torch, spec)
    N = dev.numel()
    _say("case c3: gpu stats, 65536 bins")
    res, counts, outl = tsa.stats(dev, 65536)
    assert res["status"] == 0
    assert res["count"] + res["nan_count"] == N and res["nan_count"] == nan
    assert int(counts.sum().item()) == res["count"] and int(outl.sum().item()) == 0
    rng = np.random.default_rng(9)
    for z0 in sorted(rng.choice(spec.nz - 8, 2, replace=False)):
        z0 = int(z0)
        box = (0, 0, z0, spec.nx, spec.ny, z0 + 8)
        _say("case c3: slab", box)
        host, _ = synth.generate(spec, z0, z0 + 8)
        want = oracle.stats(host, 65536)
        got, c, o = tsa.stats(dev, 65536, box)
        check_moments(got, want, "f32", f"c3 slab {z0}")
        check_median(got["median"], want["median"], "f32", f"c3 slab {z0}")
        check_hist(c, o, want["counts"], want["outliers"], f"c3 slab {z0}")
        assert res["min"] <= want["min"] and want["max"] <= res["max"]
