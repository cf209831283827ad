"""Full-size workloads in the launch configuration the benchmark times, checked
on sampled outputs the oracle computes one by one."""
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


def _check_box_results(res, hists, want, counts, what, idx=None):
    """GPU batch results against oracle.stats_boxes output, query by query."""
    idx = range(len(want)) if idx is None else idx
    for i in idx:
        w = want[i]
        r = {k: res[i][k].item() for k in res.dtype.names}
        check_moments(r, w, "f32", f"{what} q{i}")
        check_median(r["median"], w["median"], "f32", f"{what} q{i}")
        assert bool(r["flags"] & tsa.FLAG_HIST_SKIPPED) == w["hist_skipped"], (what, i)
        if not w["hist_skipped"]:
            check_hist(hists[i], None, counts[i], None, f"{what} q{i}")


def test_c4_region_batch_every_query():
    """4096 boxes on the resident 2048^3 cube (the benchmark's batch, default
    tuning), every query against the oracle."""
    spec = synth.SPECS["c4"]
    _say("case c4: generating 2048^3")
    host, _ = synth.generate(spec)
    dev = torch.from_numpy(host).to("cuda:0")
    boxes = synth.regions(4096, (spec.nx, spec.ny, spec.nz), seed=2024, edge_lo=8, edge_hi=512)
    _say("case c4: batch")
    res, hists = tsa.region_batch(dev, boxes, 256)
    hists = hists.cpu().numpy().view(np.uint64)
    assert np.all(res["status"] == 0)
    _say("case c4: oracle over every box")
    want, counts = oracle.stats_boxes(host, boxes, 256)
    _check_box_results(res, hists, want, counts, "c4")


def test_c2_minimap_spectrum_rank_sampled():
    """The benchmark's other workloads on the resident 1024x1024x1280 cube, in
    the configuration it times: the 30^3 mini-map (52675 cells, 64 bins, every
    cell against the oracle) and its 3-sigma counts (sampled cells), the
    spectrum tool's 16384 sight lines x 2560 samples (sampled rays), and the
    0.9-quantile and MAD in full."""
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
    pick = sorted(set([0, len(boxes) - 1, 34, 35 * 35 - 1] + list(rng.choice(len(boxes), 200, replace=False))))
    h = hists.cpu().numpy().view(np.uint64)
    _say("case c2: oracle over every cell")
    want, counts = oracle.stats_boxes(host, boxes, nbins)
    _check_box_results(res, h, want, counts, "c2 cell")
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


C3_HBM_BYTES = 210 * 10**9


@pytest.mark.timeout(1200)
def test_c3_full_size_206gb():
    """The 4096x4096x3072 float32 cube (206 GB) resident on one GPU, 65536
    bins, the benchmark's call: every output of the whole cube against the
    streaming oracle (the cube regenerated slab by slab on the host; pass 1
    uploads the same slabs to the device), plus one z-slab as a region."""
    torch.cuda.empty_cache()  # blocks the earlier cases left in torch's cache
    free, _ = torch.cuda.mem_get_info(0)
    if free < C3_HBM_BYTES:
        pytest.skip(f"needs {C3_HBM_BYTES / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")
    spec = synth.SPECS["c3"]
    dev = torch.empty((spec.nz, spec.ny, spec.nx), dtype=torch.float32, device="cuda:0")

    def upload(z0, z1, arr):
        dev[z0:z1].copy_(torch.from_numpy(arr))

    _say("case c3: oracle pass 1 uploads the cube slab by slab")
    want = oracle.stats_streaming(spec, 65536, on_slab=upload, log=_say)
    torch.cuda.synchronize()
    N = dev.numel()
    _say("case c3: gpu stats, 65536 bins")
    res, counts, outl = tsa.stats(dev, 65536)
    assert res["status"] == 0
    assert res["count"] + res["nan_count"] == N and res["nan_count"] == want["generator_nan"]
    check_moments(res, want, "f32", "c3")
    check_median(res["median"], want["median"], "f32", "c3")
    assert not want["hist_skipped"]
    check_hist(counts, outl, want["counts"], want["outliers"], "c3")
    _say("case c3: moments alone and the histogram alone")
    check_moments(tsa.moments(dev), want, "f32", "c3 tsa_moments")
    c, o = tsa.histogram(dev, want["min"], want["max"], 65536)
    check_hist(c, o, want["counts"], want["outliers"], "c3 tsa_histogram")
    z0 = 1531
    box = (0, 0, z0, spec.nx, spec.ny, z0 + 8)
    _say("case c3: slab", box)
    host, _ = synth.generate(spec, z0, z0 + 8)
    w = oracle.stats_exact(host, 65536)
    got, c, o = tsa.stats(dev, 65536, box)
    check_moments(got, w, "f32", f"c3 slab {z0}")
    check_median(got["median"], w["median"], "f32", f"c3 slab {z0}")
    check_hist(c, o, w["counts"], w["outliers"], f"c3 slab {z0}")
