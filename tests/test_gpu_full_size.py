"""Full-size workloads in the launch configuration the benchmark times, checked
on sampled outputs the oracle computes one by one."""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_hist, check_median, check_moments

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
