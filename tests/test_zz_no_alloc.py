"""tsa_stats_static (the fused trio on the library's fixed per-device scratch,
for callers that cannot allocate) against tsa_stats with a caller workspace,
through the C ABI: two calls in a row, the second on a smaller input, every
output bit for bit; then a median bucket larger than the fixed scratch's
candidate list (a third pass there, compaction in tsa_stats)."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1211_4896_amd as tsa  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bufs(dev, nbins):
    out = torch.full((72,), 0xA5, dtype=torch.uint8, device=dev.device)
    counts = torch.full((nbins,), 7, dtype=torch.int64, device=dev.device)
    outl = torch.full((2,), 7, dtype=torch.int64, device=dev.device)
    return out, counts, outl


def _both(dev, nbins, region=None):
    """(workspace call, static call) outputs as host bytes."""
    api = tsa.capi()
    c = tsa.cube_of(dev)
    reg = tsa.region_of(region)
    rp = ctypes.byref(reg) if reg is not None else None
    sh = torch.cuda.current_stream().cuda_stream
    ws = tsa.workspace(tsa.OP_STATS, dev, region, nbins)
    o1, c1, l1 = _bufs(dev, nbins)
    st = api.tsa_stats(ctypes.byref(c), rp, nbins, o1.data_ptr(), c1.data_ptr(), l1.data_ptr(), ws.data_ptr(),
                       ws.numel(), sh)
    assert st == tsa.TSA_OK, tsa.status_string(st)
    o2, c2, l2 = _bufs(dev, nbins)
    st = api.tsa_stats_static(ctypes.byref(c), rp, nbins, o2.data_ptr(), c2.data_ptr(), l2.data_ptr(), sh)
    assert st == tsa.TSA_OK, tsa.status_string(st)
    torch.cuda.synchronize()
    return [(o1.cpu().numpy(), c1.cpu().numpy(), l1.cpu().numpy()),
            (o2.cpu().numpy(), c2.cpu().numpy(), l2.cpu().numpy())]


def _same(a, b, what):
    (o1, c1, l1), (o2, c2, l2) = a, b
    r1, r2 = tsa.results_to_numpy(torch.from_numpy(o1))[0], tsa.results_to_numpy(torch.from_numpy(o2))[0]
    assert r1["status"] == 0 and r2["status"] == 0, (what, r1, r2)
    assert o1.tobytes() == o2.tobytes(), (what, r1, r2)
    assert np.array_equal(c1, c2), what
    assert np.array_equal(l1, l2), what


def test_static_scratch_matches_workspace_call_twice():
    api = tsa.capi()
    assert api.tsa_stats_static_scratch_bytes() == 8 << 20
    keys = api.tsa_stats_static_candidate_keys()
    assert 1 << 20 < keys < (8 << 20) // 4
    big = synth.scaled(synth.SPECS["c1"], 256, 256, 160)
    host, _ = synth.generate(big)
    dev = torch.from_numpy(host).to("cuda:0")
    _say("case static: 256x256x160, 1024 bins")
    a, b = _both(dev, 1024)
    _same(a, b, "256x256x160")
    small = synth.scaled(synth.SPECS["c1"], 96, 64, 40)
    host2, _ = synth.generate(small)
    dev2 = torch.from_numpy(host2).to("cuda:0")
    _say("case static: 96x64x40, 256 bins (second, smaller call)")
    a, b = _both(dev2, 256)
    _same(a, b, "96x64x40")
    _say("case static: region of the first cube, 4096 bins")
    a, b = _both(dev, 4096, (3, 5, 7, 201, 250, 99))
    _same(a, b, "region")


def test_static_scratch_third_pass_bucket():
    """Three values only, 2^27 + 4099 voxels: the median's last bucket holds
    about 4.5e7 keys, far beyond the fixed list; the workspace call, with
    2^21 candidate slots, also takes the third pass.  Then 1.9e6 keys in a
    smaller cube: above the fixed list, within the workspace call's."""
    keys = tsa.capi().tsa_stats_static_candidate_keys()
    rng = np.random.default_rng(11)
    n = (1 << 27) + 4099
    host = rng.integers(0, 3, size=n, dtype=np.int8).astype(np.float32)
    host[::1001] = np.nan
    dev = torch.from_numpy(host).to("cuda:0").reshape(1, 1, n)
    _say("case static: 3 values,", n, "voxels")
    a, b = _both(dev, 64)
    _same(a, b, "three values")
    del dev
    # 150M voxels, a run of keys + 1 ties at the median surrounded by distinct values
    n2 = 150_000_001
    m = keys + 4096
    vals = np.empty(n2, dtype=np.float32)
    lo = (n2 - m) // 2
    vals[:lo] = np.linspace(-1000.0, -1.0, lo, dtype=np.float32)
    vals[lo:lo + m] = 0.5
    vals[lo + m:] = np.linspace(1.0, 1000.0, n2 - lo - m, dtype=np.float32)
    rng.shuffle(vals)
    dev = torch.from_numpy(vals).to("cuda:0").reshape(1, 1, n2)
    _say("case static: bucket of", m, "ties in", n2, "voxels")
    a, b = _both(dev, 256)
    _same(a, b, "tie bucket")
    r = tsa.results_to_numpy(torch.from_numpy(b[0]))[0]
    assert r["median"] == 0.5
