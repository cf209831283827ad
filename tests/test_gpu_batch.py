"""Batched region queries (one persistent kernel) against the CPU oracle, per query."""
import ctypes
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_hist, check_median, check_moments

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1211_4896_amd as tsa  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _boxes(dims, nq, seed, lo=1, hi=64):
    r = synth.regions(nq, dims, seed, edge_lo=lo, edge_hi=hi)
    nx, ny, nz = dims
    extra = np.array([
        [0, 0, 0, nx, ny, nz],          # whole cube
        [3, 4, 5, 4, 5, 6],             # single voxel
        [1, 0, 0, 4, ny, nz],           # narrow, unaligned
        [0, 2, 2, nx, 3, 9],            # full rows
        [nx - 5, ny - 1, nz - 1, nx, ny, nz],
    ], dtype=np.int64)
    return np.concatenate([r, extra])


def _check_batch(host, dev, boxes, nbins, dtype="f32", tune=None, what=""):
    res, hists = tsa.region_batch(dev, boxes, nbins, tune=tune)
    hists = hists.cpu().numpy().view(np.uint64)
    for i, b in enumerate(boxes):
        r = {k: res[i][k].item() for k in res.dtype.names}
        want = oracle.stats(host, nbins, tuple(int(v) for v in b))
        tag = f"{what} q{i} {tuple(int(v) for v in b)}"
        check_moments(r, want, dtype, tag)
        check_median(r["median"], want["median"], dtype, tag)
        assert bool(r["flags"] & tsa.FLAG_HIST_SKIPPED) == want["hist_skipped"], tag
        if not want["hist_skipped"]:
            check_hist(hists[i], None, want["counts"], None, tag)
    return res, hists


@pytest.mark.parametrize("seed", [1, 2])
def test_batch_matches_oracle(seed):
    spec = synth.scaled(synth.SPECS["c1"], 128, 96, 80)
    spec = synth.CubeSpec(**{**spec.__dict__, "seed": 100 + seed})
    host, _ = synth.generate(spec)
    dev = _dev(host)
    boxes = _boxes((128, 96, 80), 200, seed)
    _say("case batch f32", seed, len(boxes))
    _check_batch(host, dev, boxes, 64, what="f32")


def test_batch_invalid_boxes_flagged():
    host = np.random.default_rng(0).standard_normal((8, 9, 12)).astype(np.float32)
    dev = _dev(host)
    boxes = np.array([[0, 0, 0, 12, 9, 8], [0, 0, 0, 13, 1, 1], [2, 2, 2, 2, 3, 3], [-1, 0, 0, 1, 1, 1],
                      [1, 1, 1, 5, 5, 5]], dtype=np.int64)
    _say("case batch invalid boxes")
    res, hists = tsa.region_batch(dev, boxes, 16)
    for i in (1, 2, 3):
        assert res[i]["status"] == tsa.TSA_EINVAL and res[i]["flags"] & tsa.FLAG_BAD_REGION
    for i in (0, 4):
        b = tuple(int(v) for v in boxes[i])
        want = oracle.stats(host, 16, b)
        check_moments({k: res[i][k].item() for k in res.dtype.names}, want, "f32", f"valid {b}")
        check_median(res[i]["median"], want["median"], "f32", f"valid {b}")


def test_batch_phase3_and_small_tiles():
    """cand_max = 0 disables the candidate copy: every median takes the third
    (data) pass.  Tiny tiles give many tiles per box."""
    spec = synth.scaled(synth.SPECS["c1"], 96, 64, 48)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    boxes = _boxes((96, 64, 48), 60, 7, lo=2, hi=48)
    _say("case batch phase3")
    res, _ = _check_batch(host, dev, boxes, 32, tune=(1024, 256, 2, 0), what="phase3")
    assert any(r["flags"] & tsa.FLAG_PHASE3 for r in res)
    _say("case batch small tiles")
    _check_batch(host, dev, boxes, 32, tune=(1024, 256, 8, 65536), what="small tiles")


def test_batch_int16():
    spec = synth.scaled(synth.SPECS["c5c"], 128, 64, 40)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    boxes = _boxes((128, 64, 40), 80, 3)
    _say("case batch int16")
    _check_batch(host, dev, boxes, 128, dtype="i16", what="i16")


def test_batch_adversarial_cube():
    rng = np.random.default_rng(11)
    host = rng.integers(-2, 3, (16, 24, 40)).astype(np.float32)  # heavy ties
    host[3:5] = np.nan  # NaN slab
    host[10, :, :] = 7.0  # constant plane
    host[12, 5, 5] = -0.0
    host[14, 0:2, :] = np.inf   # constant +inf rows
    host[14, 2:4, :] = -np.inf  # constant -inf rows
    dev = _dev(host)
    boxes = np.array([[0, 0, 3, 40, 24, 5],      # all NaN
                      [0, 0, 10, 40, 24, 11],    # constant
                      [0, 0, 0, 40, 24, 16],     # everything
                      [5, 5, 12, 6, 6, 13],      # a single -0
                      [1, 2, 2, 39, 22, 14],
                      [0, 0, 14, 40, 2, 15],     # constant +inf: no histogram
                      [3, 2, 14, 9, 4, 15],      # constant -inf: no histogram
                      [0, 1, 14, 40, 3, 15]], dtype=np.int64)  # +inf and -inf
    _say("case batch adversarial")
    _check_batch(host, dev, boxes, 8, what="adv")


def test_batch_deterministic_and_equal_to_single_calls():
    spec = synth.scaled(synth.SPECS["c1"], 128, 128, 64)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    boxes = _boxes((128, 128, 64), 100, 5)
    _say("case batch determinism")
    r1, h1 = tsa.region_batch(dev, boxes, 256)
    r2, h2 = tsa.region_batch(dev, boxes, 256)
    assert r1.tobytes() == r2.tobytes() and torch.equal(h1, h2)
    for i in range(0, len(boxes), 7):
        b = tuple(int(v) for v in boxes[i])
        one, c, _ = tsa.stats(dev, 256, b)
        assert one["count"] == r1[i]["count"]
        check_median(one["median"], r1[i]["median"], "f32", f"single {b}")
        assert np.array_equal(c.cpu().numpy(), h1[i].cpu().numpy())
        assert math.isclose(one["mean"], r1[i]["mean"], rel_tol=1e-12, abs_tol=1e-14)


def test_batch_graph_replays_match_eager_inputs():
    """tsa_region_batch replays a captured launch graph for a repeated argument
    set.  Replays with eager work between them, and with the box array's
    contents changed in place, must give the same answers as fresh inputs."""
    spec = synth.scaled(synth.SPECS["c1"], 96, 96, 64)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    nq, nbins = 64, 32
    boxes_a = _boxes((96, 96, 64), nq - 5, 21)
    boxes_b = _boxes((96, 96, 64), nq - 5, 22)
    d_boxes = torch.from_numpy(boxes_a).to("cuda:0")
    ws = tsa.workspace(tsa.OP_REGION_BATCH, dev, None, nbins, nq)
    out = torch.empty(72 * nq, dtype=torch.uint8, device="cuda:0")
    hists = torch.empty((nq, nbins), dtype=torch.int64, device="cuda:0")
    api = tsa.capi()
    import ctypes
    c = tsa.cube_of(dev)

    def call():
        st = api.tsa_region_batch(ctypes.byref(c), d_boxes.data_ptr(), nq, nbins, out.data_ptr(), hists.data_ptr(),
                                  None, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
        assert st == 0
        torch.cuda.synchronize()
        return tsa.results_to_numpy(out).copy(), hists.clone()

    _say("case batch graph replays")
    ref_a = call()  # captured here
    for rep in range(4):
        tsa.stats(dev, 128)  # eager work between replays
        d_boxes.copy_(torch.from_numpy(boxes_b if rep % 2 == 0 else boxes_a))
        got = call()
        want_boxes = boxes_b if rep % 2 == 0 else boxes_a
        if rep % 2 == 1:
            assert got[0].tobytes() == ref_a[0].tobytes() and torch.equal(got[1], ref_a[1])
        for i in range(0, nq, 9):
            b = tuple(int(v) for v in want_boxes[i])
            want = oracle.stats(host, nbins, b)
            r = {k: got[0][i][k].item() for k in got[0].dtype.names}
            check_moments(r, want, "f32", f"replay {rep} q{i}")
            check_median(r["median"], want["median"], "f32", f"replay {rep} q{i}")
            check_hist(got[1][i].cpu().numpy().view(np.uint64), None, want["counts"], None, f"replay {rep} q{i}")


def test_autotuner_choice_is_used_and_correct():
    spec = synth.scaled(synth.SPECS["c1"], 128, 96, 64)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    boxes = _boxes((128, 96, 64), 123, 31, lo=4, hi=96)
    _say("case batch autotuner")
    best, ms = tsa.tune_region_batch(dev, boxes, 64, reps=1)
    assert best[0] in (0, 65536, 262144, 1048576) and best[2] in (2, 4, 6, 8) and ms > 0
    assert best[3] in (65536, 262144, 1 << 20, 4 << 20) and best[4] in (0, 1, 2, 4, 8)
    # with tracing on, calls launch directly (no graph replay), so the launch
    # choices recorded are this call's: the remembered ones
    lib = tsa.capi().lib
    lib.tsa_trace_enable.argtypes = [ctypes.c_int32, ctypes.c_int32]
    assert lib.tsa_trace_enable(1, 64) == 0
    try:
        res, hists = _check_batch(host, dev, boxes, 64, what="tuned")  # tune=None: the remembered choice
        tiles, bpc, reps, cap = tsa.batch_last_config()
    finally:
        lib.tsa_trace_enable(0, 0)
    assert bpc == best[2] and cap == best[3], (best, tsa.batch_last_config())
    assert tiles == (best[0] // 4 if best[0] >= 1024 else 0)
    assert reps == (best[4] if best[4] else 4)  # 64 bins: 4 replicas by default
    # every replica count gives the same bits
    for r in (1, 2, 4, 8):
        got, gh = tsa.region_batch(dev, boxes, 64, tune=(best[0], 256, 4, best[3], r))
        assert got.tobytes() == res.tobytes() and np.array_equal(gh.cpu().numpy().view(np.uint64), hists), r


def test_replicas_reduced_to_fit_lds():
    """4096 bins x 8 replicas would not fit a block's LDS: the batch uses as
    many as fit (here one) and stays exact."""
    spec = synth.scaled(synth.SPECS["c1"], 64, 64, 32)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    boxes = _boxes((64, 64, 32), 20, 7, lo=4, hi=48)
    _say("case batch replicas 8 at 4096 bins")
    lib = tsa.capi().lib
    lib.tsa_trace_enable.argtypes = [ctypes.c_int32, ctypes.c_int32]
    assert lib.tsa_trace_enable(1, 64) == 0  # direct launches: the recorded choices are this call's
    try:
        _check_batch(host, dev, boxes, 4096, tune=(0, 256, 4, 1 << 20, 8), what="replicas 8")
        assert tsa.batch_last_config()[2] == 1
        _check_batch(host, dev, boxes, 256, tune=(0, 256, 4, 1 << 20, 8), what="replicas 8, 256 bins")
        assert tsa.batch_last_config()[2] == 8
    finally:
        lib.tsa_trace_enable(0, 0)
    with pytest.raises(tsa.TsaError):
        tsa.region_batch(dev, boxes, 64, tune=(0, 256, 4, 1 << 20, 3))


def test_batch_candidate_pool_fills_without_wrapping():
    """5000 boxes of 2^20 voxels whose values all fall into one first-digit key
    bucket ([1, 1.125): one exponent, top three significand bits zero), so each
    box asks the shared candidate pool for its whole volume: their requests sum
    past 2^32.  The pool hands out ranges only while they fit; the boxes that
    find it full take the third pass.  Every box against the oracle."""
    rng = np.random.default_rng(31)
    nx, ny, nz = 512, 512, 256
    top = np.nextafter(np.float32(1.125), np.float32(0.0))
    host = np.minimum(np.float32(1.0) + rng.random((nz, ny, nx), dtype=np.float32) * np.float32(0.125), top)
    host = host.astype(np.float32)
    nq = 5000
    e = np.array([128, 128, 64])
    o = np.stack([rng.integers(0, n - k + 1, nq) for n, k in zip((nx, ny, nz), e)], axis=1)
    boxes = np.concatenate([o, o + e], axis=1).astype(np.int64)
    _say("case pool: batch of", nq, "boxes of", int(np.prod(e)), "voxels")
    dev = _dev(host)
    res, hists = tsa.region_batch(dev, boxes, 64)
    hists = hists.cpu().numpy().view(np.uint64)
    assert np.all(res["status"] == 0), np.unique(res["status"])
    n3 = int(np.count_nonzero(res["flags"] & tsa.FLAG_PHASE3))
    _say("case pool: boxes that took the third pass:", n3)
    assert n3 > nq // 2  # the pool (16384 keys a box) holds fewer than 80 such boxes
    _say("case pool: oracle over every box")
    want, counts = oracle.stats_boxes(host, boxes, 64)
    for i in range(nq):
        r = {k: res[i][k].item() for k in res.dtype.names}
        check_moments(r, want[i], "f32", f"pool q{i}")
        check_median(r["median"], want[i]["median"], "f32", f"pool q{i}")
        check_hist(hists[i], None, counts[i], None, f"pool q{i}")


def _solo(box, tile_voxels):
    """True when the batch plans the box as one tile (float32, 16-byte rows):
    tile_voxels / 4 vectors per tile, whole rows of ceil(x1/4) - floor(x0/4)
    vectors each."""
    x0, y0, z0, x1, y1, z1 = (int(v) for v in box)
    vpr = -(-x1 // 4) - x0 // 4
    rpt = max(1, (tile_voxels // 4) // vpr)
    return (y1 - y0) * (z1 - z0) <= rpt


def test_batch_bounded_wait_gives_up_cleanly():
    """The persistent kernel's bounded waits, forced from the host to give up
    at their first poll: the kernel still exits, every box of several tiles
    that needed its second phase reports TSA_EDEVICE, boxes finished in their
    first phase (constant or all-NaN boxes) and one-tile boxes (finished whole
    by one block, no wait) keep their results, and the next batch on the same
    workspace is correct again."""
    spec = synth.scaled(synth.SPECS["c1"], 96, 64, 48)
    host, _ = synth.generate(spec)
    host[:8, :8, :16] = np.float32(2.5)  # a constant corner
    host[40:44, 0:4, 0:8] = np.nan       # an all-NaN corner
    boxes = _boxes((96, 64, 48), 60, seed=9, lo=2, hi=40)
    const_box = np.array([[0, 0, 0, 16, 8, 8], [0, 0, 40, 8, 4, 44]], dtype=np.int64)
    boxes = np.concatenate([boxes, const_box])
    tile = 1024
    solo = [_solo(b, tile) for b in boxes]
    assert 5 < sum(solo) < len(boxes) - 5
    dev = _dev(host)
    lib = tsa.capi().lib
    lib.tsa_internal_batch_wait_limit.argtypes = [ctypes.c_int32]
    lib.tsa_internal_batch_wait_limit(0)
    try:
        _say("case wait limit 0")
        res, _ = tsa.region_batch(dev, boxes, 32, tune=(tile, 256, 4, 1 << 20, 0))
    finally:
        lib.tsa_internal_batch_wait_limit(-1)
    for i, b in enumerate(boxes):
        want = oracle.stats(host, 32, tuple(int(v) for v in b))
        r = {k: res[i][k].item() for k in res.dtype.names}
        if solo[i] or want["count"] == 0 or np.float32(want["min"]).tobytes() == np.float32(want["max"]).tobytes():
            assert r["status"] == 0, (i, b, r)
            check_moments(r, want, "f32", f"wait q{i}")
            check_median(r["median"], want["median"], "f32", f"wait q{i}")
        else:
            assert r["status"] == tsa.TSA_EDEVICE, (i, b, r)
    _say("case wait limit restored")
    _check_batch(host, dev, boxes, 32, what="after wait limit")
