"""GPU parity: every call of the C ABI against the CPU oracle on the same seeded inputs."""
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


def _dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _full_check(host, dev, nbins, region=None, dtype="f32", what="", moment_values=True):
    """moments, histogram over the oracle's [min, max], median, and the fused call."""
    want = oracle.stats(host, nbins, region)
    got = tsa.moments(dev, region)
    if moment_values:
        check_moments(got, want, dtype, what + " moments")  # one pass, lanes about their own shift
    else:
        check_moments({**got, "mean": want["mean"], "std": want["std"], "m2": want["m2"]}, want, dtype, what)
    if not want["hist_skipped"]:
        c, o = tsa.histogram(dev, want["min"], want["max"], nbins, region)
        check_hist(c, o, want["counts"], want["outliers"], what + " histogram")
    gm = tsa.median(dev, region)
    assert gm["count"] == want["count"] and gm["status"] == 0
    check_median(gm["median"], want["median"], dtype, what + " median")
    res, c, o = tsa.stats(dev, nbins, region)
    if moment_values:
        check_moments(res, want, dtype, what + " stats")  # two-pass M2: 1e-12 at any mean/std
    check_median(res["median"], want["median"], dtype, what + " stats median")
    assert bool(res["flags"] & tsa.FLAG_HIST_SKIPPED) == want["hist_skipped"], (what, res["flags"])
    if not want["hist_skipped"]:
        check_hist(c, o, want["counts"], want["outliers"], what + " stats histogram")


def test_c1_cube():
    spec = synth.SPECS["c1"]
    _say("case c1 256^3", spec)
    host, nan = synth.generate(spec)
    dev = _dev(host)
    _full_check(host, dev, 1024, what="c1")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_regions_on_small_cube(seed):
    spec = synth.scaled(synth.SPECS["c1"], 100, 72, 60)
    spec = synth.CubeSpec(**{**spec.__dict__, "seed": seed})
    host, _ = synth.generate(spec)
    dev = _dev(host)
    rng = np.random.default_rng(seed)
    boxes = [
        (0, 0, 0, 100, 72, 60),  # whole cube as a region
        (0, 0, 5, 100, 72, 17),  # whole planes (contiguous)
        (0, 9, 3, 100, 10, 4),  # one full row
        (3, 9, 3, 97, 10, 4),  # part of one row (contiguous, unaligned)
        (1, 2, 3, 4, 5, 6),  # 3 wide: first and last vector coincide
        (5, 0, 0, 6, 72, 60),  # 1 wide
        (7, 7, 7, 8, 8, 8),  # single voxel
        (2, 1, 1, 99, 71, 59),  # unaligned both ends
        (4, 4, 4, 8, 8, 8),  # aligned, one vector per row
        (0, 0, 0, 100, 1, 60),  # full rows, one y, many z
    ]
    for _ in range(10):
        e = rng.integers(1, [101, 73, 61])
        o = [rng.integers(0, n - k + 1) for n, k in zip((100, 72, 60), e)]
        boxes.append((o[0], o[1], o[2], o[0] + e[0], o[1] + e[1], o[2] + e[2]))
    for b in boxes:
        _say("case region", seed, b)
        _full_check(host, dev, 64, region=b, what=f"region {b}")


def _adversarial_cubes():
    rng = np.random.default_rng(42)
    n = 4096
    cubes = {
        "constant": np.full(n, 3.25, np.float32),
        "all_nan": np.full(n, np.nan, np.float32),
        "single": np.float32([7.5]),
        "two": np.float32([2.0, -1.0]),
        "ramp": np.arange(n, dtype=np.float32) * np.float32(0.5) - np.float32(100.0),
        "signed_zeros": rng.choice(np.float32([0.0, -0.0]), n).astype(np.float32),
        "zeros_around_median": np.concatenate([np.full(100, -1.0), np.full(50, -0.0), np.full(50, 0.0),
                                               np.full(100, 1.0)]).astype(np.float32),
        "denormals": (rng.integers(-50, 50, n) * np.float32(1e-45)).astype(np.float32),
        "with_inf": np.concatenate([rng.standard_normal(n - 3), [np.inf, -np.inf, np.nan]]).astype(np.float32),
        "heavy_ties": rng.integers(-3, 4, n).astype(np.float32),
        "one_hot_bin": np.concatenate([np.full(n - 2, 1.0), [0.0, 1000.0]]).astype(np.float32),
        "huge_range": np.float32([-3.0e38, 3.0e38, 0.0, 1.0, -1.0]),
        "nan_mixed": np.where(rng.random(n) < 0.3, np.nan, rng.standard_normal(n)).astype(np.float32),
        "odd_length": rng.standard_normal(4097).astype(np.float32),
        "large_mean": (1000.0 + rng.standard_normal(n)).astype(np.float32),
        # mean/std of 1e3, 1e5 and 1e7 (float32 spacing at 1e5 is 2^-7): the
        # one-pass moments keep 1e-12 at any ratio
        "mean_1e3_big": (1000.0 + rng.standard_normal(1 << 20)).astype(np.float32),
        "mean_1e5": (1.0e5 + rng.standard_normal(n)).astype(np.float32),
        "mean_m1e5_big": (-1.0e5 + rng.standard_normal(1 << 20)).astype(np.float32),
        "mean_1e7_ratio": (1.0e5 + 0.01 * rng.standard_normal(n)).astype(np.float32),
        # an offset cube with rare far outliers (some lanes' first values lie far out)
        "offset_outliers": np.where(rng.random(1 << 20) < 0.01, 1500.0,
                                    1000.0 + rng.standard_normal(1 << 20)).astype(np.float32),
        "only_pos_inf_and_values": np.concatenate([rng.standard_normal(n), np.full(7, np.inf)]).astype(np.float32),
        "all_pos_inf": np.full(n, np.inf, np.float32),
    }
    return cubes


@pytest.mark.parametrize("name", list(_adversarial_cubes().keys()))
def test_adversarial(name):
    host = _adversarial_cubes()[name]
    _say("case adversarial", name)
    dev = _dev(host)
    _full_check(host, dev, 32, what=name)
    if name == "constant":
        m = tsa.moments(dev)
        assert m["std"] == 0.0 and m["mean"] == 3.25


def test_unaligned_base_and_scalar_paths():
    rng = np.random.default_rng(5)
    host = rng.standard_normal(10007).astype(np.float32)
    big = _dev(host)
    for off in (1, 2, 3):
        _say("case unaligned offset", off)
        sub = big[off:]  # data pointer not 16-byte aligned: scalar path
        _full_check(host[off:], sub, 50, what=f"offset {off}")
    # odd nx: rows fall back to scalar loads
    cube = rng.standard_normal((7, 9, 13)).astype(np.float32)
    dev = _dev(cube)
    for b in [(1, 1, 1, 12, 8, 6), (0, 0, 0, 13, 9, 7), (3, 2, 0, 4, 9, 7)]:
        _say("case odd nx", b)
        _full_check(cube, dev, 17, region=b, what=f"odd nx {b}")


def test_int16():
    spec = synth.scaled(synth.SPECS["c5c"], 128, 64, 48)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    _say("case int16 cube", host.shape)
    _full_check(host, dev, 256, dtype="i16", what="int16")
    for b in [(3, 5, 7, 101, 60, 40), (8, 0, 0, 16, 64, 48), (1, 1, 1, 2, 2, 2)]:
        _say("case int16 region", b)
        _full_check(host, dev, 100, region=b, dtype="i16", what=f"int16 {b}")
    ext = np.int16([-32768, 32767, 0, -1, 1, -32768, 32767])
    _full_check(ext, _dev(ext), 8, dtype="i16", what="int16 extremes")


@pytest.mark.parametrize("nbins", [1, 3, 4096, 16384, 20000, 65536])
def test_histogram_bin_counts(nbins):
    spec = synth.scaled(synth.SPECS["c1"], 128, 128, 64)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    _say("case nbins", nbins)
    for lo, hi in [(-3.0, 9.0), (-1.0, -1.0), (0.0, 1e-3)]:
        wc, wo = oracle.histogram(host, lo, hi, nbins)
        c, o = tsa.histogram(dev, lo, hi, nbins)
        check_hist(c, o, wc, wo, f"nbins {nbins} [{lo},{hi}]")
    b = (5, 3, 2, 120, 99, 60)
    wc, wo = oracle.histogram(host, -2.0, 20.0, nbins, b)
    c, o = tsa.histogram(dev, -2.0, 20.0, nbins, b)
    check_hist(c, o, wc, wo, f"nbins {nbins} region")
    # the fused trio at this bin count (16-bit counters above ~12K bins)
    for reg in (None, b):
        want = oracle.stats(host, nbins, reg)
        res, c, o = tsa.stats(dev, nbins, reg)
        check_moments(res, want, "f32", f"stats nbins {nbins} {reg}")
        check_median(res["median"], want["median"], "f32", f"stats nbins {nbins} {reg}")
        check_hist(c, o, want["counts"], want["outliers"], f"stats nbins {nbins} {reg}")


def test_integer_grid_histogram_is_bincount():
    rng = np.random.default_rng(9)
    host = rng.integers(0, 4096, 1 << 20).astype(np.float32)
    c, o = tsa.histogram(_dev(host), 0.0, 4096.0, 4096)
    assert np.array_equal(c.cpu().numpy(), np.bincount(host.astype(np.int64), minlength=4096))
    assert o.cpu().tolist() == [0, 0]


def test_deterministic_bits():
    spec = synth.scaled(synth.SPECS["c1"], 128, 128, 128)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    a = tsa.stats(dev, 512)
    b = tsa.stats(dev, 512)
    assert a[0] == b[0] or all((a[0][k] == b[0][k]) or (a[0][k] != a[0][k] and b[0][k] != b[0][k]) for k in a[0])
    assert torch.equal(a[1], b[1])
    m1, m2 = tsa.moments(dev), tsa.moments(dev)
    assert m1["mean"] == m2["mean"] and m1["std"] == m2["std"]


@pytest.mark.slow
def test_c2_full_size():
    """The benchmark workload (1024x1024x1280, 4096 bins), in the launch
    configuration the benchmark times, against the oracle on every output."""
    spec = synth.SPECS["c2"]
    _say("case c2 full size: generating")
    host, nan = synth.generate(spec)
    dev = _dev(host)
    _say("case c2: gpu stats")
    res, c, o = tsa.stats(dev, 4096)
    _say("case c2: oracle")
    want = oracle.stats(host, 4096)
    check_moments(res, want, "f32", "c2 stats")
    check_median(res["median"], want["median"], "f32", "c2 median")
    check_hist(c, o, want["counts"], want["outliers"], "c2 histogram")
    assert res["nan_count"] == nan
    gm = tsa.median(dev)
    check_median(gm["median"], want["median"], "f32", "c2 tsa_median")


def test_read_probe_sees_every_word():
    """The bandwidth probe reads the whole buffer: the XOR of its per-block
    words is the XOR of every 32-bit word (a ragged tail of vectors included)."""
    import ctypes
    rng = np.random.default_rng(12)
    host = rng.integers(0, 2**32, 3 * 1024 * 1024 + 4 * 37, dtype=np.uint64).astype(np.uint32)
    dev = torch.from_numpy(host.view(np.int32)).to("cuda:0")
    lib = tsa.capi().lib
    lib.tsa_internal_read_probe.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
    lib.tsa_internal_probe_blocks.restype = ctypes.c_int32
    nb = lib.tsa_internal_probe_blocks()
    assert nb > 0
    sink = torch.empty(nb, dtype=torch.int32, device="cuda:0")
    assert lib.tsa_internal_read_probe(dev.data_ptr(), host.nbytes, sink.data_ptr(), None) == 0
    assert lib.tsa_internal_read_probe(dev.data_ptr(), 12, sink.data_ptr(), None) == tsa.TSA_EINVAL
    torch.cuda.synchronize()
    got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))
    assert got == np.bitwise_xor.reduce(host)


@pytest.mark.parametrize("case", ["spread", "skewed", "int16"])
def test_stats_many_bins_outside_window(case):
    """65536 bins over [min, max]: the fused pass counts a 32768-bin window in
    LDS and the rest in global memory.  Values spread over the whole range
    (half outside any window), piled at one end, and int16 must all give the
    oracle's bins."""
    rng = np.random.default_rng(21)
    if case == "spread":
        host = rng.uniform(-1e6, 1e6, (40, 96, 128)).astype(np.float32)
    elif case == "skewed":
        host = np.exp(rng.standard_normal((40, 96, 128)) * 3).astype(np.float32)  # long right tail
        host[3, 4, 5] = np.nan
    else:
        host = rng.integers(-32768, 32768, (40, 96, 128)).astype(np.int16)
    dev = _dev(host)
    _say("case many bins", case)
    res, c, o = tsa.stats(dev, 65536)
    want = oracle.stats(host, 65536)
    dt = "i16" if host.dtype == np.int16 else "f32"
    check_moments(res, want, dt, case)
    check_median(res["median"], want["median"], dt, case)
    check_hist(c, o, want["counts"], want["outliers"], case)
    # the standalone call: a window placed from a sample, the rest (and the
    # values outside a narrower range) counted apart
    vals = host[~np.isnan(host)] if host.dtype == np.float32 else host
    narrow = (float(np.float32(np.percentile(vals, 10))), float(np.float32(np.percentile(vals, 95))))
    for nb in (20000, 65536):
        for lo, hi in [(float(want["min"]), float(want["max"])), narrow]:
            wc, wo = oracle.histogram(host, lo, hi, nb)
            c, o = tsa.histogram(dev, lo, hi, nb)
            check_hist(c, o, wc, wo, f"{case} histogram {nb} [{lo}, {hi}]")
    b = (7, 5, 3, 120, 90, 37)
    wc, wo = oracle.histogram(host, narrow[0], narrow[1], 65536, b)
    c, o = tsa.histogram(dev, narrow[0], narrow[1], 65536, b)
    check_hist(c, o, wc, wo, f"{case} histogram region")


def test_stats_graph_replays_match_direct_launch():
    """tsa_stats captures its launches into a graph the second time an
    argument set comes and replays it afterwards.  Every replay, with eager
    GPU work and synchronisation between them, must equal the directly
    launched call (tracing makes a call launch directly), for the whole cube
    and for a box; the direct results match the oracle."""
    import ctypes
    spec = synth.scaled(synth.SPECS["c1"], 96, 96, 64)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    nbins = 256
    api = tsa.capi()
    lib = api.lib
    lib.tsa_trace_enable.argtypes = [ctypes.c_int32, ctypes.c_int32]
    c = tsa.cube_of(dev)
    out = torch.empty(72, dtype=torch.uint8, device="cuda:0")
    counts = torch.empty(nbins, dtype=torch.int64, device="cuda:0")
    outl = torch.empty(2, dtype=torch.int64, device="cuda:0")
    for box in (None, (5, 7, 3, 90, 81, 60)):
        _say("case stats graph replays", box)
        reg = tsa.region_of(box)
        ws = tsa.workspace(tsa.OP_STATS, dev, box, nbins)

        def call():
            st = api.tsa_stats(ctypes.byref(c), tsa._rp(reg), nbins, out.data_ptr(), counts.data_ptr(),
                               outl.data_ptr(), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
            assert st == 0
            torch.cuda.synchronize()
            return out.cpu().numpy().tobytes(), counts.cpu().numpy().tobytes(), outl.cpu().numpy().tobytes()

        assert lib.tsa_trace_enable(1, 64) == 0
        direct = call()
        assert lib.tsa_trace_enable(0, 0) == 0
        r = {k: tsa.results_to_numpy(out)[0][k].item() for k in tsa.results_to_numpy(out).dtype.names}
        want = oracle.stats(host, nbins, box)
        check_moments(r, want, "f32", f"direct {box}")
        check_median(r["median"], want["median"], "f32", f"direct {box}")
        for rep in range(5):
            x = (dev * 2.0).sum()  # eager GPU work between replays
            torch.cuda.synchronize()
            del x
            got = call()  # 1st: direct launch, 2nd: capture, then replays
            assert got == direct, (box, rep)
