"""Serving engine: every response equals the same request served alone, under
an open-loop mixed load; admission limits hold; results match the oracle."""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_hist, check_median, check_moments

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1211_4896_amd as tsa  # noqa: E402
from paper_1211_4896_amd import serve  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cubes():
    specs = [synth.scaled(synth.SPECS["c5a"], 96, 80, 64), synth.scaled(synth.SPECS["c5b"], 128, 64, 48),
             synth.scaled(synth.SPECS["c5c"], 64, 64, 64)]
    hosts = [synth.generate(s)[0] for s in specs]
    return hosts


def _workload(hosts, n, seed, full_frac=0.1):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        c = int(rng.integers(0, len(hosts)))
        nz, ny, nx = hosts[c].shape
        if rng.random() < full_frac:
            kind = serve.REQ_FULL_HIST if rng.random() < 0.5 else serve.REQ_FULL_MEDIAN
            reqs.append((c, kind, None))
        else:
            b = synth.regions(1, (nx, ny, nz), seed * 100003 + i, edge_lo=2, edge_hi=40)[0]
            reqs.append((c, serve.REQ_REGION, tuple(int(v) for v in b)))
    return reqs


def _make(srv, cube_ids, reqs, nb_region, nb_full):
    out, hists = [], []
    for i, (c, kind, box) in enumerate(reqs):
        h = np.zeros(nb_region if kind == serve.REQ_REGION else nb_full, dtype=np.uint64)
        hists.append(h)
        out.append(srv.request(cube_ids[c], kind, box, h if kind != serve.REQ_FULL_MEDIAN else None, tag=i))
    return out, hists


def _same(a, b):
    ra, rb = a.result, b.result
    for k in ("count", "nan_count", "status", "flags"):
        if getattr(ra, k) != getattr(rb, k):
            return False
    for k in ("mean", "m2", "std", "min", "max", "median"):
        x, y = getattr(ra, k), getattr(rb, k)
        if not (x == y or (x != x and y != y)):
            return False
    return a.status == b.status


def test_alone_equals_in_the_mix():
    hosts = _cubes()
    devs = [torch.from_numpy(h).to("cuda:0") for h in hosts]
    reqs = _workload(hosts, 400, seed=5)
    with serve.Server(max_batch=64, region_lanes=2, max_admitted=256, region_nbins=64, full_nbins=512) as srv:
        ids = [srv.add_cube(d) for d in devs]
        # alone: one request at a time
        _say("case serve alone")
        alone_reqs, alone_h = _make(srv, ids, reqs, 64, 512)
        alone = []
        for r in alone_reqs:
            srv.submit(r)
            srv.drain(60.0)
            got = srv.poll(4)
            assert len(got) == 1
            alone.append(got[0])
        # in the mix: open-loop arrivals far faster than service
        _say("case serve mix")
        mix_reqs, mix_h = _make(srv, ids, reqs, 64, 512)
        t = serve.poisson_arrivals(20000.0, len(mix_reqs), seed=9)
        mixed = srv.replay(mix_reqs, t)
        st = srv.stats()
        _say("server stats", st)
        assert st["max_batch"] > 1  # requests really were batched together
        for i in range(len(reqs)):
            assert alone[i].tag == mixed[i].tag == i
            assert mixed[i].status == 0, (i, mixed[i].status)
            assert _same(alone[i], mixed[i]), (i, reqs[i])
            assert np.array_equal(alone_h[i], mix_h[i]), i
            assert mixed[i].t_submit <= mixed[i].t_admit <= mixed[i].t_launch <= mixed[i].t_done
    # and the answers are right
    for i in range(0, len(reqs), 9):
        c, kind, box = reqs[i]
        host = hosts[c]
        dt = "i16" if host.dtype == np.int16 else "f32"
        r = serve.response_dict(mixed[i])["result"]
        if kind == serve.REQ_REGION:
            want = oracle.stats(host, 64, box)
            check_moments(r, want, dt, f"serve q{i}")
            check_median(r["median"], want["median"], dt, f"serve q{i}")
            if not want["hist_skipped"]:
                check_hist(mix_h[i], None, want["counts"], None, f"serve q{i}")
        elif kind == serve.REQ_FULL_MEDIAN:
            want, n = oracle.median(host)
            check_median(r["median"], want, dt, f"serve full median {i}")
            assert r["count"] == n
        else:
            mo = oracle.moments(host)
            wc, _ = oracle.histogram(host, float(np.float32(mo["min"])), float(np.float32(mo["max"])), 512)
            check_hist(mix_h[i], None, wc, None, f"serve full hist {i}")


def test_admission_limit_and_scratch_budget():
    hosts = _cubes()
    devs = [torch.from_numpy(h).to("cuda:0") for h in hosts]
    reqs = _workload(hosts, 120, seed=6, full_frac=0.2)
    with serve.Server(max_batch=8, region_lanes=1, max_admitted=4, region_nbins=32, full_nbins=256) as srv:
        ids = [srv.add_cube(d) for d in devs]
        mk, _ = _make(srv, ids, reqs, 32, 256)
        _say("case serve admission")
        out = srv.replay(mk, serve.poisson_arrivals(50000.0, len(mk), seed=1))
        st = srv.stats()
        assert st["finished"] == st["submitted"] >= len(reqs)
        assert st["max_batch"] <= 4  # never more admitted than the slots
        assert st["admission_waits"] > 0
        assert all(o.status == 0 for o in out)


def test_bad_requests():
    host = np.zeros((4, 4, 8), np.float32)
    with serve.Server(max_batch=4, region_lanes=1, max_admitted=4, region_nbins=8, full_nbins=8) as srv:
        cid = srv.add_cube(torch.from_numpy(host).to("cuda:0"))
        with pytest.raises(tsa.TsaError):
            srv.submit(srv.request(cid + 5, serve.REQ_REGION, (0, 0, 0, 1, 1, 1)))
        with pytest.raises(tsa.TsaError):
            srv.submit(srv.request(cid, 7, None))
        srv.submit(srv.request(cid, serve.REQ_REGION, (0, 0, 0, 9, 1, 1), tag=3))  # box outside the cube
        srv.drain(30.0)
        r = srv.poll(4)
        assert len(r) == 1 and r[0].result.status == tsa.TSA_EINVAL and r[0].tag == 3


def test_scratch_budget_limits_admission():
    """A scratch budget of three region requests: admission waits on the
    budget (the slot limit is far above it), the budget in use never exceeds
    it, every answer equals the same request served alone, and a request that
    costs more than the whole budget is refused at submission (TSA_ENOMEM)
    instead of holding up its class."""
    hosts = _cubes()
    devs = [torch.from_numpy(h).to("cuda:0") for h in hosts]
    reqs = [r for r in _workload(hosts, 150, seed=7, full_frac=0.0)]
    with serve.Server(max_batch=16, region_lanes=2, max_admitted=4096, region_nbins=32, full_nbins=256) as probe:
        cost = probe.stats()["region_cost"]
    budget = 3 * cost
    with serve.Server(max_batch=16, region_lanes=2, max_admitted=4096, region_nbins=32, full_nbins=256,
                      scratch_bytes=budget) as srv:
        ids = [srv.add_cube(d) for d in devs]
        # a full-cube request needs the full-cube workspace: far above three region requests
        with pytest.raises(tsa.TsaError) as e:
            srv.submit(srv.request(ids[0], serve.REQ_FULL_MEDIAN, None))
        assert e.value.status == tsa.TSA_ENOMEM
        mk, mh = _make(srv, ids, reqs, 32, 256)
        _say("case serve scratch budget", budget)
        out = srv.replay(mk, serve.poisson_arrivals(50000.0, len(mk), seed=2))
        st = srv.stats()
        _say("server stats", st)
        assert st["scratch_bytes"] == budget and 0 < st["budget_peak"] <= budget
        assert st["admission_waits"] > 0 and st["max_batch"] <= 3
        assert st["finished"] == st["submitted"] == len(reqs)
        alone_mk, alone_h = _make(srv, ids, reqs, 32, 256)
        for i, r in enumerate(alone_mk):
            srv.submit(r)
            srv.drain(60.0)
            a = srv.poll(4)
            assert len(a) == 1 and out[i].status == 0
            assert _same(a[0], out[i]), (i, reqs[i])
            assert np.array_equal(alone_h[i], mh[i]), i


def test_full_scans_in_slab_launches():
    """Full-cube requests answered with each pass cut into z-slab launches of
    a voxel budget (17 KiB voxels here: many slabs, the last one short; the
    median's candidate list and its third pass over the slabs, a histogram of
    more bins than one LDS copy holds) give the same bits as one launch per
    pass, and the oracle's answers."""
    rng = np.random.default_rng(12)
    hosts = [synth.generate(synth.scaled(synth.SPECS["c5a"], 64, 48, 40))[0],
             rng.integers(0, 3, size=(37, 40, 64)).astype(np.float32),  # ties: the last digit over the slabs
             synth.generate(synth.scaled(synth.SPECS["c5c"], 64, 32, 33))[0]]
    devs = [torch.from_numpy(h).to("cuda:0") for h in hosts]
    kinds = [serve.REQ_FULL_HIST, serve.REQ_FULL_MEDIAN]
    for nbins in (512, 20000):
        outs = []
        for chunk in (0, 17):
            with serve.Server(max_batch=8, region_lanes=1, max_admitted=64, region_nbins=16, full_nbins=nbins,
                              full_chunk_kvoxels=chunk) as srv:
                ids = [srv.add_cube(d) for d in devs]
                reqs = [(c, k, None) for c in range(len(hosts)) for k in kinds]
                mk, mh = _make(srv, ids, reqs, 16, nbins)
                _say("case serve slabs", nbins, chunk)
                for r in mk:
                    srv.submit(r)
                srv.drain(60.0)
                got = sorted(srv.poll(64), key=lambda r: r.tag)
                assert len(got) == len(reqs) and all(g.status == 0 for g in got)
                outs.append((got, mh))
        (a, ah), (b, bh) = outs
        for i, (c, kind, _) in enumerate(reqs):
            assert _same(a[i], b[i]), (nbins, i)
            assert np.array_equal(ah[i], bh[i]), (nbins, i)
            host = hosts[c]
            dt = "i16" if host.dtype == np.int16 else "f32"
            r = serve.response_dict(b[i])["result"]
            if kind == serve.REQ_FULL_MEDIAN:
                want, n = oracle.median(host)
                check_median(r["median"], want, dt, f"slabs median {c}")
                assert r["count"] == n
            else:
                mo = oracle.moments(host)
                wc, _ = oracle.histogram(host, float(np.float32(mo["min"])), float(np.float32(mo["max"])), nbins)
                check_hist(bh[i], None, wc, None, f"slabs hist {c} {nbins}")
