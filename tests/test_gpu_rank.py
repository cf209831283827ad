"""Quantiles (arbitrary rank, early stop) and the median absolute deviation vs the oracle."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_median

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1211_4896_amd as tsa  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


QS = [0.0, 0.001, 0.1, 0.25, 0.29, 0.5, 0.75, 0.9, 0.999, 1.0]


def test_quantiles_exact_and_early():
    spec = synth.scaled(synth.SPECS["c1"], 128, 96, 64)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    for reg in (None, (3, 5, 7, 101, 90, 60)):
        for q in QS:
            _say("case quantile", q, reg)
            want, n = oracle.quantile(host, q, reg)
            v, w, cnt = tsa.quantile(dev, q, reg)
            assert cnt == n and w == 0.0
            check_median(v, want, "f32", f"q={q} {reg}")
            for digits in (1, 2):
                v, w, cnt = tsa.quantile(dev, q, reg, digits=digits)
                assert cnt == n and w >= 0.0
                assert v <= want <= v + w, (q, digits, v, w, want)


def test_quantile_median_equals_median_call_and_int16():
    rng = np.random.default_rng(4)
    host = rng.integers(-30000, 30000, (24, 40, 64)).astype(np.int16)
    dev = _dev(host)
    for q in QS:
        want, n = oracle.quantile(host, q)
        v, w, cnt = tsa.quantile(dev, q)
        assert v == want and cnt == n and w == 0.0
    assert tsa.quantile(dev, 0.5)[0] == tsa.median(dev)["median"]
    with pytest.raises(tsa.TsaError):
        tsa.quantile(dev, 1.5)
    empty = _dev(np.full(64, np.nan, np.float32))
    v, w, cnt = tsa.quantile(empty, 0.3)
    assert math.isnan(v) and cnt == 0


@pytest.mark.parametrize("seed", [0, 1])
def test_mad_matches_oracle(seed):
    spec = synth.scaled(synth.SPECS["c1"], 96, 80, 64)
    spec = synth.CubeSpec(**{**spec.__dict__, "seed": 300 + seed})
    host, _ = synth.generate(spec)
    dev = _dev(host)
    for reg in (None, (2, 3, 4, 90, 77, 60), (5, 5, 5, 6, 9, 9)):
        _say("case mad", seed, reg)
        m, mad, n = oracle.mad(host, reg)
        gm, gmad, gn = tsa.mad(dev, reg)
        assert gn == n
        check_median(gm, m, "f32", f"mad median {reg}")
        check_median(gmad, mad, "f32", f"mad {reg}")


def test_mad_int16_and_edges():
    spec = synth.scaled(synth.SPECS["c5c"], 64, 48, 32)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    m, mad, n = oracle.mad(host)
    assert tsa.mad(dev) == (m, mad, n)
    ext = np.int16([-32768, 32767, 0, 5, -5, 100])
    assert tsa.mad(_dev(ext)) == oracle.mad(ext)
    const = np.full(1000, 2.5, np.float32)
    assert tsa.mad(_dev(const)) == (2.5, 0.0, 1000)
    allnan = np.full(100, np.nan, np.float32)
    gm, gmad, gn = tsa.mad(_dev(allnan))
    assert math.isnan(gm) and math.isnan(gmad) and gn == 0
    ties = np.float32([1, 1, 1, 2, 2, 3, 10, np.nan, -0.0, 0.0])
    assert tsa.mad(_dev(ties)) == oracle.mad(ties)


def test_mad_infinite_median():
    """A value equal to an infinite median deviates by zero (no NaN
    deviations), as the oracle defines it."""
    cases = {
        "inf3_1": np.float32([np.inf, np.inf, np.inf, 1]),
        "minf2_0": np.float32([-np.inf, -np.inf, 0]),
        "inf_majority_nan": np.float32([1, 2, np.inf, np.inf, np.inf, np.nan]),
        "finite_median_infs": np.float32([1, 2, 3, np.inf, -np.inf]),
    }
    rng = np.random.default_rng(17)
    big = rng.standard_normal(50000).astype(np.float32)
    big[rng.random(big.size) < 0.6] = np.inf
    big[rng.random(big.size) < 0.01] = np.nan
    cases["inf_majority_50k"] = big
    neg = -big
    cases["minf_majority_50k"] = neg
    for name, x in cases.items():
        _say("case mad inf", name)
        want = oracle.mad(x)
        got = tsa.mad(_dev(x))
        assert got[2] == want[2], (name, got, want)
        check_median(got[0], want[0], "f32", f"{name} median")
        check_median(got[1], want[1], "f32", f"{name} mad")
