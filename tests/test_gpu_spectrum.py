"""3-D spectrum tool (Section 4.4) against the oracle, sample by sample.

Both sides form the positions, weights and sums with the same IEEE double
operations in the order the definition states, so the samples are compared
bit for bit (NaN where the oracle has NaN)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1211_4896_amd as tsa  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _rays(n, dims, seed, step=0.5, inside=True):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    if inside:
        o = rng.uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1], (n, 3))
    else:
        o = rng.uniform([-5, -5, -5], [nx + 4, ny + 4, nz + 4], (n, 3))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([o, d * step], axis=1)


def _check(host, rays, nsamples, what):
    dev = _dev(host)
    _say("case spectrum", what, host.shape, len(rays), nsamples)
    got = tsa.spectrum(dev, rays, nsamples).cpu().numpy()
    want = oracle.spectrum(host, rays[:, :3], rays[:, 3:], nsamples)
    assert got.shape == want.shape
    bad = ~((got == want) | (np.isnan(got) & np.isnan(want)))
    assert not bad.any(), (what, np.argwhere(bad)[:5], got[bad][:5], want[bad][:5])
    return got


def test_spectrum_survey_cube():
    spec = synth.scaled(synth.SPECS["c3"], 96, 80, 72)
    host, _ = synth.generate(spec)
    dims = (96, 80, 72)
    got = _check(host, _rays(64, dims, 1), 300, "inside origins")  # 300: a ragged second block
    assert np.isfinite(got).mean() > 0.2
    _check(host, _rays(64, dims, 2, step=1.7, inside=False), 77, "outside origins")


def test_spectrum_axis_rays_hit_voxels_exactly():
    rng = np.random.default_rng(5)
    host = rng.standard_normal((40, 30, 20)).astype(np.float32)
    host[7, 3, 4] = np.nan
    rays = np.array([[4, 3, 0, 0, 0, 1],       # along frequency: a plain spectrum
                     [0, 3, 7, 1, 0, 0],       # along x through the NaN voxel
                     [19, 29, 39, -1, -1, -1],  # from the far corner
                     [2.5, 0, 0, 0, 0.5, 0.5],
                     [0, 0, 0, 0, 0, 0]], dtype=np.float64)  # a zero step: one point repeated
    got = _check(host, rays, 45, "axis rays")
    assert np.array_equal(got[0, :40], host[:, 3, 4].astype(np.float64), equal_nan=True)
    assert np.all(np.isnan(got[0, 40:]))


def test_spectrum_int16_thin_axes_and_empty():
    spec = synth.scaled(synth.SPECS["c5c"], 64, 48, 40)
    host, _ = synth.generate(spec)
    _check(host, _rays(32, (64, 48, 40), 3, step=0.9), 130, "int16")
    rng = np.random.default_rng(6)
    flat = rng.standard_normal((1, 7, 9)).astype(np.float32)  # one plane: z must be exactly 0
    rays = np.array([[0.5, 0.5, 0.0, 0.25, 0.2, 0.0], [0.5, 0.5, 0.0, 0.25, 0.2, 1e-9],
                     [8.0, 6.0, 0.0, -0.5, -0.5, 0.0]])
    _check(flat, rays, 20, "one plane")
    dev = _dev(flat)
    assert tsa.spectrum(dev, np.zeros((0, 6)), 10).shape == (0, 10)
    assert tsa.spectrum(dev, rays, 0).shape == (3, 0)


def test_spectrum_deterministic():
    spec = synth.scaled(synth.SPECS["c1"], 64, 64, 64)
    host, _ = synth.generate(spec)
    dev = _dev(host)
    rays = _rays(200, (64, 64, 64), 9)
    a = tsa.spectrum(dev, rays, 257)
    b = tsa.spectrum(dev, rays, 257)
    assert torch.equal(a.nan_to_num(7.5), b.nan_to_num(7.5))
