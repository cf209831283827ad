"""Seeded synthetic cubes and region lists (inputs only; no statistics here).

The paper's HIPASS, LMC and GASS cubes (Section 5, Table 2) are not available,
so these generators stand in for them with the same shapes and value
structure: Gaussian noise, compact bright sources, NULL (NaN) slabs.  Both the
HIP path and the CPU oracle take the arrays made here unchanged.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libsynth.so with gcc (in-tree)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.synth_cube.restype = ctypes.c_int64
        lib.synth_cube.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


@dataclass(frozen=True)
class CubeSpec:
    nx: int
    ny: int
    nz: int
    seed: int
    n_sources: int = 200
    amp: tuple = (5.0, 50.0)
    amp_log: bool = False
    sigma: tuple = (2.0, 6.0)
    nan_frac: float = 0.005
    dtype: str = "f32"  # "f32" or "i16"

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def np_dtype(self):
        return np.float32 if self.dtype == "f32" else np.int16


# The workloads: shapes and value distributions of the paper's cubes.
SPECS = {
    # 256^3: N(0,1) + 200 sources, A ~ U[5,50], sigma ~ U[2,6], 0.5% NaN slabs
    "c1": CubeSpec(256, 256, 256, seed=11),
    # 1024x1024x1280 (5.37 GB): one GPU's 1/96 share of a ~0.5 TB cube; the 256^3 recipe at the
    # same source density (200 per 256^3)
    "c2": CubeSpec(1024, 1024, 1280, seed=12, n_sources=200 * 80),
    # 4096x4096x3072 (206 GB): 20000 sources, A log-uniform [3,500], 0.1% NaN
    "c3": CubeSpec(4096, 4096, 3072, seed=13, n_sources=20000, amp=(3.0, 500.0), amp_log=True,
                   nan_frac=0.001),
    # resident cube for batched region queries
    "c4": CubeSpec(2048, 2048, 2048, seed=14, n_sources=200 * 512),
    # serving cubes
    "c5a": CubeSpec(1024, 1024, 1024, seed=15, n_sources=200 * 64),
    "c5b": CubeSpec(2048, 2048, 1024, seed=16, n_sources=200 * 256),
    "c5c": CubeSpec(2048, 2048, 2048, seed=17, n_sources=200 * 512, amp=(5000.0, 50000.0),
                    nan_frac=0.0, dtype="i16"),
}


def scaled(spec: CubeSpec, nx: int, ny: int, nz: int, keep_density: bool = True) -> CubeSpec:
    """Same recipe at another shape (sources scaled to keep their density)."""
    ns = spec.n_sources
    if keep_density:
        ns = max(1, int(round(spec.n_sources * (nx * ny * nz) / spec.n)))
    return replace(spec, nx=nx, ny=ny, nz=nz, n_sources=ns)


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def generate(spec: CubeSpec, z0: int = 0, z1: int | None = None, out: np.ndarray | None = None,
             threads: int | None = None):
    """Return (array of shape (z1-z0, ny, nx), nan_count) for slices [z0, z1)."""
    lib = _load()
    if z1 is None:
        z1 = spec.nz
    shape = (z1 - z0, spec.ny, spec.nx)
    if out is None:
        out = np.empty(shape, dtype=spec.np_dtype)
    assert out.shape == shape and out.dtype == spec.np_dtype and out.flags.c_contiguous
    nan = lib.synth_cube(spec.nx, spec.ny, spec.nz, spec.seed, spec.n_sources, spec.amp[0], spec.amp[1],
                         int(spec.amp_log), spec.sigma[0], spec.sigma[1], spec.nan_frac,
                         0 if spec.dtype == "f32" else 1, z0, z1, out.ctypes.data,
                         threads or default_threads())
    if nan < 0:
        raise ValueError("synth_cube rejected its arguments")
    return out, int(nan)


def regions(nq: int, dims, seed: int, edge_lo: int = 8, edge_hi: int = 512) -> np.ndarray:
    """nq half-open boxes (x0,y0,z0,x1,y1,z1) as int64[nq,6].

    Edge lengths round(exp(U[ln lo, ln hi])) per axis (clipped to the cube),
    origins uniform so that the box fits.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    out = np.empty((nq, 6), dtype=np.int64)
    for a, n in enumerate((nx, ny, nz)):
        e = np.rint(np.exp(rng.uniform(np.log(edge_lo), np.log(edge_hi), nq))).astype(np.int64)
        e = np.clip(e, 1, n)
        o = (rng.random(nq) * (n - e + 1)).astype(np.int64)
        out[:, a] = o
        out[:, a + 3] = o + e
    return out


def sight_lines(nrays: int, dims, seed: int, step: float = 0.5, max_angle_deg: float = 45.0) -> np.ndarray:
    """Rays for the spectrum tool as float64[nrays, 6] = origin (x, y, z) and
    step vector: origins uniform on the z = 0 face, directions uniform over
    the cap within max_angle of +z, step length `step` voxels."""
    rng = np.random.default_rng(seed)
    nx, ny, _ = dims
    o = np.stack([rng.uniform(0, nx - 1, nrays), rng.uniform(0, ny - 1, nrays), np.zeros(nrays)], axis=1)
    th = np.arccos(rng.uniform(np.cos(np.radians(max_angle_deg)), 1.0, nrays))
    ph = rng.uniform(0, 2 * np.pi, nrays)
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1) * step
    return np.concatenate([o, d], axis=1)


def key_order_values(rng: np.random.Generator, n: int) -> np.ndarray:
    """Adversarial float32 values: +-0, denormals, +-inf, ties, NaN."""
    pool = np.array([0.0, -0.0, 1e-45, -1e-45, 1.17e-38, -3.4e38, 3.4e38, np.inf, -np.inf, 1.0, -1.0,
                     0.5, 2.0, np.nan], dtype=np.float32)
    return pool[rng.integers(0, len(pool), n)]
