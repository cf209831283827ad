"""Tera-scale cube statistics on MI355X (gfx950): Python binding of libtsa.so.

The statistics of Hassan et al., "Tera-scale astronomical data analysis and
visualization" (arXiv 1211.4896), Section 4: global histogram (4.1), mean and
standard deviation (4.2), exact median (4.3), and batched queries over
sub-cube regions.  Every step runs in the HIP kernels of libtsa.so; this
module only marshals arguments.  PyTorch supplies device memory and streams.

Two layers:

* ``capi`` -- the C functions of include/tsa.h under their own names
  (``tsa_moments``, ``tsa_histogram``, ``tsa_median``, ``tsa_stats``,
  ``tsa_region_batch``, ``tsa_workspace_bytes``, ...), taking ctypes
  structures and raw device pointers;
* ``moments``, ``histogram``, ``median``, ``stats``, ``region_batch`` --
  conveniences taking torch tensors, allocating outputs and workspace with
  torch, and synchronising before they return.

A missing or unloadable libtsa.so raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TSA_LIB names another build of the same library (for timing one build against another)
LIB_PATH = os.environ.get("TSA_LIB") or os.path.join(_HERE, "libtsa.so")

TSA_OK, TSA_EINVAL, TSA_ENOMEM, TSA_EDEVICE, TSA_ENOTSUP, TSA_EBUSY = 0, -1, -2, -3, -4, -5
TSA_F32, TSA_I16 = 0, 1
OP_MOMENTS, OP_HISTOGRAM, OP_MEDIAN, OP_STATS, OP_REGION_BATCH, OP_QUANTILE, OP_MAD = 0, 1, 2, 3, 4, 5, 6
FLAG_HIST_SKIPPED, FLAG_BAD_REGION, FLAG_PHASE3 = 1, 2, 4


class Cube(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Region(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int64), ("y0", ctypes.c_int64), ("z0", ctypes.c_int64),
                ("x1", ctypes.c_int64), ("y1", ctypes.c_int64), ("z1", ctypes.c_int64)]


class Tune(ctypes.Structure):
    _fields_ = [("tile_voxels", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("cand_max", ctypes.c_int32), ("replicas", ctypes.c_int32)]


# tsa_result as a numpy record (72 bytes)
RESULT_DTYPE = np.dtype([("count", "<u8"), ("nan_count", "<u8"), ("mean", "<f8"), ("m2", "<f8"), ("std", "<f8"),
                         ("min", "<f8"), ("max", "<f8"), ("median", "<f8"), ("status", "<i4"), ("flags", "<i4")])
assert RESULT_DTYPE.itemsize == 72


class TsaError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class _CAPI:
    """The C ABI, loaded once."""

    def __init__(self, path: str):
        if not os.path.exists(path):
            raise RuntimeError(f"libtsa.so not built ({path}); run paper_1211_4896_amd.build.build()")
        lib = ctypes.CDLL(path)
        P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        CP = ctypes.POINTER(Cube)
        RP = ctypes.POINTER(Region)
        sig = {
            "tsa_workspace_bytes": (SZ, [I32, CP, RP, I32, I32]),
            "tsa_moments": (ctypes.c_int, [CP, RP, P, P, SZ, P]),
            "tsa_histogram": (ctypes.c_int, [CP, RP, ctypes.c_float, ctypes.c_float, I32, P, P, P, SZ, P]),
            "tsa_median": (ctypes.c_int, [CP, RP, P, P, SZ, P]),
            "tsa_stats": (ctypes.c_int, [CP, RP, I32, P, P, P, P, SZ, P]),
            "tsa_stats_static": (ctypes.c_int, [CP, RP, I32, P, P, P, P]),
            "tsa_stats_static_scratch_bytes": (SZ, []),
            "tsa_stats_static_candidate_keys": (I64, []),
            "tsa_region_batch": (ctypes.c_int, [CP, P, I32, I32, P, P, ctypes.POINTER(Tune), P, SZ, P]),
            "tsa_status_string": (ctypes.c_char_p, [I32]),
            "tsa_version": (ctypes.c_char_p, []),
            "tsa_internal_magic_div": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32]),
            "tsa_tune_region_batch": (ctypes.c_int, [CP, P, I32, I32, P, P, P, SZ, P, I32, ctypes.POINTER(Tune),
                                                     ctypes.POINTER(ctypes.c_float)]),
            "tsa_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
            "tsa_quantile": (ctypes.c_int, [CP, RP, ctypes.c_double, I32, P, P, SZ, P]),
            "tsa_mad": (ctypes.c_int, [CP, RP, P, P, SZ, P]),
            "tsa_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
            "tsa_minimap_workspace_bytes": (SZ, [CP, I32, I32, I32, I32]),
            "tsa_minimap_cells": (I64, [CP, I32, I32, I32]),
            "tsa_minimap": (ctypes.c_int, [CP, I32, I32, I32, I32, P, P, P, SZ, P]),
            "tsa_sigma_count": (ctypes.c_int, [CP, I32, I32, I32, P, ctypes.c_double, P, P]),
            "tsa_spectrum": (ctypes.c_int, [CP, P, I32, I32, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
            setattr(self, name, f)
        self.lib = lib
        self.path = path


_capi: Optional[_CAPI] = None


def capi() -> _CAPI:
    global _capi
    if _capi is None:
        _capi = _CAPI(LIB_PATH)
    return _capi


def status_string(status: int) -> str:
    return capi().tsa_status_string(status).decode()


def _check(st: int, what: str):
    if st != TSA_OK:
        raise TsaError(st, what)


# ---------------------------------------------------------------------------
# torch conveniences
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def cube_of(t) -> Cube:
    """Describe a (nz, ny, nx) contiguous float32/int16 CUDA tensor (or a 1-D one)."""
    torch = _torch()
    if not t.is_cuda:
        raise ValueError("cube tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("cube tensor must be contiguous")
    if t.dtype == torch.float32:
        dt = TSA_F32
    elif t.dtype == torch.int16:
        dt = TSA_I16
    else:
        raise TypeError("cube dtype must be float32 or int16")
    if t.dim() == 1:
        nz, ny, nx = 1, 1, t.shape[0]
    elif t.dim() == 3:
        nz, ny, nx = t.shape
    else:
        raise ValueError("cube must be 1-D or (nz, ny, nx)")
    return Cube(t.data_ptr(), dt, 0, nx, ny, nz)


def region_of(r) -> Optional[Region]:
    if r is None:
        return None
    x0, y0, z0, x1, y1, z1 = (int(v) for v in r)
    return Region(x0, y0, z0, x1, y1, z1)


def _rp(reg: Optional[Region]):
    return ctypes.byref(reg) if reg is not None else None


def _stream(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def workspace(op: int, t, region=None, nbins: int = 0, nq: int = 0):
    torch = _torch()
    c = cube_of(t)
    reg = region_of(region)
    n = capi().tsa_workspace_bytes(op, ctypes.byref(c), _rp(reg), nbins, nq)
    if n == 0:
        raise TsaError(TSA_EINVAL, "tsa_workspace_bytes")
    return torch.empty(n, dtype=torch.uint8, device=t.device)


def results_to_numpy(buf) -> np.ndarray:
    """Device uint8 buffer of n tsa_result records -> numpy record array."""
    return buf.cpu().numpy().view(RESULT_DTYPE)


def _result_buf(t, n: int = 1):
    torch = _torch()
    buf = torch.empty(72 * n, dtype=torch.uint8, device=t.device)
    # NaN-filled doubles, zero counts/status/flags: untouched fields read as NaN
    v = buf.view(torch.float64).view(n, 9)
    v.fill_(float("nan"))
    buf.view(torch.int64).view(n, 9)[:, 0:2].zero_()
    buf.view(torch.int64).view(n, 9)[:, 8].zero_()
    return buf


def _rec(r) -> dict:
    return {k: (r[k].item() if hasattr(r[k], "item") else r[k]) for k in RESULT_DTYPE.names}


def moments(t, region=None, stream=None) -> dict:
    torch = _torch()
    c, reg = cube_of(t), region_of(region)
    ws = workspace(OP_MOMENTS, t, region)
    out = _result_buf(t)
    _check(capi().tsa_moments(ctypes.byref(c), _rp(reg), out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)),
           "tsa_moments")
    torch.cuda.synchronize(t.device)
    return _rec(results_to_numpy(out)[0])


def histogram(t, lo: float, hi: float, nbins: int, region=None, stream=None):
    """Returns (counts int64 tensor [nbins] holding uint64 bits, outliers [2])."""
    torch = _torch()
    c, reg = cube_of(t), region_of(region)
    ws = workspace(OP_HISTOGRAM, t, region, nbins)
    counts = torch.empty(nbins, dtype=torch.int64, device=t.device)
    outl = torch.empty(2, dtype=torch.int64, device=t.device)
    _check(capi().tsa_histogram(ctypes.byref(c), _rp(reg), lo, hi, nbins, counts.data_ptr(), outl.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream(stream)), "tsa_histogram")
    torch.cuda.synchronize(t.device)
    return counts, outl


def median(t, region=None, stream=None) -> dict:
    torch = _torch()
    c, reg = cube_of(t), region_of(region)
    ws = workspace(OP_MEDIAN, t, region)
    out = _result_buf(t)
    _check(capi().tsa_median(ctypes.byref(c), _rp(reg), out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)),
           "tsa_median")
    torch.cuda.synchronize(t.device)
    return _rec(results_to_numpy(out)[0])


def stats(t, nbins: int, region=None, stream=None):
    """Moments, nbins histogram over [min, max] and lower median together.

    Returns (result dict, counts tensor, outliers tensor)."""
    torch = _torch()
    c, reg = cube_of(t), region_of(region)
    ws = workspace(OP_STATS, t, region, nbins)
    out = _result_buf(t)
    counts = torch.empty(nbins, dtype=torch.int64, device=t.device)
    outl = torch.empty(2, dtype=torch.int64, device=t.device)
    _check(capi().tsa_stats(ctypes.byref(c), _rp(reg), nbins, out.data_ptr(), counts.data_ptr(), outl.data_ptr(),
                            ws.data_ptr(), ws.numel(), _stream(stream)), "tsa_stats")
    torch.cuda.synchronize(t.device)
    return _rec(results_to_numpy(out)[0]), counts, outl


def stats_static(t, nbins: int, region=None, stream=None):
    """``stats`` through tsa_stats_static: no workspace, the library's fixed
    per-device scratch instead.  Returns (result dict, counts, outliers)."""
    torch = _torch()
    c, reg = cube_of(t), region_of(region)
    out = _result_buf(t)
    counts = torch.empty(nbins, dtype=torch.int64, device=t.device)
    outl = torch.empty(2, dtype=torch.int64, device=t.device)
    _check(capi().tsa_stats_static(ctypes.byref(c), _rp(reg), nbins, out.data_ptr(), counts.data_ptr(),
                                   outl.data_ptr(), _stream(stream)), "tsa_stats_static")
    torch.cuda.synchronize(t.device)
    return _rec(results_to_numpy(out)[0]), counts, outl


def quantile(t, q: float, region=None, digits: int = 3, stream=None):
    """Lower q-quantile (rank floor(q (n-1))).  Returns (value, width, count):
    the exact value lies in [value, value + width] (width 0 when digits = 3)."""
    torch = _torch()
    c, reg = cube_of(t), region_of(region)
    ws = workspace(OP_QUANTILE, t, region)
    out = torch.empty(3, dtype=torch.float64, device=t.device)
    _check(capi().tsa_quantile(ctypes.byref(c), _rp(reg), q, digits, out.data_ptr(), ws.data_ptr(), ws.numel(),
                               _stream(stream)), "tsa_quantile")
    torch.cuda.synchronize(t.device)
    v = out.cpu().tolist()
    return v[0], v[1], int(v[2])


def mad(t, region=None, stream=None):
    """Median absolute deviation.  Returns (median, mad, count)."""
    torch = _torch()
    c, reg = cube_of(t), region_of(region)
    ws = workspace(OP_MAD, t, region)
    out = torch.empty(3, dtype=torch.float64, device=t.device)
    _check(capi().tsa_mad(ctypes.byref(c), _rp(reg), out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)),
           "tsa_mad")
    torch.cuda.synchronize(t.device)
    v = out.cpu().tolist()
    return v[0], v[1], int(v[2])


def region_batch(t, regions, nbins: int, tune: Optional[Sequence[int]] = None, stream=None, ws=None):
    """Batched region queries.  regions: int64 [nq, 6] (host or device).

    Returns (numpy record array of nq results, hists int64 tensor [nq, nbins])."""
    torch = _torch()
    c = cube_of(t)
    reg = torch.as_tensor(regions, dtype=torch.int64).to(t.device).contiguous()
    nq = reg.shape[0]
    if ws is None:
        ws = workspace(OP_REGION_BATCH, t, None, nbins, nq)
    out = torch.empty(72 * nq, dtype=torch.uint8, device=t.device)
    hists = torch.empty((nq, nbins), dtype=torch.int64, device=t.device)
    tp = ctypes.byref(Tune(*tune)) if tune is not None else None
    _check(capi().tsa_region_batch(ctypes.byref(c), reg.data_ptr(), nq, nbins, out.data_ptr(), hists.data_ptr(), tp,
                                   ws.data_ptr(), ws.numel(), _stream(stream)), "tsa_region_batch")
    torch.cuda.synchronize(t.device)
    return results_to_numpy(out), hists


def tune_region_batch(t, regions, nbins: int, reps: int = 3, stream=None):
    """Run the autotuner on this batch; returns ((tile_voxels, block_threads,
    blocks_per_cu, cand_max, replicas), best ms).  Later region_batch calls of
    the same shape class use the choice when no tune is given."""
    torch = _torch()
    c = cube_of(t)
    reg = torch.as_tensor(regions, dtype=torch.int64).to(t.device).contiguous()
    nq = reg.shape[0]
    ws = workspace(OP_REGION_BATCH, t, None, nbins, nq)
    out = torch.empty(72 * nq, dtype=torch.uint8, device=t.device)
    hists = torch.empty((nq, nbins), dtype=torch.int64, device=t.device)
    best = Tune()
    ms = ctypes.c_float()
    _check(capi().tsa_tune_region_batch(ctypes.byref(c), reg.data_ptr(), nq, nbins, out.data_ptr(), hists.data_ptr(),
                                        ws.data_ptr(), ws.numel(), _stream(stream), reps, ctypes.byref(best),
                                        ctypes.byref(ms)), "tsa_tune_region_batch")
    return (best.tile_voxels, best.block_threads, best.blocks_per_cu, best.cand_max, best.replicas), ms.value


def batch_last_config():
    """(tile units requested, blocks per CU, LDS replicas per bin, candidate
    cap) of the last region batch this thread enqueued (testing support)."""
    out = (ctypes.c_int32 * 4)()
    _check(capi().lib.tsa_internal_batch_last_config(out), "tsa_internal_batch_last_config")
    return tuple(out)


def minimap(t, cell: Sequence[int], nbins: int, stream=None, ws=None):
    """Statistical mini-map: cells of cell = (cx, cy, cz) voxels, x fastest.

    Returns (numpy record array of the cells' results, hists int64 tensor
    [ncells, nbins], the device result buffer for sigma_count)."""
    torch = _torch()
    c = cube_of(t)
    cx, cy, cz = (int(v) for v in cell)
    ncells = capi().tsa_minimap_cells(ctypes.byref(c), cx, cy, cz)
    _check(int(ncells) if ncells < 0 else TSA_OK, "tsa_minimap_cells")
    if ws is None:
        nb = capi().tsa_minimap_workspace_bytes(ctypes.byref(c), cx, cy, cz, nbins)
        if nb == 0:
            raise TsaError(TSA_EINVAL, "tsa_minimap_workspace_bytes")
        ws = torch.empty(nb, dtype=torch.uint8, device=t.device)
    out = torch.empty(72 * ncells, dtype=torch.uint8, device=t.device)
    hists = torch.empty((ncells, nbins), dtype=torch.int64, device=t.device)
    _check(capi().tsa_minimap(ctypes.byref(c), cx, cy, cz, nbins, out.data_ptr(), hists.data_ptr(), ws.data_ptr(),
                              ws.numel(), _stream(stream)), "tsa_minimap")
    torch.cuda.synchronize(t.device)
    return results_to_numpy(out), hists, out


def sigma_count(t, cell: Sequence[int], cells_dev, k: float, stream=None):
    """Per mini-map cell, the voxels above its mean + k*std; cells_dev is the
    device result buffer that minimap returned.  Returns a uint64 numpy array."""
    torch = _torch()
    c = cube_of(t)
    cx, cy, cz = (int(v) for v in cell)
    ncells = capi().tsa_minimap_cells(ctypes.byref(c), cx, cy, cz)
    _check(int(ncells) if ncells < 0 else TSA_OK, "tsa_minimap_cells")
    above = torch.empty(ncells, dtype=torch.int64, device=t.device)
    _check(capi().tsa_sigma_count(ctypes.byref(c), cx, cy, cz, cells_dev.data_ptr(), float(k), above.data_ptr(),
                                  _stream(stream)), "tsa_sigma_count")
    torch.cuda.synchronize(t.device)
    return above.cpu().numpy().view(np.uint64)


def spectrum(t, rays, nsamples: int, stream=None):
    """Trilinear samples along rays.  rays: float64 [nrays, 6] = origin (x, y, z)
    and step (x, y, z) in voxel units.  Returns a float64 tensor [nrays, nsamples]."""
    torch = _torch()
    c = cube_of(t)
    r = torch.as_tensor(rays, dtype=torch.float64).reshape(-1, 6).to(t.device).contiguous()
    out = torch.empty((r.shape[0], nsamples), dtype=torch.float64, device=t.device)
    _check(capi().tsa_spectrum(ctypes.byref(c), r.data_ptr(), r.shape[0], nsamples, out.data_ptr(), _stream(stream)),
           "tsa_spectrum")
    torch.cuda.synchronize(t.device)
    return out


def version() -> str:
    return capi().tsa_version().decode()
