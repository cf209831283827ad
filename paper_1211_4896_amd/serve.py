"""Python binding of the serving engine (include/tsa_serve.h): argument
marshalling only; the scheduler runs in libtsa.so's own thread."""
from __future__ import annotations

import ctypes
import json
from typing import Optional, Sequence

import numpy as np

from . import TSA_OK, Cube, Region, TsaError, capi, cube_of, status_string

REQ_REGION, REQ_FULL_HIST, REQ_FULL_MEDIAN = 0, 1, 2


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("region_lanes", ctypes.c_int32), ("max_admitted", ctypes.c_int32),
                ("region_nbins", ctypes.c_int32), ("full_nbins", ctypes.c_int32),
                ("full_chunk_kvoxels", ctypes.c_int32),
                ("scratch_bytes", ctypes.c_size_t)]


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("nan_count", ctypes.c_uint64), ("mean", ctypes.c_double),
                ("m2", ctypes.c_double), ("std", ctypes.c_double), ("min", ctypes.c_double),
                ("max", ctypes.c_double), ("median", ctypes.c_double), ("status", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("cube", ctypes.c_int32), ("kind", ctypes.c_int32), ("region", Region),
                ("h_hist", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class Response(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("result", _Result), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double),
                ("kind", ctypes.c_int32), ("status", ctypes.c_int32)]


def _bind():
    api = capi()
    lib = api.lib
    if getattr(api, "_serve_bound", False):
        return lib
    P = ctypes.c_void_p
    sigs = {
        "tsa_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]),
        "tsa_server_add_cube": (ctypes.c_int, [P, ctypes.POINTER(Cube), ctypes.POINTER(ctypes.c_int32)]),
        "tsa_server_submit": (ctypes.c_int, [P, ctypes.POINTER(Request)]),
        "tsa_server_poll": (ctypes.c_int, [P, ctypes.POINTER(Response), ctypes.c_int32]),
        "tsa_server_drain": (ctypes.c_int, [P, ctypes.c_double]),
        "tsa_server_replay": (ctypes.c_int, [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_int32, ctypes.POINTER(Response)]),
        "tsa_server_stats": (ctypes.c_int, [P, ctypes.c_char_p, ctypes.c_size_t]),
        "tsa_server_destroy": (ctypes.c_int, [P]),
        "tsa_server_now": (ctypes.c_double, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    api._serve_bound = True
    return lib


def response_dict(r: Response) -> dict:
    res = {k: getattr(r.result, k) for k, _ in _Result._fields_}
    return {"tag": r.tag, "kind": r.kind, "status": r.status, "result": res, "t_submit": r.t_submit,
            "t_admit": r.t_admit, "t_launch": r.t_launch, "t_done": r.t_done}


class Server:
    """A serving engine over resident cubes (torch tensors kept alive here)."""

    def __init__(self, max_batch=1024, region_lanes=2, max_admitted=4096, region_nbins=256, full_nbins=4096,
                 scratch_bytes=0, full_chunk_kvoxels=0):
        self.lib = _bind()
        self.cfg = ServerConfig(max_batch, region_lanes, max_admitted, region_nbins, full_nbins, full_chunk_kvoxels,
                                scratch_bytes)
        h = ctypes.c_void_p()
        st = self.lib.tsa_server_create(ctypes.byref(self.cfg), ctypes.byref(h))
        if st != TSA_OK:
            raise TsaError(st, "tsa_server_create")
        self.h = h
        self._cubes = []

    def add_cube(self, t) -> int:
        c = cube_of(t)
        cid = ctypes.c_int32()
        st = self.lib.tsa_server_add_cube(self.h, ctypes.byref(c), ctypes.byref(cid))
        if st != TSA_OK:
            raise TsaError(st, "tsa_server_add_cube")
        self._cubes.append(t)
        return cid.value

    @staticmethod
    def request(cube: int, kind: int, region: Optional[Sequence[int]] = None, hist: Optional[np.ndarray] = None,
                tag: int = 0) -> Request:
        reg = Region(*(int(v) for v in region)) if region is not None else Region(0, 0, 0, 0, 0, 0)
        hp = hist.ctypes.data if hist is not None else None
        return Request(cube, kind, reg, hp, tag)

    def submit(self, req: Request):
        st = self.lib.tsa_server_submit(self.h, ctypes.byref(req))
        if st != TSA_OK:
            raise TsaError(st, "tsa_server_submit")

    def poll(self, cap: int = 1024):
        buf = (Response * cap)()
        n = self.lib.tsa_server_poll(self.h, buf, cap)
        if n < 0:
            raise TsaError(n, "tsa_server_poll")
        return [buf[i] for i in range(n)]

    def drain(self, timeout_s: float = 0.0):
        st = self.lib.tsa_server_drain(self.h, timeout_s)
        if st != TSA_OK:
            raise TsaError(st, "tsa_server_drain")

    def replay(self, reqs: Sequence[Request], t_arrival: np.ndarray):
        n = len(reqs)
        arr = (Request * n)(*reqs)
        ta = np.ascontiguousarray(t_arrival, dtype=np.float64)
        out = (Response * n)()
        st = self.lib.tsa_server_replay(self.h, arr, ta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, out)
        if st != TSA_OK:
            raise TsaError(st, "tsa_server_replay")
        return out

    def stats(self) -> dict:
        buf = ctypes.create_string_buffer(1024)
        n = self.lib.tsa_server_stats(self.h, buf, len(buf))
        if n < 0:
            raise TsaError(n, "tsa_server_stats")
        return json.loads(buf.value.decode())

    def close(self):
        if self.h:
            self.lib.tsa_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def poisson_arrivals(rate_qps: float, n: int, seed: int) -> np.ndarray:
    """Open-loop arrival times (seconds from 0): seeded exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_qps, n))


def status_text(st: int) -> str:
    return status_string(st)
