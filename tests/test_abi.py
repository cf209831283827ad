"""The C ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before touching the device (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1211_4896_amd as tsa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(tsa_[a-z0-9_]+)\s*\(", src))
    return names


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(tsa.LIB_PATH)
    names = _declared()
    assert {"tsa_moments", "tsa_histogram", "tsa_median", "tsa_stats", "tsa_region_batch",
            "tsa_workspace_bytes"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_status_strings_and_version():
    assert tsa.status_string(tsa.TSA_OK) == "ok"
    assert tsa.status_string(tsa.TSA_EINVAL) == "invalid argument"
    assert "gfx950" in tsa.version()


@pytest.mark.parametrize("d", [1, 2, 3, 5, 7, 48, 129, 512, 4095, 65537, 1000003, (1 << 31) - 1, 1 << 30])
def test_magic_division(d):
    c = tsa.capi()
    for n in [0, 1, d - 1, d, d + 1, 2 * d + 5, 123456789, (1 << 32) - 1, (1 << 31) + 7]:
        n &= 0xFFFFFFFF
        assert c.tsa_internal_magic_div(n, d) == n // d, (n, d)


def _cube(nx=8, ny=4, nz=2, dtype=tsa.TSA_F32, ptr=0x10000):
    return tsa.Cube(ptr, dtype, 0, nx, ny, nz)


def test_workspace_bytes_checks():
    c = tsa.capi()
    cube = _cube()
    assert c.tsa_workspace_bytes(tsa.OP_MOMENTS, ctypes.byref(cube), None, 0, 0) > 0
    assert c.tsa_workspace_bytes(tsa.OP_HISTOGRAM, ctypes.byref(cube), None, 0, 0) == 0  # nbins 0
    assert c.tsa_workspace_bytes(tsa.OP_HISTOGRAM, ctypes.byref(cube), None, 65537, 0) == 0
    bad = tsa.Region(0, 0, 0, 9, 1, 1)
    assert c.tsa_workspace_bytes(tsa.OP_MEDIAN, ctypes.byref(cube), ctypes.byref(bad), 0, 0) == 0
    nul = tsa.Cube(0, 0, 0, 8, 4, 2)
    assert c.tsa_workspace_bytes(tsa.OP_MOMENTS, ctypes.byref(nul), None, 0, 0) == 0
    i8 = tsa.Cube(0x10000, 7, 0, 8, 4, 2)
    assert c.tsa_workspace_bytes(tsa.OP_MOMENTS, ctypes.byref(i8), None, 0, 0) == 0


@pytest.mark.parametrize("reg", [(0, 0, 0, 0, 1, 1), (0, 0, 0, 9, 1, 1), (-1, 0, 0, 1, 1, 1), (2, 0, 0, 1, 1, 1),
                                 (0, 0, 0, 1, 5, 1), (0, 0, 1, 1, 1, 1)])
def test_bad_regions_rejected_before_launch(reg):
    c = tsa.capi()
    cube = _cube()
    r = tsa.Region(*reg)
    ws = 0x20000
    assert c.tsa_moments(ctypes.byref(cube), ctypes.byref(r), 0x30000, ws, 1 << 30, None) == tsa.TSA_EINVAL
    assert c.tsa_median(ctypes.byref(cube), ctypes.byref(r), 0x30000, ws, 1 << 30, None) == tsa.TSA_EINVAL


@pytest.mark.parametrize("lo,hi,nb", [(0.0, 1.0, 0), (0.0, 1.0, 65537), (1.0, 0.0, 8), (float("nan"), 1.0, 8),
                                      (0.0, float("inf"), 8), (-3.0e38, 3.0e38, 8), (0.0, 1e-45, 65536)])
def test_bad_histogram_ranges_rejected(lo, hi, nb):
    c = tsa.capi()
    cube = _cube()
    st = c.tsa_histogram(ctypes.byref(cube), None, lo, hi, nb, 0x40000, 0x50000, 0x20000, 1 << 30, None)
    assert st == tsa.TSA_EINVAL


def test_null_pointers_rejected():
    c = tsa.capi()
    cube = _cube()
    assert c.tsa_moments(ctypes.byref(cube), None, None, 0x20000, 1 << 30, None) == tsa.TSA_EINVAL
    assert c.tsa_histogram(ctypes.byref(cube), None, 0.0, 1.0, 8, None, None, 0x20000, 1 << 30, None) == tsa.TSA_EINVAL
    assert c.tsa_moments(None, None, 0x30000, 0x20000, 1 << 30, None) == tsa.TSA_EINVAL
    assert c.tsa_stats(ctypes.byref(cube), None, 0, 0x30000, 0x40000, None, 0x20000, 1 << 30, None) == tsa.TSA_EINVAL


def test_server_config_rejected_before_device():
    from paper_1211_4896_amd import serve
    lib = serve._bind()
    h = ctypes.c_void_p()
    for bad in [serve.ServerConfig(0, 1, 1, 8, 8, 0, 0), serve.ServerConfig(8, 0, 1, 8, 8, 0, 0),
                serve.ServerConfig(8, 5, 1, 8, 8, 0, 0), serve.ServerConfig(8, 1, 0, 8, 8, 0, 0),
                serve.ServerConfig(8, 1, 1, 5000, 8, 0, 0), serve.ServerConfig(8, 1, 1, 8, 70000, 0, 0),
                serve.ServerConfig(8, 1, 1, 8, 8, -1, 0)]:
        assert lib.tsa_server_create(ctypes.byref(bad), ctypes.byref(h)) == tsa.TSA_EINVAL
    assert lib.tsa_server_now() > 0


def test_batch_workspace_bytes():
    c = tsa.capi()
    cube = _cube(64, 64, 64)
    n1 = c.tsa_workspace_bytes(tsa.OP_REGION_BATCH, ctypes.byref(cube), None, 256, 1)
    n2 = c.tsa_workspace_bytes(tsa.OP_REGION_BATCH, ctypes.byref(cube), None, 256, 4096)
    assert 0 < n1 < n2
    assert c.tsa_workspace_bytes(tsa.OP_REGION_BATCH, ctypes.byref(cube), None, 4097, 8) == 0
    assert c.tsa_workspace_bytes(tsa.OP_REGION_BATCH, ctypes.byref(cube), None, 256, 65537) == 0


def test_tune_cache_roundtrip(tmp_path):
    c = tsa.capi()
    p = tmp_path / "tune.json"
    # entries of four numbers (written before the replica count was tuned) load with replicas 0
    p.write_text('{\n  "gfx950|f32|nbins=256|nq2=12": [65536, 256, 4, 65536],\n'
                 '  "gfx950|i16|nbins=128|nq2=3": [16384, 256, 8, 0, 2]\n}\n')
    assert c.tsa_tune_load(str(p).encode()) == 2
    q = tmp_path / "out.json"
    assert c.tsa_tune_save(str(q).encode()) == 0
    txt = q.read_text()
    assert '"gfx950|f32|nbins=256|nq2=12": [65536, 256, 4, 65536, 0]' in txt
    assert '"gfx950|i16|nbins=128|nq2=3": [16384, 256, 8, 0, 2]' in txt
    assert c.tsa_tune_load(str(tmp_path / "missing.json").encode()) == tsa.TSA_EINVAL


def test_minimap_grid_and_workspace():
    c = tsa.capi()
    cube = _cube(100, 64, 61)
    assert c.tsa_minimap_cells(ctypes.byref(cube), 30, 30, 30) == 4 * 3 * 3
    assert c.tsa_minimap_cells(ctypes.byref(cube), 1000, 1000, 1000) == 1
    assert c.tsa_minimap_cells(ctypes.byref(cube), 0, 30, 30) == tsa.TSA_EINVAL
    assert c.tsa_minimap_cells(ctypes.byref(cube), 1, 1, 1) == tsa.TSA_EINVAL  # 390400 cells
    n1 = c.tsa_minimap_workspace_bytes(ctypes.byref(cube), 30, 30, 30, 64)
    n2 = c.tsa_workspace_bytes(tsa.OP_REGION_BATCH, ctypes.byref(cube), None, 64, 36)
    assert n1 >= n2 + 36 * 48 > 0
    assert c.tsa_minimap_workspace_bytes(ctypes.byref(cube), 30, 30, 30, 0) == 0
    assert c.tsa_minimap_workspace_bytes(ctypes.byref(cube), 30, 30, 30, 4097) == 0
    # argument errors come back before anything is launched
    dummy = ctypes.c_void_p(16)
    assert c.tsa_minimap(ctypes.byref(cube), 30, 30, 30, 64, dummy, dummy, dummy, 16, None) == tsa.TSA_ENOMEM
    assert c.tsa_minimap(ctypes.byref(cube), 30, 30, 30, 64, None, dummy, dummy, n1, None) == tsa.TSA_EINVAL
    assert c.tsa_sigma_count(ctypes.byref(cube), 30, 30, 30, dummy, float("nan"), dummy, None) == tsa.TSA_EINVAL
    assert c.tsa_sigma_count(ctypes.byref(cube), 30, 30, 30, None, 3.0, dummy, None) == tsa.TSA_EINVAL
    big = _cube(70000, 70000, 2)
    assert c.tsa_minimap_cells(ctypes.byref(big), 70000, 70000, 1) == tsa.TSA_EINVAL  # cell >= 2^32 voxels


def test_spectrum_arguments_checked_on_host():
    c = tsa.capi()
    cube = _cube(16, 16, 16)
    dummy = ctypes.c_void_p(16)
    assert c.tsa_spectrum(ctypes.byref(cube), dummy, -1, 4, dummy, None) == tsa.TSA_EINVAL
    assert c.tsa_spectrum(ctypes.byref(cube), dummy, 4, -1, dummy, None) == tsa.TSA_EINVAL
    assert c.tsa_spectrum(ctypes.byref(cube), None, 4, 4, dummy, None) == tsa.TSA_EINVAL
    assert c.tsa_spectrum(ctypes.byref(cube), dummy, 4, 4, None, None) == tsa.TSA_EINVAL
    assert c.tsa_spectrum(ctypes.byref(cube), None, 0, 4, None, None) == tsa.TSA_OK  # nothing to do
    assert c.tsa_spectrum(ctypes.byref(cube), dummy, 1 << 30, 1 << 30, dummy, None) == tsa.TSA_EINVAL
