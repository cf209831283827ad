#!/usr/bin/env python3
"""Benchmark of the cube-statistics hot path on one MI355X.

A step is one pass of the whole analysis path of the paper's Section 4 over a
resident float32 cube: global moments, the N-bin histogram over [min, max],
and the exact lower median -- one tsa_stats call (two passes over the data
plus small selection kernels).  The headline cube is the largest that fits one
GPU: 4096x4096x3072 (206 GB in HBM, 65536 bins; the 8-way share of a 1.6 TB
cube).  Inputs are synthetic and seeded (noise + Gaussian sources + NaN
slabs) and already resident in HBM when the timed region starts.

Prints one JSON line: whole-step throughput in GVoxel/s, the roofline entry of
the dominant kernel (its duration measured with HIP events on its launch
stream during the timed steps), the separate-call rates of the histogram,
median and moments, the CPU oracle timed on a bounded sample of the same cube
on the host's cores, and, as extra keys, the 1024x1024x1280 cube (one GPU's
share at 96 GPUs), the 256^3 cube, the mini-map, the spectrum tool, batched
region queries and the serving loop.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload c3|c2|c1]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "GVoxel/s + % HBM peak (hist, median); region queries/s batched vs plain, p99"
KERNEL_SOURCES = ["tsa_device.hpp", "tsa_walk.hpp", "tsa_ops.hpp", "tsa_kernels.hip"]
_COMMON = ["tsa_device.hpp", "tsa_walk.hpp", "tsa_ops.hpp"]
# sources whose text decides each profiled kernel's code (a counter summary
# taken on other sources no longer describes the kernel)
SOURCES_FOR = {"batch": _COMMON + ["tsa_batch.hip"], "minimap_cells": _COMMON + ["tsa_minimap.hip"],
               "sigma": _COMMON + ["tsa_minimap.hip"], "spectrum": ["tsa_device.hpp", "tsa_spectrum.hip"]}


def sources_for(kernel: str):
    return SOURCES_FOR.get(kernel, KERNEL_SOURCES)


def _src_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for s in sources:
        with open(os.path.join(ROOT, "paper_1211_4896_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _counter_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("src_sha256_16") != _src_hash(sources_for(kernel)):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _trace(lib, on: bool, cap: int = 0):
    st = lib.tsa_trace_enable(1 if on else 0, cap)
    if st != 0:
        raise RuntimeError(f"tsa_trace_enable failed ({st})")


def _trace_read(lib) -> dict:
    buf = ctypes.create_string_buffer(1 << 16)
    n = lib.tsa_trace_read(buf, len(buf))
    if n < 0:
        raise RuntimeError(f"tsa_trace_read failed ({n})")
    return json.loads(buf.value.decode())


def _cpu_baseline(spec, nbins: int, target_s: float = 1.5, max_planes: int = 256) -> dict:
    """The oracle timed on the host's cores: ``oracle.stats_exact`` (exact sums
    for the moments, the histogram over [min, max], the lower median by a
    two-level key count; the oracle the 206 GB cube is checked against),
    threads over the values, on a z-slab from the middle of the same cube,
    generated outside the timed region.  The slab grows until one run takes
    about target_s seconds of wall time."""
    import oracle
    import synth

    threads = synth.default_threads()
    plane = spec.nx * spec.ny
    planes = max(1, (1 << 24) // plane)
    while True:
        z0 = max(0, spec.nz // 2 - planes // 2)
        z1 = min(spec.nz, z0 + planes)
        host, _ = synth.generate(spec, z0, z1)
        t0 = time.perf_counter()
        oracle.stats_exact(host, nbins, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= target_s or planes >= max_planes or z1 - z0 == spec.nz:
            break
        planes = int(min(max_planes, max(planes + 1, planes * target_s / max(dt, 1e-3) * 1.1)))
        del host
    nvox = (z1 - z0) * plane
    return {"value": round(nvox / dt / 1e9, 4), "unit": "GVoxel/s", "cores": threads, "kind": "oracle",
            "sample": f"z-slices [{z0}, {z1}) of the {spec.nx}x{spec.ny}x{spec.nz} cube ({nvox} voxels), "
                      f"oracle.stats_exact on {threads} threads: moments (exact sums) + {nbins}-bin histogram over "
                      f"[min,max] + lower median (two-level 16+16-bit key count), {dt:.2f} s wall",
            "host_cpus": os.cpu_count()}


def _workload_text(name: str, spec, nbins: int) -> str:
    return (f"{name}: {spec.nx}x{spec.ny}x{spec.nz} float32 cube ({spec.nx * spec.ny * spec.nz * 4 / 1e9:.1f} GB "
            f"resident; seeded noise + {spec.n_sources} Gaussian sources + {spec.nan_frac:.1%} NaN slabs); moments + "
            f"{nbins}-bin histogram over [min,max] + exact lower median (tsa_stats)")


# algorithmic bytes of one launch of the streaming passes of tsa_stats: one read
# of the cube plus the histogram the pass produces (8 bytes per bin)
def _pass_bytes(kernel: str, N: int, nbins: int) -> float:
    if kernel == "pass_a":
        return 4.0 * N + 8.0 * 4096
    if kernel in ("pass_b", "pass_bwin", "pass_b16"):
        return 4.0 * N + 8.0 * nbins
    return 4.0 * N


def _timed_stats(tsa, torch, lib, dev, nbins: int, steps: int, warmup: int, workload: str) -> dict:
    """warmup untimed tsa_stats calls, then exactly `steps` timed ones bracketed
    by device synchronisation; per-kernel times from HIP events on the launch
    stream (tsa_trace); the roofline entry of the dominant kernel."""
    api = tsa.capi()
    c = tsa.cube_of(dev)
    cp = ctypes.byref(c)
    ws = tsa.workspace(tsa.OP_STATS, dev, None, nbins)
    out = torch.empty(72, dtype=torch.uint8, device=dev.device)
    counts = torch.empty(nbins, dtype=torch.int64, device=dev.device)
    outl = torch.empty(2, dtype=torch.int64, device=dev.device)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    def step():
        st = api.tsa_stats(cp, None, nbins, out.data_ptr(), counts.data_ptr(), outl.data_ptr(), ws.data_ptr(),
                           ws.numel(), sh)
        if st != 0:
            raise RuntimeError(f"tsa_stats failed: {tsa.status_string(st)}")

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    _trace(lib, True, cap=steps * 32)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    ev_ms = e0.elapsed_time(e1) / steps
    kern = _trace_read(lib)
    _trace(lib, False)
    res = tsa.results_to_numpy(out)[0]
    if res["status"] != 0:
        raise RuntimeError("device status %d" % res["status"])
    N = dev.numel()
    dom_name, (dom_n, dom_tot, _, _) = max(kern.items(), key=lambda kv: kv[1][1])
    dom_avg_ms = dom_tot / dom_n
    per_launch = _pass_bytes(dom_name, N, nbins)
    achieved = per_launch / (dom_avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _counter_traffic(dom_name, workload),
                "kernel": dom_name, "avg_ms": round(dom_avg_ms, 4), "bytes_per_launch": per_launch}
    probe = _read_probe(lib, dev, sh, torch)
    roofline["achievable_read_GBps"] = probe["GBps"]
    roofline["frac_of_achievable"] = round(achieved / probe["GBps"], 4)
    hist_total = int(counts.sum().item()) + int(outl.sum().item())
    return {"ms_per_step": wall_ms, "event_ms_per_step": round(ev_ms, 4), "roofline": roofline,
            "kernels_ms": {k: round(v[1] / v[0], 4) for k, v in kern.items()}, "res": res,
            "checks": {"count_plus_nan_is_N": int(res["count"]) + int(res["nan_count"]) == N,
                       "hist_total_is_count": hist_total == int(res["count"])},
            "api": api, "cp": cp, "sh": sh}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"],
                    help="headline cube: c3 = 4096x4096x3072 (206 GB, 65536 bins), c2 = 1024x1024x1280 "
                         "(5.4 GB, 4096 bins), c1 = 256^3 (1024 bins)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ops", action="store_true", help="skip the separate-call measurements")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run 3 plain 1 GiB device copies (reference dispatches for byte counters)")
    ap.add_argument("--no-c2", action="store_true", help="skip the 1024x1024x1280 cube and what runs on it "
                                                         "(mini-map, spectrum) when it is not the headline")
    ap.add_argument("--no-region", action="store_true", help="skip the batched-vs-plain region queries (c4)")
    ap.add_argument("--region-reps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run (c5)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-warmup", type=float, default=10.0)
    ap.add_argument("--serve-qps", type=float, default=2000.0)
    ap.add_argument("--serve-chunk-kvoxels", type=int, default=0,
                    help="voxels (x1024) per launch of a full-cube scan's passes in the serving run (0: one launch)")
    ap.add_argument("--no-minimap", action="store_true", help="skip the mini-map + k-sigma measurement")
    ap.add_argument("--no-spectrum", action="store_true", help="skip the spectrum-tool measurement")
    ap.add_argument("--no-c1", action="store_true", help="skip the 256^3 cache-resident case")
    ap.add_argument("--hw-queues", type=int, default=8,
                    help="raise the process's hardware queues to at least this many (0: leave the environment's)")
    args = ap.parse_args()
    # The serving run keeps three streams busy at once (two region lanes and the
    # full-scan lane) beside torch's own.  With HIP's default of four hardware
    # queues per process a region lane can land on the full-scan lane's queue and
    # wait behind its kernels (region service p99 5.3 ms against 2.4 ms with eight
    # queues); a server process is configured with a queue per stream.  Read by
    # the HIP runtime when it starts, so it is set before anything touches the GPU.
    if args.hw_queues > 0:
        try:
            have = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
        except ValueError:
            have = 4
        if have < args.hw_queues:
            os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this path does not shard)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1211_4896_amd as tsa

    lib = tsa.capi().lib
    lib.tsa_trace_enable.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.tsa_trace_read.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    NBINS = {"c1": 1024, "c2": 4096, "c3": 65536}

    def load(name):
        spec = synth.SPECS[name]
        t0 = time.perf_counter()
        if name == "c3":
            dev, _ = generate_on_device(synth, torch, spec)
        else:
            host, _ = synth.generate(spec)
            dev = torch.from_numpy(host).to("cuda:0")
            del host
        torch.cuda.synchronize()
        print(f"[bench] {name}: generated {spec.nx}x{spec.ny}x{spec.nz} in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        return spec, dev

    head = args.workload
    nbins = NBINS[head]
    spec, dev = load(head)
    N = dev.numel()
    t = _timed_stats(tsa, torch, lib, dev, nbins, args.steps, args.warmup, head)
    ms_per_step = t["ms_per_step"]
    line = {"metric": METRIC, "value": round(N / (ms_per_step * 1e-3) / 1e9, 2), "unit": "GVoxel/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": _workload_text(head, spec, nbins), "voxels": N, "nbins": nbins, "parallelism": "1 GPU"},
            "roofline": t["roofline"], "event_ms_per_step": t["event_ms_per_step"], "kernels_ms": t["kernels_ms"],
            "checks": t["checks"]}
    print(f"[bench] {head}: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)
    res = t["res"]
    if not args.no_ops:
        line["ops"] = _separate_ops(tsa, t["api"], dev, t["cp"], N, float(res["min"]), float(res["max"]), nbins,
                                    t["sh"])
    if args.calib_copy:
        line["calib_copy_bytes"] = _calib_copy(lib, dev.device, t["sh"])
    if head != "c2":
        del dev, t
        torch.cuda.empty_cache()
        dev = None
        if not args.no_c2:
            _, dev = load("c2")
            t2 = _timed_stats(tsa, torch, lib, dev, 4096, args.steps, args.warmup, "c2")
            line["c2"] = {"workload": _workload_text("c2", synth.SPECS["c2"], 4096),
                          "ms_per_step": round(t2["ms_per_step"], 4),
                          "gvoxel_s": round(dev.numel() / (t2["ms_per_step"] * 1e-3) / 1e9, 2),
                          "roofline": t2["roofline"], "kernels_ms": t2["kernels_ms"], "checks": t2["checks"]}
            if not args.no_ops:
                r2 = t2["res"]
                line["c2"]["ops"] = _separate_ops(tsa, t2["api"], dev, t2["cp"], dev.numel(), float(r2["min"]),
                                                  float(r2["max"]), 4096, t2["sh"])
            del t2
    sh = torch.cuda.current_stream().cuda_stream
    if not args.no_c1 and head != "c1":
        line["c1"] = _c1_bench(tsa, torch, synth, lib, sh)
    if dev is not None and dev.numel() == synth.SPECS["c2"].n:
        api = tsa.capi()
        if not args.no_minimap:
            # 2 ms calls: 20 of them, so one slow call does not move the mean much
            line["minimap"] = _minimap_bench(tsa, torch, api, lib, dev, sh, max(args.region_reps, 20))
        if not args.no_spectrum:
            line["spectrum"] = _spectrum_bench(tsa, torch, np, synth, api, lib, dev, sh, args.region_reps)
    dev = None
    torch.cuda.empty_cache()
    if not args.no_region:
        line["region_batch"] = _region_batch_bench(tsa, torch, np, synth, args.region_reps)
        torch.cuda.empty_cache()
    if not args.no_serve:
        line["serving"] = _serving_bench(torch, np, synth, args.serve_seconds, args.serve_qps, args.serve_warmup,
                                         args.serve_chunk_kvoxels)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = _cpu_baseline(spec, nbins)
    print(json.dumps(line), flush=True)


def _region_batch_bench(tsa, torch, np, synth, reps: int) -> dict:
    """c4: 4096 boxes (edges log-uniform [8,512]) on a resident 2048^3 float32
    cube, each getting moments + 256-bin histogram over its own [min,max] +
    median.  Batched = one tsa_region_batch call (one persistent launch).
    Plain = the same library per box: tsa_moments, host sync and read of
    min/max, tsa_histogram, tsa_median, host sync."""
    spec = synth.SPECS["c4"]
    t0 = time.perf_counter()
    host, _ = synth.generate(spec)
    t_gen = time.perf_counter() - t0
    dev = torch.from_numpy(host).to("cuda:0")
    del host
    torch.cuda.synchronize()
    nq, nbins = 4096, 256
    boxes = synth.regions(nq, (spec.nx, spec.ny, spec.nz), seed=2024, edge_lo=8, edge_hi=512)
    vox = int(np.prod(boxes[:, 3:] - boxes[:, :3], axis=1).sum())
    d_boxes = torch.from_numpy(boxes).to(dev.device)
    ws = tsa.workspace(tsa.OP_REGION_BATCH, dev, None, nbins, nq)
    res_buf = torch.empty(72 * nq, dtype=torch.uint8, device=dev.device)
    hists = torch.empty((nq, nbins), dtype=torch.int64, device=dev.device)
    api = tsa.capi()
    c = tsa.cube_of(dev)
    sh = torch.cuda.current_stream().cuda_stream

    def batch():
        st = api.tsa_region_batch(ctypes.byref(c), d_boxes.data_ptr(), nq, nbins, res_buf.data_ptr(),
                                  hists.data_ptr(), None, ws.data_ptr(), ws.numel(), sh)
        if st != 0:
            raise RuntimeError(f"tsa_region_batch: {tsa.status_string(st)}")

    batch()
    torch.cuda.synchronize()
    # untuned (library defaults), then the autotuner's choice for this batch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch()
    e1.record()
    torch.cuda.synchronize()
    default_ms = e0.elapsed_time(e1) / reps
    t0 = time.perf_counter()
    best, best_ms = tsa.tune_region_batch(dev, d_boxes, nbins, reps=2)
    t_tune = time.perf_counter() - t0
    batch()  # the tuned choice is now the library's choice for this shape class
    torch.cuda.synchronize()
    lib = api.lib
    e0.record()
    for _ in range(reps):
        batch()  # replays of the captured launch graph
    e1.record()
    torch.cuda.synchronize()
    b_ms = e0.elapsed_time(e1) / reps
    _trace(lib, True, cap=reps * 16)  # eager launches, each kernel bracketed by events
    for _ in range(reps):
        batch()
    torch.cuda.synchronize()
    kern = _trace_read(lib)
    _trace(lib, False)
    res = tsa.results_to_numpy(res_buf)
    bad = int(np.count_nonzero(res["status"] != 0))
    phase3 = int(np.count_nonzero(res["flags"] & tsa.FLAG_PHASE3))

    # plain per-query path over the same boxes
    ws1 = torch.empty(max(api.tsa_workspace_bytes(op, ctypes.byref(c), None, nbins, 0) for op in (0, 1, 2)),
                      dtype=torch.uint8, device=dev.device)
    out = torch.empty(72, dtype=torch.uint8, device=dev.device)
    counts = torch.empty(nbins, dtype=torch.int64, device=dev.device)
    outl = torch.empty(2, dtype=torch.int64, device=dev.device)
    host_out = torch.empty(72, dtype=torch.uint8, pin_memory=True)

    def plain(b):
        reg = tsa.Region(*(int(v) for v in b))
        rp = ctypes.byref(reg)
        api.tsa_moments(ctypes.byref(c), rp, out.data_ptr(), ws1.data_ptr(), ws1.numel(), sh)
        host_out.copy_(out)  # synchronous: min/max needed on the host
        r = host_out.numpy().view(tsa.RESULT_DTYPE)[0]
        if r["count"] > 0 and np.isfinite(r["min"]) and np.isfinite(r["max"]):
            api.tsa_histogram(ctypes.byref(c), rp, float(r["min"]), float(r["max"]), nbins, counts.data_ptr(),
                              outl.data_ptr(), ws1.data_ptr(), ws1.numel(), sh)
        api.tsa_median(ctypes.byref(c), rp, out.data_ptr(), ws1.data_ptr(), ws1.numel(), sh)
        host_out.copy_(out)

    for b in boxes[:16]:
        plain(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in boxes:
        plain(b)
    torch.cuda.synchronize()
    p_s = time.perf_counter() - t0
    batched_qps = nq / (b_ms * 1e-3)
    plain_qps = nq / p_s
    kb = kern.get("batch", [1, b_ms, 0, 0])
    batch_kernel_ms = kb[1] / kb[0]
    return {"workload": "c4: 2048^3 float32 cube (noise + sources + 0.5% NaN), 4096 boxes, edges round(exp U[ln 8, "
                        "ln 512]) per axis; moments + 256-bin histogram over own [min,max] + exact median each",
            "queries": nq, "voxels_per_batch": vox, "batched_ms": round(b_ms, 3),
            "batched_qps": round(batched_qps, 1), "plain_qps": round(plain_qps, 1),
            "ratio": round(batched_qps / plain_qps, 2),
            "batched_gvoxel_s": round(vox / (b_ms * 1e-3) / 1e9, 1),
            "persistent_kernel_ms": round(batch_kernel_ms, 3),
            "hbm_frac_2_passes": round(2 * 4.0 * vox / (batch_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic_bytes_per_launch": _counter_traffic("batch", "c4"),
            "kernels_ms": {k: round(v[1] / v[0], 4) for k, v in kern.items()},
            "status_errors": bad, "phase3_queries": phase3, "generate_s": round(t_gen, 1),
            "untuned_ms": round(default_ms, 3), "tuned": {"tile_voxels": best[0], "block_threads": best[1],
                                                          "blocks_per_cu": best[2], "cand_max": best[3],
                                                          "replicas": best[4],
                                                          "tuner_best_ms": round(best_ms, 3),
                                                          "tuning_s": round(t_tune, 1)}}


def _minimap_bench(tsa, torch, api, lib, dev, sh, reps: int) -> dict:
    """The statistical mini-map of the resident cube: 30x30x30-voxel cells
    (the partition size of the paper's sigma-clipping example), each with
    moments + 64-bin histogram over its own [min,max] + median, then the
    local 3-sigma counts."""
    cell, nbins, k = MINIMAP_CELL, MINIMAP_NBINS, MINIMAP_K
    c = tsa.cube_of(dev)
    cp = ctypes.byref(c)
    ncells = int(api.tsa_minimap_cells(cp, *cell))
    ws = torch.empty(api.tsa_minimap_workspace_bytes(cp, *cell, nbins), dtype=torch.uint8, device=dev.device)
    cells = torch.empty(72 * ncells, dtype=torch.uint8, device=dev.device)
    hists = torch.empty((ncells, nbins), dtype=torch.int64, device=dev.device)
    above = torch.empty(ncells, dtype=torch.int64, device=dev.device)

    def mm():
        st = api.tsa_minimap(cp, *cell, nbins, cells.data_ptr(), hists.data_ptr(), ws.data_ptr(), ws.numel(), sh)
        if st != 0:
            raise RuntimeError(f"tsa_minimap: {tsa.status_string(st)}")

    def sig():
        st = api.tsa_sigma_count(cp, *cell, cells.data_ptr(), k, above.data_ptr(), sh)
        if st != 0:
            raise RuntimeError(f"tsa_sigma_count: {tsa.status_string(st)}")

    mm()
    sig()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        mm()
    e1.record(stream)
    torch.cuda.synchronize()
    mm_ms = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        sig()
    e1.record(stream)
    torch.cuda.synchronize()
    sig_ms = e0.elapsed_time(e1) / reps
    _trace(lib, True, cap=reps * 16)
    for _ in range(reps):
        mm()
        sig()
    torch.cuda.synchronize()
    kern = _trace_read(lib)
    _trace(lib, False)
    res = tsa.results_to_numpy(cells)
    N = dev.numel()
    ks = kern.get("sigma", [1, sig_ms, 0, 0])
    sig_kernel_ms = ks[1] / ks[0]
    sig_bytes = 4.0 * N + 8.0 * ncells
    return {"workload": f"mini-map of the resident {c.nx}x{c.ny}x{c.nz} float32 cube: {ncells} cells of "
                        f"30x30x30 voxels, moments + {nbins}-bin histogram over own [min,max] + median each; "
                        f"then per-cell counts above mean + 3 std",
            "cells": ncells, "minimap_ms": round(mm_ms, 3), "minimap_gvoxel_s": round(N / (mm_ms * 1e-3) / 1e9, 1),
            "cells_per_s": round(ncells / (mm_ms * 1e-3), 1),
            "sigma_ms": round(sig_ms, 4), "sigma_kernel_ms": round(sig_kernel_ms, 4),
            "sigma_hbm_frac": round(sig_bytes / (sig_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernels_ms": {kk: round(v[1] / v[0], 4) for kk, v in kern.items()},
            "status_errors": int((res["status"] != 0).sum()), "above_total": int(above.sum().item())}


SPECTRUM_RAYS, SPECTRUM_SAMPLES, SPECTRUM_SEED = 16384, 2560, 4404
MINIMAP_CELL, MINIMAP_NBINS, MINIMAP_K = (30, 30, 30), 64, 3.0


def _spectrum_bench(tsa, torch, np, synth, api, lib, dev, sh, reps: int) -> dict:
    """The 3-D spectrum tool over the resident cube: 16384 lines of sight
    entering through the z = 0 face at seeded random points, directions within
    45 degrees of the frequency axis, 0.5-voxel steps, 2560 trilinear samples
    each."""
    nrays, nsamples = SPECTRUM_RAYS, SPECTRUM_SAMPLES
    c = tsa.cube_of(dev)
    rays = torch.from_numpy(synth.sight_lines(nrays, (c.nx, c.ny, c.nz), SPECTRUM_SEED)).to(dev.device)
    out = torch.empty((nrays, nsamples), dtype=torch.float64, device=dev.device)

    def run():
        st = api.tsa_spectrum(ctypes.byref(c), rays.data_ptr(), nrays, nsamples, out.data_ptr(), sh)
        if st != 0:
            raise RuntimeError(f"tsa_spectrum: {tsa.status_string(st)}")

    run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    _trace(lib, True, cap=reps * 2)
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    kern = _trace_read(lib)
    _trace(lib, False)
    inside = int(torch.isfinite(out).sum().item())
    ns = nrays * nsamples
    kk = kern.get("spectrum", [1, ms, 0, 0])
    kms = kk[1] / kk[0]
    return {"workload": f"{nrays} rays x {nsamples} samples (0.5-voxel step, within 45 deg of the z axis, entering "
                        f"at z = 0) through the resident {c.nx}x{c.ny}x{c.nz} float32 cube",
            "samples": ns, "inside_samples": inside, "ms": round(ms, 3), "kernel_ms": round(kms, 4),
            "gsamples_s": round(ns / (kms * 1e-3) / 1e9, 2),
            "inside_gsamples_s": round(inside / (kms * 1e-3) / 1e9, 2),
            "out_gb_s": round(8.0 * ns / (kms * 1e-3) / 1e9, 1),
            "gathered_gb_s": round((32.0 * inside + 8.0 * ns) / (kms * 1e-3) / 1e9, 1)}


def _serving_bench(torch, np, synth, seconds: float, qps: float, warm: float = 10.0, chunk_kvoxels: int = 0) -> dict:
    """c5: open-loop Poisson arrivals over three resident cubes (float32 1024^3,
    float32 2048x2048x1024, int16 2048^3): 90% region requests (c4 boxes), 10%
    full-cube requests (half 4096-bin histograms over the cube's [min,max],
    half medians).  Latency = completion - submission."""
    from paper_1211_4896_amd import serve

    names = ["c5a", "c5b", "c5c"]
    devs = []
    for nm in names:
        host, _ = synth.generate(synth.SPECS[nm])
        devs.append(torch.from_numpy(host).to("cuda:0"))
        del host
    torch.cuda.synchronize()
    n = int((warm + seconds) * qps)
    rng = np.random.default_rng(77)
    t_arr = serve.poisson_arrivals(qps, n, seed=78)
    srv = serve.Server(max_batch=1024, region_lanes=2, max_admitted=8192, region_nbins=256, full_nbins=4096,
                       full_chunk_kvoxels=chunk_kvoxels)
    try:
        ids = [srv.add_cube(d) for d in devs]
        reqs = []
        for i in range(n):
            ci = int(rng.integers(0, 3))
            spec = synth.SPECS[names[ci]]
            if rng.random() < 0.1:
                kind = serve.REQ_FULL_HIST if rng.random() < 0.5 else serve.REQ_FULL_MEDIAN
                reqs.append(srv.request(ids[ci], kind, None, None, tag=i))
            else:
                b = synth.regions(1, (spec.nx, spec.ny, spec.nz), seed=1000003 + i, edge_lo=8, edge_hi=512)[0]
                reqs.append(srv.request(ids[ci], serve.REQ_REGION, b, None, tag=i))
        out = srv.replay(reqs, t_arr)
        st = srv.stats()
    finally:
        srv.close()
    # capacity of the full-cube lane: one call of each full request kind per cube, alone
    import paper_1211_4896_amd as tsa
    single = {}
    for nm, d in zip(names, devs):
        mo = tsa.moments(d)
        for kind, f in (("hist", lambda: tsa.histogram(d, float(np.float32(mo["min"])), float(np.float32(mo["max"])),
                                                       4096)),
                        ("median", lambda: tsa.median(d))):
            f()
            t0 = time.perf_counter()
            f()
            single[f"{nm}_{kind}_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    keep = [o for o, t in zip(out, t_arr) if t >= warm]
    svc = np.array([o.t_done - o.t_launch for o in keep]) * 1e3
    qwait = np.array([o.t_launch - o.t_submit for o in keep]) * 1e3
    lat = np.array([o.t_done - o.t_submit for o in keep]) * 1e3
    kinds = np.array([o.kind for o in keep])
    t_first = min(o.t_submit for o in keep)
    t_last = max(o.t_done for o in keep)
    errs = sum(1 for o in out if o.status != 0)

    def pct(x, q):
        return round(float(np.percentile(x, q)), 3) if x.size else None

    return {"workload": "c5: float32 1024^3 + float32 2048x2048x1024 + int16 2048^3 resident; Poisson arrivals; 90% "
                        "region (c4 boxes, 256 bins), 5% full-cube 4096-bin histogram, 5% full-cube median",
            "offered_qps": qps, "measured_s": seconds, "warmup_s": warm, "requests": len(keep),
            "full_scan_launch_voxels": chunk_kvoxels * 1024,
            "achieved_qps": round(len(keep) / (t_last - t_first), 1),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "p999_ms": pct(lat, 99.9),
            "p50_region_ms": pct(lat[kinds == 0], 50), "p99_region_ms": pct(lat[kinds == 0], 99),
            "p50_full_ms": pct(lat[kinds != 0], 50), "p99_full_ms": pct(lat[kinds != 0], 99),
            "errors": errs, "scheduler": st,
            "service_p50_region_ms": pct(svc[kinds == 0], 50), "service_p50_full_ms": pct(svc[kinds != 0], 50),
            "queue_p50_full_ms": pct(qwait[kinds != 0], 50),
            # where a region request's p99 goes: waiting for its launch, or the launch itself
            "queue_p99_region_ms": pct(qwait[kinds == 0], 99), "service_p99_region_ms": pct(svc[kinds == 0], 99),
            "single_call_ms": single}


def _c1_bench(tsa, torch, synth, lib, sh, reps: int = 20) -> dict:
    """The small 256^3 cube (67 MB, inside the 256 MB Infinity Cache): tsa_stats
    with 1024 bins back to back (cache-resident) and after a 1 GiB copy that
    scrubs the caches before each call."""
    spec = synth.SPECS["c1"]
    host, _ = synth.generate(spec)
    dev = torch.from_numpy(host).to("cuda:0")
    api = tsa.capi()
    c = tsa.cube_of(dev)
    nbins = 1024
    ws = tsa.workspace(tsa.OP_STATS, dev, None, nbins)
    out = torch.empty(72, dtype=torch.uint8, device=dev.device)
    counts = torch.empty(nbins, dtype=torch.int64, device=dev.device)
    scrub = torch.empty(2 << 30, dtype=torch.uint8, device=dev.device)
    lib.tsa_internal_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]

    def run(n, cold):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tot = 0.0
        for _ in range(n):
            if cold:
                lib.tsa_internal_copy(scrub.data_ptr() + (1 << 30), scrub.data_ptr(), 1 << 30, sh)
            e0.record()
            st = api.tsa_stats(ctypes.byref(c), None, nbins, out.data_ptr(), counts.data_ptr(), None,
                               ws.data_ptr(), ws.numel(), sh)
            e1.record()
            if st != 0:
                raise RuntimeError(f"tsa_stats: {tsa.status_string(st)}")
            torch.cuda.synchronize()
            tot += e0.elapsed_time(e1)
        return tot / n

    run(3, False)
    hot = run(reps, False)
    cold = run(reps // 2, True)
    N = dev.numel()
    return {"workload": "c1: 256^3 float32 (67 MB) cube; moments + 1024-bin histogram over [min,max] + median",
            "hot_ms": round(hot, 4), "hot_gvoxel_s": round(N / (hot * 1e-3) / 1e9, 1),
            "cold_ms": round(cold, 4), "cold_gvoxel_s": round(N / (cold * 1e-3) / 1e9, 1)}


def generate_on_device(synth, torch, spec, planes: int = 16):
    """A cube generated in z-slabs straight into one device tensor: the host
    generates the next slab into one of two pinned buffers while the other's
    copy to the device runs.  Returns (tensor, nan count)."""
    dt = torch.float32 if spec.dtype == "f32" else torch.int16
    dev = torch.empty((spec.nz, spec.ny, spec.nx), dtype=dt, device="cuda:0")
    bufs = [torch.empty((planes, spec.ny, spec.nx), dtype=dt, pin_memory=True) for _ in range(2)]
    copied = [None, None]
    stream = torch.cuda.Stream()
    nan = 0
    for i, z0 in enumerate(range(0, spec.nz, planes)):
        z1 = min(spec.nz, z0 + planes)
        b = i % 2
        if copied[b] is not None:
            copied[b].synchronize()  # this buffer's previous copy has finished
        _, n = synth.generate(spec, z0, z1, out=bufs[b][: z1 - z0].numpy())
        nan += n
        with torch.cuda.stream(stream):
            dev[z0:z1].copy_(bufs[b][: z1 - z0], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        copied[b] = ev
    stream.synchronize()
    torch.cuda.synchronize()
    return dev, nan


def _read_probe(lib, dev, sh, torch, reps: int = 10) -> dict:
    """Achievable HBM read bandwidth: the passes' load pattern over the same
    cube with the least possible work (tsa_internal_read_probe)."""
    lib.tsa_internal_read_probe.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
    lib.tsa_internal_probe_blocks.restype = ctypes.c_int32
    nbytes = dev.numel() * dev.element_size() // 16 * 16
    sink = torch.empty(max(1, lib.tsa_internal_probe_blocks()), dtype=torch.int32, device=dev.device)
    for _ in range(2):
        lib.tsa_internal_read_probe(dev.data_ptr(), nbytes, sink.data_ptr(), sh)
    torch.cuda.synchronize()
    _trace(lib, True, cap=reps + 1)
    for _ in range(reps):
        if lib.tsa_internal_read_probe(dev.data_ptr(), nbytes, sink.data_ptr(), sh) != 0:
            raise RuntimeError("tsa_internal_read_probe failed")
    torch.cuda.synchronize()
    k = _trace_read(lib).get("read_probe", [1, 0.0])
    _trace(lib, False)
    ms = k[1] / k[0]
    return {"ms": round(ms, 4), "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}


def _calib_copy(lib, device, sh, nbytes: int = 1 << 30) -> int:
    """Three plain copies of nbytes: their FETCH_SIZE / WRITE_SIZE per dispatch
    calibrate the counters against a known byte count."""
    import torch

    lib.tsa_internal_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    for _ in range(3):
        st = lib.tsa_internal_copy(dst.data_ptr(), src.data_ptr(), nbytes, sh)
        if st != 0:
            raise RuntimeError(f"tsa_internal_copy failed ({st})")
    torch.cuda.synchronize()
    return nbytes


def _separate_ops(tsa, api, dev, cp, N, lo, hi, nbins, sh, reps: int = 10) -> dict:
    """Rates of the separate calls: tsa_histogram (one pass), tsa_median
    (radix selection), tsa_moments (one pass)."""
    import torch

    ws = tsa.workspace(tsa.OP_HISTOGRAM, dev, None, nbins)
    out = torch.empty(72, dtype=torch.uint8, device=dev.device)
    counts = torch.empty(nbins, dtype=torch.int64, device=dev.device)
    outl = torch.empty(2, dtype=torch.int64, device=dev.device)
    calls = {
        "histogram": lambda: api.tsa_histogram(cp, None, lo, hi, nbins, counts.data_ptr(), outl.data_ptr(),
                                               ws.data_ptr(), ws.numel(), sh),
        "median": lambda: api.tsa_median(cp, None, out.data_ptr(), ws.data_ptr(), ws.numel(), sh),
        "moments": lambda: api.tsa_moments(cp, None, out.data_ptr(), ws.data_ptr(), ws.numel(), sh),
    }
    res = {}
    for name, f in calls.items():
        for _ in range(2):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            st = f()
            if st != 0:
                raise RuntimeError(f"{name}: {tsa.status_string(st)}")
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gvs = N / (ms * 1e-3) / 1e9
        # bytes actually required: one read of the cube per full pass
        passes = {"histogram": 1, "moments": 1, "median": 2}[name]
        res[name] = {"ms": round(ms, 4), "gvoxel_s": round(gvs, 2),
                     "hbm_frac": round(passes * 4.0 * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "full_passes": passes}
    return res


if __name__ == "__main__":
    main()
