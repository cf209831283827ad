"""Build libtsa.so (hipcc, gfx950) in-tree.

Each source compiles to its own object in parallel (under _build/), then one
link step makes the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtsa.so")
OBJDIR = os.path.join(ROOT, "_build")

SOURCES = ["tsa_kernels.hip", "tsa_hist_wide.hip", "tsa_batch.hip", "tsa_serve.hip", "tsa_tune.hip",
           "tsa_minimap.hip", "tsa_spectrum.hip", "tsa_trace.hip", "tsa_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # IEEE arithmetic exactly as written: no contraction into FMA (the
    # histogram bin formula), denormals kept (bins and sums of denormal values)
    "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout)


def build(out: str = LIB, verbose: bool = False, extra_flags=(), jobs: int = 0) -> str:
    """Compile every source and link one shared library (extra_flags: e.g. -D
    switches of kernel variants, for timing one build against another)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tag = "default" if not extra_flags else str(abs(hash(tuple(extra_flags))))
    objdir = os.path.join(OBJDIR, tag)
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    cmds = [[hipcc, *HIPCC_FLAGS, *extra_flags, *inc, "-c", "-o", o, os.path.join(CSRC, s)]
            for s, o in zip(SOURCES, objs)]
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = out + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
