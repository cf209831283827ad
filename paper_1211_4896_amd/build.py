"""Build libtsa.so (hipcc, gfx950) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtsa.so")

SOURCES = ["tsa_kernels.hip", "tsa_hist_wide.hip", "tsa_batch.hip", "tsa_serve.hip", "tsa_tune.hip", "tsa_minimap.hip", "tsa_spectrum.hip", "tsa_trace.hip", "tsa_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # IEEE arithmetic exactly as written: no contraction into FMA (the
    # histogram bin formula), denormals kept (bins and sums of denormal values)
    "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(out: str = LIB, verbose: bool = False, extra_flags=()) -> str:
    """Compile every source into one shared library (extra_flags: e.g. -D
    switches of kernel variants, for timing one build against another)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *extra_flags, "-I", os.path.join(ROOT, "include"), "-o", tmp,
           *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
