"""Build the gfx950 shared library in-tree with hipcc (no JIT, no torch extension).

    python -m paper_2606_04801_amd.build

Produces paper_2606_04801_amd/libflashcubical.so from csrc/ (kernels + C ABI + table
generator).  Packed FP32 instructions are disabled for every HIP translation unit.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libflashcubical.so")
SOURCES = ["fc_kernels.hip", "fc_lut.cpp"]
ARCH = os.environ.get("FC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    # a fixed command line: clang names the library's device-code symbols with a hash of it, so
    # the same sources give the same library bytes (profiles/ figures are tied to that digest)
    out_tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=%s" % ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function",
           "-o", out_tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        if os.path.exists(out_tmp):
            os.remove(out_tmp)
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs:
        print(msgs)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
