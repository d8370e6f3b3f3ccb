"""Build the CPU emulation of the library's kernels (test infrastructure, never shipped).

The kernels of paper_2606_04801_amd/csrc are compiled as host C++ against the emulated HIP
runtime in this folder and linked with driver.cpp.  Variants:
  asan   g++, AddressSanitizer + UBSan (fatal), a redzone around every LDS array
  poison g++ -O2, LDS refilled with a poison byte before every block
  msan   clang++, MemorySanitizer (LDS, workspace and outputs start uninitialised)
  trace  clang++, every load and store of kernel code must hit device memory, LDS or the
         thread's own private memory; EMU_LOCKSTEP=1 switches threads after every access
  so     the library's C ABI as a host shared object (no driver), for the binding tests
  isa    the library's host code as a shared object whose kernel launches and device
         allocations go to hooks (tests/isa_emulation runs the gfx950 code object there)
Every build leaves 256 unused bytes after each workspace array (FC_ARRAY_GAP), which the driver
poisons.  Executables go to tests/cpu_emulation/_build/ and are rebuilt when a source changes.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2606_04801_amd", "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "_build")
SOURCES = [os.path.join(CSRC, "fc_kernels.hip"), os.path.join(CSRC, "fc_lut.cpp"), os.path.join(HERE, "runtime.cpp")]
DEPS = SOURCES + [os.path.join(HERE, "driver.cpp"), os.path.join(CSRC, "fc_common.h"), os.path.join(INC, "flashcubical.h"),
                  os.path.join(HERE, "hip", "hip_runtime.h"), os.path.join(HERE, "trace_ignore.txt")]

COMMON = ["-std=c++20", "-D__HIPCC__", "-DFC_ARRAY_GAP=256", "-I", HERE, "-I", INC, "-I", CSRC, "-pthread"]
VARIANTS = {
    "asan": ("g++", ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=undefined", "-DEMU_LDS_REDZONE"]),
    "poison": ("g++", ["-O2"]),
    "msan": ("/opt/rocm/llvm/bin/clang++", ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=memory",
                                            "-fsanitize-memory-track-origins=2"]),
    # every load and store of kernel code checked against GPU-visible memory (runtime.cpp)
    "trace": ("/opt/rocm/llvm/bin/clang++", ["-O1", "-g", "-fno-omit-frame-pointer", "-rdynamic", "-DEMU_TRACE",
                                             "-fsanitize=address", "-mllvm", "-asan-instrumentation-with-call-threshold=0",
                                             "-mllvm", "-asan-memory-access-callback-prefix=__emu_",
                                             "-mllvm", "-asan-stack=0", "-mllvm", "-asan-globals=0",
                                             "-fsanitize-ignorelist=" + os.path.join(HERE, "trace_ignore.txt")]),
    # the library's host code as a shared object whose launches go to the gfx950 interpreter
    "isa": ("g++", ["-O1", "-g", "-fPIC", "-shared", "-DEMU_ISA"]),
    # the library's C ABI as a host shared object, for driving the Python binding on the CPU
    "so": ("g++", ["-O2", "-g", "-fPIC", "-shared"]),
}


def build(variant: str = "asan") -> str:
    cxx, flags = VARIANTS[variant]
    if not (os.path.exists(cxx) or shutil.which(cxx)):
        raise RuntimeError("compiler %s not found" % cxx)
    h = hashlib.sha256((cxx + " ".join(flags)).encode())
    for p in DEPS:
        h.update(open(p, "rb").read())
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "driver_" + variant)
    stamp = exe + ".sha256"
    if os.path.exists(exe) and os.path.exists(stamp) and open(stamp).read() == h.hexdigest():
        return exe
    srcs = []
    for s in SOURCES + ([] if variant in ("so", "isa") else [os.path.join(HERE, "driver.cpp")]):
        srcs += ["-x", "c++", s]
    if variant in ("so", "isa"):
        exe = os.path.join(OUT, "libflashcubical_emulated.so" if variant == "so" else "libflashcubical_isa_host.so")
        stamp = exe + ".sha256"
        if os.path.exists(exe) and os.path.exists(stamp) and open(stamp).read() == h.hexdigest():
            return exe
    cmd = [cxx] + COMMON + flags + srcs + ["-o", exe + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("emulation build failed:\n" + r.stderr[-4000:])
    os.replace(exe + ".tmp", exe)
    open(stamp, "w").write(h.hexdigest())
    return exe


if __name__ == "__main__":
    import sys
    for v in (sys.argv[1:] or ["asan"]):
        print(build(v))
