"""Audit of the library's own gfx950 machine code (built here), read back from the shared
library with the ROCm LLVM tools: no scratch memory, no packed FP32 arithmetic, no stores or
atomics through the scalar data cache, no PC-relative data references, and every kernel's
static LDS within the device limit.  No GPU needed."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

fc = pytest.importorskip("paper_2606_04801_amd")
LLVM = "/opt/rocm/llvm/bin"
if not (os.path.exists(fc.LIB_PATH) and os.path.exists(os.path.join(LLVM, "llvm-objdump"))):
    pytest.skip("library or ROCm LLVM tools missing", allow_module_level=True)

FORBIDDEN = [
    r"^scratch_", r"^buffer_",                                    # private (scratch) memory
    r"^v_pk_(add|mul|fma)_f32",                                   # packed FP32 arithmetic
    r"^s_(buffer_)?store", r"^s_(buffer_)?atomic", r"^s_dcache_(wb|discard)",   # scalar-cache writes
    r"^s_getpc",                                                  # PC-relative addressing
]


@pytest.fixture(scope="module")
def code_object():
    d = tempfile.mkdtemp()
    fb, co = os.path.join(d, "fatbin"), os.path.join(d, "gfx950.co")
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section=.hip_fatbin=" + fb, fc.LIB_PATH],
                   check=True, capture_output=True)
    subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o", "--input=" + fb,
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--output=" + co], check=True, capture_output=True)
    yield co
    shutil.rmtree(d, ignore_errors=True)


def test_no_forbidden_instructions(code_object):
    dis = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", code_object],
                         check=True, capture_output=True, text=True).stdout
    mnemonics = set(re.findall(r"^\s+([a-z][a-z0-9_]*)\s", dis, flags=re.M))
    assert len(mnemonics) > 50
    bad = sorted(m for m in mnemonics if any(re.match(p, m) for p in FORBIDDEN))
    assert not bad, bad


def test_kernel_descriptors(code_object):
    out = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", code_object], check=True,
                         capture_output=True, text=True).stdout
    lds = [int(x) for x in re.findall(r"\.group_segment_fixed_size:\s+(\d+)", out)]
    priv = [int(x) for x in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", out)]
    assert len(lds) >= 15 and len(priv) == len(lds)
    assert max(lds) <= 64 * 1024            # well inside the 160 KiB a gfx950 workgroup may use
    assert max(priv) == 0
    assert "uses_dynamic_stack: true" not in out.replace(".", "")


def test_no_device_globals(code_object):
    out = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--dyn-syms", "-S", code_object], check=True,
                         capture_output=True, text=True).stdout
    objs = [l.split()[-1] for l in out.splitlines() if " OBJECT " in l and ".kd" not in l]
    assert all(o.startswith("__hip_cuid") for o in objs), objs
