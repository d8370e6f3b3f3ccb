"""Audit of the library's own gfx950 machine code (built here), read back from the shared
library with the ROCm LLVM tools: no packed FP32 arithmetic, no stores or atomics through the
scalar data cache, no PC-relative data references, every kernel's static LDS within the device
limit, and no scratch memory except a bounded register spill in the 3D classify kernels (built
for seven workgroups per compute unit).  No GPU needed."""
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
    r"^buffer_",                                                  # buffer-descriptor memory
    r"^v_pk_(add|mul|fma)_f32",                                   # packed FP32 arithmetic
    r"^s_(buffer_)?store", r"^s_(buffer_)?atomic", r"^s_dcache_(wb|discard)",   # scalar-cache writes
    r"^s_getpc",                                                  # PC-relative addressing
]


@pytest.fixture(scope="module")
def code_object():
    d = tempfile.mkdtemp()
    fb, co = os.path.join(d, "fatbin"), os.path.join(d, "gfx950.co")
    # an explicit output: without one llvm-objcopy rewrites the library in place
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section=.hip_fatbin=" + fb, fc.LIB_PATH,
                    os.path.join(d, "copy.so")], check=True, capture_output=True)
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


def test_scratch_only_in_classify3d(code_object):
    """Private memory appears only as the 3D classify kernels' spill, through architected flat
    scratch (no buffer descriptor)."""
    dis = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", code_object],
                         check=True, capture_output=True, text=True).stdout
    fn, users = None, set()
    for line in dis.splitlines():
        m = re.match(r"^[0-9a-f]+ <(\S+)>:", line)
        if m:
            fn = m.group(1)
        elif re.match(r"^\s+scratch_", line):
            users.add(fn)
    assert all("k_classify3d" in f for f in users), users


def test_kernel_descriptors(code_object):
    out = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", code_object], check=True,
                         capture_output=True, text=True).stdout
    lds = [int(x) for x in re.findall(r"\.group_segment_fixed_size:\s+(\d+)", out)]
    priv = [int(x) for x in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", out)]
    names = re.findall(r"^\s+\.name:\s+(\S+)", out, flags=re.M)
    names = [n for n in names if n.startswith("_Z") or n.startswith("k_")]
    assert len(lds) >= 12 and len(priv) == len(lds) == len(names)
    assert max(lds) <= 160 * 1024           # the LDS a gfx950 workgroup may use
    for n, p in zip(names, priv):           # a spill of a few registers at most
        assert p == 0 or ("k_classify3d" in n and p <= 32), (n, p)
    assert "uses_dynamic_stack: true" not in out.replace(".", "")


def test_no_device_globals(code_object):
    """The only device variable is the no-allocation entry point's workspace (`scratch`, 64 MiB,
    reached by its address from hipGetSymbolAddress); the kernels keep no other state."""
    out = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--dyn-syms", "-S", code_object], check=True,
                         capture_output=True, text=True).stdout
    rows = [l.split() for l in out.splitlines() if " OBJECT " in l and ".kd" not in l]
    objs = {r[-1]: int(r[2], 0) for r in rows}
    others = [o for o in objs if not o.startswith("__hip_cuid")]
    assert others == ["_ZL7scratch"], objs
    assert objs["_ZL7scratch"] == 64 << 20
