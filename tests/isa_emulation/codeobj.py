"""Read the library's own gfx950 code object: kernel metadata, kernel descriptors and the
disassembly (ROCm LLVM tools).  Test infrastructure for the ISA-level CPU interpreter."""
from __future__ import annotations

import os
import re
import struct
import subprocess
import tempfile

LLVM = "/opt/rocm/llvm/bin"


def _run(args):
    return subprocess.run(args, check=True, capture_output=True, text=True).stdout


def extract(so_path: str, arch: str = "gfx950") -> str:
    """Path of the unbundled gfx950 code object of a HIP shared library (in a temp dir)."""
    d = tempfile.mkdtemp(prefix="fc_co_")
    fb, co = os.path.join(d, "fatbin"), os.path.join(d, arch + ".co")
    # an explicit output: without one llvm-objcopy rewrites its input in place
    _run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section=.hip_fatbin=" + fb, so_path, os.path.join(d, "copy.so")])
    _run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o", "--input=" + fb,
          "--targets=hipv4-amdgcn-amd-amdhsa--" + arch, "--output=" + co])
    return co


class KernelInfo:
    def __init__(self, name):
        self.name = name
        self.args = []            # (offset, size, value_kind)
        self.kernarg_size = 0
        self.group_segment = 0
        self.private_segment = 0
        self.desc = None          # raw 64-byte kernel descriptor
        self.entry = None         # address of the first instruction


def _metadata(co: str):
    """Kernels of the code object's metadata note (YAML as printed by llvm-readelf): an entry
    of amdhsa.kernels starts with "- ." at indent 2, an argument with "- ." at indent 6."""
    text = _run([os.path.join(LLVM, "llvm-readelf"), "--notes", co])
    kernels, cur, arg, in_kernels = {}, None, None, False
    for line in text.splitlines():
        if line.strip().startswith("amdhsa.kernels:"):
            in_kernels = True
            continue
        if not in_kernels:
            continue
        m = re.match(r"^(\s*)(- )?\.(\w+):\s*(.*)$", line)
        if not m:
            if line and not line.startswith(" "):
                in_kernels = False
            continue
        indent = len(m.group(1)) + (2 if m.group(2) else 0)
        key, val = m.group(3), m.group(4).strip()
        if m.group(2) and len(m.group(1)) == 2:
            cur = KernelInfo(None)
            arg = None
        if cur is None:
            continue
        if m.group(2) and len(m.group(1)) == 6:
            arg = {}
            cur.args.append(arg)
        if indent >= 8 and arg is not None:
            arg[key] = val
        elif indent == 4:
            arg = None if key != "args" else arg
            if key == "name":
                cur.name = val
            elif key == "symbol":
                kernels[val[:-3] if val.endswith(".kd") else val] = cur
            elif key == "kernarg_segment_size":
                cur.kernarg_size = int(val)
            elif key == "group_segment_fixed_size":
                cur.group_segment = int(val)
            elif key == "private_segment_fixed_size":
                cur.private_segment = int(val)
    for k in kernels.values():
        k.args = [(int(a["offset"]), int(a["size"]), a["value_kind"]) for a in k.args]
    return kernels


def _sections(co: str):
    text = _run([os.path.join(LLVM, "llvm-readelf"), "-S", "--wide", co])
    secs = {}
    for line in text.splitlines():
        m = re.match(r"\s*\[\s*\d+\]\s+(\S+)\s+\S+\s+([0-9a-f]+)\s+([0-9a-f]+)\s+([0-9a-f]+)", line)
        if m:
            secs[m.group(1)] = (int(m.group(2), 16), int(m.group(3), 16), int(m.group(4), 16))
    return secs


def _symbols(co: str):
    text = _run([os.path.join(LLVM, "llvm-readelf"), "-s", "--wide", co])
    syms = {}
    for line in text.splitlines():
        p = line.split()
        if len(p) >= 8 and p[3] in ("FUNC", "OBJECT"):
            syms[p[7]] = int(p[1], 16)
    return syms


def disassemble(co: str, arch: str = "gfx950"):
    """[(address, text)] of every instruction of .text (comments and encodings stripped)."""
    text = _run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=" + arch, co])
    out = []
    for line in text.splitlines():
        if not line.startswith("\t"):
            continue
        body, _, comment = line[1:].partition("//")
        m = re.match(r"\s*([0-9A-Fa-f]+):", comment)
        if not m:
            continue
        out.append((int(m.group(1), 16), body.strip()))
    return out


def load(so_path: str, arch: str = "gfx950"):
    """(kernels by mangled name, instructions) of the library's code object."""
    co = extract(so_path, arch)
    kernels = _metadata(co)
    secs = _sections(co)
    syms = _symbols(co)
    raw = open(co, "rb").read()
    for name, k in kernels.items():
        kd = syms[name + ".kd"]
        addr, off, _ = secs[".rodata"]
        desc = raw[off + kd - addr: off + kd - addr + 64]
        k.desc = desc
        entry_off = struct.unpack_from("<q", desc, 16)[0]
        k.entry = kd + entry_off
        if k.entry != syms[name]:
            raise RuntimeError("kernel entry mismatch for " + name)
    return kernels, disassemble(co, arch)
