"""Interpreter for the library's own gfx950 machine code, on the CPU.

It executes the instructions that llvm-objdump prints for the code object built here: one
wavefront of 64 lanes at a time in lockstep (numpy vectors), the waves of a workgroup
interleaved between barriers (or every few instructions), workgroups one after another.  So the
compiled kernels themselves, not a host rebuild of their source, run against the oracle.
Every global access must fall inside a registered device allocation and every LDS access
inside the kernel's LDS segment; anything else stops the run with the kernel, instruction and
address.  Only the instructions these kernels use are implemented; an unknown one stops the
run as well.  Test infrastructure, never part of the library.
"""
from __future__ import annotations

import bisect
import ctypes
import re
import struct

import numpy as np

np.seterr(all="ignore")

U8, U16, U32, U64, I32, I64 = np.uint8, np.uint16, np.uint32, np.uint64, np.int32, np.int64
F32 = np.float32
LANES = 64
M32 = 0xFFFFFFFF
M64 = 0xFFFFFFFFFFFFFFFF
SPECIAL = {"vcc_lo": (106, 1), "vcc_hi": (107, 1), "vcc": (106, 2), "exec_lo": (126, 1),
           "exec_hi": (127, 1), "exec": (126, 2), "m0": (124, 1)}
FLOAT_INLINE = {"0.5": 0x3F000000, "-0.5": 0xBF000000, "1.0": 0x3F800000, "-1.0": 0xBF800000,
                "2.0": 0x40000000, "-2.0": 0xC0000000, "4.0": 0x40800000, "-4.0": 0xC0800000,
                "0.15915494": 0x3E22F983}
# Flat addresses in [SHARED_APERTURE, SHARED_APERTURE + 2^32) are LDS: flat loads and stores
# there go to the workgroup's LDS (bounds-checked against the kernel's LDS segment); other
# instructions that reach the aperture (flat atomics) are refused, as Memory has no allocation
# there.
SHARED_APERTURE = 0x10000 << 32
LANE = np.arange(LANES, dtype=np.int64)
BIT = (np.uint64(1) << np.arange(LANES, dtype=np.uint64))


class Fault(Exception):
    pass


class Unsupported(Exception):
    pass


def mask_of(b) -> int:
    """64-bit lane mask of a bool vector"""
    return int(np.bitwise_or.reduce(np.where(b, BIT, np.uint64(0))))


def bools_of(m: int) -> np.ndarray:
    return ((np.uint64(m) >> np.arange(LANES, dtype=np.uint64)) & np.uint64(1)).astype(bool)


# ------------------------------------------------------------------------ memory --
class Memory:
    """Device allocations by address.  The interpreter reads and writes the host memory that
    stands for device memory and refuses any address outside a registered allocation."""

    def __init__(self):
        self.bases, self.regions = [], []      # sorted bases; (base, size, uint8 view)

    def add(self, base: int, size: int, view=None):
        if view is None:
            view = np.ctypeslib.as_array((ctypes.c_uint8 * max(size, 1)).from_address(base))
        k = bisect.bisect_left(self.bases, base)
        if k < len(self.bases) and self.bases[k] == base:
            self.regions[k] = (base, size, view)
            return
        self.bases.insert(k, base)
        self.regions.insert(k, (base, size, view))

    def remove(self, base: int):
        k = bisect.bisect_left(self.bases, base)
        if k < len(self.bases) and self.bases[k] == base:
            del self.bases[k]
            del self.regions[k]

    def region(self, lo: int, hi: int, what: str):
        k = bisect.bisect_right(self.bases, lo) - 1
        if k >= 0:
            base, size, view = self.regions[k]
            if lo >= base and hi <= base + size:
                return view, base
        near = ""
        if k >= 0:
            base, size, _ = self.regions[k]
            near = " (nearest allocation below: 0x%x, %d bytes, access at +%d)" % (base, size, lo - base)
        if SHARED_APERTURE <= lo < SHARED_APERTURE + (1 << 32):
            raise Fault("%s: this flat access to LDS (0x%x) is not emulated" % (what, lo))
        raise Fault("%s outside device memory: [0x%x, 0x%x)%s" % (what, lo, hi, near))

    def _idx(self, addrs, nbytes, what):
        lo, hi = int(addrs.min()), int(addrs.max()) + nbytes
        try:
            view, base = self.region(lo, hi, what)
            return [(view, (addrs.astype(np.int64) - base)[:, None] + np.arange(nbytes), slice(None))]
        except Fault:
            if len(addrs) == 1:
                raise
        out = []
        for k in range(len(addrs)):
            view, base = self.region(int(addrs[k]), int(addrs[k]) + nbytes, what)
            out.append((view, (np.int64(addrs[k]) - base) + np.arange(nbytes)[None, :], slice(k, k + 1)))
        return out

    def gather(self, addrs, nbytes, what):
        """bytes at each address -> (k, nbytes) uint8"""
        res = np.zeros((len(addrs), nbytes), U8)
        if len(addrs):
            for view, idx, sl in self._idx(addrs, nbytes, what):
                res[sl] = view[idx]
        return res

    def scatter(self, addrs, data, what):
        """data (k, nbytes) uint8 to each address, in lane order (the highest lane wins)"""
        if len(addrs) == 0:
            return
        for view, idx, sl in self._idx(addrs, data.shape[1], what):
            view[idx] = data[sl]

    def read(self, addr: int, nbytes: int, what: str) -> bytes:
        view, base = self.region(addr, addr + nbytes, what)
        return view[addr - base: addr - base + nbytes].tobytes()

    def write(self, addr: int, data: bytes, what: str):
        view, base = self.region(addr, addr + len(data), what)
        view[addr - base: addr - base + len(data)] = np.frombuffer(data, U8)


# ---------------------------------------------------------------------- operands --
class Opd:
    """A parsed operand: kind 'v' / 's' (register index, count), 'imm' (value), 'off'."""
    __slots__ = ("kind", "idx", "cnt", "val", "neg", "abs", "sext", "lit", "text")

    def __init__(self, text):
        self.text = text
        self.neg = self.abs = self.sext = self.lit = False
        self.kind, self.idx, self.cnt, self.val = None, 0, 1, 0
        t = text
        if t.startswith("sext(") and t.endswith(")"):
            self.sext, t = True, t[5:-1]
        if t.startswith("-|") and t.endswith("|"):
            self.neg, self.abs, t = True, True, t[2:-1]
        elif t.startswith("|") and t.endswith("|"):
            self.abs, t = True, t[1:-1]
        elif t.startswith("-") and re.match(r"^-[vs]", t):
            self.neg, t = True, t[1:]
        m = re.match(r"^([vs])(\d+)$", t)
        if m:
            self.kind, self.idx = m.group(1), int(m.group(2))
            return
        m = re.match(r"^([vs])\[(\d+):(\d+)\]$", t)
        if m:
            self.kind, self.idx = m.group(1), int(m.group(2))
            self.cnt = int(m.group(3)) - self.idx + 1
            return
        if t in SPECIAL:
            self.kind = "s"
            self.idx, self.cnt = SPECIAL[t]
            return
        if t == "off":
            self.kind = "off"
            return
        if t == "src_shared_base":             # base of the flat aperture that maps LDS
            self.kind, self.val, self.lit = "imm", SHARED_APERTURE, True
            return
        if t in FLOAT_INLINE:
            self.kind, self.val = "imm", FLOAT_INLINE[t]
            return
        m = re.match(r"^(-?)(0x[0-9a-fA-F]+|\d+)$", t)
        if m:
            v = int(m.group(2), 0)
            self.lit = m.group(2).startswith("0x")
            self.kind, self.val = "imm", (-v if m.group(1) else v)
            return
        raise Unsupported("operand " + text)


def split_ops(rest: str):
    """operands and trailing modifiers of an instruction's text"""
    if not rest:
        return [], {}
    parts = [p.strip() for p in rest.split(",")]
    tail = parts[-1].split()
    parts[-1] = tail[0] if tail else ""
    mods = {}
    for t in tail[1:]:
        k, _, v = t.partition(":")
        mods[k] = v if v else True
    if parts == [""]:
        parts = []
    # a first token that is itself a modifier (instructions without operands)
    if parts and ":" in parts[0] and not parts[0].startswith(("v[", "s[")):
        k, _, v = parts[0].partition(":")
        mods[k] = v
        parts = []
    return parts, mods


class Wave:
    __slots__ = ("s", "v", "scc", "pc", "done", "barrier", "wid", "wg", "lds", "_em", "_eb", "priv")

    def __init__(self, nvgpr):
        self.s = [0] * 128
        self.v = np.zeros((max(nvgpr, 1) + 4, LANES), U32)
        self.scc = 0
        self.pc = 0
        self.done = False
        self.barrier = False
        self._em = None
        self._eb = None
        self.priv = None          # (64, private segment bytes): each lane's scratch memory

    def exec(self) -> np.ndarray:
        m = self.s[126] | (self.s[127] << 32)
        if m != self._em:
            self._em, self._eb = m, bools_of(m)
        return self._eb


# ------------------------------------------------------------ operand accessors --
def r32(o: Opd):
    """value reader for a 32-bit source: vector (64,) for VGPRs, uint32 scalar otherwise"""
    if o.kind == "v":
        i = o.idx
        f = lambda w: w.v[i]
    elif o.kind == "s":
        i = o.idx
        f = lambda w: U32(w.s[i])
    elif o.kind == "imm":
        c = U32(o.val & M32)
        f = lambda w: c
    else:
        raise Unsupported("source " + o.text)
    if o.abs or o.neg:
        a, n, g = o.abs, o.neg, f

        def f(w):
            x = g(w)
            if a:
                x = x & U32(0x7FFFFFFF)
            if n:
                x = x ^ U32(0x80000000)
            return x
    return f


def r64(o: Opd):
    if o.kind == "v":
        i = o.idx
        return lambda w: w.v[i].astype(U64) | (w.v[i + 1].astype(U64) << U64(32))
    if o.kind == "s":
        i = o.idx
        return lambda w: U64(w.s[i] | (w.s[i + 1] << 32))
    if o.kind == "imm":
        c = U64((o.val & M32) if o.lit else (o.val & M64))
        return lambda w: c
    raise Unsupported("source64 " + o.text)


def rs(o: Opd):
    """scalar reader (python int) for SALU operands; 64-bit for pairs"""
    if o.kind == "s":
        i = o.idx
        if o.cnt == 2:
            return lambda w: w.s[i] | (w.s[i + 1] << 32)
        return lambda w: w.s[i]
    if o.kind == "imm":
        c = o.val & M32 if (o.lit or o.val >= 0) else o.val & M64
        c32 = o.val & M32
        return (lambda w: c) if o.cnt == 2 else (lambda w: c32)
    raise Unsupported("scalar source " + o.text)


def rs64(o: Opd):
    if o.kind == "s":
        i = o.idx
        return lambda w: w.s[i] | (w.s[i + 1] << 32)
    if o.kind == "imm":
        c = (o.val & M32) if o.lit and o.val != SHARED_APERTURE else (o.val & M64)
        return lambda w: c
    raise Unsupported("scalar source64 " + o.text)


def ws(o: Opd):
    """scalar writer; a pair takes a 64-bit value"""
    if o.kind != "s":
        raise Unsupported("scalar dest " + o.text)
    i, n = o.idx, o.cnt

    def f(w, x):
        for k in range(n):
            w.s[i + k] = (x >> (32 * k)) & M32
    return f


def wv(o: Opd):
    """vector writer honouring EXEC; 64-bit pairs take uint64 vectors"""
    if o.kind != "v":
        raise Unsupported("vector dest " + o.text)
    i, n = o.idx, o.cnt
    if n == 1:
        def f(w, x):
            e = w.exec()
            w.v[i] = np.where(e, x, w.v[i])
        return f

    def f2(w, x):
        e = w.exec()
        x = np.broadcast_to(np.asarray(x, U64), (LANES,))
        w.v[i] = np.where(e, (x & U64(M32)).astype(U32), w.v[i])
        w.v[i + 1] = np.where(e, (x >> U64(32)).astype(U32), w.v[i + 1])
    return f2


def vec(x, dt=U32):
    return np.broadcast_to(np.asarray(x, dt), (LANES,))


def s32(x):
    return vec(x).view(I32)


def f32(x):
    return vec(x).view(F32)


def bits(x):
    return np.asarray(x, F32).view(U32)


# ------------------------------------------------------------------ VALU table --
def _sx(x, b):
    """sign-extend the low b bits of uint32 values to int64"""
    x = np.asarray(x).astype(np.int64) & ((1 << b) - 1)
    return np.where(x >= (1 << (b - 1)), x - (1 << b), x)


def _bfe_u(a, off, wid):
    off = np.asarray(off, U32) & U32(31)
    wid = np.asarray(wid, U32) & U32(31)
    m = (U64(1) << wid.astype(U64)) - U64(1)
    return ((np.asarray(a, U32).astype(U64) >> off.astype(U64)) & m).astype(U32)


def _bfe_i(a, off, wid):
    u = _bfe_u(a, off, wid).astype(np.int64)
    wid = (np.asarray(wid, U32) & U32(31)).astype(np.int64)
    sign = np.where(wid > 0, (u >> np.maximum(wid - 1, 0)) & 1, 0)
    r = np.where(sign == 1, u - (np.int64(1) << wid), u)
    return np.where(wid == 0, 0, r).astype(np.int64).astype(U32)


def _popc32(x):
    x = np.asarray(x, U32).astype(U64)
    c = np.zeros_like(x)
    for k in range(32):
        c += (x >> U64(k)) & U64(1)
    return c.astype(U32)


def _mbcnt(lo):
    lanes = LANE if lo else np.maximum(LANE - 32, 0)
    lanes = np.minimum(lanes, 32)
    masks = ((np.uint64(1) << lanes.astype(U64)) - U64(1)).astype(U64)
    if not lo:
        masks = np.where(LANE >= 32, masks, U64(0))

    def f(a, b):
        return (_popc32(np.asarray(a, U32).astype(U64) & masks) + np.asarray(b, U32)).astype(U32)
    return f


def _bitop3(tt):
    def f(a, b, c):
        a, b, c = vec(a), vec(b), vec(c)
        r = np.zeros(LANES, U32)
        for i in range(8):
            if (tt >> i) & 1:
                t = (a if i & 4 else ~a) & (b if i & 2 else ~b) & (c if i & 1 else ~c)
                r |= t
        return r
    return f


def _cvt_u32_f32(a):
    x = f32(a).astype(np.float64)
    x = np.where(np.isnan(x), 0.0, x)
    x = np.trunc(np.clip(x, 0.0, 4294967295.0))
    return x.astype(np.uint64).astype(U32)


def _rcp(a):
    x = f32(a).astype(np.float64)
    with np.errstate(divide="ignore"):
        return bits((1.0 / x).astype(F32))


VALU2 = {   # D = f(S0, S1)
    "v_add_u32": lambda a, b: vec(a) + b,
    "v_sub_u32": lambda a, b: vec(a) - b,
    "v_subrev_u32": lambda a, b: vec(b) - a,
    "v_and_b32": lambda a, b: vec(a) & b,
    "v_or_b32": lambda a, b: vec(a) | b,
    "v_xor_b32": lambda a, b: vec(a) ^ b,
    "v_lshlrev_b32": lambda a, b: vec(b) << (vec(a) & U32(31)),
    "v_lshrrev_b32": lambda a, b: vec(b) >> (vec(a) & U32(31)),
    "v_ashrrev_i32": lambda a, b: (s32(b) >> (vec(a) & U32(31)).astype(I32)).view(U32),
    "v_max_i32": lambda a, b: np.maximum(s32(a), s32(b)).view(U32),
    "v_min_i32": lambda a, b: np.minimum(s32(a), s32(b)).view(U32),
    "v_max_u32": lambda a, b: np.maximum(vec(a), vec(b)),
    "v_min_u32": lambda a, b: np.minimum(vec(a), vec(b)),
    "v_mul_lo_u32": lambda a, b: ((vec(a).astype(U64) * vec(b).astype(U64)) & U64(M32)).astype(U32),
    "v_mul_hi_u32": lambda a, b: ((vec(a).astype(U64) * vec(b).astype(U64)) >> U64(32)).astype(U32),
    "v_mul_hi_i32": lambda a, b: ((s32(a).astype(I64) * s32(b).astype(I64)) >> 32).astype(I64).astype(U32),
    "v_mul_u32_u24": lambda a, b: (((vec(a) & U32(0xFFFFFF)).astype(U64) * (vec(b) & U32(0xFFFFFF)).astype(U64)) & U64(M32)).astype(U32),
    "v_mul_hi_u32_u24": lambda a, b: (((vec(a) & U32(0xFFFFFF)).astype(U64) * (vec(b) & U32(0xFFFFFF)).astype(U64)) >> U64(32)).astype(U32),
    "v_mul_i32_i24": lambda a, b: ((_sx(a, 24) * _sx(b, 24)) & M32).astype(U32),
    "v_bcnt_u32_b32": lambda a, b: _popc32(a) + vec(b),
    "v_mbcnt_lo_u32_b32": _mbcnt(True),
    "v_mbcnt_hi_u32_b32": _mbcnt(False),
    "v_mul_f32": lambda a, b: bits(f32(a) * f32(b)),
    "v_add_f32": lambda a, b: bits(f32(a) + f32(b)),      # IEEE, subnormals kept (as the kernels' mode)
    "v_sub_f32": lambda a, b: bits(f32(a) - f32(b)),
    "v_subrev_f32": lambda a, b: bits(f32(b) - f32(a)),
    "v_add_u16": lambda a, b: ((vec(a) + vec(b)) & U32(0xFFFF)),
    "v_mul_lo_u16": lambda a, b: (((vec(a) & U32(0xFFFF)) * (vec(b) & U32(0xFFFF))) & U32(0xFFFF)),
    "v_sub_u16": lambda a, b: ((vec(a) - vec(b)) & U32(0xFFFF)),
    "v_lshrrev_b16": lambda a, b: ((vec(b) & U32(0xFFFF)) >> (vec(a) & U32(15))),
    "v_ashrrev_i16": lambda a, b: ((_sx(b, 16) >> (vec(a) & U32(15)).astype(np.int64)) & 0xFFFF).astype(U32),
}
VALU1 = {   # D = f(S0)
    "v_mov_b32": lambda a: vec(a),
    "v_not_b32": lambda a: ~vec(a),
    "v_bfrev_b32": lambda a: _brev32(vec(a)),
    "v_cvt_f32_u32": lambda a: bits(vec(a).astype(np.float64).astype(F32)),
    "v_cvt_f32_ubyte0": lambda a: bits((vec(a) & U32(0xFF)).astype(F32)),
    "v_cvt_f32_ubyte1": lambda a: bits(((vec(a) >> U32(8)) & U32(0xFF)).astype(F32)),
    "v_cvt_f32_ubyte2": lambda a: bits(((vec(a) >> U32(16)) & U32(0xFF)).astype(F32)),
    "v_cvt_f32_ubyte3": lambda a: bits((vec(a) >> U32(24)).astype(F32)),
    "v_cvt_f32_i32": lambda a: bits(s32(a).astype(np.float64).astype(F32)),
    "v_cvt_u32_f32": _cvt_u32_f32,
    "v_rcp_iflag_f32": _rcp,
    "v_rcp_f32": _rcp,
    "v_trunc_f32": lambda a: bits(np.trunc(f32(a))),
    "v_ffbl_b32": lambda a: _ffbl(vec(a)),          # lowest set bit, -1 for zero
    "v_ffbh_u32": lambda a: _ffbh(vec(a)),          # leading zeros, -1 for zero
}


def _ffbl(x):
    r = np.full(LANES, M32, dtype=U32)
    for k in range(31, -1, -1):
        r = np.where((x >> U32(k)) & U32(1), U32(k), r)
    return r


def _ffbh(x):
    r = np.full(LANES, M32, dtype=U32)
    for k in range(32):
        r = np.where((x >> U32(k)) & U32(1), U32(31 - k), r)
    return r
VALU3 = {   # D = f(S0, S1, S2)
    "v_add3_u32": lambda a, b, c: vec(a) + b + c,
    "v_add_lshl_u32": lambda a, b, c: (vec(a) + b) << (vec(c) & U32(31)),
    "v_lshl_add_u32": lambda a, b, c: (vec(a) << (vec(b) & U32(31))) + c,
    "v_lshl_or_b32": lambda a, b, c: (vec(a) << (vec(b) & U32(31))) | c,
    "v_and_or_b32": lambda a, b, c: (vec(a) & b) | c,
    "v_or3_b32": lambda a, b, c: vec(a) | b | c,
    "v_max3_i32": lambda a, b, c: np.maximum(np.maximum(s32(a), s32(b)), s32(c)).astype(U32),
    "v_min3_i32": lambda a, b, c: np.minimum(np.minimum(s32(a), s32(b)), s32(c)).astype(U32),
    "v_max3_u32": lambda a, b, c: np.maximum(np.maximum(vec(a), vec(b)), vec(c)),
    "v_min3_u32": lambda a, b, c: np.minimum(np.minimum(vec(a), vec(b)), vec(c)),
    "v_med3_i32": lambda a, b, c: np.median(np.stack(np.broadcast_arrays(s32(a), s32(b), s32(c))), axis=0).astype(np.int64).astype(U32),
    "v_xad_u32": lambda a, b, c: (vec(a) ^ b) + c,
    "v_bfe_u32": lambda a, b, c: _bfe_u(vec(a), b, c),
    "v_bfe_i32": lambda a, b, c: _bfe_i(vec(a), b, c),
    "v_perm_b32": lambda a, b, c: _perm_b32(vec(a), vec(b), vec(c)),
    "v_bfi_b32": lambda a, b, c: (vec(a) & vec(b)) | (~vec(a) & vec(c)),
    "v_alignbit_b32": lambda a, b, c: (((vec(a).astype(U64) << U64(32)) | vec(b).astype(U64)) >> (vec(c) & U32(31)).astype(U64)).astype(U64).__and__(U64(M32)).astype(U32),
    "v_mad_u32_u24": lambda a, b, c: ((((vec(a) & U32(0xFFFFFF)).astype(U64) * (vec(b) & U32(0xFFFFFF)).astype(U64)) + vec(c).astype(U64)) & U64(M32)).astype(U32),
    "v_mad_i32_i24": lambda a, b, c: ((_sx(a, 24) * _sx(b, 24) + vec(c).astype(np.int64)) & M32).astype(U32),
}


def _brev32(x):
    r = np.zeros_like(x)
    for k in range(32):
        r |= ((x >> U32(k)) & U32(1)) << U32(31 - k)
    return r


# float compares: lt..lg are ordered (false when either side is NaN), the n-forms are their
# negations (true when either side is NaN); ne is the integer compare
CMP = {"lt": np.less, "le": np.less_equal, "gt": np.greater, "ge": np.greater_equal,
       "eq": np.equal, "ne": np.not_equal,
       "lg": lambda x, y: np.less(x, y) | np.greater(x, y),
       "neq": lambda x, y: ~np.equal(x, y), "nlt": lambda x, y: ~np.less(x, y),
       "nle": lambda x, y: ~np.less_equal(x, y), "ngt": lambda x, y: ~np.greater(x, y),
       "nge": lambda x, y: ~np.greater_equal(x, y),
       "nlg": lambda x, y: ~(np.less(x, y) | np.greater(x, y))}


def _perm_b32(a, b, c):
    """v_perm_b32: byte i of the result is chosen by byte i of c from the eight bytes of
    {a (high), b (low)}; 8..11 replicate the sign bit of bytes 1, 3, 5, 7, 12 gives 0, 13.. 0xFF"""
    data = (a.astype(U64) << U64(32)) | b.astype(U64)
    out = np.zeros(a.shape, U32)
    for i in range(4):
        sel = ((c >> U32(8 * i)) & U32(0xFF)).astype(U64)
        byte = (data >> (U64(8) * np.minimum(sel, U64(7)))) & U64(0xFF)
        for s_, bit in ((8, 15), (9, 31), (10, 47), (11, 63)):
            byte = np.where(sel == s_, np.where((data >> U64(bit)) & U64(1), U64(0xFF), U64(0)), byte)
        byte = np.where(sel == 12, U64(0), np.where(sel >= 13, U64(0xFF), byte))
        out |= (byte.astype(U32) << U32(8 * i))
    return out


def _cmp_vals(ty, o):
    if ty == "i32":
        f = r32(o)
        return lambda w: s32(f(w))
    if ty == "u32":
        f = r32(o)
        return lambda w: vec(f(w))
    if ty == "i64":
        f = r64(o)
        return lambda w: vec(f(w), U64).view(I64)
    if ty == "u64":
        f = r64(o)
        return lambda w: vec(f(w), U64)
    if ty == "f32":
        f = r32(o)
        return lambda w: f32(f(w))
    if ty == "u16":
        f = r32(o)
        return lambda w: vec(f(w)) & U32(0xFFFF)
    if ty == "i16":
        f = r32(o)
        return lambda w: ((vec(f(w)) & U32(0xFFFF)).astype(I64) ^ 0x8000) - 0x8000
    raise Unsupported("compare type " + ty)


# ------------------------------------------------------------------ compilation --
class Instr:
    __slots__ = ("pc", "text", "op", "fn", "next")


def compile_instr(pc: int, text: str, nxt: int):
    op, _, rest = text.partition(" ")
    parts, mods = split_ops(rest.strip())
    ins = Instr()
    ins.pc, ins.text, ins.op, ins.next = pc, text, op, nxt
    ins.fn = _compile(op, parts, mods, pc, nxt)
    return ins


def _branch_target(pc, parts):
    simm = int(parts[0], 0)
    if simm >= 0x8000:
        simm -= 0x10000
    return pc + 4 + 4 * simm


def _compile(op, parts, mods, pc, nxt):
    O = [Opd(p) for p in parts] if not op.startswith(("s_waitcnt", "s_nop", "s_branch", "s_cbranch")) else None
    # ---------------------------------------------------------------- control
    if op in ("s_nop", "s_waitcnt"):
        return lambda w: nxt
    if op == "s_endpgm":
        def f(w):
            w.done = True
            return None
        return f
    if op == "s_barrier":
        def f(w):
            w.barrier = True
            return nxt
        return f
    if op == "s_branch":
        t = _branch_target(pc, parts)
        return lambda w: t
    if op.startswith("s_cbranch_"):
        t = _branch_target(pc, parts)
        cond = op[len("s_cbranch_"):]
        if cond == "scc0":
            return lambda w: nxt if w.scc else t
        if cond == "scc1":
            return lambda w: t if w.scc else nxt
        if cond == "vccz":
            return lambda w: nxt if (w.s[106] | w.s[107]) else t
        if cond == "vccnz":
            return lambda w: t if (w.s[106] | w.s[107]) else nxt
        if cond == "execz":
            return lambda w: nxt if (w.s[126] | w.s[127]) else t
        if cond == "execnz":
            return lambda w: t if (w.s[126] | w.s[127]) else nxt
        raise Unsupported(op)
    if op.startswith("s_"):
        return _compile_salu(op, O, mods, nxt)
    if op.startswith(("global_", "flat_")):
        return _compile_global(op, O, mods, nxt)
    if op.startswith("scratch_"):
        return _compile_scratch(op, O, mods, nxt)
    if op.startswith("ds_"):
        return _compile_ds(op, O, mods, nxt)
    if op.startswith("v_"):
        return _compile_valu(op, O, mods, nxt)
    raise Unsupported(op)


# ---------------------------------------------------------------------- SALU --
def _scc_nz(w, x):
    w.scc = 1 if x else 0
    return x


def _compile_salu(op, O, mods, nxt):
    if op.startswith("s_load_dword"):
        n = {"s_load_dword": 1, "s_load_dwordx2": 2, "s_load_dwordx4": 4, "s_load_dwordx8": 8}[op]
        d, base = O[0], rs64(O[1])
        offr = rs(O[2]) if len(O) > 2 else (lambda w: 0)
        di = d.idx

        def f(w):
            addr = (base(w) + offr(w)) & ~3
            raw = w.wg.mem.read(addr, 4 * n, "s_load at pc 0x%x" % w.pc)
            vals = struct.unpack("<%dI" % n, raw)
            for k in range(n):
                w.s[di + k] = vals[k]
            return nxt
        return f
    if op in ("s_and_saveexec_b64", "s_or_saveexec_b64", "s_andn2_saveexec_b64"):
        d, a = ws(O[0]), rs64(O[1])
        kind = op.split("_")[1]

        def f(w):
            e = w.s[126] | (w.s[127] << 32)
            x = a(w)
            d(w, e)
            ne = (x & e) if kind == "and" else ((x | e) if kind == "or" else (x & ~e & M64))
            w.s[126], w.s[127] = ne & M32, ne >> 32
            w.scc = 1 if ne else 0
            return nxt
        return f
    if op == "s_cselect_b32" or op == "s_cselect_b64":
        d, a, b = ws(O[0]), rs(O[1]), rs(O[2])
        if op.endswith("64"):
            a, b = rs64(O[1]), rs64(O[2])
        return lambda w: (d(w, a(w) if w.scc else b(w)), nxt)[1]
    if op.startswith(("s_cmp_", "s_cmpk_")):
        _, kind, cmpop, ty = op.split("_")
        a = rs64(O[0]) if ty.endswith("64") else rs(O[0])
        if kind == "cmpk":
            k = O[1].val & 0xFFFF
            if ty == "i32" and k >= 0x8000:
                k -= 0x10000
            b = lambda w: k
        else:
            b = rs64(O[1]) if ty.endswith("64") else rs(O[1])
        c = CMP[cmpop]
        if ty == "i32":
            def f(w):
                x, y = a(w), b(w)
                x = x - (1 << 32) if x >= 1 << 31 else x
                y = y - (1 << 32) if y >= 1 << 31 else y
                w.scc = 1 if c(x, y) else 0
                return nxt
        else:
            def f(w):
                w.scc = 1 if c(a(w), b(w)) else 0
                return nxt
        return f
    if op in ("s_bitcmp1_b32", "s_bitcmp0_b32"):
        a, b = rs(O[0]), rs(O[1])
        want = 1 if op == "s_bitcmp1_b32" else 0

        def f(w):
            w.scc = 1 if ((a(w) >> (b(w) & 31)) & 1) == want else 0
            return nxt
        return f
    d = ws(O[0])
    if op in ("s_movk_i32", "s_addk_i32", "s_mulk_i32"):
        k = O[1].val & 0xFFFF
        k = k - 0x10000 if k >= 0x8000 else k
        di = O[0].idx
        if op == "s_movk_i32":
            return lambda w: (d(w, k & M32), nxt)[1]
        if op == "s_mulk_i32":
            return lambda w: (d(w, (w.s[di] * k) & M32), nxt)[1]

        def f(w):
            x = w.s[di]
            xs = x - (1 << 32) if x >= 1 << 31 else x
            r = xs + k
            w.scc = 1 if (r >= 1 << 31 or r < -(1 << 31)) else 0
            d(w, r & M32)
            return nxt
        return f
    is64 = op.endswith("_b64")
    if op in ("s_mov_b32", "s_mov_b64"):
        a = rs64(O[1]) if is64 else rs(O[1])
        return lambda w: (d(w, a(w)), nxt)[1]
    if op in ("s_not_b32", "s_brev_b32", "s_abs_i32", "s_ff1_i32_b64", "s_bcnt1_i32_b64", "s_flbit_i32_b64",
              "s_flbit_i32_b32", "s_ff1_i32_b32", "s_bcnt1_i32_b32"):
        a = rs64(O[1]) if op.endswith("b64") else rs(O[1])
        if op == "s_not_b32":
            return lambda w: (d(w, _scc_nz(w, ~a(w) & M32)), nxt)[1]
        if op == "s_brev_b32":
            return lambda w: (d(w, int("{:032b}".format(a(w))[::-1], 2)), nxt)[1]
        if op == "s_abs_i32":
            def f(w):
                x = a(w)
                x = x - (1 << 32) if x >= 1 << 31 else x
                d(w, _scc_nz(w, abs(x) & M32))
                return nxt
            return f
        if op in ("s_ff1_i32_b64", "s_ff1_i32_b32"):
            def f(w):
                x = a(w)
                d(w, ((x & -x).bit_length() - 1) & M32 if x else M32)
                return nxt
            return f
        if op in ("s_flbit_i32_b64", "s_flbit_i32_b32"):   # leading zeros, -1 for zero
            width = 64 if op.endswith("64") else 32

            def f(w):
                x = a(w)
                d(w, (width - x.bit_length()) if x else M32)
                return nxt
            return f
        return lambda w: (d(w, _scc_nz(w, bin(a(w)).count("1"))), nxt)[1]
    if len(O) < 3:
        raise Unsupported(op)
    a, b = O[1], O[2]
    if op in ("s_lshl_b64", "s_lshr_b64"):
        ra, rb = rs64(a), rs(b)
        if op == "s_lshl_b64":
            return lambda w: (d(w, _scc_nz(w, (ra(w) << (rb(w) & 63)) & M64)), nxt)[1]
        return lambda w: (d(w, _scc_nz(w, ra(w) >> (rb(w) & 63))), nxt)[1]
    if is64:
        ra, rb = rs64(a), rs64(b)
        M = M64
    else:
        ra, rb = rs(a), rs(b)
        M = M32
    base = op[2:op.rindex("_")]
    if base in ("and", "or", "xor", "andn2", "orn2", "nand", "nor", "xnor"):
        fn = {"and": lambda x, y: x & y, "or": lambda x, y: x | y, "xor": lambda x, y: x ^ y,
              "andn2": lambda x, y: x & ~y & M, "orn2": lambda x, y: (x | ~y) & M,
              "nand": lambda x, y: ~(x & y) & M, "nor": lambda x, y: ~(x | y) & M,
              "xnor": lambda x, y: ~(x ^ y) & M}[base]
        return lambda w: (d(w, _scc_nz(w, fn(ra(w), rb(w)))), nxt)[1]
    if op == "s_add_u32":
        def f(w):
            r = ra(w) + rb(w)
            w.scc = r >> 32
            d(w, r & M32)
            return nxt
        return f
    if op == "s_addc_u32":
        def f(w):
            r = ra(w) + rb(w) + w.scc
            w.scc = r >> 32
            d(w, r & M32)
            return nxt
        return f
    if op == "s_sub_u32":
        def f(w):
            x, y = ra(w), rb(w)
            w.scc = 1 if y > x else 0
            d(w, (x - y) & M32)
            return nxt
        return f
    if op == "s_subb_u32":
        def f(w):
            x, y = ra(w), rb(w) + w.scc
            w.scc = 1 if y > x else 0
            d(w, (x - y) & M32)
            return nxt
        return f
    if op in ("s_add_i32", "s_sub_i32"):
        sub = op == "s_sub_i32"

        def f(w):
            x, y = ra(w), rb(w)
            x = x - (1 << 32) if x >= 1 << 31 else x
            y = y - (1 << 32) if y >= 1 << 31 else y
            r = x - y if sub else x + y
            w.scc = 1 if (r >= 1 << 31 or r < -(1 << 31)) else 0
            d(w, r & M32)
            return nxt
        return f
    if op == "s_mul_i32":
        return lambda w: (d(w, (ra(w) * rb(w)) & M32), nxt)[1]
    if op == "s_mul_hi_u32":
        return lambda w: (d(w, (ra(w) * rb(w)) >> 32), nxt)[1]
    if op == "s_mul_hi_i32":
        def f(w):
            x, y = ra(w), rb(w)
            x = x - (1 << 32) if x >= 1 << 31 else x
            y = y - (1 << 32) if y >= 1 << 31 else y
            d(w, ((x * y) >> 32) & M32)
            return nxt
        return f
    if op == "s_lshl_b32":
        return lambda w: (d(w, _scc_nz(w, (ra(w) << (rb(w) & 31)) & M32)), nxt)[1]
    if op == "s_lshr_b32":
        return lambda w: (d(w, _scc_nz(w, ra(w) >> (rb(w) & 31))), nxt)[1]
    if op == "s_ashr_i32":
        def f(w):
            x = ra(w)
            x = x - (1 << 32) if x >= 1 << 31 else x
            d(w, _scc_nz(w, (x >> (rb(w) & 31)) & M32))
            return nxt
        return f
    if op in ("s_bfe_u32", "s_bfe_i32"):
        signed = op.endswith("i32")

        def f(w):
            x, c = ra(w), rb(w)
            off, wid = c & 31, (c >> 16) & 0x7F
            r = (x >> off) & ((1 << wid) - 1) if wid else 0
            if signed and wid and (r >> (wid - 1)) & 1:
                r -= 1 << wid
            d(w, _scc_nz(w, r & M32))
            return nxt
        return f
    if op in ("s_min_i32", "s_max_i32", "s_min_u32", "s_max_u32"):
        signed, take_max = op.endswith("i32"), op.startswith("s_max")

        def f(w):
            x, y = ra(w), rb(w)
            xs = x - (1 << 32) if signed and x >= 1 << 31 else x
            ys = y - (1 << 32) if signed and y >= 1 << 31 else y
            first = xs > ys if take_max else xs < ys     # SCC: the first operand was taken
            w.scc = 1 if first else 0
            d(w, x if first else y)
            return nxt
        return f
    raise Unsupported(op)


# ---------------------------------------------------------------------- VALU --
def _compile_valu(op, O, mods, nxt):
    enc = ""
    for suf in ("_e32", "_e64", "_sdwa", "_dpp"):
        if op.endswith(suf):
            enc, op = suf[1:], op[: -len(suf)]
    if enc == "dpp":
        return _compile_dpp(op, O, mods, nxt)
    if enc == "sdwa":
        return _compile_sdwa(op, O, mods, nxt)
    if op.startswith("v_cmp_"):
        _, _, cmpop, ty = op.split("_")
        dst = ws(O[0])
        if cmpop == "u":
            a, b = _cmp_vals(ty, O[1]), _cmp_vals(ty, O[2])

            def f(w):
                x, y = a(w), b(w)
                dst(w, mask_of((np.isnan(x) | np.isnan(y)) & w.exec()))
                return nxt
            return f
        a, b, c = _cmp_vals(ty, O[1]), _cmp_vals(ty, O[2]), CMP[cmpop]

        def f(w):
            dst(w, mask_of(c(a(w), b(w)) & w.exec()))
            return nxt
        return f
    if op == "v_cndmask_b32":
        d, a, b = wv(O[0]), r32(O[1]), r32(O[2])
        m = rs64(O[3]) if len(O) > 3 else (lambda w: w.s[106] | (w.s[107] << 32))

        def f(w):
            d(w, np.where(bools_of(m(w)), b(w), a(w)))
            return nxt
        return f
    if op == "v_readfirstlane_b32":
        d, a = ws(O[0]), r32(O[1])

        def f(w):
            e = w.exec()
            x = vec(a(w))
            k = int(np.argmax(e)) if e.any() else 0
            d(w, int(x[k]))
            return nxt
        return f
    if op == "v_readlane_b32":
        d, a, l = ws(O[0]), r32(O[1]), rs(O[2])
        return lambda w: (d(w, int(vec(a(w))[l(w) & 63])), nxt)[1]
    if op == "v_writelane_b32":
        i, a, l = O[0].idx, rs(O[1]), rs(O[2])

        def f(w):
            w.v[i][l(w) & 63] = a(w)
            return nxt
        return f
    if op == "v_mov_b64":
        d, a = wv(O[0]), r64(O[1])
        return lambda w: (d(w, a(w)), nxt)[1]
    if op in ("v_lshlrev_b64", "v_lshrrev_b64", "v_ashrrev_i64"):
        d, a, b = wv(O[0]), r32(O[1]), r64(O[2])

        def f(w):
            s = (vec(a(w)) & U32(63)).astype(U64)
            x = vec(b(w), U64)
            if op == "v_lshlrev_b64":
                r = x << s
            elif op == "v_lshrrev_b64":
                r = x >> s
            else:
                r = (x.view(I64) >> s.astype(I64)).view(U64)
            d(w, r)
            return nxt
        return f
    if op == "v_lshl_add_u64":
        d, a, b, c = wv(O[0]), r64(O[1]), r32(O[2]), r64(O[3])

        def f(w):
            d(w, (vec(a(w), U64) << (vec(b(w)) & U32(63)).astype(U64)) + c(w))
            return nxt
        return f
    if op in ("v_mad_u64_u32", "v_mad_i64_i32"):
        d, sd, a, b, c = wv(O[0]), ws(O[1]), r32(O[2]), r32(O[3]), r64(O[4])
        signed = op == "v_mad_i64_i32"

        def f(w):
            e = w.exec()
            if signed:
                p = s32(a(w)).astype(object) * s32(b(w)).astype(object)
                cc = vec(c(w), U64).view(I64).astype(object)
                full = p + cc
                r = np.array([int(x) & M64 for x in full], dtype=U64)
                car = np.array([((int(x) >> 64) & 1) for x in full], dtype=bool)
            else:
                p = vec(a(w)).astype(U64) * vec(b(w)).astype(U64)
                r = p + c(w)
                car = r < p
            d(w, r)
            sd(w, mask_of(car & e))
            return nxt
        return f
    if op in ("v_add_co_u32", "v_sub_co_u32", "v_subrev_co_u32"):
        d, sd, a, b = wv(O[0]), ws(O[1]), r32(O[2]), r32(O[3])

        def f(w):
            x, y = vec(a(w)).astype(np.int64), vec(b(w)).astype(np.int64)
            if op == "v_add_co_u32":
                r = x + y
                car = r > M32
            elif op == "v_sub_co_u32":
                r = x - y
                car = r < 0
            else:
                r = y - x
                car = r < 0
            d(w, (r & M32).astype(U32))
            sd(w, mask_of(car & w.exec()))
            return nxt
        return f
    if op in ("v_addc_co_u32", "v_subb_co_u32", "v_subbrev_co_u32"):
        d, sd, a, b = wv(O[0]), ws(O[1]), r32(O[2]), r32(O[3])
        cin = rs64(O[4])

        def f(w):
            x, y = vec(a(w)).astype(np.int64), vec(b(w)).astype(np.int64)
            ci = bools_of(cin(w)).astype(np.int64)
            if op == "v_addc_co_u32":
                r = x + y + ci
                car = r > M32
            elif op == "v_subb_co_u32":
                r = x - y - ci
                car = r < 0
            else:
                r = y - x - ci
                car = r < 0
            d(w, (r & M32).astype(U32))
            sd(w, mask_of(car & w.exec()))
            return nxt
        return f
    if op == "v_bitop3_b32":
        d, a, b, c = wv(O[0]), r32(O[1]), r32(O[2]), r32(O[3])
        fn = _bitop3(int(mods["bitop3"], 0))
        return lambda w: (d(w, fn(a(w), b(w), c(w))), nxt)[1]
    if op == "v_fmac_f32":
        d, a, b = wv(O[0]), r32(O[1]), r32(O[2])
        di = O[0].idx

        def f(w):
            x = f32(a(w)).astype(np.longdouble) * f32(b(w)).astype(np.longdouble) + w.v[di].view(F32).astype(np.longdouble)
            d(w, bits(x.astype(F32)))
            return nxt
        return f
    if op in VALU1:
        d, a, fn = wv(O[0]), r32(O[1]), VALU1[op]
        return lambda w: (d(w, fn(a(w))), nxt)[1]
    if op in VALU2:
        d, a, b, fn = wv(O[0]), r32(O[1]), r32(O[2]), VALU2[op]
        return lambda w: (d(w, fn(a(w), b(w))), nxt)[1]
    if op in VALU3:
        d, a, b, c, fn = wv(O[0]), r32(O[1]), r32(O[2]), r32(O[3]), VALU3[op]
        return lambda w: (d(w, fn(a(w), b(w), c(w))), nxt)[1]
    raise Unsupported(op)


def _dpp_src(ctrl):
    """source lane of every lane for a DPP control; -1 where the source is out of range"""
    p = LANE % 16
    if ctrl.startswith("row_shl:"):
        n = int(ctrl.split(":")[1])
        return np.where(p + n < 16, LANE + n, -1)
    if ctrl.startswith("row_shr:"):
        n = int(ctrl.split(":")[1])
        return np.where(p - n >= 0, LANE - n, -1)
    if ctrl == "row_mirror":
        return LANE - p + (15 - p)
    if ctrl == "row_half_mirror":
        q = LANE % 8
        return LANE - q + (7 - q)
    if ctrl == "row_bcast:15":                 # lane 15 of the row below (rows 1..3)
        r = LANE // 16
        return np.where(r >= 1, 16 * r - 1, -1)
    if ctrl == "row_bcast:31":                 # lane 31 (rows 2 and 3)
        return np.where(LANE >= 32, 31, -1)
    if ctrl == "wave_shl:1":
        return np.where(LANE + 1 < 64, LANE + 1, -1)
    if ctrl == "wave_shr:1":
        return np.where(LANE - 1 >= 0, LANE - 1, -1)
    raise Unsupported("dpp " + ctrl)


def _compile_dpp(op, O, mods, nxt):
    ctrl = [k + (":" + v if v is not True else "") for k, v in mods.items()
            if k.startswith(("row_", "wave_", "quad_")) and k not in ("row_mask",)]
    if len(ctrl) != 1:
        raise Unsupported("dpp controls %s" % mods)
    src = _dpp_src(ctrl[0])
    if mods.get("bank_mask", "0xf") != "0xf":
        raise Unsupported("dpp bank mask")
    row_on = ((int(mods.get("row_mask", "0xf"), 16) >> (LANE // 16)) & 1).astype(bool)   # rows written
    bound0 = mods.get("bound_ctrl") in ("1", True, "0")
    d = wv(O[0])
    a = r32(O[1])
    b = r32(O[2]) if len(O) > 2 else None
    fn = VALU1.get(op) if b is None else VALU2.get(op)
    if fn is None:
        raise Unsupported("dpp op " + op)
    di = O[0].idx

    def f(w):
        e = w.exec()
        x = vec(a(w))
        ok = (src >= 0) & e[np.clip(src, 0, 63)]
        moved = np.where(ok, x[np.clip(src, 0, 63)], U32(0))
        r = fn(moved) if b is None else fn(moved, b(w))
        if not bound0:
            keep = ~ok
            r = np.where(keep, w.v[di], r)
        r = np.where(row_on, r, w.v[di])
        d(w, r)
        return nxt
    return f


def _sdwa_sel(x, sel, sext):
    x = vec(x)
    if sel == "DWORD":
        return x
    sh = {"BYTE_0": 0, "BYTE_1": 8, "BYTE_2": 16, "BYTE_3": 24, "WORD_0": 0, "WORD_1": 16}[sel]
    nb = 8 if sel.startswith("BYTE") else 16
    v = (x >> U32(sh)) & U32((1 << nb) - 1)
    if sext:
        return (_sx(v, nb) & M32).astype(U32)
    return v


def _compile_sdwa(op, O, mods, nxt):
    if op == "v_cndmask_b32":
        # lane-wise select of the two selected source fields by VCC, written whole
        if mods.get("dst_sel", "DWORD") != "DWORD":
            raise Unsupported("sdwa dst_sel for " + op)
        d, a, b = wv(O[0]), r32(O[1]), r32(O[2])
        s0, s1 = mods.get("src0_sel", "DWORD"), mods.get("src1_sel", "DWORD")
        x0, x1 = O[1].sext, O[2].sext

        def f(w):
            m = bools_of(w.s[106] | (w.s[107] << 32))
            d(w, np.where(m, _sdwa_sel(b(w), s1, x1), _sdwa_sel(a(w), s0, x0)))
            return nxt
        return f
    if op.startswith("v_cmp_"):
        # VOPC with operand selects: compare the selected fields, write the lane mask
        _, _, cmpop, ty = op.split("_")
        if ty not in ("u16", "i16", "u32", "i32") or cmpop not in CMP:
            raise Unsupported("sdwa compare " + op)
        dst = ws(O[0])
        a, b = r32(O[1]), r32(O[2])
        s0, s1 = mods.get("src0_sel", "DWORD"), mods.get("src1_sel", "DWORD")
        x0, x1 = O[1].sext, O[2].sext
        c = CMP[cmpop]
        nb = 16 if ty.endswith("16") else 32

        def val(x):
            x = vec(x).astype(I64) & ((1 << nb) - 1)
            return ((x ^ (1 << (nb - 1))) - (1 << (nb - 1))) if ty[0] == "i" else x

        def f(w):
            dst(w, mask_of(c(val(_sdwa_sel(a(w), s0, x0)), val(_sdwa_sel(b(w), s1, x1))) & w.exec()))
            return nxt
        return f
    if op in VALU1 and len(O) == 2:
        # one source with an operand select, written whole (dst_sel DWORD only)
        f1 = VALU1[op]
        a1, s01, x01 = r32(O[1]), mods.get("src0_sel", "DWORD"), O[1].sext
        if mods.get("dst_sel", "DWORD") != "DWORD":
            raise Unsupported("sdwa dst_sel for " + op)
        w1 = wv(O[0])
        return lambda w: (w1(w, vec(f1(_sdwa_sel(a1(w), s01, x01)))), nxt)[1]
    fn = VALU2.get(op)
    if fn is None:
        raise Unsupported("sdwa op " + op)
    d = O[0]
    a, b = r32(O[1]), r32(O[2])
    s0, s1 = mods.get("src0_sel", "DWORD"), mods.get("src1_sel", "DWORD")
    x0, x1 = O[1].sext, O[2].sext
    dsel, dun = mods.get("dst_sel", "DWORD"), mods.get("dst_unused", "UNUSED_PAD")
    wd = wv(d)
    di = d.idx

    def f(w):
        r = vec(fn(_sdwa_sel(a(w), s0, x0), _sdwa_sel(b(w), s1, x1)))
        if dsel != "DWORD":
            sh = {"BYTE_0": 0, "BYTE_1": 8, "BYTE_2": 16, "BYTE_3": 24, "WORD_0": 0, "WORD_1": 16}[dsel]
            nb = 8 if dsel.startswith("BYTE") else 16
            m = U32(((1 << nb) - 1) << sh)
            val = (r << U32(sh)) & m
            if dun == "UNUSED_PRESERVE":
                r = (w.v[di] & ~m) | val
            elif dun == "UNUSED_PAD":
                r = val
            else:
                raise Unsupported("sdwa dst_unused " + dun)
        wd(w, r)
        return nxt
    return f


# -------------------------------------------------------------------- memory --
def _offset(mods):
    return int(mods.get("offset", "0"), 0)


def _compile_scratch(op, O, mods, nxt):
    """Private (scratch) memory: every lane has its own bytes, w.priv[lane]; the address is
    vaddr + saddr + offset (either may be off), checked against the private segment size."""
    off = _offset(mods)
    kind = op.split("_", 1)[1]
    load = kind.startswith("load_")
    nbytes = {"dword": 4, "dwordx2": 8, "dwordx3": 12, "dwordx4": 16}.get(kind.split("_", 1)[1])
    if nbytes is None:
        raise Unsupported(op)
    vo, so = (O[1], O[2]) if load else (O[0], O[2])
    va = (lambda w: np.zeros(LANES, np.int64)) if vo.kind == "off" else (lambda w, r=r32(vo): vec(r(w)).astype(np.int64))
    sa = (lambda w: 0) if so.kind == "off" else (lambda w, r=rs(so): int(r(w)))
    reg = (O[0] if load else O[1]).idx

    def f(w):
        e = w.exec()
        if not e.any():
            return nxt
        addr = va(w) + sa(w) + off
        lanes = np.nonzero(e)[0]
        a = addr[lanes]
        if (a < 0).any() or (a + nbytes > w.priv.shape[1]).any():
            raise Fault("%s at pc 0x%x: outside the private segment (%d bytes)" % (op, w.pc, w.priv.shape[1]))
        for k in range(nbytes // 4):
            for j, ln in enumerate(lanes):
                p = int(a[j]) + 4 * k
                if load:
                    w.v[reg + k][ln] = w.priv[ln, p:p + 4].view("<u4")[0]
                else:
                    w.priv[ln, p:p + 4] = np.frombuffer(np.uint32(w.v[reg + k][ln]).tobytes(), U8)
        return nxt
    return f


def _flat_lds(w, addrs, nbytes, what):
    """(mask of the flat addresses that fall in the LDS aperture, their byte indices into the
    workgroup's LDS); an LDS address outside the kernel's LDS segment stops the run"""
    m = (addrs >= SHARED_APERTURE) & (addrs < SHARED_APERTURE + (1 << 32))
    if not m.any():
        return m, None
    offs = addrs[m] - SHARED_APERTURE
    if (offs + nbytes > w.wg.lds_size).any():
        raise Fault("%s: flat LDS access past the %d-byte segment" % (what, w.wg.lds_size))
    return m, offs[:, None] + np.arange(nbytes)


def _compile_global(op, O, mods, nxt):
    off = _offset(mods)
    flat = op.startswith("flat_")
    kind = op.split("_", 1)[1]

    def addr_of(vo: Opd, so: Opd | None):
        if so is None or so.kind == "off":
            va = r64(vo)
            return lambda w: vec(va(w), U64).astype(np.int64) + off
        sa, vv = rs64(so), r32(vo)
        return lambda w: np.int64(sa(w)) + vec(vv(w)).astype(np.int64) + off

    if kind.startswith("load_"):
        nbytes = {"load_dword": 4, "load_dwordx2": 8, "load_dwordx3": 12, "load_dwordx4": 16,
                  "load_ushort": 2, "load_ubyte": 1, "load_sshort": 2, "load_sbyte": 1}[kind]
        d = O[0]
        ad = addr_of(O[1], None if flat else O[2])
        di = d.idx

        def f(w):
            e = w.exec()
            if not e.any():
                return nxt
            addrs = ad(w)[e]
            what = "%s at pc 0x%x" % (op, w.pc)
            m, li = _flat_lds(w, addrs, nbytes, what) if flat else (None, None)
            if li is None:
                raw = w.wg.mem.gather(addrs, nbytes, what)
            else:                                   # flat: LDS lanes from the LDS, the rest from memory
                raw = np.empty((len(addrs), nbytes), U8)
                raw[m] = w.wg.lds[li]
                if (~m).any():
                    raw[~m] = w.wg.mem.gather(addrs[~m], nbytes, what).reshape(-1, nbytes)
                raw = raw.reshape(-1)
            if nbytes >= 4:
                vals = raw.view("<u4").reshape(len(addrs), nbytes // 4)
                for k in range(nbytes // 4):
                    w.v[di + k][e] = vals[:, k]
            else:
                v = raw.view("<u2" if nbytes == 2 else "<u1").reshape(-1).astype(np.int64)
                if kind in ("load_sshort", "load_sbyte"):
                    v = _sx(v, 8 * nbytes)
                w.v[di][e] = (v & M32).astype(U32)
            return nxt
        return f
    if kind.startswith("store_"):
        nbytes = {"store_dword": 4, "store_dwordx2": 8, "store_dwordx3": 12, "store_dwordx4": 16,
                  "store_short": 2, "store_byte": 1}[kind]
        ad = addr_of(O[0], None if flat else O[2])
        si = O[1].idx

        def f(w):
            e = w.exec()
            if not e.any():
                return nxt
            addrs = ad(w)[e]
            if nbytes >= 4:
                data = np.stack([w.v[si + k][e] for k in range(nbytes // 4)], axis=1).astype("<u4").view(U8)
            else:
                data = (w.v[si][e] & U32((1 << (8 * nbytes)) - 1)).astype("<u2" if nbytes == 2 else "<u1").view(U8)
            data = data.reshape(len(addrs), nbytes)
            what = "%s at pc 0x%x" % (op, w.pc)
            m, li = _flat_lds(w, addrs, nbytes, what) if flat else (None, None)
            if li is None:
                w.wg.mem.scatter(addrs, data, what)
            else:
                w.wg.lds[li] = data[m]
                if (~m).any():
                    w.wg.mem.scatter(addrs[~m], data[~m], what)
            return nxt
        return f
    if kind.startswith("atomic_"):
        aop = kind[len("atomic_"):]
        ret = len(O) == 4 or (flat and len(O) == 3)
        if ret:
            d, vo, do, so = O[0], O[1], O[2], (O[3] if not flat else None)
        else:
            d, vo, do, so = None, O[0], O[1], (O[2] if not flat else None)
        ad = addr_of(vo, so)
        di = d.idx if d is not None else None
        dd = do.idx
        is64 = aop.endswith("_x2")
        if is64 or aop not in ("add", "smin", "umin", "smax", "umax", "cmpswap", "add_f32", "or", "and"):
            raise Unsupported(op)             # refused when the code object is read, not when run

        def f(w):
            e = w.exec()
            lanes = np.nonzero(e)[0]
            addrs = ad(w)
            what = "%s at pc 0x%x" % (op, w.pc)
            for l in lanes:
                a = int(addrs[l])
                old = struct.unpack("<I", w.wg.mem.read(a, 4, what))[0]
                x = int(w.v[dd][l])
                if aop == "add":
                    new = (old + x) & M32
                elif aop == "smin":
                    os_ = old - (1 << 32) if old >= 1 << 31 else old
                    xs = x - (1 << 32) if x >= 1 << 31 else x
                    new = old if os_ <= xs else x
                elif aop == "umin":
                    new = min(old, x)
                elif aop == "smax":
                    os_ = old - (1 << 32) if old >= 1 << 31 else old
                    xs = x - (1 << 32) if x >= 1 << 31 else x
                    new = old if os_ >= xs else x
                elif aop == "umax":
                    new = max(old, x)
                elif aop == "and":
                    new = old & x
                elif aop == "cmpswap":
                    cmp = int(w.v[dd + 1][l])
                    new = x if old == cmp else old
                elif aop == "add_f32":
                    new = int(np.array([np.array(old, U32).view(F32) + np.array(x, U32).view(F32)], F32).view(U32)[0])
                elif aop == "or":
                    new = old | x
                else:
                    raise Unsupported(op)
                w.wg.mem.write(a, struct.pack("<I", new), what)
                if di is not None:
                    w.v[di][l] = old
            return nxt
        return f
    raise Unsupported(op)


def _compile_ds(op, O, mods, nxt):
    # LDS addresses are 32-bit: the offset field is added to the address register modulo 2^32
    # (the compiler folds constants into the offset against a base below them)
    kind = op[3:]
    off = _offset(mods)

    if kind == "bpermute_b32":
        # lane l of the result takes data from lane ((addr[l] + offset) / 4) mod 64; a source
        # lane outside exec gives 0; no LDS memory is touched
        di, va, vd = O[0].idx, r32(O[1]), r32(O[2])

        def f(w):
            e = w.exec()
            lane = ((vec(va(w)).astype(np.int64) + off) >> 2) & 63
            data = np.where(e, vec(vd(w)), U32(0)).astype(U32)
            w.v[di] = np.where(e, data[lane], w.v[di])
            return nxt
        return f

    def lds(w, addrs, n, what):
        lim = w.wg.lds_size
        bad = (addrs < 0) | (addrs + n > lim)
        if bad.any():
            raise Fault("%s at pc 0x%x: LDS [%d, %d) outside the %d-byte segment" %
                        (what, w.pc, int(addrs[bad][0]), int(addrs[bad][0]) + n, lim))
        return w.wg.lds

    if kind in ("read_b32", "read_b64", "read_b96", "read_b128", "read_u16", "read_u8"):
        n = {"read_b32": 4, "read_b64": 8, "read_b96": 12, "read_b128": 16, "read_u16": 2, "read_u8": 1}[kind]
        di, va = O[0].idx, r32(O[1])

        def f(w):
            e = w.exec()
            if not e.any():
                return nxt
            addrs = (vec(va(w)).astype(np.int64)[e] + off) & M32
            mem = lds(w, addrs, n, op)
            raw = mem[addrs[:, None] + np.arange(n)]
            if n >= 4:
                vals = raw.view("<u4").reshape(len(addrs), n // 4)
                for k in range(n // 4):
                    w.v[di + k][e] = vals[:, k]
            else:
                w.v[di][e] = raw.view("<u2" if n == 2 else "<u1").reshape(-1).astype(U32)
            return nxt
        return f
    if kind in ("read2_b32", "read2_b64", "read2st64_b32", "read2st64_b64"):
        esz = 8 if kind.endswith("b64") else 4
        unit = esz * (64 if "st64" in kind else 1)
        di, va = O[0].idx, r32(O[1])
        o0, o1 = int(mods.get("offset0", "0"), 0) * unit, int(mods.get("offset1", "0"), 0) * unit

        def f(w):
            e = w.exec()
            if not e.any():
                return nxt
            base = vec(va(w)).astype(np.int64)[e]
            for k, o in enumerate((o0, o1)):
                addrs = (base + o) & M32
                mem = lds(w, addrs, esz, op)
                vals = mem[addrs[:, None] + np.arange(esz)].view("<u4").reshape(len(addrs), esz // 4)
                for j in range(esz // 4):
                    w.v[di + k * (esz // 4) + j][e] = vals[:, j]
            return nxt
        return f
    if kind in ("write_b32", "write_b64", "write_b96", "write_b128", "write_b16", "write_b8"):
        n = {"write_b32": 4, "write_b64": 8, "write_b96": 12, "write_b128": 16, "write_b16": 2, "write_b8": 1}[kind]
        va, si = r32(O[0]), O[1].idx

        def f(w):
            e = w.exec()
            if not e.any():
                return nxt
            addrs = (vec(va(w)).astype(np.int64)[e] + off) & M32
            mem = lds(w, addrs, n, op)
            if n >= 4:
                data = np.stack([w.v[si + k][e] for k in range(n // 4)], axis=1).astype("<u4").view(U8)
            else:
                data = (w.v[si][e] & U32((1 << (8 * n)) - 1)).astype("<u2" if n == 2 else "<u1").view(U8)
            data = data.reshape(len(addrs), n)
            for k in range(len(addrs)):            # lane order: the highest lane wins
                mem[addrs[k]:addrs[k] + n] = data[k]
            return nxt
        return f
    if kind in ("write2_b32", "write2_b64", "write2st64_b32", "write2st64_b64"):
        esz = 8 if kind.endswith("b64") else 4
        unit = esz * (64 if "st64" in kind else 1)
        va, s0, s1 = r32(O[0]), O[1].idx, O[2].idx
        o0, o1 = int(mods.get("offset0", "0"), 0) * unit, int(mods.get("offset1", "0"), 0) * unit

        def f(w):
            e = w.exec()
            if not e.any():
                return nxt
            base = vec(va(w)).astype(np.int64)[e]
            for o, si in ((o0, s0), (o1, s1)):
                addrs = (base + o) & M32
                mem = lds(w, addrs, esz, op)
                data = np.stack([w.v[si + j][e] for j in range(esz // 4)], axis=1).astype("<u4").view(U8)
                data = data.reshape(len(addrs), esz)
                for k in range(len(addrs)):
                    mem[addrs[k]:addrs[k] + esz] = data[k]
            return nxt
        return f
    if kind == "bpermute_b32":
        di, va, da = O[0].idx, r32(O[1]), r32(O[2])

        def f(w):
            e = w.exec()
            idx = ((vec(va(w)).astype(np.int64) + off) >> 2) & 63
            data = vec(da(w))
            srcok = e[idx]
            w.v[di] = np.where(e, np.where(srcok, data[idx], U32(0)), w.v[di])
            return nxt
        return f
    if kind in ("add_rtn_u32", "and_rtn_b32", "or_rtn_b32", "xor_rtn_b32", "cmpst_rtn_b32"):
        # the old word goes to vdst; cmpst stores data1 where the word equals data0
        di, va, da = O[0].idx, r32(O[1]), r32(O[2])
        db = r32(O[3]) if kind == "cmpst_rtn_b32" else None

        def f(w):
            e = w.exec()
            lanes = np.nonzero(e)[0]
            addrs = (vec(va(w)).astype(np.int64) + off) & M32
            data = vec(da(w))
            data1 = vec(db(w)) if db is not None else None
            mem = lds(w, addrs[e], 4, op) if len(lanes) else None
            out = w.v[di].copy()
            for l in lanes:                        # lanes in order, one at a time
                a = int(addrs[l])
                old = int(mem[a:a + 4].view("<u4")[0])
                x = int(data[l])
                if kind == "add_rtn_u32":
                    new = (old + x) & M32
                elif kind == "and_rtn_b32":
                    new = old & x
                elif kind == "or_rtn_b32":
                    new = old | x
                elif kind == "xor_rtn_b32":
                    new = old ^ x
                else:
                    new = int(data1[l]) if old == x else old
                mem[a:a + 4] = np.array([new], "<u4").view(U8)
                out[l] = old
            w.v[di] = out
            return nxt
        return f
    if kind == "min_u64":
        va, da = r32(O[0]), O[1]
        di = da.idx

        def f(w):
            e = w.exec()
            lanes = np.nonzero(e)[0]
            addrs = (vec(va(w)).astype(np.int64) + off) & M32
            mem = lds(w, addrs[e], 8, op) if len(lanes) else None
            for l in lanes:
                a = int(addrs[l])
                old = int(mem[a:a + 8].view("<u8")[0])
                x = int(w.v[di][l]) | (int(w.v[di + 1][l]) << 32)
                mem[a:a + 8] = np.array([min(old, x)], "<u8").view(U8)
            return nxt
        return f
    if kind in ("or_b32", "min_i32", "add_u32", "max_i32", "min_u32", "and_b32"):
        va, da = r32(O[0]), r32(O[1])

        def f(w):
            e = w.exec()
            lanes = np.nonzero(e)[0]
            addrs = (vec(va(w)).astype(np.int64) + off) & M32
            data = vec(da(w))
            mem = lds(w, addrs[e], 4, op) if len(lanes) else None
            for l in lanes:
                a = int(addrs[l])
                old = int(mem[a:a + 4].view("<u4")[0])
                x = int(data[l])
                if kind == "or_b32":
                    new = old | x
                elif kind == "and_b32":
                    new = old & x
                elif kind == "add_u32":
                    new = (old + x) & M32
                elif kind == "min_u32":
                    new = min(old, x)
                else:
                    os_ = old - (1 << 32) if old >= 1 << 31 else old
                    xs = x - (1 << 32) if x >= 1 << 31 else x
                    new = (min if kind == "min_i32" else max)(os_, xs) & M32
                mem[a:a + 4] = np.array([new], "<u4").view(U8)
            return nxt
        return f
    raise Unsupported(op)


# ------------------------------------------------------------------- program --
class Program:
    """The code object's instructions, compiled lazily, by address."""

    def __init__(self, kernels, instrs):
        self.kernels = kernels
        self.text = {}
        self.next = {}
        for k, (pc, t) in enumerate(instrs):
            self.text[pc] = t
            self.next[pc] = instrs[k + 1][0] if k + 1 < len(instrs) else None
        self.compiled = {}

    def at(self, pc):
        ins = self.compiled.get(pc)
        if ins is None:
            if pc not in self.text:
                raise Fault("jump to 0x%x, not an instruction" % pc)
            ins = compile_instr(pc, self.text[pc], self.next[pc])
            self.compiled[pc] = ins
        return ins


class Workgroup:
    __slots__ = ("mem", "lds", "lds_size")


class Dispatch:
    """One kernel launch: kernarg segment and dispatch packet in registered memory."""

    def __init__(self, prog: Program, mem: Memory, name: str, grid, block, explicit: bytes, slice_=0):
        self.prog, self.mem, self.name = prog, mem, name
        self.k = k = prog.kernels[name]
        self.grid, self.block = tuple(grid), tuple(block)
        self.slice = slice_
        # kernarg: explicit arguments as packed by the caller, hidden ones from the metadata
        ka = bytearray(max(k.kernarg_size, 16) + 64)
        ka[:len(explicit)] = explicit
        for off, size, kind in k.args:
            val = None
            g, b = self.grid, self.block
            if kind.startswith("hidden_block_count_"):
                val = g["xyz".index(kind[-1])]
            elif kind.startswith("hidden_group_size_"):
                val = b["xyz".index(kind[-1])]
            elif kind.startswith("hidden_remainder_"):
                val = 0
            elif kind.startswith("hidden_global_offset_"):
                val = 0
            elif kind == "hidden_grid_dims":
                val = 3 if g[2] > 1 or b[2] > 1 else (2 if g[1] > 1 or b[1] > 1 else 1)
            elif kind.startswith("hidden_"):
                raise Unsupported("hidden argument " + kind)
            if val is not None:
                ka[off:off + size] = int(val).to_bytes(size, "little")
        self.kernarg = np.frombuffer(bytes(ka), U8).copy()
        self.ka_addr = self.kernarg.ctypes.data
        mem.add(self.ka_addr, len(self.kernarg), self.kernarg)
        pk = bytearray(64)
        struct.pack_into("<HHHHHH", pk, 0, 0, 3, b[0], b[1], b[2], 0)
        struct.pack_into("<III", pk, 12, g[0] * b[0], g[1] * b[1], g[2] * b[2])
        struct.pack_into("<II", pk, 24, 0, k.group_segment)
        struct.pack_into("<Q", pk, 40, self.ka_addr)
        self.packet = np.frombuffer(bytes(pk), U8).copy()
        self.pk_addr = self.packet.ctypes.data
        mem.add(self.pk_addr, 64, self.packet)
        d = k.desc
        self.rsrc1, self.rsrc2 = struct.unpack_from("<II", d, 48)
        self.kcp = struct.unpack_from("<H", d, 56)[0]
        if struct.unpack_from("<H", d, 58)[0]:
            raise Unsupported("kernarg preload")
        # a private segment is only supported with architected flat scratch (scratch_* with no
        # buffer descriptor or flat-scratch SGPRs); every lane's bytes live in Wave.priv
        if self.kcp & 1 or self.kcp & 0x20:
            raise Unsupported("private segment buffer / flat scratch init SGPRs")
        self.nvgpr = 512

    def done(self):
        self.mem.remove(self.ka_addr)
        self.mem.remove(self.pk_addr)

    def _init_wave(self, wid, wg_id, nthreads):
        w = Wave(self.nvgpr)
        w.wid = wid
        s = w.s
        k = 0
        kcp = self.kcp
        if kcp & 2:                                # dispatch ptr
            s[k], s[k + 1] = self.pk_addr & M32, self.pk_addr >> 32
            k += 2
        if kcp & 4:                                # queue ptr
            k += 2
        if kcp & 8:                                # kernarg segment ptr
            s[k], s[k + 1] = self.ka_addr & M32, self.ka_addr >> 32
            k += 2
        if kcp & 16:                               # dispatch id
            k += 2
        if kcp & 64:
            k += 1
        nuser = (self.rsrc2 >> 1) & 31
        if k != nuser:
            raise Unsupported("user SGPR layout (%d set up, %d declared)" % (k, nuser))
        for axis in range(3):
            if self.rsrc2 & (1 << (7 + axis)):
                s[k] = wg_id[axis]
                k += 1
        if self.rsrc2 & (1 << 10):
            raise Unsupported("workgroup info SGPR")
        if self.rsrc2 & 1:                         # private segment wave offset: scratch is per wave here
            s[k] = 0
            k += 1
        bx, by, bz = self.block
        t = wid * 64 + LANE
        tx, ty, tz = t % bx, (t // bx) % by, t // (bx * by)
        w.v[0] = (tx | (ty << 10) | (tz << 20)).astype(U32)
        active = t < nthreads
        m = mask_of(active)
        s[126], s[127] = m & M32, m >> 32
        w.pc = self.k.entry
        return w

    def run(self, max_instr=50_000_000):
        bx, by, bz = self.block
        nthreads = bx * by * bz
        nwaves = (nthreads + 63) // 64
        count = 0
        gx, gy, gz = self.grid
        for z in range(gz):
            for y in range(gy):
                for x in range(gx):
                    wg = Workgroup()
                    wg.mem = self.mem
                    wg.lds_size = self.k.group_segment
                    wg.lds = np.full(max(self.k.group_segment, 4), 0x5A, U8)
                    waves = [self._init_wave(i, (x, y, z), nthreads) for i in range(nwaves)]
                    for w in waves:
                        w.wg = wg
                        w.priv = np.full((LANES, max(self.k.private_segment, 4)), 0x5A, U8)
                    count += self._run_group(waves, max_instr - count, (x, y, z))
        return count

    trace = None      # callable(dispatch, wave, instr) called before every instruction

    def _run_group(self, waves, budget, wg_id):
        prog = self.prog
        count = 0
        tr = Dispatch.trace
        sl = self.slice if self.slice > 0 else 1 << 62
        while True:
            live = [w for w in waves if not w.done]
            if not live:
                return count
            if all(w.barrier for w in live):
                for w in live:
                    w.barrier = False
                continue
            progressed = False
            for w in live:
                if w.barrier:
                    continue
                n = 0
                while not w.done and not w.barrier and n < sl:
                    ins = prog.at(w.pc)
                    if tr is not None:
                        tr(self, w, ins)
                    try:
                        nx = ins.fn(w)
                    except Fault as e:
                        raise Fault("%s, workgroup %s wave %d: %s [%s]" % (self.name, wg_id, w.wid, e, ins.text)) from None
                    except Unsupported as e:
                        raise Unsupported("%s [%s at 0x%x]" % (e, ins.text, ins.pc)) from None
                    n += 1
                    if nx is None:
                        break
                    w.pc = nx
                count += n
                progressed = progressed or n > 0
                if count > budget:
                    raise Fault("%s: instruction budget exhausted (a wave that never ends)" % self.name)
            if not progressed:
                raise Fault("%s: no wave can progress" % self.name)
