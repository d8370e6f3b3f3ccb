"""Run the library's C ABI with its kernels executed by the gfx950 interpreter.

The host side is the library's own host code, built for the CPU as a shared object whose
kernel launches and device allocations go to hooks (tests/cpu_emulation, variant "isa").  Each
launch runs the matching kernel of the real code object (paper_2606_04801_amd/
libflashcubical.so) instruction by instruction.  Inputs, outputs and the workspace are numpy
arrays registered as device memory; nothing else is addressable by the kernels.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.join(os.path.dirname(HERE), "cpu_emulation"))
sys.path.insert(0, ROOT)

import build as emu_build  # noqa: E402
import codeobj  # noqa: E402
from gfx950_sim import Dispatch, Fault, Memory, Program  # noqa: E402

LIB = os.path.join(ROOT, "paper_2606_04801_amd", "libflashcubical.so")
LAUNCH = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint), ctypes.c_void_p, ctypes.c_size_t)
ALLOC = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int)


class ph_shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("ext", ctypes.c_int32 * 3)]


class ph_pairs(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_void_p), ("birth", ctypes.c_void_p), ("death", ctypes.c_void_p),
                ("birth_cell", ctypes.c_void_p), ("death_cell", ctypes.c_void_p),
                ("birth_vertex", ctypes.c_void_p), ("death_vertex", ctypes.c_void_p)]


class ph_tuning(ctypes.Structure):
    _fields_ = [("tile2d", ctypes.c_int32), ("tile3d", ctypes.c_int32)]


PAIR_FIELDS = [("dim", np.int8), ("birth", np.float32), ("death", np.float32), ("birth_cell", np.int64),
               ("death_cell", np.int64), ("birth_vertex", np.int32), ("death_vertex", np.int32)]


IN_FLAGS = {np.dtype(np.float32): 0, np.dtype(np.uint8): 4, np.dtype(np.uint16): 8}   # PH_IN_U8, PH_IN_U16


def as_input(a):
    """the array in its input element type: uint8 and uint16 stay, anything else is float32"""
    a = np.ascontiguousarray(a)
    return a if a.dtype in (np.uint8, np.uint16) else a.astype(np.float32)


def make_shape(shape):
    ext = list(shape) + [0] * (3 - len(shape))
    return ph_shape(len(shape), (ctypes.c_int32 * 3)(*ext))


class IsaRunner:
    """slice_: instructions a wave runs before the next wave of its workgroup gets a turn
    (0: run to the next barrier)."""

    # one host library per process: its device allocations (the lookup tables, made once)
    # live in one memory map shared by every runner, and its hooks call the newest runner
    _mem = Memory()
    _current = None
    _hooks = None

    def __init__(self, slice_: int = 0, lib_path: str = LIB):
        kernels, instrs = codeobj.load(lib_path)
        self.prog = Program(kernels, instrs)
        self.host = ctypes.CDLL(emu_build.build("isa"))
        self.mem = IsaRunner._mem
        self.slice = slice_
        self.error = None
        self.launches = []
        self.keep = []
        IsaRunner._current = self
        if IsaRunner._hooks is None:
            IsaRunner._hooks = (LAUNCH(lambda *a: IsaRunner._current._on_launch(*a)),
                                ALLOC(lambda *a: IsaRunner._current._on_alloc(*a)))
            self.host.emu_isa_set_hooks(*IsaRunner._hooks)
        H = self.host
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        H.ph_capacity_bound.argtypes = [ph_shape]
        H.ph_capacity_bound.restype = i64
        H.ph_capacity_bound_flags.argtypes = [ph_shape, u32]
        H.ph_capacity_bound_flags.restype = i64
        H.ph_workspace_bytes.argtypes = [ctypes.POINTER(ph_shape), i32, u32]
        H.ph_workspace_bytes.restype = ctypes.c_size_t
        H.ph_diagram.argtypes = [vp, ph_shape, u32, ph_pairs, i64, vp, vp, vp, ctypes.c_size_t, vp]
        H.ph_diagram_batch.argtypes = [i32, vp, vp, vp, ctypes.POINTER(ph_shape), u32, ph_pairs, vp, vp, vp,
                                       ctypes.POINTER(ph_tuning), vp, ctypes.c_size_t, vp]
        H.ph_backward.argtypes = [i32, ph_pairs, vp, vp, vp, vp, vp, vp, i64, vp]
        
    # ------------------------------------------------------------------ hooks --
    def _on_launch(self, name, dims, args, n):
        if self.error is not None:
            return
        try:
            nm = name.decode()
            if nm not in self.prog.kernels:
                raise Fault("launch of %s: no such kernel in the code object" % nm)
            k = self.prog.kernels[nm]
            explicit = [(o, s) for o, s, kind in k.args if not kind.startswith("hidden_")]
            end = max(o + s for o, s in explicit) if explicit else 0
            if end != n:
                raise Fault("%s: host packed %d argument bytes, the kernel takes %d" % (nm, n, end))
            d = Dispatch(self.prog, self.mem, nm, [dims[i] for i in range(3)], [dims[i] for i in range(3, 6)],
                         ctypes.string_at(args, n), self.slice)
            try:
                cnt = d.run()
            finally:
                d.done()
            self.launches.append((nm, tuple(dims[i] for i in range(6)), cnt))
        except BaseException as e:            # reported after the C call returns
            self.error = e

    def _on_alloc(self, p, n, free):
        if free:
            self.mem.remove(p)
        else:
            self.mem.add(p, n)

    def dev(self, arr: np.ndarray) -> np.ndarray:
        """register a numpy array as device memory"""
        arr = np.ascontiguousarray(arr)
        self.mem.add(arr.ctypes.data, max(arr.nbytes, 1), arr.reshape(-1).view(np.uint8))
        self.keep.append(arr)
        return arr

    def release(self):
        for a in self.keep:
            self.mem.remove(a.ctypes.data)
        self.keep = []

    def _check(self, rc, what):
        if self.error is not None:
            e, self.error = self.error, None
            raise e
        if rc != 0:
            raise RuntimeError("%s returned %d" % (what, rc))

    def _pairs(self, cap):
        bufs = {f: self.dev(np.full(max(cap, 1), 0x7B, dtype=t) if t != np.float32 else
                            np.full(max(cap, 1), np.nan, dtype=t)) for f, t in PAIR_FIELDS}
        return bufs, ph_pairs(*[bufs[f].ctypes.data for f, _ in PAIR_FIELDS])

    @staticmethod
    def _records(bufs, start, count):
        import oracle
        out = np.zeros(count, oracle.PAIR_DTYPE)
        for f, _ in PAIR_FIELDS:
            out[f] = bufs[f][start:start + count]
        return out

    # -------------------------------------------------------------- entry points --
    def diagram(self, img: np.ndarray, capacity: int | None = None, tfilt: bool = False, h1: bool = False):
        """(pairs, status, count) of ph_diagram on one image or volume (T-filtration with
        tfilt, flag 16; a volume's H1 with h1, flag 32)"""
        img = self.dev(as_input(img))
        flags = 3 | IN_FLAGS[img.dtype] | (16 if tfilt else 0) | (32 if h1 else 0)
        shp = make_shape(img.shape)
        if capacity is not None:
            cap = capacity
        elif h1:
            cap = int(self.host.ph_capacity_bound_flags(shp, flags))
        else:
            bound = make_shape(tuple(e + 2 for e in img.shape)) if tfilt else shp
            cap = int(self.host.ph_capacity_bound(bound))
        bufs, pr = self._pairs(cap)
        count = self.dev(np.full(1, -7, np.int64))
        status = self.dev(np.full(1, -77, np.int32))
        nb = int(self.host.ph_workspace_bytes(ctypes.byref(shp), 1, flags))
        ws = self.dev(np.frombuffer(np.random.default_rng(5).bytes(nb), np.uint8).copy())
        rc = self.host.ph_diagram(img.ctypes.data, shp, flags, pr, cap, count.ctypes.data, status.ctypes.data,
                                  ws.ctypes.data, nb, None)
        self._check(rc, "ph_diagram")
        n = int(count[0])
        res = self._records(bufs, 0, min(n, cap)) if status[0] in (0, -3) else None
        self.release()
        return res, int(status[0]), n

    def batch(self, imgs, tuning=None, backward=False):
        """per-instance (pairs, status) of ph_diagram_batch, and the gradient of the loss sum
        over finite pairs of (death - birth)^2 from ph_backward when asked"""
        imgs = [as_input(a) for a in imgs]
        assert len({a.dtype for a in imgs}) == 1, "one element type per batch"
        flags = 3 | IN_FLAGS[imgs[0].dtype]
        n = len(imgs)
        shapes = (ph_shape * n)(*[make_shape(a.shape) for a in imgs])
        sizes = [a.size for a in imgs]
        caps = [int(self.host.ph_capacity_bound(shapes[i])) for i in range(n)]
        img_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        out_off = np.concatenate([[0], np.cumsum(caps)]).astype(np.int64)
        flat = self.dev(np.concatenate([a.reshape(-1) for a in imgs]))
        d_img_off = self.dev(img_off[:-1].copy())
        d_out_off = self.dev(out_off.copy())
        d_shapes = self.dev(np.array([[len(a.shape)] + list(a.shape) + [0] * (3 - a.ndim) for a in imgs], np.int32))
        bufs, pr = self._pairs(int(out_off[-1]))
        counts = self.dev(np.full(n, -7, np.int64))
        status = self.dev(np.full(n, -77, np.int32))
        nb = int(self.host.ph_workspace_bytes(shapes, n, 3))
        ws = self.dev(np.frombuffer(np.random.default_rng(6).bytes(nb), np.uint8).copy())
        tp = ctypes.byref(ph_tuning(*tuning)) if tuning is not None else None
        rc = self.host.ph_diagram_batch(n, flat.ctypes.data, d_img_off.ctypes.data, d_shapes.ctypes.data, shapes, flags, pr,
                                        d_out_off.ctypes.data, counts.ctypes.data, status.ctypes.data, tp,
                                        ws.ctypes.data, nb, None)
        self._check(rc, "ph_diagram_batch")
        res = [(self._records(bufs, int(out_off[i]), int(counts[i])) if status[i] == 0 else None, int(status[i]))
               for i in range(n)]
        grad = None
        if backward:
            gb = self.dev(np.zeros(int(out_off[-1]) or 1, np.float32))
            gd = self.dev(np.zeros(int(out_off[-1]) or 1, np.float32))
            for i in range(n):
                for j in range(int(counts[i])):
                    k = int(out_off[i]) + j
                    if bufs["death_cell"][k] < 0:
                        continue
                    dlt = np.float32(bufs["death"][k] - bufs["birth"][k])
                    gb[k], gd[k] = -2 * dlt, 2 * dlt
            g = self.dev(np.full(int(img_off[-1]), np.nan, np.float32))
            rc = self.host.ph_backward(n, pr, d_out_off.ctypes.data, counts.ctypes.data, gb.ctypes.data,
                                       gd.ctypes.data, g.ctypes.data, d_img_off.ctypes.data, int(img_off[-1]), None)
            self._check(rc, "ph_backward")
            grad = g.copy()
        self.release()
        return res, grad
