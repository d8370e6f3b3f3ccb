"""CPU oracle for V- and T-filtration cubical persistence over F2 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The GPU library never links, loads or calls it, and it shares no
code with that library.

``diagram`` wraps the plain C column reduction in ``cubical_oracle.c``:
  * the cubical complex and V-filtration of paper Sec. 2.2 (cell value = max of its
    vertices' pixel values);
  * the fully refined order of paper Sec. 2.3 (lower-star vertex by value then pixel index,
    then dimension, then doubled-grid cell index);
  * standard F2 boundary-matrix reduction (paper Sec. 2.1), zero-persistence pairs omitted
    (paper Sec. 2.3).

``diagram(..., filtration="T")`` takes the pixels as the top cells instead (paper Sec. 2.2):
a cell's value is the minimum over the top cells containing it, the first-order tie-break is
the top cell through which it enters (the pixel order's minimum of those), and pairs come
sorted by (dim, death key), essential classes last.

``gradient`` is the reference backward: scatter of dL/dbirth and dL/ddeath to the pixel that
attains each critical cell's value, accumulated in FP32 in output order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cubical_oracle.c")
_LIB = os.path.join(_HERE, "libcubical_oracle.so")

FULL = 0    # reduce the whole boundary matrix (all dimensions)
SPLIT = 1   # reduce only the blocks of the requested dimensions (top dim by coboundary)

PAIR_DTYPE = np.dtype([
    ("dim", np.int8), ("birth", np.float32), ("death", np.float32),
    ("birth_cell", np.int64), ("death_cell", np.int64),
    ("birth_vertex", np.int32), ("death_vertex", np.int32),
])


class _Pair(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("birth", ctypes.c_float), ("death", ctypes.c_float),
                ("birth_cell", ctypes.c_int64), ("death_cell", ctypes.c_int64),
                ("birth_vertex", ctypes.c_int32), ("death_vertex", ctypes.c_int32)]


_C_DTYPE = np.dtype([("dim", np.int32), ("birth", np.float32), ("death", np.float32),
                     ("birth_cell", np.int64), ("death_cell", np.int64),
                     ("birth_vertex", np.int32), ("death_vertex", np.int32)], align=True)
assert _C_DTYPE.itemsize == ctypes.sizeof(_Pair)


class OracleError(RuntimeError):
    pass


_ERRORS = {-1: "invalid argument", -2: "NaN in input", -4: "out of memory"}


def build(force: bool = False) -> str:
    """Compile the oracle with the host C compiler (plain C99, -O3; ISO C mode keeps every
    floating-point operation as written, no contraction into fused multiply-adds)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.or_diagram.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.POINTER(_Pair)),
                                   ctypes.POINTER(ctypes.c_int64)]
        lib.or_diagram.restype = ctypes.c_int
        lib.or_diagram_t.argtypes = lib.or_diagram.argtypes
        lib.or_diagram_t.restype = ctypes.c_int
        lib.or_free.argtypes = [ctypes.c_void_p]
        lib.or_gradient.argtypes = [ctypes.POINTER(_Pair), ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        lib.or_gradient.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_dims(ndim: int) -> tuple:
    """H0 and the top dimension (H1 for images, H2 for volumes)."""
    return (0, ndim - 1)


def diagram(img, dims=None, method: int = SPLIT, keep_zero: bool = False,
            filtration: str = "V") -> np.ndarray:
    """Persistence pairs of ``img`` (2D or 3D float32) under the V- or T-filtration; V pairs
    sorted by (dim, birth key), T pairs by (dim, death key) with essential classes last.

    Returns a structured array with fields of ``PAIR_DTYPE``.  ``dims`` lists the homology
    dimensions wanted (default: H0 and H_top).  ``keep_zero`` keeps zero-persistence pairs
    (used only by the pair-count checks).
    """
    a = np.ascontiguousarray(img, dtype=np.float32)
    if a.ndim not in (2, 3):
        raise OracleError("ndim must be 2 or 3")
    if dims is None:
        dims = default_dims(a.ndim)
    mask = 0
    for d in dims:
        mask |= 1 << int(d)
    if filtration not in ("V", "T"):
        raise OracleError("filtration must be 'V' or 'T'")
    lib = _load()
    fn = lib.or_diagram if filtration == "V" else lib.or_diagram_t
    ext = (ctypes.c_int64 * a.ndim)(*a.shape)
    out = ctypes.POINTER(_Pair)()
    cnt = ctypes.c_int64(0)
    rc = fn(a.ctypes.data, a.ndim, ext, mask, int(method), int(bool(keep_zero)),
                        ctypes.byref(out), ctypes.byref(cnt))
    if rc != 0:
        raise OracleError(_ERRORS.get(rc, "error %d" % rc))
    n = cnt.value
    res = np.zeros(n, dtype=PAIR_DTYPE)
    if n:
        raw = np.frombuffer(ctypes.string_at(out, n * ctypes.sizeof(_Pair)), dtype=_C_DTYPE)
        for f in PAIR_DTYPE.names:
            res[f] = raw[f]
    lib.or_free(out)
    return res


def gradient(pairs: np.ndarray, grad_birth, grad_death, shape) -> np.ndarray:
    """Reference backward of the pair values with respect to the pixels (FP32)."""
    n = len(pairs)
    cp = (_Pair * max(n, 1))()
    for i in range(n):
        p = pairs[i]
        cp[i] = _Pair(int(p["dim"]), float(p["birth"]), float(p["death"]), int(p["birth_cell"]),
                      int(p["death_cell"]), int(p["birth_vertex"]), int(p["death_vertex"]))
    gb = np.ascontiguousarray(grad_birth, dtype=np.float32)
    gd = np.ascontiguousarray(grad_death, dtype=np.float32)
    nvox = int(np.prod(shape))
    g = np.zeros(nvox, dtype=np.float32)
    rc = _load().or_gradient(cp, n, gb.ctypes.data, gd.ctypes.data, g.ctypes.data, nvox)
    if rc != 0:
        raise OracleError(_ERRORS.get(rc, "error %d" % rc))
    return g.reshape(shape)
