"""MI355X (gfx950) cubical persistence: thin Python binding of libflashcubical.so.

Every step of the computation runs in the library's HIP kernels; this module only marshals
arguments (torch tensors for device memory and streams, ctypes for the C ABI declared in
include/flashcubical.h).  It raises if the library has not been built: there is no CPU
fallback.

Entry points (same names as the C ABI):
  ph_diagram(img)                 one image or volume -> Diagram (device tensors)
  ph_diagram_noalloc              the same into caller-owned outputs, library-owned workspace
  Batch(shapes).ph_diagram_batch  many instances of uneven sizes in one set of launches
  Batch.ph_autotune               tile choice timed on the batch, kept for its size class
  Batch.ph_backward / ph_backward gradient scatter to the critical pixels
  PHDiagramFn                     torch.autograd.Function around ph_diagram / ph_backward
  BatchDiagramFn                  torch.autograd.Function around ph_diagram_batch / ph_backward
  Batch.work_counters, profile / profile_read, device_report: inspection
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflashcubical.so")

PH_OK, PH_EINVAL, PH_ENAN, PH_ECAPACITY, PH_ENOMEM, PH_EHIP, PH_EINTERNAL, PH_ELISTS = 0, -1, -2, -3, -4, -5, -6, -7
PH_H0, PH_HTOP = 1, 2
PH_IN_U8, PH_IN_U16 = 4, 8          # input element type (float32 when neither is set)
PH_TFILT = 16                       # T-filtration: pixels are the top cells (default: V)
PH_H1 = 32                          # volumes: H1 as well (images: H1 is the top dimension)
PH_WIDE = 64                        # union-finds of 2^20+ voxel instances with many nodes start over the whole GPU
STATUS_NAMES = {0: "ok", -1: "invalid argument", -2: "NaN in input", -3: "capacity exceeded",
                -4: "workspace too small", -5: "HIP error", -6: "internal bound exceeded",
                -7: "lists outgrew the list fraction"}


def PH_LIST_FRACTION(k: int) -> int:
    """flags bits sizing the per-instance lists to k/256 of their worst case (C ABI
    PH_LIST_FRACTION): a smaller workspace; an instance whose lists outgrow it gets PH_ELISTS."""
    if not 0 <= int(k) <= 255:
        raise ValueError("list fraction k must be in 0..255")
    return (int(k) & 0xFF) << 8

PAIR_DTYPE = np.dtype([
    ("dim", np.int8), ("birth", np.float32), ("death", np.float32),
    ("birth_cell", np.int64), ("death_cell", np.int64),
    ("birth_vertex", np.int32), ("death_vertex", np.int32),
])


class PHError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__("%s: %s (%d)" % (what, STATUS_NAMES.get(code, "error"), code))
        self.code = code


class ph_shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("ext", ctypes.c_int32 * 3)]


class ph_pairs(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_void_p), ("birth", ctypes.c_void_p), ("death", ctypes.c_void_p),
                ("birth_cell", ctypes.c_void_p), ("death_cell", ctypes.c_void_p),
                ("birth_vertex", ctypes.c_void_p), ("death_vertex", ctypes.c_void_p)]


class ph_tuning(ctypes.Structure):
    _fields_ = [("tile2d", ctypes.c_int32), ("tile3d", ctypes.c_int32)]


class ph_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double)]


_lib = None


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln and "/" in ln})
    except OSError:
        return []


def lib():
    """The loaded C library; raises when it is missing (build it first).

    The library must share the HIP runtime of torch, which provides the device memory and
    streams: torch is imported first, so the loader binds the library to torch's copy of the
    runtime.  Loaded the other way round, the process would hold two runtimes, and the
    library's would not see torch's allocations."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libflashcubical.so is not built: run `python -m paper_2606_04801_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        runtimes = _hip_runtimes()
        if len(runtimes) > 1:
            raise ImportError("two HIP runtimes are loaded (%s): import torch before this library is "
                              "loaded" % ", ".join(runtimes))
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        L.ph_capacity_bound.argtypes = [ph_shape]
        L.ph_capacity_bound.restype = i64
        L.ph_capacity_bound_flags.argtypes = [ph_shape, u32]
        L.ph_capacity_bound_flags.restype = i64
        L.ph_workspace_bytes.argtypes = [ctypes.POINTER(ph_shape), i32, u32]
        L.ph_workspace_bytes.restype = ctypes.c_size_t
        L.ph_diagram.argtypes = [vp, ph_shape, u32, ph_pairs, i64, vp, vp, vp, ctypes.c_size_t, vp]
        L.ph_diagram.restype = ctypes.c_int
        L.ph_diagram_noalloc.argtypes = [vp, ph_shape, u32, ph_pairs, i64, vp, vp, vp]
        L.ph_diagram_noalloc.restype = ctypes.c_int
        L.ph_diagram_batch.argtypes = [i32, vp, vp, vp, ctypes.POINTER(ph_shape), u32, ph_pairs, vp, vp, vp,
                                       ctypes.POINTER(ph_tuning), vp, ctypes.c_size_t, vp]
        L.ph_diagram_batch.restype = ctypes.c_int
        L.ph_autotune.argtypes = [i32, vp, vp, vp, ctypes.POINTER(ph_shape), u32, ph_pairs, vp, vp, vp, vp,
                                  ctypes.c_size_t, i32, ctypes.POINTER(ph_tuning), vp]
        L.ph_autotune.restype = ctypes.c_int
        L.ph_backward.argtypes = [i32, ph_pairs, vp, vp, vp, vp, vp, vp, i64, vp]
        L.ph_backward.restype = ctypes.c_int
        L.ph_diagram_batch_grad.argtypes = [i32, vp, vp, vp, ctypes.POINTER(ph_shape), u32, ph_pairs, vp, vp, vp,
                                            ctypes.POINTER(ph_tuning), vp, ctypes.c_size_t, vp, vp]
        L.ph_diagram_batch_grad.restype = ctypes.c_int
        L.ph_backward_scatter.argtypes = [i32, ph_pairs, vp, vp, vp, vp, vp, vp, i64, vp]
        L.ph_backward_scatter.restype = ctypes.c_int
        L.ph_lut_entry.argtypes = [i32, u32, ctypes.POINTER(ctypes.c_uint64)]
        L.ph_lut_entry.restype = ctypes.c_int
        L.ph_lut_config_count.argtypes = [i32]
        L.ph_lut_config_count.restype = i32
        L.ph_version.restype = ctypes.c_char_p
        L.ph_init_device.restype = ctypes.c_int
        L.ph_device_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        L.ph_device_report.restype = ctypes.c_int
        L.ph_work_counters.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.ph_work_counters.restype = ctypes.c_int
        L.ph_profile.argtypes = [i32]
        L.ph_profile.restype = ctypes.c_int
        L.ph_profile_read.argtypes = [ctypes.POINTER(ph_kernel_time), i32, ctypes.POINTER(i32)]
        L.ph_profile_read.restype = ctypes.c_int
        _lib = L
    return _lib


def make_shape(shape) -> ph_shape:
    shape = tuple(int(x) for x in shape)
    if len(shape) not in (2, 3):
        raise PHError(PH_EINVAL, "shape")
    ext = list(shape) + [0] * (3 - len(shape))
    return ph_shape(len(shape), (ctypes.c_int32 * 3)(*ext))


def capacity_bound(shape, filtration: str = "V", flags: int = PH_H0 | PH_HTOP) -> int:
    """Pairs one instance can hold at most (C ABI ph_capacity_bound_flags): under the
    T-filtration the bound of the framed dual image (every extent + 2); with PH_H1 a volume's
    H1 pairs are added."""
    return int(lib().ph_capacity_bound_flags(make_shape(shape), _filtration_flags(flags, filtration)))


def _filtration_flags(flags: int, filtration: str) -> int:
    if filtration not in ("V", "T"):
        raise PHError(PH_EINVAL, "filtration must be 'V' or 'T'")
    return (int(flags) & ~PH_TFILT) | (PH_TFILT if filtration == "T" else 0)


def workspace_bytes(shapes, flags=PH_H0 | PH_HTOP) -> int:
    arr = (ph_shape * len(shapes))(*[make_shape(s) for s in shapes])
    return int(lib().ph_workspace_bytes(arr, len(shapes), flags))


def lut_entry(ndim: int, raw_mask: int) -> int:
    e = ctypes.c_uint64(0)
    rc = lib().ph_lut_entry(ndim, raw_mask, ctypes.byref(e))
    if rc != PH_OK:
        raise PHError(rc, "ph_lut_entry")
    return int(e.value)


def device_report():
    """(status, text): device limits and per-kernel resources (launches nothing)."""
    buf = ctypes.create_string_buffer(8192)
    rc = lib().ph_device_report(buf, len(buf))
    return rc, buf.value.decode()


def lut_config_count(ndim: int) -> int:
    return int(lib().ph_lut_config_count(ndim))


def profile(enable: bool) -> None:
    """Start (clearing earlier records) or stop per-launch event timing (C ABI ph_profile)."""
    lib().ph_profile(1 if enable else 0)


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} of the launches recorded since profile(True)."""
    buf = (ph_kernel_time * 32)()
    cnt = ctypes.c_int32(0)
    rc = lib().ph_profile_read(buf, 32, ctypes.byref(cnt))
    if rc != PH_OK:
        raise PHError(rc, "ph_profile_read")
    return {buf[k].name.decode(): (int(buf[k].launches), float(buf[k].total_ms))
            for k in range(min(cnt.value, 32))}


# ------------------------------------------------------------------- device side --

def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None and not torch.cuda.is_available():
        return ctypes.c_void_p(None)             # no device: the library reports it, not the binding
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class PairBuffers:
    """SoA device tensors holding `cap` pairs."""

    def __init__(self, cap: int, device):
        torch = _torch()
        cap = max(int(cap), 1)
        self.cap = cap
        self.dim = torch.empty(cap, dtype=torch.int8, device=device)
        self.birth = torch.empty(cap, dtype=torch.float32, device=device)
        self.death = torch.empty(cap, dtype=torch.float32, device=device)
        self.birth_cell = torch.empty(cap, dtype=torch.int64, device=device)
        self.death_cell = torch.empty(cap, dtype=torch.int64, device=device)
        self.birth_vertex = torch.empty(cap, dtype=torch.int32, device=device)
        self.death_vertex = torch.empty(cap, dtype=torch.int32, device=device)

    def c(self) -> ph_pairs:
        return ph_pairs(*[t.data_ptr() for t in (self.dim, self.birth, self.death, self.birth_cell,
                                                 self.death_cell, self.birth_vertex, self.death_vertex)])

    def to_numpy(self, start: int, count: int) -> np.ndarray:
        out = np.zeros(count, dtype=PAIR_DTYPE)
        for f in PAIR_DTYPE.names:
            out[f] = getattr(self, f)[start:start + count].cpu().numpy()
        return out


class Diagram:
    """Result of ph_diagram: device SoA buffers plus the device count and status."""

    def __init__(self, bufs: PairBuffers, count, status, shape):
        self.bufs, self.count_t, self.status_t, self.shape = bufs, count, status, tuple(shape)

    def check(self) -> int:
        st = int(self.status_t.item())
        if st != PH_OK:
            raise PHError(st, "ph_diagram")
        return int(self.count_t.item())

    def numpy(self) -> np.ndarray:
        n = self.check()
        return self.bufs.to_numpy(0, n)


class Workspace:
    """Reusable device workspace (grown on demand)."""

    def __init__(self):
        self.t = None

    def get(self, nbytes: int, device):
        torch = _torch()
        if self.t is None or self.t.numel() < nbytes or self.t.device != torch.device(device):
            self.t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        return self.t


_default_ws = Workspace()


def ph_diagram(img, flags: int = PH_H0 | PH_HTOP, capacity: int | None = None, ws: Workspace | None = None,
               stream=None, filtration: str = "V") -> Diagram:
    """Persistence diagram of one image (H, W) or volume (D, H, W) on the GPU: float32, or
    uint8 / uint16 (read as such, results those of the same values as float32), under the
    V-filtration (pixels are vertices) or the T-filtration (pixels are top cells)."""
    torch = _torch()
    # a host tensor would hand the kernels a host pointer; without a GPU the library itself
    # reports that it cannot run, so the check only matters when one is present
    on_device = img.is_cuda or not torch.cuda.is_available()
    kinds = _input_flags()
    if not (on_device and img.dtype in kinds and img.dim() in (2, 3)):
        raise PHError(PH_EINVAL, "ph_diagram expects a 2D/3D float32, uint8 or uint16 CUDA tensor")
    flags = _filtration_flags((int(flags) & ~(PH_IN_U8 | PH_IN_U16)) | kinds[img.dtype], filtration)
    img = img.contiguous()
    shp = make_shape(img.shape)
    cap = capacity_bound(img.shape, filtration, flags) if capacity is None else int(capacity)
    bufs = PairBuffers(cap, img.device)
    count = torch.zeros(1, dtype=torch.int64, device=img.device)
    status = torch.zeros(1, dtype=torch.int32, device=img.device)
    nb = int(lib().ph_workspace_bytes(ctypes.byref(shp), 1, flags))
    w = (ws or _default_ws).get(nb, img.device)
    rc = lib().ph_diagram(_ptr(img), shp, flags, bufs.c(), cap, _ptr(count), _ptr(status), _ptr(w),
                          w.numel(), _stream_ptr(stream))
    if rc != PH_OK:
        raise PHError(rc, "ph_diagram")
    return Diagram(bufs, count, status, img.shape)


def ph_diagram_noalloc(img, bufs: PairBuffers, count, status, flags: int = PH_H0 | PH_HTOP,
                       capacity: int | None = None, stream=None, filtration: str = "V") -> int:
    """C ABI ph_diagram_noalloc: the diagram of one image or volume into caller-owned outputs
    (bufs, count, status: device tensors), with the library's own per-device workspace
    (ph_init_device must have run on the device); the call allocates nothing.  Returns the
    C status (PH_OK once the work is enqueued); the kernels' status lands in `status`."""
    kinds = _input_flags()
    if img.dtype not in kinds or img.dim() not in (2, 3) or not img.is_contiguous():
        raise PHError(PH_EINVAL, "ph_diagram_noalloc expects a contiguous 2D/3D float32, uint8 or uint16 tensor")
    flags = _filtration_flags((int(flags) & ~(PH_IN_U8 | PH_IN_U16)) | kinds[img.dtype], filtration)
    cap = bufs.cap if capacity is None else int(capacity)
    return int(lib().ph_diagram_noalloc(_ptr(img), make_shape(img.shape), flags, bufs.c(), cap, _ptr(count),
                                        _ptr(status), _stream_ptr(stream)))


def _input_flags():
    torch = _torch()
    return {torch.float32: 0, torch.uint8: PH_IN_U8, torch.uint16: PH_IN_U16}


def ph_backward(bufs: PairBuffers, counts, out_off, img_off, grad_birth, grad_death, grad_img, stream=None,
                zeroed: bool = False):
    """Scatter dL/dbirth, dL/ddeath into grad_img (overwritten) -- C ABI ph_backward; with
    zeroed, grad_img already holds zeros (ph_diagram_batch_grad) and only the scatter runs --
    C ABI ph_backward_scatter."""
    n = int(counts.numel())
    fn = lib().ph_backward_scatter if zeroed else lib().ph_backward
    rc = fn(n, bufs.c(), _ptr(out_off), _ptr(counts), _ptr(grad_birth), _ptr(grad_death),
            _ptr(grad_img), _ptr(img_off), int(grad_img.numel()), _stream_ptr(stream))
    if rc != PH_OK:
        raise PHError(rc, "ph_backward_scatter" if zeroed else "ph_backward")


class Batch:
    """Buffers and launches for a fixed list of instance shapes (2D and 3D may be mixed).

    Inputs live in one packed buffer (`images`) of the batch's element type (float32, uint8
    or uint16), outputs in one SoA buffer with a
    per-instance capacity of pixels + top cells, so nothing depends on the host between
    launches and the forward + backward pair can be captured in a HIP graph.
    """

    def __init__(self, shapes, flags: int = PH_H0 | PH_HTOP, tuning=None, device="cuda", capacities=None,
                 dtype=None, filtration: str = "V"):
        """capacities: pairs stored per instance (default: the bound pixels + top cells, which
        never overflows); a smaller one, e.g. the counts of an earlier call on the same
        inputs, keeps the pair buffers small.  dtype: element type of the inputs (float32,
        uint8 or uint16; integer inputs use the default tiles).  filtration: "V" (pixels are
        vertices) or "T" (pixels are top cells)."""
        torch = _torch()
        self.dtype = torch.float32 if dtype is None else dtype
        kinds = _input_flags()
        if self.dtype not in kinds:
            raise PHError(PH_EINVAL, "Batch dtype must be float32, uint8 or uint16")
        flags = _filtration_flags((int(flags) & ~(PH_IN_U8 | PH_IN_U16)) | kinds[self.dtype], filtration)
        self.filtration = filtration
        self.shapes = [tuple(int(x) for x in s) for s in shapes]
        self.n = len(self.shapes)
        self.flags = flags
        self.device = torch.device(device)
        sizes = [int(np.prod(s)) for s in self.shapes]
        caps = [capacity_bound(s, filtration, flags) for s in self.shapes] if capacities is None else [max(int(c), 1) for c in capacities]
        if len(caps) != self.n:
            raise PHError(PH_EINVAL, "capacities")
        self.img_off_h = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.out_off_h = np.concatenate([[0], np.cumsum(caps)]).astype(np.int64)
        self.total_voxels = int(self.img_off_h[-1])
        self.h_shapes = (ph_shape * self.n)(*[make_shape(s) for s in self.shapes])
        d = np.zeros((self.n, 4), np.int32)
        for i, s in enumerate(self.shapes):
            d[i, 0] = len(s)
            d[i, 1:1 + len(s)] = s
        self.d_shapes = torch.from_numpy(d).to(self.device)
        self.img_off = torch.from_numpy(self.img_off_h[:-1].copy()).to(self.device)
        self.out_off = torch.from_numpy(self.out_off_h).to(self.device)
        self.images = torch.zeros(self.total_voxels, dtype=self.dtype, device=self.device)
        self.grad = torch.zeros(self.total_voxels, dtype=torch.float32, device=self.device)
        self.pairs = PairBuffers(int(self.out_off_h[-1]), self.device)
        self.counts = torch.zeros(self.n, dtype=torch.int64, device=self.device)
        self.status = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        self.ws_bytes = int(lib().ph_workspace_bytes(self.h_shapes, self.n, flags))
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.tuning = None if tuning is None else ph_tuning(int(tuning[0]), int(tuning[1]))

    def set_images(self, imgs):
        torch = _torch()
        for i, a in enumerate(imgs):
            t = torch.as_tensor(a).to(self.dtype).reshape(-1)
            self.images[self.img_off_h[i]:self.img_off_h[i + 1]].copy_(t, non_blocking=False)

    def image(self, i):
        return self.images[self.img_off_h[i]:self.img_off_h[i + 1]].view(self.shapes[i])

    def ph_diagram_batch(self, stream=None, grad=None):
        """The batch's diagrams (C ABI ph_diagram_batch); with grad (a float32 tensor of
        total_voxels elements, e.g. self.grad), also set it to zero inside the classify passes
        for ph_backward(..., zeroed=True) (C ABI ph_diagram_batch_grad)."""
        tp = ctypes.byref(self.tuning) if self.tuning is not None else None
        if grad is None:
            rc = lib().ph_diagram_batch(self.n, _ptr(self.images), _ptr(self.img_off), _ptr(self.d_shapes),
                                        self.h_shapes, self.flags, self.pairs.c(), _ptr(self.out_off),
                                        _ptr(self.counts), _ptr(self.status), tp, _ptr(self.ws), self.ws_bytes,
                                        _stream_ptr(stream))
        else:
            if grad.dtype != _torch().float32 or grad.numel() != self.total_voxels or not grad.is_contiguous():
                raise PHError(PH_EINVAL, "ph_diagram_batch: grad must be a contiguous float32 tensor of total_voxels")
            rc = lib().ph_diagram_batch_grad(self.n, _ptr(self.images), _ptr(self.img_off), _ptr(self.d_shapes),
                                             self.h_shapes, self.flags, self.pairs.c(), _ptr(self.out_off),
                                             _ptr(self.counts), _ptr(self.status), tp, _ptr(self.ws), self.ws_bytes,
                                             _ptr(grad), _stream_ptr(stream))
        if rc != PH_OK:
            raise PHError(rc, "ph_diagram_batch")

    def ph_autotune(self, reps: int = 3, stream=None):
        """Time every tile choice on this batch and keep the fastest (C ABI ph_autotune); later
        ph_diagram_batch calls of this size class use it.  Synchronises the stream."""
        best = ph_tuning(0, 0)
        rc = lib().ph_autotune(self.n, _ptr(self.images), _ptr(self.img_off), _ptr(self.d_shapes),
                               self.h_shapes, self.flags, self.pairs.c(), _ptr(self.out_off),
                               _ptr(self.counts), _ptr(self.status), _ptr(self.ws), self.ws_bytes,
                               int(reps), ctypes.byref(best), _stream_ptr(stream))
        if rc != PH_OK:
            raise PHError(rc, "ph_autotune")
        return (int(best.tile2d), int(best.tile3d))

    def ph_backward(self, grad_birth, grad_death, stream=None, zeroed: bool = False):
        """Gradient into self.grad; zeroed: the last forward cleared it (grad=self.grad)."""
        ph_backward(self.pairs, self.counts, self.out_off, self.img_off, grad_birth, grad_death, self.grad,
                    stream, zeroed)

    def work_counters(self):
        """Per-instance counters of the last call (C ABI ph_work_counters), as an (n, 16) array:
        KEEP edges, KEEP squares, H0 nodes, dual nodes, H0 rounds, dual rounds, sequential
        edges, error word, and for 3D H1: columns, columns reduced one by one, most steps of
        one column, pool entries, columns that needed the large tables, reduction rounds
        (column additions when it ran one column at a time), and the forest links the
        resolve passes followed (H0 endpoints, top-dimension cofacets).  Synchronises."""
        out = (ctypes.c_int32 * (16 * self.n))()
        rc = lib().ph_work_counters(_ptr(self.ws), self.n, out)
        if rc != PH_OK:
            raise PHError(rc, "ph_work_counters")
        return np.frombuffer(out, dtype=np.int32).reshape(self.n, 16).copy()

    def valid_mask(self):
        """Device bool mask over the packed pair slots holding a stored pair (no sync).  The
        slot -> (instance, position) map is fixed by the capacities and made once."""
        torch = _torch()
        if getattr(self, "_slot_inst", None) is None:
            idx = torch.arange(self.pairs.cap, device=self.device)
            inst = torch.clamp(torch.searchsorted(self.out_off[1:], idx, right=True), max=self.n - 1)
            self._slot_inst, self._slot_pos = inst, idx - self.out_off[inst]
        return self._slot_pos < self.counts[self._slot_inst]

    def check(self):
        st = self.status.cpu().numpy()
        bad = np.nonzero(st != PH_OK)[0]
        if len(bad):
            raise PHError(int(st[bad[0]]), "instance %d" % int(bad[0]))

    def result(self, i):
        """Pairs of instance i (raises if its own status is not PH_OK; the others are not looked at)."""
        st = int(self.status[i].item())
        if st != PH_OK:
            raise PHError(st, "instance %d" % i)
        return self.pairs.to_numpy(int(self.out_off_h[i]), int(self.counts[i].item()))

    def results(self):
        self.check()
        cnt = self.counts.cpu().numpy()
        return [self.pairs.to_numpy(int(self.out_off_h[i]), int(cnt[i])) for i in range(self.n)]


def _autograd():
    torch = _torch()

    class PHDiagramFn(torch.autograd.Function):
        """(birth, death, dim) of the pairs of one image/volume; backward scatters dL/dbirth
        and dL/ddeath to the pixels attaining each critical cell's value (ph_backward).

        Upstream gradients pass through unchanged, non-finite ones included: only the death
        of the essential class (+inf, no death pixel) has nothing to receive its gradient,
        which ph_backward skips."""

        @staticmethod
        def forward(ctx, img, filtration="V"):
            d = ph_diagram(img.detach(), filtration=filtration)
            n = d.check()
            b = d.bufs
            ctx.save_for_backward(b.birth_vertex[:n].clone(), b.death_vertex[:n].clone())
            ctx.shape = img.shape
            ctx.bufs, ctx.n = b, n
            return b.birth[:n].clone(), b.death[:n].clone(), b.dim[:n].clone()

        @staticmethod
        def backward(ctx, g_birth, g_death, g_dim):
            torch = _torch()
            dev = g_birth.device if g_birth is not None else g_death.device
            n = ctx.n
            gb = g_birth.contiguous() if g_birth is not None else torch.zeros(n, device=dev)
            gd = g_death.contiguous() if g_death is not None else torch.zeros(n, device=dev)
            gimg = torch.empty(ctx.shape, dtype=torch.float32, device=dev)
            counts = torch.tensor([n], dtype=torch.int64, device=dev)
            out_off = torch.tensor([0, max(n, 1)], dtype=torch.int64, device=dev)
            img_off = torch.zeros(1, dtype=torch.int64, device=dev)
            ph_backward(ctx.bufs, counts, out_off, img_off, gb, gd, gimg)
            return gimg, None

    class BatchDiagramFn(torch.autograd.Function):
        """Diagrams of every instance of a Batch in one ph_diagram_batch call, with the
        packed pixels as the differentiable input.

        forward(images, batch) -> (birth, death): float32 over every pair slot of the batch
        (batch.pairs.cap entries, instance i from batch.out_off_h[i]); slots past an
        instance's count hold no pair: batch.valid_mask() marks the stored ones, and
        batch.pairs.death_cell >= 0 the finite ones.  `images` is the batch's packed float32
        input; when it is not batch.images itself it is copied there first.  When a gradient
        is wanted, the forward also allocates the gradient tensor and has the classify passes
        clear it (ph_diagram_batch_grad); backward then scatters dL/dbirth and dL/ddeath to the
        critical pixels (ph_backward_scatter) from the pair vertices and counts this forward
        saved, so a later forward on the same batch does not change it.  Captured in a HIP
        graph together with the loss and its backward, a replay recomputes everything in
        place."""

        @staticmethod
        def forward(ctx, images, batch):
            if batch.dtype != torch.float32 or images.dtype != torch.float32 or images.numel() != batch.total_voxels:
                raise PHError(PH_EINVAL, "BatchDiagramFn: float32 images of the batch's total size")
            if images.data_ptr() != batch.images.data_ptr():
                batch.images.copy_(images.detach().reshape(-1))
            gimg = None
            if ctx.needs_input_grad[0]:
                gimg = torch.empty(batch.total_voxels, dtype=torch.float32, device=batch.images.device)
            batch.ph_diagram_batch(grad=gimg)
            ctx.batch = batch
            ctx.gimg = gimg
            ctx.save_for_backward(batch.pairs.birth_vertex.clone(), batch.pairs.death_vertex.clone(),
                                  batch.counts.clone())
            ctx.img_shape = images.shape
            return batch.pairs.birth.clone(), batch.pairs.death.clone()

        @staticmethod
        def backward(ctx, g_birth, g_death):
            b = ctx.batch
            bv, dv, counts = ctx.saved_tensors
            cap = bv.numel()
            dev = bv.device
            gb = g_birth.contiguous() if g_birth is not None else torch.zeros(cap, device=dev)
            gd = g_death.contiguous() if g_death is not None else torch.zeros(cap, device=dev)
            pairs = ph_pairs(None, None, None, None, None, bv.data_ptr(), dv.data_ptr())
            gimg = ctx.gimg                          # cleared by the forward's classify passes
            ctx.gimg = None
            if gimg is None:
                raise PHError(PH_EINVAL, "BatchDiagramFn: backward without a gradient buffer")
            rc = lib().ph_backward_scatter(b.n, pairs, _ptr(b.out_off), _ptr(counts), _ptr(gb), _ptr(gd),
                                           _ptr(gimg), _ptr(b.img_off), b.total_voxels, _stream_ptr(None))
            if rc != PH_OK:
                raise PHError(rc, "ph_backward_scatter")
            return gimg.view(ctx.img_shape), None

    return PHDiagramFn, BatchDiagramFn


_fn_cache = []


def __getattr__(name):
    # the autograd classes are made on first use so that importing this module needs no torch
    if name in ("PHDiagramFn", "BatchDiagramFn"):
        if not _fn_cache:
            _fn_cache.extend(_autograd())
        return _fn_cache[0] if name == "PHDiagramFn" else _fn_cache[1]
    raise AttributeError(name)
