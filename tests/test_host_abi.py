"""Host side of the C ABI (no GPU, no kernel launch): the library loads, exports every entry
point its header declares, sizes its buffers consistently and validates arguments on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

fc = pytest.importorskip("paper_2606_04801_amd")
try:
    fc.lib()
except (ImportError, OSError) as e:
    pytest.skip("library not built: %s" % e, allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flashcubical.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ph_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    names = declared_functions()
    assert {"ph_diagram", "ph_diagram_batch", "ph_backward", "ph_workspace_bytes"} <= set(names)
    L = ctypes.CDLL(fc.LIB_PATH)
    for n in names:
        assert hasattr(L, n), "missing export " + n


def test_version():
    assert fc.lib().ph_version().startswith(b"flashcubical")


def test_capacity_bound_closed_form():
    # pixels + top cells
    assert fc.capacity_bound((1, 4)) == 4
    assert fc.capacity_bound((3, 3)) == 9 + 4
    assert fc.capacity_bound((2048, 2048)) == 2048 * 2048 + 2047 * 2047
    assert fc.capacity_bound((256, 256, 256)) == 256 ** 3 + 255 ** 3
    assert fc.capacity_bound((1, 5, 5)) == 25          # a volume with a unit extent has no cubes


def test_invalid_shapes_rejected():
    L = fc.lib()
    for bad in [(0, 4), (4, 0), (0, 1, 1), (-1, 3)]:
        assert fc.capacity_bound(bad) == 0
        assert fc.workspace_bytes([bad]) == 0
    big = (1 << 14, (1 << 13) + 1)                     # above 2^27 pixels: the key's pixel field
    assert fc.capacity_bound(big) == 0
    assert fc.capacity_bound((512, 512, 512)) == 512 ** 3 + 511 ** 3     # 2^27 voxels: accepted
    assert fc.capacity_bound((512, 512, 512), "T") == 0                  # framed: 514^3
    huge = (1 << 30, 1 << 30, 1 << 30)                 # extents whose product overflows 64 bits
    assert fc.capacity_bound(huge) == 0 and fc.workspace_bytes([huge]) == 0
    with pytest.raises(fc.PHError):
        fc.make_shape((4,))
    assert L.ph_workspace_bytes(None, 1, 3) == 0


def test_workspace_grows_with_size_and_batch():
    a = fc.workspace_bytes([(64, 64)])
    b = fc.workspace_bytes([(128, 128)])
    c = fc.workspace_bytes([(64, 64), (128, 128)])
    assert 0 < a < b < c
    assert c >= a + b - 4096                           # one header for the batch
    d3 = fc.workspace_bytes([(16, 16, 16)])
    assert d3 > fc.workspace_bytes([(64, 64)])
    mixed = fc.workspace_bytes([(16, 16, 16), (64, 64)])
    assert mixed > d3


def _call_diagram():
    L = fc.lib()
    return L.ph_diagram(None, fc.make_shape((4, 4)), 3, fc.ph_pairs(), 16, None, None, None, 0, None)


def test_host_validation_before_any_device_call():
    # every call below fails argument checks on the host before touching HIP
    L = fc.lib()
    assert _call_diagram() == fc.PH_EINVAL                      # null buffers
    assert L.ph_diagram(None, fc.make_shape((4, 4)), 3, fc.ph_pairs(), -1, None, None, None, 0,
                        None) == fc.PH_EINVAL                   # negative capacity
    sh = (fc.ph_shape * 1)(fc.make_shape((4, 4)))
    assert L.ph_diagram_batch(1, None, None, None, sh, 3, fc.ph_pairs(), None, None, None, None, None, 0,
                              None) == fc.PH_EINVAL
    assert L.ph_diagram_batch(0, None, None, None, sh, 3, fc.ph_pairs(), None, None, None, None, None, 0,
                              None) == fc.PH_EINVAL
    many = (fc.ph_shape * 65536)(*([fc.make_shape((2, 2))] * 65536))
    one = ctypes.c_void_p(1)                                    # never dereferenced: rejected first
    assert L.ph_diagram_batch(65536, one, one, one, many, 3, fc.ph_pairs(one, one, one, one, one, one, one),
                              one, one, one, None, one, 1 << 30, None) == fc.PH_EINVAL
    assert L.ph_backward(1, fc.ph_pairs(), None, None, None, None, None, None, 16, None) == fc.PH_EINVAL
    assert L.ph_backward(1, fc.ph_pairs(), None, None, None, None, None, None, 0, None) == fc.PH_EINVAL
    assert L.ph_backward_scatter(1, fc.ph_pairs(), None, None, None, None, None, None, 16, None) == fc.PH_EINVAL
    pr = fc.ph_pairs(one, one, one, one, one, one, one)
    assert L.ph_diagram_batch_grad(1, one, one, one, sh, 3, pr, one, one, one, None, one, 1 << 30, None,
                                   None) == fc.PH_EINVAL       # no gradient buffer
    assert L.ph_diagram_batch_grad(0, one, one, one, sh, 3, pr, one, one, one, None, one, 1 << 30, one,
                                   None) == fc.PH_EINVAL
    best = fc.ph_tuning(0, 0)
    assert L.ph_autotune(1, None, None, None, sh, 3, fc.ph_pairs(), None, None, None, None, 0, 1,
                         ctypes.byref(best), None) == fc.PH_EINVAL
    assert L.ph_autotune(1, None, None, None, sh, 3, fc.ph_pairs(), None, None, None, None, 0, 1,
                         None, None) == fc.PH_EINVAL


def test_binding_raises_without_gpu_tensor():
    torch = pytest.importorskip("torch")
    with pytest.raises(fc.PHError):
        fc.ph_diagram(torch.zeros(4, 4))                        # CPU tensor: refused, no fallback


def test_status_names_cover_codes():
    for code in (fc.PH_OK, fc.PH_EINVAL, fc.PH_ENAN, fc.PH_ECAPACITY, fc.PH_ENOMEM, fc.PH_EHIP,
                 fc.PH_EINTERNAL):
        assert code in fc.STATUS_NAMES


def test_work_counters_validation():
    L = fc.lib()
    out = (ctypes.c_int32 * 8)()
    assert L.ph_work_counters(None, 1, out) == fc.PH_EINVAL
    assert L.ph_work_counters(ctypes.c_void_p(1), 0, out) == fc.PH_EINVAL
    assert L.ph_work_counters(ctypes.c_void_p(1), 1, None) == fc.PH_EINVAL


def test_one_hip_runtime_shared_with_torch():
    """The library binds to torch's HIP runtime: one libamdhip64 in the process (a second
    copy would not see torch's device allocations)."""
    pytest.importorskip("torch")
    fc.lib()
    assert len(fc._hip_runtimes()) <= 1, fc._hip_runtimes()


def test_library_loaded_before_torch_still_shares_its_runtime():
    """In a fresh process, the first use of the binding without importing torch still ends with
    one runtime: lib() imports torch before loading the library."""
    import subprocess
    import sys
    pytest.importorskip("torch")
    code = ("import sys; sys.path.insert(0, %r); import paper_2606_04801_amd as fc; fc.lib(); "
            "print(len(fc._hip_runtimes()))" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().splitlines()[-1] in ("0", "1"), r.stdout + r.stderr[-2000:]


def test_both_integer_input_flags_rejected():
    """PH_IN_U8 with PH_IN_U16 names no element type: refused on the host, before any device
    call (the pointers are never dereferenced)."""
    L = fc.lib()
    one = ctypes.c_void_p(1)
    pr = fc.ph_pairs(one, one, one, one, one, one, one)
    flags = fc.PH_H0 | fc.PH_HTOP | fc.PH_IN_U8 | fc.PH_IN_U16
    assert L.ph_diagram(one, fc.make_shape((4, 4)), flags, pr, 16, one, one, one, 1 << 20, None) == fc.PH_EINVAL
    sh = (fc.ph_shape * 1)(fc.make_shape((4, 4)))
    assert L.ph_diagram_batch(1, one, one, one, sh, flags, pr, one, one, one, None, one, 1 << 20,
                              None) == fc.PH_EINVAL


def test_t_filtration_sizes():
    """Under PH_TFILT the workspace holds the framed dual images (extents + 2) and their lists,
    and the capacity bound is that of the framed shape."""
    sh = [(64, 64), (16, 16, 16)]
    v = fc.workspace_bytes(sh)
    t = fc.workspace_bytes(sh, fc.PH_H0 | fc.PH_HTOP | fc.PH_TFILT)
    assert t > v + 4 * (66 * 66 + 18 ** 3)
    assert fc.capacity_bound((3, 3), "T") == fc.capacity_bound((5, 5))
    big = (1 << 13, (1 << 14) - 2)                     # fits, its frame does not
    assert fc.workspace_bytes([big], fc.PH_H0 | fc.PH_HTOP | fc.PH_TFILT) == 0
