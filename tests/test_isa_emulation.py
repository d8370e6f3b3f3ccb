"""The library's gfx950 machine code, executed instruction by instruction on the CPU.

tests/isa_emulation interprets the code object of paper_2606_04801_amd/libflashcubical.so (the
AMD assembly of this build, read with the ROCm LLVM tools): 64-lane waves in lockstep, waves of
a workgroup interleaved between barriers, every global access checked against the registered
device buffers and every LDS access against the kernel's LDS segment.  The library's own host
code issues the launches (tests/cpu_emulation, variant "isa").  Results must equal the
oracle's bit for bit.  This is how the node-key sort was found to load its count through a
scalar register pair that its branch never set (see sort_list).
"""
import os
import shutil
import sys

import numpy as np
import pytest

import fixtures
import oracle
import synthetic as S
from gpu_util import diff_pairs

pytestmark = pytest.mark.slow
HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(os.path.dirname(HERE), "paper_2606_04801_amd", "libflashcubical.so")
if not (os.path.exists(LIB) and os.path.exists("/opt/rocm/llvm/bin/llvm-objdump") and shutil.which("g++")):
    pytest.skip("library, ROCm LLVM tools or host compiler missing", allow_module_level=True)
sys.path.insert(0, os.path.join(HERE, "isa_emulation"))


@pytest.fixture(scope="module")
def isa():
    from runner import IsaRunner
    return IsaRunner()


def staircase(n):
    a = np.zeros(2 * n + 1, np.float32)
    a[0::2] = np.linspace(0.5, 0.1, n + 1).astype(np.float32)
    a[1::2] = np.linspace(1.0, 2.0, n).astype(np.float32)
    return a.reshape(1, -1)


def test_fixtures(isa):
    for name, img, _, _ in fixtures.load():
        got, st, _ = isa.diagram(img)
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, name


def test_every_kernel_of_a_diagram_runs(isa):
    isa.launches = []
    isa.diagram(S.grf((12, 10, 14), 1.5, 8))
    names = {n for n, _, _ in isa.launches}
    for k in ("k_plan", "k_classify3d", "k_sort_lists", "k_resolve", "k_unionfind", "k_output"):
        assert any(k in n for n in names), k


def test_fields_and_edge_cases(isa):
    specials = np.array([[np.inf, -np.inf, -0.0, 0.0, 1e-45, -1e-45, 3.4e38, -3.4e38]] * 5, np.float32)
    specials[2:] = specials[2:, ::-1]
    cb = (np.indices((33, 47)).sum(axis=0) % 2).astype(np.float32)
    for img in (S.grf((48, 40), 2.0, 7), S.grf((12, 10, 14), 1.5, 8), staircase(150), specials, cb,
                S.levels((2, 2, 300), 3, 5), S.uniform((128, 128), 4)):
        got, st, _ = isa.diagram(img)
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape


def test_long_lists_and_lds_forest(isa):
    """180 x 180 uniform noise: 10k KEEP edges sorted in three runs and two merge passes, and
    6.5k H0 nodes, past the keyed LDS capacity, in the union-find's node-only LDS layout."""
    img = S.uniform((180, 180), 24)
    got, st, _ = isa.diagram(img)
    assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None


def test_status_words(isa):
    img = S.grf((20, 20), 2.0, 3)
    img[4, 5] = np.nan
    assert isa.diagram(img)[1] == -2                                        # PH_ENAN
    img = S.uniform((40, 40), 9)
    ref = oracle.diagram(img)
    got, st, n = isa.diagram(img, capacity=25)
    assert st == -3 and n == len(ref) and diff_pairs(got, ref[:25]) is None  # PH_ECAPACITY


@pytest.mark.parametrize("tuning", [None, (2, 1)])
def test_batch_with_backward(isa, tuning):
    imgs = [S.levels((5, 9), 3, 7100), S.grf((40, 33), 2.0, 7101), S.levels((4, 3, 5), 2, 7102),
            S.grf((9, 12, 10), 1.5, 7103), S.levels((1, 7), 5, 7104), S.uniform((20, 21), 7105)]
    res, grad = isa.batch(imgs, tuning=tuning, backward=True)
    off = 0
    for img, (got, st) in zip(imgs, res):
        ref = oracle.diagram(img)
        assert st == 0 and diff_pairs(got, ref) is None, img.shape
        f = ref["death_cell"] >= 0
        d = np.where(f, ref["death"] - ref["birth"], 0).astype(np.float32)
        g = oracle.gradient(ref, -2 * d, 2 * d, img.shape).reshape(-1)
        np.testing.assert_allclose(grad[off:off + img.size], g, rtol=1e-6, atol=1e-7)
        off += img.size


def test_waves_interleaved_every_instruction():
    """Waves of a workgroup switched after every instruction instead of at barriers."""
    from runner import IsaRunner
    r = IsaRunner(slice_=1)
    for img in (S.grf((48, 40), 2.0, 7), S.levels((4, 3, 5), 2, 7102)):
        got, st, _ = r.diagram(img)
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape


def test_access_outside_device_memory_is_reported(isa):
    """Negative control: k_zero handed a buffer that was never registered stops the run."""
    import struct
    from gfx950_sim import Dispatch, Fault
    name = [k for k in isa.prog.kernels if "k_zero" in k][0]
    buf = np.zeros(64, np.float32)                  # host memory, not registered
    d = Dispatch(isa.prog, isa.mem, name, (1, 1, 1), (256, 1, 1), struct.pack("<Qq", buf.ctypes.data, 64))
    with pytest.raises(Fault, match="outside device memory"):
        try:
            d.run()
        finally:
            d.done()


def test_interpreter_covers_every_instruction(isa):
    """Every instruction of the code object parses into an implemented operation, so no
    path of any kernel can stop on an unknown one."""
    from gfx950_sim import Unsupported, compile_instr
    missing = {}
    pcs = sorted(isa.prog.text)
    for k, pc in enumerate(pcs):
        try:
            compile_instr(pc, isa.prog.text[pc], pcs[k + 1] if k + 1 < len(pcs) else None)
        except (Unsupported, IndexError, ValueError, KeyError) as e:
            missing.setdefault(isa.prog.text[pc].split()[0], "%s: %s" % (type(e).__name__, e))
    assert not missing, missing


def test_integer_inputs(isa):
    """uint8 and uint16 inputs (PH_IN_U8, PH_IN_U16) give the oracle's pairs of the same
    values as float32; the coarse 7-level copies are dense in ties."""
    for shape, sigma in (((48, 40), 2.0), ((12, 10, 14), 1.5)):
        g = S.grf(shape, sigma, 77)
        for dt, levels in ((np.uint8, 255), (np.uint16, 65535), (np.uint8, 7)):
            q = np.round(g * levels).astype(dt)
            got, st, _ = isa.diagram(q)
            assert st == 0 and diff_pairs(got, oracle.diagram(q.astype(np.float32))) is None, (shape, dt, levels)
    imgs = [np.round(S.grf((20, 21), 2.0, 5) * 9).astype(np.uint16),
            np.round(S.grf((6, 7, 8), 1.2, 6) * 9).astype(np.uint16)]
    res, grad = isa.batch(imgs, backward=True)
    off = 0
    for img, (got, st) in zip(imgs, res):
        ref = oracle.diagram(img.astype(np.float32))
        assert st == 0 and diff_pairs(got, ref) is None, img.shape
        f = ref["death_cell"] >= 0
        d = np.where(f, ref["death"] - ref["birth"], 0).astype(np.float32)
        g = oracle.gradient(ref, -2 * d, 2 * d, img.shape).reshape(-1)
        np.testing.assert_allclose(grad[off:off + img.size], g, rtol=1e-6, atol=1e-7)
        off += img.size


def test_t_filtration(isa):
    """PH_TFILT: the framed dual image (read through the reflection by the classify passes)
    and back (k_output) gives the oracle's T-filtration pairs, for float32 and uint8 inputs."""
    for shape, sigma in (((30, 26), 2.0), ((9, 8, 11), 1.5)):
        g = S.grf(shape, sigma, 81)
        for img in (g, np.round(g * 7).astype(np.uint8)):
            got, st, _ = isa.diagram(img, tfilt=True)
            ref = oracle.diagram(np.asarray(img, np.float32), filtration="T")
            assert st == 0 and diff_pairs(got, ref) is None, (shape, img.dtype)


def test_h1_volumes(isa):
    """PH_H1 on the code object: the Morse expansion of each column (k_h1_morse) and the
    reduction rounds over the unsafe columns (k_h1_reduce, which reads a column either from
    the workspace or from LDS through one generic pointer), against the oracle's every
    dimension, on noise (hundreds of H1 columns, several of them unsafe) and a field."""
    for img in (S.uniform((10, 11, 12), 5), S.grf((20, 18, 16), 1.5, 5)):
        got, st, _ = isa.diagram(img, h1=True)
        assert st == 0 and diff_pairs(got, oracle.diagram(img, dims=(0, 1, 2))) is None, img.shape
