"""uint8 and uint16 inputs on the GPU (PH_IN_U8, PH_IN_U16): the oracle's pairs of the same
values as float32, and bit for bit the float32 path's results (pairs and gradient)."""
import numpy as np
import pytest

import oracle
import synthetic as S
from gpu_util import diff_pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2606_04801_amd as fc  # noqa: E402
from gpu_util import device_for_tests  # noqa: E402

DEV, HOST_MODE = device_for_tests(fc, torch)
if DEV is None:
    pytest.skip("no GPU", allow_module_level=True)

CASES = [(np.uint8, 255), (np.uint16, 65535), (np.uint8, 6)]


def gpu_diagram(img):
    print("case", img.shape, img.dtype, flush=True)
    return fc.ph_diagram(torch.from_numpy(np.ascontiguousarray(img)).to(DEV)).numpy()


@pytest.mark.parametrize("shape, sigma", [((200, 170), 3.0), ((40, 36, 44), 2.0)])
@pytest.mark.parametrize("dt, levels", CASES)
def test_integer_image(shape, sigma, dt, levels):
    q = np.round(S.grf(shape, sigma, 11) * levels).astype(dt)
    got = gpu_diagram(q)
    msg = diff_pairs(got, oracle.diagram(q.astype(np.float32)))
    assert msg is None, msg
    same = gpu_diagram(q.astype(np.float32))
    for f in got.dtype.names:
        assert np.array_equal(got[f], same[f]), f


@pytest.mark.parametrize("dt, levels", CASES)
def test_integer_batch_with_backward(dt, levels):
    shapes = [(96, 96, 96), (512, 512), (33, 17, 9), (7, 300)]
    qs = [np.round(S.grf(s, 3.0, 100 + k) * levels).astype(dt) for k, s in enumerate(shapes)]
    out = []
    for kind in (torch.float32, getattr(torch, np.dtype(dt).name)):
        print("batch", kind, flush=True)
        bt = fc.Batch(shapes, device=DEV, dtype=kind)
        bt.set_images([torch.from_numpy(q) for q in qs])
        bt.ph_diagram_batch()
        fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
        diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
        bt.ph_backward(-2.0 * diff, 2.0 * diff)
        torch.cuda.synchronize()
        out.append((bt.results(), bt.grad.cpu().numpy().copy()))
    (rf, gf), (ri, gi) = out
    for k, (a, b) in enumerate(zip(rf, ri)):
        for f in a.dtype.names:
            assert np.array_equal(a[f], b[f]), (k, f)
    assert np.array_equal(gf, gi)
    for k in (2, 3):                                    # the small ones against the oracle too
        assert diff_pairs(ri[k], oracle.diagram(qs[k].astype(np.float32))) is None, shapes[k]


def test_autotune_with_integer_input_keeps_defaults():
    """An integer batch always runs the default tiles: ph_autotune returns them, the results
    are the oracle's, and nothing is recorded for the size class."""
    shapes = [(64, 80), (12, 10, 14)]
    qs = [np.round(S.grf(s, 2.0, 300 + k) * 255).astype(np.uint8) for k, s in enumerate(shapes)]
    bt = fc.Batch(shapes, device=DEV, dtype=torch.uint8)
    bt.set_images([torch.from_numpy(q) for q in qs])
    assert bt.ph_autotune(reps=1) == (0, 0)
    torch.cuda.synchronize()
    for q, got in zip(qs, bt.results()):
        assert diff_pairs(got, oracle.diagram(q.astype(np.float32))) is None, q.shape
