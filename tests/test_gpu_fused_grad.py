"""ph_diagram_batch_grad + ph_backward_scatter (the input gradient cleared inside the classify
passes, then only the scatter) against ph_diagram_batch + ph_backward through the C ABI: the
same pairs bit for bit and the same gradient, on a gradient buffer first filled with NaNs, for
float32, uint8 and uint16 inputs, both filtrations, every tile choice, PH_H1 and PH_WIDE, in a
HIP graph, and through the batched autograd Function; the gradient also against the oracle's."""
import numpy as np
import pytest

import oracle
import synthetic as S
from gpu_util import diff_pairs, device_for_tests

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2606_04801_amd as fc  # noqa: E402

DEV, HOST_MODE = device_for_tests(fc, torch)
if DEV is None:
    pytest.skip("no GPU", allow_module_level=True)
NAN = float("nan")


def sync():
    if not HOST_MODE:
        torch.cuda.synchronize()


def step(bt, fused):
    bt.ph_diagram_batch(grad=bt.grad if fused else None)
    fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
    diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
    bt.ph_backward((-2.0 * diff).contiguous(), (2.0 * diff).contiguous(), zeroed=fused)


def same_grad(a, b):
    # additions to one pixel are atomic, so with three or more their order (last bits) may differ
    return bool(torch.isfinite(a).all()) and torch.allclose(a, b, rtol=1e-6, atol=1e-7)


def fused_against_plain(imgs, label, **kw):
    bt = fc.Batch([a.shape for a in imgs], device=DEV, **kw)
    bt.set_images([torch.from_numpy(np.ascontiguousarray(a)) for a in imgs])
    print("fused grad:", label, [a.shape for a in imgs][:4], flush=True)
    step(bt, False)
    sync()
    ref, g_ref = bt.results(), bt.grad.clone()
    for rep in range(2):                             # twice: the second call finds the first's gradient
        if rep == 0:
            bt.grad.fill_(NAN)
        step(bt, True)
        sync()
        for k, (a, b) in enumerate(zip(bt.results(), ref)):
            assert diff_pairs(a, b) is None, (label, k)
        assert same_grad(bt.grad, g_ref), (label, rep)
    return bt, ref


def mixed_float():
    rng = np.random.default_rng(70_000)
    imgs = [S.grf((130, 70), 3.0, 70_001), S.grf((33, 20, 41), 2.0, 70_002), S.uniform((1, 300), 70_003),
            S.uniform((9, 1, 13), 70_004), S.grf((64, 16), 2.0, 70_005), S.uniform((2, 2, 2), 70_006)]
    for k in range(4):
        nd = int(rng.integers(2, 4))
        shape = tuple(int(v) for v in rng.integers(1, 24, size=nd))
        imgs.append(S.levels(shape, int(rng.choice([2, 5, 1 << 20])), 70_010 + k))
    return imgs


@pytest.mark.parametrize("tuning", [None, (1, 1), (2, 2)])
def test_float_batch_every_tile(tuning):
    imgs = mixed_float()
    bt, ref = fused_against_plain(imgs, "float %s" % (tuning,), tuning=tuning)
    for i in (0, 1, 3, 6):                           # the gradient itself against the oracle's
        img, r = imgs[i], ref[i]
        f = r["death_cell"] >= 0
        d = np.where(f, r["death"] - r["birth"], 0).astype(np.float32)
        want = oracle.gradient(oracle.diagram(img), -2 * d, 2 * d, img.shape).reshape(-1)
        got = bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]].cpu().numpy()
        np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("dt, levels", [(np.uint8, 255), (np.uint16, 65535), (np.uint8, 6)])
def test_integer_inputs(dt, levels):
    shapes = [(96, 80), (33, 17, 9), (7, 300), (1, 1, 5)]
    qs = [np.round(S.grf(s, 3.0, 71_000 + k) * levels).astype(dt) for k, s in enumerate(shapes)]
    fused_against_plain(qs, np.dtype(dt).name, dtype=getattr(torch, np.dtype(dt).name))


@pytest.mark.parametrize("tuning", [None, (1, 2), (2, 1)])
def test_t_filtration(tuning):
    """Under the T-filtration the kernels see the framed grid: only its inner pixels, through
    the reflection, are the caller's."""
    imgs = [S.grf((120, 64), 3.0, 72_001), S.grf((18, 30, 16), 2.0, 72_002), S.uniform((1, 9), 72_003),
            S.uniform((1, 1, 1), 72_004), S.levels((13, 11, 7), 3, 72_005)]
    bt, ref = fused_against_plain(imgs, "T %s" % (tuning,), tuning=tuning, filtration="T")
    for i in (0, 1, 4):
        img, r = imgs[i], ref[i]
        f = r["death_cell"] >= 0
        d = np.where(f, r["death"] - r["birth"], 0).astype(np.float32)
        want = oracle.gradient(oracle.diagram(img, filtration="T"), -2 * d, 2 * d, img.shape).reshape(-1)
        got = bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]].cpu().numpy()
        np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-7)


def test_h1_batch():
    imgs = [S.grf((22, 20, 24), 2.0, 73_001), S.grf((50, 41), 2.0, 73_002), S.uniform((12, 11, 13), 73_003)]
    fused_against_plain(imgs, "H1", flags=fc.PH_H0 | fc.PH_HTOP | fc.PH_H1)


@pytest.mark.skipif(HOST_MODE, reason="2^20 voxels against the host build take minutes")
def test_wide_batch():
    imgs = [S.uniform((1024, 1024), 74_001), S.grf((40, 30, 20), 2.0, 74_002), S.uniform((5, 7), 74_003)]
    fused_against_plain(imgs, "wide", flags=fc.PH_H0 | fc.PH_HTOP | fc.PH_WIDE)


def test_graph_replay():
    """Forward with the clear and the scatter captured in one HIP graph: every replay, on a
    gradient full of NaNs, gives the eager plain path's gradient and pairs."""
    if HOST_MODE:
        pytest.skip("graph capture needs the GPU")
    imgs = mixed_float()
    bt = fc.Batch([a.shape for a in imgs], device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    step(bt, False)
    sync()
    ref, g_ref = bt.results(), bt.grad.clone()
    step(bt, True)                                   # warm-up outside the capture
    sync()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(bt, True)
    for rep in range(3):
        bt.pairs.birth.fill_(NAN)
        bt.grad.fill_(NAN)
        bt.ws.fill_(0x5A)
        sync()
        graph.replay()
        sync()
        for a, b in zip(bt.results(), ref):
            assert diff_pairs(a, b) is None, "replay %d" % rep
        assert same_grad(bt.grad, g_ref), "replay %d" % rep


def test_autograd_function_uses_the_fused_clear():
    """BatchDiagramFn allocates its gradient uninitialised and has the forward clear it: the
    gradient of loss.backward() is the plain path's, and a forward without requires_grad
    takes no gradient buffer."""
    imgs = mixed_float()
    bt = fc.Batch([a.shape for a in imgs], device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    step(bt, False)
    sync()
    ref, g_ref = bt.results(), bt.grad.clone()
    x = bt.images.detach().clone().requires_grad_(True)
    b, d = fc.BatchDiagramFn.apply(x, bt)
    fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
    (torch.where(fin, d - b, torch.zeros_like(d)) ** 2).sum().backward()
    sync()
    for a, r in zip(bt.results(), ref):
        assert diff_pairs(a, r) is None
    assert same_grad(x.grad, g_ref)
    with torch.no_grad():
        b2, d2 = fc.BatchDiagramFn.apply(bt.images, bt)
    v = bt.valid_mask()                             # slots past a count hold no pair
    assert torch.equal(b2[v], b.detach()[v]) and torch.equal(d2[v], d.detach()[v])


def test_null_gradient_is_rejected():
    bt = fc.Batch([(8, 8)], device=DEV)
    L = fc.lib()
    tp = None
    rc = L.ph_diagram_batch_grad(bt.n, fc._ptr(bt.images), fc._ptr(bt.img_off), fc._ptr(bt.d_shapes), bt.h_shapes,
                                 bt.flags, bt.pairs.c(), fc._ptr(bt.out_off), fc._ptr(bt.counts),
                                 fc._ptr(bt.status), tp, fc._ptr(bt.ws), bt.ws_bytes, None, None)
    assert rc == fc.PH_EINVAL
    with pytest.raises(fc.PHError):
        bt.ph_diagram_batch(grad=torch.zeros(bt.total_voxels + 1, device=DEV))


def test_failed_instance_is_cleared_too():
    """An instance that stops on a NaN (PH_ENAN, its other tiles skip their work) still has
    every pixel of its gradient cleared, as ph_backward's fill would: the clear comes before the
    classify passes look at the instance's error word."""
    imgs = [S.grf((70, 90), 2.0, 75_001), S.grf((300, 200), 3.0, 75_002), S.grf((40, 36, 44), 2.0, 75_003),
            S.grf((24, 24, 24), 2.0, 75_004)]
    imgs[1][5, 7] = np.nan
    imgs[3][1, 2, 3] = np.nan
    bt = fc.Batch([a.shape for a in imgs], device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    print("fused grad: NaN instances", flush=True)

    def step_ok(fused):
        bt.ph_diagram_batch(grad=bt.grad if fused else None)
        fin = bt.valid_mask() & (bt.pairs.death_cell >= 0) & (bt.status[bt._slot_inst] == fc.PH_OK)
        diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
        bt.ph_backward((-2.0 * diff).contiguous(), (2.0 * diff).contiguous(), zeroed=fused)

    step_ok(False)
    sync()
    st = bt.status.cpu().numpy()
    assert list(st) == [fc.PH_OK, fc.PH_ENAN, fc.PH_OK, fc.PH_ENAN], st
    ref, g_ref = [bt.result(i) for i in (0, 2)], bt.grad.clone()
    bt.grad.fill_(NAN)
    step_ok(True)
    sync()
    assert list(bt.status.cpu().numpy()) == list(st)
    for k, i in enumerate((0, 2)):
        assert diff_pairs(bt.result(i), ref[k]) is None
    assert same_grad(bt.grad, g_ref)
    for i in (1, 3):
        assert not bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]].any()
