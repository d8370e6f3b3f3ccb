"""GPU tests beyond the small parity sweeps: full-size workloads against stored oracle digests,
batching (bitwise equal to per-image calls, for every tile choice and after autotuning), graph
replay, the backward scatter against the oracle's reference gradient and against finite
differences, and the status words (NaN, capacity).  All go through the C ABI."""
import json
import os

import numpy as np
import pytest

import oracle
import synthetic as S
from gpu_util import diff_pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2606_04801_amd as fc  # noqa: E402
from golden.make_digests import instances, make, pair_digest, input_digest  # noqa: E402
from gpu_util import device_for_tests  # noqa: E402

DEV, HOST_MODE = device_for_tests(fc, torch)
if DEV is None:
    pytest.skip("no GPU", allow_module_level=True)
# against the host build, the full-size workloads take minutes: only with FC_EMULATE_FULL=1
full_size = pytest.mark.skipif(HOST_MODE and os.environ.get("FC_EMULATE_FULL") != "1",
                               reason="full size against the host build: set FC_EMULATE_FULL=1")
DIGESTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.json")


def sync():
    if not HOST_MODE:
        torch.cuda.synchronize()


def gpu(img):
    print("case", img.shape, flush=True)
    return fc.ph_diagram(torch.from_numpy(np.ascontiguousarray(img)).to(DEV)).numpy()


def digests():
    if not os.path.exists(DIGESTS):
        pytest.skip("no stored digests (run tests/golden/make_digests.py)")
    return json.load(open(DIGESTS))


def check_digest(cfg, idx, img, pairs):
    rec = digests().get(cfg, {}).get(str(idx))
    if rec is None:
        pytest.skip("no digest for %s/%d" % (cfg, idx))
    assert rec["input_sha256"] == input_digest(img), "input generator changed"
    top = img.ndim - 1
    assert (int((pairs["dim"] == 0).sum()), int((pairs["dim"] == top).sum())) == (rec["h0"], rec["htop"])
    assert pair_digest(pairs) == rec["pairs_sha256"]


def items(cfg):
    return [it for it in instances() if it[0] == cfg]


@full_size
@pytest.mark.parametrize("cfg", ["c1", "c2", "c2u8", "c3"])
def test_single_full_size(cfg):
    (_, idx, kind, args), = items(cfg)
    img = make(kind, args)
    check_digest(cfg, idx, img, gpu(img))


@full_size
def test_c2u8_through_the_uint8_input_path():
    """Config 2's 256-level copy read as uint8 (PH_IN_U8) gives the stored digest of the same
    values as float32."""
    (_, idx, kind, args), = items("c2u8")
    img = make(kind, args)
    q = img.astype(np.uint8)
    assert np.array_equal(q.astype(np.float32), img)            # the copy holds integers 0..255
    check_digest("c2u8", idx, img, gpu(q))


def run_batch(imgs, tuning=None, autotune=False):
    bt = fc.Batch([a.shape for a in imgs], tuning=tuning, device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    if autotune:
        bt.ph_autotune(reps=1)
    bt.ph_diagram_batch()
    sync()
    return bt, bt.results()


@full_size
@pytest.mark.parametrize("cfg", ["c4", "c5"])
def test_batch_full_size(cfg):
    its = items(cfg)
    imgs = [make(kind, args) for _, _, kind, args in its]
    bt, res = run_batch(imgs)
    for (c, idx, _, _), img, r in zip(its, imgs, res):
        check_digest(c, idx, img, r)


def small_mixed_batch():
    rng = np.random.default_rng(77)
    imgs = []
    for k in range(12):
        if k % 3 == 2:
            shape = tuple(int(x) for x in rng.integers(1, 14, size=3))
        else:
            shape = tuple(int(x) for x in rng.integers(1, 90, size=2))
        lev = int(rng.choice([2, 5, 1 << 20]))
        imgs.append(S.levels(shape, lev, 5000 + k))
    imgs.append(S.grf((130, 70), 3.0, 5100))
    imgs.append(S.grf((20, 33, 17), 2.0, 5101))
    return imgs


def test_batch_equals_single_and_oracle():
    imgs = small_mixed_batch()
    _, res = run_batch(imgs)
    for img, r in zip(imgs, res):
        assert diff_pairs(r, gpu(img)) is None
        assert diff_pairs(r, oracle.diagram(img)) is None


@pytest.mark.parametrize("t2,t3", [(a, b) for a in range(3) for b in range(3)])
def test_tile_choice_never_changes_results(t2, t3):
    imgs = small_mixed_batch()
    _, res = run_batch(imgs, tuning=(t2, t3))
    for img, r in zip(imgs, res):
        assert diff_pairs(r, oracle.diagram(img)) is None


def test_autotune_then_batch():
    imgs = small_mixed_batch()
    _, res = run_batch(imgs, autotune=True)
    for img, r in zip(imgs, res):
        assert diff_pairs(r, oracle.diagram(img)) is None


def loss_grads(bt):
    fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
    diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
    return (-2.0 * diff).contiguous(), (2.0 * diff).contiguous()


def test_backward_against_reference_gradient():
    imgs = small_mixed_batch()
    bt, res = run_batch(imgs)
    gb, gd = loss_grads(bt)
    bt.ph_backward(gb, gd)
    sync()
    for i, (img, r) in enumerate(zip(imgs, res)):
        f = r["death_cell"] >= 0
        d = np.where(f, r["death"] - r["birth"], 0).astype(np.float32)
        ref = oracle.gradient(oracle.diagram(img), -2 * d, 2 * d, img.shape).reshape(-1)
        got = bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]].cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-7)


def test_graph_replay_matches_eager():
    if HOST_MODE:
        pytest.skip("graph capture needs the GPU")
    imgs = small_mixed_batch()
    bt, ref = run_batch(imgs)
    gb, gd = loss_grads(bt)
    bt.ph_backward(gb, gd)
    sync()
    g_ref = bt.grad.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bt.ph_diagram_batch()
        gb2, gd2 = loss_grads(bt)
        bt.ph_backward(gb2, gd2)
    for rep in range(4):
        bt.pairs.birth.fill_(float("nan"))
        bt.grad.fill_(123.0)
        sync()
        graph.replay()
        sync()
        res = bt.results()
        for a, b in zip(res, ref):
            assert diff_pairs(a, b) is None, "replay %d" % rep
        assert torch.equal(bt.grad, g_ref) or torch.allclose(bt.grad, g_ref, rtol=1e-6, atol=1e-7)


def test_finite_differences():
    """dL/dx on tie-free 16x16 inputs, L = sum over finite pairs of (d - b)^2."""
    Fn = fc.PHDiagramFn
    for k in range(4):
        x0 = S.tie_free((16, 16), 4000 + k).astype(np.float64)
        x = torch.tensor(x0, dtype=torch.float32, device=DEV, requires_grad=True)
        b, d, dim = Fn.apply(x)
        fin = torch.isfinite(d)
        loss = ((d - b)[fin] ** 2).sum()
        loss.backward()
        g = x.grad.cpu().numpy().reshape(-1)

        def L(v):
            p = oracle.diagram(v.astype(np.float32))
            f = p["death_cell"] >= 0
            return float(((p["death"][f].astype(np.float64) - p["birth"][f]) ** 2).sum())

        # values are (k + 1/2)/256, so every d - b is a multiple of 1/256 and a non-zero
        # gradient is at least 2/256 in magnitude: a relative tolerance applies to it, and a
        # small absolute one (the rounding of the float32 steps) only where it is zero
        h = 1e-4
        nonzero = 0
        for j in range(256):
            xp, xm = x0.reshape(-1).copy(), x0.reshape(-1).copy()
            xp[j] += h
            xm[j] -= h
            step = float(np.float32(xp[j])) - float(np.float32(xm[j]))
            fd = (L(xp.reshape(16, 16)) - L(xm.reshape(16, 16))) / step
            tol = 1e-3 * abs(fd) if g[j] != 0 else 1e-6
            assert abs(fd - g[j]) <= tol, (k, j, fd, g[j])
            nonzero += g[j] != 0
        assert nonzero >= 16, "too few critical pixels to test"


def test_nan_sets_status():
    img = S.grf((40, 40), 2.0, 1)
    img[7, 9] = np.nan
    d = fc.ph_diagram(torch.from_numpy(img).to(DEV))
    with pytest.raises(fc.PHError) as e:
        d.check()
    assert e.value.code == fc.PH_ENAN


def test_capacity_overflow_reports_true_count():
    img = S.uniform((64, 64), 3)
    full = gpu(img)
    d = fc.ph_diagram(torch.from_numpy(img).to(DEV), capacity=10)
    sync()
    assert int(d.status_t.item()) == fc.PH_ECAPACITY
    assert int(d.count_t.item()) == len(full)
    got = d.bufs.to_numpy(0, 10)
    assert diff_pairs(got, full[:10]) is None


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (2, 2), (1, 1, 1), (1, 1, 7), (7, 1, 1),
                                   (1, 6, 6), (6, 1, 6), (2, 2, 2)])
def test_degenerate_extents(shape):
    for lev in (2, 1 << 20):
        img = S.levels(shape, lev, 6000 + sum(shape))
        assert diff_pairs(gpu(img), oracle.diagram(img)) is None


def _batch_loss(bt, b, d):
    # masked before squaring: a where() after the square would send 0 * inf = NaN back
    # through the essential pair (death +inf) and through unused pair slots
    fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
    return (torch.where(fin, d - b, torch.zeros_like(d)) ** 2).sum()


def test_batch_autograd_finite_differences():
    """BatchDiagramFn on a mixed tie-free batch (two 16x16 images, one 6x6x6 volume):
    L = sum over finite pairs of (d - b)^2, dL/dx from loss.backward() against central
    differences of the oracle's L (step 1e-4 over the exact float32 step), relative 1e-3."""
    imgs = [S.tie_free((16, 16), 4100), S.tie_free((6, 6, 6), 4101), S.tie_free((16, 16), 4102)]
    bt = fc.Batch([a.shape for a in imgs], device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    x = bt.images.detach().clone().requires_grad_(True)
    b, d = fc.BatchDiagramFn.apply(x, bt)
    _batch_loss(bt, b, d).backward()
    g = x.grad.cpu().numpy()

    def L(v):
        p = oracle.diagram(v.astype(np.float32))
        f = p["death_cell"] >= 0
        return float(((p["death"][f].astype(np.float64) - p["birth"][f]) ** 2).sum())

    h = 1e-4
    nonzero = 0
    for i, a in enumerate(imgs):
        x0 = a.astype(np.float64).reshape(-1)
        gi = g[bt.img_off_h[i]:bt.img_off_h[i + 1]]
        for j in range(a.size):
            xp, xm = x0.copy(), x0.copy()
            xp[j] += h
            xm[j] -= h
            step = float(np.float32(xp[j])) - float(np.float32(xm[j]))
            fd = (L(xp.reshape(a.shape)) - L(xm.reshape(a.shape))) / step
            tol = 1e-3 * abs(fd) if gi[j] != 0 else 1e-6
            assert abs(fd - gi[j]) <= tol, (i, j, fd, gi[j])
            nonzero += gi[j] != 0
    assert nonzero >= 24


def test_batch_autograd_equals_manual_backward():
    """loss.backward() through BatchDiagramFn gives bitwise the gradient of the manual path
    (the loss gradient computed by hand, then ph_backward), and the diagrams of a plain call."""
    imgs = small_mixed_batch()
    bt, res = run_batch(imgs)
    gb, gd = loss_grads(bt)
    bt.ph_backward(gb, gd)
    sync()
    g_manual = bt.grad.clone()
    x = bt.images.detach().clone().requires_grad_(True)
    b, d = fc.BatchDiagramFn.apply(x, bt)
    _batch_loss(bt, b, d).backward()
    sync()
    for a, r in zip(bt.results(), res):
        assert diff_pairs(a, r) is None
    # additions to one pixel are atomic, so their order (and last bits) may differ
    assert torch.allclose(x.grad, g_manual, rtol=1e-6, atol=1e-7)


def test_batch_autograd_graph_replay():
    """Forward, loss and loss.backward() through BatchDiagramFn captured in one graph over the
    batch's own input tensor; every replay (inputs changed in place between replays) gives the
    eager gradient and diagrams of the same inputs."""
    if HOST_MODE:
        pytest.skip("graph capture needs the GPU")
    sets = [small_mixed_batch(), [S.grf(a.shape, 1.7, 77 + k) for k, a in enumerate(small_mixed_batch())]]
    bt = fc.Batch([a.shape for a in sets[0]], device=DEV)
    refs = []
    for imgs in sets:
        bt.set_images([torch.from_numpy(a) for a in imgs])
        x = bt.images.detach().clone().requires_grad_(True)
        b, d = fc.BatchDiagramFn.apply(x, bt)
        _batch_loss(bt, b, d).backward()
        sync()
        refs.append((bt.results(), x.grad.clone()))
    bt.set_images([torch.from_numpy(a) for a in sets[0]])
    bt.images.requires_grad_(True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                       # warm-up on a side stream, as capture requires
        b, d = fc.BatchDiagramFn.apply(bt.images, bt)
        _batch_loss(bt, b, d).backward()
    torch.cuda.current_stream().wait_stream(s)
    bt.images.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b, d = fc.BatchDiagramFn.apply(bt.images, bt)
        _batch_loss(bt, b, d).backward()
    for rep in range(4):
        k = rep % 2
        with torch.no_grad():
            bt.images.copy_(torch.cat([torch.from_numpy(a).reshape(-1) for a in sets[k]]).to(DEV))
        bt.pairs.birth.fill_(float("nan"))
        sync()
        graph.replay()
        sync()
        for a, r in zip(bt.results(), refs[k][0]):
            assert diff_pairs(a, r) is None, "replay %d" % rep
        assert torch.allclose(bt.images.grad, refs[k][1], rtol=1e-6, atol=1e-7), "replay %d" % rep
