"""GPU parity of the T-filtration (PH_TFILT, pixels as top cells) through the C ABI against the
oracle's T-filtration, bit for bit: every field of every pair, in the T output order (by
dimension, then by death key, essential class last)."""
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


def sync():
    if not HOST_MODE:
        torch.cuda.synchronize()


def gpu_t(img, **kw):
    print("case T", img.dtype, img.shape, flush=True)
    return fc.ph_diagram(torch.from_numpy(np.ascontiguousarray(img)).to(DEV), filtration="T", **kw).numpy()


def check(img, label=""):
    ref = oracle.diagram(np.asarray(img, np.float32), filtration="T")
    msg = diff_pairs(gpu_t(img), ref)
    assert msg is None, "%s %s: %s" % (label, img.shape, msg)


def test_hand_cases():
    a = np.array([[0, 1], [1, 0]], np.float32)            # corner contact joins under T
    check(a, "diag")
    r = np.zeros((3, 3), np.float32)
    r[1, 1] = 5
    check(r, "ring")


def test_tiny_sweep_2d():
    rng = np.random.default_rng(11)
    for k in range(120):
        shape = tuple(int(x) for x in rng.integers(1, 10, size=2))
        lev = int(rng.choice([2, 3, 5, 1 << 20]))
        check(S.levels(shape, lev, 40_000 + k), "2d#%d" % k)


def test_tiny_sweep_3d():
    rng = np.random.default_rng(12)
    for k in range(100):
        shape = tuple(int(x) for x in rng.integers(1, 7, size=3))
        lev = int(rng.choice([2, 3, 5, 1 << 20]))
        check(S.levels(shape, lev, 50_000 + k), "3d#%d" % k)


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (2, 2), (1, 1, 1), (1, 1, 7), (7, 1, 1),
                                   (1, 6, 6), (6, 1, 6), (2, 2, 2)])
def test_degenerate_extents(shape):
    for lev in (2, 1 << 20):
        check(S.levels(shape, lev, 60_000 + sum(shape)), "degenerate")


def test_special_values():
    a = np.array([[0.0, -0.0, 1.0, -np.inf], [-np.inf, 0.5, -0.0, 0.0], [1e-45, -1e-45, 3.0, 0.0]], np.float32)
    check(a, "specials")
    check(np.stack([a, a[::-1], a]).astype(np.float32), "specials3d")


@pytest.mark.parametrize("shape,sigma", [((200, 300), 2.0), ((257, 131), 4.0), ((70, 1030), 1.0)])
def test_fields_2d(shape, sigma):
    x = S.grf(shape, sigma, 15)
    check(x, "grf")
    check(S.quantize_u8(x), "u8")


@pytest.mark.parametrize("shape,sigma", [((40, 35, 50), 1.5), ((17, 64, 33), 2.0), ((1, 40, 41), 1.0)])
def test_fields_3d(shape, sigma):
    x = S.grf(shape, sigma, 16)
    check(x, "grf3")
    check(S.quantize_u8(x), "u8-3")


def test_uniform_noise():
    check(S.uniform((96, 80), 17), "uniform2d")
    check(S.uniform((20, 26, 24), 18), "uniform3d")


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_integer_inputs(dtype):
    """uint8 / uint16 inputs under T give bitwise the pairs of the same values as float32."""
    rng = np.random.default_rng(19)
    hi = 255 if dtype == np.uint8 else 65535
    for shape in [(37, 53), (9, 14, 11)]:
        q = rng.integers(0, hi + 1, size=shape).astype(dtype)
        q[0, 0] = hi
        assert diff_pairs(gpu_t(q), oracle.diagram(q.astype(np.float32), filtration="T")) is None


@pytest.mark.parametrize("flags", [fc.PH_H0, fc.PH_HTOP])
def test_one_dimension_only(flags):
    for img in (S.grf((60, 45), 2.0, 20), S.grf((14, 12, 15), 1.5, 21)):
        want = oracle.diagram(img, filtration="T")
        want = want[want["dim"] == (0 if flags == fc.PH_H0 else img.ndim - 1)]
        assert diff_pairs(gpu_t(img, flags=flags), want) is None


def test_plus_infinity_is_reported():
    img = S.grf((30, 30), 2.0, 22)
    img[4, 5] = np.inf
    d = fc.ph_diagram(torch.from_numpy(img).to(DEV), filtration="T")
    with pytest.raises(fc.PHError) as e:
        d.check()
    assert e.value.code == fc.PH_ENAN


def mixed_batch():
    rng = np.random.default_rng(23)
    imgs = []
    for k in range(10):
        if k % 3 == 2:
            shape = tuple(int(x) for x in rng.integers(1, 12, size=3))
        else:
            shape = tuple(int(x) for x in rng.integers(1, 70, size=2))
        imgs.append(S.levels(shape, int(rng.choice([2, 5, 1 << 20])), 61_000 + k))
    imgs.append(S.grf((120, 64), 3.0, 61_100))
    imgs.append(S.grf((18, 30, 16), 2.0, 61_101))
    return imgs


@pytest.mark.parametrize("tuning", [None, (1, 2), (2, 1)])
def test_batch_with_backward(tuning):
    imgs = mixed_batch()
    bt = fc.Batch([a.shape for a in imgs], tuning=tuning, device=DEV, filtration="T")
    bt.set_images([torch.from_numpy(a) for a in imgs])
    bt.ph_diagram_batch()
    sync()
    res = bt.results()
    for img, r in zip(imgs, res):
        assert diff_pairs(r, oracle.diagram(img, filtration="T")) is None
    fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
    diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
    bt.ph_backward((-2.0 * diff).contiguous(), (2.0 * diff).contiguous())
    sync()
    for i, (img, r) in enumerate(zip(imgs, res)):
        f = r["death_cell"] >= 0
        d = np.where(f, r["death"] - r["birth"], 0).astype(np.float32)
        ref = oracle.gradient(oracle.diagram(img, filtration="T"), -2 * d, 2 * d, img.shape).reshape(-1)
        got = bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]].cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-7)


def test_v_and_t_batches_share_nothing():
    """A V call after a T call on the same workspace gives the V oracle's pairs (the T frame
    and the framed layout leave nothing behind)."""
    img = S.grf((50, 70), 2.0, 24)
    ws = fc.Workspace()
    t = fc.ph_diagram(torch.from_numpy(img).to(DEV), filtration="T", ws=ws).numpy()
    v = fc.ph_diagram(torch.from_numpy(img).to(DEV), ws=ws).numpy()
    assert diff_pairs(t, oracle.diagram(img, filtration="T")) is None
    assert diff_pairs(v, oracle.diagram(img)) is None


def test_autograd_function_under_t():
    x0 = S.tie_free((12, 12), 25)
    x = torch.tensor(x0, dtype=torch.float32, device=DEV, requires_grad=True)
    b, d, dim = fc.PHDiagramFn.apply(x, "T")
    fin = torch.isfinite(d)
    ((d - b)[fin] ** 2).sum().backward()
    p = oracle.diagram(x0, filtration="T")
    f = p["death_cell"] >= 0
    dd = np.where(f, p["death"] - p["birth"], 0).astype(np.float32)
    ref = oracle.gradient(p, -2 * dd, 2 * dd, x0.shape)
    np.testing.assert_allclose(x.grad.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)


def test_graph_replay_t():
    """A T forward + backward captured in a HIP graph replays to the eager results (the frame
    is written by a kernel, nothing by a memset)."""
    if HOST_MODE:
        pytest.skip("graph capture needs the GPU")
    imgs = mixed_batch()
    bt = fc.Batch([a.shape for a in imgs], device=DEV, filtration="T")
    bt.set_images([torch.from_numpy(a) for a in imgs])

    def step():
        bt.ph_diagram_batch()
        fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
        diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
        bt.ph_backward((-2.0 * diff).contiguous(), (2.0 * diff).contiguous())

    step()
    sync()
    ref, g_ref = bt.results(), bt.grad.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        bt.pairs.birth.fill_(float("nan"))
        bt.grad.fill_(123.0)
        bt.ws.fill_(0x5A)
        sync()
        graph.replay()
        sync()
        for a, b in zip(bt.results(), ref):
            assert diff_pairs(a, b) is None, "replay %d" % rep
        assert torch.equal(bt.grad, g_ref), "replay %d" % rep


@pytest.mark.skipif(HOST_MODE, reason="full size against the host build takes minutes")
def test_full_size_bench_batch_t_against_digests():
    """All 128 instances of the bench workload (64 volumes 96^3 sigma 3, 64 images 512^2
    sigma 6) in one T batch with the bench's launch configuration, each against the digest of
    the T oracle's diagram (tests/golden/make_digests.py, config c5t)."""
    import json
    import os
    from golden.make_digests import instances, make, pair_digest, input_digest
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.json")
    dig = json.load(open(path)).get("c5t")
    if not dig:
        pytest.skip("no c5t digests")
    its = [it for it in instances() if it[0] == "c5t"]
    imgs = [make(kind, args) for _, _, kind, args in its]
    bt = fc.Batch([a.shape for a in imgs], device=DEV, filtration="T")
    bt.set_images([torch.from_numpy(a) for a in imgs])
    print("T batch of", len(imgs), flush=True)
    bt.ph_diagram_batch()
    sync()
    for (c, idx, _, _), img, r in zip(its, imgs, bt.results()):
        rec = dig[str(idx)]
        assert rec["input_sha256"] == input_digest(img), "input generator changed"
        top = img.ndim - 1
        assert (int((r["dim"] == 0).sum()), int((r["dim"] == top).sum())) == (rec["h0"], rec["htop"]), idx
        assert pair_digest(r) == rec["pairs_sha256"], idx
