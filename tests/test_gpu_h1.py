"""GPU parity of 3D H1 (PH_H1, Sec. 4.2 steps 4-5) through the C ABI: every field of every pair
of H0, H1 and H2 against the oracle's full boundary-matrix reduction of all dimensions, bit for
bit (fixtures, tie-heavy sweeps with degenerate extents, fields, noise, special values, mixed
batches with images, the T-filtration, and full-size bench volumes against stored digests)."""
import json
import os

import numpy as np
import pytest

import oracle
import synthetic as S
import fixtures
from gpu_util import diff_pairs, device_for_tests

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2606_04801_amd as fc  # noqa: E402

DEV, HOST_MODE = device_for_tests(fc, torch)
if DEV is None:
    pytest.skip("no GPU", allow_module_level=True)
ALL = fc.PH_H0 | fc.PH_HTOP | fc.PH_H1


def gpu(img, filtration="V", flags=ALL):
    print("case H1", img.dtype, img.shape, filtration, flush=True)
    return fc.ph_diagram(torch.from_numpy(np.ascontiguousarray(img)).to(DEV), flags=flags,
                         filtration=filtration).numpy()


def ref(img, filtration="V"):
    dims = (0, 1, 2) if img.ndim == 3 else (0, 1)
    return oracle.diagram(np.asarray(img, np.float32), dims=dims, filtration=filtration)


def check(img, filtration="V", label=""):
    msg = diff_pairs(gpu(img, filtration), ref(img, filtration))
    assert msg is None, "%s %s %s: %s" % (label, img.shape, filtration, msg)


@pytest.mark.parametrize("name,img,expected,case", [f for f in fixtures.load() if f[1].ndim == 3],
                         ids=lambda x: x if isinstance(x, str) else "")
def test_fixtures(name, img, expected, case):
    check(img, label=name)


def test_tiny_sweep():
    rng = np.random.default_rng(31)
    for k in range(60):
        shape = tuple(int(x) for x in rng.integers(1, 7, size=3))
        img = S.levels(shape, int(rng.choice([2, 3, 5, 1 << 20])), 9000 + k)
        check(img, label="sweep %d" % k)


@pytest.mark.parametrize("shape", [(1, 6, 7), (6, 1, 7), (6, 7, 1), (1, 1, 9), (2, 2, 2), (2, 9, 9), (9, 2, 9)])
def test_degenerate_extents(shape):
    for lev in (2, 1 << 20):
        check(S.levels(shape, lev, 9100 + sum(shape)), label="degenerate")


@pytest.mark.parametrize("shape,sigma,seed", [((20, 22, 18), 2.0, 1), ((33, 30, 28), 3.0, 2), ((40, 24, 36), 4.0, 3),
                                              ((48, 48, 48), 3.0, 4)])
def test_fields(shape, sigma, seed):
    check(S.grf(shape, sigma, seed), label="field")


def test_noise_and_ties():
    check(S.uniform((16, 17, 15), 5), label="uniform")
    # more KEEP edges than the reduction keeps in LDS: the workspace path
    check(S.uniform((30, 31, 29), 25), label="uniform, reduction out of the workspace")
    check(S.levels((14, 13, 12), 3, 6), label="three levels")
    check(S.quantize_u8(S.grf((24, 26, 22), 3.0, 7)), label="quantised")


def test_special_values():
    a = S.grf((9, 10, 11), 1.5, 8)
    flat = a.reshape(-1)
    flat[[3, 50, 400, 777]] = np.array([np.inf, -np.inf, -0.0, 1e-45], np.float32)
    check(a, label="specials")


def test_integer_input():
    q = S.quantize_u8(S.grf((20, 19, 21), 2.5, 9))
    got = gpu(q.astype(np.uint8))
    assert diff_pairs(got, ref(q)) is None


def test_t_filtration():
    for k, img in enumerate([S.grf((14, 15, 13), 2.0, 10), S.levels((7, 8, 6), 3, 11), S.uniform((9, 8, 10), 12)]):
        check(img, filtration="T", label="T %d" % k)


def test_flag_ignored_by_images_and_off_by_default():
    img2 = S.grf((40, 37), 2.0, 13)
    assert diff_pairs(gpu(img2), oracle.diagram(img2)) is None
    vol = S.grf((18, 17, 19), 2.0, 14)
    assert diff_pairs(gpu(vol, flags=fc.PH_H0 | fc.PH_HTOP), oracle.diagram(vol)) is None
    only = gpu(vol, flags=fc.PH_H1)
    r = ref(vol)
    assert diff_pairs(only, r[r["dim"] == 1]) is None


def test_mixed_batch_with_counters():
    imgs = [S.grf((22, 20, 24), 2.0, 15), S.grf((50, 41), 2.0, 16), S.levels((6, 7, 5), 3, 17),
            S.uniform((12, 11, 13), 18), S.grf((1, 30, 31), 2.0, 19)]
    bt = fc.Batch([a.shape for a in imgs], flags=ALL, device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    bt.ph_diagram_batch()
    for a, got in zip(imgs, bt.results()):
        assert diff_pairs(got, ref(a)) is None, a.shape
    wc = bt.work_counters()
    assert wc[0, 8] > 0 and wc[1, 8] == 0 and wc[:, 7].sum() == 0


def test_batch_backward_with_h1():
    """The H1 pairs' gradients go to their critical pixels like the others'."""
    imgs = [S.grf((12, 13, 11), 2.0, 20), S.grf((30, 28), 2.0, 21)]
    bt = fc.Batch([a.shape for a in imgs], flags=ALL, device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    bt.ph_diagram_batch()
    fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
    diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
    bt.ph_backward((-2.0 * diff).contiguous(), (2.0 * diff).contiguous())
    res = bt.results()
    for i, (a, r) in enumerate(zip(imgs, res)):
        f = r["death_cell"] >= 0
        d = np.where(f, r["death"] - r["birth"], 0).astype(np.float32)
        g = oracle.gradient(ref(a), -2 * d, 2 * d, a.shape).reshape(-1)
        got = bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]].cpu().numpy()
        np.testing.assert_allclose(got, g, rtol=1e-6, atol=1e-7)


@pytest.mark.skipif(HOST_MODE, reason="full size against the host build takes minutes")
def test_full_size_bench_volumes_against_digests():
    """The first eight 96^3 volumes (sigma 3) of the bench workload in one batch under PH_H1,
    each against the digest of the oracle's H0 + H1 + H2 (tests/golden/make_digests.py, c5h1)."""
    from golden.make_digests import instances, make, pair_digest, input_digest
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.json")
    dig = json.load(open(path)).get("c5h1")
    if not dig:
        pytest.skip("no c5h1 digests")
    its = [it for it in instances() if it[0] == "c5h1"]
    imgs = [make(kind, args) for _, _, kind, args in its]
    bt = fc.Batch([a.shape for a in imgs], flags=ALL, device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    print("H1 batch of", len(imgs), flush=True)
    bt.ph_diagram_batch()
    for (c, idx, _, _), img, r in zip(its, imgs, bt.results()):
        rec = dig[str(idx)]
        assert rec["input_sha256"] == input_digest(img)
        assert pair_digest(r) == rec["pairs_sha256"], idx


@pytest.mark.parametrize("tuning", [(1, 1), (2, 2), "autotune"])
def test_tile_choices_under_h1(tuning):
    """A tuned 3D tile (explicit, or recorded by the autotuner for the size class) must not
    change the H1 results: volumes under PH_H1 plan and run the default 3D tile."""
    imgs = [S.grf((22, 20, 24), 2.0, 30), S.grf((50, 41), 2.0, 31), S.uniform((12, 11, 13), 32)]
    shapes = [a.shape for a in imgs]
    if tuning == "autotune":
        at = fc.Batch(shapes, device=DEV)
        at.set_images([torch.from_numpy(a) for a in imgs])
        at.ph_autotune(reps=1)
        bt = fc.Batch(shapes, flags=ALL, device=DEV)
    else:
        bt = fc.Batch(shapes, flags=ALL, tuning=tuning, device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    bt.ph_diagram_batch()
    for a, got in zip(imgs, bt.results()):
        assert diff_pairs(got, ref(a)) is None, a.shape


def ring_valley(R, depth, seed):
    """A valley along a horizontal circle of radius R: one long H1 class whose killing square
    sweeps the whole disk, so that column's running sum holds hundreds of edges at once."""
    n = 2 * R + 12
    z, y, x = np.mgrid[0:depth, 0:n, 0:n].astype(np.float64)
    c = (n - 1) / 2
    f = (np.hypot(y - c, x - c) - R) ** 2 + 4 * (z - (depth - 1) / 2) ** 2
    f += np.random.default_rng(seed).random(f.shape) * 1e-3
    return (f / f.max()).astype(np.float32)


def test_large_column_takes_the_second_pass():
    """A column whose live edges outgrow the first pass's tables is finished by the second
    pass (work counter 12 > 0), with the oracle's result."""
    a = ring_valley(100, 6, 1)
    bt = fc.Batch([a.shape], flags=ALL, device=DEV)
    bt.set_images([torch.from_numpy(a)])
    bt.ph_diagram_batch()
    (got,) = bt.results()
    assert bt.work_counters()[0, 12] > 0
    assert diff_pairs(got, ref(a)) is None
