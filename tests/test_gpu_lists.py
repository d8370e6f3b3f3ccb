"""The list fraction (PH_LIST_FRACTION): per-instance lists sized to k/256 of their worst case.

Results that fit are bitwise those of the worst-case sizing (and the oracle's); an instance
whose lists outgrow their capacities reports PH_ELISTS, its neighbours in the batch are not
affected, and the work counters give the true list sizes, from which a sufficient fraction
follows.  All through the C ABI."""
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

H = fc.PH_H0 | fc.PH_HTOP


def batch(imgs, flags, filtration="V"):
    bt = fc.Batch([a.shape for a in imgs], device=DEV, flags=flags, filtration=filtration)
    bt.set_images([torch.from_numpy(np.ascontiguousarray(a)) for a in imgs])
    print("batch", [a.shape for a in imgs], "flags", flags, filtration, flush=True)
    bt.ph_diagram_batch()
    return bt


def statuses(bt):
    return bt.status.cpu().numpy().tolist()


def fraction_needed(shape, w):
    """The smallest k whose capacities (ceil(worst k / 256), at least 4096) hold the counted
    KEEP edges, KEEP squares, H0 nodes and dual nodes (work counters 0-3)."""
    if len(shape) == 2:
        h, wd = shape
        worst = [h * (wd - 1) + (h - 1) * wd, 0, h * wd, (h - 1) * (wd - 1) + 1]
    else:
        d, h, wd = shape
        worst = [d * h * (wd - 1) + d * (h - 1) * wd + (d - 1) * h * wd,
                 d * (h - 1) * (wd - 1) + (d - 1) * h * (wd - 1) + (d - 1) * (h - 1) * wd,
                 d * h * wd, (d - 1) * (h - 1) * (wd - 1) + 1]
    k = 1
    for count, wc in zip(w[:4], worst):
        if count > 4096:
            k = max(k, -(-256 * int(count) // wc))
    return min(k, 255)


def test_workspace_shrinks_and_floor():
    full = fc.workspace_bytes([(96, 96, 96)], H)
    small = fc.workspace_bytes([(96, 96, 96)], H | fc.PH_LIST_FRACTION(1))
    assert small < full // 8                      # forest links remain: 8 B per voxel
    # lists at or below 4096 entries keep their worst case
    assert fc.workspace_bytes([(40, 40)], H | fc.PH_LIST_FRACTION(1)) == fc.workspace_bytes([(40, 40)], H)
    with pytest.raises(ValueError):
        fc.PH_LIST_FRACTION(256)


@pytest.mark.parametrize("filtration", ["V", "T"])
def test_fitting_lists_give_the_same_pairs(filtration):
    imgs = [S.grf((40, 38, 42), 2.0, 91), S.grf((300, 280), 3.0, 92), S.uniform((64, 64), 93),
            S.levels((1, 6000), 5, 94)]
    ref = batch(imgs, H, filtration).results()
    bt = batch(imgs, H | fc.PH_LIST_FRACTION(1), filtration)
    assert statuses(bt) == [fc.PH_OK] * len(imgs)
    for a, r, got in zip(imgs, ref, bt.results()):
        assert diff_pairs(got, r) is None, a.shape
        assert diff_pairs(got, oracle.diagram(a, filtration=filtration)) is None, a.shape


def test_backward_and_h1_with_fitting_lists():
    imgs = [S.grf((30, 28, 26), 2.0, 95), S.grf((120, 100), 3.0, 96)]
    flags = H | fc.PH_H1
    a = batch(imgs, flags)
    b = batch(imgs, flags | fc.PH_LIST_FRACTION(2))
    for x, y in zip(a.results(), b.results()):
        assert diff_pairs(x, y) is None
    for bt in (a, b):
        fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
        diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
        bt.ph_backward(-2.0 * diff, 2.0 * diff)
    assert torch.equal(a.grad, b.grad)


def test_overflow_reports_elists_and_true_sizes():
    """Noise keeps about a sixth of its edges: at 1/256 the lists of a 150 x 150 image and of a
    32^3 volume overflow (the smooth field beside them does not); the counters give the true
    sizes, and the fraction they imply fits."""
    imgs = [S.uniform((150, 150), 97), S.grf((50, 50), 2.0, 98), S.uniform((32, 32, 32), 99)]
    bt = batch(imgs, H | fc.PH_LIST_FRACTION(1))
    st = statuses(bt)
    assert st == [fc.PH_ELISTS, fc.PH_OK, fc.PH_ELISTS], st
    assert diff_pairs(bt.result(1), oracle.diagram(imgs[1])) is None
    wc = bt.work_counters()
    need = max(fraction_needed(a.shape, w) for a, w in zip(imgs, wc))
    assert need > 1
    ok = batch(imgs, H | fc.PH_LIST_FRACTION(need))
    assert statuses(ok) == [fc.PH_OK] * 3
    for a, got in zip(imgs, ok.results()):
        assert diff_pairs(got, oracle.diagram(a)) is None, a.shape
    # the counters of the failed call were the true sizes: the same as the successful call's
    assert (ok.work_counters()[:, :4] == wc[:, :4]).all()
