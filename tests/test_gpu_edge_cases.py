"""Edge cases on the GPU, each compared field by field with the oracle through the C ABI:
the union-find's sequential finish (a staircase row whose H0 merges each wait for the one
before, so the parallel rounds run out: the work counters must show edges finished
sequentially), long strips along every axis, an all-ties checkerboard, a constant image,
a 64x64 permutation, a thin volume with few levels, and IEEE special values; the same cases
batched together, and under the T-filtration.  Then noise large enough for the sorts' merge
passes and for every layout of the union-find."""
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


def staircase(n):
    """1 x (2n+1) row: minima decreasing to the right, saddles increasing to the right."""
    a = np.zeros(2 * n + 1, np.float32)
    a[0::2] = np.linspace(0.5, 0.1, n + 1).astype(np.float32)
    a[1::2] = np.linspace(1.0, 2.0, n).astype(np.float32)
    return a.reshape(1, -1)


def specials():
    s = np.array([[np.inf, -np.inf, -0.0, 0.0, 1e-45, -1e-45, 3.4e38, -3.4e38]] * 5, np.float32)
    s[2:] = s[2:, ::-1]
    return s


CASES = {
    "staircase": lambda: staircase(150),
    "staircase_mirror": lambda: staircase(150)[:, ::-1].copy(),
    "staircase_column": lambda: staircase(150).T.copy(),
    "staircase_volume_x": lambda: staircase(150).reshape(1, 1, -1),
    "staircase_volume_z": lambda: staircase(150).reshape(-1, 1, 1).copy(),
    "zeros": lambda: np.zeros((17, 23), np.float32),
    "checkerboard": lambda: (np.indices((33, 47)).sum(axis=0) % 2).astype(np.float32),
    "checkerboard_3d": lambda: (np.indices((9, 11, 10)).sum(axis=0) % 2).astype(np.float32),
    "strip_1x5000": lambda: S.levels((1, 5000), 7, 1),
    "strip_5000x1": lambda: S.levels((5000, 1), 7, 2),
    "strip_1x1x3000": lambda: S.levels((1, 1, 3000), 5, 3),
    "strip_3000x1x1": lambda: S.levels((3000, 1, 1), 5, 4),
    "strip_1x3000x1": lambda: S.levels((1, 3000, 1), 5, 6),
    "thin_2x2x700": lambda: S.levels((2, 2, 700), 3, 5),
    "specials": specials,
    "permutation_64": lambda: np.random.default_rng(5).permutation(64 * 64).reshape(64, 64).astype(np.float32),
}
SEQUENTIAL = {"staircase", "staircase_mirror", "staircase_column", "staircase_volume_x", "staircase_volume_z"}


def single(img, filtration="V"):
    print("case", img.shape, filtration, flush=True)
    return fc.ph_diagram(torch.from_numpy(np.ascontiguousarray(img)).to(DEV), filtration=filtration).numpy()


@pytest.mark.parametrize("name", sorted(CASES))
def test_edge_case_single(name):
    img = CASES[name]()
    assert diff_pairs(single(img), oracle.diagram(img)) is None, name


@pytest.mark.parametrize("name", sorted(SEQUENTIAL))
def test_sequential_finish_runs(name):
    """The staircases leave live edges after the parallel rounds: the work counters show
    edges finished by the sequential pass, and the result is still the oracle's."""
    img = CASES[name]()
    bt = fc.Batch([img.shape], device=DEV)
    bt.set_images([torch.from_numpy(img)])
    bt.ph_diagram_batch()
    (got,) = bt.results()
    assert diff_pairs(got, oracle.diagram(img)) is None
    wc = bt.work_counters()
    assert wc[0, 4] == 48 and wc[0, 6] > 0, wc[0]          # rounds at the limit, edges finished in order


def test_edge_cases_batched():
    """Every case in one batch: each instance bitwise the oracle's."""
    imgs = [CASES[k]() for k in sorted(CASES)]
    bt = fc.Batch([a.shape for a in imgs], device=DEV)
    bt.set_images([torch.from_numpy(np.ascontiguousarray(a)) for a in imgs])
    print("batch of", len(imgs), flush=True)
    bt.ph_diagram_batch()
    for name, a, got in zip(sorted(CASES), imgs, bt.results()):
        assert diff_pairs(got, oracle.diagram(a)) is None, name
    assert bt.work_counters()[:, 6].sum() > 0


@pytest.mark.parametrize("name", sorted(k for k in CASES if k != "specials"))
def test_edge_case_t_filtration(name):
    img = CASES[name]()
    assert diff_pairs(single(img, "T"), oracle.diagram(img, filtration="T")) is None, name


def test_specials_t_filtration_without_plus_inf():
    img = specials()
    img[np.isposinf(img)] = 3.0e38
    assert diff_pairs(single(img, "T"), oracle.diagram(img, filtration="T")) is None


# Lists past one LDS sort (4096 keys) and forests past the union-find's LDS capacities, from
# uniform noise (about a sixth of the edges kept): (KEEP edges, H0 nodes) of each, and which
# layout the union-find takes (par, moe and keys in LDS up to 5120 nodes; par and moe alone up
# to 20440; else the workspace, after six rounds over many workgroups when the instance has
# 2^20 voxels or more).
LARGE = {
    "noise_200x230": lambda: S.uniform((200, 230), 21),        # 14k edges, 9k nodes
    "noise_350x360": lambda: S.uniform((350, 360), 22),        # 39k edges, 25k nodes
    "noise_34x35x33": lambda: S.uniform((34, 35, 33), 23),     # 13k edges, 8k squares, 6k nodes
    "noise_1024x1024": lambda: S.uniform((1024, 1024), 25),    # 330k edges: 81 runs, 7 passes
    "noise_80x80x80": lambda: S.uniform((80, 80, 80), 26),     # long lists of all three kinds
    "noise_128x128x128": lambda: S.uniform((128, 128, 128), 27),   # 2^21 voxels
}
WIDE = {"noise_1024x1024", "noise_128x128x128"}   # 2^20 voxels or more: PH_WIDE applies


@pytest.mark.parametrize("name", sorted(LARGE))
def test_long_lists_and_large_forests(name):
    img = LARGE[name]()
    ref = oracle.diagram(img)
    for flags in ((fc.PH_H0 | fc.PH_HTOP, fc.PH_H0 | fc.PH_HTOP | fc.PH_WIDE) if name in WIDE else (fc.PH_H0 | fc.PH_HTOP,)):
        bt = fc.Batch([img.shape], flags=flags, device=DEV)
        bt.set_images([torch.from_numpy(img)])
        print("case", name, "flags", flags, flush=True)
        bt.ph_diagram_batch()
        (got,) = bt.results()
        assert diff_pairs(got, ref) is None, (name, flags)
        wc = bt.work_counters()
        assert wc[0, 0] > 4096 and wc[0, 2] > 5120, wc[0]
        if flags & fc.PH_WIDE:                      # both forests past one workgroup's LDS
            assert wc[0, 2] > 20440 and wc[0, 3] > 20440 and wc[0, 4] > 0 and wc[0, 5] > 0, wc[0]


def test_wide_rounds_beside_small_instances():
    """PH_WIDE on a batch whose largest instance takes the wide union-find rounds, with
    instances that stay in one workgroup (each kernel decides per instance), twice in a row on
    one batch, and the large image under the T-filtration."""
    imgs = [LARGE["noise_200x230"](), LARGE["noise_1024x1024"](), S.grf((40, 30, 20), 2.0, 91),
            LARGE["noise_34x35x33"]()]
    refs = [oracle.diagram(a) for a in imgs]
    bt = fc.Batch([a.shape for a in imgs], flags=fc.PH_H0 | fc.PH_HTOP | fc.PH_WIDE, device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    print("batch with a wide instance", flush=True)
    for _ in range(2):
        bt.ph_diagram_batch()
        for a, got, ref in zip(imgs, bt.results(), refs):
            assert diff_pairs(got, ref) is None, a.shape
    img = LARGE["noise_1024x1024"]()
    print("wide instance, T-filtration", flush=True)
    got = fc.ph_diagram(torch.from_numpy(img).to(DEV), flags=fc.PH_H0 | fc.PH_HTOP | fc.PH_WIDE, filtration="T").numpy()
    assert diff_pairs(got, oracle.diagram(img, filtration="T")) is None


def test_wide_with_uint8_backward_and_list_fraction():
    """PH_WIDE beside the other flags on 1024^2 noise quantised to 256 levels (heavy ties): uint8
    input, the backward scatter, and a list fraction, against the same calls without PH_WIDE
    (pairs, gradient, counters bitwise); a fraction too small for the lists gives PH_ELISTS
    with the true list sizes, as without the flag."""
    img = S.quantize_u8(LARGE["noise_1024x1024"]())
    base = fc.PH_H0 | fc.PH_HTOP | fc.PH_LIST_FRACTION(64)
    got = {}
    for flags in (base, base | fc.PH_WIDE):
        bt = fc.Batch([img.shape], flags=flags, device=DEV, dtype=torch.uint8)
        bt.set_images([torch.from_numpy(img)])
        print("uint8 noise, flags", flags, flush=True)
        bt.ph_diagram_batch()
        (res,) = bt.results()
        fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
        diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
        bt.ph_backward(-2.0 * diff, 2.0 * diff)
        got[flags] = (res, bt.grad.cpu().numpy().copy(), bt.work_counters()[0, :4].copy())
    (r0, g0, w0), (r1, g1, w1) = got[base], got[base | fc.PH_WIDE]
    assert diff_pairs(r1, r0) is None and diff_pairs(r0, oracle.diagram(img.astype(np.float32))) is None
    assert np.array_equal(g0, g1) and np.array_equal(w0, w1) and w0[2] > 20440, (w0, w1)
    for flags in (fc.PH_H0 | fc.PH_HTOP | fc.PH_LIST_FRACTION(8), fc.PH_H0 | fc.PH_HTOP | fc.PH_LIST_FRACTION(8) | fc.PH_WIDE):
        bt = fc.Batch([img.shape], flags=flags, device=DEV, dtype=torch.uint8)
        bt.set_images([torch.from_numpy(img)])
        print("uint8 noise, too small a fraction, flags", flags, flush=True)
        bt.ph_diagram_batch()
        torch.cuda.synchronize()
        assert int(bt.status[0]) == fc.PH_ELISTS
        assert np.array_equal(bt.work_counters()[0, :4], w0), bt.work_counters()[0, :4]


def test_long_lists_batched_and_t_filtration():
    """The large cases side by side in one batch (each list with its own merge scratch), and
    two of them under the T-filtration."""
    imgs = [LARGE[k]() for k in ("noise_200x230", "noise_350x360", "noise_34x35x33")]
    bt = fc.Batch([a.shape for a in imgs], device=DEV)
    bt.set_images([torch.from_numpy(a) for a in imgs])
    print("batch of large cases", flush=True)
    bt.ph_diagram_batch()
    for a, got in zip(imgs, bt.results()):
        assert diff_pairs(got, oracle.diagram(a)) is None, a.shape
    for k in ("noise_350x360", "noise_34x35x33"):
        img = LARGE[k]()
        assert diff_pairs(single(img, "T"), oracle.diagram(img, filtration="T")) is None, k
