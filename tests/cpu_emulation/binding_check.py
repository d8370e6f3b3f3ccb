"""Drive the Python binding's Batch class end to end on the CPU against the host build of the
library's C ABI (tests/cpu_emulation, variant "so"): marshalling of shapes, offsets, pair and
gradient buffers, autotuning, work counters and profiling, checked against the oracle.

    python binding_check.py path/to/libflashcubical_emulated.so
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TESTS = os.path.dirname(HERE)
ROOT = os.path.dirname(TESTS)
sys.path[:0] = [ROOT, TESTS]

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
import paper_2606_04801_amd as fc  # noqa: E402
import synthetic as S  # noqa: E402
from gpu_util import diff_pairs  # noqa: E402


def main(so):
    fc.LIB_PATH = so
    imgs = [S.grf((40, 33), 2.0, 1), S.levels((4, 3, 5), 2, 2), S.levels((1, 9), 3, 3), S.grf((9, 12, 10), 1.5, 4),
            S.uniform((24, 30), 5)]
    bt = fc.Batch([a.shape for a in imgs], device="cpu")
    bt.set_images([torch.from_numpy(a) for a in imgs])
    best = bt.ph_autotune(reps=1)
    assert all(0 <= t <= 2 for t in best), best
    fc.profile(True)
    bt.ph_diagram_batch()
    prof = fc.profile_read()
    fc.profile(False)
    assert "k_classify2d" in prof and "k_classify3d" in prof and "k_output" in prof, prof
    res = bt.results()
    refs = [oracle.diagram(a) for a in imgs]
    for a, r, ref in zip(imgs, res, refs):
        assert diff_pairs(r, ref) is None, a.shape
    wc = bt.work_counters()
    assert wc.shape == (len(imgs), 16) and (wc[:, 7] == 0).all() and (wc[:, 2] >= 1).all(), wc
    assert (wc[:, 14] >= 2 * wc[:, 0]).all(), wc     # each KEEP edge reads the forest at both endpoints
    fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
    assert int(bt.valid_mask().sum()) == sum(len(r) for r in refs)
    diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
    bt.ph_backward((-2.0 * diff).contiguous(), (2.0 * diff).contiguous())
    for i, (a, ref) in enumerate(zip(imgs, refs)):
        f = ref["death_cell"] >= 0
        d = np.where(f, ref["death"] - ref["birth"], 0).astype(np.float32)
        g = oracle.gradient(ref, -2 * d, 2 * d, a.shape).reshape(-1)
        got = bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]].numpy()
        np.testing.assert_allclose(got, g, rtol=1e-6, atol=1e-7)
    # an explicit tuning gives the same pairs
    bt2 = fc.Batch([a.shape for a in imgs], tuning=(2, 1), device="cpu")
    bt2.set_images([torch.from_numpy(a) for a in imgs])
    bt2.ph_diagram_batch()
    for r, ref in zip(bt2.results(), refs):
        assert diff_pairs(r, ref) is None
    # autograd: PHDiagramFn forward + backward against finite differences of the oracle's loss
    Fn = fc.PHDiagramFn
    for k in range(2):
        x0 = S.tie_free((16, 16), 4000 + k).astype(np.float64)
        x = torch.tensor(x0, dtype=torch.float32, requires_grad=True)
        b, d, dim = Fn.apply(x)
        ref = oracle.diagram(x0.astype(np.float32))
        assert torch.equal(b, torch.from_numpy(ref["birth"].copy()))
        fin = torch.isfinite(d)
        ((d - b)[fin] ** 2).sum().backward()
        g = x.grad.numpy().reshape(-1)

        def loss(v):
            p = oracle.diagram(v.astype(np.float32))
            f = p["death_cell"] >= 0
            return float(((p["death"][f].astype(np.float64) - p["birth"][f]) ** 2).sum())

        h = 1e-4
        for j in np.random.default_rng(k).choice(256, size=20, replace=False):
            xp, xm = x0.reshape(-1).copy(), x0.reshape(-1).copy()
            xp[j] += h
            xm[j] -= h
            step = float(np.float32(xp[j])) - float(np.float32(xm[j]))
            fd = (loss(xp.reshape(16, 16)) - loss(xm.reshape(16, 16))) / step
            assert abs(fd - g[j]) <= 1e-3 * max(1.0, abs(fd)), (k, j, fd, g[j])
    print("binding ok")


if __name__ == "__main__":
    main(sys.argv[1])
