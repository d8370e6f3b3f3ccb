"""ph_diagram_noalloc (the entry point for callers that cannot allocate) through the C ABI:
its pairs, counts and status equal ph_diagram's bitwise on two calls in a row on one device,
the second on a smaller instance (so a stale first call in the library's workspace would
show), under both filtrations; an instance beyond the workspace is refused on the host."""
import numpy as np
import pytest

import synthetic as S
from gpu_util import diff_pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2606_04801_amd as fc  # noqa: E402

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
DEV = torch.device("cuda:0")


def noalloc(img, filtration="V"):
    t = torch.from_numpy(np.ascontiguousarray(img)).to(DEV)
    cap = fc.capacity_bound(img.shape, filtration)
    bufs = fc.PairBuffers(cap, DEV)
    count = torch.full((1,), -7, dtype=torch.int64, device=DEV)
    status = torch.full((1,), 99, dtype=torch.int32, device=DEV)
    print("noalloc", img.shape, filtration, flush=True)
    rc = fc.ph_diagram_noalloc(t, bufs, count, status, filtration=filtration)
    assert rc == fc.PH_OK
    torch.cuda.synchronize()
    assert int(status.item()) == fc.PH_OK
    return bufs.to_numpy(0, int(count.item()))


def reference(img, filtration="V"):
    return fc.ph_diagram(torch.from_numpy(np.ascontiguousarray(img)).to(DEV), filtration=filtration).numpy()


def test_noalloc_equals_ph_diagram_twice_shrinking():
    torch.zeros(1, device=DEV)
    assert fc.lib().ph_init_device() == fc.PH_OK
    for filtration in ("V", "T"):
        first = S.grf((40, 44, 36), 2.0, 11)               # a volume, then a smaller image
        second = S.grf((50, 61), 2.5, 12)
        a = noalloc(first, filtration)
        b = noalloc(second, filtration)
        assert len(a) > 1 and len(b) > 1
        assert diff_pairs(a, reference(first, filtration)) is None
        assert diff_pairs(b, reference(second, filtration)) is None
        # and the smaller instance once more right after a larger one of its own kind
        third = S.levels((20, 23), 3, 13)
        assert diff_pairs(noalloc(third, filtration), reference(third, filtration)) is None


def test_noalloc_refuses_beyond_workspace():
    assert fc.lib().ph_init_device() == fc.PH_OK
    shape = (1024, 1024)
    need = fc.workspace_bytes([shape])
    assert need > (64 << 20)
    t = torch.zeros(shape, dtype=torch.float32, device=DEV)
    bufs = fc.PairBuffers(1, DEV)
    count = torch.zeros(1, dtype=torch.int64, device=DEV)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    assert fc.ph_diagram_noalloc(t, bufs, count, status, capacity=1) == fc.PH_ENOMEM
