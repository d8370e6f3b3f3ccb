"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import synthetic as S
import fixtures
from gpu_util import diff_pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2606_04801_amd as fc  # noqa: E402
from gpu_util import device_for_tests  # noqa: E402

DEV, HOST_MODE = device_for_tests(fc, torch)
if DEV is None:
    pytest.skip("no GPU", allow_module_level=True)

def gpu_diagram(img, **kw):
    print("case", img.shape, flush=True)
    return fc.ph_diagram(torch.from_numpy(np.ascontiguousarray(img)).to(DEV), **kw).numpy()


def check(img, label=""):
    got = gpu_diagram(img)
    ref = oracle.diagram(img)
    msg = diff_pairs(got, ref)
    assert msg is None, "%s %s: %s" % (label, img.shape, msg)


def test_library_is_native():
    if HOST_MODE:
        pytest.skip("host build of the C ABI")
    assert fc.lib()._name.endswith("libflashcubical.so")
    assert fc.lut_config_count(3) == 15935


def test_kernels_fit_device():
    """Every kernel's static LDS and block size fit the device (no kernel is launched)."""
    torch.zeros(1, device=DEV)
    rc, text = fc.device_report()
    print(text, flush=True)
    assert rc == fc.PH_OK, text


def test_tables_uploaded():
    """The lookup tables on the device equal the host tables (copy, read back, compare)."""
    assert fc.lib().ph_init_device() == fc.PH_OK


@pytest.mark.parametrize("name,img,expected,case", fixtures.load(), ids=lambda x: x if isinstance(x, str) else "")
def test_fixtures(name, img, expected, case):
    check(img, name)


def test_tiny_sweep_2d():
    rng = np.random.default_rng(1)
    for k in range(150):
        shape = tuple(int(x) for x in rng.integers(1, 10, size=2))
        lev = int(rng.choice([2, 3, 5, 1 << 20]))
        check(S.levels(shape, lev, 10_000 + k), "2d#%d" % k)


def test_tiny_sweep_3d():
    rng = np.random.default_rng(2)
    for k in range(120):
        shape = tuple(int(x) for x in rng.integers(1, 7, size=3))
        lev = int(rng.choice([2, 3, 5, 1 << 20]))
        check(S.levels(shape, lev, 20_000 + k), "3d#%d" % k)


def test_special_values():
    a = np.array([[0.0, -0.0, 1.0, np.inf], [-np.inf, 0.5, -0.0, 0.0], [1e-45, -1e-45, 3.0, 0.0]], np.float32)
    check(a, "specials")
    v = np.tile(a[:, :3], (2, 1, 1)).astype(np.float32)
    check(v, "specials3d")


def test_uniform_128():
    check(S.uniform((128, 128), 0), "uniform128")


@pytest.mark.parametrize("shape,sigma", [((200, 300), 2.0), ((257, 131), 4.0), ((70, 1030), 1.0)])
def test_fields_2d(shape, sigma):
    x = S.grf(shape, sigma, 5)
    check(x, "grf")
    check(S.quantize_u8(x), "u8")


@pytest.mark.parametrize("shape,sigma", [((40, 35, 50), 1.5), ((17, 64, 33), 2.0), ((1, 40, 41), 1.0)])
def test_fields_3d(shape, sigma):
    x = S.grf(shape, sigma, 6)
    check(x, "grf3")
    check(S.quantize_u8(x), "u8-3")


def test_uniform_3d():
    check(S.uniform((24, 30, 28), 9), "uniform3d")
