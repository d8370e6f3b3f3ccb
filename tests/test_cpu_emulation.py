"""The library's kernels run on the CPU against the oracle, under AddressSanitizer and UBSan.

tests/cpu_emulation compiles csrc/fc_kernels.hip as host C++ against an emulated HIP runtime
(one fiber per GPU thread, cooperative barriers and wave exchanges; see its header) with a
redzone around every LDS array and poisoned gaps after the workspace arrays.  This
checks the kernels' indexing and synchronisation, and their results bit for bit, without a GPU.
It is not a parity claim for the GPU build (compiler and hardware differ) and nothing in the
library uses it.
"""
import os
import shutil
import struct
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import fixtures
import oracle
import synthetic as S
from gpu_util import diff_pairs

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "cpu_emulation"))
import build as emu_build  # noqa: E402

pytestmark = pytest.mark.slow
if shutil.which("g++") is None:
    pytest.skip("no host C++ compiler", allow_module_level=True)

REC = np.dtype([("dim", "<i4"), ("birth", "<f4"), ("death", "<f4"), ("birth_cell", "<i8"),
                ("death_cell", "<i8"), ("birth_vertex", "<i4"), ("death_vertex", "<i4")])


@pytest.fixture(scope="module")
def driver():
    return emu_build.build("asan")


def run(exe, imgs, mode=0, tuning=None, backward=False, capacity=-1, with_count=False, flags=3):
    """(per-instance (pairs, status), gradient or None) from the emulated kernels.  With
    with_count, each instance gives (pairs, status, count) instead."""
    imgs = [np.ascontiguousarray(a, dtype=np.float32) for a in imgs]
    hdr = struct.pack("<7i", len(imgs), flags, mode, *(tuning if tuning else (-1, -1)), int(backward), capacity)
    for a in imgs:
        ext = list(a.shape) + [1] * (3 - a.ndim)
        hdr += struct.pack("<4i", a.ndim, *ext)
    with tempfile.TemporaryDirectory() as d:
        fi, fo = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        with open(fi, "wb") as f:
            f.write(hdr)
            for a in imgs:
                f.write(a.tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
        r = subprocess.run([exe, fi, fo], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stderr[-4000:]
        raw = open(fo, "rb").read()
    out, pos = [], 0
    for a in imgs:
        cnt, st = struct.unpack_from("<qi", raw, pos)
        pos += 12
        m = cnt if st == 0 else (min(cnt, capacity) if st == -3 and capacity >= 0 else 0)
        rec = np.frombuffer(raw, REC, count=m, offset=pos)
        pos += m * REC.itemsize
        res = np.zeros(m, oracle.PAIR_DTYPE)
        for f in oracle.PAIR_DTYPE.names:
            res[f] = rec[f]
        out.append((res, st, cnt) if with_count else (res, st))
    grad = None
    if backward:
        grad = np.frombuffer(raw, "<f4", offset=pos)
    return out, grad


def test_fixtures(driver):
    for name, img, _, _ in fixtures.load():
        (got, st), = run(driver, [img])[0]
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, name


def test_tiny_sweep(driver):
    rng = np.random.default_rng(31)
    for k in range(10):
        nd = 2 if k % 2 == 0 else 3
        shape = tuple(int(x) for x in rng.integers(1, 10 if nd == 2 else 6, size=nd))
        img = S.levels(shape, int(rng.choice([2, 3, 1 << 20])), 7000 + k)
        (got, st), = run(driver, [img])[0]
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, (k, shape)


def test_fields_multi_tile(driver):
    for img in (S.grf((48, 40), 2.0, 7), S.grf((12, 10, 14), 1.5, 8), S.quantize_u8(S.grf((70, 130), 3.0, 2))):
        (got, st), = run(driver, [img])[0]
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape


def mixed_batch():
    return [S.levels((5, 9), 3, 7100), S.grf((40, 33), 2.0, 7101), S.levels((4, 3, 5), 2, 7102),
            S.grf((9, 12, 10), 1.5, 7103), S.levels((1, 7), 5, 7104), S.uniform((20, 21), 7105)]


@pytest.mark.parametrize("tuning, fused", [(None, 0), ((1, 2), 0), ((2, 1), 0), (None, 1), ((2, 1), 1)])
def test_batch_with_backward(driver, tuning, fused):
    """ph_backward after ph_diagram_batch, or (fused) ph_backward_scatter after
    ph_diagram_batch_grad cleared a gradient full of NaNs: the oracle's gradient."""
    imgs = mixed_batch()
    out, grad = run(driver, imgs, mode=1, tuning=tuning, backward=2 if fused else True)
    off = 0
    for img, (got, st) in zip(imgs, out):
        ref = oracle.diagram(img)
        assert st == 0 and diff_pairs(got, ref) is None, img.shape
        f = ref["death_cell"] >= 0
        d = np.where(f, ref["death"] - ref["birth"], 0).astype(np.float32)
        g = oracle.gradient(ref, -2 * d, 2 * d, img.shape).reshape(-1)
        np.testing.assert_allclose(grad[off:off + img.size], g, rtol=1e-6, atol=1e-7)
        off += img.size


@pytest.mark.parametrize("variant", ["asan", "poison"])
def test_t_filtration_fused_gradient(variant):
    """Under the T-filtration (PH_TFILT) the classify passes clear the caller's pixels through
    the reflection of the framed grid: ph_diagram_batch_grad then ph_backward_scatter, on a
    gradient full of NaNs, under AddressSanitizer and on a garbage workspace, give the oracle's
    T pairs and gradient."""
    exe = emu_build.build(variant)
    imgs = mixed_batch()
    out, grad = run(exe, imgs, mode=1, flags=3 | 16, backward=2)
    off = 0
    for img, (got, st) in zip(imgs, out):
        ref = oracle.diagram(img, filtration="T")
        assert st == 0 and diff_pairs(got, ref) is None, img.shape
        f = ref["death_cell"] >= 0
        d = np.where(f, ref["death"] - ref["birth"], 0).astype(np.float32)
        g = oracle.gradient(ref, -2 * d, 2 * d, img.shape).reshape(-1)
        np.testing.assert_allclose(grad[off:off + img.size], g, rtol=1e-6, atol=1e-7)
        off += img.size


def test_autotune_then_batch(driver):
    imgs = mixed_batch()[:4]
    out, _ = run(driver, imgs, mode=2)
    for img, (got, st) in zip(imgs, out):
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None


def test_nan_status(driver):
    img = S.grf((20, 20), 2.0, 3)
    img[4, 5] = np.nan
    (got, st), = run(driver, [img])[0]
    assert st == -2                                   # PH_ENAN


@pytest.mark.skipif(os.environ.get("FC_EMULATE_FULL") != "1",
                    reason="about 9 minutes: set FC_EMULATE_FULL=1 to run every full-size workload")
def test_full_size_workloads_against_digests():
    """Every instance of the full-size workloads (2048^2 with and without ties, 256^3, the
    512-image batch, the 128-instance mixed batch) through the emulated kernels, compared with
    the oracle's stored digests."""
    import json
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    from make_digests import instances, make, pair_digest
    exe = emu_build.build("poison")
    D = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.json")))
    its = instances()
    for cfg in ("c1", "c2", "c2u8", "c3"):
        (c, idx, kind, args), = [it for it in its if it[0] == cfg]
        (got, st), = run(exe, [make(kind, args)])[0]
        assert st == 0 and pair_digest(got) == D[c][str(idx)]["pairs_sha256"], cfg
    for cfg, chunk in (("c4", 128), ("c5", 32)):
        items = [it for it in its if it[0] == cfg]
        for k in range(0, len(items), chunk):
            part = items[k:k + chunk]
            out, _ = run(exe, [make(kind, args) for _, _, kind, args in part], mode=1)
            for (c, idx, _, _), (got, st) in zip(part, out):
                assert st == 0 and pair_digest(got) == D[c][str(idx)]["pairs_sha256"], (c, idx)


def staircase(n):
    """1 x (2n+1) row: minima decreasing to the right, saddles increasing.  Every H0 merge waits
    for the previous one, so the parallel rounds run out and the sequential finish is used."""
    a = np.zeros(2 * n + 1, np.float32)
    a[0::2] = np.linspace(0.5, 0.1, n + 1).astype(np.float32)
    a[1::2] = np.linspace(1.0, 2.0, n).astype(np.float32)
    return a.reshape(1, -1)


def test_edge_cases(driver):
    rng = np.random.default_rng(5)
    cb = (np.indices((33, 47)).sum(axis=0) % 2).astype(np.float32)          # checkerboard, all ties
    specials = np.array([[np.inf, -np.inf, -0.0, 0.0, 1e-45, -1e-45, 3.4e38, -3.4e38]] * 5, np.float32)
    specials[2:] = specials[2:, ::-1]
    cases = [staircase(150), staircase(150)[:, ::-1].copy(), np.zeros((17, 23), np.float32), cb,
             S.levels((1, 5000), 7, 1), S.levels((5000, 1), 7, 2), S.levels((1, 1, 3000), 5, 3),
             S.levels((3000, 1, 1), 5, 4), S.levels((2, 2, 700), 3, 5), specials,
             rng.permutation(64 * 64).reshape(64, 64).astype(np.float32)]
    for img in cases:
        (got, st), = run(driver, [img])[0]
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape


def test_long_lists_and_large_forests(driver):
    """Lists past one LDS sort (4096 keys) through several merge passes with ragged runs, and
    union-finds past the LDS node capacities: uniform noise keeps about a sixth of the edges.
    200 x 230: ~15k KEEP edges (4 runs), ~9k H0 nodes (par, moe in LDS, keys and live edges in
    the workspace); 350 x 360: ~40k edges (10 runs, 4 passes), ~26k nodes (all in the
    workspace); a 26 x 27 x 25 volume: long KEEP-square and node lists side by side."""
    for img in (S.uniform((200, 230), 21), S.uniform((350, 360), 22), S.uniform((34, 35, 33), 23)):
        (got, st), = run(driver, [img])[0]
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape


@pytest.mark.parametrize("seed", [3, 4])
def test_long_lists_random_interleavings(driver, monkeypatch, seed):
    """The merge passes and the union-find with LDS nodes under random thread interleavings,
    side by side in one batch."""
    monkeypatch.setenv("EMU_SHUFFLE", str(seed))
    imgs = [S.uniform((200, 230), 21), S.uniform((34, 35, 33), 23)]
    out, _ = run(driver, imgs, mode=1)
    for img, (got, st) in zip(imgs, out):
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape


def test_long_lists_touch_device_memory_only():
    """Every access of the merge passes (each list with its own scratch) and of the large
    union-finds lands in a device allocation or LDS (trace build)."""
    exe = emu_build.build("trace")
    imgs = [S.uniform((200, 230), 21), S.uniform((34, 35, 33), 23)]
    out, _ = run(exe, imgs, mode=1)
    for img, (got, st) in zip(imgs, out):
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape


def test_capacity_overflow_keeps_true_count(driver):
    img = S.uniform((40, 40), 9)
    ref = oracle.diagram(img)
    (got, st, cnt), = run(driver, [img], capacity=25, with_count=True)[0]
    assert st == -3 and cnt == len(ref)                                     # PH_ECAPACITY
    assert diff_pairs(got, ref[:25]) is None


def test_binding_batch_end_to_end():
    """The Python binding's Batch (offsets, buffers, autotune, counters, profiling, backward)
    against the host build of the C ABI, in a separate process."""
    so = emu_build.build("so")
    script = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cpu_emulation", "binding_check.py")
    r = subprocess.run([sys.executable, script, so], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "binding ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]


@pytest.mark.parametrize("seed", [1, 2])
def test_random_interleavings(driver, monkeypatch, seed):
    """Threads resumed in random order, with turns given up at atomics: the results must not
    depend on the interleaving between barriers."""
    monkeypatch.setenv("EMU_SHUFFLE", str(seed))
    imgs = mixed_batch() + [staircase(60), S.uniform((48, 48), 11)]
    out, grad = run(driver, imgs, mode=1, backward=True)
    off = 0
    for img, (got, st) in zip(imgs, out):
        ref = oracle.diagram(img)
        assert st == 0 and diff_pairs(got, ref) is None, img.shape
        f = ref["death_cell"] >= 0
        d = np.where(f, ref["death"] - ref["birth"], 0).astype(np.float32)
        g = oracle.gradient(ref, -2 * d, 2 * d, img.shape).reshape(-1)
        np.testing.assert_allclose(grad[off:off + img.size], g, rtol=1e-6, atol=1e-7)
        off += img.size


def test_bench_flow_against_host_library():
    """bench.py's measuring path (sizing pass, batched and per-image forms, parity with each
    other and with the oracle, profiling, counters, JSON line) run on the CPU against the host
    build of the C ABI, on a reduced workload."""
    import json
    so = emu_build.build("so")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ)
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--host-library", so, "--steps", "1",
                        "--warmup", "1", "--cpu-workers", "2"], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["value"] > 0 and line["roofline"]["kernel"].startswith("k_")
    assert set(line["forms"]) == {"batched_fwd_bwd", "batched_fwd_bwd_manual", "batched_fwd", "per_image_fwd_bwd",
                                  "batched_fwd_bwd_list_fraction", "per_image_fwd_bwd_graph",
                                  "batched_fwd_bwd_u8", "batched_fwd_bwd_tfilt", "batched_fwd_h1", "c1_single",
                                  "c2_single", "c2u8_single", "c3_single", "c4_batch",
                                  "noise_20x20", "noise_40x44", "noise_10x11x12"}
    assert line["parity"]["autograd_eq_manual"] and line["forms"]["batched_fwd_h1"]["h1_columns"] > 0
    assert all(k["bytes"] > 0 for n, k in line["kernels"].items() if n not in ("k_plan",))
    assert line["cpu_baseline"]["kind"] == "oracle" and line["work"]["pairs"] > 0


def test_random_shapes_and_ties_hypothesis(driver):
    """Random extents (1..12 per axis, 2D and 3D), value counts (2 levels to all distinct),
    +-0 and infinities, in batches of 16 through the emulated kernels against the oracle."""
    hyp = pytest.importorskip("hypothesis")
    from hypothesis import strategies as st

    @hyp.settings(max_examples=12, deadline=None, derandomize=True)
    @hyp.given(st.lists(st.tuples(st.lists(st.integers(1, 12), min_size=2, max_size=3),
                                  st.sampled_from([2, 3, 7, 1 << 20]), st.integers(0, 2 ** 31 - 1),
                                  st.booleans()), min_size=1, max_size=16))
    def check(spec):
        imgs = []
        for shape, lev, seed, specials in spec:
            a = S.levels(tuple(shape), lev, seed)
            if specials and a.size > 2:
                r = np.random.default_rng(seed)
                flat = a.reshape(-1)
                flat[r.integers(0, a.size, 2)] = np.array([-0.0, np.inf], np.float32)
            imgs.append(a)
        out, _ = run(driver, imgs, mode=1)
        for a, (got, status) in zip(imgs, out):
            assert status == 0 and diff_pairs(got, oracle.diagram(a)) is None, a.shape

    check()


def test_gpu_suites_against_host_library():
    """The GPU test modules themselves, run against the host build of the C ABI on host tensors
    (graph capture and the full-size workloads excepted), in a separate process."""
    so = emu_build.build("so")
    tests = os.path.dirname(os.path.abspath(__file__))
    env = dict(os.environ, FC_TEST_HOST_LIBRARY=so)
    env.pop("FC_EMULATE_FULL", None)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "gpu", "-p", "no:cacheprovider",
                        os.path.join(tests, "test_gpu_parity.py"), os.path.join(tests, "test_gpu_full.py"),
                        os.path.join(tests, "test_gpu_tfilt.py"), os.path.join(tests, "test_gpu_lists.py")],
                       capture_output=True, text=True, timeout=1200, env=env, cwd=os.path.dirname(tests))
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert " passed" in r.stdout and " failed" not in r.stdout


def test_smoke_diagram_checks_against_host_library():
    """The diagram half of __graft_entry__.smoke() on host tensors against the host build."""
    so = emu_build.build("so")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, torch; sys.path.insert(0, %r); import paper_2606_04801_amd as fc; "
            "fc.LIB_PATH = %r; import __graft_entry__ as g; g.diagram_checks(torch.device('cpu')); "
            "print('checks ok')" % (root, so))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600,
                       cwd=root)
    assert r.returncode == 0 and "checks ok" in r.stdout, r.stdout[-2000:] + r.stderr[-3000:]


@pytest.mark.parametrize("lockstep", ["0", "1"])
def test_kernels_touch_device_memory_only(monkeypatch, lockstep):
    """Every load, store and struct copy of kernel code lands in a device allocation, LDS or the
    thread's own private memory (trace build); with EMU_LOCKSTEP=1 the threads of a block also
    advance one memory access at a time."""
    exe = emu_build.build("trace")
    monkeypatch.setenv("EMU_LOCKSTEP", lockstep)
    for name, img, _, _ in fixtures.load():
        (got, st), = run(exe, [img])[0]
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, name
    imgs = mixed_batch()
    out, grad = run(exe, imgs, mode=1, tuning=(2, 1), backward=True)
    for img, (got, st) in zip(imgs, out):
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape


def h1_batch():
    rng = np.random.default_rng(21)
    imgs = [S.grf((14, 15, 13), 2.0, 7201), S.levels((6, 7, 5), 3, 7202), S.uniform((9, 10, 8), 7203),
            S.grf((30, 28), 2.0, 7204), S.levels((1, 9, 8), 2, 7205)]
    for k in range(4):
        shape = tuple(int(x) for x in rng.integers(1, 7, size=3))
        imgs.append(S.levels(shape, int(rng.choice([2, 3, 1 << 20])), 7210 + k))
    return imgs


def h1_ref(a):
    return oracle.diagram(a, dims=(0, 1, 2) if a.ndim == 3 else (0, 1))


@pytest.mark.parametrize("variant", ["asan", "poison"])
def test_h1_batch(variant):
    """3D H1 (PH_H1) in a mixed batch through the emulated kernels, under AddressSanitizer
    and on a workspace filled with garbage, against the oracle's every dimension."""
    exe = emu_build.build(variant)
    imgs = h1_batch()
    out, _ = run(exe, imgs, mode=1, flags=3 | 32)
    for img, (got, st) in zip(imgs, out):
        assert st == 0 and diff_pairs(got, h1_ref(img)) is None, img.shape


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_h1_random_interleavings(monkeypatch, seed):
    """The H1 column kernels (LDS table and queue shared by the 64 threads, claims by atomics)
    with the threads resumed in random order and turns given up at every atomic."""
    exe = emu_build.build("poison")
    monkeypatch.setenv("EMU_SHUFFLE", str(seed))
    imgs = h1_batch()
    out, _ = run(exe, imgs, mode=1, flags=3 | 32)
    for img, (got, st) in zip(imgs, out):
        assert st == 0 and diff_pairs(got, h1_ref(img)) is None, img.shape


def test_h1_touches_device_memory_only():
    """Every access of the H1 kernels lands in device memory, LDS or private memory."""
    exe = emu_build.build("trace")
    imgs = h1_batch()[:4]
    out, _ = run(exe, imgs, mode=1, flags=3 | 32)
    for img, (got, st) in zip(imgs, out):
        assert st == 0 and diff_pairs(got, h1_ref(img)) is None, img.shape


def test_wide_union_find_rounds():
    """PH_WIDE on an image of 2^20 pixels of uniform noise (about 160k H0 nodes and as many
    dual ones) beside a small image: both union-finds of the large one take the rounds spread
    over many workgroups, then finish in one.  Built without the sanitizers (the instance is
    large), against the oracle."""
    exe = emu_build.build("poison")
    imgs = [S.uniform((1024, 1024), 25), S.uniform((20, 21), 26)]
    for img, (got, st) in zip(imgs, run(exe, imgs, mode=1, flags=3 | 64)[0]):
        assert st == 0 and diff_pairs(got, oracle.diagram(img)) is None, img.shape
