"""Benchmark: Mvoxels/s to H0 + H_top diagrams, batched forward + backward versus per-image
plain calls, on one MI355X; prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--traffic-json F]

Workload: 64 volumes 96^3 (random field, sigma 3, seeds 2000+i) and 64 images 512^2 (sigma 6,
seeds 3000+i) in one batch; loss = sum over finite pairs of (death - birth)^2, so the backward
scatters -2(d-b) to each birth pixel and +2(d-b) to each death pixel.  A step is one pass of
the whole path over the batch: forward (ph_diagram_batch), loss gradient, backward
(ph_backward).  The batched step is captured once in a HIP graph and replayed; the per-image
form is a plain loop of ph_diagram + ph_backward calls per instance on one stream; the forward
alone is timed as well.  Pair capacities come from a sizing pass on the same inputs, and timed
steps alternate between two copies of inputs and buffers.  All forms are compared bit for bit
before any timing.

roofline: the dominant kernel of the batched step (largest event-timed total over the timed
profiled steps), its algorithmic bytes per launch divided by its mean launch duration, against
8 TB/s.  traffic: HBM bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE, read from
profiles/hbm_traffic.json (or --traffic-json) only when it was taken on the library build that
is loaded (its sha256 is recorded), else null (see --profile-steps and --traffic-from).

cpu_baseline: the CPU oracle (single-threaded C, one process per host core, at most 16) on a
bounded sample of the same workload (one instance per core, half volumes and half images,
forward + reference gradient, about 30 s), in Mvoxels/s.  The GPU results of those instances
are also compared with the oracle's, bit for bit.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthetic as S  # noqa: E402

METRIC = "Mvoxels/s to H0+H_top diagrams, batched fwd+bwd vs per-image, bit-exact"
HBM_PEAK_GBS = 8000.0
N3, N2 = 64, 64
SHAPE3, SIG3, SHAPE2, SIG2 = (96, 96, 96), 3.0, (512, 512), 6.0


def use_small_workload():
    """A reduced workload of the same kind, for checking this script against the host build of
    the library (--host-library); never used for a reported number."""
    global N3, N2, SHAPE3, SHAPE2
    N3, N2, SHAPE3, SHAPE2 = 3, 3, (20, 18, 22), (64, 70)


def workload_shapes():
    return [SHAPE3] * N3 + [SHAPE2] * N2


def workload_desc():
    return "%d x %s field sigma 3 + %d x %s field sigma 6, H0+H_top, batched fwd+bwd" % (
        N3, "x".join(map(str, SHAPE3)), N2, "x".join(map(str, SHAPE2)))


def _oracle_instance(item):
    """One workload instance through the oracle: forward + reference gradient, timed."""
    import oracle
    idx, shape, sig, seed = item
    img = S.grf(shape, sig, seed)
    t0 = time.perf_counter()
    p = oracle.diagram(img)
    fin = p["death_cell"] >= 0
    d = np.where(fin, p["death"] - p["birth"], 0).astype(np.float32)
    g = oracle.gradient(p, -2 * d, 2 * d, img.shape)
    return idx, img.size, time.perf_counter() - t0, p, g


def cpu_baseline(workers: int):
    """The oracle on a bounded sample of the workload, one instance per host core.

    The sample is `workers` instances, half volumes and half images (first seeds of each),
    each run single-threaded in its own process; the rate is sample voxels over wall time.
    Returns the baseline record and {batch index: (pairs, gradient)} for the parity check."""
    from multiprocessing import get_context
    n3 = min((workers + 1) // 2, N3)
    n2 = min(workers - n3, N2)
    items = [(i, SHAPE3, SIG3, 2000 + i) for i in range(n3)] + \
            [(N3 + i, SHAPE2, SIG2, 3000 + i) for i in range(n2)]
    t0 = time.perf_counter()
    with get_context("spawn").Pool(workers) as pool:     # fresh processes: no HIP state is forked
        res = pool.map(_oracle_instance, items, chunksize=1)
    wall = time.perf_counter() - t0
    vox = sum(r[1] for r in res)
    ref = {r[0]: (r[3], r[4]) for r in res}
    rec = {"value": round(vox / wall / 1e6, 5), "unit": "Mvoxels/s", "cores": min(workers, len(items)),
           "kind": "oracle",
           "sample": "%d x %s volumes (seeds 2000..) + %d x %s images (seeds 3000..) of the workload, "
                     "forward + gradient, one single-threaded C process per core, %.1f s wall "
                     "(single-process sum %.1f s)" % (n3, "x".join(map(str, SHAPE3)), n2,
                                                     "x".join(map(str, SHAPE2)), wall, sum(r[2] for r in res))}
    return rec, ref


def algorithmic_bytes(name, wc, npairs, shapes):
    """Bytes one launch of `name` must move over the whole batch: the unavoidable reads and
    writes of its inputs and outputs (pixels, forest arrays, list keys, pairs), no re-reads.

    wc: per-instance work counters (KEEP edges, KEEP squares, H0 nodes, dual nodes, ...)."""
    is3 = np.array([len(s) == 3 for s in shapes])
    N = sum(int(np.prod(s)) for s in shapes)
    T = sum(int(np.prod([e - 1 for e in s])) for s in shapes)
    ke, kf, m0, mt = (int(wc[:, k].sum()) for k in range(4))
    facets = int(wc[~is3, 0].sum()) + kf                 # 2D walks the KEEP edges, 3D the KEEP squares
    if name == "k_classify2d" or name == "k_classify3d":
        sel = is3 if name == "k_classify3d" else ~is3
        n = sum(int(np.prod(s)) for s, k in zip(shapes, sel) if k)
        t = sum(int(np.prod([e - 1 for e in s])) for s, k in zip(shapes, sel) if k)
        return 4 * n + 4 * n + 4 * t + 8 * (int(wc[sel, 0].sum()) + int(wc[sel, 1].sum())
                                            + int(wc[sel, 2].sum()) + int(wc[sel, 3].sum()))
    if name == "k_sort":
        return 16 * (ke + kf + m0)
    f3 = int(wc[is3, 1].sum())                          # facets of the volumes (walked beside H0)
    if name in ("k_resolve", "k_unionfind"):
        return 16 * (ke + f3)
    if name in ("k_resolve(2d top)", "k_unionfind(2d top)"):
        return 16 * (facets - f3)
    if name == "k_output":
        return 8 * (m0 + facets) + 32 * npairs
    if name == "k_zero":
        return 4 * N
    if name == "k_scatter":
        return 32 * npairs
    return 0


# ------------------------------------------------------------------ HBM traffic --
# Under `rocprofv3 --pmc FETCH_SIZE` (then `--pmc WRITE_SIZE`) run `bench.py --profile-steps K`:
# K eager batched steps, then one elementwise kernel (torch.neg) over COPY_BYTES, which must read
# and write exactly COPY_BYTES.  --traffic-from reads the two counter CSVs, scales each counter
# by what it reads for that kernel and writes bytes per launch per kernel for --traffic-json.
COPY_BYTES = 1 << 30
KERNEL_KEYS = ["k_classify2d", "k_classify3d", "k_sort", "k_resolve", "k_unionfind", "k_output", "k_plan",
               "k_zero", "k_scatter"]
PROFILE_NAMES = {}


def profile_steps(steps):
    import torch
    import paper_2606_04801_amd as fc
    shapes = workload_shapes()
    bt = fc.Batch(shapes, device="cuda:0")
    imgs = [S.grf(SHAPE3, SIG3, 2000 + i) for i in range(N3)] + [S.grf(SHAPE2, SIG2, 3000 + i) for i in range(N2)]
    bt.set_images([torch.from_numpy(a) for a in imgs])
    for k in range(steps):
        bt.ph_diagram_batch()
        fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
        diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
        bt.ph_backward(-2.0 * diff, 2.0 * diff)
        torch.cuda.synchronize()
        print("bench: profile step %d done" % k, file=sys.stderr, flush=True)
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)                          # one elementwise kernel: reads and writes COPY_BYTES
    torch.cuda.synchronize()
    bt.check()
    print("bench: profile run done", file=sys.stderr, flush=True)


def _counter_means(path, counter):
    """{kernel key: mean counter value (KiB) per dispatch}, plus the copy kernel's under 'copy'."""
    import csv
    acc = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row.get("Kernel_Name", "")
            key = "copy" if "neg_kernel" in name else next((k for k in KERNEL_KEYS if k in name), None)
            if key is None:
                continue
            v = acc.setdefault(key, [0.0, 0])
            v[0] += float(row["Counter_Value"])
            v[1] += 1
    return {k: v[0] / v[1] for k, v in acc.items()}


def library_sha256():
    import hashlib
    import paper_2606_04801_amd as fc
    with open(fc.LIB_PATH, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_from(fetch_csv, write_csv, out_json):
    fetch, write = _counter_means(fetch_csv, "FETCH_SIZE"), _counter_means(write_csv, "WRITE_SIZE")
    if "copy" not in fetch or "copy" not in write:
        raise SystemExit("bench: no copy kernel in the counter files")
    fs, ws = COPY_BYTES / (fetch["copy"] * 1024), COPY_BYTES / (write["copy"] * 1024)
    # the counters belong to this library build: bench.py uses them only while it is loaded
    res = {"_library_sha256": library_sha256(), "_scale": {"fetch": fs, "write": ws}}
    for k in fetch:
        if k == "copy" or k not in write:
            continue
        res[PROFILE_NAMES.get(k, k)] = round(fetch[k] * 1024 * fs + write[k] * 1024 * ws)
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes (0: host cores, at most 16)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "hbm_traffic.json"),
                    help="HBM bytes per launch from the counter passes (used only for the library build they were taken on)")
    ap.add_argument("--profile-steps", type=int, default=0, help="only run K eager steps and a calibration copy")
    ap.add_argument("--traffic-from", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"))
    ap.add_argument("--host-library", default=None,
                    help="check this script on the CPU against a host build of the C ABI (small workload)")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from)
        return
    if args.profile_steps:
        profile_steps(args.profile_steps)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the batch would shard by instance "
              "across GPUs; no multi-GPU path is built)", file=sys.stderr)
        sys.exit(2)

    if args.host_library:
        use_small_workload()
    shapes = workload_shapes()
    nvox = sum(int(np.prod(s)) for s in shapes)
    line = {"metric": METRIC, "value": None, "unit": "Mvoxels/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": workload_desc(), "instances": len(shapes), "voxels": nvox}}

    ref = {}
    if not args.no_cpu_baseline:                 # before this process loads HIP
        workers = args.cpu_workers or min(16, len(os.sched_getaffinity(0)))
        print("bench: cpu baseline (oracle on %d cores, about 30 s)" % workers, file=sys.stderr, flush=True)
        line["cpu_baseline"], ref = cpu_baseline(workers)
    import torch
    import paper_2606_04801_amd as fc
    if args.host_library:
        fc.LIB_PATH = args.host_library
    fc.lib()
    gpu = torch.cuda.is_available()
    if args.host_library:
        line.update(run_gpu(fc, torch, shapes, args, ref, dev=torch.device("cpu")))
        line["status"] = "host-library check, not a measurement"
    elif not gpu:
        line["status"] = "no GPU"
    else:
        line.update(run_gpu(fc, torch, shapes, args, ref))
    print(json.dumps(line), flush=True)


def same_bits(a, b):
    """Pair arrays equal field by field, floats compared by their bits."""
    return len(a) == len(b) and all(np.array_equal(np.ascontiguousarray(a[f]).view(np.uint8),
                                                   np.ascontiguousarray(b[f]).view(np.uint8))
                                    for f in a.dtype.names)


def step_bytes(prof_names, wc, npairs, shapes):
    """Algorithmic bytes of one batched forward + backward step (kernel models summed)."""
    return sum(algorithmic_bytes(k, wc, npairs, shapes) for k in prof_names)


def run_gpu(fc, torch, shapes, args, ref, dev=None):
    dev = dev or torch.device("cuda:0")
    cuda = dev.type == "cuda"
    sync = torch.cuda.synchronize if cuda else (lambda: None)
    print("bench: generating %d instances" % len(shapes), file=sys.stderr, flush=True)
    imgs = [S.grf(SHAPE3, SIG3, 2000 + i) for i in range(N3)] + [S.grf(SHAPE2, SIG2, 3000 + i) for i in range(N2)]
    host = [torch.from_numpy(a) for a in imgs]
    if cuda:
        torch.zeros(1, device=dev)               # the device context exists before the library's first call
    rc = fc.lib().ph_init_device()
    if rc != fc.PH_OK:
        raise fc.PHError(rc, "ph_init_device")

    # sizing pass with the never-overflowing capacity, then exact capacities: the pair buffers
    # (and the loss-gradient arithmetic over them) stay as small as the diagrams
    print("bench: sizing pass", file=sys.stderr, flush=True)
    sizing = fc.Batch(shapes, device=dev)
    sizing.set_images(host)
    sizing.ph_diagram_batch()
    sync()
    sizing.check()
    caps = sizing.counts.cpu().numpy().tolist()
    del sizing
    if cuda:
        torch.cuda.empty_cache()

    # two copies of inputs and buffers; timed steps alternate between them so that a step does
    # not find its inputs in the caches from the step before
    bts = []
    for _ in range(2):
        bt = fc.Batch(shapes, device=dev, capacities=caps)
        bt.set_images(host)
        bts.append(bt)

    def batched_step(bt, backward=True):
        bt.ph_diagram_batch()
        if backward:
            fin = bt.valid_mask() & (bt.pairs.death_cell >= 0)
            diff = torch.where(fin, bt.pairs.death - bt.pairs.birth, 0.0)
            bt.ph_backward(-2.0 * diff, 2.0 * diff)

    # per-image plain calls on the same inputs, one stream, no graph
    singles = [[], []]
    for c in range(2):
        for i in range(len(imgs)):
            singles[c].append(dict(img=bts[c].image(i), cap=int(caps[i]), ws=fc.Workspace(),
                                   grad=torch.empty(imgs[i].shape, dtype=torch.float32, device=dev),
                                   off=torch.tensor([0, max(int(caps[i]), 1)], dtype=torch.int64, device=dev),
                                   ioff=torch.zeros(1, dtype=torch.int64, device=dev)))

    def per_image_step(c):
        for s in singles[c]:
            d = fc.ph_diagram(s["img"], capacity=s["cap"], ws=s["ws"])
            s["diag"] = d
            idx = torch.arange(d.bufs.cap, device=dev)
            fin = (idx < d.count_t) & (d.bufs.death_cell >= 0)
            diff = torch.where(fin, d.bufs.death - d.bufs.birth, 0.0)
            fc.ph_backward(d.bufs, d.count_t, s["off"], s["ioff"], -2.0 * diff, 2.0 * diff, s["grad"])

    # parity: batched, per-image and (for the sampled instances) the oracle, bit for bit
    print("bench: parity", file=sys.stderr, flush=True)
    bt = bts[0]
    batched_step(bt)
    per_image_step(0)
    sync()
    bt.check()
    res = bt.results()
    for i, s in enumerate(singles[0]):
        if not same_bits(res[i], s["diag"].numpy()):
            raise SystemExit("bench: batched and per-image diagrams differ on instance %d" % i)
        g1 = bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]]
        if not torch.allclose(g1, s["grad"].reshape(-1), rtol=1e-6, atol=1e-7):
            raise SystemExit("bench: batched and per-image gradients differ on instance %d" % i)
    for i, (p, g) in ref.items():
        if not same_bits(res[i], p):
            raise SystemExit("bench: instance %d differs from the oracle" % i)
        g1 = bt.grad[bt.img_off_h[i]:bt.img_off_h[i + 1]].cpu().numpy()
        if not np.allclose(g1, g.reshape(-1), rtol=1e-6, atol=1e-7):
            raise SystemExit("bench: gradient of instance %d differs from the oracle" % i)

    def capture(fn):
        """A replayable step: a captured HIP graph on the GPU (the host check replays eagerly)."""
        for _ in range(args.warmup):
            fn()
        sync()
        if not cuda:
            return fn
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        return g.replay

    def timed(run):
        for k in range(args.warmup):
            run(k)
        sync()
        t0 = time.perf_counter()
        for k in range(args.steps):
            run(k)
        sync()
        return (time.perf_counter() - t0) / args.steps

    print("bench: batched forward + backward (graph replay)", file=sys.stderr, flush=True)
    g_fb = [capture(lambda b=b: batched_step(b)) for b in bts]
    t_b = timed(lambda k: g_fb[k % 2]())
    for b in bts:
        b.check()
    print("bench: batched forward only (graph replay)", file=sys.stderr, flush=True)
    g_f = [capture(lambda b=b: batched_step(b, backward=False)) for b in bts]
    t_f = timed(lambda k: g_f[k % 2]())
    print("bench: per-image plain calls", file=sys.stderr, flush=True)
    t_p = timed(lambda k: per_image_step(k % 2))

    # per-kernel event timing of the batched step (eager, the same launches as the graph)
    fc.profile(True)
    for k in range(args.steps):
        batched_step(bts[k % 2])
    sync()
    prof = fc.profile_read()
    fc.profile(False)
    npairs = int(bt.counts.cpu().numpy().sum())
    wc = bt.work_counters()
    name, (launches, total_ms) = max(prof.items(), key=lambda kv: kv[1][1])
    mean_s = total_ms / launches / 1e3
    algo = algorithmic_bytes(name, wc, npairs, shapes)
    achieved = algo / mean_s / 1e9 if mean_s > 0 else 0.0
    traffic = None
    if args.traffic_json and os.path.exists(args.traffic_json):
        tj = json.load(open(args.traffic_json))
        if tj.get("_library_sha256") == library_sha256():
            traffic = tj.get(name)
    # the same instances quantised to 256 levels and read as uint8 (PH_IN_U8), checked bit for
    # bit against the float32 path on the same values, then timed like the batched form
    print("bench: batched forward + backward, uint8 input (graph replay)", file=sys.stderr, flush=True)
    q8 = [torch.from_numpy(np.round(a * 255.0).astype(np.uint8)) for a in imgs]
    sz = fc.Batch(shapes, device=dev)
    sz.set_images([q.float() for q in q8])
    batched_step(sz)
    sync()
    ref8 = sz.results()
    gref8 = sz.grad.cpu().numpy().copy()
    caps8 = sz.counts.cpu().numpy().tolist()
    del sz
    b8 = []
    for _ in range(2):
        b = fc.Batch(shapes, device=dev, capacities=caps8, dtype=torch.uint8)
        b.set_images(q8)
        b8.append(b)
    batched_step(b8[0])
    sync()
    for i, r in enumerate(b8[0].results()):
        if not same_bits(r, ref8[i]):
            raise SystemExit("bench: uint8 and float32 inputs give different diagrams on instance %d" % i)
    if not np.array_equal(b8[0].grad.cpu().numpy(), gref8):
        raise SystemExit("bench: uint8 and float32 inputs give different gradients")
    g_8 = [capture(lambda b=b: batched_step(b)) for b in b8]
    t_8 = timed(lambda k: g_8[k % 2]())
    for b in b8:
        b.check()

    # the same instances under the T-filtration (pixels as top cells, PH_TFILT): sized by a
    # first call, then timed like the batched form (parity of this path is the T test suite's)
    print("bench: batched forward + backward, T-filtration (graph replay)", file=sys.stderr, flush=True)
    src = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)) for a in imgs]
    sz = fc.Batch(shapes, device=dev, filtration="T")
    sz.set_images(src)
    batched_step(sz)
    sync()
    sz.check()
    caps_t = sz.counts.cpu().numpy().tolist()
    del sz
    b_t = []
    for _ in range(2):
        b = fc.Batch(shapes, device=dev, capacities=caps_t, filtration="T")
        b.set_images(src)
        b_t.append(b)
    g_t = [capture(lambda b=b: batched_step(b)) for b in b_t]
    t_t = timed(lambda k: g_t[k % 2]())
    for b in b_t:
        b.check()
        if not np.array_equal(b.counts.cpu().numpy(), np.asarray(caps_t)):
            raise SystemExit("bench: T-filtration pair counts changed between calls")

    nvox = sum(int(np.prod(s)) for s in shapes)
    sb = step_bytes(prof.keys(), wc, npairs, shapes)
    fb = sb - algorithmic_bytes("k_zero", wc, npairs, shapes) - algorithmic_bytes("k_scatter", wc, npairs, shapes)
    frac = lambda b, t: round(b / t / (HBM_PEAK_GBS * 1e9), 5)
    return {
        "value": round(nvox / t_b / 1e6, 3),
        "ms_per_step": round(t_b * 1e3, 4),
        "forms": {
            "batched_fwd_bwd": {"value": round(nvox / t_b / 1e6, 3), "ms": round(t_b * 1e3, 4), "hbm_frac": frac(sb, t_b)},
            "batched_fwd": {"value": round(nvox / t_f / 1e6, 3), "ms": round(t_f * 1e3, 4), "hbm_frac": frac(fb, t_f)},
            "per_image_fwd_bwd": {"value": round(nvox / t_p / 1e6, 3), "ms": round(t_p * 1e3, 4), "hbm_frac": frac(sb, t_p)},
            "batched_fwd_bwd_u8": {"value": round(nvox / t_8 / 1e6, 3), "ms": round(t_8 * 1e3, 4),
                                   "input": "the same instances quantised to 256 levels, uint8"},
            "batched_fwd_bwd_tfilt": {"value": round(nvox / t_t / 1e6, 3), "ms": round(t_t * 1e3, 4),
                                      "input": "the same instances under the T-filtration"},
        },
        "roofline": {"bound": "hbm", "kernel": name, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic},
        "kernels_ms": {k: round(v[1] / v[0], 4) for k, v in prof.items()},
        "work": {"keep_edges": int(wc[:, 0].sum()), "keep_squares": int(wc[:, 1].sum()),
                 "h0_nodes": int(wc[:, 2].sum()), "dual_nodes": int(wc[:, 3].sum()),
                 "pairs": npairs, "max_rounds": int(wc[:, 4:6].max()),
                 "sequential_edges": int(wc[:, 6].sum())},
    }


if __name__ == "__main__":
    main()
