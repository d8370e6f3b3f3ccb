"""Write tests/golden/digests.json: the oracle's diagrams of the full-size workloads, as digests.

    python tests/golden/make_digests.py [--jobs 6] [--only c1,c2,...]

Configs c1..c5 are under the V-filtration; c5t is c5's 128 instances under the T-filtration
(pixels as top cells), whose pairs come in the T output order (dim, death key); c5h1 is c5's
first eight volumes with every dimension (H0, H1, H2).

Calls only the CPU oracle (oracle/) and the seeded generators (synthetic.py).  For every
instance it stores the digest of its input pixels (so a change of generator is caught), the
number of H0 and top-dimension pairs, and a SHA-256 over the pairs in output order, packed
little-endian as dim int8, birth and death float32 bits, birth and death cell int64, birth and
death vertex int32.  The full-size GPU parity tests compare the GPU output with these digests.
The 256^3 volume takes about ten minutes and a few GB of memory.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from multiprocessing import get_context

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PACKED = np.dtype([("dim", "<i1"), ("birth", "<u4"), ("death", "<u4"), ("birth_cell", "<i8"),
                   ("death_cell", "<i8"), ("birth_vertex", "<i4"), ("death_vertex", "<i4")])


def pair_digest(pairs) -> str:
    """SHA-256 of a pair array (any dtype with the PAIR_DTYPE field names), packed."""
    a = np.zeros(len(pairs), PACKED)
    for f in PACKED.names:
        v = np.asarray(pairs[f])
        a[f] = v.view(np.uint32) if v.dtype == np.float32 else v
    return hashlib.sha256(a.tobytes()).hexdigest()


def input_digest(img) -> str:
    return hashlib.sha256(np.ascontiguousarray(img, dtype="<f4").tobytes()).hexdigest()


def instances():
    """(config, index, generator name, args) of every instance of the full-size workloads."""
    import synthetic as S
    out = [("c1", 0, "uniform", ((128, 128), 0)),
           ("c2", 0, "grf", ((2048, 2048), 8.0, 1)),
           ("c2u8", 0, "grf_u8", ((2048, 2048), 8.0, 1)),
           ("c3", 0, "grf", ((256, 256, 256), 4.0, 2))]
    for i, (shape, s) in enumerate(S.batch_shapes_512()):
        out.append(("c4", i, "grf", (shape, s, 1000 + i)))
    for i in range(64):
        out.append(("c5", i, "grf", ((96, 96, 96), 3.0, 2000 + i)))
    for i in range(64):
        out.append(("c5", 64 + i, "grf", ((512, 512), 6.0, 3000 + i)))
    out += [("c5t",) + it[1:] for it in out if it[0] == "c5"]
    out += [("c5h1",) + it[1:] for it in out if it[0] == "c5" and it[1] < 8]
    return out


def dims_of(cfg, ndim):
    """The dimensions a config's digest covers: every one for the H1 configs (name ending in
    h1), else H0 and the top dimension."""
    return tuple(range(ndim)) if cfg.endswith("h1") else (0, ndim - 1)


def filtration_of(cfg) -> str:
    """"T" for the T-filtration configs (name ending in t), else "V"."""
    return "T" if cfg.endswith("t") else "V"


def make(kind, args):
    import synthetic as S
    if kind == "uniform":
        return S.uniform(*args)
    if kind == "grf":
        return S.grf(*args)
    if kind == "grf_u8":
        return S.quantize_u8(S.grf(*args))
    raise ValueError(kind)


def job(item):
    import oracle
    cfg, idx, kind, args = item
    img = make(kind, args)
    t0 = time.perf_counter()
    p = oracle.diagram(img, dims=dims_of(cfg, img.ndim), filtration=filtration_of(cfg))
    dt = time.perf_counter() - t0
    top = img.ndim - 1
    return cfg, idx, {"shape": list(img.shape), "input_sha256": input_digest(img),
                      "h0": int((p["dim"] == 0).sum()), "htop": int((p["dim"] == top).sum()),
                      "pairs_sha256": pair_digest(p), "oracle_s": round(dt, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--only", default=None)
    a = ap.parse_args()
    items = instances()
    if a.only:
        keep = set(a.only.split(","))
        items = [it for it in items if it[0] in keep]
    items.sort(key=lambda it: 0 if it[0] == "c3" else (1 if len(it[3][0]) == 3 else 2))   # longest first
    path = os.path.join(HERE, "digests.json")
    doc = json.load(open(path)) if os.path.exists(path) else {}
    doc["_about"] = ("oracle diagrams of the full-size workloads (H0 + top dimension), written by "
                     "tests/golden/make_digests.py from oracle/ and synthetic.py only")
    with get_context("fork").Pool(a.jobs) as pool:
        for cfg, idx, rec in pool.imap_unordered(job, items):
            doc.setdefault(cfg, {})[str(idx)] = rec
            print(cfg, idx, rec["shape"], rec["h0"], rec["htop"], rec["oracle_s"], flush=True)
            with open(path + ".tmp", "w") as f:
                json.dump(doc, f, indent=0, sort_keys=True)
            os.replace(path + ".tmp", path)


if __name__ == "__main__":
    main()
