"""Loader for the hand-derived golden fixtures in tests/golden/fixtures.json."""
import json
import os

import numpy as np

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fixtures.json")


def _values(case):
    shape = tuple(case["shape"])
    v = case["values"]
    if isinstance(v, list):
        return np.asarray(v, np.float32).reshape(shape)
    n = int(np.prod(shape))
    if v == "pixidx/100, centre 0.9":
        a = (np.arange(n) / 100.0).astype(np.float32)
        a[n // 2] = np.float32(0.9)
        return a.reshape(shape)
    if v in ("annulus", "hollow_cube"):
        c = np.indices(shape) - 3
        r = np.abs(c).max(axis=0)
        a = np.full(shape, 1.0, np.float32)
        a[r == 2] = 0.0
        a[r <= 1] = 0.5
        return a
    if v == "ramp":
        return np.arange(n, dtype=np.float32).reshape(shape)
    raise ValueError(v)


def load():
    with open(_PATH) as f:
        doc = json.load(f)
    out = []
    for case in doc["cases"]:
        pairs = [tuple(float("inf") if x == "inf" else x for x in p) for p in case["pairs"]]
        out.append((case["name"], _values(case), pairs, case))
    return out
