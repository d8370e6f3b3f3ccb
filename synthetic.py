"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the persistence method: it only makes pixel arrays.
Every generator is exact integer arithmetic up to one final, correctly rounded float
division, so the same seed gives bit-identical arrays on any x86-64 host.

Workloads (stand-ins for the real images and volumes the paper benchmarks on, which are not
available here):
  * ``uniform``  : i.i.d. uniform [0,1) pixels, the paper's synthetic workload.
  * ``grf``      : a smooth random field, standing in for natural images and volumes: centred
                   uniform integer white noise, smoothed by a separable integer-quantised
                   Gaussian kernel of radius ceil(4 sigma) with periodic wrap, rescaled to
                   [0,1) and rounded to float32.
  * ``quantize_u8``: 256-level copy of a field in [0,1) (heavy ties), returned as float32.
"""
from __future__ import annotations

import math

import numpy as np

_NOISE_BITS = 20      # white noise in [-2^20, 2^20)
_W_BITS = 16          # kernel weights scaled by 2^16


def uniform(shape, seed: int) -> np.ndarray:
    """i.i.d. uniform [0,1) float32 pixels (numpy PCG64)."""
    return np.random.default_rng(seed).random(tuple(shape), dtype=np.float32)


def _kernel(sigma: float) -> np.ndarray:
    r = int(math.ceil(4.0 * sigma))
    w = [int(round(math.exp(-0.5 * (t / sigma) ** 2) * (1 << _W_BITS))) for t in range(-r, r + 1)]
    return np.asarray(w, dtype=np.int64)


def _smooth_axis(g: np.ndarray, w: np.ndarray, axis: int) -> np.ndarray:
    r = (len(w) - 1) // 2
    acc = np.zeros_like(g)
    for t in range(len(w)):
        acc += w[t] * np.roll(g, r - t, axis=axis)     # periodic (wrap) boundary
    return acc >> _W_BITS                              # exact rescale (floor)


def grf(shape, sigma: float, seed: int) -> np.ndarray:
    """Smooth random field in [0,1) as float32, deterministic from ``seed``."""
    rng = np.random.default_rng(seed)
    g = rng.integers(-(1 << _NOISE_BITS), 1 << _NOISE_BITS, size=tuple(shape), dtype=np.int64)
    w = _kernel(sigma)
    for ax in range(g.ndim):
        g = _smooth_axis(g, w, ax)
    lo, hi = int(g.min()), int(g.max())
    if hi == lo:
        return np.zeros(tuple(shape), np.float32)
    x = (g - lo).astype(np.float64) / float(hi - lo)   # exact integers, one rounded division
    return (x * (1.0 - 2.0 ** -24)).astype(np.float32)


def quantize_u8(x: np.ndarray) -> np.ndarray:
    """256-level quantisation of a [0,1) field, as exact float32 integers 0..255."""
    q = np.minimum(np.floor(x.astype(np.float64) * 256.0), 255.0)
    return q.astype(np.float32)


def tie_free(shape, seed: int) -> np.ndarray:
    """Distinct values (perm + 0.5)/n: minimum gap 1/n, for finite-difference checks."""
    n = int(np.prod(shape))
    p = np.random.default_rng(seed).permutation(n)
    return ((p.astype(np.float64) + 0.5) / n).astype(np.float32).reshape(tuple(shape))


def levels(shape, nlev: int, seed: int) -> np.ndarray:
    """Random values on ``nlev`` levels (heavy ties) for edge-case tests."""
    r = np.random.default_rng(seed).integers(0, nlev, size=tuple(shape))
    return (r.astype(np.float64) / nlev).astype(np.float32)


# --------------------------------------------------------------------------- workloads --

def workload_2d_uniform_128():
    """128x128 i.i.d. uniform, seed 0: H0 and H1."""
    return [uniform((128, 128), 0)]


def workload_2d_grf_2048(quantized: bool = False):
    """2048x2048 field, sigma 8 px, seed 1 (and its 256-level copy)."""
    x = grf((2048, 2048), 8.0, 1)
    return [quantize_u8(x) if quantized else x]


def workload_3d_grf_256():
    """256^3 field, sigma 4 voxels, seed 2: H0 and H2."""
    return [grf((256, 256, 256), 4.0, 2)]


def batch_shapes_512(n: int = 512):
    """Sizes and sigmas of the uneven 2D batch: H, W ~ U{64..512}, sigma in {2,4,8}."""
    rng = np.random.default_rng(999)
    hw = rng.integers(64, 513, size=(n, 2))
    sig = rng.choice(np.array([2.0, 4.0, 8.0]), size=n)
    return [((int(h), int(w)), float(s)) for (h, w), s in zip(hw, sig)]


def workload_batch_512(n: int = 512):
    """512 fields of uneven sizes, image i from seed 1000+i."""
    return [grf(shape, s, 1000 + i) for i, (shape, s) in enumerate(batch_shapes_512(n))]


def workload_mixed_fwd_bwd(n3: int = 64, n2: int = 64):
    """64 volumes 96^3 (sigma 3, seeds 2000+i) then 64 images 512^2 (sigma 6, seeds 3000+i)."""
    vols = [grf((96, 96, 96), 3.0, 2000 + i) for i in range(n3)]
    imgs = [grf((512, 512), 6.0, 3000 + i) for i in range(n2)]
    return vols + imgs
