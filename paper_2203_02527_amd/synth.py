"""Seeded synthetic point clouds for the H0 barcode workloads.

This module only draws integer point clouds; it holds none of the barcode
arithmetic (no distances, no sorting, no reduction), so that the GPU library
and the CPU oracle can both consume exactly the same bytes.

The paper measures on real-valued points drawn uniformly from (0,1)^2
(Sections 3.1 and 4.1).  The workloads here replace them with integer clouds
so that squared distances are exact; their shapes follow the five workloads
the library is measured on:

* ``uniform``   -- N=256, d=3, int16 coordinates uniform in [-100, 100].
* ``mixture``   -- int8 coordinates from a mixture of isotropic Gaussian
  clusters (centres uniform in [-100, 100]^d, rounded half-to-even, clipped
  to [-127, 127]); N=4096/d=16/8 clusters/std 10 and N=16384/d=64/32
  clusters/std 12 are the two large single-cloud workloads.
* ``batch``     -- many clouds, N uniform in [32, 512], d=3 int16, each either
  a noisy circle (radius 80, noise std 5) or 2-4 Gaussian blobs (std 10).
* ``serving``   -- a request mix: N log-uniform in [64, 8192], d in {3,16,64},
  int8 or int16 Gaussian mixtures with 2-8 clusters.

Every generator takes an explicit seed and uses numpy's PCG64 stream.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "uniform_cloud",
    "unit_square_cloud",
    "mixture_cloud",
    "batch_clouds",
    "circle_cloud",
    "blobs_cloud",
    "serving_requests",
    "workload",
    "WORKLOADS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_cloud(n: int = 256, d: int = 3, lo: int = -100, hi: int = 100,
                  seed: int = 0, dtype=np.int16) -> np.ndarray:
    """n x d integer points uniform in [lo, hi] (inclusive)."""
    rng = _rng(seed)
    return rng.integers(lo, hi + 1, size=(n, d)).astype(dtype)


UNIT_SCALE = 32767  # fixed-point grid of the unit-square workload


def unit_square_cloud(n: int, seed: int = 0, scale: int = UNIT_SCALE) -> np.ndarray:
    """n points uniform in [0, 1]^2 (the paper's experiments), on a
    fixed-point grid: each coordinate is rint(u * scale) as int16, so that
    squared distances, their order and their ties are exact integers."""
    rng = _rng(seed)
    u = rng.random((n, 2))
    return np.rint(u * scale).astype(np.int16)


def _mixture(rng: np.random.Generator, n: int, d: int, k: int, std: float,
             centre_lo: float, centre_hi: float, clip: int, dtype) -> np.ndarray:
    centres = rng.uniform(centre_lo, centre_hi, size=(k, d))
    labels = rng.integers(0, k, size=n)
    x = centres[labels] + std * rng.standard_normal(size=(n, d))
    x = np.clip(np.rint(x), -clip, clip)
    return x.astype(dtype)


def mixture_cloud(n: int = 4096, d: int = 16, k: int = 8, std: float = 10.0,
                  seed: int = 0, dtype=np.int8, clip: int = 127,
                  centre_range: float = 100.0) -> np.ndarray:
    """Gaussian-mixture cloud: k centres uniform in [-R, R]^d, isotropic noise."""
    rng = _rng(seed)
    return _mixture(rng, n, d, k, std, -centre_range, centre_range, clip, dtype)


def circle_cloud(rng: np.random.Generator, n: int, radius: float = 80.0,
                 noise: float = 5.0, dtype=np.int16) -> np.ndarray:
    """Noisy circle in the x-y plane of R^3 (third coordinate is noise only)."""
    theta = rng.uniform(0.0, 2.0 * math.pi, size=n)
    base = np.stack([radius * np.cos(theta), radius * np.sin(theta),
                     np.zeros(n)], axis=1)
    x = base + noise * rng.standard_normal(size=(n, 3))
    return np.rint(x).astype(dtype)


def blobs_cloud(rng: np.random.Generator, n: int, std: float = 10.0,
                dtype=np.int16) -> np.ndarray:
    """2-4 Gaussian blobs with centres uniform in [-100, 100]^3."""
    k = int(rng.integers(2, 5))
    centres = rng.uniform(-100.0, 100.0, size=(k, 3))
    labels = rng.integers(0, k, size=n)
    x = centres[labels] + std * rng.standard_normal(size=(n, 3))
    return np.rint(x).astype(dtype)


def batch_clouds(count: int = 10000, n_lo: int = 32, n_hi: int = 512,
                 seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Many uneven d=3 int16 clouds, concatenated.

    Returns (points, offsets): points is sum(N) x 3 int16 and cloud c owns
    rows offsets[c]:offsets[c+1].
    """
    rng = _rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    kinds = rng.integers(0, 2, size=count)
    parts = []
    for n, kind in zip(sizes, kinds):
        if kind == 0:
            parts.append(circle_cloud(rng, int(n)))
        else:
            parts.append(blobs_cloud(rng, int(n)))
    offsets = np.zeros(count + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    points = np.concatenate(parts, axis=0) if parts else np.zeros((0, 3), np.int16)
    return points, offsets


def serving_requests(count: int, seed: int = 0, n_lo: int = 64,
                     n_hi: int = 8192) -> list[np.ndarray]:
    """A request mix of clouds with log-uniform N, d in {3,16,64}, int8/int16.

    int8 clouds: centres uniform in [-100,100]^d, std 10, clip +-127.
    int16 clouds: centres uniform in [-6400,6400]^d, std 640, clip +-16383.
    """
    rng = _rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(rng.choice([3, 16, 64]))
        k = int(rng.integers(2, 9))
        if int(rng.integers(0, 2)) == 0:
            out.append(_mixture(rng, n, d, k, 10.0, -100.0, 100.0, 127, np.int8))
        else:
            out.append(_mixture(rng, n, d, k, 640.0, -6400.0, 6400.0, 16383,
                                np.int16))
    return out


# Named single-cloud workloads (the batched and serving mixes are above).
WORKLOADS = {
    "uniform_n256_d3_i16": dict(kind="uniform", n=256, d=3),
    "mixture_n4096_d16_i8": dict(kind="mixture", n=4096, d=16, k=8, std=10.0),
    "mixture_n16384_d64_i8": dict(kind="mixture", n=16384, d=64, k=32, std=12.0),
}


def workload(name: str, seed: int = 0) -> np.ndarray:
    """Points of a named single-cloud workload (C-contiguous)."""
    w = WORKLOADS[name]
    if w["kind"] == "uniform":
        x = uniform_cloud(w["n"], w["d"], seed=seed)
    else:
        x = mixture_cloud(w["n"], w["d"], w["k"], w["std"], seed=seed)
    return np.ascontiguousarray(x)
