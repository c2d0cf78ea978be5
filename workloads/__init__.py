"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and describes workload shapes; it holds
none of the FMM's arithmetic.  Every array is produced in float64 by numpy's
PCG64 generator (``numpy.random.default_rng``) from a fixed seed, so the oracle
and the HIP library are fed bit-identical inputs.

Seed convention: points ``1000 + c``, charges ``2000 + c``, sampled targets
``3000 + c`` and the batched-problem draw ``5000``, where ``c`` is the workload
number below.  The paper's benchmark problems are uniform points in the unit
box with sources equal to targets and random source densities (Section 4);
the sphere-surface cloud stands in for its non-uniform mesh, which is not
available here.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_POINTS = 1000
SEED_CHARGES = 2000
SEED_SAMPLES = 3000
SEED_BATCH = 5000


def uniform_cube(n: int, seed: int) -> np.ndarray:
    """``n`` points uniform in [0, 1)^3, shape (n, 3), float64."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 3))


def sphere_surface(n: int, seed: int) -> np.ndarray:
    """``n`` points on the unit sphere (normalised standard-normal vectors)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def charges(n: int, nvec: int, seed: int, dist: str) -> np.ndarray:
    """Charge vectors, shape (nvec, n) C-contiguous (column-major [nvec][n])."""
    rng = np.random.default_rng(seed)
    if dist == "u01":
        q = rng.random((nvec, n))
    elif dist == "upm1":
        q = rng.uniform(-1.0, 1.0, (nvec, n))
    elif dist == "normal":
        q = rng.standard_normal((nvec, n))
    else:
        raise ValueError(dist)
    return np.ascontiguousarray(q)


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """``k`` distinct target indices out of ``n``, sorted."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False))


@dataclass
class Workload:
    """One problem: points, charges and the tree / expansion parameters."""

    name: str
    points: np.ndarray          # (n, 3) float64; sources == targets
    q: np.ndarray               # (nvec, n) float64
    depth: int
    order: int                  # expansion order p
    origin: tuple
    width: float
    m2l: str                    # "dense" | "fft" | "blas"
    svd_rel_tol: float = 0.0
    svd_rel_tol_dir: float = -1.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.points.shape[0]

    @property
    def nvec(self) -> int:
        return self.q.shape[0]


def config(c: int, n: int | None = None, nvec: int | None = None,
           depth: int | None = None) -> Workload:
    """The five benchmark workloads; ``n``/``nvec``/``depth`` shrink them for tests.

    1: plain kiFMM, 20,000 uniform points, depth 3, p=3, dense M2L, 1 vector.
    2: FFT-M2L, 1,000,000 uniform points, depth 5, p=6, 1 vector in [0,1).
    3: BLAS-M2L (relative SVD threshold 1e-6), 1,000,000 uniform points,
       depth 5, p=6, 32 vectors in [-1,1).
    4: 4,000,000 points on the unit sphere in [-1,1]^3, depth 6, p=6,
       64 standard-normal vectors.
    6: 8,000,000 uniform points, depth 6, p=6, FFT-M2L, 1 vector in [0,1)
       (the paper's larger problem size, for runs at scale).
    """
    if c == 1:
        n = 20_000 if n is None else n
        nv = 1 if nvec is None else nvec
        pts = uniform_cube(n, SEED_POINTS + c)
        q = charges(n, nv, SEED_CHARGES + c, "u01")
        return Workload("uniform-20k-d3-p3-dense", pts, q, 3 if depth is None else depth,
                        3, (0.0, 0.0, 0.0), 1.0, "dense")
    if c == 2:
        n = 1_000_000 if n is None else n
        nv = 1 if nvec is None else nvec
        pts = uniform_cube(n, SEED_POINTS + c)
        q = charges(n, nv, SEED_CHARGES + c, "u01")
        return Workload("uniform-1M-d5-p6-fft", pts, q, 5 if depth is None else depth,
                        6, (0.0, 0.0, 0.0), 1.0, "fft")
    if c == 3:
        n = 1_000_000 if n is None else n
        nv = 32 if nvec is None else nvec
        pts = uniform_cube(n, SEED_POINTS + c)
        q = charges(n, nv, SEED_CHARGES + c, "upm1")
        return Workload("uniform-1M-d5-p6-blas-32rhs", pts, q, 5 if depth is None else depth,
                        6, (0.0, 0.0, 0.0), 1.0, "blas", svd_rel_tol=1e-6,
                        svd_rel_tol_dir=1e-6)
    if c == 4:
        n = 4_000_000 if n is None else n
        nv = 64 if nvec is None else nvec
        pts = sphere_surface(n, SEED_POINTS + c)
        q = charges(n, nv, SEED_CHARGES + c, "normal")
        return Workload("sphere-4M-d6-p6-64rhs", pts, q, 6 if depth is None else depth,
                        6, (-1.0, -1.0, -1.0), 2.0, "fft")
    if c == 6:
        n = 8_000_000 if n is None else n
        nv = 1 if nvec is None else nvec
        pts = uniform_cube(n, SEED_POINTS + c)
        q = charges(n, nv, SEED_CHARGES + c, "u01")
        return Workload("uniform-8M-d6-p6-fft", pts, q, 6 if depth is None else depth,
                        6, (0.0, 0.0, 0.0), 1.0, "fft")
    raise ValueError(f"unknown workload {c}")


def batch_problems(count: int = 128, seed: int = SEED_BATCH) -> list[dict]:
    """Problem shapes of the batched serving workload.

    N is log-uniform in [1e4, 2e5); depth = clamp(round(log8(N/40)), 3, 4);
    p uniform over {4, 5, 6}; 1..8 charge vectors.  Points and charges of
    problem i are drawn with seeds ``seed + 1 + 2i`` and ``seed + 2 + 2i``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(1e4), math.log(2e5)))))
        depth = int(min(4, max(3, round(math.log(n / 40.0, 8)))))
        p = int(rng.integers(4, 7))
        nvec = int(rng.integers(1, 9))
        out.append(dict(n=n, depth=depth, order=p, nvec=nvec,
                        seed_points=seed + 1 + 2 * i, seed_charges=seed + 2 + 2 * i))
    return out
