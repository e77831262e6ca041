"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds none of the method's arithmetic: only reproducible random numbers with the
shapes of the method's inputs (white noise on the particle grid, particle
displacements).  Both the HIP path and the oracle receive the same float32 arrays.
"""
from __future__ import annotations

import numpy as np


def white_noise(np_side: int, seed: int) -> np.ndarray:
    """N(0, 1) white noise on the np^3 particle grid, float32, particle order."""
    return np.random.default_rng(seed).standard_normal(np_side**3).astype(np.float32)


def displacements(np_side: int, box: float, seed: int, rms: float, clump_frac: float = 0.2,
                  clump_width: float = 0.5) -> np.ndarray:
    """Random displacements (3, np^3), float32: Gaussian of the given rms plus a
    fraction of particles pulled into one tight clump (many particles per cell)."""
    rng = np.random.default_rng(seed)
    n = np_side**3
    s = rms * rng.standard_normal((3, n))
    ax = np.arange(np_side) * (box / np_side)
    q = np.stack(np.meshgrid(ax, ax, ax, indexing="ij")).reshape(3, n)
    centre = np.array([0.31, 0.62, 0.13])[:, None] * box
    clump = rng.random(n) < clump_frac
    s[:, clump] = (centre - q[:, clump]) + clump_width * rng.standard_normal((3, int(clump.sum())))
    return s.astype(np.float32)


def mesh_field(n: int, seed: int) -> np.ndarray:
    """Random real field on an n^3 mesh, float32."""
    return np.random.default_rng(seed).standard_normal((n, n, n)).astype(np.float32)
