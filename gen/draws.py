"""Seeded vertex and vertex-pair draws (uniform over the grid, Eq. 3's U(Omega^2)
restricted to grid vertices)."""
from __future__ import annotations

import numpy as np

SEED_REFS = 2311
SEED_TRAIN = 2312
SEED_HELDOUT = 2399


def random_vertices(n_vertices: int, n: int, seed: int = SEED_REFS) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_vertices, size=n, dtype=np.int64)


def random_pairs(n_vertices: int, n: int, seed: int) -> np.ndarray:
    """int64 [n][2]: independent uniform endpoints (p1, p2)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_vertices, size=(n, 2), dtype=np.int64)
