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


def random_positions(n: int, seed: int, spread: float = 1.0) -> np.ndarray:
    """float32 [n][3]: continuous positions uniform in [-spread, spread]^3 (the
    network's domain is [-1, 1]^3; spread > 1 also draws points outside it)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-spread, spread, size=(n, 3)).astype(np.float32)


def ray_positions(n_rays: int, n_steps: int, seed: int) -> np.ndarray:
    """float32 [n_rays * n_steps][3]: equally spaced samples along straight rays
    through the domain [-1, 1]^3 (per ray a random axis; entry point on that
    axis' face at -1, exit point on the face at +1, the other coordinates
    uniform), in ray-major order as a ray marcher visits them."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(n_rays, 3))
    b = rng.uniform(-1.0, 1.0, size=(n_rays, 3))
    ax = rng.integers(0, 3, size=n_rays)
    a[np.arange(n_rays), ax] = -1.0
    b[np.arange(n_rays), ax] = 1.0
    t = (np.arange(n_steps) + 0.5) / n_steps
    p = a[:, None, :] + t[None, :, None] * (b - a)[:, None, :]
    return p.reshape(-1, 3).astype(np.float32)
