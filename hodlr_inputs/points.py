"""Seeded point sets (numpy PCG64 via ``default_rng``)."""
from __future__ import annotations

import numpy as np


def uniform_1d_sorted(n: int, seed: int) -> np.ndarray:
    """n points uniform on [0, 1], sorted ascending; shape (n, 1)."""
    x = np.sort(np.random.default_rng(seed).uniform(0.0, 1.0, n))
    return x[:, None]


def morton_order(P: np.ndarray, bits: int = 16) -> np.ndarray:
    """Stable argsort of 2D points in [0,1]^2 by their Morton (Z-order) key.

    Coordinates are quantised to ``bits`` bits; x bits go to even key
    positions and y bits to odd ones.
    """
    q = np.minimum((P * (1 << bits)).astype(np.int64), (1 << bits) - 1)
    key = np.zeros(len(P), dtype=np.int64)
    for b in range(bits):
        key |= ((q[:, 0] >> b) & 1) << (2 * b)
        key |= ((q[:, 1] >> b) & 1) << (2 * b + 1)
    return np.argsort(key, kind="stable")


def uniform_2d_morton(n: int, seed: int) -> np.ndarray:
    """n points uniform in the unit square, in Morton order; shape (n, 2)."""
    P = np.random.default_rng(seed).uniform(0.0, 1.0, (n, 2))
    return P[morton_order(P)]


def clustered_1d(n: int, seed: int, centres=(0.2, 0.4, 0.6, 0.8), sd: float = 0.02) -> np.ndarray:
    """Equal-weight mixture of Gaussians, clipped to [0,1], sorted; (n, 1)."""
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, len(centres), n)
    x = np.clip(np.asarray(centres)[lab] + sd * rng.standard_normal(n), 0.0, 1.0)
    return np.sort(x)[:, None]


def grid_1d(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n uniform grid points on [lo, hi]; (n, 1)."""
    return np.linspace(lo, hi, n)[:, None]


def grid_2d(nx: int, ny: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """nx * ny uniform grid points on [lo,hi]^2, row by row; (nx*ny, 2)."""
    gx, gy = np.meshgrid(np.linspace(lo, hi, nx), np.linspace(lo, hi, ny), indexing="xy")
    return np.stack([gx.ravel(), gy.ravel()], axis=1)
