"""Kernel functions k(p, q) and dense evaluation of blocks A[I, J].

A kernel is evaluated off the diagonal by ``offdiag(P, Q)`` on the point
coordinates, and on the diagonal (i == j, same point index) by
``diag_value`` (a constant) plus an optional ``diag_shift``.  Blocks are
addressed by half-open index ranges into the point array.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable

import numpy as np


def _dist(P, Q):
    if P.shape[1] == 1:
        return np.abs(P[:, 0][:, None] - Q[:, 0][None, :])
    d2 = (P[:, 0][:, None] - Q[:, 0][None, :]) ** 2
    d2 += (P[:, 1][:, None] - Q[:, 1][None, :]) ** 2
    return np.sqrt(d2)


def _dist2(P, Q):
    if P.shape[1] == 1:
        return (P[:, 0][:, None] - Q[:, 0][None, :]) ** 2
    d2 = (P[:, 0][:, None] - Q[:, 0][None, :]) ** 2
    d2 += (P[:, 1][:, None] - Q[:, 1][None, :]) ** 2
    return d2


@dataclass(frozen=True)
class Kernel:
    name: str
    offdiag: Callable          # (P (m,d), Q (c,d)) -> (m, c)
    diag_value: float | None   # value at i == j instead of offdiag (None: use offdiag)
    diag_shift: float = 0.0    # added at i == j
    symmetric: bool = True     # A[J, I] == A[I, J]^T
    antisymmetric: bool = False  # A[J, I] == -A[I, J]^T

    def block(self, P: np.ndarray, r0: int, r1: int, c0: int, c1: int) -> np.ndarray:
        """Dense A[r0:r1, c0:c1] in fp64."""
        B = self.offdiag(P[r0:r1], P[c0:c1])
        lo, hi = max(r0, c0), min(r1, c1)
        if lo < hi:
            idx = np.arange(lo, hi)
            if self.diag_value is not None:
                B[idx - r0, idx - c0] = self.diag_value
            B[idx - r0, idx - c0] += self.diag_shift
        return B

    def dense(self, P: np.ndarray) -> np.ndarray:
        n = len(P)
        return self.block(P, 0, n, 0, n)


def inv_dist_reg(delta: float, shift: float = 0.0) -> Kernel:
    """1 / (|p - q| + delta), plus ``shift`` on the diagonal."""
    return Kernel(f"1/(r+{delta:g})", lambda P, Q: 1.0 / (_dist(P, Q) + delta), None, shift)


def gaussian(denom: float, shift: float = 0.0) -> Kernel:
    """exp(-|p - q|^2 / denom), plus ``shift`` on the diagonal."""
    return Kernel(f"exp(-r^2/{denom:g})", lambda P, Q: np.exp(-_dist2(P, Q) / denom), None, shift)


def log_reg(delta: float, shift: float = 0.0) -> Kernel:
    """log(|p - q| + delta), plus ``shift`` on the diagonal."""
    return Kernel(f"log(r+{delta:g})", lambda P, Q: np.log(_dist(P, Q) + delta), None, shift)


def exp_neg(shift: float = 0.0) -> Kernel:
    """exp(-|p - q|)."""
    return Kernel("exp(-r)", lambda P, Q: np.exp(-_dist(P, Q)), None, shift)


# The paper's test kernels, eq. (4.1).
def paper_inverse_1d() -> Kernel:
    """(i): 1 / (x - y) off the diagonal, 1 on it (signed, 1D)."""
    def f(P, Q):
        d = P[:, 0][:, None] - Q[:, 0][None, :]
        with np.errstate(divide="ignore"):
            return np.where(d != 0, 1.0 / np.where(d != 0, d, 1.0), 1.0)
    return Kernel("1/(x-y)", f, 1.0, 0.0, symmetric=False, antisymmetric=True)


def paper_log() -> Kernel:
    """(ii): log |x_i - x_j| off the diagonal, 0 on it."""
    def f(P, Q):
        d = _dist(P, Q)
        with np.errstate(divide="ignore"):
            return np.where(d > 0, np.log(np.where(d > 0, d, 1.0)), 0.0)
    return Kernel("log r", f, 0.0, 0.0)


def paper_gaussian(h: float) -> Kernel:
    """(iii): exp(-|x_i - x_j|^2 / (2 h^2))."""
    return Kernel(f"exp(-r^2/(2*{h:g}^2))", lambda P, Q: np.exp(-_dist2(P, Q) / (2 * h * h)), None, 0.0)
