"""Error bounds of the paper and the GPU-vs-oracle tolerance (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

* ``global_bound_adaptive``: eq. (3.5) (Thm. 3.1 with rule (3.3)),
  ||H - H^||_F <~ (2 sqrt(2 l) + 1) eps ||H||_F.
* ``global_bound_given``: eq. (3.2), for arbitrary per-level precisions,
  ||H - H^||_F <~ (2 sqrt 2 (sum_k 2^k xi_k^2 u_k^2)^(1/2) + eps) ||H||_F.
* ``block_quant_bound``: eq. (3.4), per block,
  ||H~_b - H^_b||_F <= (2 + sqrt(p) u_k) u_k ||H~_b||_F.
* ``block_bound_adaptive``: eq. (3.6), per block of level k,
  ||H_b - H^_b||_F <~ (2^(1-k/2) + 1) eps ||H||_F.
* ``matvec_backward_bound``: Thm. 3.5, for working precision u <= eps/n,
  ||Delta H||_F <= 2 (sqrt 2 + 1) sqrt(2^(l+1) + 2^(l-1)) eps ||H||_F.
* ``tolerance``: componentwise acceptance bound between a computed product
  and the oracle's fp64 product, from the standard model of Sect. 1
  (gamma_n = n u / (1 - n u)): a chain of at most M rounded operations per
  output entry gives |y^ - y| <= gamma_M(u_acc) z + u_out |y| + gamma_M(2^-53) z
  with z = |H^| |x| (``matvec.matvec_abs``).
* ``tolerance_prob``: the same chain under the probabilistic model of
  rounding errors (independent, mean-zero relative errors; Higham and Mary,
  SIAM J. Sci. Comput. 41 (2019)): |y^ - y| <= lambda sqrt(M) u_acc z +
  u_out |y| + gamma_M(2^-53) z with probability at least 1 - delta for each
  of N entries when lambda = sqrt(2 log(2 M N / delta)); delta = 1e-6.
"""
from __future__ import annotations

import math

import numpy as np


def gamma(n: int, u: float) -> float:
    """gamma_n = n u / (1 - n u) (Sect. 1 notation); inf when n u >= 1."""
    nu = n * u
    return math.inf if nu >= 1 else nu / (1 - nu)


def global_bound_adaptive(depth: int, eps: float) -> float:
    return (2 * math.sqrt(2 * depth) + 1) * eps


def global_bound_given(xi, u_levels, eps: float) -> float:
    s = sum((2.0 ** k) * (x ** 2) * (u ** 2)
            for k, (x, u) in enumerate(zip(xi, u_levels), start=1))
    return 2 * math.sqrt(2) * math.sqrt(s) + eps


def block_quant_bound(p: int, u_k: float) -> float:
    return (2 + math.sqrt(p) * u_k) * u_k


def block_bound_adaptive(k: int, eps: float) -> float:
    return (2.0 ** (1 - k / 2) + 1) * eps


def matvec_backward_bound(depth: int, eps: float) -> float:
    return 2 * (math.sqrt(2) + 1) * math.sqrt(2.0 ** (depth + 1) + 2.0 ** (depth - 1)) * eps


def chain_length(blocks, ranks, leaf_sizes, depth: int) -> int:
    """M: the longest chain of rounded operations behind one output entry.

    A leaf row is an m-term dot product; a low-rank term is a c_b-term dot
    product followed by a p_b-term one; then the depth+1 terms of a row are
    summed.  So M = max(max_i m_i, max_b (c_b + p_b)) + depth + 1.
    """
    m = max([0] + list(leaf_sizes))
    for b, p in zip(blocks, ranks):
        m = max(m, b.ncols + p)
    return m + depth + 1


def tolerance(z: np.ndarray, y_ref: np.ndarray, M: int, u_acc: float,
              u_out: float) -> np.ndarray:
    """Componentwise acceptance bound (see module docstring)."""
    return gamma(M, u_acc) * z + u_out * np.abs(y_ref) + gamma(M, 2.0 ** -53) * z


def tolerance_prob(z: np.ndarray, y_ref: np.ndarray, M: int, u_acc: float, u_out: float,
                   delta: float = 1e-6) -> np.ndarray:
    """Probabilistic componentwise bound (see module docstring)."""
    N = max(1, int(np.size(z)))
    lam = math.sqrt(2.0 * math.log(2.0 * M * N / delta))
    return lam * math.sqrt(M) * u_acc * z + u_out * np.abs(y_ref) + gamma(M, 2.0 ** -53) * z
