"""Adaptive precision assignment (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Follows Alg. "Adaptive-precision HODLR Format" and eq. (3.3): with
nrmAll = ||H||_F^2 and, for each level k, nrm_k the largest squared
Frobenius norm of a level-k off-diagonal block,

    xi_k = sqrt(nrm_k / nrmAll),   u'_k = eps / (2^(k/2) xi_k),
    u_k  = the largest u* <= u'_k among {u} and the allowed set,

where u is the working precision (fp64 here) and the level's generators are
stored in u_k.  Readings where the paper is silent:

* A tie u* == u'_k selects that format (the rule reads "u* <= u'").
* If no candidate satisfies u* <= u'_k (possible for deep trees), the level
  falls back to fp64 and ``insufficient[k]`` is set: the bound of Thm. 3.1
  is then not guaranteed for that level.
* If xi_k == 0 (every block of the level is zero), u'_k is +inf and the
  coarsest candidate is taken; nothing is stored for such a level anyway.
* 2^(k/2) is evaluated as sqrt(2^k) (correctly rounded), and the formula is
  evaluated left to right in fp64, so that any other implementation doing
  the same IEEE operations reaches the same decision bit for bit.

``norms_from_factors`` gives the alternative reading in which xi is taken
from the stored factors (the H~ of Thm. 3.1) instead of the original blocks.

``assign_blocks`` is the per-block variant (not in the paper's algorithm):
the same rule with each block's own norm in place of the level maximum,
xi_b = ||H_b||_F / ||H||_F and u'_b = eps / (2^(k/2) xi_b).  Since
xi_b <= xi_k, every block gets a format at least as coarse as its level's.
The proof of Thm. 3.1 bounds the error of each block separately by about
2 u_b ||H_b||_F <= 2 eps ||H||_F / 2^(k/2) and adds the squares over the
2^k blocks of each level, so the global bound (3.5) holds unchanged.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import formats as F


@dataclass
class Assignment:
    xi: list            # xi_k, k = 1..depth (index k-1)
    u_prime: list       # u'_k
    fmt: list           # chosen format name per level
    insufficient: list  # True where no candidate met u* <= u'_k


def level_max_norm2(norm2_blocks, levels) -> list:
    """nrm_k = max over the level's blocks of ||H_b||_F^2 (k = 1..depth)."""
    depth = max(levels) if len(levels) else 0
    out = [0.0] * depth
    for v, k in zip(norm2_blocks, levels):
        out[k - 1] = max(out[k - 1], float(v))
    return out


def _candidates(allowed, working):
    return sorted({F.fmt(working).name, *[F.fmt(a).name for a in allowed]},
                  key=lambda nm: F.FORMATS[nm].u)


def _choose(nrm: float, norm2_all: float, k: int, eps: float, cands):
    """(xi, u', format, insufficient) for squared norm nrm at level k."""
    xi = math.sqrt(nrm / norm2_all) if norm2_all > 0 else 0.0
    if xi == 0.0:
        up = math.inf
    else:
        up = eps / (math.sqrt(float(2 ** k)) * xi)
    ok = [c for c in cands if F.FORMATS[c].u <= up]
    if ok:
        return xi, up, max(ok, key=lambda nm: F.FORMATS[nm].u), False
    return xi, up, "fp64", True


def assign(norm2_all: float, nrm_levels, eps: float, allowed,
           working: str = "fp64") -> Assignment:
    """Alg. "Adaptive-precision HODLR Format", the per-level precision choice."""
    cands = _candidates(allowed, working)
    xis, ups, fmts, bad = [], [], [], []
    for k, nrm in enumerate(nrm_levels, start=1):
        xi, up, choice, insufficient = _choose(nrm, norm2_all, k, eps, cands)
        xis.append(xi)
        ups.append(up)
        fmts.append(choice)
        bad.append(insufficient)
    return Assignment(xis, ups, fmts, bad)


def assign_from_xi(xi_levels, eps: float, allowed, working: str = "fp64") -> Assignment:
    """The rule of Alg. "Adaptive-precision HODLR Format" from the point
    where xi_k is known: u'_k = eps / (2^(k/2) xi_k) and the largest
    candidate unit roundoff <= u'_k, for xi given per level (k = 1..depth)."""
    cands = _candidates(allowed, working)
    xis, ups, fmts, bad = [], [], [], []
    for k, xi in enumerate(xi_levels, start=1):
        xi = float(xi)
        up = math.inf if xi == 0.0 else eps / (math.sqrt(float(2 ** k)) * xi)
        ok = [c for c in cands if F.FORMATS[c].u <= up]
        xis.append(xi)
        ups.append(up)
        fmts.append(max(ok, key=lambda nm: F.FORMATS[nm].u) if ok else "fp64")
        bad.append(not ok)
    return Assignment(xis, ups, fmts, bad)


def assign_blocks(norm2_all: float, norm2_blocks, levels, eps: float, allowed,
                  working: str = "fp64") -> Assignment:
    """Per-block variant (module docstring): one entry per block, in the
    order of ``norm2_blocks`` / ``levels``."""
    cands = _candidates(allowed, working)
    xis, ups, fmts, bad = [], [], [], []
    for nrm, k in zip(norm2_blocks, levels):
        xi, up, choice, insufficient = _choose(float(nrm), norm2_all, int(k), eps, cands)
        xis.append(xi)
        ups.append(up)
        fmts.append(choice)
        bad.append(insufficient)
    return Assignment(xis, ups, fmts, bad)


def norms_from_factors(leaves, U, V):
    """||H~||_F^2 and ||U_b V_b^T||_F^2 computed from the stored fp64 factors.

    ||U V^T||_F^2 = trace(U^T U V^T V) = sum((U^T U) * (V^T V)).
    """
    nb = np.array([float(np.sum((u.T @ u) * (v.T @ v))) for u, v in zip(U, V)])
    total = float(sum(float(np.sum(d * d)) for d in leaves) + nb.sum())
    return total, nb
