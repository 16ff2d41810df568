"""Dense construction of an eps-HODLR matrix by truncated SVD (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Follows:
* Def. 2.3: every off-diagonal block of the approximation is within relative
  eps of the original block.
* Eq. (3.1): the block is stored as U V^T with U having orthonormal columns;
  V carries the singular values (U = W_p, V = Z_p Sigma_p for B = W Sigma Z^T).
* Sect. 4: blocks are truncated with an SVD and a user-given eps.
* Alg. "Mixed-precision HODLR Format": the leaves are the original diagonal
  blocks, kept in the working precision (fp64).

Truncation rules (the paper fixes eps but not the norm; readings):
* ``"frob"`` (default): the smallest p with
  (sum_{i>p} sigma_i^2)^(1/2) <= eps * ||B||_F, which makes Lemma 2.2 hold
  exactly in the Frobenius norm.
* ``"spec_global"``: keep sigma_i > eps * ||A||_2 (a threshold relative to
  the whole matrix in the 2-norm).

The whole matrix is materialised, so this is for small n only.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import tree as _tree


@dataclass
class Hodlr:
    """An eps-HODLR matrix in factored fp64 form plus the norms Alg. 3.2 needs."""
    n: int
    depth: int
    bounds: list                    # node_bounds(n, depth)
    blocks: list                    # tree.Block, canonical order
    leaves: list                    # fp64 D_i, m_i x m_i
    U: list                         # fp64 r_b x p_b, orthonormal columns
    V: list                         # fp64 c_b x p_b
    norm2_all: float = 0.0          # ||A||_F^2
    norm2_blocks: np.ndarray = field(default_factory=lambda: np.zeros(0))  # ||A_b||_F^2

    @property
    def ranks(self):
        return [u.shape[1] for u in self.U]


def truncation_rank(s: np.ndarray, eps: float, rule: str, norm_b_f: float,
                    norm_a_2: float | None = None) -> int:
    """Rank kept from singular values ``s`` (descending) under ``rule``."""
    if s.size == 0:
        return 0
    if rule == "frob":
        # tails[p] = sqrt(sum_{i >= p} s_i^2), summed smallest first
        sq = (s[::-1] ** 2).cumsum()[::-1]
        tails = np.sqrt(np.append(sq, 0.0))
        thr = eps * norm_b_f
        for p in range(s.size + 1):
            if tails[p] <= thr:
                return p
        return s.size
    if rule == "spec_global":
        if norm_a_2 is None:
            raise ValueError("spec_global needs ||A||_2")
        return int(np.count_nonzero(s > eps * norm_a_2))
    raise ValueError(f"unknown truncation rule {rule!r}")


def construct(A: np.ndarray, depth: int, eps: float, rule: str = "frob",
              leaf_bounds=None) -> Hodlr:
    """Compress every off-diagonal block of dense ``A`` (Def. 2.3, eq. (3.1))."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    nb = _tree.node_bounds(n, depth, leaf_bounds)
    blks = _tree.blocks(n, depth, leaf_bounds)
    norm_a_2 = float(np.linalg.norm(A, 2)) if rule == "spec_global" else None
    Us, Vs, nb2 = [], [], []
    for b in blks:
        B = A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols]
        nrm2 = float(np.sum(B * B))
        nb2.append(nrm2)
        if B.size == 0:
            Us.append(np.zeros((b.nrows, 0)))
            Vs.append(np.zeros((b.ncols, 0)))
            continue
        W, s, Zt = np.linalg.svd(B, full_matrices=False)
        p = truncation_rank(s, eps, rule, np.sqrt(nrm2), norm_a_2)
        Us.append(np.ascontiguousarray(W[:, :p]))
        Vs.append(np.ascontiguousarray(Zt[:p].T * s[:p]))
    lv = [A[a:a + m, a:a + m].copy() for a, m in _tree.leaves(n, depth, leaf_bounds)]
    return Hodlr(n, depth, nb, blks, lv, Us, Vs, float(np.sum(A * A)), np.array(nb2))


def assemble_tilde(h: Hodlr) -> np.ndarray:
    """Dense H~ from the fp64 factors and leaves (before any rounding)."""
    H = np.zeros((h.n, h.n))
    for (a, m), D in zip(_tree.leaves(h.n, h.depth, h.bounds[h.depth]), h.leaves):
        H[a:a + m, a:a + m] = D
    for b, U, V in zip(h.blocks, h.U, h.V):
        H[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols] = U @ V.T
    return H
