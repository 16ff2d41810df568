"""HODLR matrix-vector product (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Follows Alg. "HODLR_MATVEC": b <- 0; for every level k and sibling pair i,
b_{2i-1} += U_{2i-1} (V_{2i}^T x_{2i}) and b_{2i} += U_{2i} (V_{2i-1}^T
x_{2i-1}); then every leaf adds H_ii x_i.  Everything is done in fp64 on
the stored (dequantised) values, in the algorithm's order.  Several right-
hand sides are treated column by column (the algorithm is stated for one
vector; the block form below is the same arithmetic per column).

``matvec_abs`` is the same loop on absolute values, z = |H^| |x| evaluated
blockwise (|D| |x| + sum |U| (|V|^T |x|)), used by the componentwise
tolerance.  ``assemble`` builds the dense stored operator H^ so the product
can be checked against a plain dense multiply.
"""
from __future__ import annotations

import numpy as np


def _as2d(X):
    X = np.asarray(X, dtype=np.float64)
    return (X[:, None], True) if X.ndim == 1 else (X, False)


def matvec(n, blocks, leaves_bounds, leaves, U, V, X) -> np.ndarray:
    """b = H^ X by Alg. "HODLR_MATVEC" (fp64).

    ``blocks``: canonical block list (oracle.tree.Block); ``leaves_bounds``:
    (start, size) per leaf; ``leaves``: fp64 D_i; ``U``/``V``: dequantised
    generators per block.
    """
    X, vec = _as2d(X)
    b = np.zeros((n, X.shape[1]))
    for blk, Ub, Vb in zip(blocks, U, V):
        r = slice(blk.row0, blk.row0 + blk.nrows)
        c = slice(blk.col0, blk.col0 + blk.ncols)
        b[r] += Ub @ (Vb.T @ X[c])
    for (a, m), D in zip(leaves_bounds, leaves):
        b[a:a + m] += D @ X[a:a + m]
    return b[:, 0] if vec else b


def matvec_abs(n, blocks, leaves_bounds, leaves, U, V, X) -> np.ndarray:
    """z = |D||x| + sum_b |U_b| (|V_b|^T |x|), blockwise, fp64."""
    return matvec(n, blocks, leaves_bounds, [np.abs(d) for d in leaves],
                  [np.abs(u) for u in U], [np.abs(v) for v in V], np.abs(X))


def assemble(n, blocks, leaves_bounds, leaves, U, V) -> np.ndarray:
    """Dense n x n matrix with the leaves on the diagonal and U_b V_b^T off it."""
    H = np.zeros((n, n))
    for (a, m), D in zip(leaves_bounds, leaves):
        H[a:a + m, a:a + m] = D
    for blk, Ub, Vb in zip(blocks, U, V):
        H[blk.row0:blk.row0 + blk.nrows, blk.col0:blk.col0 + blk.ncols] = Ub @ Vb.T
    return H


def matvec_rows(rows, blocks, leaves_bounds, leaves, U, V, X, *, absolute=False):
    """Selected rows of H^ X (or of |H^| |X|), each computed on its own.

    Row r receives, from each level, the row of U_b of the block whose rows
    contain r times V_b^T x_cols, plus the row of its leaf times x_leaf: the
    same sum as Alg. "HODLR_MATVEC" restricted to one output entry.  Used to
    check full-size results on a sample of rows.
    """
    X, vec = _as2d(X)
    ab = np.abs if absolute else (lambda a: a)
    Xa = ab(X)
    out = np.zeros((len(rows), X.shape[1]))
    # T_b per block, computed once
    cache = {}
    for t, r in enumerate(rows):
        acc = np.zeros(X.shape[1])
        for bi, blk in enumerate(blocks):
            if blk.row0 <= r < blk.row0 + blk.nrows:
                if bi not in cache:
                    c = slice(blk.col0, blk.col0 + blk.ncols)
                    cache[bi] = ab(V[bi]).T @ Xa[c]
                acc += ab(U[bi][r - blk.row0]) @ cache[bi]
        for (a, m), D in zip(leaves_bounds, leaves):
            if a <= r < a + m:
                acc += ab(D[r - a]) @ Xa[a:a + m]
        out[t] = acc
    return out[:, 0] if vec else out
