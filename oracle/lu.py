"""LU factorization of a HODLR matrix and the triangular solves (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Follows Alg. "HODLR_LU" (Sect. 3.4) in fp64:

* at a leaf, a dense LU factorization (no pivoting, unit lower triangular L
  as in Doolittle's method: the algorithm performs no row exchanges);
* otherwise, with H = [[H11, H12], [H21, H22]], H12 = U12 V12^T and
  H21 = U21 V21^T from the stored generators:
    L11, U11 = HODLR_LU(H11);
    U12 <- L11^-1 H12 = (L11^-1 U12) V12^T   (solve with a lower triangular
                                              HODLR matrix, one right-hand
                                              side per rank column);
    L21 <- H21 U11^-1 = U21 (U11^-T V21)^T   (solve with the transpose of an
                                              upper triangular HODLR matrix);
    S   <- H22 - L21 U12 = H22 - U21 C V12^T with C = (U11^-T V21)^T (L11^-1 U12):
          a low-rank update of the HODLR matrix H22, applied down its tree
          (leaves updated densely, each off-diagonal block's generators
          extended by the update's and then truncated);
    L22, U22 = HODLR_LU(S).
* L = [[L11, 0], [L21, L22]], U = [[U11, U12], [0, U22]].

Truncation of the Schur complement's blocks (reading of the truncation
assumption of Sect. 3.4): each block B = [U_b, -A] [V_b, B2]^T is
recompressed by QR of both factors and an SVD of the small core, keeping
the smallest rank p with (sum_{i>p} sigma_i^2)^(1/2) <= eps ||B||_F; summed
over the blocks this gives ||S^ - S~||_F <= eps ||S~||_F as the assumption
states.  eps = 0 keeps every nonzero singular value (an exact update).

Triangular solves: L X = B by forward substitution over the tree
(X1 = L11^-1 B1, B2 -= U21 (Y21^T X1), X2 = L22^-1 B2); U X = B by back
substitution; U^T X = B likewise with the transposed blocks.  The solution
of A x = b is U^-1 (L^-1 b).

``lu_backward_bound`` is Cor. "LU of mixed-precision HODLR matrices":
||L^ U^ - H||_F <~ 2 (2^l - 1) eps ||H||_F + 11 (2^l - 1) eps ||L^||_F ||U^||_F.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Node:
    """A HODLR matrix on m consecutive indices: a dense leaf, or two
    children with off-diagonal blocks H12 = U12 V12^T and H21 = U21 V21^T."""
    m: int
    dense: np.ndarray | None = None
    c1: "Node | None" = None
    c2: "Node | None" = None
    U12: np.ndarray | None = None
    V12: np.ndarray | None = None
    U21: np.ndarray | None = None
    V21: np.ndarray | None = None


def from_stored(n, depth, blocks, leaves, U, V) -> Node:
    """The tree of a stored operator (canonical block order, fp64 values)."""
    byk = {}
    for b, u, v in zip(blocks, U, V):
        byk[(b.level, b.row_node)] = (u, v)

    def build(k, j, size_from):
        if k == depth:
            D = leaves[j]
            return Node(D.shape[0], dense=np.array(D, dtype=np.float64))
        c1 = build(k + 1, 2 * j, None)
        c2 = build(k + 1, 2 * j + 1, None)
        u12, v12 = byk[(k + 1, 2 * j)]          # rows of child 1, columns of child 2
        u21, v21 = byk[(k + 1, 2 * j + 1)]
        return Node(c1.m + c2.m, c1=c1, c2=c2, U12=np.array(u12), V12=np.array(v12), U21=np.array(u21),
                    V21=np.array(v21))
    return build(0, 0, None)


def to_dense(N: Node) -> np.ndarray:
    if N.dense is not None:
        return N.dense.copy()
    m1 = N.c1.m
    out = np.zeros((N.m, N.m))
    out[:m1, :m1] = to_dense(N.c1)
    out[m1:, m1:] = to_dense(N.c2)
    out[:m1, m1:] = N.U12 @ N.V12.T
    out[m1:, :m1] = N.U21 @ N.V21.T
    return out


# ---------------------------------------------------------------------------
# dense pieces
# ---------------------------------------------------------------------------
def dense_lu(A: np.ndarray):
    """Doolittle LU without pivoting: A = L U, L unit lower triangular."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    L = np.eye(n)
    U = np.zeros_like(A)
    for k in range(n):
        U[k, k:] = A[k, k:] - L[k, :k] @ U[:k, k:]
        L[k + 1:, k] = (A[k + 1:, k] - L[k + 1:, :k] @ U[:k, k]) / U[k, k]
    return L, U


def _forward(L, B):          # L lower triangular (dense), L X = B
    X = np.array(B, dtype=np.float64)
    for i in range(L.shape[0]):
        X[i] = (X[i] - L[i, :i] @ X[:i]) / L[i, i]
    return X


def _backward(U, B):         # U upper triangular (dense), U X = B
    X = np.array(B, dtype=np.float64)
    for i in range(U.shape[0] - 1, -1, -1):
        X[i] = (X[i] - U[i, i + 1:] @ X[i + 1:]) / U[i, i]
    return X


# ---------------------------------------------------------------------------
# triangular solves with HODLR factors
# ---------------------------------------------------------------------------
def solve_lower(L: Node, B):
    """X with L X = B (L lower triangular HODLR: its U12 is empty)."""
    B = np.asarray(B, dtype=np.float64)
    if L.dense is not None:
        return _forward(L.dense, B)
    m1 = L.c1.m
    X1 = solve_lower(L.c1, B[:m1])
    B2 = B[m1:] - L.U21 @ (L.V21.T @ X1)
    return np.concatenate([X1, solve_lower(L.c2, B2)])


def solve_upper(U: Node, B):
    """X with U X = B (U upper triangular HODLR: its U21 is empty)."""
    B = np.asarray(B, dtype=np.float64)
    if U.dense is not None:
        return _backward(U.dense, B)
    m1 = U.c1.m
    X2 = solve_upper(U.c2, B[m1:])
    B1 = B[:m1] - U.U12 @ (U.V12.T @ X2)
    return np.concatenate([solve_upper(U.c1, B1), X2])


def solve_upper_t(U: Node, B):
    """X with U^T X = B: U^T is lower triangular with (2,1) block V12 U12^T."""
    B = np.asarray(B, dtype=np.float64)
    if U.dense is not None:
        return _forward(U.dense.T, B)
    m1 = U.c1.m
    X1 = solve_upper_t(U.c1, B[:m1])
    B2 = B[m1:] - U.V12 @ (U.U12.T @ X1)
    return np.concatenate([X1, solve_upper_t(U.c2, B2)])


def solve(L: Node, U: Node, b):
    """x with (L U) x = b."""
    return solve_upper(U, solve_lower(L, b))


# ---------------------------------------------------------------------------
# the Schur complement's update and truncation
# ---------------------------------------------------------------------------
def truncate(A, B, eps):
    """A B^T as U V^T with orthonormal U and the smallest rank meeting
    ||A B^T - U V^T||_F <= eps ||A B^T||_F (eps = 0: every nonzero singular
    value)."""
    m, n = A.shape[0], B.shape[0]
    if A.shape[1] == 0:
        return np.zeros((m, 0)), np.zeros((n, 0))
    Qa, Ra = np.linalg.qr(A)
    Qb, Rb = np.linalg.qr(B)
    W, s, Zt = np.linalg.svd(Ra @ Rb.T)
    if eps > 0:
        tail = np.append((s[::-1] ** 2).cumsum()[::-1], 0.0)
        p = int(np.nonzero(tail <= (eps * eps) * float(np.sum(s * s)))[0][0])
    else:
        p = int(np.count_nonzero(s > 0))
    return Qa @ W[:, :p], (Qb @ Zt[:p].T) * s[:p]


def subtract_lowrank(N: Node, A, B, eps, stats=None) -> Node:
    """The HODLR matrix N - A B^T (A, B: N.m x q), off-diagonal blocks truncated."""
    if A.shape[1] == 0:
        return N
    if N.dense is not None:
        return Node(N.m, dense=N.dense - A @ B.T)
    m1 = N.c1.m
    U12, V12 = truncate(np.hstack([N.U12, -A[:m1]]), np.hstack([N.V12, B[m1:]]), eps)
    U21, V21 = truncate(np.hstack([N.U21, -A[m1:]]), np.hstack([N.V21, B[:m1]]), eps)
    if stats is not None:
        stats["max_rank"] = max(stats.get("max_rank", 0), U12.shape[1], U21.shape[1])
    return Node(N.m, c1=subtract_lowrank(N.c1, A[:m1], B[:m1], eps, stats),
                c2=subtract_lowrank(N.c2, A[m1:], B[m1:], eps, stats), U12=U12, V12=V12, U21=U21, V21=V21)


# ---------------------------------------------------------------------------
# Alg. HODLR_LU
# ---------------------------------------------------------------------------
def hodlr_lu(H: Node, eps: float, stats=None):
    """(L, U) of the HODLR matrix H; eps truncates the Schur complements."""
    if H.dense is not None:
        L, U = dense_lu(H.dense)
        return Node(H.m, dense=L), Node(H.m, dense=U)
    L11, U11 = hodlr_lu(H.c1, eps, stats)
    X12 = solve_lower(L11, H.U12)                # U12 of U: X12 V12^T
    Y21 = solve_upper_t(U11, H.V21)              # L21 of L: U21 Y21^T
    C = Y21.T @ X12                               # L21 U12 = U21 C V12^T
    S = subtract_lowrank(H.c2, H.U21 @ C, H.V12, eps, stats)
    L22, U22 = hodlr_lu(S, eps, stats)
    z1, z2 = np.zeros((H.c1.m, 0)), np.zeros((H.c2.m, 0))
    L = Node(H.m, c1=L11, c2=L22, U12=z1, V12=z2, U21=H.U21.copy(), V21=Y21)
    U = Node(H.m, c1=U11, c2=U22, U12=X12, V12=H.V12.copy(), U21=z2, V21=z1)
    return L, U


def lu_backward_bound(depth: int, eps: float, norm_h: float, norm_l: float, norm_u: float) -> float:
    """Right-hand side of Cor. "LU of mixed-precision HODLR matrices"."""
    c = 2 ** depth - 1
    return 2 * c * eps * norm_h + 11 * c * eps * norm_l * norm_u
