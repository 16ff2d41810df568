"""Pins for the oracle's dense eps-HODLR construction (no GPU)."""
import numpy as np
import pytest
import scipy.linalg

from hodlr_inputs import kernels as K
from hodlr_inputs import points as Pt
from oracle import construct as C
from oracle import tree as T


def _diag_blocks(n, depth, k):
    b = T.node_bounds(n, depth)[k]
    return [(b[i], b[i + 1]) for i in range(len(b) - 1)]


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-8])
def test_lemma_2_2_every_level(eps):
    """Lemma 2.2: ||H~_ii^(k) - H_ii^(k)||_F <= eps ||H_ii^(k)||_F, k = 0..l."""
    n, depth = 600, 4
    P = Pt.uniform_1d_sorted(n, 3)
    A = K.inv_dist_reg(1e-3).dense(P)
    h = C.construct(A, depth, eps)
    Ht = C.assemble_tilde(h)
    for k in range(depth + 1):
        for a, b in _diag_blocks(n, depth, k):
            err = np.linalg.norm(Ht[a:b, a:b] - A[a:b, a:b])
            assert err <= eps * np.linalg.norm(A[a:b, a:b]) * (1 + 1e-10) + 1e-13


def test_rank_one_exactness_exp_kernel():
    """exp(-|x-y|) on sorted 1D points: every off-diagonal block is exactly
    exp(x_i) exp(-y_j) (upper) or exp(-x_i) exp(y_j) (lower), i.e. rank 1."""
    n, depth = 512, 4
    P = Pt.uniform_1d_sorted(n, 4)
    A = K.exp_neg().dense(P)
    for eps in (1e-2, 1e-8, 1e-12):
        h = C.construct(A, depth, eps)
        assert set(h.ranks) == {1}
        Ht = C.assemble_tilde(h)
        assert np.linalg.norm(Ht - A) <= 1e-13 * np.linalg.norm(A)


def test_exact_low_rank_operator_recovered():
    rng = np.random.default_rng(5)
    n, depth = 300, 3
    blks = T.blocks(n, depth)
    ranks = [int(rng.integers(0, 6)) for _ in blks]
    A = np.zeros((n, n))
    for a, m in T.leaves(n, depth):
        A[a:a + m, a:a + m] = rng.standard_normal((m, m))
    for b, p in zip(blks, ranks):
        A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols] = (
            rng.standard_normal((b.nrows, p)) @ rng.standard_normal((p, b.ncols)))
    h = C.construct(A, depth, 1e-10)
    assert h.ranks == ranks
    assert np.linalg.norm(C.assemble_tilde(h) - A) <= 1e-12 * np.linalg.norm(A)


def test_factor_convention_orthonormal_u_and_rule():
    """Eq. (3.1): U has orthonormal columns; the kept rank p is the smallest
    meeting the Frobenius rule, checked against scipy's SVD of each block."""
    n, depth, eps = 400, 3, 1e-5
    P = Pt.uniform_2d_morton(n, 6)
    A = K.gaussian(0.04, 0.01).dense(P)
    h = C.construct(A, depth, eps)
    for b, U, V in zip(h.blocks, h.U, h.V):
        p = U.shape[1]
        assert np.allclose(U.T @ U, np.eye(p), atol=1e-12)
        B = A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols]
        s = scipy.linalg.svd(B, compute_uv=False, lapack_driver="gesvd")
        nb = np.linalg.norm(B)
        tail = lambda q: np.sqrt(np.sum(s[q:] ** 2))
        assert tail(p) <= eps * nb * (1 + 1e-9)
        if p > 0:
            assert tail(p - 1) > eps * nb * (1 - 1e-9)
        assert abs(np.linalg.norm(B - U @ V.T) - tail(p)) <= 1e-12 * nb + 1e-3 * tail(p)


def test_spec_global_rule_and_zero_blocks():
    n, depth, eps = 256, 2, 1e-6
    P = Pt.uniform_1d_sorted(n, 7)
    A = K.inv_dist_reg(1e-3).dense(P)
    h = C.construct(A, depth, eps, rule="spec_global")
    a2 = np.linalg.norm(A, 2)
    for b, U, V in zip(h.blocks, h.U, h.V):
        B = A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols]
        s = np.linalg.svd(B, compute_uv=False)
        p = U.shape[1]
        assert np.all(s[:p] > eps * a2) and np.all(s[p:] <= eps * a2)
    Z = np.zeros((64, 64))
    hz = C.construct(Z, 2, 1e-3)
    assert set(hz.ranks) == {0}


def test_norms_recorded():
    n, depth = 200, 3
    P = Pt.uniform_1d_sorted(n, 8)
    A = K.log_reg(1e-4, float(n)).dense(P)
    h = C.construct(A, depth, 1e-3)
    assert h.norm2_all == pytest.approx(np.sum(A * A), rel=1e-14)
    for b, v in zip(h.blocks, h.norm2_blocks):
        B = A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols]
        assert v == pytest.approx(np.sum(B * B), rel=1e-14)
