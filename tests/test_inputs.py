"""The input generator's compressor against the oracle's own construction.

The compressor (``hodlr_inputs.compress``) and the oracle's construction
(``oracle.construct``) are separate implementations; on small dense cases
they must agree on ranks and on the approximated blocks, and the
randomised path must meet the same truncation rule it certifies.
"""
import numpy as np
import pytest

from hodlr_inputs import compress as CP
from hodlr_inputs import configs as CF
from hodlr_inputs import kernels as K
from hodlr_inputs import points as Pt
from oracle import construct as C
from oracle import tree as T


def _part(n, depth):
    blks = [(b.row0, b.nrows, b.col0, b.ncols) for b in T.blocks(n, depth)]
    return blks, T.leaves(n, depth)


@pytest.mark.parametrize("kern,pts", [
    (K.gaussian(0.04, 0.01), lambda n: Pt.uniform_2d_morton(n, 0)),
    (K.inv_dist_reg(1e-3), lambda n: Pt.uniform_1d_sorted(n, 0)),
    (K.paper_inverse_1d(), lambda n: Pt.grid_1d(n)),
    (K.log_reg(1e-4, 700.0), lambda n: Pt.uniform_1d_sorted(n, 0)),
])
def test_dense_path_matches_oracle(kern, pts):
    n, depth, eps = 700, 4, 1e-6
    P = pts(n)
    A = kern.dense(P)
    h = C.construct(A, depth, eps)
    blks, lv = _part(n, depth)
    op = CP.compress(kern, P, blks, lv, eps)
    assert op.ranks == h.ranks
    assert op.norm2_all == pytest.approx(h.norm2_all, rel=1e-13)
    assert np.allclose(op.norm2_blocks, h.norm2_blocks, rtol=1e-13)
    for b, U, V, Uo, Vo in zip(h.blocks, op.U, op.V, h.U, h.V):
        B = A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols]
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
        assert np.linalg.norm(U @ V.T - Uo @ Vo.T) <= 1e-9 * np.linalg.norm(B) + 1e-12
    for D, Do in zip(op.leaves, h.leaves):
        assert np.array_equal(D, Do)


@pytest.mark.parametrize("eps", [1e-3, 1e-8])
def test_randomised_path_meets_rule(eps):
    n, depth = 1500, 2
    P = Pt.uniform_2d_morton(n, 1)
    kern = K.gaussian(0.04, 0.01)
    A = kern.dense(P)
    blks, lv = _part(n, depth)
    op = CP.compress(kern, P, blks, lv, eps, dense_limit=100 * 100)
    assert any(op.sketch)
    h = C.construct(A, depth, eps)
    for (r0, nr, c0, nc), U, V, p_or in zip(blks, op.U, op.V, h.ranks):
        B = A[r0:r0 + nr, c0:c0 + nc]
        assert np.linalg.norm(B - U @ V.T) <= eps * np.linalg.norm(B) * (1 + 1e-6)
        assert abs(U.shape[1] - p_or) <= 1
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-11)


@pytest.mark.parametrize("eps", [1e-4, 1e-10])
def test_cross_approximation_path_meets_rule(eps):
    """method="aca" (used where blocks are too large to evaluate whole):
    checked here against the dense blocks, where they can be formed."""
    c = CF.get("c5_s")
    n, depth = 4096, 3
    P = c.points()[:n]
    blks, lv = _part(n, depth)
    op = CP.compress(c.kernel, P, blks, lv, eps, "frob", dense_limit=64 * 64, method="aca")
    ref = CP.compress(c.kernel, P, blks, lv, eps, "frob")
    A = c.kernel.dense(P)
    for (r0, nr, c0, nc), U, V, p_ref in zip(blks, op.U, op.V, ref.ranks):
        B = A[r0:r0 + nr, c0:c0 + nc]
        assert np.linalg.norm(B - U @ V.T) <= 1.05 * eps * np.linalg.norm(B)
        assert abs(U.shape[1] - p_ref) <= 1
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
    assert max(op.certificate) < eps


def test_spec_global_config_c1_small():
    c = CF.get("c1_s")
    P = c.points()
    blks, lv = _part(c.n, c.depth)
    A = c.kernel.dense(P)
    op = CP.compress(c.kernel, P, blks, lv, c.eps, c.rule, CF.norm_a_2(c, P))
    h = C.construct(A, c.depth, c.eps, rule="spec_global")
    assert op.ranks == h.ranks


def test_x_generation_is_seeded_and_typed():
    c = CF.get("c2_s")
    X1, X2 = c.X(3), c.X(3)
    assert np.array_equal(X1, X2)
    assert np.array_equal(X1, X1.astype(np.float32).astype(np.float64))
    assert X1.shape == (c.n, 3)
