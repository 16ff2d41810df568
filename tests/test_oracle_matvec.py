"""Pins for the oracle's stored operator and HODLR_MATVEC (no GPU).

* brute force: the product equals a dense multiply by the assembled H^;
* exactness: on an operator that is exactly HODLR and stored in fp64 the
  product equals A x;
* the paper's bounds: eq. (3.4) per block, (3.5) globally, (3.6) per block
  and Thm. 3.5 for the product, on the paper's own kernels (4.1);
* planted mistakes (on the CPU, in the oracle's inputs): a swapped
  generator or a dropped level is caught by the brute-force pin.
"""
import numpy as np
import pytest

from hodlr_inputs import configs as CF
from hodlr_inputs import kernels as K
from hodlr_inputs import points as Pt
from oracle import assign as AS
from oracle import bounds as BD
from oracle import construct as C
from oracle import formats as F
from oracle import matvec as MV
from oracle import quantize as Q
from oracle import tree as T


def _stored(A, depth, eps, allowed, rule="frob"):
    h = C.construct(A, depth, eps, rule)
    a = AS.assign(h.norm2_all, AS.level_max_norm2(h.norm2_blocks, [b.level for b in h.blocks]),
                  eps, allowed)
    return h, a, Q.store(h, a.fmt)


def _mv(s, X):
    lb = T.leaves(s.n, s.depth)
    return MV.matvec(s.n, s.blocks, lb, s.leaves, s.U, s.V, X)


def _dense(s):
    return MV.assemble(s.n, s.blocks, T.leaves(s.n, s.depth), s.leaves, s.U, s.V)


@pytest.mark.parametrize("cfg", ["mat1", "mat3", "c2_s"])
def test_matvec_equals_dense_product(cfg):
    c = CF.get(cfg)
    n = min(c.n, 2048)
    P = c.points()[:n] if c.n > 2048 else c.points()
    A = c.kernel.dense(P)
    _, _, s = _stored(A, min(c.depth, 6), 1e-4, c.allowed)
    X = np.random.default_rng(1).uniform(-1, 1, (n, 3))
    y = _mv(s, X)
    yd = _dense(s) @ X
    assert np.linalg.norm(y - yd) <= 1e-14 * np.linalg.norm(np.abs(_dense(s)) @ np.abs(X))


def test_matvec_abs_is_abs_dense():
    c = CF.get("mat2")
    A = c.kernel.dense(c.points())
    _, _, s = _stored(A, 5, 1e-3, c.allowed)
    X = np.random.default_rng(2).uniform(-1, 1, (c.n, 2))
    z = MV.matvec_abs(s.n, s.blocks, T.leaves(s.n, s.depth), s.leaves, s.U, s.V, X)
    # |U_b V_b^T| <= |U_b| |V_b|^T, so z dominates the dense |H^| |x|
    zd = np.abs(_dense(s)) @ np.abs(X)
    assert np.all(z >= zd * (1 - 1e-14))


def test_matvec_rows_equals_full():
    c = CF.get("c2_s")
    P = c.points()[:1024]
    A = c.kernel.dense(P)
    _, _, s = _stored(A, 4, 1e-6, c.allowed)
    X = c.X(2)[:1024]
    lb = T.leaves(s.n, s.depth)
    rows = [0, 5, 511, 512, 1023]
    full = _mv(s, X)
    part = MV.matvec_rows(rows, s.blocks, lb, s.leaves, s.U, s.V, X)
    assert np.allclose(part, full[rows], rtol=1e-14, atol=1e-14 * np.abs(full).max())


def test_exact_operator_fp64_storage_gives_ax():
    rng = np.random.default_rng(3)
    n, depth = 257, 3
    A = np.zeros((n, n))
    for a, m in T.leaves(n, depth):
        A[a:a + m, a:a + m] = rng.standard_normal((m, m))
    for b in T.blocks(n, depth):
        p = 3
        A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols] = (
            rng.standard_normal((b.nrows, p)) @ rng.standard_normal((p, b.ncols)))
    _, _, s = _stored(A, depth, 1e-12, ())
    x = rng.standard_normal(n)
    assert np.linalg.norm(_mv(s, x) - A @ x) <= 1e-13 * np.linalg.norm(np.abs(A) @ np.abs(x))


@pytest.mark.parametrize("cfg", ["mat1", "mat2", "mat3", "mat4"])
@pytest.mark.parametrize("eps", [1e-2, 1e-5, 1e-8])
def test_paper_bounds_on_paper_kernels(cfg, eps):
    """Eqs. (3.4), (3.5), (3.6) and Thm. 3.5 on kernels (4.1), n=2000, l=8."""
    c = CF.get(cfg)
    A = c.kernel.dense(c.points())
    h, a, s = _stored(A, c.depth, eps, c.allowed)
    nA = np.sqrt(h.norm2_all)
    Hh = _dense(s)
    # (3.5) global representation error
    assert np.linalg.norm(A - Hh) <= BD.global_bound_adaptive(c.depth, eps) * nA
    for b, U, V, QU, QV in zip(h.blocks, h.U, h.V, s.QU, s.QV):
        k = b.level
        Bt = U @ V.T
        Bh = QU.values @ QV.values.T
        uk = F.FORMATS[a.fmt[k - 1]].u
        # (3.4) quantisation of one block
        assert np.linalg.norm(Bt - Bh) <= BD.block_quant_bound(U.shape[1], uk) * np.linalg.norm(Bt) + 1e-300
        # (3.6) block error against the original
        B = A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols]
        assert np.linalg.norm(B - Bh) <= BD.block_bound_adaptive(k, eps) * nA
    # Thm 3.5: fp64 working precision satisfies u <= eps / n
    assert 2.0 ** -53 <= eps / c.n
    X = c.X(4)
    Y = _mv(s, X)
    for j in range(X.shape[1]):
        eta = np.linalg.norm(Y[:, j] - A @ X[:, j]) / (nA * np.linalg.norm(X[:, j]))
        assert eta <= BD.matvec_backward_bound(c.depth, eps)


@pytest.mark.parametrize("cfg", ["mat1", "mat2", "mat3", "mat4"])
def test_per_block_variant_keeps_paper_bounds(cfg):
    """Per-block formats (``assign_blocks``): eq. (3.4) per block with the
    block's own u_b, eq. (3.5) globally and Thm 3.5 still hold, and the
    stored generators never take more bits than with one format per level."""
    c = CF.get(cfg)
    A = c.kernel.dense(c.points())
    nA = None
    for eps in (1e-2, 1e-5):
        h = C.construct(A, c.depth, eps)
        nA = np.sqrt(h.norm2_all)
        levels = [b.level for b in h.blocks]
        blk = AS.assign_blocks(h.norm2_all, h.norm2_blocks, levels, eps, c.allowed)
        lvl = AS.assign(h.norm2_all, AS.level_max_norm2(h.norm2_blocks, levels), eps, c.allowed)
        s = Q.store_blocks(h, blk.fmt)
        assert np.linalg.norm(A - _dense(s)) <= BD.global_bound_adaptive(c.depth, eps) * nA
        for b, U, V, QU, QV, f in zip(h.blocks, h.U, h.V, s.QU, s.QV, blk.fmt):
            Bt = U @ V.T
            Bh = QU.values @ QV.values.T
            assert np.linalg.norm(Bt - Bh) <= BD.block_quant_bound(U.shape[1], F.FORMATS[f].u) * \
                np.linalg.norm(Bt) + 1e-300
            B = A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols]
            assert np.linalg.norm(B - Bh) <= BD.block_bound_adaptive(b.level, eps) * nA
        X = c.X(2)
        Y = _mv(s, X)
        for j in range(X.shape[1]):
            eta = np.linalg.norm(Y[:, j] - A @ X[:, j]) / (nA * np.linalg.norm(X[:, j]))
            assert eta <= BD.matvec_backward_bound(c.depth, eps)
        assert Q.storage_bits(s) <= Q.storage_bits(Q.store(h, lvl.fmt))


def test_eq_3_2_bound_for_forced_precisions():
    """Eq. (3.2) holds for any per-level precisions (Alg. "Mixed-precision
    HODLR Format"), here every level forced to bf16."""
    c = CF.get("mat3")
    A = c.kernel.dense(c.points())
    h = C.construct(A, c.depth, 1e-6)
    s = Q.store(h, ["bf16"] * c.depth)
    nA = np.sqrt(h.norm2_all)
    lvl = AS.level_max_norm2(h.norm2_blocks, [b.level for b in h.blocks])
    xi = [np.sqrt(v / h.norm2_all) for v in lvl]
    bound = BD.global_bound_given(xi, [F.BF16.u] * c.depth, 1e-6)
    assert np.linalg.norm(A - _dense(s)) <= bound * nA


def test_planted_mistakes_are_caught():
    c = CF.get("mat3")
    A = c.kernel.dense(c.points())
    _, _, s = _stored(A, 4, 1e-6, c.allowed)
    X = np.random.default_rng(4).uniform(-1, 1, (c.n, 1))
    good = _dense(s) @ X
    lb = T.leaves(s.n, s.depth)
    # swap the V generators of the first sibling pair (upper <-> lower roles)
    V = list(s.V)
    V[0], V[1] = V[1], V[0]
    bad1 = MV.matvec(s.n, s.blocks, lb, s.leaves, s.U, V, X) if V[0].shape == V[1].shape else None
    # drop the deepest level
    keep = [i for i, b in enumerate(s.blocks) if b.level < s.depth]
    bad2 = MV.matvec(s.n, [s.blocks[i] for i in keep], lb, s.leaves,
                     [s.U[i] for i in keep], [s.V[i] for i in keep], X)
    tol = 1e-12 * np.linalg.norm(good)
    if bad1 is not None:
        assert np.linalg.norm(bad1 - good) > tol
    assert np.linalg.norm(bad2 - good) > tol
