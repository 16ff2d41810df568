"""Pins of the oracle's HODLR LU and triangular solves (CPU).

* The dense Doolittle LU equals scipy's pivoted LU where partial pivoting
  makes no exchange (a column diagonally dominant matrix), so it is the
  LU without pivoting that Alg. "HODLR_LU" asks for at the leaves.
* With no truncation (eps = 0) the recursive block LU must reproduce the
  dense LU without pivoting of the same matrix (that LU is unique), on
  several kernels, depths and uneven leaves; a sign mistake in the Schur
  complement, or a missing Schur update, breaks it.
* The triangular solves give the dense solution.
* With truncation, Cor. "LU of mixed-precision HODLR matrices" holds for
  the adaptive mixed-precision operators of several kernels and eps.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from hodlr_inputs import configs as CF
from hodlr_inputs import kernels as K
from hodlr_inputs import points as Pt
from oracle import assign as AS
from oracle import construct as C
from oracle import lu as LU
from oracle import quantize as Q
from oracle import tree as T


def _node(A, depth, eps, fmt=None):
    h = C.construct(A, depth, eps)
    if fmt is None:
        U, V = h.U, h.V
    else:
        s = Q.store(h, fmt)
        U, V = s.U, s.V
    return LU.from_stored(h.n, depth, h.blocks, h.leaves, U, V), h


def test_doolittle_equals_scipy_without_exchanges():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((40, 40))
    A += np.diag(np.abs(A).sum(axis=0) + 1.0)        # column diagonally dominant: no row exchange
    P, L, U = sl.lu(A)
    assert np.array_equal(P, np.eye(40))
    L2, U2 = LU.dense_lu(A)
    assert np.allclose(L2, L, rtol=0, atol=1e-13) and np.allclose(U2, U, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("kind,n,depth", [("exp", 300, 3), ("gauss", 256, 4), ("log", 200, 2), ("inv", 333, 3)])
def test_block_lu_without_truncation_is_the_dense_lu(kind, n, depth):
    x = Pt.uniform_1d_sorted(n, 1)
    ker = {"exp": K.exp_neg(0.5), "gauss": K.gaussian(0.04, 0.5), "log": K.log_reg(1e-3, float(n)),
           "inv": K.inv_dist_reg(1e-2, 50.0)}[kind]
    A = ker.dense(x)
    H, h = _node(A, depth, 1e-15)
    Hd = LU.to_dense(H)
    Lh, Uh = LU.hodlr_lu(H, 0.0)
    Ld, Ud = LU.dense_lu(Hd)
    Lx, Ux = LU.to_dense(Lh), LU.to_dense(Uh)
    assert np.allclose(Lx, Ld, rtol=0, atol=1e-10 * np.abs(Ld).max())
    assert np.allclose(Ux, Ud, rtol=0, atol=1e-10 * np.abs(Ud).max())
    assert np.allclose(np.triu(Lx, 1), 0) and np.allclose(np.tril(Ux, -1), 0)
    b = np.random.default_rng(3).standard_normal((n, 2))
    xs = LU.solve(Lh, Uh, b)
    assert np.allclose(xs, np.linalg.solve(Hd, b), rtol=1e-9, atol=1e-9 * np.abs(xs).max())


def test_planted_mistakes_in_the_recursion_are_caught():
    x = Pt.uniform_1d_sorted(256, 4)
    A = K.gaussian(0.04, 0.5).dense(x)
    H, _ = _node(A, 3, 1e-15)
    Ld, Ud = LU.dense_lu(LU.to_dense(H))
    good = LU.hodlr_lu
    orig = LU.subtract_lowrank
    try:
        LU.subtract_lowrank = lambda N, A_, B_, eps, stats=None: orig(N, -A_, B_, eps, stats)   # wrong sign
        Lb, Ub = good(H, 0.0)
        assert not np.allclose(LU.to_dense(Ub), Ud, atol=1e-6)
        LU.subtract_lowrank = lambda N, A_, B_, eps, stats=None: N                              # no update
        Lb, Ub = good(H, 0.0)
        assert not np.allclose(LU.to_dense(Ub), Ud, atol=1e-6)
    finally:
        LU.subtract_lowrank = orig


def test_truncation_meets_its_rule():
    rng = np.random.default_rng(5)
    A0 = rng.standard_normal((60, 12)) * np.logspace(0, -9, 12)
    B0 = rng.standard_normal((50, 12))
    for eps in (1e-2, 1e-5, 1e-8):
        U, V = LU.truncate(A0, B0, eps)
        E = A0 @ B0.T
        assert np.linalg.norm(E - U @ V.T) <= eps * np.linalg.norm(E) * (1 + 1e-12)
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)
        # the smallest such rank: one column fewer breaks the rule
        s = np.linalg.svd(E, compute_uv=False)
        p = U.shape[1]
        assert np.sqrt(np.sum(s[p - 1:] ** 2)) > eps * np.linalg.norm(E) if p > 0 else True


@pytest.mark.parametrize("name,n,depth", [("c3", 1024, 4), ("c5", 1024, 4), ("c2", 1024, 3)])
@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6, 1e-8])
def test_corollary_bound_with_mixed_precision_factors(name, n, depth, eps):
    cfg = {"c2": CF._c2, "c3": CF._c3, "c5": CF._c5}[name](n, depth)
    A = cfg.kernel.dense(cfg.points())
    h = C.construct(A, depth, eps)
    a = AS.assign(h.norm2_all, AS.level_max_norm2(h.norm2_blocks, [b.level for b in h.blocks]), eps,
                  ("fp32", "bf16", "fp16"))
    s = Q.store(h, a.fmt)
    H = LU.from_stored(h.n, depth, h.blocks, h.leaves, s.U, s.V)
    stats = {}
    Lh, Uh = LU.hodlr_lu(H, eps, stats)
    Lx, Ux = LU.to_dense(Lh), LU.to_dense(Uh)
    err = np.linalg.norm(Lx @ Ux - A)
    bound = LU.lu_backward_bound(depth, eps, np.linalg.norm(A), np.linalg.norm(Lx), np.linalg.norm(Ux))
    assert err <= bound, (err, bound)
    # the solve's backward error is of the same order
    b = np.random.default_rng(6).standard_normal(n)
    xs = LU.solve(Lh, Uh, b)
    assert np.linalg.norm(A @ xs - b) <= bound * np.linalg.norm(xs) + 1e-300


def test_corollary_bound_value_pin():
    # 2 (2^l - 1) eps ||H|| + 11 (2^l - 1) eps ||L|| ||U||: l = 3 -> 7 (2 + 11 * 6) eps with norms 1, 2, 3
    assert LU.lu_backward_bound(3, 1e-3, 1.0, 2.0, 3.0) == pytest.approx(7 * (2 + 66) * 1e-3, rel=1e-15)
