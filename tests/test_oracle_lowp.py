"""Pins for the oracle's product in a low working precision (no GPU).

* brute force: on an operator whose every value and partial sum is exact in
  bf16 (small integers), the W product equals a dense multiply built here
  from the blocks, with no rounding anywhere;
* a hand-worked case where the rounding of T_b decides the result (ties to
  even), so a dropped, moved or extra rounding point fails;
* the paper's Sect. 4 observation on the matrix-vector backward error: the
  finite-precision error of a working precision u dominates until eps
  reaches about u, and the approximation error dominates beyond (mat-1 and
  mat-3, bf16 and fp16 against fp64);
* the tolerance holds between the oracle's W result and a second,
  independently ordered evaluation of the same model with fp32 sums.
"""
import numpy as np
import pytest

from hodlr_inputs import configs as CF
from oracle import assign as AS
from oracle import bounds as BD
from oracle import construct as C
from oracle import formats as F
from oracle import lowp as LP
from oracle import matvec as MV
from oracle import quantize as Q
from oracle import tree as T


def _integer_operator(n, depth, rank, seed):
    rng = np.random.default_rng(seed)
    blocks = T.blocks(n, depth)
    lb = T.leaves(n, depth)
    leaves = [rng.integers(-1, 2, (m, m)).astype(np.float64) for _, m in lb]
    U = [rng.integers(-1, 2, (b.nrows, rank)).astype(np.float64) for b in blocks]
    V = [rng.integers(-1, 2, (b.ncols, rank)).astype(np.float64) for b in blocks]
    return blocks, lb, leaves, U, V


@pytest.mark.parametrize("w", ["bf16", "fp16"])
def test_exact_on_integer_operator(w):
    n, depth, rank = 64, 2, 2
    blocks, lb, leaves, U, V = _integer_operator(n, depth, rank, 3)
    QU = [Q.quantize(u, "fp32") for u in U]
    QV = [Q.quantize(v, "fp32") for v in V]
    X = np.random.default_rng(4).integers(-1, 2, (n, 3)).astype(np.float64)
    # dense operator from the blocks, by hand
    A = np.zeros((n, n))
    for (a, m), D in zip(lb, leaves):
        A[a:a + m, a:a + m] = D
    for b, u, v in zip(blocks, U, V):
        A[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols] = u @ v.T
    # every |T| <= 32 and |y| <= 16 + 2 * 2 * 32: integers exact in bf16 and fp16
    prod = LP.matvec_lowp(n, blocks, lb, leaves, QU, QV, X, w)
    assert np.array_equal(prod.y, A @ X)
    assert np.array_equal(LP.round_result(prod, w), A @ X)


def test_rounding_of_T_hand_worked():
    """n = 4, depth 1, zero leaves, U_b = (1, 0)^T, V_b = (1, 1)^T for both
    blocks, x = (1, 2^-8, 1, 2^-8).  In fp64 each T_b = 1 + 2^-8 and
    y = (1 + 2^-8, 0, 1 + 2^-8, 0).  In bf16 (8 significand bits, spacing
    2^-7 above 1) 1 + 2^-8 is halfway between 1 and 1 + 2^-7; ties to even
    give T_b = 1 and y = (1, 0, 1, 0).  In fp16 (11 bits) 1 + 2^-8 is exact."""
    blocks = T.blocks(4, 1)
    lb = T.leaves(4, 1)
    leaves = [np.zeros((2, 2)), np.zeros((2, 2))]
    QU = [Q.quantize(np.array([[1.0], [0.0]]), "fp32") for _ in blocks]
    QV = [Q.quantize(np.array([[1.0], [1.0]]), "fp32") for _ in blocks]
    x = np.array([1.0, 2.0 ** -8, 1.0, 2.0 ** -8])
    y16 = LP.round_result(LP.matvec_lowp(4, blocks, lb, leaves, QU, QV, x, "bf16"), "bf16")
    assert np.array_equal(y16, [1.0, 0.0, 1.0, 0.0])
    yh = LP.round_result(LP.matvec_lowp(4, blocks, lb, leaves, QU, QV, x, "fp16"), "fp16")
    assert np.array_equal(yh, [1.0 + 2.0 ** -8, 0.0, 1.0 + 2.0 ** -8, 0.0])
    y64 = MV.matvec(4, blocks, lb, leaves, [q.values for q in QU], [q.values for q in QV], x)
    assert np.array_equal(y64, [1.0 + 2.0 ** -8, 0.0, 1.0 + 2.0 ** -8, 0.0])


def _backward_errors(A, cfg, eps, X):
    h = C.construct(A, cfg.depth, eps)
    a = AS.assign(h.norm2_all, AS.level_max_norm2(h.norm2_blocks, [b.level for b in h.blocks]), eps,
                  cfg.allowed)
    s = Q.store(h, a.fmt)
    lb = T.leaves(s.n, s.depth)
    nA = np.sqrt(h.norm2_all)

    def eta(Y, Xs):
        return np.mean([np.linalg.norm(Y[:, j] - A @ Xs[:, j]) / (nA * np.linalg.norm(Xs[:, j]))
                        for j in range(Xs.shape[1])])
    out = {"fp64": eta(MV.matvec(s.n, s.blocks, lb, s.leaves, s.U, s.V, X), X)}
    for w in ("bf16", "fp16"):
        Xw = F.round_rne(w, X)
        pr = LP.matvec_lowp(s.n, s.blocks, lb, s.leaves, s.QU, s.QV, Xw, w)
        out[w] = eta(LP.round_result(pr, w), Xw)
    return out


@pytest.mark.parametrize("cfg", ["mat3", "mat1"])
def test_working_precision_crossover(cfg):
    """Sect. 4: with working precision u the backward error is the finite-
    precision one (well above fp64's, at most u) while eps << u, and the
    approximation one (that of fp64) once eps >> u; u_bf16 = 2^-8 ~ 3.9e-3,
    u_fp16 = 2^-11 ~ 4.9e-4 (Table 1.1)."""
    c = CF.get(cfg)
    A = c.kernel.dense(c.points())
    X = np.random.default_rng(0).uniform(-1, 1, (c.n, 3))
    e = {eps: _backward_errors(A, c, eps, X) for eps in (1e-8, 1e-4, 1e-3, 1e-1)}
    for w in ("bf16", "fp16"):
        u = F.fmt(w).u
        assert e[1e-8][w] > 100 * e[1e-8]["fp64"]         # finite precision dominates
        assert e[1e-8][w] <= u
        assert e[1e-1][w] <= 1.1 * e[1e-1]["fp64"]       # approximation dominates
    assert e[1e-3]["bf16"] > 2 * e[1e-3]["fp64"]          # eps = 1e-3 < u_bf16: still bf16's
    assert e[1e-4]["fp16"] > 2 * e[1e-4]["fp64"]          # eps = 1e-4 < u_fp16: still fp16's


def test_tolerance_covers_fp32_sums():
    """The device sums in fp32 in its own order; an fp32 evaluation of the
    same model (contraction and final sums in float32, left to right per
    block and leaf) stays inside ``tolerance`` of the oracle's result."""
    c = CF.get("c2_s")
    A = c.kernel.dense(c.points())
    h = C.construct(A, 3, 1e-4)
    s = Q.store(h, ["bf16", "fp16", "e4m3"])
    lb = T.leaves(s.n, s.depth)
    w = "bf16"
    X = F.round_rne(w, np.random.default_rng(5).standard_normal((s.n, 4)))
    pr = LP.matvec_lowp(s.n, s.blocks, lb, s.leaves, s.QU, s.QV, X, w)
    y32 = np.zeros((s.n, 4), dtype=np.float32)
    for b, qu, qv in zip(s.blocks, s.QU, s.QV):
        Uw = F.round_rne(w, F.decode(qu.fmt, qu.codes)).astype(np.float32)
        Vw = F.round_rne(w, F.decode(qv.fmt, qv.codes)).astype(np.float32)
        scale = np.ldexp(1.0, -(qv.exps + qu.exps))
        sums = (Vw.T @ X[b.col0:b.col0 + b.ncols].astype(np.float32)).astype(np.float64)
        Tb = F.round_rne(w, sums * scale[:, None]).astype(np.float32)
        y32[b.row0:b.row0 + b.nrows] += Uw @ Tb
    for (a, m), D in zip(lb, s.leaves):
        y32[a:a + m] += F.round_rne(w, D).astype(np.float32) @ X[a:a + m].astype(np.float32)
    yw = F.round_rne(w, y32.astype(np.float64))
    M = BD.chain_length(s.blocks, [q.codes.shape[1] for q in s.QU], [m for _, m in lb], s.depth)
    Cl = max(b.ncols for b in s.blocks)
    tol = LP.tolerance(pr, w, M, Cl)
    assert (np.abs(yw - pr.y) <= tol).all()
    # a rounding error far above u_W is not tolerated
    assert not (np.abs((yw * (1 + 64 * F.fmt(w).u)) - pr.y) <= tol).all()
