"""Pins of the GPU-vs-oracle gate and of the paper's bounds (CPU).

Two kinds of checks:

* value pins: every bound function and every piece of the gate evaluated at
  a point where its value was worked out by hand from the paper's formula
  (Sect. 1 for gamma_n, eqs. (3.2)-(3.6), Thm. 3.5) or from the stated
  chain of rounded operations, so that a wrong constant, exponent or chain
  length fails;
* planted errors: an independent fp32 evaluation of a stored 8192-point
  operator (numpy float32 products in another summation order) must pass
  the gate, and the same evaluation with a mistake planted in the operator
  must be rejected whenever the mistake's exact effect on Y (computed by
  the oracle in fp64) clearly exceeds the gate, and accepted when it is
  clearly below it.  The gate's resolving power on this operator is
  measured and pinned in a range: at this size it is about 530 fp32 units
  of z per entry, so single-ulp changes of one generator entry are below
  it while indexing, sibling, transposition and dropped-level mistakes are
  far above it; a wrong scale of one T_b entry shows once it reaches a few
  per mille of that term (the term's share of z decides).
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from hodlr_inputs import compress as CP
from hodlr_inputs import configs as CF
from oracle import bounds as BD
from oracle import matvec as MV
from oracle import quantize as Q
from oracle import tree as T

U24 = 2.0 ** -24
U53 = 2.0 ** -53


# ---------------------------------------------------------------------------
# value pins
# ---------------------------------------------------------------------------
def test_gamma_value_pins():
    # gamma_n = n u / (1 - n u): exact rational values
    for n, u in ((10, Fr(1, 2 ** 24)), (4096, Fr(1, 2 ** 24)), (7, Fr(1, 2 ** 53)), (3, Fr(1, 8))):
        want = float(n * u / (1 - n * u))
        assert BD.gamma(n, float(u)) == pytest.approx(want, rel=1e-15)
    assert BD.gamma(8, 0.125) == math.inf          # n u = 1
    assert BD.gamma(9, 0.125) == math.inf


def test_thm_3_5_value_pins():
    # 2 (sqrt 2 + 1) sqrt(2^(l+1) + 2^(l-1)) eps; at l = 4: sqrt(32 + 8) = sqrt 40
    assert BD.matvec_backward_bound(4, 1e-4) == pytest.approx(3.0537654460671836e-3, rel=1e-14)
    # l = 1: sqrt(4 + 1) = sqrt 5
    assert BD.matvec_backward_bound(1, 1.0) == pytest.approx(2 * (2 ** 0.5 + 1) * 5 ** 0.5, rel=1e-15)
    # l = 8: sqrt(512 + 128) = 8 sqrt 10
    assert BD.matvec_backward_bound(8, 1e-6) == pytest.approx(16 * (2 ** 0.5 + 1) * 10 ** 0.5 * 1e-6, rel=1e-14)


def test_eq_3_5_and_3_6_value_pins():
    # (3.5): (2 sqrt(2 l) + 1) eps: l = 2 -> 5 eps, l = 8 -> 9 eps, l = 18 -> 13 eps
    assert BD.global_bound_adaptive(2, 1e-3) == pytest.approx(5e-3, rel=1e-15)
    assert BD.global_bound_adaptive(8, 1e-6) == pytest.approx(9e-6, rel=1e-15)
    assert BD.global_bound_adaptive(18, 1.0) == pytest.approx(13.0, rel=1e-15)
    # (3.6): (2^(1 - k/2) + 1) eps: k = 2 -> 2 eps, k = 4 -> 1.5 eps, k = 6 -> 1.25 eps, k = 1 -> (sqrt 2 + 1) eps
    assert BD.block_bound_adaptive(2, 1e-4) == pytest.approx(2e-4, rel=1e-15)
    assert BD.block_bound_adaptive(4, 1.0) == pytest.approx(1.5, rel=1e-15)
    assert BD.block_bound_adaptive(6, 1.0) == pytest.approx(1.25, rel=1e-15)
    assert BD.block_bound_adaptive(1, 1.0) == pytest.approx(2 ** 0.5 + 1, rel=1e-15)


def test_eq_3_4_value_pins():
    # (2 + sqrt(p) u) u: p = 4, u = 2^-8 -> 2^-7 + 2^-15; p = 9, u = 2^-4 -> 2^-3 + 3 * 2^-8
    assert BD.block_quant_bound(4, 2.0 ** -8) == 2.0 ** -7 + 2.0 ** -15
    assert BD.block_quant_bound(9, 2.0 ** -4) == 2.0 ** -3 + 3 * 2.0 ** -8
    assert BD.block_quant_bound(0, 2.0 ** -11) == 2.0 ** -10


def test_eq_3_2_value_pin():
    # 2 sqrt 2 (sum_k 2^k xi_k^2 u_k^2)^(1/2) + eps with xi = (1/2, 1/4),
    # u = (2^-11, 2^-8): the sum is 2^-23 + 2^-18 = 33 * 2^-23, so the first
    # term is 2 sqrt(66 * 2^-23) = 2^-10.5 sqrt 66
    got = BD.global_bound_given([0.5, 0.25], [2.0 ** -11, 2.0 ** -8], 1e-3)
    assert got == pytest.approx(2.0 ** -10.5 * 66 ** 0.5 + 1e-3, rel=1e-15)


def test_chain_length_hand_example():
    # n = 10, depth 2 (ceil split): leaves 3, 2, 3, 2; level 1 blocks have
    # 5 columns, level 2 blocks 2, 3, 2, 3 columns
    blocks = T.blocks(10, 2)
    assert [b.ncols for b in blocks] == [5, 5, 2, 3, 2, 3]
    ranks = [2, 1, 1, 2, 0, 1]
    # max(max m_i = 3, max(c_b + p_b) = 5 + 2 = 7) + depth + 1
    assert BD.chain_length(blocks, ranks, [3, 2, 3, 2], 2) == 10
    # a leaf longer than every c_b + p_b decides M
    assert BD.chain_length(blocks, ranks, [9, 1, 0, 0], 2) == 12


def test_tolerance_value_pins():
    z = np.array([1.0, 2.0, 0.0])
    y = np.array([0.5, -1.0, 3.0])
    M = 10
    g24 = float(Fr(10, 2 ** 24) / (1 - Fr(10, 2 ** 24)))
    g53 = float(Fr(10, 2 ** 53) / (1 - Fr(10, 2 ** 53)))
    want = g24 * z + U24 * np.abs(y) + g53 * z
    assert np.allclose(BD.tolerance(z, y, M, U24, U24), want, rtol=1e-14, atol=0)
    # the fp64 term alone, and the output rounding alone
    assert np.allclose(BD.tolerance(z, y, M, 0.0, 0.0), g53 * z, rtol=1e-14, atol=0)
    assert np.allclose(BD.tolerance(0 * z, y, M, U24, 2.0 ** -11), 2.0 ** -11 * np.abs(y), rtol=0, atol=0)


def test_tolerance_prob_value_pins():
    z = np.array([1.0, 2.0])
    y = np.array([0.5, -1.0])
    M = 10
    # lambda = sqrt(2 ln(2 M N / delta)) with N = 2 entries, delta = 1e-6: ln(4e7)
    lam = math.sqrt(2.0 * (math.log(4.0) + 7.0 * math.log(10.0)))
    assert lam == pytest.approx(5.916821, rel=1e-6)
    g53 = float(Fr(10, 2 ** 53) / (1 - Fr(10, 2 ** 53)))
    want = lam * math.sqrt(10) * U24 * z + U24 * np.abs(y) + g53 * z
    assert np.allclose(BD.tolerance_prob(z, y, M, U24, U24), want, rtol=1e-13, atol=0)
    # another delta and size: N = 1, M = 1000, delta = 1e-3: ln(2e6)
    lam2 = math.sqrt(2.0 * (math.log(2.0) + 6.0 * math.log(10.0)))
    got = BD.tolerance_prob(np.array([1.0]), np.array([0.0]), 1000, U24, 0.0, delta=1e-3)
    g53b = float(Fr(1000, 2 ** 53) / (1 - Fr(1000, 2 ** 53)))
    assert got[0] == pytest.approx(lam2 * math.sqrt(1000) * U24 + g53b, rel=1e-13)


def test_storage_bits_hand_sized_operator():
    # n = 8, depth 1: two 4 x 4 blocks, ranks 1 and 2
    rng = np.random.default_rng(3)
    blocks = T.blocks(8, 1)
    U = [rng.standard_normal((4, 1)), rng.standard_normal((4, 2))]
    V = [rng.standard_normal((4, 1)), rng.standard_normal((4, 2))]

    class H:
        pass
    h = H()
    h.n, h.depth, h.blocks, h.leaves, h.U, h.V = 8, 1, blocks, [np.eye(4), np.eye(4)], U, V
    # fp16 with column scales: 16 bits per code, 8 per column of each factor
    # codes: (4 + 4) * 1 + (4 + 4) * 2 = 24 codes; scaled columns: 2 * 1 + 2 * 2 = 6
    assert Q.storage_bits(Q.store(h, ["fp16"])) == 24 * 16 + 6 * 8
    assert Q.storage_bits(Q.store(h, ["fp16"], scale_columns=False)) == 24 * 16
    assert Q.storage_bits(Q.store(h, ["fp32"])) == 24 * 32        # never scaled
    assert Q.storage_bits(Q.store(h, ["e4m3"])) == 24 * 8 + 6 * 8
    assert Q.storage_bits(Q.store(h, ["fp64"])) == 24 * 64


# ---------------------------------------------------------------------------
# planted errors on a stored 8192-point operator
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def stored():
    c = CF.get("c2_s")
    blocks = T.blocks(c.n, c.depth)
    lb = T.leaves(c.n, c.depth)
    op = CP.compress(c.kernel, c.points(), [(b.row0, b.nrows, b.col0, b.ncols) for b in blocks], lb, c.eps,
                     "frob")
    U = [Q.quantize(u, "fp32").values for u in op.U]
    V = [Q.quantize(v, "fp32").values for v in op.V]
    X = c.X(1)
    y = MV.matvec(c.n, blocks, lb, op.leaves, U, V, X)
    z = MV.matvec_abs(c.n, blocks, lb, op.leaves, U, V, X)
    M = BD.chain_length(blocks, op.ranks, [m for _, m in lb], c.depth)
    return dict(c=c, blocks=blocks, lb=lb, op=op, U=U, V=V, X=X, y=y, z=z, M=M)


def fp32_eval(n, blocks, lb, leaves, U, V, X):
    """An independent evaluation as the fp32 path computes it: T_b = V^T x and
    U T_b in float32 (numpy BLAS order), summed over the levels in float32,
    plus the fp64 leaf products, rounded to float32 once."""
    x32 = X.astype(np.float32)
    acc = np.zeros(X.shape, dtype=np.float32)
    for b, u, v in zip(blocks, U, V):
        if u.shape[1] == 0:
            continue
        t = v.astype(np.float32).T @ x32[b.col0:b.col0 + b.ncols]
        acc[b.row0:b.row0 + b.nrows] += u.astype(np.float32) @ t
    w = np.zeros(X.shape)
    for (r0, m), D in zip(lb, leaves):
        w[r0:r0 + m] = D @ X[r0:r0 + m]
    return (acc + w.astype(np.float32)).astype(np.float64)


def gate(s, y_test):
    """(accepted by both gates, max |err| / tau_prob)."""
    tau = BD.tolerance(s["z"], s["y"], s["M"], U24, U24)
    taup = BD.tolerance_prob(s["z"], s["y"], s["M"], U24, U24)
    err = np.abs(y_test - s["y"])
    return bool((err <= tau).all() and (err <= taup).all()), float((err / taup).max())


def test_resolving_power_of_the_gate(stored):
    s = stored
    taup = BD.tolerance_prob(s["z"], s["y"], s["M"], U24, U24)
    nz = s["z"] > 0
    power = taup[nz] / (U24 * s["z"][nz])
    # lambda sqrt(M) plus the output rounding's share: ~530 fp32 units of z at this size
    lam = math.sqrt(2 * math.log(2 * s["M"] * s["c"].n / 1e-6))
    assert s["M"] == 4096 + max(p for p in s["op"].ranks) + s["c"].depth + 1 or s["M"] > 4096
    assert lam * math.sqrt(s["M"]) <= power.min() <= power.max() <= lam * math.sqrt(s["M"]) + 1.0 + 1e-6
    assert 400 < power.min() < 700


def test_independent_fp32_evaluation_passes(stored):
    s = stored
    ok, r = gate(s, fp32_eval(s["c"].n, s["blocks"], s["lb"], s["op"].leaves, s["U"], s["V"], s["X"]))
    assert ok, r
    assert r < 0.05           # the rounding errors of a correct fp32 evaluation sit far below the gate


def _planted(s, U=None, V=None, blocks=None, leaves=None):
    """(gate verdict on the fp32 evaluation of the planted operator, exact
    effect of the mistake on Y over tau_prob)."""
    U = s["U"] if U is None else U
    V = s["V"] if V is None else V
    blocks = s["blocks"] if blocks is None else blocks
    leaves = s["op"].leaves if leaves is None else leaves
    n = s["c"].n
    y_bad = MV.matvec(n, blocks, s["lb"], leaves, U, V, s["X"])
    taup = BD.tolerance_prob(s["z"], s["y"], s["M"], U24, U24)
    effect = float((np.abs(y_bad - s["y"]) / taup).max())
    ok, _ = gate(s, fp32_eval(n, blocks, s["lb"], leaves, U, V, s["X"]))
    return ok, effect


def _check(ok, effect):
    if effect >= 2.0:
        assert not ok, effect
    if effect <= 0.5:
        assert ok, effect


def test_one_ulp_generator_change_is_below_the_gate(stored):
    s = stored
    deepest = [i for i, b in enumerate(s["blocks"]) if b.level == s["c"].depth and s["U"][i].shape[1]]
    i = max(deepest, key=lambda k: np.abs(s["U"][k]).max())
    U = list(s["U"])
    u = U[i].copy()
    r, j = np.unravel_index(np.argmax(np.abs(u)), u.shape)
    u32 = np.float32(u[r, j])
    u[r, j] = float(np.nextafter(u32, np.float32(np.inf) if u32 > 0 else np.float32(-np.inf)))
    U[i] = u
    ok, effect = _planted(s, U=U)
    _check(ok, effect)
    assert ok and effect < 0.01


@pytest.mark.parametrize("shift,expect_reject", [(20, False), (10, False), (6, True)])
def test_scaled_t_entry(stored, shift, expect_reject):
    """T_b of the level-1 upper block, first column, times (1 + 2^-shift)
    (the effect of a wrong column scale).  That term is about 1 % of z on
    this operator (the leaf term dominates), so the gate resolves a relative
    error of it only above about 2^-7.5: 2^-10 (effect 0.22 tau) passes,
    2^-6 (3.6 tau) is rejected."""
    s = stored
    V = list(s["V"])
    v = V[0].copy()
    v[:, 0] *= 1.0 + 2.0 ** -shift
    V[0] = v
    ok, effect = _planted(s, V=V)
    _check(ok, effect)
    assert ok != expect_reject, effect


def test_dropped_rank_column(stored):
    """The last rank column of every level-1 block dropped."""
    s = stored
    U, V = list(s["U"]), list(s["V"])
    for i in (0, 1):
        U[i], V[i] = U[i][:, :-1], V[i][:, :-1]
    ok, effect = _planted(s, U=U, V=V)
    _check(ok, effect)


def test_structural_mistakes_are_rejected(stored):
    s = stored
    U, V = list(s["U"]), list(s["V"])
    cases = []
    # wrong sibling: the deepest pair's V generators exchanged
    k = len(s["blocks"]) - 2
    if V[k].shape == V[k + 1].shape:
        V2 = list(V)
        V2[k], V2[k + 1] = V[k + 1], V[k]
        cases.append(("sibling", _planted(s, V=V2)))
    # off by one row: a level-2 block's U shifted down by one row
    i = 2
    u = np.vstack([np.zeros((1, U[i].shape[1])), U[i][:-1]])
    U2 = list(U)
    U2[i] = u
    cases.append(("row shift", _planted(s, U=U2)))
    # a dropped level
    keep = [q for q, b in enumerate(s["blocks"]) if b.level != 3]
    cases.append(("dropped level", _planted(s, U=[U[q] for q in keep], V=[V[q] for q in keep],
                                            blocks=[s["blocks"][q] for q in keep])))
    # two leaves exchanged (the kernel is symmetric, so a transposed leaf would not show)
    L2 = list(s["op"].leaves)
    L2[1], L2[2] = L2[2], L2[1]
    cases.append(("exchanged leaves", _planted(s, leaves=L2)))
    # a transposed low-rank block: U and V of the level-2 lower block exchanged
    i = 4
    if U[i].shape == V[i].shape:
        U3, V3 = list(U), list(V)
        U3[i], V3[i] = V[i], U[i]
        cases.append(("transposed block", _planted(s, U=U3, V=V3)))
    for name, (ok, effect) in cases:
        assert not ok and effect > 2.0, (name, effect)
