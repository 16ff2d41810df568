"""Pins for the oracle's adaptive precision rule (no GPU).

Expected picks are worked out by hand from eq. (3.3): u'_k = eps /
(2^(k/2) xi_k) and the largest unit roundoff not above it.
"""
import math

import numpy as np
import pytest

from oracle import assign as A
from oracle import formats as F

PAPER_SET = ("e5m2", "bf16", "fp16", "fp32")   # q52, bf16, fp16, fp32 (+ fp64)


def test_hand_worked_levels():
    # nrmAll = 1, xi = (0.1, 0.05, 0.001)
    # u'_1 = 1e-4 / (sqrt2 * 0.1)  = 7.07e-4  -> fp16 (4.88e-4); bf16 3.9e-3 too big
    # u'_2 = 1e-4 / (2 * 0.05)     = 1.0e-3   -> fp16
    # u'_3 = 1e-4 / (2sqrt2 * 1e-3)= 3.54e-2  -> bf16 (e5m2 1.25e-1 too big)
    a = A.assign(1.0, [0.01, 0.0025, 1e-6], 1e-4, PAPER_SET)
    assert a.fmt == ["fp16", "fp16", "bf16"]
    assert a.xi == pytest.approx([0.1, 0.05, 0.001], rel=1e-15)
    assert a.u_prime == pytest.approx([7.0710678e-4, 1e-3, 3.5355339e-2], rel=1e-7)
    assert not any(a.insufficient)
    # adding e4m3 (u = 2^-4 = 6.25e-2) changes nothing: still above 3.54e-2
    assert A.assign(1.0, [0.01, 0.0025, 1e-6], 1e-4, PAPER_SET + ("e4m3",)).fmt[2] == "bf16"
    # a smaller xi at level 3 admits e4m3 then e5m2
    assert A.assign(1.0, [0.01, 0.0025, 1e-8], 1e-4, ("e4m3",)).fmt[2] == "e4m3"   # u'=0.354
    assert A.assign(1.0, [0.01, 0.0025, 1e-8], 1e-4, PAPER_SET).fmt[2] == "e5m2"


def test_tie_selects_the_format():
    # level 2: 2^(k/2) = 2 exactly; xi = 0.5 -> u' = eps exactly
    eps = 2.0 ** -11
    a = A.assign(1.0, [0.0, 0.25], eps, ("fp16", "fp32"))
    assert a.u_prime[1] == eps and a.fmt[1] == "fp16"
    b = A.assign(1.0, [0.0, 0.25], math.nextafter(eps, 0), ("fp16", "fp32"))
    assert b.fmt[1] == "fp32"


def test_fallback_and_zero_xi():
    a = A.assign(1.0, [0.5, 0.0], 1e-17, ("fp32",))
    assert a.fmt[0] == "fp64" and a.insufficient[0]       # u' < 2^-53
    assert a.u_prime[1] == math.inf and a.fmt[1] == "fp32" and not a.insufficient[1]


def test_only_working_precision_when_set_empty():
    a = A.assign(1.0, [0.01, 0.01], 1e-3, ())
    assert a.fmt == ["fp64", "fp64"]


def test_rule_meets_theorem_3_1_premise():
    """Every pick satisfies u_k <= eps / (2^(k/2) xi_k) (eq. (3.3)), so
    sum_k 2^k xi_k^2 u_k^2 <= l eps^2 and eq. (3.2) reduces to (3.5)."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        depth = int(rng.integers(1, 13))
        nrm = list(10.0 ** rng.uniform(-12, -0.5, depth))
        eps = 10.0 ** rng.uniform(-12, -1)
        a = A.assign(1.0, nrm, eps, PAPER_SET + ("e4m3",))
        us = [F.FORMATS[f].u for f in a.fmt]
        for k, (x, u, bad) in enumerate(zip(a.xi, us, a.insufficient), start=1):
            if not bad:
                assert u * (2.0 ** (k / 2)) * x <= eps * (1 + 1e-15)
        s = sum(2.0 ** k * x * x * u * u for k, (x, u) in enumerate(zip(a.xi, us), 1))
        if not any(a.insufficient):
            assert s <= depth * eps * eps * (1 + 1e-12)


def test_norms_from_factors_match_dense():
    rng = np.random.default_rng(10)
    U = [rng.standard_normal((30, 4)), rng.standard_normal((20, 0))]
    V = [rng.standard_normal((25, 4)), rng.standard_normal((10, 0))]
    D = [rng.standard_normal((7, 7))]
    tot, nb = A.norms_from_factors(D, U, V)
    assert nb[0] == pytest.approx(np.sum((U[0] @ V[0].T) ** 2), rel=1e-13)
    assert nb[1] == 0.0
    assert tot == pytest.approx(np.sum(D[0] ** 2) + nb.sum(), rel=1e-14)


def test_per_block_hand_worked():
    """Per-block variant: each block's own xi in eq. (3.3)."""
    levels = [1, 1, 2, 2, 2, 2]
    nrm = [0.01, 1e-6, 0.0025, 0.0025, 1e-8, 0.0]
    a = A.assign_blocks(1.0, nrm, levels, 1e-4, PAPER_SET + ("e4m3",))
    # block 0 is its level's maximum: fp16 as in test_hand_worked_levels
    # block 1: u' = 1e-4 / (sqrt2 * 1e-3) = 7.07e-2 -> e4m3 (6.25e-2); e5m2 (0.125) too big
    # blocks 2, 3: level 2's maximum -> fp16; block 4: u' = 1e-4 / (2 * 1e-4) = 0.5 -> e5m2
    # block 5: xi = 0 -> coarsest candidate (e5m2)
    assert a.fmt == ["fp16", "e4m3", "fp16", "fp16", "e5m2", "e5m2"]
    assert a.u_prime[1] == pytest.approx(7.0710678e-2, rel=1e-7)
    assert math.isinf(a.u_prime[5])


def test_per_block_never_finer_than_its_level():
    rng = np.random.default_rng(5)
    levels = [k for k in range(1, 6) for _ in range(2 ** k)]
    for eps in (1e-2, 1e-5, 1e-9):
        nrm = rng.uniform(0, 1, len(levels)) ** 6
        tot = float(nrm.sum() * 3)
        lvl = A.assign(tot, A.level_max_norm2(nrm, levels), eps, PAPER_SET)
        blk = A.assign_blocks(tot, nrm, levels, eps, PAPER_SET)
        for f, k, v in zip(blk.fmt, levels, nrm):
            assert F.FORMATS[f].u >= F.FORMATS[lvl.fmt[k - 1]].u
            if v == max(x for x, kk in zip(nrm, levels) if kk == k):
                assert f == lvl.fmt[k - 1]
