"""HODLR matrix-vector product in a low working precision (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Alg. "HODLR_MATVEC" computed in a working precision W (bf16 or fp16): the
setting of Thm. 3.5 and of the Sect. 4 matrix-vector experiment, where the
working precision u is swept (fp64, fp32, bf16) against the approximation
parameter eps.  Reading taken here (the paper simulates each operation
rounded to u; matrix cores round the operands and sum in fp32), the model
of a W product with fp32 accumulation:

* X is given in W;
* the leaf D_i enters as round_W(D_i);
* a stored generator enters as round_W of its code value (the stored value
  times 2^e_j, i.e. before the column scale is taken off);
* T_b = round_W(2^(-e^V_j - e^U_j) sum_r round_W(V code)_rj x_r): the
  column scales of V_b and U_b are folded into T_b, which is rounded once;
* y = round_W(D_i^W x_i + sum_b U_b^W T_b), rounded once at the end.

The sums here are exact up to fp64 rounding (products of two W numbers are
exact in fp64); the device's fp32 sums are accounted for by
``tolerance``, which also allows T_b to land one W quantum away (its
rounding decision follows an fp32 sum).  ``matvec_lowp`` returns the value
before the final rounding of y and the magnitudes the tolerance needs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import formats as F
from .bounds import gamma


@dataclass
class LowpProduct:
    y: np.ndarray       # D^W x + sum_b U_b^W T_b (exact sums), before the final rounding
    zl: np.ndarray      # |D^W| |x| + sum_b |U_b^W| |T_b|: terms of the final fp32 sum
    zt: np.ndarray      # sum_b |U_b^W| |T_b|: where T_b's rounding enters
    zv: np.ndarray      # sum_b |U_b^W| (scale_b |V_b^W|^T |x|): the contraction sums
    T: list             # T_b per block (rounded to W)


def _code_values(q) -> np.ndarray:
    """The stored code values of a quantised factor (value times 2^e_j)."""
    return F.decode(q.fmt, q.codes)


def matvec_lowp(n, blocks, leaves_bounds, leaves, QU, QV, X, w: str) -> LowpProduct:
    """The product of the module docstring for ``X`` (n x nrhs, values in W).

    ``QU``, ``QV``: the stored generators per block (``quantize.QFactor``),
    ``leaves``: fp64 D_i, ``leaves_bounds``: (start, size) per leaf.
    """
    W = F.fmt(w)
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    assert np.array_equal(F.round_rne(W, X), X), "X must hold W values"
    y = np.zeros((n, X.shape[1]))
    zl = np.zeros_like(y)
    zt = np.zeros_like(y)
    zv = np.zeros_like(y)
    Ts = []
    for blk, qu, qv in zip(blocks, QU, QV):
        r = slice(blk.row0, blk.row0 + blk.nrows)
        c = slice(blk.col0, blk.col0 + blk.ncols)
        Uw = F.round_rne(W, _code_values(qu))
        Vw = F.round_rne(W, _code_values(qv))
        scale = np.ldexp(1.0, -(np.asarray(qv.exps, dtype=np.int64) + np.asarray(qu.exps, dtype=np.int64)))
        s = Vw.T @ X[c]
        T = F.round_rne(W, s * scale[:, None])
        Ts.append(T)
        y[r] += Uw @ T
        zl[r] += np.abs(Uw) @ np.abs(T)
        zt[r] += np.abs(Uw) @ np.abs(T)
        zv[r] += np.abs(Uw) @ (scale[:, None] * (np.abs(Vw).T @ np.abs(X[c])))
    for (a, m), D in zip(leaves_bounds, leaves):
        Dw = F.round_rne(W, D)
        y[a:a + m] += Dw @ X[a:a + m]
        zl[a:a + m] += np.abs(Dw) @ np.abs(X[a:a + m])
    if vec:
        y, zl, zt, zv = y[:, 0], zl[:, 0], zt[:, 0], zv[:, 0]
    return LowpProduct(y, zl, zt, zv, Ts)


def tolerance(prod: LowpProduct, w: str, M: int, C: int) -> np.ndarray:
    """Componentwise bound on |y_W - y| for a device result y_W.

    With u = u_W, v = 2^-24 (fp32 sums), M the longest chain of the final
    sum (``bounds.chain_length``) and C the longest contraction sum:

    * the contraction sum s_b carries at most gamma_C(v) |V^W|^T |x|, so
      the two sides round values at most gamma_C(v) scale |V^W|^T |x|
      apart, and their roundings to W differ by at most that plus
      u |T| on each side: |dT| <= 2u |T| + (1 + 2u) gamma_C(v) zv-terms;
    * the final fp32 sum adds gamma_M(v) (zl + |U^W| |dT|);
    * the final rounding adds u |y_W| <= u (|y| + the above);
    * fp64 sums on the oracle side, gamma_M(2^-53) zl.
    """
    u = F.fmt(w).u
    v = F.FP32.u
    dT = 2.0 * u * prod.zt + (1.0 + 2.0 * u) * gamma(C, v) * prod.zv
    e = dT + gamma(M, v) * (prod.zl + dT)
    return (1.0 + u) * e + u * np.abs(prod.y) + gamma(M, 2.0 ** -53) * prod.zl


def round_result(prod: LowpProduct, w: str) -> np.ndarray:
    """y rounded once to W (the oracle's own W result)."""
    return F.round_rne(F.fmt(w), prod.y, check_overflow=False)
