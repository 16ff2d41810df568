"""Storing each level's generators in its assigned precision (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Follows Alg. "Mixed-precision HODLR Format" / "Adaptive-precision HODLR
Format": the generators U_b, V_b of a level-k block are stored in u_k and
the leaves in the working precision; the stored values are cast back to
the working precision when used (Sect. 3.3, casting on the fly).

Reading (not in the paper): for the narrow formats (fp16, e4m3, e5m2) each
column j of a factor is first multiplied by 2^e_j, the largest power of two
that keeps the column's largest magnitude within the format's range
(``formats.column_scale_exponent``); the stored value is
round(F[:, j] * 2^e_j) and its fp64 meaning is decode(code) * 2^-e_j.
Power-of-2 scaling changes no relative error, so the per-element model
behind eq. (3.4) still holds.  Without scaling, a value that overflows the
format raises ``formats.OverflowInFormat``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import formats as F


@dataclass
class QFactor:
    fmt: str
    codes: np.ndarray     # rows x p unsigned bit patterns
    exps: np.ndarray      # p int column exponents (zeros when unscaled)
    values: np.ndarray    # rows x p fp64: decode(codes) * 2^-exps
    scaled: bool = False  # True when the columns carry stored exponents


def quantize(Fm: np.ndarray, fmt: str, scale_columns: bool = True) -> QFactor:
    Fm = np.asarray(Fm, dtype=np.float64)
    f = F.fmt(fmt)
    p = Fm.shape[1]
    scaled = bool(scale_columns and f.name in F.SCALED)
    if scaled and Fm.size:
        exps = F.column_scale_exponent(f, np.abs(Fm).max(axis=0))
    else:
        exps = np.zeros(p, dtype=np.int64)
    shifted = np.ldexp(Fm, exps[None, :]) if p else Fm
    r = F.round_rne(f, shifted)
    codes = F.encode(f, r)
    values = np.ldexp(F.decode(f, codes), -exps[None, :]) if p else r
    return QFactor(f.name, codes, exps, values, scaled)


@dataclass
class StoredHodlr:
    """The stored operator H^: fp64 leaves plus quantised generators."""
    n: int
    depth: int
    blocks: list
    leaves: list
    level_fmt: list       # per level k = 1..depth
    QU: list
    QV: list

    @property
    def U(self):
        return [q.values for q in self.QU]

    @property
    def V(self):
        return [q.values for q in self.QV]


def store(h, level_fmt, scale_columns: bool = True) -> StoredHodlr:
    """Quantise every block's generators in its level's format."""
    QU, QV = [], []
    for b, U, V in zip(h.blocks, h.U, h.V):
        f = level_fmt[b.level - 1]
        QU.append(quantize(U, f, scale_columns))
        QV.append(quantize(V, f, scale_columns))
    return StoredHodlr(h.n, h.depth, h.blocks, h.leaves, list(level_fmt), QU, QV)


def store_blocks(h, block_fmt, scale_columns: bool = True) -> StoredHodlr:
    """Quantise every block's generators in its own format (the per-block
    variant of ``oracle.assign.assign_blocks``); ``level_fmt`` is left empty."""
    QU, QV = [], []
    for U, V, f in zip(h.U, h.V, block_fmt):
        QU.append(quantize(U, f, scale_columns))
        QV.append(quantize(V, f, scale_columns))
    return StoredHodlr(h.n, h.depth, h.blocks, h.leaves, [], QU, QV)


def storage_bits(stored: StoredHodlr) -> int:
    """Bits of the stored generators: codes plus one 8-bit exponent per
    column of a factor stored with column scales."""
    bits = 0
    for q in list(stored.QU) + list(stored.QV):
        f = F.fmt(q.fmt)
        bits += q.codes.size * 8 * f.nbytes
        if q.scaled:
            bits += 8 * q.codes.shape[1]
    return bits
