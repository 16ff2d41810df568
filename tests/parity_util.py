"""Shared helpers of the parity tests: build a workload over the oracle's
partition, run the oracle's stored-operator product, and compare a GPU
result with it under the componentwise tolerance of ``oracle.bounds``."""
from __future__ import annotations

import numpy as np

from hodlr_inputs import compress as CP
from hodlr_inputs import configs as CF
from oracle import assign as AS
from oracle import bounds as BD
from oracle import formats as F
from oracle import matvec as MV
from oracle import quantize as Q
from oracle import tree as T


class Case:
    """A compressed workload plus the oracle's view of it."""

    def __init__(self, cfg, n=None, depth=None, eps=None, leaf_bounds=None, points=None):
        c = CF.get(cfg) if isinstance(cfg, str) else cfg
        self.cfg = c
        self.n = c.n if n is None else n
        self.depth = c.depth if depth is None else depth
        self.eps = c.eps if eps is None else eps
        P = c.points() if points is None else points
        self.P = P[: self.n]
        self.leaf_bounds = leaf_bounds
        self.blocks = T.blocks(self.n, self.depth, leaf_bounds)
        self.leaves_b = T.leaves(self.n, self.depth, leaf_bounds)
        na2 = None
        if c.rule == "spec_global":
            na2 = float(np.linalg.norm(c.kernel.dense(self.P), 2))
        self.op = CP.compress(c.kernel, self.P, [(b.row0, b.nrows, b.col0, b.ncols) for b in self.blocks],
                              self.leaves_b, self.eps, c.rule, na2, method=c.extra.get("compress", "random"))
        self.norms2 = np.concatenate([[self.op.norm2_all], self.op.norm2_blocks])

    def oracle_assign(self, allowed):
        lv = AS.level_max_norm2(self.op.norm2_blocks, [b.level for b in self.blocks])
        return AS.assign(self.op.norm2_all, lv, self.eps, allowed)

    def stored(self, level_fmt, scale=True):
        QU = [Q.quantize(u, level_fmt[b.level - 1], scale) for b, u in zip(self.blocks, self.op.U)]
        QV = [Q.quantize(v, level_fmt[b.level - 1], scale) for b, v in zip(self.blocks, self.op.V)]
        return [q.values for q in QU], [q.values for q in QV]

    def oracle_product(self, level_fmt, X, scale=True):
        U, V = self.stored(level_fmt, scale)
        y = MV.matvec(self.n, self.blocks, self.leaves_b, self.op.leaves, U, V, X)
        z = MV.matvec_abs(self.n, self.blocks, self.leaves_b, self.op.leaves, U, V, X)
        return y, z, U, V

    def chain(self):
        return BD.chain_length(self.blocks, self.op.ranks, [m for _, m in self.leaves_b], self.depth)

    def library_op(self, device=0):
        import paper_2407_21637_amd as H
        return H.Operator(self.n, self.depth, self.op.leaves, self.op.U, self.op.V, device=device,
                          leaf_bounds=None if self.leaf_bounds is None else
                          T.node_bounds(self.n, self.depth, self.leaf_bounds)[self.depth])


class RandomCase(Case):
    """Random factors with a chosen rank per level over the oracle's
    partition (no compression), for the kernels' rank-dependent paths:
    U_b, V_b with N(0, 1) entries (U_b scaled by 1/sqrt(rows)), leaves
    I + N(0, 1/m)."""

    def __init__(self, n, depth, ranks_per_level, seed=0):
        from types import SimpleNamespace
        rng = np.random.default_rng(seed)
        self.cfg = None
        self.n, self.depth, self.eps, self.leaf_bounds = n, depth, 0.0, None
        self.blocks = T.blocks(n, depth)
        self.leaves_b = T.leaves(n, depth)
        U = [rng.standard_normal((b.nrows, ranks_per_level[b.level - 1])) / np.sqrt(max(b.nrows, 1))
             for b in self.blocks]
        V = [rng.standard_normal((b.ncols, ranks_per_level[b.level - 1])) for b in self.blocks]
        leaves = [np.eye(m) + rng.standard_normal((m, m)) / np.sqrt(max(m, 1)) for _, m in self.leaves_b]
        self.op = SimpleNamespace(leaves=leaves, U=U, V=V, ranks=[u.shape[1] for u in U])
        self.norms2 = None


# (format, ranks per level, accumulation flag): operators whose every leaf's
# ancestor ranks fit one pass of stacked 16-row tiles, 1 to 4 tiles per leaf
STACKED_CASES = [
    ("e4m3", [16, 16, 16, 16], 0x2),     # four tiles
    ("e5m2", [5, 4, 4, 3], 0x2),         # one
    ("bf16", [12, 12, 12, 12], 0x2),     # three
    ("fp16", [9, 9, 9, 8], 0x2),         # three, a partial last tile
    ("fp32", [16, 16, 16, 16], 0x2),     # four, fp32 sums
    ("fp32", [8, 8, 8, 8], 0x4),         # two, fp64 sums
    ("fp64", [8, 8, 8, 8], 0x2),         # two, fp64 arithmetic
]

# depth 7, 3072 rows (leaves of 24 rows): level 1's 40 ranks over the 64
# leaves of its column node exceed the 32 outputs a slice of the bf16
# reduction's 8 interleaved slices would hold, so it takes fewer slices
DEEP_STACKED = (3072, 7, [40, 3, 3, 3, 3, 3, 3])


def check(y_gpu, y_ora, z, M, acc, xy, label=""):
    """Assert both componentwise gates; return error statistics.

    * tau: the worst-case bound (``oracle.bounds.tolerance``);
    * tau_prob: the probabilistic bound (``oracle.bounds.tolerance_prob``),
      about sqrt(M) times tighter, met with probability >= 1 - 1e-6 under
      the model of independent rounding errors.
    """
    u_acc = F.FP64.u if acc == "fp64" else F.FP32.u
    u_out = F.FP64.u if xy == "fp64" else F.FP32.u
    y_gpu = np.asarray(y_gpu, dtype=np.float64)
    tau = BD.tolerance(z, y_ora, M, u_acc, u_out)
    taup = BD.tolerance_prob(z, y_ora, M, u_acc, u_out)
    err = np.abs(y_gpu - y_ora)
    nz = lambda t: np.where(t > 0, t, 1)
    stats = {
        "max_err_over_tau": float((err / nz(tau)).max()) if err.size else 0.0,
        "max_err_over_tau_prob": float((err / nz(taup)).max()) if err.size else 0.0,
        "norm_err_over_uz": float(np.linalg.norm(err) / (u_acc * np.linalg.norm(z))) if err.size else 0.0,
        "rel_err": float(np.linalg.norm(err) / max(np.linalg.norm(y_ora), 1e-300)),
    }
    assert np.isfinite(y_gpu).all(), (label, "non-finite output")
    assert not (err > tau).any(), (label, int((err > tau).sum()), stats)
    assert not (err > taup).any(), (label, "prob", int((err > taup).sum()), stats)
    return stats
