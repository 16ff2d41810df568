"""Named synthetic workloads.

Each workload fixes the points, kernel, size, depth, eps, truncation rule,
the set of storage formats the adaptive rule may choose from, and the
right-hand sides.  Points use seed 0 and right-hand sides seed 1 of numpy's
``default_rng`` (PCG64) unless stated.

* ``c1`` -- n=2048 sorted uniform 1D points, A_ij = 1/(|x_i-x_j|+1e-3),
  depth 4 (leaf 128), eps=1e-8 relative to ||A||_2, uniform fp64, one fp64
  right-hand side ~ N(0,1).  Small enough for a dense oracle.
* ``c2`` -- n=65536 uniform 2D points in Morton order, Gaussian kernel
  exp(-r^2/0.04) + 0.01 on the diagonal, depth 8 (leaf 256), eps=1e-6,
  formats {fp32, bf16, fp16}, fp32 right-hand sides ~ N(0,1), nrhs 1 or 32.
* ``c3`` -- n=262144 sorted uniform 1D points, log(|x_i-x_j|+1e-4) with n
  added on the diagonal, depth 9 (leaf 512), eps=1e-3, formats {fp16, bf16,
  e4m3}, 128 fp32 right-hand sides ~ U(-1,1).
* ``c5`` -- n=2^20 points from a mixture of four Gaussians (centres 0.2,
  0.4, 0.6, 0.8, sd 0.02, clipped, sorted), 1/(|x_i-x_j|+1e-5) + n on the
  diagonal, depth 12 (leaf 256), eps=1e-10, formats {fp32, fp16}, fp64
  accumulation, 16 fp64 right-hand sides ~ N(0,1); compressed by adaptive
  cross approximation (too large to evaluate every entry).
* ``mat1``..``mat4`` -- the paper's matrix-vector experiments (Sect. 4,
  kernels (4.1)): n=2000, depth 8; (i) on a 1D grid, (ii) and (iii) with
  h=1 and h=20 on a 40x50 grid of [-1,1]^2; x ~ U(-1,1); formats
  {e5m2 (q52), bf16, fp16, fp32}.
* ``*_s`` variants -- the same recipe at a smaller n for fast tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from . import kernels as K
from . import points as Pt


@dataclass
class Config:
    name: str
    n: int
    depth: int
    points: Callable[[], np.ndarray]
    kernel: K.Kernel
    eps: float
    rule: str
    allowed: tuple
    nrhs: tuple
    x_dtype: str                 # "fp32" or "fp64"
    x_dist: str                  # "normal" or "uniform11"
    acc: str = "auto"            # accumulation policy: auto | fp32 | fp64
    seed_x: int = 1
    description: str = ""
    extra: dict = field(default_factory=dict)

    def X(self, nrhs: int) -> np.ndarray:
        """Right-hand sides, (n, nrhs) fp64 holding values of ``x_dtype``."""
        rng = np.random.default_rng(self.seed_x)
        if self.x_dist == "normal":
            X = rng.standard_normal((self.n, nrhs))
        else:
            X = rng.uniform(-1.0, 1.0, (self.n, nrhs))
        if self.x_dtype == "fp32":
            X = X.astype(np.float32).astype(np.float64)
        return X


def _c1(n=2048, depth=4):
    return Config("c1" if n == 2048 else f"c1_{n}", n, depth, lambda: Pt.uniform_1d_sorted(n, 0),
                  K.inv_dist_reg(1e-3), 1e-8, "spec_global", (), (1,), "fp64", "normal",
                  acc="fp64", description="1/(r+1e-3), 1D sorted uniform, uniform fp64")


def _c2(n=65536, depth=8):
    return Config("c2" if n == 65536 else f"c2_{n}", n, depth, lambda: Pt.uniform_2d_morton(n, 0),
                  K.gaussian(0.04, 0.01), 1e-6, "frob", ("fp32", "bf16", "fp16"), (1, 32),
                  "fp32", "normal", description="exp(-r^2/0.04)+0.01 I, 2D Morton, adaptive")


def _c3(n=262144, depth=9):
    return Config("c3" if n == 262144 else f"c3_{n}", n, depth, lambda: Pt.uniform_1d_sorted(n, 0),
                  K.log_reg(1e-4, float(n)), 1e-3, "frob", ("fp16", "bf16", "e4m3"), (128,),
                  "fp32", "uniform11", description="log(r+1e-4)+n I, 1D sorted, low accuracy")


def _c5(n=1 << 20, depth=12):
    # blocks far too large to evaluate whole: adaptive cross approximation
    return Config("c5" if n == 1 << 20 else f"c5_{n}", n, depth, lambda: Pt.clustered_1d(n, 0),
                  K.inv_dist_reg(1e-5, float(n)), 1e-10, "frob", ("fp32", "fp16"), (16,),
                  "fp64", "normal", acc="fp64",
                  description="1/(r+1e-5)+n I, clustered 1D, high accuracy",
                  extra={"compress": "aca"})


def _mat(i):
    n, depth = 2000, 8
    allowed = ("e5m2", "bf16", "fp16", "fp32")
    if i == 1:
        pts, ker = (lambda: Pt.grid_1d(n)), K.paper_inverse_1d()
    elif i == 2:
        pts, ker = (lambda: Pt.grid_2d(40, 50)), K.paper_log()
    else:
        h = 1.0 if i == 3 else 20.0
        pts, ker = (lambda: Pt.grid_2d(40, 50)), K.paper_gaussian(h)
    return Config(f"mat{i}", n, depth, pts, ker, 1e-6, "frob", allowed, (1,), "fp64",
                  "uniform11", description=f"paper kernel matrix mat-{i}")


CONFIGS = {
    "c1": _c1(),
    "c2": _c2(),
    "c3": _c3(),
    "c5": _c5(),
    "c1_s": _c1(512, 2),
    "c2_s": _c2(8192, 5),
    "c3_s": _c3(8192, 4),
    "c5_s": _c5(8192, 5),
    "mat1": _mat(1), "mat2": _mat(2), "mat3": _mat(3), "mat4": _mat(4),
}


def get(name: str) -> Config:
    return CONFIGS[name]


def with_eps(cfg: Config, eps: float) -> Config:
    """Copy of ``cfg`` at another eps (the paper sweeps eps)."""
    import dataclasses
    return dataclasses.replace(cfg, eps=eps, name=f"{cfg.name}@{eps:g}")


def norm_a_2(cfg: Config, P: np.ndarray) -> float | None:
    """||A||_2 for the rule that needs it (dense; small n only)."""
    if cfg.rule != "spec_global":
        return None
    return float(np.linalg.norm(cfg.kernel.dense(P), 2))


def build(cfg: Config, blocks, leaves, seed: int = 12345):
    """Points and the compressed operator over the caller's partition."""
    from .compress import compress
    P = cfg.points()
    op = compress(cfg.kernel, P, blocks, leaves, cfg.eps, cfg.rule, norm_a_2(cfg, P), seed=seed,
                  method=cfg.extra.get("compress", "random"))
    return P, op
