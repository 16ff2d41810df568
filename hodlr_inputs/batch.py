"""Batches of independent operators of uneven size, depth, rank and format.

The batched workload: ``count`` operators, each drawn from its own child of
``numpy.random.SeedSequence(seed)``:

* n = round(exp(U(ln n_lo, ln n_hi))), points in 1 or 2 dimensions (sorted
  uniform on [0, 1], or uniform in the unit square in Morton order);
* kernel drawn from 1/(r + 1e-3), exp(-r) and exp(-r^2 / 0.08) (Gaussian
  with h = 0.2), no diagonal shift;
* depth = ceil(log2(n / leaf)) (leaves in (leaf/2, leaf]), at least 1;
* eps drawn from {1e-4, 1e-6, 1e-8}, Frobenius truncation per block;
* storage formats chosen by the adaptive rule from {fp32, bf16, fp16, e4m3};
* nrhs drawn from {1, 8, 32}; X ~ N(0, 1) in fp32, or fp64 for the
  eps = 1e-8 operators.

``c4`` is 512 operators with n in [1024, 16384] and leaf 256; ``c4_s`` is a
small batch for tests.  This module only draws inputs: it holds none of the
method's arithmetic beyond the compression shared with the other workloads.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import kernels as K
from . import points as Pt

ALLOWED = ("fp32", "bf16", "fp16", "e4m3")
KERNELS = (("inv", lambda: K.inv_dist_reg(1e-3)), ("exp", lambda: K.exp_neg()),
           ("gauss", lambda: K.gaussian(0.08)))
EPS = (1e-4, 1e-6, 1e-8)
NRHS = (1, 8, 32)


@dataclass
class OpSpec:
    index: int
    n: int
    dim: int
    kernel_name: str
    eps: float
    depth: int
    nrhs: int
    x_dtype: str          # "fp32" or "fp64"
    seed_points: int
    seed_x: int

    @property
    def kernel(self):
        return dict(KERNELS)[self.kernel_name]()

    def points(self) -> np.ndarray:
        if self.dim == 1:
            return Pt.uniform_1d_sorted(self.n, self.seed_points)
        return Pt.uniform_2d_morton(self.n, self.seed_points)

    def X(self) -> np.ndarray:
        X = np.random.default_rng(self.seed_x).standard_normal((self.n, self.nrhs))
        if self.x_dtype == "fp32":
            X = X.astype(np.float32).astype(np.float64)
        return X


def specs(count: int, n_lo: int, n_hi: int, leaf: int, seed: int = 0) -> list[OpSpec]:
    out = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(child)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        dim = int(rng.integers(1, 3))
        kname = KERNELS[int(rng.integers(0, len(KERNELS)))][0]
        eps = EPS[int(rng.integers(0, len(EPS)))]
        nrhs = NRHS[int(rng.integers(0, len(NRHS)))]
        depth = max(1, math.ceil(math.log2(n / leaf)))
        s_pts, s_x = (int(v) for v in rng.integers(0, 2**31 - 1, 2))
        out.append(OpSpec(i, n, dim, kname, eps, depth, nrhs, "fp64" if eps < 1e-7 else "fp32", s_pts, s_x))
    return out


BATCHES = {
    "c4": dict(count=512, n_lo=1024, n_hi=16384, leaf=256),
    "c4_s": dict(count=24, n_lo=256, n_hi=2048, leaf=128),
}


def get(name: str) -> list[OpSpec]:
    return specs(**BATCHES[name])


def build(spec: OpSpec, blocks, leaves, seed: int = 12345, workers=None):
    """Points and the compressed operator of one spec over the caller's partition."""
    from .compress import compress
    P = spec.points()
    return P, compress(spec.kernel, P, blocks, leaves, spec.eps, "frob", seed=seed, workers=workers)


def _build_one(args):
    spec, blocks, leaves = args
    return build(spec, blocks, leaves, workers=1)[1]


def build_all(specs, parts, processes=None, log=None):
    """Compressed operators of every spec, one process per operator at a
    time (``parts``: (blocks, leaves) per spec, the caller's partitions).
    Uses spawned processes: call it before the GPU is touched."""
    import multiprocessing as mp
    import os
    from concurrent.futures import ProcessPoolExecutor
    if processes is None:
        try:
            processes = max(1, min(16, len(os.sched_getaffinity(0))))
        except AttributeError:  # pragma: no cover
            processes = max(1, min(16, os.cpu_count() or 1))
    out = [None] * len(specs)
    jobs = [(s, b, l) for s, (b, l) in zip(specs, parts)]
    order = sorted(range(len(specs)), key=lambda i: -specs[i].n)       # largest first
    with ProcessPoolExecutor(processes, mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(_build_one, jobs[i]): i for i in order}
        from concurrent.futures import as_completed
        for done, f in enumerate(as_completed(futs), 1):
            out[futs[f]] = f.result()
            if log and (done % 32 == 0 or done == len(specs)):
                log(f"[batch] compressed {done}/{len(specs)} operators")
    return out
