"""Compression of a kernel matrix into an eps-HODLR operator (input generator).

Given a kernel, points, the caller's partition (canonical off-diagonal
blocks and leaves as index ranges) and eps, every off-diagonal block B is
replaced by U V^T with U having orthonormal columns and V = Z_p Sigma_p,
truncated so that the discarded part meets the rule:

* ``"frob"``: the smallest p with ||B - U V^T||_F <= eps ||B||_F;
* ``"spec_global"``: keep singular values > eps * ||A||_2 (``norm_a_2``).

Small blocks use a dense SVD.  Large blocks (more than ``dense_limit``
entries) use, with ``method="random"``, a randomised range finder evaluated
tile by tile: Y = B Omega, Q = orth(Y), M = Q^T B, SVD of M.  The residual
||B - Q M||_F is known (either exactly from a third pass, or as
||B||_F^2 - ||M||_F^2 when eps is large enough for that difference to be
accurate), so the rank chosen meets the rule exactly for the factors
produced; the sketch grows until it does.  ||B||_F^2 of every block and of
every leaf is accumulated on the way, so ||A||_F^2 = sum of them is exact.

``method="aca"`` is for operators too large to evaluate every entry (the
2^20-point workload): adaptive cross approximation with partial pivoting
(Bebendorf, Numer. Math. 86 (2000)) touches O((r + c) k) entries of a block
for k crosses, stopping when the last cross is below eps/16 of the
approximant's norm; the crosses are recompressed (QR of both sides, SVD of
the small core) and truncated by the same rule, with ||B||_F^2 taken as the
approximant's plus the residual's, the residual estimated from 16 sampled
rows (a statistical certificate, kept in ``Compressed.certificate``; exact
norms are not available at that size).

The result is the input of the library's ``hodlr_create`` (and of the
oracle's tests): fp64 leaves, fp64 U_b, V_b, and the squared norms.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

try:
    from threadpoolctl import threadpool_limits
except ImportError:  # pragma: no cover
    threadpool_limits = None


@dataclass
class Compressed:
    n: int
    leaves: list                     # fp64 D_i (m_i x m_i)
    U: list                          # fp64 r_b x p_b
    V: list                          # fp64 c_b x p_b
    norm2_all: float
    norm2_blocks: np.ndarray
    sketch: list = field(default_factory=list)   # per block: 0 dense, else sketch width / crosses
    certificate: list = field(default_factory=list)   # per block (aca): sampled residual / ||B||_F

    @property
    def ranks(self):
        return [u.shape[1] for u in self.U]


def _workers():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


def _rank(s, eps, rule, nb2, norm_a_2, res2=0.0):
    if s.size == 0:
        return 0 if res2 <= (eps * eps) * nb2 else None
    if rule == "frob":
        thr2 = (eps * eps) * nb2
        sq = np.append((s[::-1] ** 2).cumsum()[::-1], 0.0) + res2
        ok = np.nonzero(sq <= thr2)[0]
        return int(ok[0]) if ok.size else None
    if rule == "spec_global":
        return int(np.count_nonzero(s > eps * norm_a_2))
    raise ValueError(rule)


class _Pool:
    def __init__(self, workers=None):
        self.nw = workers if workers else _workers()
        self.ex = ThreadPoolExecutor(self.nw)

    def map(self, fn, items):
        return list(self.ex.map(fn, items))


def _tiles(nrows, ncols, budget=1 << 24):
    t = max(16, min(nrows, budget // max(1, ncols)))
    return [(a, min(nrows, a + t)) for a in range(0, nrows, t)]


def _dense_block(kernel, P, b, eps, rule, norm_a_2):
    r0, nr, c0, nc = b
    B = kernel.block(P, r0, r0 + nr, c0, c0 + nc)
    nb2 = float(np.sum(B * B))
    if B.size == 0:
        return np.zeros((nr, 0)), np.zeros(0), np.zeros((nc, 0)), nb2
    W, s, Zt = np.linalg.svd(B, full_matrices=False)
    p = _rank(s, eps, rule, nb2, norm_a_2)
    return W[:, :p].copy(), s[:p].copy(), Zt[:p].T.copy(), nb2


def _random_block(kernel, P, b, eps, rule, norm_a_2, pool, rng, s0):
    r0, nr, c0, nc = b
    tiles = _tiles(nr, nc)
    exact_res = eps < 1e-6 or rule != "frob"
    s = max(8, s0)
    while True:
        Om = rng.standard_normal((nc, s))

        def p1(t):
            B = kernel.block(P, r0 + t[0], r0 + t[1], c0, c0 + nc)
            return B @ Om, float(np.sum(B * B))
        out = pool.map(p1, tiles)
        Y = np.vstack([o[0] for o in out])
        nb2 = float(sum(o[1] for o in out))
        Q, _ = np.linalg.qr(Y)

        def p2(group):                   # each worker adds up its own tiles
            M = np.zeros((Q.shape[1], nc))
            for t in group:
                B = kernel.block(P, r0 + t[0], r0 + t[1], c0, c0 + nc)
                M += Q[t[0]:t[1]].T @ B
            return M
        groups = [tiles[w::pool.nw] for w in range(min(pool.nw, len(tiles)))]
        M = np.sum(pool.map(p2, groups), axis=0)
        if exact_res:
            def p3(t):
                B = kernel.block(P, r0 + t[0], r0 + t[1], c0, c0 + nc)
                R = B - Q[t[0]:t[1]] @ M
                return float(np.sum(R * R))
            res2 = float(sum(pool.map(p3, tiles)))
        else:
            res2 = max(0.0, nb2 - float(np.sum(M * M)))
        Wm, sm, Zt = np.linalg.svd(M, full_matrices=False)
        p = _rank(sm, eps, rule, nb2, norm_a_2, res2)
        # accept when the rule is met and the sketch kept some slack
        if p is not None and (p < s - 4 or s >= min(nr, nc)):
            U = Q @ Wm[:, :p]
            return U, sm[:p].copy(), Zt[:p].T.copy(), nb2, s
        if s >= min(nr, nc):
            raise RuntimeError("randomised compression could not meet eps")
        s = min(min(nr, nc), 2 * s)


def _aca_block(kernel, P, b, eps, rule, norm_a_2, rng, sample_rows=16):
    r0, nr, c0, nc = b
    Pr, Pc = P[r0:r0 + nr], P[c0:c0 + nc]
    kmax = min(nr, nc, 1024)
    Ua = np.zeros((nr, 64))
    Va = np.zeros((nc, 64))
    used_r = np.zeros(nr, dtype=bool)
    used_c = np.zeros(nc, dtype=bool)
    norm2, k, i, small = 0.0, 0, 0, 0
    tol = eps / 16.0
    while k < kmax:
        if k == Ua.shape[1]:                       # grow the cross storage
            Ua = np.hstack([Ua, np.zeros((nr, k))])
            Va = np.hstack([Va, np.zeros((nc, k))])
        used_r[i] = True
        rv = kernel.offdiag(Pr[i:i + 1], Pc)[0] - Ua[i, :k] @ Va[:, :k].T
        a = np.abs(rv)
        a[used_c] = -1.0
        j = int(np.argmax(a))
        if a[j] <= 0.0:                            # zero residual row: try another row
            free = np.flatnonzero(~used_r)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = rv / rv[j]
        u = kernel.offdiag(Pr, Pc[j:j + 1])[:, 0] - Ua[:, :k] @ Va[j, :k]
        used_c[j] = True
        uu, vv = float(u @ u), float(v @ v)
        norm2 += 2.0 * float((Ua[:, :k].T @ u) @ (Va[:, :k].T @ v)) + uu * vv
        Ua[:, k], Va[:, k] = u, v
        k += 1
        if np.sqrt(uu * vv) <= tol * np.sqrt(max(norm2, 0.0)):
            small += 1
            if small >= 2:
                break
        else:
            small = 0
        au = np.abs(u)
        au[used_r] = -1.0
        i = int(np.argmax(au))
        if au[i] < 0.0:
            break
    Ua, Va = Ua[:, :k], Va[:, :k]
    # recompress: B ~ Ua Va^T = Qu (Ru Rv^T) Qv^T
    Qu, Ru = np.linalg.qr(Ua)
    Qv, Rv = np.linalg.qr(Va)
    W, s, Zt = np.linalg.svd(Ru @ Rv.T)
    # sampled rows: the residual of the full cross approximation
    ii = rng.integers(0, nr, min(sample_rows, nr))
    R = kernel.offdiag(Pr[ii], Pc) - Ua[ii] @ Va.T
    nb2 = float(np.sum(s * s))
    res2 = float(np.sum(R * R)) * nr / len(ii)
    p = _rank(s, eps, rule, nb2 + res2, norm_a_2, res2)
    if p is None:
        p = len(s)
    U = Qu @ W[:, :p]
    Z = Qv @ Zt[:p].T
    cert = np.sqrt(res2 / max(nb2, 1e-300))
    return U, s[:p].copy(), Z, nb2, k, cert


def compress(kernel, P, blocks, leaves, eps, rule="frob", norm_a_2=None,
             seed=12345, dense_limit=512 * 512, workers=None, method="random") -> Compressed:
    """Compress every off-diagonal block of the kernel matrix over ``P``.

    ``blocks``: (row0, nrows, col0, ncols) per off-diagonal block in the
    library's canonical order; ``leaves``: (start, size) per leaf;
    ``workers``: threads (default: the usable cores, at most 16).
    """
    if rule == "spec_global" and norm_a_2 is None:
        raise ValueError("spec_global needs norm_a_2")
    n = len(P)
    blocks = [tuple(int(v) for v in b) for b in blocks]
    index = {b: i for i, b in enumerate(blocks)}
    nb = len(blocks)
    U, S, Z, nb2 = [None] * nb, [None] * nb, [None] * nb, np.zeros(nb)
    sk = [0] * nb
    cert = [0.0] * nb
    pool = _Pool(workers)
    rng = np.random.default_rng(seed)
    twin = {}                      # lower block j derived from upper block i
    if kernel.symmetric or kernel.antisymmetric:
        for i, (r0, nr, c0, nc) in enumerate(blocks):
            j = index.get((c0, nc, r0, nr))
            if j is not None and j > i and i not in twin.values():
                twin[j] = i
    own = [i for i in range(nb) if i not in twin]
    small = [i for i in own if blocks[i][1] * blocks[i][3] <= dense_limit]
    large = [i for i in own if blocks[i][1] * blocks[i][3] > dense_limit]
    limiter = threadpool_limits(1) if threadpool_limits else None
    try:
        for i, res in zip(small, pool.map(
                lambda i: _dense_block(kernel, P, blocks[i], eps, rule, norm_a_2), small)):
            U[i], S[i], Z[i], nb2[i] = res
        if method == "aca":
            seeds = rng.integers(0, 2**31 - 1, len(large))
            for i, res in zip(large, pool.map(
                    lambda t: _aca_block(kernel, P, blocks[t[0]], eps, rule, norm_a_2,
                                         np.random.default_rng(int(t[1]))), list(zip(large, seeds)))):
                U[i], S[i], Z[i], nb2[i], sk[i], cert[i] = res
        else:
            prev_rank = 16
            for i in large:
                U[i], S[i], Z[i], nb2[i], sk[i] = _random_block(
                    kernel, P, blocks[i], eps, rule, norm_a_2, pool, rng, prev_rank + 16)
                prev_rank = max(8, U[i].shape[1])
    finally:
        if limiter is not None:
            limiter.restore_original_limits()
    sign = -1.0 if kernel.antisymmetric else 1.0
    for j, i in twin.items():
        U[j], S[j], Z[j], nb2[j], sk[j], cert[j] = Z[i], S[i], sign * U[i], nb2[i], sk[i], cert[i]
    Vs = [np.ascontiguousarray(z * s[None, :]) for z, s in zip(Z, S)]
    Us = [np.ascontiguousarray(u) for u in U]
    lv = []
    leaf_n2 = 0.0
    for a, m in leaves:
        D = kernel.block(P, a, a + m, a, a + m)
        leaf_n2 += float(np.sum(D * D))
        lv.append(D)
    pool.ex.shutdown()
    return Compressed(n, lv, Us, Vs, float(leaf_n2 + nb2.sum()), nb2, sk, cert)
