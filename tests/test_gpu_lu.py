"""Triangular solves on the GPU with the LU factors (``hodlr_solve``).

* Without truncation the factors of the stored matrix are unique, so the
  GPU's X = U^-1 L^-1 B must equal the oracle's solve with its own factors
  (oracle.lu) to 1e-10 relative, for 1, 3, 17 and 40 right-hand sides (the
  library applies the inverse factors as two fp64 products: the wave path
  below 8 columns, the matrix-core path above, ragged column groups);
* fp32 B and X: the solve runs in fp64 from the widened B, so X must be
  the fp64 solution of the same B rounded to fp32, bit for bit;
* with truncation, the GPU solution equals the dense triangular solves with
  the library's own factors (hodlr_lu_dense) to 1e-10 relative;
* at 8192 and 65536 points (the 2D Gaussian workload, built on the GPU), the
  residual of the solution against the stored operator's product obeys
  Cor. "LU of mixed-precision HODLR matrices" with the factor norms the
  library reports, and a repeated solve is bit-identical;
* refusals: no factors, bfloat16 operands.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from hodlr_inputs import configs as CF  # noqa: E402
from oracle import assign as AS  # noqa: E402
from oracle import construct as OC  # noqa: E402
from oracle import lu as LU  # noqa: E402
from oracle import quantize as Q  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2407_21637_amd as H  # noqa: E402

DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(cfg, eps, allowed=("fp32", "bf16", "fp16")):
    A = cfg.kernel.dense(cfg.points())
    h = OC.construct(A, cfg.depth, eps)
    op = H.Operator(h.n, cfg.depth, h.leaves, h.U, h.V, device=0)
    norms = np.concatenate([[h.norm2_all], h.norm2_blocks])
    op.assign_precision(eps, allowed, norms2=norms)
    a = AS.assign(h.norm2_all, AS.level_max_norm2(h.norm2_blocks, [b.level for b in h.blocks]), eps, allowed)
    assert [x[0] for x in op.levels()] == a.fmt
    s = Q.store(h, a.fmt)
    return A, op, LU.from_stored(h.n, cfg.depth, h.blocks, h.leaves, s.U, s.V)


def _dev(b, dtype=torch.float64):
    X = H.colmajor_empty(b.shape[0], b.shape[1], dtype, DEV)
    X.copy_(torch.from_numpy(np.asfortranarray(b)).to(dtype))
    return X


def test_untruncated_solve_equals_the_oracle():
    cfg = CF._c2(1024, 3)
    A, op, Ho = _pair(cfg, 1e-6)
    rep = op.lu(0.0)
    _say(f"[lu] {cfg.name} eps=0: {rep}")
    Lo, Uo = LU.hodlr_lu(Ho, 0.0)
    rng = np.random.default_rng(11)
    for nrhs in (1, 3, 17, 40):
        b = rng.standard_normal((cfg.n, nrhs))
        x = op.solve(_dev(b)).cpu().numpy()
        xo = LU.solve(Lo, Uo, b)
        err = np.linalg.norm(x - xo, axis=0) / np.linalg.norm(xo, axis=0)
        _say(f"    nrhs={nrhs}: max rel diff {err.max():.2e}")
        assert (err <= 1e-10).all(), err
    # fp32 operands: the fp64 solve of the widened B, rounded once
    b32 = rng.standard_normal((cfg.n, 5)).astype(np.float32)
    x32 = op.solve(_dev(b32, torch.float32))
    x64 = op.solve(_dev(b32.astype(np.float64)))
    assert torch.equal(x32, x64.to(torch.float32))
    # a 1-D right-hand side, and B aliasing X
    v = _dev(b[:, :1]).reshape(-1)
    xv = op.solve(v.clone())
    op.solve(v, v)
    assert torch.equal(v, xv)


@pytest.mark.parametrize("name,n,depth,eps", [("c3", 2048, 4, 1e-6), ("c5", 2048, 4, 1e-4)])
def test_truncated_solve_equals_the_dense_triangular_solves(name, n, depth, eps):
    import scipy.linalg as sl
    cfg = {"c3": CF._c3, "c5": CF._c5}[name](n, depth)
    A, op, _ = _pair(cfg, eps)
    rep = op.lu(eps)
    L, U = op.lu_dense()
    b = np.random.default_rng(12).standard_normal((n, 6))
    xr = sl.solve_triangular(U, sl.solve_triangular(L, b, lower=True, unit_diagonal=True))
    x = op.solve(_dev(b)).cpu().numpy()
    err = np.linalg.norm(x - xr, axis=0) / np.linalg.norm(xr, axis=0)
    _say(f"[lu] {cfg.name} eps={eps:g}: {rep}; max rel diff {err.max():.2e}")
    assert (err <= 1e-10).all(), err
    bound = LU.lu_backward_bound(depth, eps, np.linalg.norm(A), rep["norm_l"], rep["norm_u"])
    assert (np.linalg.norm(A @ x - b, axis=0) <= bound * np.linalg.norm(x, axis=0) + 1e-12 *
            np.linalg.norm(b, axis=0)).all()


@pytest.mark.parametrize("n,depth", [(8192, 5), (65536, 8)])
def test_solve_residual_at_scale(n, depth):
    cfg = CF._c2(n, depth)
    eps = cfg.eps
    op, brep = H.build_kernel(cfg.points(), depth, "gaussian", a=0.04, diag_shift=0.01, eps=eps, seed=3)
    op.assign_precision(eps, cfg.allowed)
    rep = op.lu(eps)
    _say(f"[lu] {cfg.name} eps={eps:g} formats {[x[0] for x in op.levels()]}: {rep}")
    norm_h = float(np.sqrt(op.norms2()[0]))
    b = np.random.default_rng(13).standard_normal((n, 4))
    B = _dev(b)
    X = op.solve(B)                                   # first call: workspaces
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    X2 = op.solve(B)
    t1.record()
    torch.cuda.synchronize()
    assert torch.equal(X, X2)                         # deterministic
    R = op.matvec(X) - B
    res = torch.linalg.vector_norm(R, dim=0).cpu().numpy()
    xn = torch.linalg.vector_norm(X, dim=0).cpu().numpy()
    bound = LU.lu_backward_bound(depth, eps, norm_h, rep["norm_l"], rep["norm_u"])
    _say(f"    solve {t0.elapsed_time(t1):.2f} ms; ||Hx-b||/||x|| {(res / xn).max():.2e}, bound {bound:.2e}")
    assert (res <= bound * xn + 1e-12 * np.linalg.norm(b, axis=0)).all()


def test_refusals():
    cfg = CF._c2(256, 2)
    A, op, _ = _pair(cfg, 1e-6, ("fp32",))
    b = _dev(np.ones((256, 1)))
    with pytest.raises(H.HodlrError) as e:
        op.solve(b)                                    # no factors yet
    assert e.value.status == 2
    op.lu(1e-8)
    with pytest.raises(H.HodlrError) as e:
        op.solve(b.to(torch.bfloat16))
    assert e.value.status == 6
    op.assign_precision(1e-6, ("fp32", "bf16"))        # reassignment drops the factors
    with pytest.raises(H.HodlrError) as e:
        op.solve(b)
    assert e.value.status == 2
