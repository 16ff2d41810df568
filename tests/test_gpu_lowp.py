"""GPU parity of the product in a low working precision (X, Y in bf16 or
fp16; hodlr_matvec with HODLR_BF16 / HODLR_FP16), through the C ABI.

Every case compares the library's Y with the oracle's W product of the same
stored operator (``oracle.lowp``: leaves, generator code values and T_b
rounded to W, exact sums) entry by entry under ``oracle.lowp.tolerance``:
the fp32 sums of the device, a T_b that may round one W quantum apart, and
the final rounding of Y.  Operators: the adaptive fp32 recipe, the e4m3
recipe, every stored format including fp64 levels, the paper's kernels with
padded leaves, large leaves, strided X and Y; nrhs from 1 to 128.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.parity_util import DEEP_STACKED, STACKED_CASES, Case, RandomCase  # noqa: E402
from oracle import bounds as BD  # noqa: E402
from oracle import formats as F  # noqa: E402
from oracle import lowp as LP  # noqa: E402
from oracle import quantize as Q  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2407_21637_amd as H  # noqa: E402

DEV = torch.device("cuda:0")
TD = {"bf16": torch.bfloat16, "fp16": torch.float16}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle(case, fmts, Xw, w):
    QU = [Q.quantize(u, fmts[b.level - 1]) for b, u in zip(case.blocks, case.op.U)]
    QV = [Q.quantize(v, fmts[b.level - 1]) for b, v in zip(case.blocks, case.op.V)]
    prod = LP.matvec_lowp(case.n, case.blocks, case.leaves_b, case.op.leaves, QU, QV, Xw, w)
    Cl = max([b.ncols for b in case.blocks] or [1])
    return prod, LP.tolerance(prod, w, case.chain(), Cl)


def _check(label, yg, prod, tol):
    err = np.abs(yg - prod.y)
    assert np.isfinite(yg).all(), (label, "non-finite output")
    bad = err > tol
    ratio = float((err / np.where(tol > 0, tol, 1)).max()) if err.size else 0.0
    assert not bad.any(), (label, int(bad.sum()), ratio)
    return ratio


def _run(case, h, fmts, nrhs, w, label, X=None):
    if X is None:
        X = np.random.default_rng(7).standard_normal((case.n, nrhs))
    Xw = F.round_rne(w, X)
    _say(f"[lowp] {label} n={case.n} depth={case.depth} nrhs={nrhs} fmts={fmts} w={w}")
    Xd = H.colmajor_empty(case.n, nrhs, TD[w], DEV)
    Xd.copy_(torch.from_numpy(np.asfortranarray(Xw)).to(TD[w]))
    Y = h.matvec(Xd)
    torch.cuda.synchronize()
    yg = Y.cpu().double().numpy()
    prod, tol = _oracle(case, fmts, Xw, w)
    r = _check(label, yg, prod, tol)
    # the device result is a W value of every entry
    assert np.array_equal(F.round_rne(w, yg), yg)
    _say(f"    ok max err/tol {r:.3g}")
    return yg


@pytest.mark.parametrize("w", ["bf16", "fp16"])
@pytest.mark.parametrize("nrhs", [1, 7, 16, 33, 64])
def test_adaptive_fp32_recipe(w, nrhs):
    case = Case("c2_s")
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    fm = [lv[0] for lv in h.levels()]
    _run(case, h, fm, nrhs, w, "c2_s")


@pytest.mark.parametrize("w", ["bf16", "fp16"])
@pytest.mark.parametrize("nrhs", [16, 128])
def test_low_accuracy_e4m3_recipe(w, nrhs):
    case = Case("c3_s")
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    fm = [lv[0] for lv in h.levels()]
    _run(case, h, fm, nrhs, w, "c3_s")


@pytest.mark.parametrize("fmt,ranks,flags", STACKED_CASES)
def test_leaf_stacked_contraction(fmt, ranks, flags):
    """The contraction on leaf-stacked tiles (k_contract_lp_stack and
    k_reduce_lp_stack): every code format, 1 to 4 tiles per leaf, ragged
    leaves, 1, 3 and 8 column groups."""
    case = RandomCase(3000, 4, ranks, seed=5)
    h = case.library_op()
    h.set_level_precisions([fmt] * 4, flags)
    assert h.query()["leaf_stacked"]
    for w, nrhs in (("bf16", 5), ("fp16", 40), ("bf16", 128)):
        _run(case, h, [fmt] * 4, nrhs, w, f"stacked-{fmt}")


def test_leaf_stacked_contraction_deep_tree():
    """A level whose rank exceeds what the reduction's slices hold at that
    many leaves (fewer slices), four tiles per leaf, ragged small leaves."""
    n, depth, ranks = DEEP_STACKED
    case = RandomCase(n, depth, ranks, seed=9)
    h = case.library_op()
    h.set_level_precisions(["bf16"] * depth, H.ACC_FP32)
    assert h.query()["leaf_stacked"]
    for w, nrhs in (("bf16", 3), ("fp16", 70)):
        _run(case, h, ["bf16"] * depth, nrhs, w, "stacked-deep")


@pytest.mark.parametrize("w", ["bf16", "fp16"])
def test_every_stored_format(w):
    """fp64 levels reach W directly, the others through their exact fp32 value."""
    case = Case("c2_s", n=4096, depth=5, eps=1e-5)
    h = case.library_op()
    fm = ["fp64", "fp32", "bf16", "fp16", "e4m3"]
    h.set_level_precisions(fm)
    for nrhs in (3, 40):
        _run(case, h, fm, nrhs, w, "formats")
    fm2 = ["e5m2", "fp16", "fp64", "bf16", "fp32"]
    h.set_level_precisions(fm2)
    _run(case, h, fm2, 24, w, "formats-2")


@pytest.mark.parametrize("cfg", ["mat1", "mat3"])
def test_paper_kernels_padded_leaves(cfg):
    """n = 2000, depth 8: leaves of 7-8 rows padded to 16, one half-used
    32-column step per leaf."""
    case = Case(cfg)
    h = case.library_op()
    h.assign_precision(1e-3, case.cfg.allowed, case.norms2)
    fm = [lv[0] for lv in h.levels()]
    for w in ("bf16", "fp16"):
        _run(case, h, fm, 9, w, cfg)


def test_large_leaves_and_ragged():
    """Leaves of 1024 rows (several expansion tiles and contraction items)
    and a ragged n with padded leaves."""
    case = Case("c2_s", n=4096, depth=2, eps=1e-5)
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    fm = [lv[0] for lv in h.levels()]
    _run(case, h, fm, 20, "bf16", "large-leaves")
    case2 = Case("c2_s", n=999, depth=3, eps=1e-4)
    h2 = case2.library_op()
    h2.set_level_precisions(["fp32", "bf16", "e4m3"])
    _run(case2, h2, ["fp32", "bf16", "e4m3"], 5, "fp16", "ragged")


def test_strided_x_and_y():
    """ld of X and Y not a multiple of 8 elements: X goes through the padded
    copy; nothing is written past the n rows of each Y column."""
    case = Case("c2_s", n=4096, depth=4, eps=1e-4)
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    fm = [lv[0] for lv in h.levels()]
    nrhs, w = 18, "bf16"
    Xw = F.round_rne(w, np.random.default_rng(9).standard_normal((4096, nrhs)))
    Xb = torch.zeros(nrhs, 4096 + 1, dtype=TD[w], device=DEV)
    Xv = Xb[:, :4096].t()
    Xv.copy_(torch.from_numpy(Xw).to(TD[w]))
    Yb = torch.full((nrhs, 4096 + 3), 7.0, dtype=TD[w], device=DEV)
    Yv = Yb[:, :4096].t()
    _say(f"[lowp] strided n=4096 nrhs={nrhs} ldx=4097 ldy=4099")
    h.matvec(Xv, Yv)
    torch.cuda.synchronize()
    prod, tol = _oracle(case, fm, Xw, w)
    _check("strided", Yv.cpu().double().numpy(), prod, tol)
    assert (Yb[:, 4096:] == 7.0).all()


def test_deterministic():
    case = Case("c3_s")
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    X = torch.randn(case.n, 48, device=DEV).to(torch.bfloat16)
    Xd = H.colmajor_empty(case.n, 48, torch.bfloat16, DEV)
    Xd.copy_(X)
    y1 = h.matvec(Xd)
    y2 = h.matvec(Xd)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


def test_fp16_range_is_checked():
    """A leaf entry beyond fp16's range is refused (E_RANGE) before any
    work; bf16 takes the same operator."""
    rng = np.random.default_rng(3)
    D = [rng.standard_normal((32, 32)) for _ in range(2)]
    D[1][3, 3] = 1.0e6
    U = [rng.standard_normal((32, 2)), rng.standard_normal((32, 2))]
    V = [rng.standard_normal((32, 2)), rng.standard_normal((32, 2))]
    h = H.Operator(64, 1, D, U, V)
    h.set_level_precisions(["fp32"])
    X = torch.ones(64, 16, device=DEV).to(torch.float16)
    Xd = H.colmajor_empty(64, 16, torch.float16, DEV)
    Xd.copy_(X)
    with pytest.raises(RuntimeError, match="range"):
        h.matvec(Xd)
    Xb = H.colmajor_empty(64, 16, torch.bfloat16, DEV)
    Xb.copy_(X.to(torch.bfloat16))
    y = h.matvec(Xb)
    torch.cuda.synchronize()
    assert torch.isfinite(y.float()).all()


def test_first_call_on_two_streams_at_once():
    """The first bf16 product after an assignment builds the bf16 operand;
    a product enqueued at the same time on a second stream must not read it
    before the build has finished."""
    case = Case("c2_s", n=2048, depth=3, eps=1e-5)
    ref = case.library_op()
    ref.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    X = case.cfg.X(2)[:2048]
    Xd = H.colmajor_empty(2048, 2, torch.bfloat16, DEV)
    Xd.copy_(torch.from_numpy(np.asfortranarray(X)).to(torch.bfloat16))
    want = ref.matvec(Xd).clone()
    torch.cuda.synchronize()
    for rep in range(3):
        h = case.library_op()
        h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        Y1 = H.colmajor_empty(2048, 2, torch.bfloat16, DEV)
        Y2 = H.colmajor_empty(2048, 2, torch.bfloat16, DEV)
        with torch.cuda.stream(s1):
            h.matvec(Xd, Y1, stream=s1)
        with torch.cuda.stream(s2):
            h.matvec(Xd, Y2, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(Y1, want) and torch.equal(Y2, want), rep
        h.close()


def _gpu_backward_errors(A, cfg, eps, X):
    """eta = ||y - A x|| / (||A||_F ||x||) of the library's products of the
    eps-HODLR operator of A (adaptive formats), per working precision,
    averaged over the columns of X."""
    from oracle import construct as OC
    h = OC.construct(A, cfg.depth, eps)
    lib = H.Operator(cfg.n, cfg.depth, h.leaves, h.U, h.V, device=0)
    lib.assign_precision(eps, cfg.allowed, np.concatenate([[h.norm2_all], h.norm2_blocks]))
    nA = np.sqrt(h.norm2_all)
    out = {}
    for w, dt in (("fp64", torch.float64), ("fp32", torch.float32), ("bf16", torch.bfloat16),
                  ("fp16", torch.float16)):
        Xw = X if w == "fp64" else F.round_rne(w, X)
        Xd = H.colmajor_empty(cfg.n, X.shape[1], dt, DEV)
        Xd.copy_(torch.from_numpy(np.asfortranarray(Xw)).to(dt))
        Y = lib.matvec(Xd)
        torch.cuda.synchronize()
        Yh = Y.double().cpu().numpy()
        out[w] = float(np.mean([np.linalg.norm(Yh[:, j] - A @ Xw[:, j]) / (nA * np.linalg.norm(Xw[:, j]))
                                for j in range(X.shape[1])]))
    lib.close()
    return out


@pytest.mark.parametrize("cfg", ["mat3", "mat1"])
def test_working_precision_crossover_on_the_device(cfg):
    """Sect. 4's matrix-vector experiment on the GPU path: with a working
    precision u the backward error is the finite-precision one (well above
    fp64's, at most u) while eps << u, and the approximation one once
    eps >> u; fp64 always meets Thm. 3.5 (u = 2^-53 <= eps / n)."""
    from hodlr_inputs import configs as CF
    c = CF.get(cfg)
    A = c.kernel.dense(c.points())
    X = np.random.default_rng(0).uniform(-1, 1, (c.n, 3))
    e = {}
    for eps in (1e-8, 1e-6, 1e-4, 1e-3, 1e-2, 1e-1):
        e[eps] = _gpu_backward_errors(A, c, eps, X)
        _say(f"[crossover] {cfg} eps={eps:g}: " + ", ".join(f"{w} {v:.2e}" for w, v in e[eps].items()))
        assert e[eps]["fp64"] <= BD.matvec_backward_bound(c.depth, eps)
    for w in ("bf16", "fp16"):
        u = F.fmt(w).u
        assert e[1e-8][w] > 100 * e[1e-8]["fp64"]         # finite precision dominates
        assert e[1e-8][w] <= u
        assert e[1e-1][w] <= 1.1 * e[1e-1]["fp64"]       # approximation dominates
    assert e[1e-3]["bf16"] > 2 * e[1e-3]["fp64"]          # eps = 1e-3 < u_bf16: still bf16's
    assert e[1e-4]["fp16"] > 2 * e[1e-4]["fp64"]          # eps = 1e-4 < u_fp16: still fp16's
    # fp32 working precision: its roundoff shows only below eps ~ 1e-7
    assert e[1e-8]["fp32"] <= 2 * F.fmt("fp32").u and e[1e-2]["fp32"] <= 1.1 * e[1e-2]["fp64"]
