"""GPU parity: the HIP product against the oracle, through the C ABI.

Products with nrhs >= 8 take the matrix-core path (fp64 MFMA leaf GEMMs,
fp32/fp64 MFMA low-rank tiles); smaller ones the wave-reduction path.  Both
are checked here, on the same operators.

Every case compares the library's Y with the oracle's fp64 product of the
same stored operator (same fp64 factors, same formats, same codes), entry
by entry, under the componentwise tolerance of ``oracle.bounds.tolerance``
(the standard-model bound for a chain of M rounded operations in the
accumulation precision, plus the output rounding).  Layouts are compared
bit for bit.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.parity_util import DEEP_STACKED, STACKED_CASES, Case, RandomCase, check  # noqa: E402
from oracle import bounds as BD  # noqa: E402
from oracle import quantize as Q  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2407_21637_amd as H  # noqa: E402

DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu_product(h, X, xy):
    dt = torch.float64 if xy == "fp64" else torch.float32
    Xt = torch.from_numpy(np.asfortranarray(X)).to(dt)
    Xd = H.colmajor_empty(X.shape[0], X.shape[1], dt, DEV)
    Xd.copy_(Xt)
    Y = h.matvec(Xd)
    torch.cuda.synchronize()
    return Y.cpu().double().numpy()


def _run(case, h, fmts, nrhs, xy, acc, label, X=None):
    if X is None:
        X = case.cfg.X(nrhs)[: case.n] if case.cfg.n >= case.n else None
        if X is None or X.shape[0] != case.n:
            rng = np.random.default_rng(1)
            X = rng.standard_normal((case.n, nrhs))
        if xy == "fp32":
            X = X.astype(np.float32).astype(np.float64)
    _say(f"[parity] {label} n={case.n} depth={case.depth} nrhs={nrhs} fmts={fmts} acc={acc}")
    y, z, _, _ = case.oracle_product(fmts, X)
    yg = _gpu_product(h, X, xy)
    st = check(yg, y, z, case.chain(), acc, xy, label)
    _say(f"    ok {st}")
    return X, yg, y, st


def test_c1_uniform_fp64_full_size_and_layout():
    case = Case("c1")
    h = case.library_op()
    assert h.info()["acc_dtype"] == "fp64"
    fm = ["fp64"] * case.depth
    X, yg, y, _ = _run(case, h, fm, 1, "fp64", "fp64", "c1")
    # Thm 3.5 against the original matrix (fp64 working precision)
    A = case.cfg.kernel.dense(case.P)
    nA = np.sqrt(case.op.norm2_all)
    eta = np.linalg.norm(yg[:, 0] - A @ X[:, 0]) / (nA * np.linalg.norm(X[:, 0]))
    assert eta <= BD.matvec_backward_bound(case.depth, case.eps)
    # the uploaded image equals the oracle's codes bit for bit
    for b in range(h.nblocks):
        uc, ue, vc, ve = h.export_block(b, from_device=True)
        assert np.array_equal(uc, Q.quantize(case.op.U[b], "fp64").codes)
        assert np.array_equal(vc, Q.quantize(case.op.V[b], "fp64").codes)


@pytest.mark.parametrize("nrhs", [1, 2, 3, 8, 16, 17, 32, 33, 128])
def test_c2_small_adaptive(nrhs):
    case = Case("c2_s")
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    a = case.oracle_assign(case.cfg.allowed)
    assert [lv[0] for lv in h.levels()] == a.fmt
    _run(case, h, a.fmt, nrhs, "fp32", "fp32", "c2_s")


def test_c3_recipe_small_e4m3_matrix_cores():
    """The low-accuracy recipe (log kernel, eps 1e-3, {fp16, bf16, e4m3}) at
    n = 8192: the adaptive rule picks e4m3; 128 right-hand sides take the
    128-column matrix-core tiles."""
    case = Case("c3_s")
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    a = case.oracle_assign(case.cfg.allowed)
    assert [lv[0] for lv in h.levels()] == a.fmt
    for nrhs in (1, 128):
        _run(case, h, a.fmt, nrhs, "fp32", h.info()["acc_dtype"], "c3_s")


def test_c5_recipe_small_fp64():
    """The high-accuracy recipe (clustered 1/(r+1e-5) + n I, eps 1e-10,
    {fp32, fp16}) at n = 8192: fp64 X and Y, fp64 accumulation, 1 and 16
    right-hand sides; Thm 3.5 against the dense matrix."""
    case = Case("c5_s")
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    a = case.oracle_assign(case.cfg.allowed)
    assert [lv[0] for lv in h.levels()] == a.fmt
    assert h.info()["acc_dtype"] == "fp64"
    A = case.cfg.kernel.dense(case.P)
    nA = np.sqrt(case.op.norm2_all)
    for nrhs in (1, 16):
        X, yg, _, _ = _run(case, h, a.fmt, nrhs, "fp64", "fp64", "c5_s")
        for j in range(nrhs):
            eta = np.linalg.norm(yg[:, j] - A @ X[:, j]) / (nA * np.linalg.norm(X[:, j]))
            assert eta <= BD.matvec_backward_bound(case.depth, case.eps)


@pytest.mark.parametrize("nrhs", [1, 3, 24])
def test_per_block_formats(nrhs):
    """Per-block precision (HODLR_PER_BLOCK): formats differ inside a level;
    both product paths against the oracle's per-block stored operator."""
    from oracle import assign as AS
    from oracle import matvec as MV
    # clustered points: block norms vary inside a level, so do the formats
    case = Case("c5_s", n=4096, depth=4, eps=1e-4)
    allowed = ("e4m3", "e5m2", "fp16", "bf16", "fp32")
    h = case.library_op()
    h.assign_precision(case.eps, allowed, case.norms2, H.PER_BLOCK)
    levels = [b.level for b in case.blocks]
    a = AS.assign_blocks(case.op.norm2_all, case.op.norm2_blocks, levels, case.eps, allowed)
    assert [h.block(b)["dtype"] for b in range(h.nblocks)] == a.fmt
    assert any(len({f for f, k in zip(a.fmt, levels) if k == kk}) > 1 for kk in range(1, case.depth + 1))
    assert h.info()["acc_dtype"] == "fp32"
    U = [Q.quantize(u, f).values for u, f in zip(case.op.U, a.fmt)]
    V = [Q.quantize(v, f).values for v, f in zip(case.op.V, a.fmt)]
    X = case.cfg.X(nrhs)[: case.n]
    y = MV.matvec(case.n, case.blocks, case.leaves_b, case.op.leaves, U, V, X)
    z = MV.matvec_abs(case.n, case.blocks, case.leaves_b, case.op.leaves, U, V, X)
    _say(f"[parity] per-block n={case.n} nrhs={nrhs} formats {sorted(set(a.fmt))}")
    yg = _gpu_product(h, X, "fp64")
    st = check(yg, y, z, case.chain(), "fp32", "fp64", "per-block")
    _say(f"    ok {st}")


@pytest.mark.parametrize("fmt", ["fp64", "fp32", "bf16", "fp16", "e4m3", "e5m2"])
def test_forced_format_every_level(fmt):
    """Alg. "Mixed-precision HODLR Format" with one format at every level."""
    case = Case("c2_s", n=4096, depth=4, eps=1e-3)
    h = case.library_op()
    h.set_level_precisions([fmt] * case.depth, H.ACC_FP32)
    for b in (0, h.nblocks - 1):
        uc, ue, vc, ve = h.export_block(b, from_device=True)
        qu = Q.quantize(case.op.U[b], fmt)
        assert np.array_equal(uc, qu.codes) and np.array_equal(ue, qu.exps)
    for nrhs in (1, 4, 24):
        _run(case, h, [fmt] * case.depth, nrhs, "fp32", "fp32", f"forced-{fmt}")


@pytest.mark.parametrize("fmt,ranks,flags", STACKED_CASES)
def test_leaf_stacked_contraction_matrix_cores(fmt, ranks, flags):
    """The matrix-core contraction on leaf-stacked tiles (k_contract_w and
    k_reduce_stack): every code format, 1 to 4 tiles per leaf, fp32 and
    fp64 sums, ragged leaves, fp32 and fp64 X."""
    case = RandomCase(3000, 4, ranks, seed=6)
    h = case.library_op()
    h.set_level_precisions([fmt] * 4, flags)
    assert h.query()["leaf_stacked"]
    acc = "fp64" if flags == H.ACC_FP64 else "fp32"
    rng = np.random.default_rng(8)
    for xy, nrhs in (("fp32", 8), ("fp32", 40), ("fp64", 16)):
        X = rng.standard_normal((case.n, nrhs))
        if xy == "fp32":
            X = X.astype(np.float32).astype(np.float64)
        _run(case, h, [fmt] * 4, nrhs, xy, acc, f"stacked-{fmt}", X=X)


def test_leaf_stacked_contraction_deep_tree():
    """Depth 7 with a large top-level rank: many leaves per column node and
    four stacked tiles per leaf on the matrix cores."""
    n, depth, ranks = DEEP_STACKED
    case = RandomCase(n, depth, ranks, seed=10)
    h = case.library_op()
    h.set_level_precisions(["e4m3"] * depth, H.ACC_FP32)
    assert h.query()["leaf_stacked"]
    X = np.random.default_rng(11).standard_normal((n, 40)).astype(np.float32).astype(np.float64)
    _run(case, h, ["e4m3"] * depth, 40, "fp32", "fp32", "stacked-deep", X=X)


def test_mixed_formats_and_fp64_accumulation():
    case = Case("c2_s", n=4096, depth=5, eps=1e-3)
    fm = ["fp64", "fp32", "bf16", "fp16", "e4m3"]
    h = case.library_op()
    h.set_level_precisions(fm, H.ACC_FP64)
    assert h.info()["acc_dtype"] == "fp64"
    _run(case, h, fm, 3, "fp32", "fp64", "mixed-acc64")
    _run(case, h, fm, 19, "fp32", "fp64", "mixed-acc64-wide")
    _run(case, h, fm, 16, "fp64", "fp64", "mixed-acc64-xy64-wide")
    h.set_level_precisions(["e5m2", "fp16", "bf16", "fp32", "fp64"])
    _run(case, h, ["e5m2", "fp16", "bf16", "fp32", "fp64"], 2, "fp64", "fp32", "mixed-xy64")
    _run(case, h, ["e5m2", "fp16", "bf16", "fp32", "fp64"], 40, "fp64", "fp32", "mixed-xy64-wide")


@pytest.mark.parametrize("cfg", ["mat1", "mat2", "mat3", "mat4"])
def test_paper_kernels_padded_leaves(cfg):
    """n = 2000, depth 8: leaves of 7-8 rows, padded to 16 on the device."""
    case = Case(cfg)
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    a = case.oracle_assign(case.cfg.allowed)
    assert [lv[0] for lv in h.levels()] == a.fmt
    X, yg, _, _ = _run(case, h, a.fmt, 2, "fp64", h.info()["acc_dtype"], cfg)
    X2, yg2, _, _ = _run(case, h, a.fmt, 20, "fp64", h.info()["acc_dtype"], cfg + "-wide")
    A = case.cfg.kernel.dense(case.P)
    nA = np.sqrt(case.op.norm2_all)
    for j in range(20):
        eta = np.linalg.norm(yg2[:, j] - A @ X2[:, j]) / (nA * np.linalg.norm(X2[:, j]))
        assert eta <= BD.matvec_backward_bound(case.depth, case.eps)
    for j in range(2):
        eta = np.linalg.norm(yg[:, j] - A @ X[:, j]) / (nA * np.linalg.norm(X[:, j]))
        assert eta <= BD.matvec_backward_bound(case.depth, case.eps)


def test_edge_cases_depth0_n1_rank0_empty_leaves():
    # depth 0: a single dense leaf
    rng = np.random.default_rng(3)
    D = rng.standard_normal((37, 37))
    h = H.Operator(37, 0, [D], [], [])
    for nrhs in (2, 16, 21):
        X = rng.standard_normal((37, nrhs))
        yg = _gpu_product(h, X, "fp64")
        assert np.allclose(yg, D @ X, rtol=0, atol=1e-13 * np.abs(D).sum())
    # n = 1
    h1 = H.Operator(1, 0, [np.array([[2.5]])], [], [])
    assert _gpu_product(h1, np.array([[4.0]]), "fp64")[0, 0] == 10.0
    assert (_gpu_product(h1, np.full((1, 16), 4.0), "fp64") == 10.0).all()
    # rank-0 blocks everywhere, ragged leaves
    case = Case("c2_s", n=999, depth=3, eps=0.99)
    h2 = case.library_op()
    h2.set_level_precisions(["fp32"] * 3)
    _run(case, h2, ["fp32"] * 3, 1, "fp32", "fp32", "eps0.99")
    _run(case, h2, ["fp32"] * 3, 17, "fp32", "fp32", "eps0.99-wide")
    # empty leaves (given leaf bounds)
    case3 = Case("c2_s", n=600, depth=2, eps=1e-4, leaf_bounds=[0, 0, 250, 250, 600])
    h3 = case3.library_op()
    h3.set_level_precisions(["fp32", "fp16"])
    _run(case3, h3, ["fp32", "fp16"], 3, "fp32", "fp32", "empty-leaves")
    _run(case3, h3, ["fp32", "fp16"], 16, "fp32", "fp32", "empty-leaves-wide")


@pytest.mark.parametrize("nrhs", [16, 40])
def test_wide_large_leaves(nrhs):
    """Leaves of 1024 rows (eight 128-row expansion tiles per leaf, V chunks
    of several items per block) on the matrix-core path, fp32 and fp64."""
    case = Case("c2_s", n=4096, depth=2, eps=1e-5)
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    fm = [lv[0] for lv in h.levels()]
    _run(case, h, fm, nrhs, "fp32", "fp32", "large-leaves")
    h.set_level_precisions(["fp64", "e4m3"], H.ACC_FP64)
    _run(case, h, ["fp64", "e4m3"], nrhs, "fp64", "fp64", "large-leaves-fp64")


@pytest.mark.parametrize("nrhs", [5, 20])
def test_strided_unaligned_x_and_y(nrhs):
    """ld of X and Y not a multiple of 4 elements (unpadded operator): the
    wave path reads X in place, the matrix-core path through its copy."""
    case = Case("c2_s", n=4096, depth=4, eps=1e-4)
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    fm = [lv[0] for lv in h.levels()]
    X = case.cfg.X(nrhs)[:4096]
    Xb = torch.zeros(nrhs, 4096 + 1, dtype=torch.float32, device=DEV)
    Xv = Xb[:, :4096].t()
    Xv.copy_(torch.from_numpy(X).float())
    Yb = torch.full((nrhs, 4096 + 3), 7.0, dtype=torch.float32, device=DEV)
    Yv = Yb[:, :4096].t()
    _say(f"[parity] strided n=4096 nrhs={nrhs} ldx=4097 ldy=4099")
    h.matvec(Xv, Yv)
    torch.cuda.synchronize()
    y, z, _, _ = case.oracle_product(fm, X.astype(np.float32).astype(np.float64))
    st = check(Yv.cpu().double().numpy(), y, z, case.chain(), "fp32", "fp32", "strided")
    assert (Yb[:, 4096:] == 7.0).all()       # nothing written past the n rows of each column
    _say(f"    ok {st}")


def test_deterministic_and_stream_safe():
    case = Case("c2_s", n=4096, depth=4, eps=1e-5)
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    X = case.cfg.X(4)[:4096]
    Xd = H.colmajor_empty(4096, 4, torch.float32, DEV)
    Xd.copy_(torch.from_numpy(np.asfortranarray(X)).float())
    y1 = h.matvec(Xd).clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        y2 = h.matvec(Xd, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    X = case.cfg.X(32)[:4096]
    Xw = H.colmajor_empty(4096, 32, torch.float32, DEV)
    Xw.copy_(torch.from_numpy(np.asfortranarray(X)).float())
    w1 = h.matvec(Xw).clone()
    with torch.cuda.stream(s):
        w2 = h.matvec(Xw, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(w1, w2)


@pytest.mark.slow
def test_c2_full_size_bench_workload():
    """The benchmarked workload at full size (n = 65536, depth 8)."""
    case = Case("c2")
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    a = case.oracle_assign(case.cfg.allowed)
    assert [lv[0] for lv in h.levels()] == a.fmt
    for nrhs in (1, 32):
        _run(case, h, a.fmt, nrhs, "fp32", "fp32", "c2-full")


def test_captured_product_survives_workspace_growth():
    """A product captured into a graph keeps its workspace: a later call on
    the same stream with more right-hand sides replaces the stream's
    workspace, and the graph must still replay correctly."""
    case = Case("c2_s", n=4096, depth=4, eps=1e-5)
    h = case.library_op()
    h.assign_precision(case.eps, case.cfg.allowed, case.norms2)
    X = case.cfg.X(32)[:4096]
    X1 = H.colmajor_empty(4096, 1, torch.float32, DEV)
    X1.copy_(torch.from_numpy(np.asfortranarray(X[:, :1])).float())
    Xw = H.colmajor_empty(4096, 32, torch.float32, DEV)
    Xw.copy_(torch.from_numpy(np.asfortranarray(X)).float())
    Y1 = H.colmajor_empty(4096, 1, torch.float32, DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        h.matvec(X1, Y1, stream=s)                # sizes this stream's workspace, outside capture
    s.synchronize()
    ref = Y1.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        h.matvec(X1, Y1, stream=s)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        Yw = h.matvec(Xw, stream=s)               # grows the workspace of stream s
    s.synchronize()
    for rep in range(3):
        Y1.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y1, ref), rep
        with torch.cuda.stream(s):
            h.matvec(Xw, Yw, stream=s)
        s.synchronize()
    del g
