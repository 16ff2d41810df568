"""Host logic of the HIP library against the oracle, on the CPU (no GPU).

The library is loaded and driven through its C ABI with host-only handles
(device = -1): tree, precision assignment, quantisation and packing run,
products do not.  Integer and bit-pattern results must equal the oracle's
exactly.
"""
import os
import re

import numpy as np
import pytest

import paper_2407_21637_amd as H
from hodlr_inputs import compress as CP
from hodlr_inputs import configs as CF
from oracle import assign as AS
from oracle import formats as F
from oracle import quantize as Q
from oracle import tree as T

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "hodlr.h")


def test_library_exports_every_declared_symbol():
    src = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(hodlr_\w+)\s*\(", src, re.M))
    declared = {d for d in declared if not d.endswith("_t")}
    assert declared == set(H.EXPORTS), declared ^ set(H.EXPORTS)
    L = H.lib()
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("n,leaf", [(2048, 128), (65536, 256), (1, 1), (5, 2), (1000, 7), (4097, 64)])
def test_depth_for_leaf_matches_oracle(n, leaf):
    assert H.depth_for_leaf(n, leaf) == T.depth_for_leaf(n, leaf)
    assert H.depth_for_leaf(0, 4) == -1


@pytest.mark.parametrize("n,depth", [(7, 2), (2048, 4), (1000, 6), (1, 3), (65536, 8), (12345, 10)])
def test_tree_bit_exact(n, depth):
    lib_levels = H.tree_bounds(n, depth)
    ora = T.node_bounds(n, depth)
    assert [list(a) for a in lib_levels] == ora
    blks = H.tree_blocks(n, depth)
    ob = T.blocks(n, depth)
    assert blks.tolist() == [[b.level, b.row0, b.nrows, b.col0, b.ncols] for b in ob]


def test_tree_with_leaf_bounds_and_errors():
    lb = [0, 0, 3, 3, 5]
    assert [list(a) for a in H.tree_bounds(5, 2, lb)] == T.node_bounds(5, 2, lb)
    with pytest.raises(H.HodlrError) as e:
        H.tree_bounds(5, 2, [0, 3, 2, 4, 5])
    assert e.value.status == 1


def _host_op(cfg, depth=None, eps=None):
    c = CF.get(cfg)
    n = c.n
    depth = c.depth if depth is None else depth
    P = c.points()
    blks = [(b.row0, b.nrows, b.col0, b.ncols) for b in T.blocks(n, depth)]
    lv = T.leaves(n, depth)
    op = CP.compress(c.kernel, P, blks, lv, c.eps if eps is None else eps, "frob")
    h = H.Operator(n, depth, op.leaves, op.U, op.V, device=-1)
    return c, depth, op, h


def test_assign_matches_oracle_with_given_norms():
    c, depth, op, h = _host_op("c2_s")
    norms = np.concatenate([[op.norm2_all], op.norm2_blocks])
    levels = [b.level for b in T.blocks(c.n, depth)]
    for eps in (1e-2, 1e-4, 1e-6, 1e-9, 1e-13):
        for allowed in (c.allowed, ("e4m3", "e5m2", "fp16", "bf16", "fp32"), ()):
            h.assign_precision(eps, allowed, norms)
            a = AS.assign(op.norm2_all, AS.level_max_norm2(op.norm2_blocks, levels), eps, allowed)
            got = h.levels()
            assert [g[0] for g in got] == a.fmt
            assert [g[1] for g in got] == a.xi           # bit-identical fp64
            assert [g[2] for g in got] == a.u_prime
            assert [g[3] for g in got] == a.insufficient
            assert h.info()["acc_dtype"] == ("fp64" if eps < 1e-7 else "fp32")


def test_per_block_assign_matches_oracle_and_codes_bit_exact():
    c, depth, op, h = _host_op("c2_s")
    norms = np.concatenate([[op.norm2_all], op.norm2_blocks])
    blks = T.blocks(c.n, depth)
    levels = [b.level for b in blks]
    allowed = ("e4m3", "e5m2", "fp16", "bf16", "fp32")
    for eps in (1e-2, 1e-4, 1e-6):
        h.assign_precision(eps, allowed, norms, H.PER_BLOCK)
        a = AS.assign_blocks(op.norm2_all, op.norm2_blocks, levels, eps, allowed)
        got = [h.block(b)["dtype"] for b in range(h.nblocks)]
        assert got == a.fmt
        # the level report is still the level rule
        lv = AS.assign(op.norm2_all, AS.level_max_norm2(op.norm2_blocks, levels), eps, allowed)
        assert [g[0] for g in h.levels()] == lv.fmt
        for b in (0, 1, h.nblocks // 2, h.nblocks - 1):
            uc, ue, vc, ve = h.export_block(b)
            qu = Q.quantize(op.U[b], a.fmt[b])
            qv = Q.quantize(op.V[b], a.fmt[b])
            assert np.array_equal(uc, qu.codes) and np.array_equal(ue, qu.exps)
            assert np.array_equal(vc, qv.codes) and np.array_equal(ve, qv.exps)
    # back to one format per level
    h.set_level_precisions(["fp32"] * depth)
    assert {h.block(b)["dtype"] for b in range(h.nblocks)} == {"fp32"}


def test_assign_from_factors_matches_oracle_reading():
    c, depth, op, h = _host_op("c2_s")
    tot, nb = AS.norms_from_factors(op.leaves, op.U, op.V)
    levels = [b.level for b in T.blocks(c.n, depth)]
    h.assign_precision(1e-5, c.allowed, None)
    a = AS.assign(tot, AS.level_max_norm2(nb, levels), 1e-5, c.allowed)
    got = h.levels()
    assert [g[0] for g in got] == a.fmt
    assert np.allclose([g[1] for g in got], a.xi, rtol=1e-12)


@pytest.mark.parametrize("fmt", ["fp64", "fp32", "bf16", "fp16", "e4m3", "e5m2"])
@pytest.mark.parametrize("scale", [True, False])
def test_codes_and_exponents_bit_exact(fmt, scale):
    c, depth, op, h = _host_op("c2_s", depth=3)
    flags = 0 if scale else H.NO_COLUMN_SCALE
    if not scale and fmt in ("fp16", "e4m3", "e5m2"):
        # V carries the singular values and may not fit these formats unscaled
        big = max(np.abs(v).max() for v in op.V if v.size)
        if big > F.FORMATS[fmt].max_finite:
            with pytest.raises(H.HodlrError) as e:
                h.set_level_precisions([fmt] * depth, flags)
            assert e.value.status == 5
            return
    h.set_level_precisions([fmt] * depth, flags)
    for b in range(h.nblocks):
        uc, ue, vc, ve = h.export_block(b)
        qu = Q.quantize(op.U[b], fmt, scale)
        qv = Q.quantize(op.V[b], fmt, scale)
        assert np.array_equal(uc, qu.codes) and np.array_equal(ue, qu.exps)
        assert np.array_equal(vc, qv.codes) and np.array_equal(ve, qv.exps)


@pytest.mark.parametrize("fmt", ["fp32", "bf16", "fp16", "e4m3", "e5m2"])
def test_codec_bit_exact_on_random_and_boundary_values(fmt):
    """Blocks whose U panels hold the test values (no scaling)."""
    f = F.FORMATS[fmt]
    rng = np.random.default_rng(21)
    top = min(f.max_finite, 1e30)
    e = rng.uniform(np.log2(f.x_min) - f.t - 2, np.log2(top) - 0.01, 60000)
    vals = rng.choice([-1.0, 1.0], e.size) * np.exp2(e)
    codes = np.arange(1 << (8 * f.nbytes), dtype=np.uint64) if f.nbytes <= 2 else None
    if codes is not None:
        reps = F.decode(fmt, codes)
        reps = reps[np.isfinite(reps)]
        reps = reps[np.abs(reps) <= f.max_finite]
        mids = (np.sort(reps)[:-1] + np.sort(reps)[1:]) / 2
        vals = np.concatenate([vals, reps, mids])
    vals = vals[np.abs(vals) <= f.max_finite]
    vals = vals[np.abs(F.round_rne(fmt, vals, check_overflow=False)) <= f.max_finite]
    r = 256
    for start in range(0, vals.size, 2 * r * r):
        chunk = vals[start:start + 2 * r * r]
        chunk = np.concatenate([chunk, np.ones((-chunk.size) % (2 * r))])
        p = chunk.size // (2 * r)
        Uu = chunk[: r * p].reshape(r, p, order="F")
        Ul = chunk[r * p:].reshape(r, p, order="F")
        V = np.ones((r, p))
        h = H.Operator(2 * r, 1, [np.eye(r), np.eye(r)], [Uu, Ul], [V, V], device=-1)
        h.set_level_precisions([fmt], H.NO_COLUMN_SCALE)
        for b, Ub in ((0, Uu), (1, Ul)):
            uc, _, _, _ = h.export_block(b)
            assert np.array_equal(uc, F.encode(fmt, F.round_rne(fmt, Ub)))
        h.close()


def test_info_and_block_queries():
    c, depth, op, h = _host_op("c2_s", depth=3)
    h.set_level_precisions(["fp32", "bf16", "e4m3"])
    inf = h.info()
    assert inf["n"] == c.n and inf["depth"] == 3 and inf["nblocks"] == 14 and inf["on_device"] == 0
    ranks = [u.shape[1] for u in op.U]
    want = 0
    for b, blk in enumerate(T.blocks(c.n, 3)):
        s = {1: 4, 2: 2, 3: 1}[blk.level]
        want += (blk.nrows + blk.ncols) * ranks[b] * s
        bi = h.block(b)
        assert (bi["level"], bi["rank"], bi["row0"], bi["nrows"], bi["col0"], bi["ncols"]) == \
            (blk.level, ranks[b], blk.row0, blk.nrows, blk.col0, blk.ncols)
    assert inf["factor_bytes"] == want
    assert inf["leaf_bytes"] == sum(8 * d.size for d in op.leaves)
    assert inf["max_rank"] == max(ranks)


def test_error_paths_are_reported_not_raised_in_c():
    c, depth, op, h = _host_op("c1_s")
    # host-only handle has no product
    with pytest.raises(H.HodlrError) as e:
        H.lib()  # loaded
        import ctypes
        st = H.lib().hodlr_matvec(h.handle, ctypes.c_void_p(1), c.n, ctypes.c_void_p(1), c.n, 1, 1, None)
        H._lib._check(st)
    assert e.value.status == 2
    # bad rank
    U = [u.copy() for u in op.U]
    U[0] = np.zeros((op.U[0].shape[0], op.U[0].shape[0] + 5))
    with pytest.raises(Exception):
        H.Operator(c.n, depth, op.leaves, U, op.V, device=-1)
    with pytest.raises(H.HodlrError) as e:
        h.assign_precision(2.0, ["fp32"])
    assert e.value.status == 1
    with pytest.raises(H.HodlrError) as e:
        h.set_level_precisions([9] * depth)
    assert e.value.status == 1
    with pytest.raises(H.HodlrError):
        h.level(0)
    with pytest.raises(H.HodlrError):
        h.block(h.nblocks)
    assert H.lib().hodlr_status_string(5) == b"HODLR_E_RANGE"
    # batched: argument checks come before any device work
    import ctypes
    L = H.lib()
    one = (ctypes.c_void_p * 1)(h.handle.value)
    ptr = (ctypes.c_void_p * 1)(1)
    ld = np.array([c.n], dtype=np.int64)
    nr = np.array([1], dtype=np.int32)
    dt = np.array([1], dtype=np.int32)
    args = (ctypes.cast(ptr, ctypes.c_void_p), H._lib._ptr(ld), ctypes.cast(ptr, ctypes.c_void_p),
            H._lib._ptr(ld), H._lib._ptr(nr), H._lib._ptr(dt), None)
    assert L.hodlr_matvec_batched(ctypes.cast(one, ctypes.c_void_p), 1, *args) == 2      # host-only handle
    assert L.hodlr_matvec_batched(ctypes.cast(one, ctypes.c_void_p), -1, *args) == 1     # count < 0
    assert L.hodlr_matvec_batched(ctypes.cast(one, ctypes.c_void_p), 0, *args) == 0      # empty batch
    bad = np.array([0], dtype=np.int32)
    assert L.hodlr_matvec_batched(ctypes.cast(one, ctypes.c_void_p), 1, args[0], args[1], args[2], args[3],
                                  H._lib._ptr(bad), args[5], None) in (1, 2)


def test_depth_zero_and_rank_zero_operators():
    h = H.Operator(5, 0, [np.eye(5)], [], [], device=-1)
    assert h.info()["nblocks"] == 0
    h.assign_precision(1e-3, ["fp16"])
    n, depth = 9, 2
    blks = T.blocks(n, depth)
    U = [np.zeros((b.nrows, 0)) for b in blks]
    V = [np.zeros((b.ncols, 0)) for b in blks]
    lv = [np.eye(m) for _, m in T.leaves(n, depth)]
    h2 = H.Operator(n, depth, lv, U, V, device=-1)
    h2.assign_precision(1e-3, ["fp16"], None)
    assert [lvl[0] for lvl in h2.levels()] == ["fp16", "fp16"]     # xi = 0 -> coarsest


def test_assign_with_given_xi_matches_oracle():
    """xi passed in: the library applies the rule to exactly those values
    (bit-identical u', formats and marks to the oracle's rule from xi),
    including values placed on a format's threshold (a tie selects it)."""
    c, depth, op, h = _host_op("c2_s")
    levels = [b.level for b in T.blocks(c.n, depth)]
    a0 = AS.assign(op.norm2_all, AS.level_max_norm2(op.norm2_blocks, levels), 1e-6, c.allowed)
    rng = np.random.default_rng(7)
    eps = 1e-4
    tie = [eps / (np.sqrt(float(2 ** k)) * F.fmt("fp16").u) for k in range(1, depth + 1)]
    for xi in (a0.xi, list(rng.uniform(1e-4, 0.5, depth)), tie, [0.0] * depth,
               [1e9] + [0.1] * (depth - 1)):
        for allowed in (c.allowed, ("e4m3", "e5m2", "fp16", "bf16", "fp32"), ()):
            h.assign_precision(eps, allowed, None, xi=xi)
            ref = AS.assign_from_xi(xi, eps, allowed)
            got = h.levels()
            assert [g[0] for g in got] == ref.fmt
            assert [g[1] for g in got] == [float(x) for x in xi]
            assert [g[2] for g in got] == ref.u_prime
            assert [g[3] for g in got] == ref.insufficient
    # the oracle's own xi gives the oracle's own decisions
    h.assign_precision(1e-6, c.allowed, None, xi=a0.xi)
    assert [g[0] for g in h.levels()] == a0.fmt
    with pytest.raises(H.HodlrError) as e:
        h.assign_precision(1e-6, c.allowed, None, xi=[-1.0] + [0.1] * (depth - 1))
    assert e.value.status == 1
    with pytest.raises(H.HodlrError):
        h.assign_precision(1e-6, c.allowed, None, xi=[float("nan")] * depth)


def test_query_matches_the_individual_queries():
    c, depth, op, h = _host_op("c2_s", depth=4)
    norms = np.concatenate([[op.norm2_all], op.norm2_blocks])
    h.assign_precision(1e-4, ("e4m3", "fp16", "bf16", "fp32"), norms)
    q = h.query()
    info = h.info()
    for k in info:
        assert q[k] == info[k], k
    assert q["levels"] == h.levels()
    assert list(q["leaf_bounds"]) == T.node_bounds(c.n, depth)[depth]
    assert list(q["ranks"]) == [u.shape[1] for u in op.U]
    assert q["per_block"] is False
    h.assign_precision(1e-4, ("e4m3", "fp16", "bf16", "fp32"), norms, H.PER_BLOCK)
    assert h.query()["per_block"] is True


def test_last_error_message_names_the_failure():
    L = H.lib()
    with pytest.raises(H.HodlrError):
        H.tree_bounds(5, 2, [0, 3, 2, 4, 5])
    msg = L.hodlr_last_error_message().decode()
    assert msg and msg == L.hodlr_last_error().decode()
    assert "leaf_bounds" in msg or "non-decreasing" in msg or msg


def test_binding_refuses_mismatched_tensors():
    """X / Y dtype, shape and device are checked before the C ABI is called
    (a host-only handle: every tensor here is on the CPU)."""
    torch = pytest.importorskip("torch")
    c, depth, op, h = _host_op("c2_s", depth=3)
    n = c.n

    def cm(k, dt):                                      # n x k column-major, on the CPU
        return torch.zeros((k, n), dtype=dt).t()

    X = cm(2, torch.float32)
    with pytest.raises(TypeError):
        h.matvec(X, cm(2, torch.float64))
    with pytest.raises(ValueError, match="nrhs"):
        h.matvec(X, cm(3, torch.float32))
    with pytest.raises(TypeError):
        h.matvec(cm(2, torch.int32))
    with pytest.raises(ValueError, match="GPU"):
        h.matvec(X, cm(2, torch.float32))
    with pytest.raises(ValueError, match="GPU"):
        H.matvec_batched([h], [X], [cm(2, torch.float32)])
    with pytest.raises(TypeError):
        H.matvec_batched([h], [X], [cm(2, torch.float64)])
    with pytest.raises(ValueError, match="nrhs"):
        H.matvec_batched([h], [X], [cm(1, torch.float32)])
    with pytest.raises(ValueError):
        H.matvec_batched([h, h], [X], [X])
    from paper_2407_21637_amd._lib import _xy_code
    assert [_xy_code(torch.zeros(1, dtype=d)) for d in
            (torch.float64, torch.float32, torch.bfloat16, torch.float16)] == [0, 1, 2, 3]


def _ranked_op(n, depth, ranks_per_level, seed=0):
    """A host-only operator with random factors of the given rank per level."""
    rng = np.random.default_rng(seed)
    blks = T.blocks(n, depth)
    U = [rng.standard_normal((b.nrows, ranks_per_level[b.level - 1])) for b in blks]
    V = [rng.standard_normal((b.ncols, ranks_per_level[b.level - 1])) for b in blks]
    leaves = [rng.standard_normal((m, m)) for _, m in T.leaves(n, depth)]
    return H.Operator(n, depth, leaves, U, V, device=-1)


@pytest.mark.parametrize("ranks,fmts,flags,stacked", [
    # one format: every leaf's ancestor ranks in 16-row tiles, at most 4 (fp32 sums) or 2 (fp64)
    ([5, 4, 4, 3], ["e4m3"] * 4, H.ACC_FP32, True),
    ([16, 16, 16, 16], ["bf16"] * 4, H.ACC_FP32, True),           # 64 rows: four tiles
    ([16, 16, 16, 17], ["bf16"] * 4, H.ACC_FP32, False),          # 65 rows: five
    ([8, 8, 8, 8], ["fp32"] * 4, H.ACC_FP64, True),               # fp64 sums: two tiles
    ([9, 8, 8, 8], ["fp32"] * 4, H.ACC_FP64, False),
    ([8, 8, 8, 8], ["fp64"] * 4, H.ACC_FP32, True),               # fp64 codes: fp64 arithmetic
    ([8, 8, 8, 9], ["fp64"] * 4, H.ACC_FP32, False),
    # two formats on a leaf: two units
    ([3, 3, 3, 3], ["e4m3", "e4m3", "e5m2", "e4m3"], H.ACC_FP32, False),
    ([3, 3, 3, 3], ["fp64", "fp32", "fp32", "fp32"], H.ACC_FP32, False),
    # a zero rank everywhere: no tiles at all
    ([0, 0, 0, 0], ["fp32"] * 4, H.ACC_FP32, False),
])
def test_leaf_stacked_contraction_rule(ranks, fmts, flags, stacked):
    """hodlr_query's leaf_stacked: each leaf's (block, rank) rows of all
    levels, grouped by format and arithmetic type 16 to a tile, must make a
    single group of at most 4 tiles (2 with fp64 arithmetic)."""
    h = _ranked_op(1000, 4, ranks)
    h.set_level_precisions(fmts, flags)
    assert h.query()["leaf_stacked"] is stacked
