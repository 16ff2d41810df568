"""GPU parity of the batched product (``hodlr_matvec_batched``).

A batch of 24 operators of uneven size, depth, kernel, eps, formats, nrhs
(1, 8, 32: both product paths) and X dtype runs as a handful of persistent
launches.  Each Y_i is compared with the oracle's product of the same stored
operator under the componentwise tolerance, and with the single-operator
call on the same inputs (bit for bit: the batched kernels run the same
device code on the same data).  Repeated calls (graph replay), a capture
inside a caller's graph, and a batch whose handle set changes are covered;
so are groups of leaf-stacked operators whose units all hold at most two
tiles (the batch's 2-tile contraction kernel) or mix one and four.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.parity_util import RandomCase, check  # noqa: E402
from hodlr_inputs import batch as BT  # noqa: E402
from hodlr_inputs.compress import compress  # noqa: E402
from oracle import assign as AS  # noqa: E402
from oracle import bounds as BD  # noqa: E402
from oracle import matvec as MV  # noqa: E402
from oracle import quantize as Q  # noqa: E402
from oracle import tree as T  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2407_21637_amd as H  # noqa: E402

DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Item:
    def __init__(self, spec):
        self.spec = spec
        n, d = spec.n, spec.depth
        self.blocks = T.blocks(n, d)
        self.leaves = T.leaves(n, d)
        P = spec.points()
        self.op = compress(spec.kernel, P, [(b.row0, b.nrows, b.col0, b.ncols) for b in self.blocks],
                           self.leaves, spec.eps, "frob")
        self.norms2 = np.concatenate([[self.op.norm2_all], self.op.norm2_blocks])
        self.h = H.Operator(n, d, self.op.leaves, self.op.U, self.op.V, device=0)
        self.h.assign_precision(spec.eps, BT.ALLOWED, self.norms2)
        lv = AS.level_max_norm2(self.op.norm2_blocks, [b.level for b in self.blocks])
        self.fmts = AS.assign(self.op.norm2_all, lv, spec.eps, BT.ALLOWED).fmt
        self.X = spec.X()
        dt = torch.float64 if spec.x_dtype == "fp64" else torch.float32
        self.Xd = H.colmajor_empty(n, spec.nrhs, dt, DEV)
        self.Xd.copy_(torch.from_numpy(np.asfortranarray(self.X)).to(dt))
        self.Y = H.colmajor_empty(n, spec.nrhs, dt, DEV)

    def oracle(self):
        U = [Q.quantize(u, self.fmts[b.level - 1]).values for b, u in zip(self.blocks, self.op.U)]
        V = [Q.quantize(v, self.fmts[b.level - 1]).values for b, v in zip(self.blocks, self.op.V)]
        y = MV.matvec(self.spec.n, self.blocks, self.leaves, self.op.leaves, U, V, self.X)
        z = MV.matvec_abs(self.spec.n, self.blocks, self.leaves, self.op.leaves, U, V, self.X)
        M = BD.chain_length(self.blocks, self.op.ranks, [m for _, m in self.leaves], self.spec.depth)
        return y, z, M


@pytest.fixture(scope="module")
def batch():
    items = [Item(s) for s in BT.get("c4_s")]
    _say(f"[batched] {len(items)} operators, n {min(i.spec.n for i in items)}..{max(i.spec.n for i in items)}, "
         f"nrhs {sorted(set(i.spec.nrhs for i in items))}")
    return items


def test_batched_matches_oracle_and_single(batch):
    for it in batch:
        assert [lv[0] for lv in it.h.levels()] == it.fmts
    H.matvec_batched([it.h for it in batch], [it.Xd for it in batch], [it.Y for it in batch])
    torch.cuda.synchronize()
    first = [it.Y.clone() for it in batch]
    for k, it in enumerate(batch):
        y, z, M = it.oracle()
        acc = it.h.info()["acc_dtype"]
        st = check(it.Y.cpu().double().numpy(), y, z, M, acc, it.spec.x_dtype, f"batch[{k}]")
        single = it.h.matvec(it.Xd)
        torch.cuda.synchronize()
        assert torch.equal(single, first[k]), k
        _say(f"    [{k}] n={it.spec.n} depth={it.spec.depth} nrhs={it.spec.nrhs} {it.spec.x_dtype} "
             f"fmts={it.fmts} ok {st['max_err_over_tau_prob']:.2e}")
    # second call: the cached plan's graph is replayed
    for it in batch:
        it.Y.zero_()
    H.matvec_batched([it.h for it in batch], [it.Xd for it in batch], [it.Y for it in batch])
    torch.cuda.synchronize()
    for k, it in enumerate(batch):
        assert torch.equal(it.Y, first[k]), k


def test_batched_inside_caller_graph(batch):
    items = batch[:10]
    hs, Xs, Ys = [it.h for it in items], [it.Xd for it in items], [it.Y for it in items]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        H.matvec_batched(hs, Xs, Ys, stream=s)      # plan for this stream, outside capture
    s.synchronize()
    ref = [y.clone() for y in Ys]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        H.matvec_batched(hs, Xs, Ys, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for y in Ys:
            y.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, y in enumerate(Ys):
            assert torch.equal(y, ref[k]), (rep, k)
    del g


def test_batched_new_handle_set_and_duplicates(batch):
    # a handle twice is refused before anything runs
    items = batch[3:9]
    with pytest.raises(RuntimeError, match="more than once"):
        H.matvec_batched([items[0].h, items[0].h], [items[0].Xd, items[0].Xd],
                         [items[0].Y, torch.empty_like(items[0].Y)])
    # a different subset gets its own plan
    H.matvec_batched([it.h for it in items], [it.Xd for it in items], [it.Y for it in items])
    torch.cuda.synchronize()
    for it in items:
        single = it.h.matvec(it.Xd)
        torch.cuda.synchronize()
        assert torch.equal(single, it.Y)


def test_tuned_and_untuned_launches_agree(batch, tmp_path, monkeypatch):
    """Every launch shape the autotuner may choose gives the same result bit
    for bit: the batch with tuning off (default shapes) equals the tuned
    batch, and choices land in the tuning-cache file named by the
    environment."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HODLR_TUNE_CACHE", str(cache))
    items = batch[2:14]
    hs, Xs = [it.h for it in items], [it.Xd for it in items]
    Ya = [torch.empty_like(it.Y) for it in items]
    H.matvec_batched(hs, Xs, Ya)                  # new signature (Y pointers): a tuned plan
    torch.cuda.synchronize()
    monkeypatch.setenv("HODLR_BATCH_TUNE", "0")
    Yb = [torch.empty_like(it.Y) for it in items]
    H.matvec_batched(hs, Xs, Yb)                  # another new signature, default shapes
    torch.cuda.synchronize()
    for k in range(len(items)):
        assert torch.equal(Ya[k], Yb[k]), k
    if cache.exists():                            # shapes new to this process were timed and stored
        for line in cache.read_text().splitlines():
            key, o, m = line.split()
            assert "|x" in key and o in ("0", "1") and m in ("1", "2", "4", "8")


# (format, ranks per level, accumulation flag, X dtype, nrhs): operators whose
# every leaf is one stacked unit; "two" has no unit above 2 tiles in any
# group, "mixed" puts 1- and 4-tile units in one group
STACKED_BATCHES = {
    "two": [("e5m2", [5, 4, 4, 3], H.ACC_FP32, "fp32", 8), ("e4m3", [4, 4, 4, 4], H.ACC_FP32, "fp32", 40),
            ("fp32", [8, 8, 8, 8], H.ACC_FP64, "fp32", 16), ("fp64", [8, 8, 8, 8], H.ACC_FP32, "fp64", 16)],
    "mixed": [("e4m3", [16, 16, 16, 16], H.ACC_FP32, "fp32", 40), ("e5m2", [5, 4, 4, 3], H.ACC_FP32, "fp32", 40),
              ("bf16", [12, 12, 12, 12], H.ACC_FP32, "fp32", 24)],
}


@pytest.mark.parametrize("which", sorted(STACKED_BATCHES))
def test_batched_leaf_stacked_groups(which):
    rng = np.random.default_rng(21)
    items = []
    for i, (fmt, ranks, flags, xy, nrhs) in enumerate(STACKED_BATCHES[which]):
        case = RandomCase(3000, 4, ranks, seed=30 + i)
        h = case.library_op()
        h.set_level_precisions([fmt] * 4, flags)
        assert h.query()["leaf_stacked"]
        X = rng.standard_normal((case.n, nrhs))
        if xy == "fp32":
            X = X.astype(np.float32).astype(np.float64)
        dt = torch.float64 if xy == "fp64" else torch.float32
        Xd = H.colmajor_empty(case.n, nrhs, dt, DEV)
        Xd.copy_(torch.from_numpy(np.asfortranarray(X)).to(dt))
        items.append((case, h, fmt, xy, X, Xd, H.colmajor_empty(case.n, nrhs, dt, DEV)))
    _say(f"[batched] stacked groups '{which}': {[(it[2], it[4].shape[1]) for it in items]}")
    H.matvec_batched([it[1] for it in items], [it[5] for it in items], [it[6] for it in items])
    torch.cuda.synchronize()
    for k, (case, h, fmt, xy, X, Xd, Y) in enumerate(items):
        y, z, _, _ = case.oracle_product([fmt] * 4, X)
        st = check(Y.cpu().double().numpy(), y, z, case.chain(), h.info()["acc_dtype"], xy, f"stacked[{k}]")
        single = h.matvec(Xd)
        torch.cuda.synchronize()
        assert torch.equal(single, Y), k
        _say(f"    [{k}] {fmt} nrhs={X.shape[1]} {xy} ok {st['max_err_over_tau_prob']:.2e}")


def test_batched_low_working_precision_with_others():
    """bf16 and fp16 products in one batched call with fp32 and fp64 ones:
    each Y equals the single-operator product bit for bit (the same launches
    run), eagerly and when a caller's graph replays the batch."""
    rng = np.random.default_rng(41)
    spec = [("bf16", torch.bfloat16, 3, [6, 5, 4, 4]), ("fp32", torch.float32, 24, [9, 7, 5, 4]),
            ("fp16", torch.float16, 40, [16, 16, 16, 16]), ("fp64", torch.float64, 2, [5, 5, 5, 5]),
            ("bf16", torch.bfloat16, 64, [20, 20, 20, 20])]
    hs, Xs, Ys = [], [], []
    for i, (name, dt, nrhs, ranks) in enumerate(spec):
        case = RandomCase(2500 + 300 * i, 4, ranks, seed=50 + i)
        h = case.library_op()
        h.set_level_precisions(["e4m3", "bf16", "fp16", "fp32"], H.ACC_FP32)
        X = H.colmajor_empty(case.n, nrhs, dt, DEV)
        X.copy_(torch.from_numpy(np.asfortranarray(rng.standard_normal((case.n, nrhs)))).to(dt))
        hs.append(h)
        Xs.append(X)
        Ys.append(H.colmajor_empty(case.n, nrhs, dt, DEV))
    _say(f"[batched] mixed dtypes {[(s[0], s[2]) for s in spec]}")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        H.matvec_batched(hs, Xs, Ys, stream=s)      # plan and W operands, outside capture
    s.synchronize()
    ref = [h.matvec(X) for h, X in zip(hs, Xs)]
    torch.cuda.synchronize()
    for k, (y, r) in enumerate(zip(Ys, ref)):
        assert torch.equal(y, r), k
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        H.matvec_batched(hs, Xs, Ys, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for y in Ys:
            y.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (y, r) in enumerate(zip(Ys, ref)):
            assert torch.equal(y, r), (rep, k)
    del g
