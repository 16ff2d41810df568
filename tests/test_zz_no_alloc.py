"""The allocation-free product (``hodlr_matvec_noalloc``) against
``hodlr_matvec`` and the oracle, through the C ABI.

The entry point runs the same kernels with its workspace in the library's
static scratch array, so its result must equal hodlr_matvec's bit for bit,
and both must meet the oracle's componentwise tolerance.  Calls follow one
another on one stream with different operators and sizes (the second
smaller than the first), so a layout or counter left over from an earlier
call would show.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.parity_util import Case, check  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2407_21637_amd as H  # noqa: E402

DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cases():
    big = Case("c2_s", n=4096, depth=4, eps=1e-5)
    small = Case("c2_s", n=2048, depth=3, eps=1e-5)
    out = []
    for c in (big, small):
        h = c.library_op()
        h.assign_precision(c.eps, c.cfg.allowed, c.norms2)
        out.append((c, h, [lv[0] for lv in h.levels()]))
    return out


def _x(c, nrhs):
    X = c.cfg.X(nrhs)[: c.n].astype(np.float32).astype(np.float64)
    Xd = H.colmajor_empty(c.n, nrhs, torch.float32, DEV)
    Xd.copy_(torch.from_numpy(np.asfortranarray(X)).float())
    return X, Xd


@pytest.mark.parametrize("sizes", [((0, 16), (1, 1)), ((0, 4), (1, 2)), ((1, 8), (0, 1))])
def test_noalloc_equals_matvec_on_consecutive_calls(cases, sizes):
    for ci, nrhs in sizes + ((0, 3),):
        c, h, fm = cases[ci]
        _say(f"[noalloc] n={c.n} depth={c.depth} nrhs={nrhs} fmts={fm}")
        X, Xd = _x(c, nrhs)
        Yn = H.colmajor_empty(c.n, nrhs, torch.float32, DEV)
        Yn.fill_(-7.0)
        h.matvec_noalloc(Xd, Yn)
        Ym = h.matvec(Xd)
        torch.cuda.synchronize()
        assert torch.equal(Yn, Ym), (c.n, nrhs)
        y, z, _, _ = c.oracle_product(fm, X)
        st = check(Yn.cpu().double().numpy(), y, z, c.chain(), h.info()["acc_dtype"], "fp32", "noalloc")
        _say(f"    ok {st}")


def test_noalloc_fp64_and_strided(cases):
    c, h, fm = cases[1]
    nrhs = 2
    X = c.cfg.X(nrhs)[: c.n]
    Xb = torch.zeros((nrhs, c.n + 3), dtype=torch.float64, device=DEV)
    Xv = Xb.t()[: c.n]
    Xv.copy_(torch.from_numpy(np.asfortranarray(X)))
    Yb = torch.full((nrhs, c.n + 5), 9.0, dtype=torch.float64, device=DEV)
    Yv = Yb.t()[: c.n]
    h.matvec_noalloc(Xv, Yv)
    Ym = h.matvec(Xv)
    torch.cuda.synchronize()
    assert torch.equal(Yv, Ym)
    assert (Yb[:, c.n:] == 9.0).all()


def test_noalloc_refuses_what_it_cannot_do(cases):
    c, h, fm = cases[0]
    # a workspace beyond the scratch array: refused before anything is enqueued
    nrhs = 4096
    Xd = H.colmajor_empty(c.n, nrhs, torch.float32, DEV)
    Yd = H.colmajor_empty(c.n, nrhs, torch.float32, DEV)
    with pytest.raises(H.HodlrError) as e:
        h.matvec_noalloc(Xd, Yd)
    assert e.value.status == 1 and "bytes" in str(e.value)
    # the low working precision needs its per-assignment operand
    Xw = H.colmajor_empty(c.n, 1, torch.bfloat16, DEV)
    with pytest.raises(H.HodlrError) as e:
        h.matvec_noalloc(Xw, H.colmajor_empty(c.n, 1, torch.bfloat16, DEV))
    assert e.value.status == 6
