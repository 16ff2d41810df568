"""Pins for the oracle's formats and codecs (no GPU).

The oracle's rounding and bit patterns are checked against things that do
not come from it: the paper's printed Table 1.1, numpy's and torch's own
casts (library routines), and brute-force nearest-even search over every
code of the 8-bit formats.
"""
import os

import numpy as np
import pytest
import torch

from oracle import formats as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table_1_1_unit_roundoff.txt")


def _sig3(x):
    return float(f"{x:.2e}")


def test_table_1_1_constants():
    """Table 1.1: u, x_min, x_max, t, e_min, e_max of each format."""
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    names = {"q52": "e5m2", "bf16": "bf16", "fp16": "fp16", "fp32": "fp32", "fp64": "fp64"}
    assert len(rows) == 5
    for name, u, xmin, xmax, t, emin, emax in rows:
        f = F.FORMATS[names[name]]
        assert _sig3(f.u) == float(u), name
        assert _sig3(f.x_min) == float(xmin), name
        assert _sig3(f.max_finite) == float(xmax), name
        assert f.emin == int(emin) and f.emax == int(emax), name
        if name == "q52":
            assert int(t) == -16 and f.t == 3          # garbled row, see header
        else:
            assert f.t == int(t), name


def _all_codes(nbits):
    return np.arange(1 << nbits, dtype=np.uint64)


def _torch_decode(codes, tdtype, view_int):
    t = torch.from_numpy(codes.astype(view_int)).view(tdtype)
    return t.to(torch.float64).numpy()


@pytest.mark.parametrize("name,tdtype", [("e4m3", torch.float8_e4m3fn), ("e5m2", torch.float8_e5m2)])
def test_decode_exhaustive_fp8_vs_torch(name, tdtype):
    codes = _all_codes(8)
    mine = F.decode(name, codes)
    ref = _torch_decode(codes, tdtype, np.uint8)
    same = (mine == ref) | (np.isnan(mine) & np.isnan(ref))
    assert same.all()


def test_decode_exhaustive_fp16_vs_numpy():
    codes = _all_codes(16)
    mine = F.decode("fp16", codes)
    ref = codes.astype(np.uint16).view(np.float16).astype(np.float64)
    same = (mine == ref) | (np.isnan(mine) & np.isnan(ref))
    assert same.all()


def test_decode_exhaustive_bf16_vs_torch():
    codes = _all_codes(16)
    mine = F.decode("bf16", codes)
    ref = _torch_decode(codes.astype(np.int64).astype(np.int16), torch.bfloat16, np.int16)
    same = (mine == ref) | (np.isnan(mine) & np.isnan(ref))
    assert same.all()


def _random_doubles(rng, n, lo_exp, hi_exp):
    e = rng.uniform(lo_exp, hi_exp, n)
    return rng.choice([-1.0, 1.0], n) * np.exp2(e) * rng.uniform(1, 2, n)


def test_round_fp32_fp16_vs_numpy_casts():
    rng = np.random.default_rng(11)
    x = np.concatenate([_random_doubles(rng, 200000, -30, 15),
                        _random_doubles(rng, 50000, -26, -13)])   # fp16 subnormals
    x = x[np.abs(x) < 65504]
    r16 = F.round_rne("fp16", x)
    assert np.array_equal(r16, x.astype(np.float16).astype(np.float64))
    y = _random_doubles(rng, 200000, -150, 120)
    assert np.array_equal(F.round_rne("fp32", y), y.astype(np.float32).astype(np.float64))


def test_round_bf16_fp8_vs_torch_on_fp32_exact_inputs():
    """torch rounds fp32 -> bf16/fp8 once; on fp32-exact inputs that is the
    single rounding from fp64 the oracle does."""
    rng = np.random.default_rng(12)
    x32 = _random_doubles(rng, 100000, -140, 120).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(F.round_rne("bf16", x32.astype(np.float64)), ref)
    for name, td, top in (("e4m3", torch.float8_e4m3fn, 448.0), ("e5m2", torch.float8_e5m2, 57344.0)):
        x = _random_doubles(rng, 100000, -22, 16).astype(np.float32)
        x = x[np.abs(x) <= top]
        ref = torch.from_numpy(x).to(td).to(torch.float64).numpy()
        assert np.array_equal(F.round_rne(name, x.astype(np.float64)), ref), name


@pytest.mark.parametrize("name", ["e4m3", "e5m2"])
def test_round_fp8_brute_force_nearest_even(name):
    """Every finite code is a candidate; the nearest wins, ties go to the
    code with an even last bit."""
    f = F.FORMATS[name]
    codes = np.arange(256, dtype=np.uint64)
    vals = F.decode(name, codes)
    fin = np.isfinite(vals)
    cv, cc = vals[fin], codes[fin]
    rng = np.random.default_rng(13)
    x = np.concatenate([rng.uniform(-f.max_finite, f.max_finite, 4000),
                        _random_doubles(rng, 4000, f.emin - 4, f.emin + 2),
                        (cv[:-1] + cv[1:]) / 2])            # includes midpoints
    x = x[np.abs(x) <= f.max_finite]
    got = F.round_rne(name, x)
    for xi, gi in zip(x, got):
        d = np.abs(cv - xi)
        best = d.min()
        cand = cc[d == best]
        cvals = cv[d == best]
        if len(cand) > 1:
            even = cand[(cand & np.uint64(1)) == 0]
            want = cvals[np.isin(cand, even)]
            want = want[0] if not np.all(want == 0) else want[0]
        else:
            want = cvals[0]
        assert gi == want or (gi == 0 and want == 0), (xi, gi, want)


def test_encode_matches_library_bit_patterns():
    rng = np.random.default_rng(14)
    x = _random_doubles(rng, 50000, -24, 15)
    x = x[np.abs(x) < 65504]
    r = F.round_rne("fp16", x)
    assert np.array_equal(F.encode("fp16", r), x.astype(np.float16).view(np.uint16))
    x32 = _random_doubles(rng, 50000, -130, 120).astype(np.float32)
    rb = F.round_rne("bf16", x32.astype(np.float64))
    ref = torch.from_numpy(x32).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(F.encode("bf16", rb), ref)
    for name, td in (("e4m3", torch.float8_e4m3fn), ("e5m2", torch.float8_e5m2)):
        f = F.FORMATS[name]
        xs = rng.uniform(-f.max_finite, f.max_finite, 20000).astype(np.float32)
        rr = F.round_rne(name, xs.astype(np.float64))
        ref = torch.from_numpy(xs).to(td).view(torch.uint8).numpy()
        enc = F.encode(name, rr)
        # -0.0 and +0.0 agree as values; compare the codes of non-zeros
        nz = rr != 0
        assert np.array_equal(enc[nz], ref[nz]), name
    y = _random_doubles(rng, 1000, -100, 100)
    assert np.array_equal(F.encode("fp64", y), y.view(np.uint64))
    assert np.array_equal(F.decode("fp32", F.encode("fp32", F.round_rne("fp32", y))),
                          y.astype(np.float32).astype(np.float64))


def test_overflow_is_detected():
    assert F.round_rne("fp16", np.array([65519.0]))[0] == 65504.0
    with pytest.raises(F.OverflowInFormat):
        F.round_rne("fp16", np.array([65520.0]))
    assert F.round_rne("e4m3", np.array([464.0]))[0] == 448.0     # tie -> even
    with pytest.raises(F.OverflowInFormat):
        F.round_rne("e4m3", np.array([465.0]))
    r = F.round_rne("fp16", np.array([70000.0]), check_overflow=False)
    assert np.isinf(r[0])


@pytest.mark.parametrize("name", ["fp16", "e4m3", "e5m2"])
def test_column_scale_exponent_is_largest_safe_power(name):
    f = F.FORMATS[name]
    rng = np.random.default_rng(15)
    amax = np.concatenate([_random_doubles(rng, 20000, -60, 60), [f.max_finite, 1.0, 0.0],
                           np.nextafter(f.max_finite, np.inf) * np.ones(1)])
    amax = np.abs(amax)
    e = F.column_scale_exponent(name, amax)
    nz = amax > 0
    assert np.all(np.ldexp(amax[nz], e[nz]) <= f.max_finite)
    assert np.all(np.ldexp(amax[nz], e[nz] + 1) > f.max_finite)
    assert np.all(e[~nz] == 0)


def test_unit_roundoff_ordering_has_no_ties():
    """The candidate set has distinct unit roundoffs, so the adaptive rule
    never has to break a tie between formats."""
    us = sorted(f.u for f in F.FORMATS.values())
    assert len(set(us)) == len(us)
