"""Floating-point storage formats and simulated rounding (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The paper lists its formats with unit roundoff u = 2^-t, where t counts the
significand bits including the implicit one (Table 1.1: q52, bf16, fp16,
fp32, fp64), and simulates storage in a lower precision by rounding fp64
values (Sect. 4, experimental setup).  Readings taken here:

* The q52 row of Table 1.1 prints t as -16; its u = 1.25e-1 = 2^-3, x_min =
  2^-14 and x_max = 57344 identify the 8-bit E5M2 format, so t = 3.
* fp8 E4M3 (OCP "E4M3FN": max 448, no infinities) is not in the paper; it is
  added as one more member of the candidate set of the adaptive rule.
* Rounding is round-to-nearest, ties-to-even, applied once to the fp64 value,
  with gradual underflow.  A value whose rounding exceeds the largest finite
  number of the format is an overflow (``OverflowInFormat``).

Everything here works on numpy float64 arrays; codes are unsigned integers
holding the format's bit pattern.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Fmt:
    name: str
    t: int            # significand bits incl. the implicit leading bit
    emin: int         # exponent of the smallest positive normal number
    emax: int         # exponent of the largest finite number
    ebits: int        # width of the exponent field
    bias: int
    max_finite: float
    has_inf: bool     # IEEE-style infinities (all formats but E4M3FN)
    nbytes: int

    @property
    def u(self) -> float:
        """Unit roundoff 2^-t (Table 1.1)."""
        return 2.0 ** (-self.t)

    @property
    def mbits(self) -> int:
        return self.t - 1

    @property
    def x_min(self) -> float:
        return 2.0 ** self.emin


def _ieee_max(t: int, emax: int) -> float:
    return (2.0 - 2.0 ** (1 - t)) * 2.0 ** emax


FP64 = Fmt("fp64", 53, -1022, 1023, 11, 1023, _ieee_max(53, 1023), True, 8)
FP32 = Fmt("fp32", 24, -126, 127, 8, 127, _ieee_max(24, 127), True, 4)
BF16 = Fmt("bf16", 8, -126, 127, 8, 127, _ieee_max(8, 127), True, 2)
FP16 = Fmt("fp16", 11, -14, 15, 5, 15, _ieee_max(11, 15), True, 2)
# E4M3FN: exponent field 1111 is an ordinary binade except mantissa 111 (NaN),
# so emax = 8 and the largest finite value is 1.75 * 2^8 = 448.
E4M3 = Fmt("e4m3", 4, -6, 8, 4, 7, 448.0, False, 1)
E5M2 = Fmt("e5m2", 3, -14, 15, 5, 15, _ieee_max(3, 15), True, 1)

FORMATS = {f.name: f for f in (FP64, FP32, BF16, FP16, E4M3, E5M2)}

# Formats that receive a per-column power-of-2 scale before rounding (their
# exponent range is narrow; bf16 and fp32 share fp32's range and need none).
SCALED = ("fp16", "e4m3", "e5m2")


class OverflowInFormat(ArithmeticError):
    """A value rounds to something larger than the format's largest number."""


def fmt(name_or_fmt) -> Fmt:
    return name_or_fmt if isinstance(name_or_fmt, Fmt) else FORMATS[name_or_fmt]


def round_rne(f, x, *, check_overflow: bool = True) -> np.ndarray:
    """Round fp64 values to format ``f`` (nearest, ties to even), once.

    The quantum of a value with leading bit 2^E is 2^(max(E, emin) - t + 1):
    below 2^emin it stays at the subnormal quantum (gradual underflow).
    Scaling by that power of two is exact, ``np.rint`` rounds the scaled
    value to an integer with ties to even, and scaling back is exact.
    """
    f = fmt(f)
    x = np.asarray(x, dtype=np.float64)
    if f is FP64:
        return x.copy()
    out = x.copy()
    fin = np.isfinite(x) & (x != 0)
    xv = x[fin]
    _, e = np.frexp(xv)                       # xv = m * 2^e, 0.5 <= |m| < 1
    lead = e.astype(np.int64) - 1             # exponent of the leading bit
    qexp = np.maximum(lead, f.emin) - (f.t - 1)
    r = np.rint(np.ldexp(xv, -qexp))
    yv = np.ldexp(r, qexp)
    big = np.abs(yv) > f.max_finite
    if big.any():
        if check_overflow:
            raise OverflowInFormat(f"{f.name}: |value| up to {np.abs(xv[big]).max():.6g}"
                                   f" exceeds {f.max_finite:.6g}")
        yv = np.where(big, np.copysign(np.inf if f.has_inf else np.nan, yv), yv)
    out[fin] = yv
    return out


def encode(f, y) -> np.ndarray:
    """Bit patterns of values already representable in ``f``.

    sign | exponent field | fraction field, with the usual biased exponent;
    exponent field 0 holds zero and the subnormals.  Infinities use the
    all-ones exponent (E4M3FN has none); NaN is the all-ones pattern.
    """
    f = fmt(f)
    y = np.asarray(y, dtype=np.float64)
    nbits = 8 * f.nbytes
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[f.nbytes]
    if f is FP64:
        return y.view(np.uint64).copy()
    sign = np.signbit(y).astype(np.uint64)
    a = np.abs(y)
    expf = np.zeros(a.shape, dtype=np.int64)
    frac = np.zeros(a.shape, dtype=np.int64)
    fin = np.isfinite(a) & (a != 0)
    av = a[fin]
    _, e = np.frexp(av)
    lead = e.astype(np.int64) - 1
    sub = lead < f.emin
    ev = np.where(sub, 0, lead + f.bias)
    quantum = np.where(sub, f.emin, lead) - (f.t - 1)
    sig = np.ldexp(av, -quantum)             # integer-valued significand
    if not np.all(sig == np.floor(sig)):
        raise ValueError(f"value not representable in {f.name}")
    sig = sig.astype(np.int64)
    fv = np.where(sub, sig, sig - (1 << f.mbits))
    expf[fin] = ev
    frac[fin] = fv
    ones = (1 << f.ebits) - 1
    inf = np.isinf(a)
    if inf.any():
        if not f.has_inf:
            raise OverflowInFormat(f"{f.name} has no infinity")
        expf[inf] = ones
        frac[inf] = 0
    nan = np.isnan(a)
    if nan.any():
        expf[nan] = ones
        frac[nan] = (1 << f.mbits) - 1
    code = (sign << np.uint64(nbits - 1)) | (expf.astype(np.uint64) << np.uint64(f.mbits)) \
        | frac.astype(np.uint64)
    return code.astype(dt)


def decode(f, code) -> np.ndarray:
    """fp64 values of bit patterns of format ``f`` (exact)."""
    f = fmt(f)
    c = np.asarray(code).astype(np.uint64)
    if f is FP64:
        return c.view(np.float64).copy()
    nbits = 8 * f.nbytes
    sign = ((c >> np.uint64(nbits - 1)) & np.uint64(1)).astype(np.int64)
    expf = ((c >> np.uint64(f.mbits)) & np.uint64((1 << f.ebits) - 1)).astype(np.int64)
    frac = (c & np.uint64((1 << f.mbits) - 1)).astype(np.int64)
    sub = expf == 0
    sig = np.where(sub, frac, frac + (1 << f.mbits)).astype(np.float64)
    ex = np.where(sub, f.emin, expf - f.bias) - f.mbits
    val = np.ldexp(sig, ex)
    ones = (1 << f.ebits) - 1
    if f.has_inf:
        special = expf == ones
        val = np.where(special & (frac == 0), np.inf, val)
        val = np.where(special & (frac != 0), np.nan, val)
    else:
        val = np.where((expf == ones) & (frac == (1 << f.mbits) - 1), np.nan, val)
    return np.where(sign == 1, -val, val)


def column_scale_exponent(f, amax) -> np.ndarray:
    """Per-column power-of-2 scale for the narrow formats.

    The exponent e_j is the largest integer with amax_j * 2^e_j <= max_finite
    (0 for an all-zero column), so the scaled column cannot overflow and
    scaling back by 2^-e_j after decoding is exact.  Computed with integer
    logic on the binary exponents (no logarithms): with amax = m_a 2^E_a and
    max_finite = m_f 2^E_f (0.5 <= m < 1), e = E_f - E_a, minus one when
    m_a > m_f.
    """
    f = fmt(f)
    amax = np.asarray(amax, dtype=np.float64)
    ma, ea = np.frexp(amax)
    mf, ef = np.frexp(f.max_finite)
    e = ef - ea.astype(np.int64) - (ma > mf).astype(np.int64)
    return np.where(amax == 0, 0, e).astype(np.int64)
