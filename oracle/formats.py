"""Decoders for the stored number formats, written from the format definitions.

Oracle (test infrastructure).  Every decoder maps raw bit patterns to exact
float64 values (all three formats embed exactly in binary64):

* bfloat16: 1 sign, 8 exponent (bias 127), 7 fraction bits; IEEE-style
  subnormals, infinities and NaNs.
* binary16 ("half"): 1 sign, 5 exponent (bias 15), 10 fraction bits.
* OCP FP8 E4M3 ("fn" flavour): 1 sign, 4 exponent (bias 7), 3 fraction bits;
  no infinities, the single NaN pattern per sign is S.1111.111, the largest
  finite magnitude is 1.75 * 2**8 = 448, subnormals are m/8 * 2**-6.

The paper's kernels operate on float32 (section "Efficient Evaluation of
Element-wise Expressions"); these formats belong to the precision extension
of the map-reduce (low-precision loads with wider accumulation).
"""

from __future__ import annotations

import numpy as np


def _bits(bits):
    b = np.asarray(bits)
    if b.dtype.kind == "f":           # e.g. numpy float16: reinterpret its bytes
        b = b.view({1: np.uint8, 2: np.uint16}[b.dtype.itemsize])
    width = 8 * b.dtype.itemsize
    return b.astype(np.int64) & ((1 << width) - 1)


def _decode(bits, exp_bits, frac_bits, bias, ieee_specials, e4m3fn=False):
    b = _bits(bits)
    sign = np.where((b >> (exp_bits + frac_bits)) & 1, -1.0, 1.0)
    e = (b >> frac_bits) & ((1 << exp_bits) - 1)
    m = (b & ((1 << frac_bits) - 1)).astype(np.float64)
    emax_code = (1 << exp_bits) - 1
    normal = np.ldexp(1.0 + m / (1 << frac_bits), (e - bias).astype(np.int64))
    sub = np.ldexp(m / (1 << frac_bits), 1 - bias)
    val = np.where(e == 0, sub, normal)
    if ieee_specials:
        val = np.where(e == emax_code, np.where(m == 0, np.inf, np.nan), val)
    if e4m3fn:
        val = np.where((e == emax_code) & (m == (1 << frac_bits) - 1), np.nan, val)
    return sign * val


def decode_bf16(bits) -> np.ndarray:
    return _decode(bits, 8, 7, 127, True)


def decode_f16(bits) -> np.ndarray:
    return _decode(bits, 5, 10, 15, True)


def decode_e4m3fn(bits) -> np.ndarray:
    return _decode(bits, 4, 3, 7, False, e4m3fn=True)


# Unit roundoff (half an ulp at 1, relative) and the smallest positive
# (subnormal) magnitude of each storage format; used for error bounds on
# stores into these formats and for the low-precision error budget.
UNIT_ROUNDOFF = {"bfloat16": 2.0 ** -8, "float16": 2.0 ** -11, "fp8_e4m3": 2.0 ** -4,
                 "float32": 2.0 ** -24, "float64": 2.0 ** -53}
MIN_SUBNORMAL = {"bfloat16": 2.0 ** -133, "float16": 2.0 ** -24, "fp8_e4m3": 2.0 ** -9,
                 "float32": 2.0 ** -149, "float64": 2.0 ** -1074}
MAX_FINITE = {"bfloat16": (2 - 2.0 ** -7) * 2.0 ** 127, "float16": 65504.0,
              "fp8_e4m3": 448.0, "float32": float(np.finfo(np.float32).max),
              "float64": float(np.finfo(np.float64).max)}
