"""C value types, the usual arithmetic conversions and argument signatures.

Oracle (test infrastructure).  The paper's elementwise and reduction
facilities take "a C-style argument list" (section "Efficient Evaluation of
Element-wise Expressions"); a reduction's signature starts with the result
dtype (section "Map-Reduce").  This module parses that list on its own
(no code shared with the GPU library) and defines the value types in which
the interpreter evaluates.

Value types: ``int`` (32-bit signed), ``unsigned`` (32-bit), ``long``
(64-bit signed), ``float``, ``double`` and ``cfloat`` (complex with float
components, stored as ``complex64``; held as complex128 ideal values with a
bound on the magnitude of the error).  Integer values are held as
exact int64; floating values are held in float64 as the *ideal* value of
the expression, with a separate absolute error bound for what a float32
(or float64) evaluation may produce.
"""

from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from .lexer import CSyntaxError, tokenize
from .parser import TYPE_WORDS

INT, UINT, LONG, FLOAT, DOUBLE = "int", "unsigned", "long", "float", "double"
CFLOAT = "cfloat"            # complex with float components (section "Complex Numbers on the GPU")
INT_TYPES = (INT, UINT, LONG)
FLOAT_TYPES = (FLOAT, DOUBLE)

# storage type -> value type after an element is read (integer promotion;
# the 16- and 8-bit float formats read as their exact float value)
STORAGE_VT = {
    "float32": FLOAT, "float64": DOUBLE,
    "int8": INT, "uint8": INT, "int16": INT, "uint16": INT, "int32": INT,
    "uint32": UINT, "int64": LONG, "bool": INT,
    "bfloat16": FLOAT, "float16": FLOAT, "fp8_e4m3": FLOAT,
    "complex64": CFLOAT,
}
STORAGE_BYTES = {"float32": 4, "float64": 8, "int8": 1, "uint8": 1, "int16": 2,
                 "uint16": 2, "int32": 4, "uint32": 4, "int64": 8, "bool": 1,
                 "bfloat16": 2, "float16": 2, "fp8_e4m3": 1, "complex64": 8}
NUMPY_STORAGE = {"float32": np.float32, "float64": np.float64, "int8": np.int8,
                 "uint8": np.uint8, "int16": np.int16, "uint16": np.uint16,
                 "int32": np.int32, "uint32": np.uint32, "int64": np.int64,
                 "bfloat16": np.uint16, "float16": np.uint16, "fp8_e4m3": np.uint8,
                 "complex64": np.complex64}

UNIT = {FLOAT: 2.0 ** -24, DOUBLE: 2.0 ** -53, CFLOAT: 2.0 ** -24}
# absolute slack per rounding: covers gradual underflow and flush-to-zero
TINY = {FLOAT: 2.0 ** -126, DOUBLE: 2.0 ** -1022, CFLOAT: 2.0 ** -126}
INT_RANGE = {INT: (-2 ** 31, 2 ** 31 - 1), UINT: (0, 2 ** 32 - 1),
             LONG: (-2 ** 63, 2 ** 63 - 1)}


def common_type(a: str, b: str) -> str:
    """C usual arithmetic conversions over the value types (LP64); a complex
    operand makes the operation complex with float components."""
    if CFLOAT in (a, b):
        return CFLOAT
    if DOUBLE in (a, b):
        return DOUBLE
    if FLOAT in (a, b):
        return FLOAT
    if LONG in (a, b):
        return LONG          # 64-bit long represents every unsigned int
    if UINT in (a, b):
        return UINT
    return INT


@dataclass
class Arg:
    name: str
    storage: str
    pointer: bool
    const: bool


@dataclass
class Signature:
    result: str | None     # storage type of a reduction result, None for elementwise
    args: list

    def arg(self, name):
        for a in self.args:
            if a.name == name:
                return a
        return None


def parse_signature(dtypes: str) -> Signature:
    """``[result_type ':'] decl (',' decl)*`` with ``decl := [const] type [*] name``."""
    result = None
    text = dtypes
    if ":" in text:
        head, text = text.split(":", 1)
        words = tuple(t.text for t in tokenize(head) if t.kind != "end")
        if words not in TYPE_WORDS:
            raise CSyntaxError(f"unknown result type {head.strip()!r}")
        result = TYPE_WORDS[words]
    args = []
    if text.strip():
        for decl in text.split(","):
            toks = [t for t in tokenize(decl) if t.kind != "end"]
            const = False
            if toks and toks[0].text == "const":
                const, toks = True, toks[1:]
            pointer = False
            if len(toks) >= 2 and toks[-2].text == "*":
                pointer = True
                toks = toks[:-2] + toks[-1:]
            toks = [t for t in toks if t.text not in ("__restrict__", "restrict")]
            if not toks or toks[-1].kind != "id":
                raise CSyntaxError(f"bad declaration {decl.strip()!r}")
            words = tuple(t.text for t in toks[:-1])
            if words and words[-1] == "const":
                const, words = True, words[:-1]
            if words not in TYPE_WORDS or TYPE_WORDS[words] == "bool":
                raise CSyntaxError(f"unknown type in {decl.strip()!r}")
            args.append(Arg(toks[-1].text, TYPE_WORDS[words], pointer, const))
    names = [a.name for a in args]
    if len(set(names)) != len(names):
        raise CSyntaxError("duplicate argument name")
    return Signature(result, args)


def round_fraction(q: Fraction, p: int, emin: int, emax: int) -> float:
    """Correctly rounded (ties to even) conversion of an exact rational to a
    binary format with ``p`` significand bits and normal exponent range
    [emin, emax]; used for C float literals such as ``0.1f``."""
    if q == 0:
        return 0.0
    sign = -1.0 if q < 0 else 1.0
    q = abs(q)
    num, den = q.numerator, q.denominator
    e = num.bit_length() - den.bit_length()
    if (num << max(0, -e)) < (den << max(0, e)):
        e -= 1                                   # now 2**e <= q < 2**(e+1)
    e = max(e, emin)
    shift = e - p + 1                            # value of the last kept bit
    if shift >= 0:
        m, rem_num, rem_den = divmod(num, den << shift) + (den << shift,)
    else:
        m, rem_num, rem_den = divmod(num << -shift, den) + (den,)
    twice = 2 * rem_num
    if twice > rem_den or (twice == rem_den and m & 1):
        m += 1
    val = Fraction(m) * Fraction(2) ** shift
    if val >= Fraction(2) ** (emax + 1):
        return sign * float("inf")
    return sign * float(val)


def f32_literal(q: Fraction) -> float:
    return round_fraction(q, 24, -126, 127)
