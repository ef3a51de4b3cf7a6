"""Fold definitions for the map-reduce oracle.

Oracle (test infrastructure).  The paper's reduction folds the map values
with a reduce expression of two formal arguments ``a`` and ``b`` and a
neutral element, an identity for that operation (section "Map-Reduce" and
its footnote).  The result is

    out = neutral (+) m(0) (+) m(1) (+) ... (+) m(n-1)

with (+) the reduce expression.  The paper does not fix the order of the
fold ("tree-based"), so the library assumes (+) associative and
commutative; the oracle computes the order-free value wherever one exists:

* integer sums: the exact sum (Python integers), then the result type's rule
  (int64/int32 must not overflow; unsigned wraps modulo 2**32);
* floating sums: the exact real sum of the map values, correctly rounded to
  float64 (``math.fsum``, Shewchuk's algorithm), together with sum |m_i| and
  the sum of the per-value error bounds, which the tolerance is built from;
  complex sums the same, for the real and imaginary parts separately;
* max / min of floating values: IEEE 754-2019 ``maximum`` / ``minimum``
  (a NaN anywhere gives NaN, -0 orders below +0); of integers: exact;
* any other reduce expression: a left-to-right fold evaluated with C
  semantics on the result type (pure Python; small n only).

Canonical reduce spellings (after removing blanks): ``a+b``, ``b+a`` and
``sum`` mean the sum; ``max(a,b)``, ``max(b,a)`` and ``max`` the maximum;
``min(a,b)``, ``min(b,a)`` and ``min`` the minimum.
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

from .api import map_chunks
from .ctype import CFLOAT, FLOAT_TYPES, INT, INT_RANGE, LONG, STORAGE_VT, UINT, parse_signature
from .interp import Interp, OracleError
from .parser import parse_expression

_CANON = {"a+b": "sum", "b+a": "sum", "sum": "sum",
          "max(a,b)": "max", "max(b,a)": "max", "max": "max",
          "min(a,b)": "min", "min(b,a)": "min", "min": "min"}

GENERIC_FOLD_LIMIT = 1 << 16


def canonical_op(combine: str) -> str:
    return _CANON.get("".join(combine.split()), "generic")


@dataclass
class ReduceResult:
    value: object        # int, or float
    op: str              # 'sum' | 'max' | 'min' | 'generic'
    t: str               # value type of the result
    n: int
    abs_sum: float       # sum |m_i|           (floating sums)
    err_sum: float       # sum of map-value error bounds (sums) / their max (max, min)
    unsure: int          # lanes whose map value may legitimately differ on the GPU
    exact: bool          # whether the GPU result must match bit for bit


def eval_neutral(result_storage: str, neutral: str):
    it = Interp({}, {}, np.zeros(1, np.int64), 1)
    one = np.ones(1, bool)
    val = it.to_storage(it.eval(parse_expression(neutral), one), result_storage, one)
    return val


def _ieee_extreme(values, op):
    if np.any(np.isnan(values)):
        return math.nan
    best = float(np.max(values) if op == "max" else np.min(values))
    if best == 0.0:
        zeros = values[values == 0]
        neg = np.signbit(zeros)
        if op == "max":
            best = 0.0 if np.any(~neg) else -0.0
        else:
            best = -0.0 if np.any(neg) else 0.0
    return best


def reduce(dtypes, map_expr, combine, neutral, n, args) -> ReduceResult:
    sig = parse_signature(dtypes)
    if sig.result is None:
        raise OracleError("a map-reduce signature starts with the result type")
    rt = STORAGE_VT[sig.result]
    op = canonical_op(combine)
    neutral_val = eval_neutral(sig.result, neutral)
    chunks = map_chunks(dtypes, map_expr, n, args)
    unsure = 0

    if rt == CFLOAT and op != "generic":
        if op != "sum":
            raise OracleError("complex values have no order: only sums reduce them")
        vals, abs_sum, err_sum = [], 0.0, 0.0
        for _, val in chunks:
            unsure += int(np.count_nonzero(val.u))
            vals.append(val.v)
            abs_sum += float(np.sum(np.abs(val.v)))
            err_sum += float(np.sum(val.e))
        allv = np.concatenate([np.asarray([complex(neutral_val.v[0])])] + vals)
        value = complex(math.fsum(allv.real.tolist()), math.fsum(allv.imag.tolist()))
        return ReduceResult(value, op, rt, n, abs_sum * (1 + 1e-12), err_sum * (1 + 1e-12),
                            unsure, False)

    if op == "sum" and rt not in FLOAT_TYPES:
        total = int(neutral_val.v[0])
        for _, val in chunks:
            unsure += int(np.count_nonzero(val.u))
            v = val.v
            if v.size and float(np.max(np.abs(v.astype(np.float64)))) * v.size < 2.0 ** 62:
                total += int(np.sum(v, dtype=np.int64))
            else:
                total += sum(int(x) for x in v.tolist())
        if rt == UINT:
            total %= 2 ** 32
        else:
            lo, hi = INT_RANGE[rt]
            if not lo <= total <= hi:
                raise OracleError(f"the sum {total} overflows the result type")
        return ReduceResult(total, op, rt, n, 0.0, 0.0, unsure, True)

    if op == "sum":
        vals = []
        abs_sum = err_sum = 0.0
        for _, val in chunks:
            unsure += int(np.count_nonzero(val.u))
            vals.append(val.v)
            abs_sum += float(np.sum(np.abs(val.v)))
            err_sum += float(np.sum(val.e))
        # the two auxiliary sums only size the tolerance: pad their rounding
        abs_sum *= 1 + 1e-12
        err_sum *= 1 + 1e-12
        value = math.fsum(itertools.chain(
            [float(neutral_val.v[0])], itertools.chain.from_iterable(a.tolist() for a in vals)))
        return ReduceResult(value, op, rt, n, abs_sum, err_sum, unsure, False)

    if op in ("max", "min"):
        best = neutral_val.v[:1].copy()
        emax = 0.0
        for _, val in chunks:
            unsure += int(np.count_nonzero(val.u))
            if val.v.size:
                if rt in FLOAT_TYPES:
                    best = np.array([_ieee_extreme(np.concatenate([best, val.v]), op)])
                    emax = max(emax, float(np.max(val.e)))
                else:
                    fn = np.max if op == "max" else np.min
                    best = np.array([fn(np.concatenate([best, val.v]))])
        value = float(best[0]) if rt in FLOAT_TYPES else int(best[0])
        return ReduceResult(value, op, rt, n, 0.0, emax, unsure, emax == 0.0)

    # generic reduce expression: left-to-right fold, C semantics
    if n > GENERIC_FOLD_LIMIT:
        raise OracleError("generic folds are evaluated for small n only")
    expr = parse_expression(combine)
    storage = sig.result
    acc = neutral_val.v[0]
    one = np.ones(1, bool)
    for _, val in chunks:
        unsure += int(np.count_nonzero(val.u))
        for x in val.v.tolist():
            it = Interp({}, {}, np.zeros(1, np.int64), 1)
            it.locals["a"] = (storage, it._mk(rt, acc))
            it.locals["b"] = (storage, it._mk(rt, x))
            res = it.to_storage(it.eval(expr, one), storage, one)
            acc = res.v[0]
    value = complex(acc) if rt == CFLOAT else float(acc) if rt in FLOAT_TYPES else int(acc)
    return ReduceResult(value, op, rt, n, 0.0, 0.0, unsure, rt not in FLOAT_TYPES and rt != CFLOAT)


def exact_sum(values) -> float:
    """Correctly rounded float64 value of the exact sum of float64 values."""
    return math.fsum(np.asarray(values, dtype=np.float64).tolist())


def norm2(values) -> float:
    """sqrt of the exact sum of squares.  Squares of values with at most 26
    significant bits (every float32, bfloat16, half and FP8 value) are exact in
    float64, the sum is correctly rounded, and the square root adds one
    rounding."""
    v = np.asarray(values, dtype=np.float64)
    return math.sqrt(math.fsum((v * v).tolist()))


__all__ = ["reduce", "canonical_op", "ReduceResult", "exact_sum", "norm2",
           "eval_neutral", "LONG", "INT"]
