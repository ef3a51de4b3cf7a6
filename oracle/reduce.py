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
* any other reduce expression: a left-to-right fold with C semantics on
  the result type (pure Python; small n only).  Integer results are exact.
  For floating results the fold is evaluated in float64 (the ideal value;
  for an associative and commutative reduce expression the exact fold does
  not depend on the order) and comes with an order-free error model, below.

Error model of a floating fold under a generic reduce expression.  The
device folds in the result type along a tree whose shape the paper leaves
open.  At every step of the left-to-right fold the oracle evaluates the
reduce expression again, vectorised over all steps, with the interpreter's
running error bounds:

* r_k, the bound on one evaluation of the expression in the result type with
  exact operands a_k, b_k (one rounding per operation);
* the sensitivity to an error in either operand, which must not exceed 1
  (a non-expansive expression: sums, maxima, selections);
* |f(a, b)| <= |a| + |b| (magnitudes grow at most like a sum);
* f(neutral, b) = b (the neutral element is an identity, as the paper's
  footnote requires).

A step that violates one of them raises ``OracleError``: for such an
expression (a product, say) this model gives no order-free bound.  Under
them, in any fold tree, the error at the root is at most the sum of the
r's of its nodes plus the map values' own errors, and since every node's
operands are bounded by the sum of |m| over its leaves,

    |device - value| <= rounds * u * D * sum |m_i| + sum e_i + slack,

where u is the unit roundoff of the result type, D the depth of the tree
(the most combinations on any one map value's path), ``rounds`` the
largest r_k / (u (|a_k| + |b_k|)) over the steps (1 for ``(a)+(b)``, 2 for
``a+b+0.0f`` under the interpreter's one-rounding-per-operation rule, 0 for
a selection such as ``fmaxf(a,b)``) and ``slack`` an absolute allowance for
steps whose operands are below 2**-80, where r_k is dominated by the
absolute underflow term.  With rounds = 0 and exact map values the fold
selects one of its operands at every step, so every order gives the same
value: the result is then exact.

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
from .ctype import CFLOAT, FLOAT_TYPES, INT, INT_RANGE, LONG, STORAGE_VT, UINT, UNIT, parse_signature
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
    rounds: float = 1.0  # roundings of the result type per combination, per unit
                         # operand magnitude (floating folds; 1 for the canonical sum)
    abs_slack: float = 0.0   # absolute allowance for steps with operands below 2**-80


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
    vals, errs = [], []
    for _, val in chunks:
        unsure += int(np.count_nonzero(val.u))
        vals.append(val.v)
        errs.append(val.e)
    m = np.concatenate(vals) if vals else np.zeros(0, neutral_val.v.dtype)
    e = np.concatenate(errs) if errs else np.zeros(0)
    if rt not in FLOAT_TYPES and rt != CFLOAT:
        acc = generic_prefix(sig.result, rt, combine, neutral_val.v[0], m)[-1]
        return ReduceResult(int(acc), op, rt, n, 0.0, 0.0, unsure, True)
    prefix = generic_prefix(sig.result, rt, combine, neutral_val.v[0], m)
    rounds, slack = generic_float_model(sig.result, rt, combine, prefix, m)
    acc = prefix[-1]
    value = complex(acc) if rt == CFLOAT else float(acc)
    abs_sum = float(np.sum(np.abs(m))) * (1 + 1e-12)
    err_sum = float(np.sum(e)) * (1 + 1e-12)
    exact = rounds == 0.0 and err_sum == 0.0 and slack == 0.0
    return ReduceResult(value, op, rt, n, abs_sum, err_sum, unsure, exact, rounds, slack)


def _combine_eval(storage, rt, expr, a, b, ea=0.0, eb=0.0):
    """The reduce expression at every pair (a[k], b[k]) at once, the
    operands carrying error bounds ea, eb; returns the interpreter's value
    converted to the result type."""
    L = len(a)
    it = Interp({}, {}, np.zeros(L, np.int64), 1)
    one = np.ones(L, bool)
    it.locals["a"] = (storage, it._mk(rt, a, e=ea))
    it.locals["b"] = (storage, it._mk(rt, b, e=eb))
    return it.to_storage(it.eval(expr, one), storage, one)


def generic_prefix(storage, rt, combine, neutral, m):
    """Left-to-right fold neutral (+) m[0] (+) m[1] ...: every partial value
    (entry k holds k map terms), each step evaluated with C semantics on the
    result type (integers exact, floating values ideal in float64)."""
    expr = parse_expression(combine)
    acc = neutral
    pref = [acc]
    for x in m.tolist():
        acc = _combine_eval(storage, rt, expr, np.asarray([acc]), np.asarray([x])).v[0]
        pref.append(acc)
    dt = np.complex128 if rt == CFLOAT else np.float64 if rt in FLOAT_TYPES else object
    return np.array(pref, dtype=dt)


TINY_OPERANDS = 2.0 ** -80


def generic_float_model(storage, rt, combine, prefix, m):
    """(rounds, slack) of the error model above for the steps
    prefix[k] (+) m[k] of a floating fold; raises OracleError where a step
    leaves the model (expansive, growing faster than a sum, or a neutral
    element that is not an identity)."""
    if m.size == 0:
        return 0.0, 0.0
    expr = parse_expression(combine)
    # steps with an infinite or NaN operand (an infinite neutral element, say)
    # have no rounding to bound: they are left out
    fin = np.isfinite(prefix[:-1]) & np.isfinite(m)
    if not np.any(fin):
        return 0.0, 0.0
    a, b = prefix[:-1][fin], m[fin]
    u = UNIT[rt]
    exact = _combine_eval(storage, rt, expr, a, b)
    r = exact.e
    mag = np.abs(a) + np.abs(b)
    for which in ("a", "b"):
        delta = np.maximum(mag, 1.0) * 2.0 ** -30
        pert = _combine_eval(storage, rt, expr, a, b, *((delta, 0.0) if which == "a" else (0.0, delta)))
        with np.errstate(invalid="ignore"):
            sens = (pert.e - r) / delta
        if np.any(~(sens <= (1 + u) * (1 + 2.0 ** -20))):
            k = int(np.argmax(~(sens <= (1 + u) * (1 + 2.0 ** -20))))
            raise OracleError(f"the reduce expression amplifies an error in '{which}' at step {k} "
                              f"(sensitivity {sens[k]:.6g} > 1): no order-free bound")
    with np.errstate(invalid="ignore"):
        grows = ~(np.abs(exact.v) <= mag * (1 + 2.0 ** -40) + r)
    if np.any(grows):
        k = int(np.argmax(grows))
        raise OracleError(f"|f(a, b)| exceeds |a| + |b| at step {k}: no order-free bound")
    ident = _combine_eval(storage, rt, expr, np.full(b.size, prefix[0]), b)
    with np.errstate(invalid="ignore"):
        off = ~(np.abs(ident.v - b) <= ident.e)
    if np.any(off):
        k = int(np.argmax(off))
        raise OracleError(f"the neutral element is not an identity of the reduce expression "
                          f"(f(neutral, {b[k]!r}) = {ident.v[k]!r})")
    big = mag >= TINY_OPERANDS
    rounds = float(np.max(r[big] / (u * mag[big]))) if np.any(big) else 0.0
    slack = float(np.max(r[~big])) * (b.size + 2 ** 14) if np.any(~big) else 0.0
    return rounds, slack


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
           "eval_neutral", "generic_prefix", "generic_float_model", "LONG", "INT"]
