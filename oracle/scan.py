"""Prefix-scan definitions for the map-scan oracle.

Oracle (test infrastructure).  Besides elementwise operations and
reductions, the paper names parallel prefix sums ("parallel scan") among
the facilities generated from the same ingredients (section "Further
Facilities"): a map expression over the formal index ``i``, a combine
expression in ``a`` and ``b`` and its neutral element (section
"Map-Reduce").  For the map values m(0), ..., m(n-1), converted to the
result type, and the combine (+):

    inclusive:  y[i] = neutral (+) m(0) (+) ... (+) m(i)
    exclusive:  y[i] = neutral (+) m(0) (+) ... (+) m(i-1)    (y[0] = neutral)

As for reductions, (+) is taken associative and commutative, and the oracle
computes the order-free value of every prefix:

* integer sums: exact prefix sums (Python integers), then the result type's
  rule (int64 / int32 must not overflow; unsigned wraps modulo 2**32);
* floating sums: every prefix's exact real sum, correctly rounded to
  float64 (for complex values, the real and imaginary parts separately).
  The map values are moved to a common binary fixed point (a Python integer
  times 2**-S, exact for every float64), summed there exactly, and each
  prefix is rounded once by Python's correctly rounded integer division.  The prefix sums of |m| and of the map values' error
  bounds are returned for the tolerance;
* max / min of floating values: IEEE 754-2019 ``maximum`` / ``minimum`` of
  every prefix (a NaN propagates to every later prefix; -0 orders below
  +0); of integers: exact;
* any other combine: a left-to-right fold with C semantics on the result
  type (pure Python; small n only); for floating results every prefix
  carries the reductions' order-free error model (``reduce``): the device's
  prefix i is within rounds * u * D * sum_{j<=i} |m_j| + sum_{j<=i} e_j +
  slack of the oracle's, D being the depth of its combination tree.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .api import map_chunks
from .ctype import CFLOAT, FLOAT_TYPES, INT_RANGE, STORAGE_VT, UINT, parse_signature
from .interp import Interp, OracleError
from .parser import parse_expression
from .reduce import (GENERIC_FOLD_LIMIT, canonical_op, eval_neutral, generic_float_model,
                     generic_prefix)


@dataclass
class ScanResult:
    values: np.ndarray       # y[i]: int64 (or object for wide integers) / float64
    op: str                  # 'sum' | 'max' | 'min' | 'generic'
    t: str                   # value type of the result
    n: int
    abs_prefix: np.ndarray   # sum over the prefix of |m_j| (floating sums), else zeros
    err_prefix: np.ndarray   # sum over the prefix of the map values' error bounds
    unsure: int              # lanes whose map value may legitimately differ on the GPU
    exact: bool              # whether the GPU result must match bit for bit
    rounds: float = 1.0      # roundings per combination and unit operand magnitude
    abs_slack: float = 0.0   # absolute allowance for steps with operands below 2**-80


def _exact_float_prefix(neutral: float, values: np.ndarray) -> np.ndarray:
    """Correctly rounded float64 value of neutral + v[0] + ... + v[k] for
    every k: exact sums in binary fixed point, one rounding per prefix."""
    vals = [float(neutral)] + [float(x) for x in values.tolist()]
    ratios = [v.as_integer_ratio() for v in vals]          # (num, 2**e)
    shift = max(d.bit_length() - 1 for _, d in ratios)     # common scale 2**-shift
    acc = 0
    out = np.empty(len(vals), dtype=np.float64)
    one = 1 << shift
    for k, (num, den) in enumerate(ratios):
        acc += num << (shift - (den.bit_length() - 1))
        out[k] = acc / one                                  # correctly rounded
    return out


def _ieee_prefix_extreme(neutral: float, values: np.ndarray, op: str) -> np.ndarray:
    v = np.concatenate([[neutral], values.astype(np.float64)])
    fn = np.maximum if op == "max" else np.minimum
    best = fn.accumulate(v)                                 # NaN propagates forward
    zero = v == 0
    if op == "max":                                         # +0 once any +0 is seen
        seen = np.logical_or.accumulate(zero & ~np.signbit(v))
        best = np.where(best == 0, np.where(seen, 0.0, -0.0), best)
    else:                                                   # -0 once any -0 is seen
        seen = np.logical_or.accumulate(zero & np.signbit(v))
        best = np.where(best == 0, np.where(seen, -0.0, 0.0), best)
    return best


def scan(dtypes, map_expr, combine, neutral, n, args, exclusive=False) -> ScanResult:
    sig = parse_signature(dtypes)
    if sig.result is None:
        raise OracleError("a map-scan signature starts with the result type")
    rt = STORAGE_VT[sig.result]
    op = canonical_op(combine)
    neutral_val = eval_neutral(sig.result, neutral)
    m_vals, m_err, unsure = [], [], 0
    for _, val in map_chunks(dtypes, map_expr, n, args):
        unsure += int(np.count_nonzero(val.u))
        m_vals.append(val.v)
        m_err.append(val.e)
    m = np.concatenate(m_vals) if m_vals else np.zeros(0, neutral_val.v.dtype)
    e = np.concatenate(m_err) if m_err else np.zeros(0)

    # prefix values over [neutral, m0, ..., m(n-1)]: entry k holds k map terms
    abs_p = np.zeros(n + 1)
    err_p = np.zeros(n + 1)
    if rt == CFLOAT and op != "generic":
        if op != "sum":
            raise OracleError("complex values have no order: only sums scan them")
        neu = complex(neutral_val.v[0])
        prefix = (_exact_float_prefix(neu.real, m.real) + 1j * _exact_float_prefix(neu.imag, m.imag))
        pad = 1.0 + (n + 1) * 2.0 ** -52
        abs_p[1:] = np.cumsum(np.abs(m)) * pad
        err_p[1:] = np.cumsum(e) * pad
        exact = False
    elif op == "sum" and rt not in FLOAT_TYPES:
        acc = int(neutral_val.v[0])
        pref = [acc]
        for x in m.tolist():
            acc += int(x)
            pref.append(acc)
        if rt == UINT:
            pref = [p % 2 ** 32 for p in pref]
        else:
            lo, hi = INT_RANGE[rt]
            if pref and not (lo <= min(pref) and max(pref) <= hi):
                raise OracleError("a prefix sum overflows the result type")
        prefix = np.array(pref, dtype=np.int64)
        exact = True
    elif op == "sum":
        prefix = _exact_float_prefix(float(neutral_val.v[0]), m)
        # the auxiliary sums only size the tolerance: pad their rounding
        pad = 1.0 + (n + 1) * 2.0 ** -52
        abs_p[1:] = np.cumsum(np.abs(m.astype(np.float64))) * pad
        err_p[1:] = np.cumsum(e) * pad
        exact = False
    elif op in ("max", "min"):
        if rt in FLOAT_TYPES:
            prefix = _ieee_prefix_extreme(float(neutral_val.v[0]), m, op)
            err_p[1:] = np.maximum.accumulate(e) if e.size else e
            exact = not np.any(e > 0)
        else:
            fn = np.maximum if op == "max" else np.minimum
            prefix = fn.accumulate(np.concatenate([neutral_val.v[:1], m]).astype(np.int64))
            exact = True
    else:
        if n > GENERIC_FOLD_LIMIT:
            raise OracleError("generic scans are evaluated for small n only")
        prefix = generic_prefix(sig.result, rt, combine, neutral_val.v[0], m)
        exact = rt not in FLOAT_TYPES and rt != CFLOAT
        if exact:
            prefix = prefix.astype(np.int64)
        else:
            rounds, slack = generic_float_model(sig.result, rt, combine, prefix, m)
            pad = 1.0 + (n + 1) * 2.0 ** -52
            abs_p[1:] = np.cumsum(np.abs(m)) * pad
            err_p[1:] = np.cumsum(e) * pad
            exact = rounds == 0.0 and not np.any(e > 0) and slack == 0.0
            sl = slice(0, n) if exclusive else slice(1, n + 1)
            return ScanResult(prefix[sl], op, rt, n, abs_p[sl], err_p[sl], unsure, exact,
                              rounds, slack)

    sl = slice(0, n) if exclusive else slice(1, n + 1)
    return ScanResult(prefix[sl], op, rt, n, abs_p[sl], err_p[sl], unsure, exact)


__all__ = ["scan", "ScanResult"]
