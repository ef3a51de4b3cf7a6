"""Public oracle entry points: elementwise, map, and map-reduce.

Oracle (test infrastructure).  Definitions, from the paper:

* elementwise (section "Efficient Evaluation of Element-wise Expressions"):
  run the statement list for every i in [0, n) over same-length arrays;
* map-reduce (section "Map-Reduce"): the reduce expression in ``a``, ``b``
  folds the map values m(0) ... m(n-1), starting from the neutral element,
  into one value of the result dtype named first in the signature; for n = 0
  the result is the neutral element (the footnote defines it as the identity
  of the reduce operation).

Arrays are numpy arrays of their storage type (the 16- and 8-bit float
formats as raw ``uint16`` / ``uint8`` bit patterns); scalars are Python
numbers (raw bit patterns for those formats).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ctype import NUMPY_STORAGE, parse_signature
from .interp import Interp, OracleError
from .lexer import CSyntaxError
from .parser import parse_statements, parse_expression

CHUNK = 1 << 20


def _bind(sig, args):
    if len(args) != len(sig.args):
        raise CSyntaxError(f"expected {len(sig.args)} arguments, got {len(args)}")
    arrays, scalars = {}, {}
    for a, val in zip(sig.args, args):
        if a.pointer:
            arr = np.asarray(val)
            want = NUMPY_STORAGE[a.storage]
            if arr.dtype != want:
                raise TypeError(f"argument {a.name}: expected numpy {np.dtype(want)}, "
                                f"got {arr.dtype}")
            arrays[a.name] = (a.storage, arr.reshape(-1))
        else:
            scalars[a.name] = (a.storage, val)
    return arrays, scalars


def _lane_chunks(n, lanes):
    if lanes is not None:
        lanes = np.asarray(lanes, dtype=np.int64)
        for s in range(0, len(lanes), CHUNK):
            yield lanes[s:s + CHUNK]
        return
    for s in range(0, n, CHUNK):
        yield np.arange(s, min(n, s + CHUNK), dtype=np.int64)


@dataclass
class Lanes:
    """Per-lane oracle values of one written array (or of the map)."""
    lanes: np.ndarray
    v: np.ndarray        # ideal values (float64) or exact integers (int64)
    e: np.ndarray        # absolute error bound of a GPU evaluation
    u: np.ndarray        # unsure lanes (skip when comparing)
    t: str               # value type
    written: np.ndarray  # lanes on which the array was assigned


def elementwise(dtypes, stmt, n, args, lanes=None) -> dict:
    """Oracle for the elementwise facility.  Returns, for every array the
    statement assigns, its values over ``lanes`` (default: all of [0, n))."""
    sig = parse_signature(dtypes)
    if sig.result is not None:
        raise CSyntaxError("an elementwise signature has no result type")
    stmts = parse_statements(stmt)
    arrays, scalars = _bind(sig, args)
    parts: dict[str, list] = {}
    for chunk in _lane_chunks(n, lanes):
        it = Interp(arrays, scalars, chunk, n)
        it.run(stmts)
        for name, ov in it.overlay.items():
            parts.setdefault(name, []).append((chunk, ov))
    out = {}
    for name, items in parts.items():
        out[name] = Lanes(np.concatenate([c for c, _ in items]),
                          np.concatenate([o["val"].v for _, o in items]),
                          np.concatenate([o["val"].e for _, o in items]),
                          np.concatenate([o["val"].u for _, o in items]),
                          items[0][1]["val"].t,
                          np.concatenate([o["w"] for _, o in items]))
    return out


def map_chunks(dtypes, map_expr, n, args, lanes=None):
    """Yields (lanes, Val) of the map expression converted to the result
    type, chunk by chunk, in index order."""
    sig = parse_signature(dtypes)
    if sig.result is None:
        raise CSyntaxError("a map-reduce signature starts with the result type")
    expr = parse_expression(map_expr)
    arrays, scalars = _bind(sig, args)
    for chunk in _lane_chunks(n, lanes):
        it = Interp(arrays, scalars, chunk, n)
        val = it.eval(expr, np.ones(len(chunk), dtype=bool))
        if it.overlay:
            raise CSyntaxError("a map expression may not assign to arrays")
        val = it.to_storage(val, sig.result, np.ones(len(chunk), dtype=bool))
        yield chunk, val


def map_values(dtypes, map_expr, n, args, lanes=None) -> Lanes:
    parts = list(map_chunks(dtypes, map_expr, n, args, lanes))
    if not parts:
        e = np.zeros(0)
        return Lanes(np.zeros(0, np.int64), e, e, np.zeros(0, bool), "", np.zeros(0, bool))
    return Lanes(np.concatenate([c for c, _ in parts]),
                 np.concatenate([v.v for _, v in parts]),
                 np.concatenate([v.e for _, v in parts]),
                 np.concatenate([v.u for _, v in parts]),
                 parts[0][1].t, np.ones(sum(len(c) for c, _ in parts), bool))


__all__ = ["elementwise", "map_chunks", "map_values", "Lanes", "OracleError",
           "CSyntaxError"]
