"""Vectorised reference interpreter for elementwise statements and map
expressions, with C semantics, exact integers and float64 floating point.

Oracle (test infrastructure).  What is computed follows the paper's
elementwise facility: the user's statement list runs once for every value of
the formal index ``i`` over arrays that all have the same length (section
"Efficient Evaluation of Element-wise Expressions"); and the map part of the
map-reduce facility, an arbitrary C expression evaluated at every ``i``
(section "Map-Reduce").

Evaluation is over a vector of lanes (a set of values of ``i``) at once;
statements run one after another, each over all lanes, which equals running
the statement list per index because writes are restricted to ``name[i]``.
Control flow (``if``, ``?:``, ``&&``, ``||``) is evaluated under lane masks.

Each floating value carries

* ``v`` -- its ideal value, computed in float64 (exactly, for the inputs in
  this project, up to one float64 rounding per operation),
* ``e`` -- an absolute bound on |(value a float32/float64 GPU evaluation of
  the same C expression may produce) - v|: a running error bound in the
  manner of Wilkinson, one rounding of the operation's type per operation
  plus the propagated input bounds, with documented ulp allowances for the
  device math functions, plus the float64 rounding of ``v`` itself,
* ``u`` -- an "unsure" lane mask: lanes where a comparison, conversion to
  integer or rounding to an integer falls inside the error interval, so that
  the GPU may legitimately take the other branch.  Tests skip those lanes.

Integer values are exact; signed overflow, division by zero, out-of-range
shifts and out-of-bounds reads on active lanes raise ``OracleError``
(undefined behaviour in C, so no expected value exists).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import formats
from .ctype import (CFLOAT, DOUBLE, FLOAT, FLOAT_TYPES, INT, INT_RANGE, INT_TYPES, LONG,
                    STORAGE_VT, TINY, UINT, UNIT, common_type, f32_literal)
from .lexer import CSyntaxError
from .parser import (Assign, Binary, Block, Call, Cast, Comma, Cond, Decl, ExprStmt,
                     If, IncDec, Index, Logical, Name, Num, Unary)

EPS64 = 2.0 ** -53           # the oracle's own float64 rounding, per operation


class OracleError(ArithmeticError):
    """The C expression has no defined value on some active lane."""


@dataclass
class Val:
    t: str
    v: np.ndarray
    e: np.ndarray
    u: np.ndarray


def _bcast(x, L):
    x = np.asarray(x)
    return np.broadcast_to(x, (L,)) if x.shape != (L,) else x


# ------------------------------------------------------------ conversions
def _wrap(v, bits, signed):
    v = np.asarray(v, dtype=np.int64)
    if bits == 64:
        return v
    m = (1 << bits) - 1
    w = v & m
    if signed:
        w = np.where(w >= (1 << (bits - 1)), w - (1 << bits), w)
    return w


_NARROW = {"int8": (8, True), "uint8": (8, False), "int16": (16, True),
           "uint16": (16, False), "int32": (32, True), "uint32": (32, False),
           "int64": (64, True)}


class Interp:
    """One evaluation over a lane vector.

    ``arrays``: name -> (storage type, numpy array of raw storage) ;
    ``scalars``: name -> (storage type, python value) ;
    ``lanes``: int64 array of the index values ``i`` ; ``n``: the length.
    """

    def __init__(self, arrays, scalars, lanes, n):
        self.arrays = arrays
        self.lanes = np.asarray(lanes, dtype=np.int64)
        self.L = len(self.lanes)
        self.n = int(n)
        self.idx_t = INT if self.n < 2 ** 31 else LONG
        self.locals: dict[str, tuple[str, Val]] = {}
        for name, (storage, value) in scalars.items():
            self.locals[name] = (storage, self._scalar_val(storage, value))
        self.overlay: dict[str, dict] = {}
        self.taint = np.zeros(self.L, dtype=bool)
        self.scopes: list[set] = [set()]

    # -- construction helpers
    def _zeros_e(self):
        return np.zeros(self.L)

    def _mk(self, t, v, e=None, u=None):
        L = self.L
        if t in INT_TYPES:
            v = _bcast(np.asarray(v, dtype=np.int64), L)
            e = np.zeros(L)
        else:
            v = _bcast(np.asarray(v, dtype=np.complex128 if t == CFLOAT else np.float64), L)
            e = self._zeros_e() if e is None else _bcast(np.asarray(e, dtype=np.float64), L)
        u = np.zeros(L, dtype=bool) if u is None else _bcast(np.asarray(u, dtype=bool), L)
        return Val(t, v, e, u)

    def _scalar_val(self, storage, value):
        """Scalar kernel argument: integers and float/double by value; the
        16- and 8-bit formats are given as their raw bit pattern."""
        vt = STORAGE_VT[storage]
        if vt in INT_TYPES:
            return self._mk(vt, self.decode(storage, np.asarray([value]))[0])
        if storage in ("bfloat16", "float16", "fp8_e4m3"):
            return self._mk(vt, self.decode(storage, np.asarray([int(value)]))[0])
        if storage == "float32":
            value = float(np.float32(value))
        if storage == "complex64":
            return self._mk(vt, complex(np.complex64(value)))
        return self._mk(vt, float(value))

    def decode(self, storage, raw):
        if storage == "bfloat16":
            return formats.decode_bf16(raw)
        if storage == "float16":
            return formats.decode_f16(raw)
        if storage == "fp8_e4m3":
            return formats.decode_e4m3fn(raw)
        if STORAGE_VT[storage] in INT_TYPES:
            return np.asarray(raw).astype(np.int64)
        if storage == "complex64":
            return np.asarray(raw).astype(np.complex128)
        return np.asarray(raw).astype(np.float64)

    # -- type conversion (C rules)
    def convert(self, x: Val, t: str, active) -> Val:
        if x.t == t:
            return x
        if x.t == CFLOAT:
            raise CSyntaxError("a complex value becomes real only through real(), imag() or abs()")
        if t == CFLOAT:            # real -> complex: the float conversion, imaginary part 0
            y = self.convert(x, FLOAT, active)
            return Val(CFLOAT, y.v.astype(np.complex128), y.e, y.u)
        if t in INT_TYPES:
            if x.t in INT_TYPES:
                if t == LONG:
                    return Val(t, x.v, x.e, x.u)
                return Val(t, _wrap(x.v, 32, t == INT), x.e, x.u)
            return self._float_to_int(x, t, active)
        # to floating
        if x.t in INT_TYPES:
            v = x.v.astype(np.float64)
            limit = 2.0 ** 24 if t == FLOAT else 2.0 ** 53
            e = np.where(np.abs(v) > limit, UNIT[t] * np.abs(v), 0.0)
            if x.t == LONG:        # int64 -> float64 conversion by numpy rounds
                e = e + np.where(np.abs(v) > 2.0 ** 53, EPS64 * np.abs(v), 0.0)
            return Val(t, v, e, x.u.copy())
        if t == DOUBLE:            # float -> double: exact
            return Val(t, x.v, x.e, x.u)
        # double -> float: one rounding
        with np.errstate(invalid="ignore", over="ignore"):
            e = x.e + UNIT[FLOAT] * (np.abs(x.v) + x.e) + TINY[FLOAT]
            u = x.u | (np.abs(x.v) > formats.MAX_FINITE["float32"])
        return Val(t, x.v, e, u)

    def _float_to_int(self, x, t, active):
        lo, hi = INT_RANGE[t]
        with np.errstate(invalid="ignore"):
            bad = active & ~((x.v > lo - 1) & (x.v < hi + 1))
        if np.any(bad):
            raise OracleError("float to integer conversion out of range")
        v = np.trunc(np.where(active, x.v, 0.0))
        with np.errstate(invalid="ignore"):
            u = x.u | (np.trunc(x.v - x.e) != np.trunc(x.v + x.e))
        return Val(t, v.astype(np.int64), np.zeros(self.L), u)

    def to_storage(self, x: Val, storage: str, active) -> Val:
        """Conversion on assignment to an array element / local of a storage type."""
        if storage in _NARROW:
            bits, signed = _NARROW[storage]
            y = self.convert(x, LONG if bits == 64 else (INT if signed else UINT), active) \
                if x.t in FLOAT_TYPES else x
            if x.t in FLOAT_TYPES and bits < 32:
                lo, hi = (-(1 << (bits - 1)), (1 << (bits - 1)) - 1) if signed \
                    else (0, (1 << bits) - 1)
                if np.any(active & ((y.v < lo) | (y.v > hi))):
                    raise OracleError("float to narrow integer out of range")
            v = _wrap(y.v, bits, signed)
            return self._mk(STORAGE_VT[storage], v, u=y.u)
        if storage == "bool":
            truth = self.truth(x)
            return self._mk(INT, truth.astype(np.int64), u=self.truth_unsure(x))
        vt = STORAGE_VT[storage]
        y = self.convert(x, vt, active)
        if storage in ("bfloat16", "float16", "fp8_e4m3"):
            with np.errstate(invalid="ignore", over="ignore"):
                e = y.e + formats.UNIT_ROUNDOFF[storage] * (np.abs(y.v) + y.e) \
                    + formats.MIN_SUBNORMAL[storage] / 2
                u = y.u | (np.abs(y.v) + y.e >= formats.MAX_FINITE[storage])
            return Val(FLOAT, y.v, e, u)
        return y

    # -- truth values
    def truth(self, x: Val):
        if x.t == CFLOAT:
            raise CSyntaxError("a complex value has no truth value")
        return x.v != 0

    def truth_unsure(self, x: Val):
        if x.t in INT_TYPES:
            return x.u
        with np.errstate(invalid="ignore"):
            return x.u | ((np.abs(x.v) <= x.e) & (x.e > 0))

    # ------------------------------------------------------------ statements
    def run(self, stmts, active=None):
        active = np.ones(self.L, dtype=bool) if active is None else active
        for s in stmts:
            self.stmt(s, active)

    def stmt(self, s, active):
        if isinstance(s, ExprStmt):
            self.eval(s.expr, active)
        elif isinstance(s, Block):
            saved = dict(self.locals)
            self.scopes.append(set())
            self.run(s.stmts, active)
            declared = self.scopes.pop()
            # names declared inside the block go out of scope (shadowed outer
            # names get their outer value back)
            for name in declared:
                if name in saved:
                    self.locals[name] = saved[name]
                else:
                    del self.locals[name]
        elif isinstance(s, Decl):
            for name, init in s.items:
                if init is not None:
                    val = self.to_storage(self.eval(init, active), s.type, active)
                else:   # reading it before a store is undefined
                    val = self._mk(STORAGE_VT[s.type], 0, u=np.ones(self.L, dtype=bool))
                self.locals[name] = (s.type, val)
                self.scopes[-1].add(name)
        elif isinstance(s, If):
            c = self.eval(s.cond, active)
            truth = self.truth(c)
            unsure = self.truth_unsure(c)
            saved = self.taint
            self.taint = saved | unsure
            self.run([s.then], active & truth)
            if s.other is not None:
                self.run([s.other], active & ~truth)
            self.taint = saved
        else:
            raise CSyntaxError(f"unsupported statement {s!r}")

    # ------------------------------------------------------------ expressions
    def eval(self, node, active) -> Val:
        meth = getattr(self, "_e_" + type(node).__name__)
        return meth(node, active)

    def _e_Num(self, node, active):
        if node.is_float:
            if node.suffix == "f":
                return self._mk(FLOAT, f32_literal(node.value))
            if node.suffix == "l":
                raise CSyntaxError("long double literals are not supported")
            return self._mk(DOUBLE, float(node.value))
        value = node.value
        suffix, base = node.suffix.split("#")
        if suffix in ("", ):
            if value <= INT_RANGE[INT][1]:
                t = INT
            elif base == "nondec" and value <= INT_RANGE[UINT][1]:
                t = UINT
            elif value <= INT_RANGE[LONG][1]:
                t = LONG
            else:
                raise CSyntaxError("integer literal too large")
        elif suffix == "u":
            if value > INT_RANGE[UINT][1]:
                raise CSyntaxError("unsigned long literals are not supported")
            t = UINT
        elif suffix in ("l", "ll"):
            if value > INT_RANGE[LONG][1]:
                raise CSyntaxError("integer literal too large")
            t = LONG
        else:
            raise CSyntaxError("unsigned long literals are not supported")
        return self._mk(t, value)

    CONSTANTS = {
        "INFINITY": (FLOAT, math.inf), "NAN": (FLOAT, math.nan),
        "HUGE_VALF": (FLOAT, math.inf), "HUGE_VAL": (DOUBLE, math.inf),
        "FLT_MAX": (FLOAT, float(np.finfo(np.float32).max)),
        "FLT_MIN": (FLOAT, float(np.finfo(np.float32).tiny)),
        "DBL_MAX": (DOUBLE, float(np.finfo(np.float64).max)),
        "INT_MAX": (INT, 2 ** 31 - 1), "INT_MIN": (INT, -2 ** 31),
        "UINT_MAX": (UINT, 2 ** 32 - 1),
        "LLONG_MAX": (LONG, 2 ** 63 - 1), "LLONG_MIN": (LONG, -2 ** 63),
    }

    def _e_Name(self, node, active):
        name = node.ident
        if name in self.locals:
            return self.locals[name][1]
        if name == "i":
            return self._mk(self.idx_t, self.lanes)
        if name == "n":
            return self._mk(self.idx_t, self.n)
        if name in self.CONSTANTS:
            t, v = self.CONSTANTS[name]
            return self._mk(t, v)
        if name in self.arrays:
            raise CSyntaxError(f"array {name!r} used without a subscript")
        raise CSyntaxError(f"unknown name {name!r}")

    def _index_lane_local(self, node):
        return isinstance(node, Name) and node.ident == "i" and "i" not in self.locals

    def _e_Index(self, node, active):
        if node.base not in self.arrays:
            raise CSyntaxError(f"{node.base!r} is not an array argument")
        storage, raw = self.arrays[node.base]
        if self._index_lane_local(node.index):
            idx = self._mk(self.idx_t, self.lanes)
        else:
            idx = self.eval(node.index, active)
            if idx.t not in INT_TYPES:
                raise CSyntaxError("array subscript is not an integer")
            if node.base in self.overlay:
                raise OracleError(f"read of {node.base}[...] other than at i after a write")
        safe = np.where(active, idx.v, 0)
        if np.any(active & ((idx.v < 0) | (idx.v >= len(raw)))):
            raise OracleError(f"out-of-bounds read of {node.base}")
        v = self.decode(storage, raw[safe])
        val = self._mk(STORAGE_VT[storage], v, u=idx.u.copy())
        if self._index_lane_local(node.index) and node.base in self.overlay:
            ov = self.overlay[node.base]
            val = self._select(ov["w"], ov["val"], val)
        return val

    def _select(self, mask, a: Val, b: Val) -> Val:
        if a.t != b.t:
            raise AssertionError("select of different types")
        return Val(a.t, np.where(mask, a.v, b.v), np.where(mask, a.e, b.e),
                   np.where(mask, a.u, b.u))

    # -- assignment
    def _store(self, target, val, active):
        val = Val(val.t, val.v, val.e, val.u | self.taint)
        if isinstance(target, Name):
            name = target.ident
            if name in self.locals:
                storage, old = self.locals[name]
                new = self.to_storage(val, storage, active)
                self.locals[name] = (storage, self._select(active, new, old))
                return self.locals[name][1]
            raise CSyntaxError(f"assignment to {name!r}, which is not a local or scalar")
        if target.base not in self.arrays:
            raise CSyntaxError(f"{target.base!r} is not an array argument")
        if not self._index_lane_local(target.index):
            raise CSyntaxError("writes are supported only to name[i]")
        storage, _ = self.arrays[target.base]
        new = self.to_storage(val, storage, active)
        ov = self.overlay.get(target.base)
        if ov is None:
            ov = {"val": new, "w": active.copy()}
        else:
            ov = {"val": self._select(active, new, ov["val"]), "w": ov["w"] | active}
        self.overlay[target.base] = ov
        return new

    def _e_Assign(self, node, active):
        rhs = self.eval(node.value, active)
        if node.op != "=":
            cur = self.eval(node.target, active)
            rhs = self.binop(node.op[:-1], cur, rhs, active)
        return self._store(node.target, rhs, active)

    def _e_IncDec(self, node, active):
        cur = self.eval(node.target, active)
        one = self._mk(INT, 1)
        new = self.binop("+" if node.op == "++" else "-", cur, one, active)
        stored = self._store(node.target, new, active)
        return stored if node.prefix else cur

    def _e_Comma(self, node, active):
        self.eval(node.left, active)
        return self.eval(node.right, active)

    def _e_Cast(self, node, active):
        return self.to_storage(self.eval(node.operand, active), node.type, active)

    def _e_Cond(self, node, active):
        c = self.eval(node.cond, active)
        truth = self.truth(c)
        a = self.eval(node.then, active & truth)
        b = self.eval(node.other, active & ~truth)
        t = common_type(a.t, b.t)
        a, b = self.convert(a, t, active & truth), self.convert(b, t, active & ~truth)
        out = self._select(truth, a, b)
        out.u = out.u | self.truth_unsure(c)
        return out

    def _e_Logical(self, node, active):
        a = self.eval(node.left, active)
        ta = self.truth(a)
        right_lanes = ta if node.op == "&&" else ~ta
        b = self.eval(node.right, active & right_lanes)
        res = (ta & self.truth(b)) if node.op == "&&" else (ta | self.truth(b))
        u = self.truth_unsure(a) | (right_lanes & self.truth_unsure(b))
        return self._mk(INT, res.astype(np.int64), u=u)

    def _e_Unary(self, node, active):
        x = self.eval(node.operand, active)
        if node.op == "!":
            return self._mk(INT, (~self.truth(x)).astype(np.int64), u=self.truth_unsure(x))
        if node.op == "+":
            return x
        if node.op == "-":
            if x.t in FLOAT_TYPES or x.t == CFLOAT:
                return Val(x.t, -x.v, x.e, x.u)
            return self._int_result(x.t, -x.v, x.u, active)
        if node.op == "~":
            if x.t in FLOAT_TYPES:
                raise CSyntaxError("~ applied to a floating value")
            return self._mk(x.t, _wrap(~x.v, 32, x.t == INT) if x.t != LONG else ~x.v, u=x.u)
        raise CSyntaxError(node.op)

    def _e_Binary(self, node, active):
        a = self.eval(node.left, active)
        b = self.eval(node.right, active)
        return self.binop(node.op, a, b, active)

    # -- arithmetic
    def _int_result(self, t, v, u, active):
        """Checks a mathematically exact integer result against type t."""
        lo, hi = INT_RANGE[t]
        if t == UINT:
            return self._mk(t, np.asarray(v, dtype=np.int64) & 0xFFFFFFFF, u=u)
        if np.any(active & ((v < lo) | (v > hi))):
            raise OracleError(f"signed {t} overflow")
        return self._mk(t, v, u=u)

    def binop(self, op, a, b, active):
        if op in ("<<", ">>"):
            return self._shift(op, a, b, active)
        t = common_type(a.t, b.t)
        a, b = self.convert(a, t, active), self.convert(b, t, active)
        u = a.u | b.u
        if t == CFLOAT:
            if op not in ("+", "-", "*"):
                raise CSyntaxError(f"operator {op} is not supported on complex values")
            return self._complex_arith(op, a, b, u)
        if op in ("==", "!=", "<", ">", "<=", ">="):
            return self._compare(op, a, b, u)
        if t in FLOAT_TYPES:
            if op in ("%", "&", "|", "^"):
                raise CSyntaxError(f"operator {op} applied to floating values")
            return self._float_arith(op, a, b, t, u, active)
        return self._int_arith(op, a, b, t, u, active)

    def _compare(self, op, a, b, u):
        fn = {"==": np.equal, "!=": np.not_equal, "<": np.less, ">": np.greater,
              "<=": np.less_equal, ">=": np.greater_equal}[op]
        with np.errstate(invalid="ignore"):
            res = fn(a.v, b.v)
            if a.t in FLOAT_TYPES:
                slack = a.e + b.e
                u = u | ((np.abs(a.v - b.v) <= slack) & (slack > 0))
        return self._mk(INT, res.astype(np.int64), u=u)

    def _float_arith(self, op, a, b, t, u, active):
        ut = UNIT[t]
        with np.errstate(all="ignore"):
            if op == "+":
                v = a.v + b.v
                prop = a.e + b.e
            elif op == "-":
                v = a.v - b.v
                prop = a.e + b.e
            elif op == "*":
                v = a.v * b.v
                prop = np.abs(a.v) * b.e + np.abs(b.v) * a.e + a.e * b.e
            elif op == "/":
                v = a.v / b.v
                denom = np.abs(b.v) * (np.abs(b.v) - b.e)
                prop = np.where(np.abs(b.v) > b.e,
                                (np.abs(a.v) * b.e + np.abs(b.v) * a.e) / denom, np.inf)
                ut = 2 * ut           # allow one ulp for the device division
            else:
                raise CSyntaxError(op)
            e = prop + ut * (np.abs(v) + prop) + TINY[t] + EPS64 * np.abs(v)
            e = np.where(np.isnan(e) & np.isfinite(v), np.inf, e)
            u = u | (~np.isfinite(e) & np.isfinite(v))
        return Val(t, v, e, u)

    def _complex_arith(self, op, a, b, u):
        """Complex +, -, * with float components.  Each component of a sum
        rounds once (|error| <= u |v|); a product's components each take
        two products and a sum (with or without fused multiply-add), so its
        error is at most 2 sqrt(2) u |a| |b| in magnitude."""
        ut = UNIT[CFLOAT]
        with np.errstate(all="ignore"):
            if op in ("+", "-"):
                v = a.v + b.v if op == "+" else a.v - b.v
                prop = a.e + b.e
                e = prop + ut * (np.abs(v) + prop)
            else:
                v = a.v * b.v
                prop = np.abs(a.v) * b.e + np.abs(b.v) * a.e + a.e * b.e
                e = prop + 2 * math.sqrt(2) * ut * (np.abs(a.v) + a.e) * (np.abs(b.v) + b.e)
            e = e + 2 * TINY[CFLOAT] + EPS64 * np.abs(v)
            e = np.where(np.isnan(e) & np.isfinite(v), np.inf, e)
            u = u | (~np.isfinite(e) & np.isfinite(v))
        return Val(CFLOAT, v, e, u)

    def _int_arith(self, op, a, b, t, u, active):
        x, y = a.v, b.v
        if op in ("/", "%"):
            if np.any(active & (y == 0)):
                raise OracleError("integer division by zero")
            ys = np.where(y == 0, 1, y)
            if t == UINT:
                q, r = x // ys, x % ys
            else:
                if t == LONG and np.any(active & (x == -2 ** 63) & (ys == -1)):
                    raise OracleError("signed long overflow in division")
                q = np.abs(x) // np.abs(ys) * np.where((x < 0) != (ys < 0), -1, 1)
                r = x - q * ys
            return self._int_result(t, q if op == "/" else r, u, active)
        if op in ("&", "|", "^"):
            fn = {"&": np.bitwise_and, "|": np.bitwise_or, "^": np.bitwise_xor}[op]
            return self._mk(t, fn(x, y), u=u)
        if t == UINT:
            xu, yu = x.astype(np.uint64), y.astype(np.uint64)
            with np.errstate(over="ignore"):
                r = {"+": xu + yu, "-": xu - yu, "*": xu * yu}[op]
            return self._mk(t, (r & np.uint64(0xFFFFFFFF)).astype(np.int64), u=u)
        if t == INT:
            r = {"+": x + y, "-": x - y, "*": x * y}[op]
            return self._int_result(t, r, u, active)
        # LONG: detect wrap-around of int64 arithmetic
        with np.errstate(over="ignore"):
            if op == "+":
                r = x + y
                bad = ((x ^ r) & (y ^ r)) < 0
            elif op == "-":
                r = x - y
                bad = ((x ^ y) & (x ^ r)) < 0
            else:
                r = x * y
                xs = np.where(x == 0, 1, x)
                bad = (x != 0) & (r // xs != y)
                bad |= (x == -1) & (y == -2 ** 63)
                bad |= (y == -1) & (x == -2 ** 63)
        if np.any(active & bad):
            raise OracleError("signed long overflow")
        return self._mk(t, r, u=u)

    def _shift(self, op, a, b, active):
        if a.t in FLOAT_TYPES or b.t in FLOAT_TYPES:
            raise CSyntaxError("shift of a floating value")
        t = a.t
        bits = 64 if t == LONG else 32
        if np.any(active & ((b.v < 0) | (b.v >= bits))):
            raise OracleError("shift count out of range")
        s = np.where(active, b.v, 0)
        u = a.u | b.u
        if op == ">>":
            return self._mk(t, a.v >> s, u=u)
        if t == UINT:
            return self._mk(t, (a.v << s) & 0xFFFFFFFF, u=u)
        if np.any(active & (a.v < 0)):
            raise OracleError("left shift of a negative value")
        limit = INT_RANGE[t][1]
        with np.errstate(over="ignore"):
            big = active & (s > 0) & (a.v > (limit >> np.maximum(s, 0)))
        if np.any(big):
            raise OracleError("left shift overflow")
        return self._mk(t, a.v << s, u=u)

    # -- function calls
    # max ulp error allowed for device math functions (float, double)
    ULPS = {"sqrt": (1, 1), "exp": (4, 2), "log": (4, 2), "sin": (4, 2), "cos": (4, 2)}
    F_SUFFIX = {"sqrtf", "fabsf", "expf", "logf", "sinf", "cosf", "floorf", "ceilf",
                "truncf", "fmaxf", "fminf"}
    GENERIC = {"sqrt", "fabs", "exp", "log", "sin", "cos", "floor", "ceil", "trunc",
               "fmax", "fmin", "max", "min", "abs"}

    def _complex_call(self, f, args, active):
        """conj, real, imag and abs of a complex value (abs as the square root
        of the sum of the squared components: three roundings and the
        square root's)."""
        if len(args) != 1:
            raise CSyntaxError(f"{f} takes 1 argument")
        z = self.convert(args[0], CFLOAT, active)
        if f == "conj":
            return Val(CFLOAT, np.conj(z.v), z.e, z.u)
        if f in ("real", "imag"):
            return Val(FLOAT, z.v.real if f == "real" else z.v.imag, z.e, z.u)
        with np.errstate(all="ignore"):
            v = np.abs(z.v)
            e = z.e + 4 * UNIT[FLOAT] * (v + z.e) + TINY[FLOAT] + EPS64 * v
        return Val(FLOAT, v, e, z.u)

    def _e_Call(self, node, active):
        f = node.func
        if f in ("conj", "real", "imag"):
            return self._complex_call(f, [self.eval(x, active) for x in node.args], active)
        if f not in self.F_SUFFIX and f not in self.GENERIC:
            raise CSyntaxError(f"unsupported function {f!r}")
        args = [self.eval(x, active) for x in node.args]
        if f == "abs" and len(args) == 1 and args[0].t == CFLOAT:
            return self._complex_call(f, args, active)
        if any(x.t == CFLOAT for x in args):
            raise CSyntaxError(f"{f} of a complex value is not supported")
        base = f[:-1] if f in self.F_SUFFIX else f
        nargs = 2 if base in ("fmax", "fmin", "max", "min") else 1
        if len(args) != nargs:
            raise CSyntaxError(f"{f} takes {nargs} argument(s)")
        if f in self.F_SUFFIX:
            t = FLOAT
        elif base in ("max", "min", "abs"):
            t = args[0].t if nargs == 1 else common_type(args[0].t, args[1].t)
        else:
            t = common_type(*(x.t for x in args))
            if t in INT_TYPES:
                t = DOUBLE            # C++ <cmath>: integral arguments -> double
        args = [self.convert(x, t, active) for x in args]
        u = args[0].u if nargs == 1 else args[0].u | args[1].u
        if t in INT_TYPES:
            if base == "abs":
                return self._int_result(t, np.abs(args[0].v), u, active)
            fn = np.maximum if base == "max" else np.minimum
            return self._mk(t, fn(args[0].v, args[1].v), u=u)
        a = args[0]
        ulp = 2 * UNIT[t]
        with np.errstate(all="ignore"):
            if nargs == 2:
                fn = np.fmax if base in ("fmax", "max") else np.fmin
                v = fn(a.v, args[1].v)
                return Val(t, v, np.maximum(a.e, args[1].e), u)
            if base in ("fabs", "abs"):
                return Val(t, np.abs(a.v), a.e, u)
            if base in ("floor", "ceil", "trunc"):
                fn = {"floor": np.floor, "ceil": np.ceil, "trunc": np.trunc}[base]
                v = fn(a.v)
                u = u | (fn(a.v - a.e) != fn(a.v + a.e))
                return Val(t, v, np.zeros(self.L), u)
            k = self.ULPS[base][0 if t == FLOAT else 1]
            if base == "sqrt":
                v = np.sqrt(a.v)
                lo = np.maximum(a.v - a.e, 0.0)
                prop = np.minimum(a.e / (np.sqrt(lo) + np.sqrt(np.abs(a.v))), np.sqrt(a.e))
                prop = np.where(a.e == 0, 0.0, prop)
                u = u | ((a.v - a.e < 0) & (a.e > 0)) | (active & (a.v < 0))
            elif base == "exp":
                v = np.exp(a.v)
                prop = np.abs(v) * np.expm1(a.e)
            elif base == "log":
                v = np.log(a.v)
                prop = np.where(a.v - a.e > 0, np.log(a.v / (a.v - a.e)), np.inf)
                prop = np.where(a.e == 0, 0.0, prop)
                u = u | ((a.v - a.e <= 0) & (a.e > 0))
            else:   # sin, cos
                v = np.sin(a.v) if base == "sin" else np.cos(a.v)
                prop = a.e
            e = prop + k * ulp * (np.abs(v) + prop) + TINY[t] + EPS64 * np.abs(v)
            u = u | (~np.isfinite(e) & np.isfinite(v))
        return Val(t, v, e, u)
