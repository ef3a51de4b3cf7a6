"""Lazy array expressions fused into one generated kernel.

The paper's array objects evaluate every operator at once, so a nested
expression makes one temporary array per intermediate result, each written
to and read back from memory (section "Efficient Evaluation of Element-wise
Expressions": the temporaries problem).  Its elementwise and map-reduce
facilities are the remedy when the user writes the fused C expression by
hand.  This module writes it for them.  Operators on `LazyArray` build an
expression tree; evaluating the tree renders it as one C statement over the
formal index i, compiles it through the cached run-time path, and runs one
elementwise kernel (or one map-reduce for sum / max / min / dot).  The same
tree can also run one kernel per operator (`fused=False`), the behaviour of
eager array arithmetic, for comparison.

Values are computed in float (the storage formats bfloat16 / half / FP8 are
read as float); integer leaves are converted to float.

`shift(e, k, fill)` is e at index i + k (fill outside [0, n)): its leaves
render as shifted reads a[i + k], which the vector kernels load as
unaligned chunks, so a stencil such as x - 0.5 * (shift(x, -1) + shift(x, 1))
is one fused kernel too.
"""

from __future__ import annotations

import functools
import hashlib
import math
import numbers

from . import hipmr as _hm

_STORAGE = {"torch.float32": "float", "torch.bfloat16": "bfloat16", "torch.float16": "half",
            "torch.float8_e4m3fn": "fp8_e4m3", "torch.int32": "int", "torch.float64": "double"}

_BINARY = {"+": "+", "-": "-", "*": "*", "/": "/"}
_FUNCS = {"sqrt": "sqrtf", "exp": "expf", "log": "logf", "sin": "sinf", "cos": "cosf",
          "abs": "fabsf", "maximum": "fmaxf", "minimum": "fminf"}


def _float_literal(v: float) -> str:
    """C float literal of v rounded to float32 (the text holds the float32
    value exactly, so the compiler's one rounding gives it back)."""
    import numpy as np
    if math.isnan(v) or math.isinf(v):
        raise ValueError("non-finite constants are not supported in lazy expressions")
    with np.errstate(over="raise"):
        v32 = float(np.float32(v))
    return repr(v32) + "f"


class LazyArray:
    """A node of an elementwise expression over same-length device arrays."""

    __array_priority__ = 1000

    def __init__(self, op, args=(), tensor=None, value=None):
        self.op, self.args, self.tensor, self.value = op, tuple(args), tensor, value

    # ---- construction
    @staticmethod
    def _wrap(v):
        if isinstance(v, LazyArray):
            return v
        if isinstance(v, numbers.Real):
            return LazyArray("const", value=float(v))
        raise TypeError(f"cannot use {type(v).__name__} in a lazy expression")

    def _bin(self, op, other, swap=False):
        o = LazyArray._wrap(other)
        return LazyArray(op, (o, self) if swap else (self, o))

    def __add__(self, o): return self._bin("+", o)
    def __radd__(self, o): return self._bin("+", o, True)
    def __sub__(self, o): return self._bin("-", o)
    def __rsub__(self, o): return self._bin("-", o, True)
    def __mul__(self, o): return self._bin("*", o)
    def __rmul__(self, o): return self._bin("*", o, True)
    def __truediv__(self, o): return self._bin("/", o)
    def __rtruediv__(self, o): return self._bin("/", o, True)
    def __neg__(self): return LazyArray("neg", (self,))

    # ---- reductions (one fused map-reduce)
    def sum(self, out=None, stream=None): return _reduce(self, "a+b", "0", out, stream)
    def max(self, out=None, stream=None): return _reduce(self, "max(a,b)", "-INFINITY", out, stream)
    def min(self, out=None, stream=None): return _reduce(self, "min(a,b)", "INFINITY", out, stream)

    # ---- evaluation
    def eval(self, out=None, fused=True, stream=None):
        """Evaluates the tree into `out` (a new float32 tensor by default)."""
        return evaluate(self, out=out, fused=fused, stream=stream)

    def leaves(self):
        seen, order = set(), []

        def walk(node):
            if node.op == "leaf":
                if id(node.tensor) not in seen:
                    seen.add(id(node.tensor))
                    order.append(node.tensor)
            for a in node.args:
                walk(a)
        walk(self)
        return order


def lazy(tensor) -> LazyArray:
    """Wraps a 1-D contiguous device tensor as a lazy leaf."""
    if tensor.dim() != 1 or not tensor.is_contiguous():
        raise ValueError("lazy arrays are flat contiguous tensors")
    if str(tensor.dtype) not in _STORAGE:
        raise TypeError(f"unsupported dtype {tensor.dtype}")
    return LazyArray("leaf", tensor=tensor)


def _fn(name):
    def f(*xs):
        return LazyArray(name, tuple(LazyArray._wrap(x) for x in xs))
    f.__name__ = name
    return f


sqrt, exp, log, sin, cos, abs, maximum, minimum = (_fn(n) for n in _FUNCS)   # noqa: A001


def shift(node, k, fill=0.0):
    """The expression at index i + k (an integer), `fill` where i + k falls
    outside [0, n)."""
    if not isinstance(k, numbers.Integral) or isinstance(k, bool):
        raise TypeError("a shift distance is an integer")
    return LazyArray("shift", (LazyArray._wrap(node),), value=(int(k), float(fill)))


def dot(a, b, out=None, stream=None):
    return (LazyArray._wrap(a) * LazyArray._wrap(b)).sum(out=out, stream=stream)


# ------------------------------------------------------------------ rendering
def render(node: LazyArray):
    """(C expression text over a0[i], a1[i], ...; the leaf tensors in argument
    order).  Leaves are read as float."""
    leaves = node.leaves()
    index = {id(t): k for k, t in enumerate(leaves)}

    def text(n, at=0):            # the subtree at index i + at
        idx = "i" if at == 0 else (f"i + {at}" if at > 0 else f"i - {-at}")
        if n.op == "leaf":
            return f"(float)a{index[id(n.tensor)]}[{idx}]"
        if n.op == "const":
            return _float_literal(n.value)
        if n.op == "shift":
            k, fill = n.value
            j = at + k
            jdx = "i" if j == 0 else (f"i + {j}" if j > 0 else f"i - {-j}")
            return f"({jdx} >= 0 && {jdx} < n ? {text(n.args[0], j)} : {_float_literal(fill)})"
        if n.op == "neg":
            return f"(-{text(n.args[0], at)})"
        if n.op in _BINARY:
            return f"({text(n.args[0], at)} {_BINARY[n.op]} {text(n.args[1], at)})"
        return f"{_FUNCS[n.op]}({', '.join(text(a, at) for a in n.args)})"
    return text(node), leaves


def _decls(leaves):
    return ", ".join(f"const {_STORAGE[str(t.dtype)]} *a{k}" for k, t in enumerate(leaves))


def _name(text):
    return "lazy_" + hashlib.sha256(text.encode()).hexdigest()[:10]


@functools.lru_cache(maxsize=1024)
def _kernel(expr, dtypes, name):
    """The compiled handle of one rendered expression, kept for the next
    evaluation of the same tree shape (the library's own cache would find
    it too, after parsing and rendering the source again)."""
    return _hm.compile(expr, dtypes, name=name)


def elementwise_source(node: LazyArray):
    """(dtypes, statement, leaves) of the fused elementwise kernel."""
    expr, leaves = render(node)
    dtypes = "float *out" + (", " + _decls(leaves) if leaves else "")
    return dtypes, f"out[i] = {expr}", leaves


def reduce_source(node: LazyArray):
    """(dtypes, map expression, leaves) of the fused map-reduce kernel."""
    expr, leaves = render(node)
    if not leaves:
        raise ValueError("a reduction needs at least one array")
    return "float: " + _decls(leaves), expr, leaves


def _length(leaves):
    ns = {t.numel() for t in leaves}
    if len(ns) != 1:
        raise ValueError("lazy arrays in one expression must have the same length")
    return ns.pop()


def evaluate(node: LazyArray, out=None, fused=True, stream=None):
    import torch
    node = LazyArray._wrap(node)
    if not fused:
        return _evaluate_unfused(node, out, stream)
    dtypes, stmt, leaves = elementwise_source(node)
    if not leaves:
        raise ValueError("an expression needs at least one array")
    n = _length(leaves)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=leaves[0].device)
    k = _kernel(stmt, dtypes, _name(stmt))
    _hm.elementwise(k, n, [out, *leaves], stream=stream)
    return out


def _evaluate_unfused(node, out, stream):
    """One kernel per operator, each writing a float32 temporary (the
    behaviour of eagerly evaluated array operators); the root operator
    writes `out`."""
    import torch

    def ev(n, dst=None):
        if n.op in ("leaf", "const"):
            return n
        kids = [ev(a) for a in n.args]
        sub = LazyArray(n.op, kids, value=n.value)
        arrays = [k for k in kids if k.op == "leaf"]
        if not arrays:
            raise ValueError("an expression needs at least one array")
        length = _length([k.tensor for k in arrays])
        t = dst if dst is not None else torch.empty(length, dtype=torch.float32,
                                                    device=arrays[0].tensor.device)
        evaluate(sub, out=t, fused=True, stream=stream)
        return LazyArray("leaf", tensor=t)
    res = ev(node, out)
    if res.op != "leaf":
        raise ValueError("an expression needs at least one array")
    return res.tensor


def _reduce(node, combine, neutral, out, stream):
    import torch
    dtypes, expr, leaves = reduce_source(node)
    n = _length(leaves)
    if out is None:
        out = torch.empty((), dtype=torch.float32, device=leaves[0].device)
    k = _kernel(expr, dtypes, _name(dtypes + expr))
    _hm.reduce(k, None, combine, neutral, n, leaves, out, stream=stream)
    return out


__all__ = ["LazyArray", "lazy", "evaluate", "render", "elementwise_source", "reduce_source",
           "dot", "shift", "sqrt", "exp", "log", "sin", "cos", "abs", "maximum", "minimum"]
