"""Host side of the lazy expression front end (the temporaries problem of
section "Efficient Evaluation of Element-wise Expressions", solved by fusing
an operator tree into one generated kernel): the rendered C statement,
evaluated by the oracle, equals a float64 numpy evaluation of the same
tree; caching and error handling."""

import math

import numpy as np
import pytest
import torch

import oracle
import paper_1304_5553_amd as hm
from paper_1304_5553_amd import lazy as lz


def np_eval(node, env):
    """Independent float64 evaluation of a lazy tree with numpy."""
    if node.op == "leaf":
        return env[id(node.tensor)]
    if node.op == "const":
        return np.float64(np.float32(node.value))
    if node.op == "shift":                        # the child at i + k, fill outside [0, n)
        k, fill = node.value
        a = np.broadcast_to(np_eval(node.args[0], env), (env["n"],))
        out = np.full(env["n"], np.float64(np.float32(fill)))
        lo, hi = max(0, -k), min(env["n"], env["n"] - k)
        if lo < hi:
            out[lo:hi] = a[lo + k:hi + k]
        return out
    a = [np_eval(x, env) for x in node.args]
    ops = {"+": np.add, "-": np.subtract, "*": np.multiply, "/": np.divide, "neg": np.negative,
           "sqrt": np.sqrt, "exp": np.exp, "log": np.log, "sin": np.sin, "cos": np.cos,
           "abs": np.abs, "maximum": np.fmax, "minimum": np.fmin}
    return ops[node.op](*a)


def leaves(n, seed, dtypes=("float32", "float32", "float32")):
    rng = np.random.default_rng(seed)
    out = []
    for dt in dtypes:
        v = rng.uniform(0.1, 2.0, n).astype(np.float32)
        if dt == "bfloat16":
            t = torch.from_numpy(v).to(torch.bfloat16)
        elif dt == "int32":
            t = torch.from_numpy((v * 100).astype(np.int32))
        else:
            t = torch.from_numpy(v)
        out.append(t)
    return out


EXPRS = {
    "poly": lambda x, y, w: 2.5 * x * y + lz.sqrt(x * x + y * y) - 0.5 * w,
    "ratio": lambda x, y, w: (x - y) / (w + 1.0) + lz.maximum(x, w) - lz.minimum(y, 0.75),
    "trans": lambda x, y, w: lz.exp(-x) * lz.sin(y) + lz.log(w) * lz.cos(x) - lz.exp(y - w),
    "reuse": lambda x, y, w: (x + x) * (x - 3) + lz.abs(-y),
    "stencil": lambda x, y, w: (x - 0.5 * (lz.shift(x, -1) + lz.shift(x, 1))
                                + lz.shift(y * w + lz.shift(w, -2), 3, fill=2.0)),
}


@pytest.mark.parametrize("name", list(EXPRS))
@pytest.mark.parametrize("dts", [("float32",) * 3, ("bfloat16", "float32", "int32")])
def test_rendered_statement_is_the_tree(name, dts):
    n = 1000
    ts = leaves(n, hash(name) % 100, dts)
    node = EXPRS[name](*(lz.lazy(t) for t in ts))
    dtypes, stmt, lv = lz.elementwise_source(node)
    env = {id(t): t.to(torch.float64).numpy() for t in ts}
    env["n"] = n
    want = np_eval(node, env)
    arrays = [np.zeros(n, np.float32)] + [
        t.view(torch.int16).numpy().view(np.uint16) if t.dtype == torch.bfloat16 else t.numpy() for t in lv]
    got = oracle.elementwise(dtypes, stmt, n, arrays)["out"]
    # the oracle's ideal values are float64 evaluations of the same operations
    assert np.allclose(got.v, want, rtol=1e-12, atol=1e-300), name
    assert len(lv) == len({id(t) for t in ts if any(t is u for u in lv)})   # each tensor once


def test_constants_round_to_float32_once():
    assert lz._float_literal(0.1) == repr(float(np.float32(0.1))) + "f"
    assert float(lz._float_literal(2.5)[:-1]) == 2.5
    with pytest.raises(ValueError):
        lz._float_literal(float("inf"))


def test_reduce_source_and_errors():
    x, y, _ = (lz.lazy(t) for t in leaves(10, 1))
    dtypes, expr, lv = lz.reduce_source(x * y)
    assert dtypes.startswith("float: ") and len(lv) == 2
    with pytest.raises(TypeError):
        _ = x + "a"
    with pytest.raises(ValueError):
        lz.lazy(torch.zeros(2, 2))


def test_shift_renders_shifted_reads():
    x, y, _ = (lz.lazy(t) for t in leaves(10, 3))
    node = x - 0.5 * (lz.shift(x, -1) + lz.shift(x, 1))
    dtypes, stmt, lv = lz.elementwise_source(node)
    assert "a0[i - 1]" in stmt and "a0[i + 1]" in stmt and "i - 1 >= 0" in stmt
    k = hm.compile(stmt, dtypes)
    assert k.vectorizable and "hipmr_loadu" in k.source(0)     # shifted chunk loads
    nested = lz.shift(lz.shift(y, 2) * x, -5, fill=1.0)          # distances add up
    assert "a0[i - 3]" in lz.render(nested)[0] and "a1[i - 5]" in lz.render(nested)[0]
    with pytest.raises(TypeError):
        lz.shift(x, 1.5)


def test_same_tree_same_kernel():
    x, y, w = (lz.lazy(t) for t in leaves(10, 2))
    a = lz.elementwise_source(2.5 * x * y - w)
    b = lz.elementwise_source(2.5 * x * y - w)
    assert a[:2] == b[:2]
    k1 = hm.compile(a[1], a[0], name=lz._name(a[1]))
    k2 = hm.compile(b[1], b[0], name=lz._name(b[1]))
    assert k1.source(0) == k2.source(0)


def test_repeated_evaluation_reuses_the_compiled_handle():
    # a tree of the same shape over other arrays renders the same statement,
    # so its evaluation reuses the handle compiled for the first one
    x, y, w = (lz.lazy(t) for t in leaves(10, 2))
    p, q, r = (lz.lazy(t) for t in leaves(20, 3))
    a = lz.elementwise_source(2.5 * x * y - w)
    b = lz.elementwise_source(2.5 * p * q - r)
    assert a[:2] == b[:2]
    k1 = lz._kernel(a[1], a[0], lz._name(a[1]))
    k2 = lz._kernel(b[1], b[0], lz._name(b[1]))
    assert k1 is k2
    c = lz.elementwise_source(2.5 * x * y + w)
    assert lz._kernel(c[1], c[0], lz._name(c[1])) is not k1
