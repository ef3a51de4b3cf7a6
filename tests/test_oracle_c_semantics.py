"""Property tests of the oracle's C integer arithmetic (no GPU): for random
int32 and uint32 operands, every binary operator either gives the value C
defines (truncating division, modulo with the dividend's sign, unsigned
wrap-around, shifts within the width) or, where C leaves the result
undefined (signed overflow, division by zero, shift counts outside the
width), raises instead of inventing a value.  The reference is plain Python
integer arithmetic written out from the C rules."""

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import OracleError

I32 = st.integers(-(2 ** 31), 2 ** 31 - 1)
U32 = st.integers(0, 2 ** 32 - 1)
OPS = ["+", "-", "*", "/", "%", "&", "|", "^", "<<", ">>"]


def c_int(op, a, b):
    """int op int in C, or None where the behaviour is undefined."""
    if op in ("/", "%"):
        if b == 0 or (a == -(2 ** 31) and b == -1):
            return None
        q = abs(a) // abs(b) * (1 if (a < 0) == (b < 0) else -1)
        r = q if op == "/" else a - q * b
    elif op in ("<<", ">>"):
        if not 0 <= b < 32 or (op == "<<" and a < 0):
            return None
        r = a << b if op == "<<" else a >> b
    else:
        r = {"+": a + b, "-": a - b, "*": a * b, "&": a & b, "|": a | b, "^": a ^ b}[op]
    return r if -(2 ** 31) <= r < 2 ** 31 else None


def c_uint(op, a, b):
    """unsigned op unsigned in C (arithmetic modulo 2^32)."""
    if op in ("/", "%"):
        if b == 0:
            return None
        return a // b if op == "/" else a % b
    if op in ("<<", ">>"):
        if not 0 <= b < 32:
            return None
        return (a << b) % 2 ** 32 if op == "<<" else a >> b
    return {"+": a + b, "-": a - b, "*": a * b, "&": a & b, "|": a | b, "^": a ^ b}[op] % 2 ** 32


def run(ctype, op, a, b, np_t):
    x, y = np.array([a], np_t), np.array([b], np_t)
    out = np.zeros(1, np.int64)
    sig = f"const {ctype} *x, const {ctype} *y, long *o"
    return oracle.elementwise(sig, f"o[i] = x[i] {op} y[i]", 1, [x, y, out])["o"].v.tolist()[0]


@settings(max_examples=300, deadline=None)
@given(st.sampled_from(OPS), I32, st.one_of(I32, st.integers(-3, 40)))
def test_int32_operators_follow_c(op, a, b):
    want = c_int(op, a, b)
    if want is None:
        with pytest.raises(OracleError):
            run("int", op, a, b, np.int32)
    else:
        assert run("int", op, a, b, np.int32) == want


@settings(max_examples=300, deadline=None)
@given(st.sampled_from(OPS), U32, st.one_of(U32, st.integers(0, 40)))
def test_uint32_operators_follow_c(op, a, b):
    want = c_uint(op, a, b)
    if want is None:
        with pytest.raises(OracleError):
            run("unsigned", op, a, b, np.uint32)
    else:
        assert run("unsigned", op, a, b, np.uint32) == want


@settings(max_examples=300, deadline=None)
@given(st.one_of(I32, st.integers(-(2 ** 62), 2 ** 62)))
def test_integer_to_float_bound_holds_the_rounded_value(v):
    # (float) of an int / long: the oracle keeps the exact value with an
    # allowance of one float32 rounding, which must contain numpy's
    # round-to-nearest-even conversion and be no wider than 2^-24 |v|
    ctype, np_t = ("int", np.int32) if -(2 ** 31) <= v < 2 ** 31 else ("long", np.int64)
    k = np.array([v], np_t)
    out = np.zeros(1, np.float32)
    o = oracle.elementwise(f"const {ctype} *k, float *o", "o[i] = (float)k[i]", 1, [k, out])["o"]
    exact, e = o.v.tolist()[0], float(o.e[0])
    assert exact == float(v) or abs(exact - v) <= abs(v) * 2.0 ** -53
    # (plus, above 2^53, the float64 representation error of the value itself)
    assert abs(float(np.float32(v)) - exact) <= e <= (2.0 ** -24 + 2.0 ** -52) * abs(v) * (1 + 1e-9) + 2.0 ** -126


@settings(max_examples=300, deadline=None)
@given(st.floats(-3e9, 3e9, width=32, allow_nan=False))
def test_float_to_int_truncates_or_raises(f):
    # (int) of a float truncates toward zero; outside the int range C leaves
    # the conversion undefined and the oracle raises
    x = np.array([f], np.float32)
    out = np.zeros(1, np.int32)
    t = int(np.trunc(np.float64(x[0])))
    if -(2 ** 31) <= t < 2 ** 31:
        o = oracle.elementwise("const float *x, int *o", "o[i] = (int)x[i]", 1, [x, out])["o"]
        assert o.v.tolist()[0] == t
    else:
        with pytest.raises(OracleError):
            oracle.elementwise("const float *x, int *o", "o[i] = (int)x[i]", 1, [x, out])
