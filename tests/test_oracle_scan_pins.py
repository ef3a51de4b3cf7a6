"""Pins of the oracle's prefix scan (section "Further Facilities": parallel
prefix sums over a map expression, a combine expression and its neutral
element).  Each pin is fixed by something other than the oracle's own
arithmetic: closed forms, the oracle's independently pinned reduce,
Python's correctly rounded math.fsum per prefix, brute-force Python folds and
exact integer identities."""

import math

import numpy as np
import pytest

import oracle
from oracle import OracleError

LONG_K = "long: const int *k"


def test_inclusive_and_exclusive_sum_of_index_closed_form():
    n = 10007
    k = np.arange(n, dtype=np.int32)
    inc = oracle.scan(LONG_K, "k[i]", "a+b", "0", n, [k])
    exc = oracle.scan(LONG_K, "k[i]", "a+b", "0", n, [k], exclusive=True)
    i = np.arange(n, dtype=np.int64)
    assert inc.exact and inc.values.tolist() == (i * (i + 1) // 2).tolist()
    assert exc.values.tolist() == (i * (i - 1) // 2).tolist()


def test_count_scan_closed_form():
    n = 5000
    k = np.arange(n, dtype=np.int32)
    r = oracle.scan(LONG_K, "k[i] % 7 == 3", "a+b", "0", n, [k])
    i = np.arange(n)
    want = np.where(i >= 3, (i - 3) // 7 + 1, 0)
    assert r.values.tolist() == want.tolist()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_last_inclusive_prefix_is_the_reduce(seed):
    rng = np.random.default_rng(seed)
    n = 3001
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    sig = "float: const float *x, const float *y"
    for mp, comb, neu in (("x[i]*y[i]", "a+b", "0"), ("x[i]", "max(a,b)", "-INFINITY"),
                          ("x[i]+y[i]", "min", "INFINITY")):
        s = oracle.scan(sig, mp, comb, neu, n, [x, y])
        r = oracle.reduce(sig, mp, comb, neu, n, [x, y])
        assert s.values[-1] == r.value, (mp, comb)


@pytest.mark.parametrize("seed", [3, 4])
def test_float_prefixes_are_correctly_rounded_exact_sums(seed):
    rng = np.random.default_rng(seed)
    n = 700
    # wide dynamic range and cancellation
    x = (rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n))).astype(np.float32)
    x[1::2] = -x[0::2][: n // 2] * np.float32(1.0 + 2.0 ** -20)
    sig = "float: const float *x"
    r = oracle.scan(sig, "x[i]", "a+b", "0", n, [x])
    vals = x.astype(np.float64).tolist()
    for k in range(n):
        assert r.values[k] == math.fsum(vals[: k + 1]), k
    e = oracle.scan(sig, "x[i]", "a+b", "0", n, [x], exclusive=True)
    assert e.values[0] == 0.0
    assert np.array_equal(e.values[1:], r.values[:-1])
    assert np.allclose(r.abs_prefix, np.cumsum(np.abs(vals)), rtol=1e-12)


def test_products_of_float32_are_summed_exactly():
    # the map value x*y of two float32 has up to 48 significant bits: still
    # exact in float64, so the prefix is fsum of the exact products
    rng = np.random.default_rng(5)
    n = 400
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    r = oracle.scan("float: const float *x, const float *y", "x[i]*y[i]", "a+b", "0", n, [x, y])
    p = (x.astype(np.float64) * y.astype(np.float64)).tolist()
    for k in range(0, n, 7):
        assert r.values[k] == math.fsum(p[: k + 1])
    assert np.all(r.err_prefix > 0)


def test_walsh_prefix_sums_are_integers():
    n = 1 << 12
    i = np.arange(n)
    x = np.where(np.array([bin(v & 0x5A5).count("1") for v in i]) % 2 == 0, 1.0, -1.0).astype(np.float32)
    r = oracle.scan("float: const float *x", "x[i]", "a+b", "0", n, [x])
    assert r.values.tolist() == np.cumsum(x.astype(np.int64)).astype(np.float64).tolist()


def test_max_min_prefix_brute_force_with_signed_zero_and_nan():
    x = np.array([-0.0, 0.0, -1.0, -0.0, 3.0, np.nan, 5.0], np.float32)
    sig = "float: const float *x"
    mx = oracle.scan(sig, "x[i]", "max(a,b)", "-INFINITY", x.size, [x])
    mn = oracle.scan(sig, "x[i]", "min(a,b)", "INFINITY", x.size, [x])
    got_mx = mx.values.tolist()
    assert got_mx[0] == 0.0 and math.copysign(1, got_mx[0]) < 0       # max(-0) = -0
    assert got_mx[1] == 0.0 and math.copysign(1, got_mx[1]) > 0       # max(-0, +0) = +0
    assert got_mx[2] == 0.0 and math.copysign(1, got_mx[2]) > 0
    assert got_mx[4] == 3.0 and math.isnan(got_mx[5]) and math.isnan(got_mx[6])
    got_mn = mn.values.tolist()
    assert math.copysign(1, got_mn[0]) < 0 and math.copysign(1, got_mn[1]) < 0
    assert got_mn[2] == -1.0 and math.isnan(got_mn[5]) and math.isnan(got_mn[6])
    # integer max: brute force
    rng = np.random.default_rng(6)
    k = rng.integers(-1000, 1000, 300).astype(np.int32)
    r = oracle.scan("int: const int *k", "k[i]", "max", "INT_MIN", k.size, [k])
    assert r.values.tolist() == [max(k[: j + 1].tolist()) for j in range(k.size)]


def test_generic_combine_product_is_factorial():
    n = 20
    k = np.arange(1, n + 1, dtype=np.int32)
    r = oracle.scan(LONG_K, "k[i]", "a*b", "1", n, [k])
    assert r.op == "generic" and r.values.tolist() == [math.factorial(j + 1) for j in range(n)]
    e = oracle.scan(LONG_K, "k[i]", "a*b", "1", n, [k], exclusive=True)
    assert e.values.tolist() == [math.factorial(j) for j in range(n)]


def test_empty_and_neutral():
    z = np.zeros(0, np.int32)
    r = oracle.scan(LONG_K, "k[i]", "a+b", "0", 0, [z])
    assert r.values.size == 0
    k = np.array([5], np.int32)
    e = oracle.scan(LONG_K, "k[i]", "a+b", "7", 1, [k], exclusive=True)
    assert e.values.tolist() == [7]
    i = oracle.scan(LONG_K, "k[i]", "a+b", "7", 1, [k])
    assert i.values.tolist() == [12]


def test_prefix_overflow_has_no_value():
    k = np.full(3, 2 ** 30, np.int32)
    with pytest.raises(OracleError):
        oracle.scan("int: const int *k", "k[i]", "a+b", "0", 3, [k])
    # the same data into a long result is fine
    r = oracle.scan(LONG_K, "k[i]", "a+b", "0", 3, [k])
    assert r.values.tolist() == [2 ** 30, 2 ** 31, 3 * 2 ** 30]


def test_unsigned_prefix_wraps():
    k = np.array([2 ** 31, 2 ** 31, 5], np.uint32)
    r = oracle.scan("unsigned int: const unsigned int *k", "k[i]", "a+b", "0", 3, [k])
    assert r.values.tolist() == [2 ** 31, 0, 5]
