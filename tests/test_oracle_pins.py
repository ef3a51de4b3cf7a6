"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these tests call the GPU library.  Each pin is chosen so that a
plausible mistake in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a missing rounding allowance) fails at least one of them.
"""

import functools
import math
import operator
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import OracleError

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                key, *vals = line.split()
                out[key] = [int(v) for v in vals] if len(vals) > 1 else int(vals[0])
    return out


# ------------------------------------------------------------ paper listings
def test_listing3b_dot_of_arange():
    g = golden("listing3b_dot.txt")
    n = g["n"]
    a = np.arange(n, dtype=np.float32)
    r = oracle.reduce("float: float *x, float *y", "x[i]*y[i]", "a+b", "0", n, [a, a])
    assert r.value == g["value"] == (n - 1) * n * (2 * n - 1) // 6
    assert r.op == "sum" and r.abs_sum >= r.value


def test_listing4_unrolled_add_is_the_rounded_sum():
    g = golden("listing4_add.txt")
    n = g["block_size"] * g["thread_block_size"] * g["macroblock_count"]
    assert n == g["n"]
    rng = np.random.default_rng(44)
    a = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    c = np.zeros(n, np.float32)
    o = oracle.elementwise("float *tgt, float *op1, float *op2",
                           "tgt[i] = op1[i] + op2[i]", n, [c, a, b])["tgt"]
    # one float32 addition is correctly rounded: rounding the exact value the
    # oracle holds must give numpy's float32 sum bit for bit
    assert np.array_equal(o.v.astype(np.float32), a + b)
    assert np.all(np.abs(o.v - (a + b).astype(np.float64)) <= o.e)


def test_listing1_multiply_by_two_exact():
    g = golden("listing1_multiply2.txt")
    rng = np.random.default_rng(1)
    a = rng.standard_normal(g["shape"]).astype(np.float32).reshape(-1)
    o = oracle.elementwise("float *a", "a[i] *= 2", a.size, [a])["a"]
    assert np.array_equal(o.v, 2.0 * a.astype(np.float64))
    assert np.array_equal(o.v.astype(np.float32), 2 * a)


def test_listing3a_linear_combination_bound_contains_float32_result():
    g = golden("listing3a_lincomb.txt")
    n = g["n"]
    rng = np.random.default_rng(2)
    x = rng.random(n).astype(np.float32)
    y = rng.random(n).astype(np.float32)
    z = np.zeros(n, np.float32)
    o = oracle.elementwise("float a, float *x, float b, float *y, float *z",
                           "z[i] = a*x[i] + b*y[i]", n, [g["a"], x, g["b"], y, z])["z"]
    exact = [Fraction(g["a"]) * Fraction(float(xi)) + Fraction(g["b"]) * Fraction(float(yi))
             for xi, yi in zip(x, y)]
    assert np.array_equal(o.v, np.array([float(q) for q in exact]))
    f32 = np.float32(g["a"]) * x + np.float32(g["b"]) * y          # one GPU-like order
    fma = (np.float32(g["a"]) * x).astype(np.float64) + np.float64(g["b"]) * y
    assert np.all(np.abs(f32 - o.v) <= o.e)
    assert np.all(np.abs(fma.astype(np.float32) - o.v) <= o.e)
    # and the bound is not vacuous: a few float32 ulps
    assert np.all(o.e <= 4 * 2.0 ** -24 * (5 * x + 6 * y) + 1e-30)


# ------------------------------------------------------------ closed forms
def test_sum_of_index_closed_form():
    n = 1 << 22
    r = oracle.reduce("long: int *unused", "i", "a+b", "0", n, [np.zeros(1, np.int32)])
    assert r.value == n * (n - 1) // 2 and r.exact


def test_sum_of_int32_k_closed_form():
    n = 1 << 20
    k = np.arange(n, dtype=np.int32)
    r = oracle.reduce("long: const int *k", "k[i]", "a+b", "0", n, [k])
    assert r.value == n * (n - 1) // 2


@pytest.mark.parametrize("n", list(range(0, 60)) + [199, 1 << 16, (1 << 22) + 5])
def test_count_mod7_closed_form(n):
    k = np.arange(n, dtype=np.int32)
    r = oracle.reduce("long: const int *k", "k[i] % 7 == 3", "a+b", "0", n, [k])
    expected = 0 if n < 4 else (n - 4) // 7 + 1
    assert r.value == expected
    if n < 200:
        assert r.value == sum(1 for v in range(n) if v % 7 == 3)


def test_geometric_series():
    r, n = 0.999, 1000
    # stored terms: the float32 rounding of r**k (float64 power, error ~1e-16)
    q = np.array([np.float32(r ** k) for k in range(n)], dtype=np.float32)
    res = oracle.reduce("double: const float *q", "q[i]", "a+b", "0", n, [q])
    closed = (1 - r ** n) / (1 - r)
    tol = (2.0 ** -24 + 1e-12) * closed          # one float32 rounding per stored term
    assert abs(res.value - closed) <= tol
    # a dropped first term (1.0), a dropped last term (r**999 ~ 0.368) and an
    # index shifted by one (sum over k = 1..n) all move the sum by more than tol
    assert abs(res.value - (closed - 1.0)) > tol
    assert abs(res.value - (closed - r ** (n - 1))) > tol
    assert abs(res.value - (r * closed)) > tol


@pytest.mark.parametrize("a_bits,b_bits,k", [(1, 2, 10), (5, 12, 14), (3, 3, 12), (0, 7, 9)])
def test_walsh_vectors_dot(a_bits, b_bits, k):
    n = 1 << k
    idx = np.arange(n)
    pop = np.vectorize(lambda v: bin(v).count("1"))
    x = np.where(pop(idx & a_bits) % 2, -1.0, 1.0).astype(np.float32)
    y = np.where(pop(idx & b_bits) % 2, -1.0, 1.0).astype(np.float32)
    r = oracle.reduce("float: const float *x, const float *y", "x[i]*y[i]", "a+b", "0", n, [x, y])
    assert r.value == (n if a_bits == b_bits else 0)
    assert r.abs_sum == pytest.approx(n)


def test_max_min_of_arange():
    n = 1000
    a = np.arange(n, dtype=np.float32)
    assert oracle.reduce("float: const float *x", "x[i]", "max", "-INFINITY", n, [a]).value == n - 1
    assert oracle.reduce("float: const float *x", "x[i]", "min(a,b)", "INFINITY", n, [a]).value == 0
    rev = a[::-1].copy()
    assert oracle.reduce("float: const float *x", "x[i]", "max(b,a)", "-INFINITY", n, [rev]).value == n - 1
    k = np.arange(-5, 5, dtype=np.int32)
    assert oracle.reduce("int: const int *k", "k[i]", "max", "INT_MIN", 10, [k]).value == 4
    assert oracle.reduce("int: const int *k", "k[i]", "min", "INT_MAX", 10, [k]).value == -5


def test_neutral_for_empty_input():
    z = np.zeros(0, np.float32)
    assert oracle.reduce("float: const float *x", "x[i]", "a+b", "0", 0, [z]).value == 0
    assert oracle.reduce("float: const float *x", "x[i]", "max", "-INFINITY", 0, [z]).value == -math.inf
    zi = np.zeros(0, np.int32)
    assert oracle.reduce("int: const int *k", "k[i]", "min", "INT_MAX", 0, [zi]).value == 2 ** 31 - 1
    assert oracle.reduce("int: const int *k", "k[i]", "a|b", "0", 0, [zi]).value == 0


def test_ieee_maximum_nan_and_signed_zero():
    x = np.array([-0.0, 0.0, -0.0], np.float32)
    assert math.copysign(1, oracle.reduce("float: const float *x", "x[i]", "max", "-INFINITY",
                                          3, [x]).value) == 1
    assert math.copysign(1, oracle.reduce("float: const float *x", "x[i]", "min", "INFINITY",
                                          3, [x]).value) == -1
    x = np.array([1.0, np.nan, 3.0], np.float32)
    assert math.isnan(oracle.reduce("float: const float *x", "x[i]", "max", "-INFINITY", 3, [x]).value)


# ------------------------------------------------------------ brute force
@pytest.mark.parametrize("seed", range(6))
def test_float_sum_is_the_correctly_rounded_exact_sum(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(0, 60))
    x = (rng.standard_normal(n) * 10.0 ** rng.integers(-8, 8, n)).astype(np.float32)
    y = (rng.standard_normal(n) * 10.0 ** rng.integers(-8, 8, n)).astype(np.float32)
    r = oracle.reduce("double: const float *x, const float *y", "x[i]*y[i]", "a+b", "0", n, [x, y])
    exact = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    assert r.value == float(exact)
    assert r.abs_sum >= float(abs(exact))


@pytest.mark.parametrize("seed", range(4))
def test_float_sum_permutation_invariant(seed):
    rng = np.random.default_rng(seed)
    n = 5000
    x = (rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))).astype(np.float32)
    p = rng.permutation(n)
    sig = "float: const float *x"
    a = oracle.reduce(sig, "x[i]", "a+b", "0", n, [x]).value
    b = oracle.reduce(sig, "x[i]", "a+b", "0", n, [x[p]]).value
    assert a == b
    k = rng.integers(-1000, 1000, n).astype(np.int32)
    s1 = oracle.reduce("long: const int *k", "k[i]*k[i] - 3", "a+b", "0", n, [k]).value
    s2 = oracle.reduce("long: const int *k", "k[i]*k[i] - 3", "a+b", "0", n, [k[p]]).value
    assert s1 == s2 == int(np.sum(k.astype(np.int64) ** 2)) - 3 * n


def _py_c_div(a, b):
    q = abs(a) // abs(b)
    return q if (a < 0) == (b < 0) else -q


def test_integer_c_semantics_brute_force():
    vals = np.array([-9, -7, -2, -1, 1, 2, 3, 7, 9], np.int32)
    a = np.repeat(vals, len(vals))
    b = np.tile(vals, len(vals))
    q = np.zeros_like(a)
    o = oracle.elementwise("const int *a, const int *b, int *q", "q[i] = a[i] / b[i]",
                           len(a), [a, b, q])["q"]
    assert o.v.tolist() == [_py_c_div(int(x), int(y)) for x, y in zip(a, b)]
    o = oracle.elementwise("const int *a, const int *b, int *q", "q[i] = a[i] % b[i]",
                           len(a), [a, b, q])["q"]
    assert o.v.tolist() == [int(x) - _py_c_div(int(x), int(y)) * int(y) for x, y in zip(a, b)]


def test_c_conversions_and_promotions():
    k = np.array([0, 1, 200, -1], np.int32)
    out = np.zeros(4, np.int64)
    ev = lambda stmt: oracle.elementwise("const int *k, long *o", stmt, 4, [k, out])["o"].v.tolist()
    assert ev("o[i] = (unsigned)k[i]") == [0, 1, 200, 2 ** 32 - 1]
    assert ev("o[i] = (char)k[i]") == [0, 1, -56, -1]
    assert ev("o[i] = (unsigned char)k[i]") == [0, 1, 200, 255]
    assert ev("o[i] = k[i] < 0u") == [0, 0, 0, 0]            # -1 converts to UINT_MAX
    assert ev("o[i] = k[i] < 0") == [0, 0, 0, 1]
    assert ev("o[i] = 0u - 1") == [2 ** 32 - 1] * 4
    assert ev("o[i] = k[i] > 0 ? k[i] : -k[i]") == [0, 1, 200, 1]
    assert ev("o[i] = (k[i] != 0) && (10 / k[i] > 2)") == [0, 1, 0, 0]
    assert ev("o[i] = k[i] == 0 || 10 % k[i] == 0") == [1, 1, 0, 1]
    assert ev("o[i] = 7 >> 1 << 2") == [12] * 4
    assert ev("o[i] = ~k[i] & 0xff") == [255, 254, 55, 0]
    assert ev("o[i] = (long)k[i] * 3000000000") == [0, 3000000000, 600000000000, -3000000000]
    assert ev("o[i] = (int)(2.75f * k[i])") == [0, 2, 550, -2]
    assert ev("o[i] = max(k[i], 5) + min(k[i], -3)") == [2, 2, 197, 2]


def test_signed_overflow_is_not_given_a_value():
    k = np.array([2 ** 30], np.int32)
    out = np.zeros(1, np.int32)
    with pytest.raises(OracleError):
        oracle.elementwise("const int *k, int *o", "o[i] = k[i] * 4", 1, [k, out])
    with pytest.raises(OracleError):
        oracle.elementwise("const int *k, int *o", "o[i] = k[i] / (k[i] - k[i])", 1, [k, out])
    with pytest.raises(OracleError):
        oracle.elementwise("const int *k, int *o", "o[i] = k[i + 1]", 1, [k, out])
    # the unselected branch of ?: may divide by zero
    o = oracle.elementwise("const int *k, int *o", "o[i] = k[i] - k[i] != 0 ? 1 / (k[i] - k[i]) : 7",
                           1, [k, out])["o"]
    assert o.v.tolist() == [7]


def test_float_literals_round_once():
    assert oracle.f32_literal(Fraction("0.1")) == float(np.float32(0.1))
    # just above the midpoint between 1 and 1 + 2**-23: double rounding would give 1
    q = Fraction(1) + Fraction(2) ** -24 + Fraction(1, 10 ** 30)
    assert oracle.f32_literal(q) == 1 + 2.0 ** -23
    assert float(np.float32(float(q))) == 1.0
    assert oracle.f32_literal(Fraction(2) ** -149) == 2.0 ** -149
    assert oracle.f32_literal(Fraction(2) ** -151) == 0.0
    assert oracle.f32_literal(Fraction(3) * Fraction(2) ** -151) == 2.0 ** -149
    assert oracle.f32_literal(Fraction(2) ** 128) == math.inf
    rng = np.random.default_rng(9)
    for v in rng.standard_normal(200) * 10.0 ** rng.integers(-30, 30, 200):
        assert oracle.f32_literal(Fraction(float(v))) == float(np.float32(v))


# ------------------------------------------------------------ error bounds
@pytest.mark.parametrize("stmt,f32", [
    ("z[i] = 2.5f*x[i] - 0.5f*y[i]", lambda x, y: np.float32(2.5) * x - np.float32(0.5) * y),
    ("z[i] = sqrtf(x[i]*x[i] + y[i]*y[i])", lambda x, y: np.sqrt(x * x + y * y)),
    ("z[i] = (x[i] - y[i]) / (1.5f + x[i]*y[i])", lambda x, y: (x - y) / (np.float32(1.5) + x * y)),
    ("z[i] = expf(x[i]) * logf(2.0f + y[i])", lambda x, y: np.exp(x) * np.log(np.float32(2) + y)),
    ("float t = x[i] + y[i]; z[i] = t*t - fabsf(x[i])",
     lambda x, y: (x + y) * (x + y) - np.abs(x)),
])
def test_error_bound_contains_float32_evaluations(stmt, f32):
    rng = np.random.default_rng(5)
    n = 20000
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    z = np.zeros(n, np.float32)
    o = oracle.elementwise("float *z, const float *x, const float *y", stmt, n, [z, x, y])["z"]
    with np.errstate(all="ignore"):
        g = f32(x, y).astype(np.float32)
    assert not np.any(o.u)
    assert np.all(np.abs(g.astype(np.float64) - o.v) <= o.e)
    # the exact value sits inside the bound as well, and the bound is tight-ish
    assert np.median(o.e / np.maximum(np.abs(o.v), 1e-30)) < 1e-5


def test_unsure_lanes_flag_rounding_sensitive_comparisons():
    x = np.array([1.0 / 3.0, 0.25, 0.4], np.float32)
    z = np.zeros(3, np.int32)
    o = oracle.elementwise("const float *x, int *z", "z[i] = x[i] * 3.0f >= 1.0f", 3, [x, z])["z"]
    assert o.u.tolist() == [True, False, False]
    assert o.v.tolist()[1:] == [0, 1]


def test_if_else_blocks_and_locals():
    x = np.array([0.2, 0.7, -1.0], np.float32)
    z = np.zeros(3, np.float32)
    o = oracle.elementwise("const float *x, float *z",
                           "if (x[i] > 0.5f) { float t = x[i]*2; z[i] = t; } else z[i] = -1; z[i] += 1",
                           3, [x, z])["z"]
    assert o.v.tolist() == [0.0, float(np.float32(0.7)) * 2 + 1, 0.0]


# ------------------------------------------------------------ generic folds
def test_generic_integer_folds_match_python():
    rng = np.random.default_rng(3)
    k = rng.integers(0, 2 ** 31 - 1, 3000).astype(np.int32)
    sig = "int: const int *k"
    assert oracle.reduce(sig, "k[i]", "a|b", "0", 3000, [k]).value == functools.reduce(operator.or_, k.tolist(), 0)
    assert oracle.reduce(sig, "k[i]", "a^b", "0", 3000, [k]).value == functools.reduce(operator.xor, k.tolist(), 0)
    u = rng.integers(0, 2 ** 32, 500).astype(np.uint32)
    prod = functools.reduce(lambda a, b: a * b % 2 ** 32, u.tolist(), 1)
    assert oracle.reduce("unsigned: const unsigned *u", "u[i]", "a*b", "1u", 500, [u]).value == prod


def test_int32_result_overflow_has_no_value():
    k = np.full(3, 2 ** 30, np.int32)
    with pytest.raises(OracleError):
        oracle.reduce("int: const int *k", "k[i]", "a+b", "0", 3, [k])
    assert oracle.reduce("long: const int *k", "k[i]", "a+b", "0", 3, [k]).value == 3 * 2 ** 30


# ------------------------------------------------------------ formats
def test_decoders_match_torch_for_every_code():
    torch = pytest.importorskip("torch")
    b16 = np.arange(1 << 16, dtype=np.uint16)
    ref = torch.from_numpy(b16.view(np.int16)).view(torch.bfloat16).double().numpy()
    assert np.array_equal(oracle.decode_bf16(b16), ref, equal_nan=True)
    ref = torch.from_numpy(b16.view(np.int16)).view(torch.float16).double().numpy()
    assert np.array_equal(oracle.decode_f16(b16), ref, equal_nan=True)
    b8 = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(b8).view(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(oracle.decode_e4m3fn(b8), ref, equal_nan=True)


def test_e4m3_format_landmarks():
    d = oracle.decode_e4m3fn(np.array([0x7E, 0x7F, 0x01, 0x08, 0x38, 0xFE], np.uint8))
    assert d[0] == 448.0 and math.isnan(d[1]) and d[2] == 2.0 ** -9
    assert d[3] == 2.0 ** -6 and d[4] == 1.0 and d[5] == -448.0


def test_low_precision_sums_exact_in_fixed_point():
    import workloads
    v = workloads.precision_values(1 << 16, "lognormal")
    for fmt, shift in (("fp8_e4m3", 9), ("float16", 24)):
        q = workloads.quantize(fmt, v)
        dec = oracle.decode_e4m3fn(q.bits) if fmt == "fp8_e4m3" else oracle.decode_f16(q.bits)
        ints = [int(x * 2 ** shift) for x in dec.tolist()]
        assert all(i == x * 2 ** shift for i, x in zip(ints, dec.tolist()))
        exact = Fraction(sum(ints), 2 ** shift)
        sig = f"double: const {fmt} *x"
        r = oracle.reduce(sig, "x[i]", "a+b", "0", len(dec), [q.bits])
        assert r.value == float(exact)
        sq = Fraction(sum(i * i for i in ints), 2 ** (2 * shift))
        nrm = oracle.norm2(dec)
        # sqrt of a correctly rounded sum: within one ulp of the exact root
        exact_root = math.sqrt(float(sq))
        assert abs(nrm - exact_root) <= 2 * math.ulp(exact_root)
    q = workloads.quantize("bfloat16", v)
    dec = oracle.decode_bf16(q.bits)
    assert np.all((np.abs(dec) >= 2.0 ** -40) & (np.abs(dec) <= 2.0 ** 40))
    exact = Fraction(sum(int(x * 2 ** 47) for x in dec.tolist()), 2 ** 47)
    r = oracle.reduce("double: const bfloat16 *x", "x[i]", "a+b", "0", len(dec), [q.bits])
    assert r.value == float(exact)


def test_norm2_pythagorean():
    assert oracle.norm2([3.0, 4.0]) == 5.0
    assert oracle.norm2([2.0, 3.0, 6.0]) == 7.0
    assert oracle.norm2([]) == 0.0


# ------------------------------------------------------------ signature
def test_signature_parser():
    s = oracle.parse_signature("long: const int *k, float a, __hip_bfloat16 *x, unsigned char *u")
    assert s.result == "int64"
    assert [(a.name, a.storage, a.pointer, a.const) for a in s.args] == [
        ("k", "int32", True, True), ("a", "float32", False, False),
        ("x", "bfloat16", True, False), ("u", "uint8", True, False)]
    assert oracle.parse_signature("float *z").result is None
    with pytest.raises(ValueError):
        oracle.parse_signature("quux *z")
    with pytest.raises(ValueError):
        oracle.parse_signature("float *z, int z")


# ------------------------------------------------------------ library cross-checks
def test_library_cross_checks_on_the_small_dot_inputs():
    # the small dot's inputs (2^20 float32 values, seed 0): the oracle's dot
    # is Python's correctly rounded fsum of the exact float64 products; its
    # max is numpy's; its sum and norm agree with torch's float64 reductions
    # to within float64 rounding
    import workloads
    torch = pytest.importorskip("torch")
    x, y = workloads.dot_1m()
    n = x.size
    r = oracle.reduce("float: const float *x, const float *y", "x[i]*y[i]", "a+b", "0", n, [x, y])
    assert r.value == math.fsum((x.astype(np.float64) * y.astype(np.float64)).tolist())
    m = oracle.reduce("float: const float *x", "x[i]", "max(a,b)", "-INFINITY", n, [x])
    assert m.value == float(np.max(x))
    s = oracle.reduce("double: const float *x", "x[i]", "a+b", "0", n, [x]).value
    t = torch.from_numpy(x).double()
    assert abs(s - float(torch.sum(t))) <= 1e-12 * float(torch.sum(t.abs()))
    # (torch's float64 reductions are not correctly rounded: allow their
    # summation error, far below what a dropped or doubled term would move)
    nrm = oracle.norm2(x)
    assert abs(nrm - float(torch.linalg.vector_norm(t))) <= 1e-12 * nrm
