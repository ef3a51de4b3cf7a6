"""Pins of the oracle's folds under a generic reduce expression with a
floating result (section "Map-Reduce": any C reduce expression in a and b
with its neutral element).  The oracle's value is a float64 left-to-right
fold; its error model bounds every float32 evaluation order of the fold by
rounds * u * D * sum |m| (D the depth of the fold tree).  These pins hold it
against what the mathematics fixes: the correctly rounded sum, numpy's
maximum, and actual float32 folds along many tree shapes, evaluated here in
numpy float32 (one rounding per C operation, as the device does)."""

import math

import numpy as np
import pytest

import oracle
from oracle.interp import OracleError

U = 2.0 ** -24
SIG = "float: const float *x"


def data(n, seed, kind="uniform"):
    rng = np.random.default_rng(seed)
    if kind == "positive":
        return rng.uniform(0.5, 1.0, n).astype(np.float32)
    if kind == "wide":
        return (rng.lognormal(0, 3, n) * rng.choice([-1, 1], n)).astype(np.float32)
    return rng.uniform(-1, 1, n).astype(np.float32)


# ----------------------------------------------------------- tree folds in float32
def fold_tree(vals, f, shape, rng=None):
    """Folds float32 values along a tree; returns (value, depth): depth is the
    largest number of combinations on one value's path."""
    items = [(np.float32(v), 0) for v in vals]
    if shape == "sequential":
        acc, d = items[0]
        for v, dv in items[1:]:
            acc, d = f(acc, v), max(d, dv) + 1
        return acc, d
    if shape == "pairwise":
        while len(items) > 1:
            nxt = [(f(a, b), max(da, db) + 1) for (a, da), (b, db) in zip(items[0::2], items[1::2])]
            if len(items) % 2:
                nxt.append(items[-1])
            items = nxt
        return items[0]
    if shape == "strided":          # lanes fold every 64th value, then a butterfly-like tree
        lanes = [fold_tree(vals[j::64], f, "sequential") for j in range(min(64, len(vals)))]
        vals2 = [v for v, _ in lanes]
        top, dtop = fold_tree(vals2, f, "pairwise")
        return top, dtop + max(d for _, d in lanes)
    # random: repeatedly combine two random items
    while len(items) > 1:
        i, j = sorted(rng.choice(len(items), 2, replace=False))
        (a, da), (b, db) = items[i], items.pop(j)
        items[i] = (f(a, b), max(da, db) + 1)
    return items[0]


PLUS = lambda a, b: np.float32(a + b)                           # noqa: E731
PLUS0 = lambda a, b: np.float32(np.float32(a + b) + np.float32(0.0))   # noqa: E731
FMAX = lambda a, b: np.float32(np.fmax(a, b))                   # noqa: E731


# ----------------------------------------------------------- value pins
@pytest.mark.parametrize("combine", ["(a)+(b)", "a+b+0.0f", "b + (a)"])
def test_sum_like_value_is_the_correctly_rounded_sum(combine):
    x = data(3000, 1)
    r = oracle.reduce(SIG, "x[i]", combine, "0", x.size, [x])
    exact = math.fsum(x.astype(np.float64).tolist())
    # the float64 left-to-right evaluation: at most n float64 roundings
    assert abs(r.value - exact) <= x.size * 2.0 ** -53 * r.abs_sum
    assert r.op == "generic" and not r.exact
    assert r.abs_sum == pytest.approx(float(np.sum(np.abs(x.astype(np.float64)))), rel=1e-9)


def test_rounds_per_combination():
    x = data(500, 2)
    assert oracle.reduce(SIG, "x[i]", "(a)+(b)", "0", x.size, [x]).rounds == pytest.approx(1, abs=1e-6)
    assert oracle.reduce(SIG, "x[i]", "a+b+0.0f", "0", x.size, [x]).rounds == pytest.approx(2, abs=1e-6)
    assert oracle.reduce(SIG, "x[i]", "fmaxf(a,b)", "-INFINITY", x.size, [x]).rounds == 0.0


@pytest.mark.parametrize("combine,neutral,fn", [("fmaxf(a,b)", "-INFINITY", np.max),
                                                ("a > b ? a : b", "-INFINITY", np.max),
                                                ("fminf(a,b)", "INFINITY", np.min),
                                                ("a < b ? a : b", "INFINITY", np.min)])
def test_selections_are_exact_and_equal_numpy(combine, neutral, fn):
    for seed, kind in ((3, "uniform"), (4, "wide")):
        x = data(4000, seed, kind)
        r = oracle.reduce(SIG, "x[i]", combine, neutral, x.size, [x])
        assert r.exact and r.rounds == 0.0 and r.abs_slack == 0.0
        assert r.value == float(fn(x))


def test_empty_fold_is_the_neutral_element():
    r = oracle.reduce(SIG, "x[i]", "fmaxf(a,b)", "-INFINITY", 0, [np.zeros(0, np.float32)])
    assert r.value == -math.inf and r.exact
    r = oracle.reduce(SIG, "x[i]", "(a)+(b)", "0", 0, [np.zeros(0, np.float32)])
    assert r.value == 0.0


# ----------------------------------------------------------- the error model
@pytest.mark.parametrize("combine,f", [("(a)+(b)", PLUS), ("a+b+0.0f", PLUS0)])
@pytest.mark.parametrize("kind", ["uniform", "positive", "wide"])
def test_model_bounds_float32_folds_in_every_tree(combine, f, kind):
    """Brute force of the bound: float32 folds along sequential, pairwise,
    lane-strided and random trees all stay within rounds * u * D * sum|m|
    of the oracle's value, D being each tree's own depth."""
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 64, 333, 1500):
        x = data(n, 100 + n, kind)
        r = oracle.reduce(SIG, "x[i]", combine, "0", n, [x])
        for shape in ("sequential", "pairwise", "strided", "random"):
            g, depth = fold_tree([0.0] + x.tolist(), f, shape, rng)   # the neutral is a leaf
            bound = r.rounds * U * depth * r.abs_sum + r.err_sum + r.abs_slack
            assert abs(float(g) - r.value) <= bound, (combine, kind, n, shape)


def test_model_bound_is_not_vacuous():
    """Rounding errors that all point one way: 1 followed by values of 3/4 of
    an ulp of 1, so that every float32 addition rounds up by a quarter ulp.
    The sequential fold then uses about half of the bound, so a bound a few
    times smaller would fail."""
    x = np.array([1.0] + [0.75 * 2.0 ** -23] * 1000, dtype=np.float32)
    r = oracle.reduce(SIG, "x[i]", "(a)+(b)", "0", x.size, [x])
    g, depth = fold_tree([0.0] + x.tolist(), PLUS, "sequential")
    used = abs(float(g) - r.value) / (r.rounds * U * depth * r.abs_sum + r.err_sum)
    assert 0.4 < used <= 1.0


def test_selection_folds_equal_in_every_tree():
    rng = np.random.default_rng(7)
    x = data(777, 8, "wide")
    r = oracle.reduce(SIG, "x[i]", "fmaxf(a,b)", "-INFINITY", x.size, [x])
    for shape in ("sequential", "pairwise", "strided", "random"):
        g, _ = fold_tree([-np.inf] + x.tolist(), FMAX, shape, rng)
        assert float(g) == r.value


def test_scan_prefixes_follow_the_model():
    x = data(400, 9, "positive")
    r = oracle.scan(SIG, "x[i]", "(a)+(b)", "0", x.size, [x])
    seq = np.cumsum(x, dtype=np.float32)            # float32 left-to-right prefixes
    depth = np.arange(1, x.size + 1) + 1            # the neutral is combined first
    bound = r.rounds * U * depth * r.abs_prefix + r.err_prefix + r.abs_slack
    assert np.all(np.abs(seq.astype(np.float64) - r.values) <= bound)
    exact = np.array([math.fsum(x[:k + 1].astype(np.float64).tolist()) for k in range(x.size)])
    assert np.all(np.abs(r.values - exact) <= (x.size + 1) * 2.0 ** -53 * r.abs_prefix)
    m = oracle.scan(SIG, "x[i]", "fmaxf(a,b)", "-INFINITY", x.size, [x])
    assert m.exact and np.array_equal(m.values, np.maximum.accumulate(x.astype(np.float64)))


# ----------------------------------------------------------- outside the model
def test_non_identity_neutral_is_refused():
    x = data(50, 10)
    with pytest.raises(OracleError, match="identity"):
        oracle.reduce(SIG, "x[i]", "(a)+(b)", "1", x.size, [x])


def test_expansive_combine_is_refused():
    x = data(50, 11, "wide")               # |x| well above 1: a product amplifies errors
    with pytest.raises(OracleError, match="amplifies"):
        oracle.reduce(SIG, "x[i]", "a*b", "1", x.size, [x])


def test_growing_combine_is_refused():
    x = data(50, 12, "positive")
    with pytest.raises(OracleError):
        oracle.reduce(SIG, "x[i]", "a+b+a*b*0.5f", "0", x.size, [x])
