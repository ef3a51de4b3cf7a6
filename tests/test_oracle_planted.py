"""Planted mistakes, on the CPU: each patches one plausible bug into the
oracle (a dropped term, C division taken as floor division, a transposed
operand, a missing rounding allowance, a lost sign bit, a naive float sum)
and checks that the pins catch it.  The GPU library is never involved."""

import math
import sys

import numpy as np
import pytest

import oracle
import oracle.interp as interp
import test_oracle_pins as pins

REDUCE_MOD = sys.modules["oracle.reduce"]


def caught(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_dropped_last_term(monkeypatch):
    real = oracle.reduce

    def planted(sig, mp, comb, neu, n, args, *a, **kw):
        return real(sig, mp, comb, neu, max(n - 1, 0), args, *a, **kw)
    monkeypatch.setattr(oracle, "reduce", planted)
    assert caught(pins.test_sum_of_index_closed_form)
    assert caught(pins.test_listing3b_dot_of_arange)
    assert caught(pins.test_count_mod7_closed_form, 46)       # element 45 counts (45 % 7 == 3)


def test_floor_division_instead_of_c_truncation(monkeypatch):
    real = interp.Interp._int_arith

    def planted(self, op, a, b, t, u, active):
        if op in ("/", "%"):
            ys = np.where(b.v == 0, 1, b.v)
            return self._int_result(t, a.v // ys if op == "/" else a.v % ys, u, active)
        return real(self, op, a, b, t, u, active)
    monkeypatch.setattr(interp.Interp, "_int_arith", planted)
    assert caught(pins.test_integer_c_semantics_brute_force)


def test_transposed_subtraction(monkeypatch):
    real = interp.Interp._float_arith

    def planted(self, op, a, b, t, u, active):
        if op == "-":
            a, b = b, a
        return real(self, op, a, b, t, u, active)
    monkeypatch.setattr(interp.Interp, "_float_arith", planted)
    stmt, f32 = "z[i] = 2.5f*x[i] - 0.5f*y[i]", lambda x, y: np.float32(2.5) * x - np.float32(0.5) * y
    assert caught(pins.test_error_bound_contains_float32_evaluations, stmt, f32)


def test_missing_rounding_allowance(monkeypatch):
    monkeypatch.setattr(interp, "UNIT", {k: 0.0 for k in interp.UNIT})
    stmt, f32 = "z[i] = sqrtf(x[i]*x[i] + y[i]*y[i])", lambda x, y: np.sqrt(x * x + y * y)
    assert caught(pins.test_error_bound_contains_float32_evaluations, stmt, f32)


def test_lost_sign_bit_in_a_decoder(monkeypatch):
    pytest.importorskip("torch")
    real = oracle.decode_bf16
    monkeypatch.setattr(oracle, "decode_bf16", lambda bits: np.abs(real(bits)))
    assert caught(pins.test_decoders_match_torch_for_every_code)


def test_naive_float_sum(monkeypatch):
    class NaiveMath:
        sqrt = staticmethod(math.sqrt)
        isnan = staticmethod(math.isnan)
        isinf = staticmethod(math.isinf)
        inf = math.inf

        @staticmethod
        def fsum(values):
            s = 0.0
            for v in values:
                s += v
            return s
    monkeypatch.setattr(REDUCE_MOD, "math", NaiveMath)
    assert any(caught(pins.test_float_sum_is_the_correctly_rounded_exact_sum, seed)
               for seed in range(6))


def test_exclusive_scan_not_shifted(monkeypatch):
    import test_oracle_scan_pins as scan_pins
    real = oracle.scan
    monkeypatch.setattr(oracle, "scan", lambda *a, exclusive=False, **kw: real(*a, **kw))
    assert caught(scan_pins.test_inclusive_and_exclusive_sum_of_index_closed_form)


def test_periodic_stencil_boundary(monkeypatch):
    # the five-point operator with wrap-around neighbours instead of the
    # Dirichlet boundary
    import test_oracle_cg_pins as cg_pins

    def planted(p, nx):
        g = np.asarray(p, np.float64).reshape(-1, nx)
        return (4 * g - np.roll(g, 1, 0) - np.roll(g, -1, 0) - np.roll(g, 1, 1)
                - np.roll(g, -1, 1)).reshape(-1)
    monkeypatch.setattr(oracle, "laplace5", planted)
    assert caught(cg_pins.test_operator_is_scipys_sparse_laplacian, 7, 5)


def test_cg_with_a_scaled_operator(monkeypatch):
    # a dropped factor inside the solver's operator (2A instead of A)
    import test_oracle_cg_pins as cg_pins
    mod = sys.modules["oracle.cg"]
    real = mod.laplace5
    monkeypatch.setattr(mod, "laplace5", lambda p, nx: 2.0 * real(p, nx))
    assert caught(cg_pins.test_cg_reaches_the_direct_solution)


def test_conj_that_does_not_conjugate(monkeypatch):
    import test_oracle_complex_pins as complex_pins
    real = interp.Interp._complex_call

    def planted(self, f, args, active):
        if f == "conj":
            return self.convert(args[0], interp.CFLOAT, active)
        return real(self, f, args, active)
    monkeypatch.setattr(interp.Interp, "_complex_call", planted)
    assert caught(complex_pins.test_conjugated_dot_is_the_exact_sum)
    assert caught(complex_pins.test_gaussian_integer_products_are_exact)


def test_generic_fold_bound_dropped(monkeypatch):
    """The generic float fold's rounding allowance dropped (rounds = 0): the
    fold would claim to be exact, and float32 folds along real trees leave it."""
    import test_oracle_generic_fold as gf
    monkeypatch.setattr(REDUCE_MOD, "generic_float_model", lambda *a, **k: (0.0, 0.0))
    assert caught(gf.test_model_bounds_float32_folds_in_every_tree, "(a)+(b)", gf.PLUS, "uniform")
    assert caught(gf.test_rounds_per_combination)


def test_generic_fold_bound_too_small(monkeypatch):
    """A bound four times too small (rounds / 4) is caught by the one-sided
    rounding sequence that uses half of the true bound."""
    import test_oracle_generic_fold as gf
    real = REDUCE_MOD.generic_float_model

    def planted(*a, **k):
        rounds, slack = real(*a, **k)
        return rounds / 4, slack
    monkeypatch.setattr(REDUCE_MOD, "generic_float_model", planted)
    assert caught(gf.test_model_bound_is_not_vacuous)


def test_generic_fold_last_term_dropped(monkeypatch):
    """A generic fold that skips its last map value is caught by the pin that
    holds the fold to the correctly rounded sum."""
    import test_oracle_generic_fold as gf
    real = REDUCE_MOD.generic_prefix

    def planted(storage, rt, combine, neutral, m):
        p = real(storage, rt, combine, neutral, m[:-1])
        return np.append(p, p[-1:]) if m.size else p
    monkeypatch.setattr(REDUCE_MOD, "generic_prefix", planted)
    assert caught(gf.test_sum_like_value_is_the_correctly_rounded_sum, "(a)+(b)")
