"""Pins of the oracle's complex arithmetic (section "Complex Numbers on the
GPU": complex values with float components inside kernels): Gaussian
integer products exact, the conjugated dot equal to an exactly summed
reference and to numpy's vdot, |z|^2 = z conj(z), the error bound containing
complex64 (float32-component) evaluations, and the conversions C++ allows."""

import math

import numpy as np
import pytest

import oracle
from oracle import CSyntaxError, OracleError

SIG = "complex64 *z, const complex64 *x, const complex64 *y"


def test_gaussian_integer_products_are_exact():
    rng = np.random.default_rng(0)
    a = rng.integers(-50, 50, (2, 500))
    b = rng.integers(-50, 50, (2, 500))
    x = (a[0] + 1j * a[1]).astype(np.complex64)
    y = (b[0] + 1j * b[1]).astype(np.complex64)
    r = oracle.elementwise(SIG, "z[i] = x[i] * y[i] - conj(y[i])", 500,
                           [np.zeros(500, np.complex64), x, y])
    want = [complex(p) * complex(q) - complex(q).conjugate() for p, q in zip(x.tolist(), y.tolist())]
    assert r["z"].v.tolist() == want


def test_conjugated_dot_is_the_exact_sum():
    rng = np.random.default_rng(1)
    n = 3000
    x = (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)).astype(np.complex64)
    y = (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)).astype(np.complex64)
    r = oracle.reduce("complex64: const complex64 *x, const complex64 *y", "conj(x[i]) * y[i]",
                      "a+b", "0", n, [x, y])
    # products of float32 components are exact in float64: sum each part exactly
    xr, xi = x.real.astype(np.float64), x.imag.astype(np.float64)
    yr, yi = y.real.astype(np.float64), y.imag.astype(np.float64)
    re = math.fsum((xr * yr).tolist() + (xi * yi).tolist())
    im = math.fsum((xr * yi).tolist() + (-xi * yr).tolist())
    assert r.value == complex(re, im)
    assert abs(r.value - np.vdot(x.astype(np.complex128), y.astype(np.complex128))) < 1e-12 * r.abs_sum
    assert r.abs_sum == pytest.approx(float(np.sum(np.abs(np.conj(x.astype(np.complex128)) * y))), rel=1e-9)


def test_norm_squared_is_real():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(200) + 1j * rng.standard_normal(200)).astype(np.complex64)
    r = oracle.elementwise("complex64 *z, const complex64 *x, const complex64 *y", "z[i] = x[i] * conj(x[i])",
                           200, [np.zeros(200, np.complex64), x, x])
    assert np.all(r["z"].v.imag == 0)
    assert np.allclose(r["z"].v.real, np.abs(x.astype(np.complex128)) ** 2, rtol=1e-15)
    f = oracle.elementwise("float *w, const complex64 *x", "w[i] = abs(x[i]) + real(x[i]) - imag(x[i])",
                           200, [np.zeros(200, np.float32), x])
    xv = x.astype(np.complex128)
    assert np.allclose(f["w"].v, np.abs(xv) + xv.real - xv.imag, rtol=1e-14)


@pytest.mark.parametrize("stmt", ["z[i] = x[i] * y[i] + x[i]", "z[i] = 2.5f * x[i] - y[i] * conj(x[i])",
                                  "z[i] = (x[i] + y[i]) * (x[i] - y[i])"])
def test_error_bound_contains_complex64_evaluations(stmt):
    rng = np.random.default_rng(3)
    n = 20000
    x = (rng.uniform(-2, 2, n) + 1j * rng.uniform(-2, 2, n)).astype(np.complex64)
    y = (rng.uniform(-2, 2, n) + 1j * rng.uniform(-2, 2, n)).astype(np.complex64)
    r = oracle.elementwise(SIG, stmt, n, [np.zeros(n, np.complex64), x, y])
    # evaluate in complex64 (float32 components) with numpy
    with np.errstate(all="ignore"):
        env = {"x": x, "y": y, "conj": np.conj}
        expr = stmt.split("=", 1)[1].replace("[i]", "").replace("2.5f", "np.float32(2.5)")
        f32 = eval(expr, {"np": np}, env).astype(np.complex64)
    err = np.abs(f32.astype(np.complex128) - r["z"].v)
    assert np.all(err <= r["z"].e), stmt
    assert np.median(r["z"].e) < 1e-5                   # not vacuous


def test_conversions_and_unsupported_operations():
    x = np.array([1 + 1j], np.complex64)
    with pytest.raises(CSyntaxError):      # complex -> float needs real()/imag()/abs()
        oracle.elementwise("float *w, const complex64 *x", "w[i] = x[i]", 1, [np.zeros(1, np.float32), x])
    with pytest.raises(CSyntaxError):
        oracle.elementwise(SIG, "z[i] = x[i] / y[i]", 1, [np.zeros(1, np.complex64), x, x])
    with pytest.raises(OracleError):
        oracle.reduce("complex64: const complex64 *x", "x[i]", "max(a,b)", "0", 1, [x])
    r = oracle.elementwise(SIG, "z[i] = 3 + x[i]", 1, [np.zeros(1, np.complex64), x, x])
    assert r["z"].v.tolist() == [4 + 1j]


def test_complex_prefix_scan_is_fsum_per_part():
    rng = np.random.default_rng(4)
    n = 300
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    r = oracle.scan("complex64: const complex64 *x", "x[i]", "a+b", "0", n, [x])
    re, im = x.real.astype(np.float64).tolist(), x.imag.astype(np.float64).tolist()
    for k in range(0, n, 13):
        assert r.values[k] == complex(math.fsum(re[:k + 1]), math.fsum(im[:k + 1]))
