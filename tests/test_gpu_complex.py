"""GPU parity of complex values with float components (section "Complex
Numbers on the GPU") in generated kernels: elementwise complex arithmetic
with complex and real operands, the conjugated dot and complex sums, a
complex prefix scan, against the oracle."""

import numpy as np
import pytest

from gpu_util import assert_lanes, assert_reduce, dev_array, host_bits, need_gpu, reduce_on_gpu, torch
import oracle
import paper_1304_5553_amd as hm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def cdata(n, seed):
    rng = np.random.default_rng(seed)
    return [(rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)).astype(np.complex64) for _ in range(2)]


@pytest.mark.parametrize("offset", [0, 1])
def test_complex_elementwise(dev, offset):
    n = 100003
    x, y = cdata(n + 2, 1)
    sig = "complex64 *z, const complex64 *x, const complex64 *y, complex64 a"
    stmt = "z[i] = conj(x[i]) * y[i] + a * x[i] - 0.5f * y[i]"
    a = 0.75 - 1.25j
    k = hm.compile(stmt, sig, name="cplx_ew")
    assert k.vectorizable and k.vec == 2
    zd = torch.full((n + 2,), complex("nan+nanj"), dtype=torch.complex64, device=dev)
    xd, yd = dev_array(x), dev_array(y)
    hm.elementwise(k, n, [zd[offset:offset + n], xd[offset:offset + n], yd[offset:offset + n], a])
    torch.cuda.synchronize()
    ref = oracle.elementwise(sig, stmt, n, [np.zeros(n, np.complex64), x[offset:offset + n],
                                            y[offset:offset + n], np.complex64(a)])
    assert_lanes(zd[offset:offset + n], ref["z"], "complex64", what=f"complex ew offset {offset}")
    assert np.isnan(host_bits(zd)[offset + n])


def test_complex_to_real_functions(dev):
    n = 50001
    x, y = cdata(n, 2)
    r = np.random.default_rng(3).uniform(0, 2, n).astype(np.float32)
    sig = "float *w, const complex64 *x, const complex64 *y, const float *r"
    stmt = "w[i] = abs(x[i]) * r[i] + real(x[i] * y[i]) - imag(conj(y[i]))"
    k = hm.compile(stmt, sig, name="cplx_real")
    w = torch.empty(n, device=dev)
    hm.elementwise(k, n, [w, dev_array(x), dev_array(y), dev_array(r)])
    torch.cuda.synchronize()
    ref = oracle.elementwise(sig, stmt, n, [np.zeros(n, np.float32), x, y, r])
    assert_lanes(w, ref["w"], "float32", what="complex to real")


@pytest.mark.parametrize("n", [1, 7, 1000, 262147])
def test_conjugated_dot_and_sum(dev, n):
    x, y = cdata(n, n)
    sig = "complex64: const complex64 *x, const complex64 *y"
    xd, yd = dev_array(x), dev_array(y)
    for mp in ("conj(x[i]) * y[i]", "x[i] + 2.0f * y[i]"):
        k = hm.compile(mp, sig, name="cplx_red")
        out = reduce_on_gpu(k, "a+b", "0", n, [xd, yd])
        assert_reduce(out, oracle.reduce(sig, mp, "a+b", "0", n, [x, y]), f"{mp} n={n}")
    k = hm.compile("x[i]", sig, name="cplx_max")
    with pytest.raises(hm.UnsupportedError):
        reduce_on_gpu(k, "max(a,b)", "0", n, [xd, yd])


def test_complex_prefix_scan(dev):
    n = 70001
    x, y = cdata(n, 4)
    sig = "complex64: const complex64 *x, const complex64 *y"
    k = hm.compile("conj(x[i]) * y[i]", sig, name="cplx_scan")
    out = torch.empty(n, dtype=torch.complex64, device=dev)
    hm.scan(k, "a+b", "0", n, [dev_array(x), dev_array(y)], out)
    torch.cuda.synchronize()
    g = host_bits(out).astype(np.complex128)
    r = oracle.scan(sig, "conj(x[i]) * y[i]", "a+b", "0", n, [x, y])
    # depth of the scan's combination tree at this size (see the float scan tests)
    tol = 80 * 2.0 ** -24 * r.abs_prefix + 2 * r.err_prefix
    assert np.all(np.abs(g - r.values) <= tol)


def test_complex_shifted_reads(dev):
    # complex64 shifted reads take the vector kernel's unaligned chunk loads
    n = 70001
    x, y = cdata(n + 2, 5)
    sig = "complex64 *z, const complex64 *x, const complex64 *y"
    stmt = "z[i] = (i >= 1 ? x[i - 1] : y[i]) * conj(x[i]) + (i + 2 < n ? y[i + 2] : x[i])"
    k = hm.compile(stmt, sig, name="cplx_shift")
    assert k.vectorizable and "hipmr_loadu" in k.source(0)
    zd = torch.full((n + 2,), complex("nan+nanj"), dtype=torch.complex64, device=dev)
    hm.elementwise(k, n, [zd[1:n + 1], dev_array(x)[1:n + 1], dev_array(y)[1:n + 1]])
    torch.cuda.synchronize()
    ref = oracle.elementwise(sig, stmt, n, [np.zeros(n, np.complex64), x[1:n + 1], y[1:n + 1]])
    assert_lanes(zd[1:n + 1], ref["z"], "complex64", what="complex shifted reads")


def test_complex_at_timed_size(dev):
    # the timed complex64 workloads at n = 2^27: z = a x + b y on the timed
    # inputs (sampled lanes against the oracle), then the conjugated dot and
    # the sum of Gaussian integers with parts in [-3, 3], whose float sums
    # are exact integers in any order (every partial sum stays far below 2^24)
    import workloads
    n = workloads.N_COMPLEX
    x, y = workloads.complex_xy(n)
    xd, yd = dev_array(x), dev_array(y)
    z = torch.empty_like(xd)
    sig, stmt = workloads.C_AXPBY
    k = hm.compile(stmt, sig, name="c_axpby")
    hm.elementwise(k, n, [z, workloads.C_A, xd, workloads.C_B, yd])
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    lanes = np.unique(np.concatenate([np.arange(4096), np.arange(n - 4096, n),
                                      rng.integers(0, n, 1 << 18)]))
    ref = oracle.elementwise(sig, stmt, n, [np.zeros(1, np.complex64), np.complex64(workloads.C_A), x,
                                            np.complex64(workloads.C_B), y], lanes=lanes)["z"]
    assert assert_lanes(z, ref, "complex64", what="complex axpby 2^27") == lanes.size
    del xd, yd, z, x, y
    parts = [rng.integers(-3, 4, n).astype(np.int64) for _ in range(4)]
    xr, xi, yr, yi = parts
    gx = (xr + 1j * xi).astype(np.complex64)
    gy = (yr + 1j * yi).astype(np.complex64)
    xd, yd = dev_array(gx), dev_array(gy)
    out = torch.empty((), dtype=torch.complex64, device=dev)
    sig, mp, comb, neu = workloads.C_DOT
    kd = hm.compile(mp, sig, name="c_conj_dot")
    got = complex(reduce_on_gpu(kd, comb, neu, n, [xd, yd], out=out).item())
    want = complex(int((xr * yr + xi * yi).sum()), int((xr * yi - xi * yr).sum()))
    assert got == want, (got, want)
    sig, mp, comb, neu = workloads.C_SUM
    ks = hm.compile(mp, sig, name="c_sum")
    got = complex(reduce_on_gpu(ks, comb, neu, n, [xd], out=out).item())
    assert got == complex(int(xr.sum()), int(xi.sum())), got
    del xd, yd
    torch.cuda.empty_cache()
