"""GPU parity of float reductions and scans under reduce expressions that are
not the canonical spellings (section "Map-Reduce": the reduce expression is
any C expression in a and b), so the generic combine is pasted into the
kernels' fold: sums spelt "(a)+(b)" and "a+b+0.0f", and the selections
"fmaxf(a,b)" / "fminf(a,b)", over the n sweep with ragged tails and
misaligned bases, against the oracle's generic fold and its order-free
error model (the proved bound at the kernels' fold depth, and the 2e-6 gate
scaled by the roundings per combination; selections bit-exact)."""

import numpy as np
import pytest

from gpu_util import (assert_reduce, dev_array, host_bits, need_gpu, reduce_depth,
                      reduce_on_gpu, torch)
import oracle
import paper_1304_5553_amd as hm

pytestmark = pytest.mark.gpu

SIG = "float: const float *x, const float *y"
SWEEP_N = sorted(set(list(range(0, 40)) + [63, 64, 65, 127, 128, 129, 255, 256, 257, 1023,
                                           1024, 1025, 4095, 4096, 4097, 8191, 8193]))
LARGE_N = [65535, 65536]      # aligned base only: the oracle's generic fold is a Python loop
COMBINES = [("(a)+(b)", "0"), ("a+b+0.0f", "0"), ("fmaxf(a,b)", "-INFINITY"),
            ("fminf(a,b)", "INFINITY")]


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def data():
    rng = np.random.default_rng(21)
    nmax = max(SWEEP_N + LARGE_N) + 8
    x = rng.uniform(-1, 1, nmax).astype(np.float32)
    y = rng.uniform(-1, 1, nmax).astype(np.float32)
    return x, y


def head_of(offset, vec=4):
    """Elements before the first 16-byte boundary of a float view that starts
    `offset` elements into a 16-byte aligned allocation."""
    return (vec - offset % vec) % vec


@pytest.mark.parametrize("combine,neutral", COMBINES, ids=[c for c, _ in COMBINES])
@pytest.mark.parametrize("mp", ["x[i]", "x[i]*y[i]"])
@pytest.mark.parametrize("offset", [0, 1, 2, 3])
def test_generic_float_reduce_sweep(dev, data, combine, neutral, mp, offset):
    x, y = data
    xd, yd = dev_array(x), dev_array(y)
    k = hm.compile(mp, SIG, name="generic_fold")
    for n in SWEEP_N + (LARGE_N if offset == 0 else []):
        xs, ys = x[offset:offset + n], y[offset:offset + n]
        out = reduce_on_gpu(k, combine, neutral, n, [xd[offset:offset + n], yd[offset:offset + n]])
        r = oracle.reduce(SIG, mp, combine, neutral, n, [xs, ys])
        if combine.startswith("fm"):
            assert r.exact or mp != "x[i]"
        d = reduce_depth(n, head_of(offset))
        assert d <= 33          # so the proved bound is inside the 2e-6 gate
        assert_reduce(out, r, f"{combine} {mp} n={n} offset={offset}", depth=d)


@pytest.mark.parametrize("combine,neutral", COMBINES, ids=[c for c, _ in COMBINES])
def test_generic_float_reduce_matches_canonical_where_exact(dev, data, combine, neutral):
    """The selections give the canonical max / min bit for bit, and the sums
    stay within the gate of the canonical sum's oracle value."""
    x, _ = data
    n = 65536
    xd = dev_array(x[:n])
    k = hm.compile("x[i]", "float: const float *x", name="generic_vs_canon")
    got = reduce_on_gpu(k, combine, neutral, n, [xd]).item()
    if combine == "fmaxf(a,b)":
        assert got == float(np.max(x[:n]))
    elif combine == "fminf(a,b)":
        assert got == float(np.min(x[:n]))
    else:
        r = oracle.reduce("float: const float *x", "x[i]", "a+b", "0", n, [x[:n]])
        assert abs(got - r.value) <= 2 * 2e-6 * r.abs_sum


@pytest.mark.parametrize("cfg", [dict(block=64, items_per_thread=1), dict(block=1024, items_per_thread=8),
                                 dict(vec=1), dict(grid=3, block=128), dict(flags=hm.CFG_FORCE_SCALAR)],
                         ids=["b64u1", "b1024u8", "v1", "g3b128", "scalar"])
def test_generic_float_reduce_geometries(dev, data, cfg):
    x, y = data
    xd, yd = dev_array(x), dev_array(y)
    k = hm.compile("x[i]*y[i]", SIG, name="generic_geom")
    for combine, neutral in COMBINES:
        for n in (1, 37, 4099, 20000):
            out = reduce_on_gpu(k, combine, neutral, n, [xd[1:1 + n], yd[1:1 + n]], config=cfg)
            r = oracle.reduce(SIG, "x[i]*y[i]", combine, neutral, n, [x[1:1 + n], y[1:1 + n]])
            assert_reduce(out, r, f"{combine} {cfg} n={n}")


@pytest.mark.parametrize("combine,neutral", COMBINES, ids=[c for c, _ in COMBINES])
@pytest.mark.parametrize("n", [1, 63, 1000, 4097, 65536])
def test_generic_float_scan(dev, data, combine, neutral, n):
    """Inclusive scans under the generic combines: selections bit-exact, sums
    within rounds * u * D * (prefix sum of |m|), D the scan's fold depth."""
    from test_gpu_scan import float_depth
    x, _ = data
    k = hm.compile("x[i]", "float: const float *x", name="generic_scan")
    buf = torch.full((n + 1,), 7.0, dtype=torch.float32, device=dev)
    hm.scan(k, combine, neutral, n, [dev_array(x[:n])], buf[:n])
    torch.cuda.synchronize()
    g = host_bits(buf).astype(np.float64)
    assert g[n] == 7.0, "wrote past the end"
    r = oracle.scan("float: const float *x", "x[i]", combine, neutral, n, [x[:n]])
    if r.exact:
        assert np.array_equal(g[:n], r.values)
    else:
        tol = r.rounds * 2.0 ** -24 * float_depth(n) * r.abs_prefix + 2 * r.err_prefix + r.abs_slack
        bad = np.nonzero(~(np.abs(g[:n] - r.values) <= tol))[0]
        assert bad.size == 0, f"{combine} n={n}: {bad.size} prefixes outside, first {bad[:3]}"
