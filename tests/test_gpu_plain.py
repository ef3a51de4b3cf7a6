"""GPU parity of the plain path (elementwise + map-reduce) against the CPU
oracle, through the C ABI: the paper's listings, the single fused dot on
2**20 elements, the plain-at-scale workload at n = 2**28, an n sweep with
ragged tails and misaligned bases, every launch-geometry knob, the scalar
fallback kernels, low-precision loads and stores, and the edge cases."""

import math

import numpy as np
import pytest

from gpu_util import (assert_lanes, assert_reduce, dev_array, host_bits, need_gpu,
                      reduce_on_gpu, torch)
import oracle
import paper_1304_5553_amd as hm
import workloads

pytestmark = pytest.mark.gpu

E1_SIG, E1_STMT = workloads.E1
E2_SIG, E2_STMT = workloads.E2

SWEEP_N = sorted(set(list(range(0, 70)) + [127, 128, 129, 255, 256, 257, 1023, 1024, 1025,
                                           4095, 4096, 4097, 8191, 8193, 65535, 65539,
                                           262144 + 17, (1 << 20) + 5]))


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def kernels():
    return {
        "e1": hm.compile(E1_STMT, E1_SIG, name="e1_lincomb"),
        "e2": hm.compile(E2_STMT, E2_SIG, name="e2_hypot"),
        "count": hm.compile(workloads.R_COUNT[1], workloads.R_COUNT[0], name="r1_count"),
        "sum": hm.compile(workloads.R_SUM[1], workloads.R_SUM[0], name="r2_sum"),
        "max": hm.compile(workloads.R_MAX[1], workloads.R_MAX[0], name="r3_max"),
        "dot": hm.compile(workloads.DOT[1], workloads.DOT[0], name="dot"),
    }


# ---------------------------------------------------------------- listings
def test_listing1_multiply_by_two(dev):
    rng = np.random.default_rng(1)
    a = rng.standard_normal((4, 4)).astype(np.float32)
    ad = dev_array(a.reshape(-1))
    k = hm.ElementwiseKernel("float *a", "a[i] *= 2", "multiply2")
    k(ad)
    torch.cuda.synchronize()
    assert np.array_equal(host_bits(ad).reshape(4, 4), 2 * a)


def test_listing3a_linear_combination(dev):
    rng = np.random.default_rng(2)
    x = rng.random(50).astype(np.float32)
    y = rng.random(50).astype(np.float32)
    lin = hm.ElementwiseKernel("float a, float *x, float b, float *y, float *z",
                               "z[i] = a*x[i] + b*y[i]", "linear_combination")
    z = torch.empty(50, dtype=torch.float32, device=dev)
    lin(5, dev_array(x), 6, dev_array(y), z)
    torch.cuda.synchronize()
    ref = oracle.elementwise("float a, float *x, float b, float *y, float *z",
                             "z[i] = a*x[i] + b*y[i]", 50, [5, x, 6, y, np.zeros(50, np.float32)])
    assert_lanes(z, ref["z"], "float32", what="listing 3a")


def test_listing3b_dot_of_arange(dev):
    a = torch.arange(400, dtype=torch.float32, device=dev)
    krnl = hm.ReductionKernel(np.float32, "float *x, float *y", "x[i]*y[i]", "a+b", "0")
    got = krnl(a, a).item()
    an = np.arange(400, dtype=np.float32)
    r = oracle.reduce("float: float *x, float *y", "x[i]*y[i]", "a+b", "0", 400, [an, an])
    assert r.value == 21253400
    assert_reduce(got, r, "listing 3b")


@pytest.mark.parametrize("force_scalar", [False, True])
def test_listing4_unrolled_add_exact(dev, force_scalar):
    n = 16 * 32 * 33
    rng = np.random.default_rng(44)
    a = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    k = hm.compile("tgt[i] = op1[i] + op2[i]", "float *tgt, float *op1, float *op2", name="add")
    c = torch.empty(n, dtype=torch.float32, device=dev)
    cfg = {"flags": hm.CFG_FORCE_SCALAR} if force_scalar else None
    hm.elementwise(k, n, [c, dev_array(a), dev_array(b)], config=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(host_bits(c), a + b)     # norm(c - (a + b)) == 0


# ---------------------------------------------------------------- dot, 2**20
def test_dot_1m(dev, kernels):
    x, y = workloads.dot_1m()
    xd, yd = dev_array(x), dev_array(y)
    out = reduce_on_gpu(kernels["dot"], "a+b", "0", x.size, [xd, yd])
    r = oracle.reduce(workloads.DOT[0], workloads.DOT[1], "a+b", "0", x.size, [x, y])
    assert_reduce(out, r, "dot 2^20", bare=True)   # the 2e-6 * sum|t| gate itself
    again = reduce_on_gpu(kernels["dot"], "a+b", "0", x.size, [xd, yd])
    assert out.item() == again.item()              # bitwise repeatable


# ---------------------------------------------------------------- sweeps
@pytest.fixture(scope="module")
def sweep_data():
    nmax = max(SWEEP_N) + 32
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, nmax).astype(np.float32)
    y = rng.uniform(-1, 1, nmax).astype(np.float32)
    k = rng.integers(0, 1 << 20, nmax, dtype=np.int32)
    return x, y, k


@pytest.mark.parametrize("name", ["e1", "e2"])
@pytest.mark.parametrize("offsets", [(0, 0, 0), (1, 1, 1), (3, 3, 3), (2, 1, 0)])
def test_elementwise_sweep(dev, kernels, sweep_data, name, offsets):
    x, y, _ = sweep_data
    sig, stmt = (E1_SIG, E1_STMT) if name == "e1" else (E2_SIG, E2_STMT)
    oz, ox, oy = offsets
    xd, yd = dev_array(x), dev_array(y)
    zfull = torch.full((x.size,), float("nan"), dtype=torch.float32, device=dev)
    for n in SWEEP_N:
        zv = zfull[oz:oz + n]
        hm.elementwise(kernels[name], n, [zv, xd[ox:ox + n], yd[oy:oy + n]])
        torch.cuda.synchronize()
        ref = oracle.elementwise(sig, stmt, n, [np.zeros(n, np.float32), x[ox:ox + n],
                                                y[oy:oy + n]])
        if n:
            assert_lanes(zv, ref["z"], "float32", what=f"{name} n={n} offsets={offsets}")
        # nothing outside [0, n) of the output was touched
        zh = host_bits(zfull)
        assert np.all(np.isnan(zh[:oz])) and np.all(np.isnan(zh[oz + n:oz + n + 8]))
        zfull.fill_(float("nan"))


@pytest.mark.parametrize("name", ["count", "sum"])
@pytest.mark.parametrize("offset", [0, 1, 2, 3])
def test_int_reduce_sweep_exact(dev, kernels, sweep_data, name, offset):
    _, _, k = sweep_data
    sig, mp, comb, neu = workloads.R_COUNT if name == "count" else workloads.R_SUM
    kd = dev_array(k)
    for n in SWEEP_N:
        out = reduce_on_gpu(kernels[name], comb, neu, n, [kd[offset:offset + n]])
        r = oracle.reduce(sig, mp, comb, neu, n, [k[offset:offset + n]])
        assert_reduce(out, r, f"{name} n={n} offset={offset}")


@pytest.mark.parametrize("offset", [0, 1, 3])
def test_max_and_dot_sweep(dev, kernels, sweep_data, offset):
    x, y, _ = sweep_data
    xd, yd = dev_array(x), dev_array(y)
    for n in SWEEP_N:
        xs, ys = x[offset:offset + n], y[offset:offset + n]
        out = reduce_on_gpu(kernels["max"], "max(a,b)", "-INFINITY", n, [xd[offset:offset + n]])
        assert_reduce(out, oracle.reduce(workloads.R_MAX[0], "x[i]", "max(a,b)", "-INFINITY",
                                         n, [xs]), f"max n={n}")
        out = reduce_on_gpu(kernels["dot"], "a+b", "0", n, [xd[offset:offset + n],
                                                            yd[offset:offset + n]])
        assert_reduce(out, oracle.reduce(workloads.DOT[0], workloads.DOT[1], "a+b", "0",
                                         n, [xs, ys]), f"dot n={n}")


# ---------------------------------------------------------------- geometry
CONFIGS = [dict(block=64, items_per_thread=1), dict(block=1024, items_per_thread=16),
           dict(block=192, items_per_thread=3), dict(vec=1), dict(vec=2), dict(vec=8),
           dict(vec=16, items_per_thread=2), dict(grid=1), dict(grid=7, block=128),
           dict(flags=hm.CFG_TEMPORAL), dict(blocks_per_cu=1), dict(flags=hm.CFG_FORCE_SCALAR)]


@pytest.mark.parametrize("cfg", CONFIGS, ids=[str(c) for c in CONFIGS])
def test_launch_configs(dev, kernels, sweep_data, cfg):
    x, y, k = sweep_data
    xd, yd, kd = dev_array(x), dev_array(y), dev_array(k)
    for n in (0, 1, 37, 4099, 100003):
        z = torch.empty(n, dtype=torch.float32, device=dev)
        hm.elementwise(kernels["e1"], n, [z, xd[1:1 + n], yd[1:1 + n]], config=cfg)
        torch.cuda.synchronize()
        ref = oracle.elementwise(E1_SIG, E1_STMT, n, [np.zeros(n, np.float32), x[1:1 + n],
                                                      y[1:1 + n]])
        if n:
            assert_lanes(z, ref["z"], "float32", what=f"e1 {cfg} n={n}")
        out = reduce_on_gpu(kernels["sum"], "a+b", "0", n, [kd[:n]], config=cfg)
        assert_reduce(out, oracle.reduce(workloads.R_SUM[0], "k[i]", "a+b", "0", n, [k[:n]]),
                      f"sum {cfg} n={n}")


# ---------------------------------------------------------------- other kernels
def test_scalar_fallback_expressions(dev):
    rng = np.random.default_rng(11)
    n = 50001
    x = rng.uniform(-1, 1, n).astype(np.float32)
    xd = dev_array(x)
    sig = "float *z, const float *x"
    for stmt in ("z[i] = x[n - 1 - i]", "z[i] = x[i + 1 < n ? i + 1 : i] - x[i]",
                 "if (i % 3 == 0) z[i] = x[i] * 2; else z[i] = -x[i]"):
        k = hm.compile(stmt, sig)
        z = torch.empty(n, dtype=torch.float32, device=dev)
        hm.elementwise(k, n, [z, xd])
        torch.cuda.synchronize()
        ref = oracle.elementwise(sig, stmt, n, [np.zeros(n, np.float32), x])["z"]
        assert_lanes(z, ref, "float32", what=stmt)
    k = hm.compile("x[n - 1 - i] * (float)(i % 5)", "double: const float *x")
    assert not k.vectorizable
    out = reduce_on_gpu(k, "a+b", "0", n, [xd])
    assert_reduce(out, oracle.reduce("double: const float *x", "x[n - 1 - i] * (float)(i % 5)",
                                     "a+b", "0", n, [x]), "scalar reduce")


def test_generic_combines_exact(dev):
    rng = np.random.default_rng(12)
    n = 40000
    k = rng.integers(0, 2 ** 31 - 1, n).astype(np.int32)
    kd = dev_array(k)
    for comb, neu in (("a|b", "0"), ("a^b", "0"), ("a&b", "-1")):
        kern = hm.compile("k[i]", "int: const int *k")
        out = reduce_on_gpu(kern, comb, neu, n, [kd])
        assert_reduce(out, oracle.reduce("int: const int *k", "k[i]", comb, neu, n, [k]), comb)
    u = rng.integers(0, 2 ** 32, 3000).astype(np.uint32)
    kern = hm.compile("u[i]", "unsigned: const unsigned *u")
    out = reduce_on_gpu(kern, "a*b", "1u", 3000, [dev_array(u)])
    r = oracle.reduce("unsigned: const unsigned *u", "u[i]", "a*b", "1u", 3000, [u])
    assert int(host_bits(out)) == r.value


def test_min_max_edge_values(dev):
    cases = [np.array([-0.0, 0.0, -0.0], np.float32), np.array([0.0, -0.0], np.float32),
             np.array([1.0, np.nan, 3.0], np.float32), np.array([-np.inf, -5.0], np.float32),
             np.array([np.inf], np.float32)]
    for x in cases:
        for comb, neu in (("max", "-INFINITY"), ("min", "INFINITY")):
            k = hm.compile("x[i]", "float: const float *x")
            out = reduce_on_gpu(k, comb, neu, x.size, [dev_array(x)])
            r = oracle.reduce("float: const float *x", "x[i]", comb, neu, x.size, [x])
            assert_reduce(out, r, f"{comb} of {x}")


def test_zero_length(dev, kernels):
    z = torch.empty(0, dtype=torch.float32, device=dev)
    hm.elementwise(kernels["e1"], 0, [z, z, z])
    for name, (sig, mp, comb, neu) in (("max", workloads.R_MAX), ("sum", workloads.R_SUM)):
        arr = torch.empty(0, dtype=torch.float32 if name == "max" else torch.int32, device=dev)
        out = reduce_on_gpu(kernels[name], comb, neu, 0, [arr])
        assert out.item() == (-math.inf if name == "max" else 0)


def test_errors(dev, kernels):
    x = torch.zeros(10, device=dev)
    y = torch.zeros(11, device=dev)
    lin = hm.ElementwiseKernel(E1_SIG, E1_STMT)
    with pytest.raises(hm.MismatchError):
        lin(x, x, y)                                  # arrays of different lengths
    out = torch.empty((), device=dev)
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(hm.WorkspaceError):
        hm.reduce(kernels["max"], None, "max", "-INFINITY", 10, [x], out, workspace_buf=small)
    with pytest.raises(hm.MismatchError):
        hm.reduce(kernels["max"], "x[i]*2", "max", "-INFINITY", 10, [x], out)
    with pytest.raises(hm.MismatchError):
        hm.elementwise(kernels["max"], 10, [x])
    with pytest.raises(hm.InvalidError):
        hm.elementwise(kernels["e1"], -1, [x, x, x])


# ---------------------------------------------------------------- formats
@pytest.mark.parametrize("fmt", ["bfloat16", "float16", "fp8_e4m3"])
def test_lowp_loads_every_code(dev, fmt):
    bits = np.arange(256 if fmt == "fp8_e4m3" else 65536).astype(
        np.uint8 if fmt == "fp8_e4m3" else np.uint16)
    n = bits.size
    sig = f"float *z, const {fmt} *x"
    k = hm.compile("z[i] = x[i]", sig)
    z = torch.empty(n, dtype=torch.float32, device=dev)
    hm.elementwise(k, n, [z, dev_array(bits, fmt)])
    torch.cuda.synchronize()
    ref = oracle.elementwise(sig, "z[i] = x[i]", n, [np.zeros(n, np.float32), bits])["z"]
    assert_lanes(z, ref, "float32", what=f"{fmt} decode")


@pytest.mark.parametrize("fmt", ["bfloat16", "float16", "fp8_e4m3"])
def test_lowp_stores_round_to_nearest_even(dev, fmt):
    rng = np.random.default_rng(13)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-8, 8, 100000))).astype(np.float32)
    x[:6] = [0.0, -0.0, 1e30, -1e30, 448.0, 465.0]
    n = x.size
    k = hm.compile("q[i] = x[i]", f"{fmt} *q, const float *x")
    q = torch.empty(n, dtype=gpu_lowp(fmt), device=dev)
    hm.elementwise(k, n, [q, dev_array(x)])
    torch.cuda.synchronize()
    xt = torch.from_numpy(x)
    if fmt == "fp8_e4m3":
        want = xt.clamp(-448, 448).to(torch.float8_e4m3fn)
    else:
        want = xt.to(gpu_lowp(fmt))
    g = host_bits(q)
    w = host_bits(want)
    assert np.array_equal(g, w), f"{fmt}: {np.count_nonzero(g != w)} stores differ"


def gpu_lowp(fmt):
    return {"bfloat16": torch.bfloat16, "float16": torch.float16,
            "fp8_e4m3": torch.float8_e4m3fn}[fmt]


# ---------------------------------------------------------------- maximum sizes
def test_64bit_index_beyond_2_31(dev):
    n = (1 << 31) + 5
    ones = torch.ones(n, dtype=torch.uint8, device=dev)
    k = hm.compile("x[i]", "long: const uint8_t *x")
    out = reduce_on_gpu(k, "a+b", "0", n, [ones])
    assert out.item() == n
    k = hm.compile("(long)i", "long: const uint8_t *x")
    out = reduce_on_gpu(k, "a+b", "0", n, [ones])
    assert out.item() == n * (n - 1) // 2
    # shifted reads with a 64-bit index: chunk loads near and beyond 2^31
    k = hm.compile("(i + 3 < n ? x[i + 3] : 0) + (i >= 7 ? x[i - 7] : 0)", "long: const uint8_t *x")
    assert k.vectorizable
    out = reduce_on_gpu(k, "a+b", "0", n, [ones])
    assert out.item() == (n - 3) + (n - 7)
    e = hm.compile("z[i] = i + 1 < n ? x[i + 1] : 0", "uint8_t *z, const uint8_t *x")
    z = torch.full((n,), 7, dtype=torch.uint8, device=dev)
    hm.elementwise(e, n, [z, ones])
    assert int(z.sum(dtype=torch.int64).item()) == n - 1 and int(z[-1].item()) == 0
    del ones, z
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- plain at scale, n = 2**28
@pytest.fixture(scope="module")
def plain_data(dev):
    x, y = workloads.plain_xy()
    k = workloads.plain_k()
    return x, y, k


def test_plain_at_scale_reductions(dev, kernels, plain_data):
    x, y, k = plain_data
    n = x.size
    kd = dev_array(k)
    for name, spec in (("count", workloads.R_COUNT), ("sum", workloads.R_SUM)):
        sig, mp, comb, neu = spec
        out = reduce_on_gpu(kernels[name], comb, neu, n, [kd])
        r = oracle.reduce(sig, mp, comb, neu, n, [k])
        assert_reduce(out, r, f"{name} 2^28")
        again = reduce_on_gpu(kernels[name], comb, neu, n, [kd])
        assert out.item() == again.item()
    del kd
    xd = dev_array(x)
    out = reduce_on_gpu(kernels["max"], "max(a,b)", "-INFINITY", n, [xd])
    assert_reduce(out, oracle.reduce(workloads.R_MAX[0], "x[i]", "max(a,b)", "-INFINITY", n, [x]),
                  "max 2^28")
    del xd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["e1", "e2"])
def test_plain_at_scale_elementwise_every_lane(dev, kernels, plain_data, name):
    """E1 / E2 at n = 2^28: every output lane against the oracle, compared
    in chunks of 2^22 lanes (the oracle's value and bound per lane)."""
    x, y, _ = plain_data
    n = x.size
    sig, stmt = (E1_SIG, E1_STMT) if name == "e1" else (E2_SIG, E2_STMT)
    xd, yd = dev_array(x), dev_array(y)
    z = torch.empty(n, dtype=torch.float32, device=dev)
    hm.elementwise(kernels[name], n, [z, xd, yd])
    torch.cuda.synchronize()
    zh = z.cpu()
    zero = np.zeros(1, np.float32)
    step = 1 << 22
    checked = 0
    for a in range(0, n, step):
        b = min(a + step, n)
        ref = oracle.elementwise(sig, stmt, n, [zero, x, y], lanes=np.arange(a, b))["z"]
        checked += assert_lanes(zh[a:b], ref, "float32", lanes=np.arange(b - a),
                                what=f"{name} 2^28 lanes [{a}, {b})")
    assert checked == n
    z2 = torch.empty_like(z)
    hm.elementwise(kernels[name], n, [z2, xd, yd])
    torch.cuda.synchronize()
    assert torch.equal(z, z2)                           # bitwise repeatable
    del xd, yd, z, z2
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- fixed-element reads
@pytest.mark.parametrize("offset", [0, 1, 3])
def test_fixed_element_reads_vector_path(dev, offset):
    """Device-resident scalars read as a[0] / a[1] stay on the 16-byte path
    (the same element for every i, read directly)."""
    n = 70001
    rng = np.random.default_rng(95 + offset)
    x = rng.uniform(-1, 1, n + 8).astype(np.float32)
    p = rng.uniform(-1, 1, n + 8).astype(np.float32)
    a = np.array([0.3125, -1.75], np.float64)
    sig = "float *x, const float *p, const double *a"
    stmt = "x[i] += (float)a[0] * p[i] - (float)a[1]"
    k = hm.compile(stmt, sig, name="fixed_ew")
    assert k.vectorizable
    xd, pd, ad = dev_array(x), dev_array(p), dev_array(a)
    xs, ps = x[offset:offset + n].copy(), p[offset:offset + n]
    hm.elementwise(k, n, [xd[offset:offset + n], pd[offset:offset + n], ad])
    torch.cuda.synchronize()
    ref = oracle.elementwise(sig, stmt, n, [xs, ps, a])
    assert_lanes(xd[offset:offset + n], ref["x"], "float32", what=f"fixed-element ew offset {offset}")
    assert k.last_symbols()[0].split("_")[-2] == "ew"       # the vector kernel ran
    # map-reduce with a fixed-element scale
    r = hm.compile("s[1] * x[i]", "float: const float *x, const float *s", name="fixed_red")
    s = np.array([9.0, 0.5], np.float32)
    x0d = dev_array(x)                                       # xd was updated above
    out = reduce_on_gpu(r, "a+b", "0", n, [x0d[offset:offset + n], dev_array(s)])
    assert_reduce(out, oracle.reduce("float: const float *x, const float *s", "s[1] * x[i]", "a+b", "0",
                                     n, [x[offset:offset + n], s]), "fixed-element reduce")


# ---------------------------------------------------------------- shifted reads
SHIFT_CASES = [
    ("z[i] = (i >= 1 ? x[i - 1] : 0.0f) + 2.0f * x[i] + (i + 1 < n ? x[i + 1] : 0.0f)",
     "float *z, const float *x", "float32", ()),
    ("z[i] = (i + k < n && i + k >= 0 ? x[i + k] : 1.5f) * 0.5f - x[i]",
     "float *z, const float *x, long k", "float32", (np.int64(1000),)),
    ("z[i] = (i + k < n && i + k >= 0 ? x[i + k] : 1.5f) * 0.5f - x[i]",
     "float *z, const float *x, long k", "float32", (np.int64(-37),)),
    ("z[i] = (i + k < n && i + k >= 0 ? x[i + k] : 1.5f) * 0.5f - x[i]",
     "float *z, const float *x, long k", "float32", (np.int64(10 ** 6),)),   # beyond n: all per element
    ("o[i] = (i + 2*m < n ? (float)b[i + 2*m] : 0.0f) + (i >= (m) ? (float)b[i - (m)] : 0.0f)",
     "bfloat16 *o, const bfloat16 *b, int m", "bfloat16", (np.int32(5),)),
    ("w[i] = (i + 3 < n ? v[i + 3] : 0) - (i >= 2 ? v[i - 2] : 0)", "int *w, const int *v", "int32", ()),
]


@pytest.mark.parametrize("case", range(len(SHIFT_CASES)))
@pytest.mark.parametrize("n,offset", [(70001, 0), (70001, 3), (5, 1), (4099, 2)])
def test_shifted_reads_vector_path(dev, case, n, offset):
    """name[i + E] reads (E uniform) run on the vector kernel: unaligned chunk
    loads, per-element evaluation within the largest distance of either end.
    Results match the oracle and, bit for bit, the one-element kernel."""
    stmt, sig, dt, scalars = SHIFT_CASES[case]
    rng = np.random.default_rng(300 + case + n + offset)
    if dt == "int32":
        src = rng.integers(-10 ** 6, 10 ** 6, n + 8).astype(np.int32)
        out_np, tdt = np.int32, torch.int32
    else:
        src = rng.uniform(-2, 2, n + 8).astype(np.float32)
        out_np, tdt = np.float32, torch.float32
    if dt == "bfloat16":
        bits = torch.from_numpy(src).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        sd = dev_array(bits, "bfloat16")
        host_in = bits[offset:offset + n]
        tdt = torch.bfloat16
        zero = np.zeros(n, np.uint16)
    else:
        sd = dev_array(src)
        host_in = src[offset:offset + n]
        zero = np.zeros(n, out_np)
    k = hm.compile(stmt, sig, name="shift_t")
    assert k.vectorizable
    outs = []
    for cfg in (None, {"flags": hm.CFG_FORCE_SCALAR}):
        buf = torch.zeros(n + 8, dtype=tdt, device=dev)
        z = buf[offset:offset + n]
        hm.elementwise(k, n, [z, sd[offset:offset + n], *[int(v) for v in scalars]], config=cfg)
        torch.cuda.synchronize()
        assert k.last_symbols()[0].split("_")[-2] == ("ew" if cfg is None else "ews")
        tail = host_bits(buf[offset + n:])
        assert np.all(tail == 0), "wrote past the end"
        outs.append(host_bits(z))
    assert np.array_equal(outs[0], outs[1]), "vector and one-element kernels differ"
    ref = oracle.elementwise(sig, stmt, n, [zero, host_in, *scalars])
    name = sig.split("*")[1].split(",")[0].strip()
    assert_lanes(z, ref[name], dt, what=f"{stmt} n={n} offset={offset} {scalars}")


@pytest.mark.parametrize("offset", [0, 1])
def test_shifted_maps(dev, offset):
    """Maps with shifted reads: the plain reduce loads them as chunks (rs1),
    the other facilities read them element by element inside their vector
    kernels; every result matches the oracle."""
    n = 300007
    rng = np.random.default_rng(400 + offset)
    x = rng.uniform(-1, 1, n + 8).astype(np.float32)
    k = rng.integers(-1000, 1000, n + 8).astype(np.int32)
    xs, ks = x[offset:offset + n], k[offset:offset + n]
    xd, kd = dev_array(x)[offset:offset + n], dev_array(k)[offset:offset + n]
    # float sum of a lag-1 product: vector (shifted chunks) and one-element kernels
    sig, mp = "float: const float *x", "(i + 1 < n ? x[i + 1] : 0.0f) * x[i]"
    h = hm.compile(mp, sig, name="lag1")
    assert h.vectorizable
    ref = oracle.reduce(sig, mp, "a+b", "0", n, [xs])
    for cfg, tag in ((None, "rs1"), ({"flags": hm.CFG_FORCE_SCALAR}, "rs1s")):
        out = reduce_on_gpu(h, "a+b", "0", n, [xd], config=cfg)
        assert h.last_symbols()[0].split("_")[-2] == tag
        assert_reduce(out, ref, f"lag-1 sum {tag}")
    # exact integer sums at positive and negative distances, and a shifted max
    isig, imp = "long: const int *k, int s", "(i + s < n && i + s >= 0 ? k[i + s] : 0) - k[i]"
    hi = hm.compile(imp, isig, name="lagk")
    for s in (4097, -3, 1 << 20):
        out = reduce_on_gpu(hi, "a+b", "0", n, [kd, s])
        assert_reduce(out, oracle.reduce(isig, imp, "a+b", "0", n, [ks, np.int32(s)]), f"int lag {s}")
    msig, mmp = "float: const float *x, long d", "i >= d ? x[i - d] : -INFINITY"
    hmx = hm.compile(mmp, msig, name="lagmax")
    out = reduce_on_gpu(hmx, "max(a,b)", "-INFINITY", n, [xd, 5])
    assert_reduce(out, oracle.reduce(msig, mmp, "max(a,b)", "-INFINITY", n, [xs, np.int64(5)]), "shifted max")
    # compensated sum (FP64 result) with the shifted map
    hc = hm.compile("(i + 1 < n ? x[i + 1] : 0.0f)", "float: const float *x", name="lagc")
    g = hm.reduce_compensated(hc, n, [xd]).item()
    want = oracle.exact_sum(xs[1:].astype(np.float64))
    assert abs(g - want) <= 1e-6 * float(np.abs(xs).sum()), (g, want)
    # segmented integer sums: the map reads across segment boundaries (i is global)
    cuts = np.sort(rng.integers(0, n, 499))
    offs = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    sseg = torch.empty(len(offs) - 1, dtype=torch.int64, device=dev)
    hm.reduce_segmented(hi, "a+b", "0", dev_array(offs), n, [kd, 7], sseg)
    torch.cuda.synchronize()
    mv = oracle.map_values(isig, imp, n, [ks, np.int32(7)]).v.astype(np.int64)
    assert host_bits(sseg).tolist() == [int(mv[a:b].sum()) for a, b in zip(offs[:-1], offs[1:])]
    # inclusive scan of the shifted map
    ssig, smp = "long: const int *k", "i >= 1 ? k[i - 1] : 0"
    hs = hm.compile(smp, ssig, name="lagscan")
    sc = torch.empty(n, dtype=torch.int64, device=dev)
    hm.scan(hs, "a+b", "0", n, [kd], sc)
    torch.cuda.synchronize()
    assert np.array_equal(host_bits(sc), oracle.scan(ssig, smp, "a+b", "0", n, [ks]).values)


def test_fp8_shifted_reads(dev):
    """FP8 arrays read at a distance (16 values per chunk, loaded by memcpy)."""
    n = 65537
    rng = np.random.default_rng(77)
    bits = rng.integers(0, 256, n + 16).astype(np.uint8)
    bits[(bits & 0x7F) == 0x7F] = 0x3C                     # no NaN codes
    sig = "float *z, const fp8_e4m3 *q"
    stmt = "z[i] = (i + 3 < n ? (float)q[i + 3] : 0.0f) - (i >= 17 ? (float)q[i - 17] : 1.0f) * (float)q[i]"
    k = hm.compile(stmt, sig, name="fp8_shift")
    assert k.vectorizable and k.vec == 16
    qd = dev_array(bits, "fp8_e4m3")
    outs = []
    for cfg in (None, {"flags": hm.CFG_FORCE_SCALAR}):
        z = torch.zeros(n, dtype=torch.float32, device=dev)
        hm.elementwise(k, n, [z, qd[5:n + 5]], config=cfg)
        torch.cuda.synchronize()
        outs.append(host_bits(z))
    assert np.array_equal(outs[0], outs[1]), "vector and one-element kernels differ"
    ref = oracle.elementwise(sig, stmt, n, [np.zeros(n, np.float32), bits[5:n + 5]])
    assert_lanes(z, ref["z"], "float32", what="fp8 shifted reads")


def test_shifted_reads_huge_distances(dev):
    """Distances near the 64-bit limits: no chunk qualifies for the vector
    loads (the bounds checks never form an overflowing sum), every element
    runs the statement with its own guard."""
    n = 10007
    rng = np.random.default_rng(501)
    x = rng.uniform(-1, 1, n).astype(np.float32)
    xd = dev_array(x)
    sig = "float *z, const float *x, long k"
    stmt = "z[i] = (i + k < n && i + k >= 0 ? x[i + k] : 2.0f) + x[i]"
    k = hm.compile(stmt, sig, name="shift_huge")
    rsig, rmap = "float: const float *x, long k", "(i + k < n && i + k >= 0 ? x[i + k] : 2.0f) * x[i]"
    r = hm.compile(rmap, rsig, name="shift_huge_r")
    for dist in ((1 << 62), -(1 << 62), (1 << 63) - (1 << 15), -(1 << 63) + (1 << 15)):   # i + k fits
        z = torch.zeros(n, dtype=torch.float32, device=dev)
        hm.elementwise(k, n, [z, xd, dist])
        out = reduce_on_gpu(r, "a+b", "0", n, [xd, dist])
        torch.cuda.synchronize()
        assert np.array_equal(host_bits(z), (np.float32(2.0) + x).astype(np.float32)), dist
        assert_reduce(out, oracle.reduce(rsig, rmap, "a+b", "0", n, [x, np.int64(dist)]), f"reduce {dist}")


@pytest.mark.parametrize("flags", [0, hm.CFG_FORCE_SCALAR])
def test_shifted_reads_at_timed_sizes(dev, flags):
    # the two timed shifted-read workloads at their measured sizes, on the
    # vector kernels and on the one-element kernels: the five-point stencil on
    # a 4096 x 4096 grid (sampled lanes against the oracle) and the lag-1
    # product sum over 2^28 float32 values of +-1, whose float sum is an exact
    # integer in any order (every partial sum is an integer far below 2^24)
    from paper_1304_5553_amd import cg as hcg
    cfg = {"flags": flags} if flags else None
    nx = 4096
    m = nx * nx
    rng = np.random.default_rng(10)
    p = rng.random(m, dtype=np.float32)
    pd, q = dev_array(p), torch.empty(m, device=dev)
    k = hm.compile(hcg.SPMV[1], hcg.SPMV[0], name="cg_spmv")
    hm.elementwise(k, m, [q, pd, nx], config=cfg)
    torch.cuda.synchronize()
    lanes = np.unique(np.concatenate([np.arange(2 * nx), np.arange(m - 2 * nx, m),
                                      rng.integers(0, m, 1 << 17)]))
    ref = oracle.elementwise(hcg.SPMV[0], hcg.SPMV[1], m, [np.zeros(1, np.float32), p, np.int32(nx)],
                             lanes=lanes)["q"]
    assert assert_lanes(q, ref, "float32", what=f"stencil 4096^2 flags={flags}") == lanes.size
    del pd, q
    n = 1 << 28
    s = (rng.integers(0, 2, n, dtype=np.int8) * 2 - 1).astype(np.int8)
    want = int((s[1:] * s[:-1]).sum(dtype=np.int64))
    xd = dev_array(s.astype(np.float32))
    r = hm.compile("(i + 1 < n ? x[i + 1] : 0.0f) * x[i]", "float: const float *x", name="lag1")
    out = reduce_on_gpu(r, "a+b", "0", n, [xd], config=cfg)
    assert r.last_symbols()[0].split("_")[-2] == ("rs1s" if flags else "rs1")
    assert out.item() == float(want), (out.item(), want)
    del xd
    torch.cuda.empty_cache()


def test_default_stream_is_torchs_current_stream(dev):
    # calls without a stream launch on torch's current stream, read as a raw
    # handle: the same stream inside and outside a stream context, and the
    # work lands there (ordered with torch's own work on that stream)
    from paper_1304_5553_amd import hipmr as binding
    assert binding._stream_ptr(None) == torch.cuda.current_stream().cuda_stream
    side = torch.cuda.Stream()
    k = hm.compile(E1_STMT, E1_SIG, name="e1_lincomb")
    n = 1 << 20
    x = torch.ones(n, device=dev)
    y = torch.full((n,), 2.0, device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        assert binding._stream_ptr(None) == side.cuda_stream != torch.cuda.default_stream().cuda_stream
        z = torch.empty(n, device=dev)
        hm.elementwise(k, n, [z, x, y])
        w = z * 2.0                                  # torch's work on the same stream
    side.synchronize()
    assert bool(torch.all(w == 3.0))
