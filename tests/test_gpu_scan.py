"""GPU parity of the prefix scan (section "Further Facilities": parallel
prefix sums over a map, a combine and its neutral element) against the
oracle's scan: integer, count and max/min scans bit-exact; float sums within
the bound derived from the depth of the kernels' combination tree."""

import math

import numpy as np
import pytest

from gpu_util import dev_array, host_bits, need_gpu, torch
import oracle
import paper_1304_5553_amd as hm

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def run_scan(k, combine, neutral, n, args, out_dtype, dev, exclusive=False, out_offset=0, config=None):
    if out_dtype == torch.uint32:      # filled as int32 (same bits), seen as uint32
        buf = torch.full((n + out_offset + 1,), 7, dtype=torch.int32, device=dev).view(torch.uint32)
    else:
        buf = torch.full((n + out_offset + 1,), 7, dtype=out_dtype, device=dev)
    out = buf[out_offset:out_offset + n]
    hm.scan(k, combine, neutral, n, args, out, exclusive=exclusive, config=config)
    torch.cuda.synchronize()
    assert host_bits(buf[out_offset + n:]).tolist() == [7], "wrote past the end"
    return out


def float_depth(n, vec=4, ipt=4):
    """Longest chain of float combinations on one output's path: wave totals
    (V P_up sequential per accumulator + the pairwise fold of the pass-1
    accumulators + 6 butterfly), the two-level scan of the totals (2 x (6 +
    4 + 1)), the block prefix (1) and the rescan (U P carries + 6 + 1 + V +
    1)."""
    sub = 64 * vec * ipt
    passes = max(1, -(-n // (sub * 65536)))
    up = min(ipt, 4)
    while ipt % up:
        up -= 1
    passes_up = passes * (ipt // up)
    fold = max(0, (up - 1).bit_length())
    return (vec * passes_up + fold + 6) + 22 + 1 + (ipt * passes + vec + 8)


def default_geometry(in_size, out_size):
    """(V, U) the library picks by default: 16 bytes of the narrowest input,
    at most 16 bytes of output per lane, up to 8 sub-tiles per pass."""
    vec = min(16 // in_size, max(1, 16 // out_size))
    return vec, min(8, 4 * ((16 // in_size) // vec))


def assert_float_scan(g, r, n, what, vec=4, ipt=4):
    d = float_depth(n, vec, ipt)
    tol = d * U24 * r.abs_prefix + 2 * r.err_prefix + 1e-30
    bad = np.nonzero(~(np.abs(g - r.values) <= tol))[0]
    assert bad.size == 0, f"{what}: {bad.size} outside, first {bad[:3]}, g {g[bad[:3]]} o {r.values[bad[:3]]}"


SIZES = [1, 5, 63, 64, 65, 1000, 1024, 4097, 65539, 300007]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("exclusive", [False, True])
def test_integer_sum_scan_exact(dev, n, exclusive):
    rng = np.random.default_rng(n)
    k = rng.integers(-(1 << 20), 1 << 20, n).astype(np.int32)
    h = hm.compile("k[i]", "long: const int *k", name="scan_isum")
    got = host_bits(run_scan(h, "a+b", "0", n, [dev_array(k)], torch.int64, dev, exclusive))
    want = oracle.scan("long: const int *k", "k[i]", "a+b", "0", n, [k], exclusive=exclusive)
    assert np.array_equal(got, want.values)


@pytest.mark.parametrize("offset", [0, 1, 2, 3])
def test_count_scan_misaligned(dev, offset):
    n = 100003
    rng = np.random.default_rng(40 + offset)
    base = rng.integers(0, 1 << 20, n + 8).astype(np.int32)
    k = base[offset:offset + n]
    kd = dev_array(base)[offset:offset + n]
    h = hm.compile("k[i] % 7 == 3", "int: const int *k", name="scan_count")
    for out_offset in (offset, 0):          # same misalignment (vector), different (scalar)
        got = host_bits(run_scan(h, "a+b", "0", n, [kd], torch.int32, dev, out_offset=out_offset))
        want = oracle.scan("int: const int *k", "k[i] % 7 == 3", "a+b", "0", n, [k])
        assert np.array_equal(got, want.values), out_offset


@pytest.mark.parametrize("n", [1000, 65539, 300007])
def test_float_sum_and_dot_scan(dev, n):
    rng = np.random.default_rng(50 + n)
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    sig = "float: const float *x, const float *y"
    xd, yd = dev_array(x), dev_array(y)
    for mp in ("x[i]", "x[i]*y[i]"):
        h = hm.compile(mp, sig, name="scan_fsum")
        for exclusive in (False, True):
            g = host_bits(run_scan(h, "a+b", "0", n, [xd, yd], torch.float32, dev, exclusive))
            r = oracle.scan(sig, mp, "a+b", "0", n, [x, y], exclusive=exclusive)
            assert_float_scan(g.astype(np.float64), r, n, f"{mp} excl={exclusive}")
            if exclusive:
                assert g[0] == 0.0


def test_max_min_scan_exact(dev):
    n = 200001
    rng = np.random.default_rng(60)
    x = rng.standard_normal(n).astype(np.float32)
    x[rng.integers(0, n, 50)] = -0.0
    sig = "float: const float *x"
    xd = dev_array(x)
    for comb, neu in (("max(a,b)", "-INFINITY"), ("min", "INFINITY")):
        h = hm.compile("x[i]", sig, name="scan_ext")
        g = host_bits(run_scan(h, comb, neu, n, [xd], torch.float32, dev))
        r = oracle.scan(sig, "x[i]", comb, neu, n, [x])
        assert np.array_equal(g.view(np.uint32), r.values.astype(np.float32).view(np.uint32)), comb


@pytest.mark.parametrize("fmt,torch_dt", [("bfloat16", None), ("fp8_e4m3", None)])
def test_low_precision_input_scan(dev, fmt, torch_dt):
    n = 70001
    rng = np.random.default_rng(70)
    v = rng.uniform(-4, 4, n).astype(np.float32)
    t = torch.from_numpy(v)
    if fmt == "bfloat16":
        bits = t.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    else:
        bits = t.to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    sig = f"float: const {fmt} *x"
    h = hm.compile("x[i]", sig, name="scan_lowp")
    g = host_bits(run_scan(h, "a+b", "0", n, [dev_array(bits, fmt)], torch.float32, dev))
    r = oracle.scan(sig, "x[i]", "a+b", "0", n, [bits])
    vec, ipt = default_geometry(bits.dtype.itemsize, 4)
    assert_float_scan(g.astype(np.float64), r, n, fmt, vec=vec, ipt=ipt)
    # max of the same values is exact
    g = host_bits(run_scan(h, "max", "-INFINITY", n, [dev_array(bits, fmt)], torch.float32, dev))
    r = oracle.scan(sig, "x[i]", "max", "-INFINITY", n, [bits])
    assert np.array_equal(g.astype(np.float64), r.values)


def test_scalar_map_and_generic_combine(dev):
    n = 5000
    rng = np.random.default_rng(80)
    k = rng.integers(0, 1 << 16, n).astype(np.uint32)
    kd = dev_array(k.view(np.int32))
    sig = "unsigned: const unsigned *k"
    h = hm.compile("k[n - 1 - i]", sig, name="scan_rev")          # not name[i]: one-element path
    g = host_bits(run_scan(h, "a+b", "0u", n, [kd], torch.uint32, dev))
    r = oracle.scan(sig, "k[n - 1 - i]", "a+b", "0u", n, [k])
    assert np.array_equal(g.astype(np.int64), r.values)
    h2 = hm.compile("k[i]", sig, name="scan_or")
    g = host_bits(run_scan(h2, "a|b", "0u", n, [kd], torch.uint32, dev))
    r = oracle.scan(sig, "k[i]", "a|b", "0u", n, [k])
    assert r.op == "generic" and np.array_equal(g.astype(np.int64), r.values)


def test_geometry_overrides_and_repeatability(dev):
    n = 123457
    rng = np.random.default_rng(90)
    x = rng.uniform(-1, 1, n).astype(np.float32)
    sig = "float: const float *x"
    h = hm.compile("x[i]", sig, name="scan_geo")
    xd = dev_array(x)
    r = oracle.scan(sig, "x[i]", "a+b", "0", n, [x])
    first = run_scan(h, "a+b", "0", n, [xd], torch.float32, dev).clone()
    again = run_scan(h, "a+b", "0", n, [xd], torch.float32, dev)
    assert torch.equal(first, again)                                 # bitwise repeatable
    for block, ipt in ((64, 1), (512, 2), (1024, 8)):
        cfg = {"block": block, "items_per_thread": ipt}
        g = host_bits(run_scan(h, "a+b", "0", n, [xd], torch.float32, dev, config=cfg))
        assert_float_scan(g.astype(np.float64), r, n, f"block {block} ipt {ipt}", ipt=ipt)


def test_empty_and_errors(dev):
    h = hm.compile("x[i]", "float: const float *x", name="scan_err")
    x = torch.zeros(4, device=dev)
    out = torch.empty(0, device=dev)
    hm.scan(h, "a+b", "0", 0, [x], out)                              # no-op
    e = hm.compile("z[i] = x[i]", "float *z, const float *x")
    with pytest.raises(hm.MismatchError):
        hm.scan(e, "a+b", "0", 4, [x, x], torch.empty(4, device=dev))
    with pytest.raises(hm.WorkspaceError):
        hm.scan(h, "a+b", "0", 4, [x], torch.empty(4, device=dev),
                workspace_buf=torch.empty(16, dtype=torch.uint8, device=dev))


def test_scan_at_scale_every_prefix(dev):
    """n = 2^28 int32 -> int64 inclusive sum (the plain workload's k, 3 GB of
    traffic): every prefix against the oracle's scan, taken in chunks of 2^24
    elements, each chunk scanned from the previous chunk's last prefix as its
    initial value (so every entry is the exact prefix over [0, i])."""
    import workloads
    n = 1 << 28
    k = workloads.plain_k(n)
    kd = dev_array(k)
    h = hm.compile("k[i]", "long: const int *k", name="scan_big")
    out = torch.empty(n, dtype=torch.int64, device=dev)
    hm.scan(h, "a+b", "0", n, [kd], out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    del out, kd
    torch.cuda.empty_cache()
    step = 1 << 24
    carry = 0
    for a in range(0, n, step):
        b = min(a + step, n)
        r = oracle.scan("long: const int *k", "k[i]", "a+b", str(carry), b - a, [k[a:b]])
        assert r.exact
        bad = np.nonzero(got[a:b] != r.values)[0]
        assert bad.size == 0, f"{bad.size} prefixes differ in [{a}, {b}), first at {a + bad[0]}"
        carry = int(r.values[-1])
    assert carry == int(np.sum(k, dtype=np.int64))
