"""GPU parity of the precision extension: compensated sums and scaled L2
norms over bfloat16, half and FP8-E4M3 inputs (per-tensor power-of-two
scale), at n = 2**27 lognormal(0, 3) values with random signs and on the
cancellation case [x; -x (1 + eps)].

Gates, per result, against the FP64 oracle:
  (i)  accumulation, vs the exact sum / norm of the dequantised values:
       sum: |g - o| <= 1e-6 * sum|q|;  norm: |g - o| <= 1e-6 * o;
  (ii) total, vs the float32 originals before rounding to the format:
       sum:  |g - sum v| <= u_q * sum|v| + N_sub * 2^-(m+1) / s + gate (i);
       norm: |g - |v|| <= u_q * |v| + sqrt(N_sub) * 2^-(m+1) / s + gate (i);
       u_q = 2^-8 (bf16), 2^-11 (half), 2^-4 (e4m3); 2^-m the format's
       smallest subnormal; N_sub the values stored as subnormals or zero.
"""

import math

import numpy as np
import pytest

from gpu_util import dev_array, need_gpu, torch
import oracle
import paper_1304_5553_amd as hm
import workloads

pytestmark = pytest.mark.gpu

FORMATS = ["bfloat16", "float16", "fp8_e4m3"]
UQ = {"bfloat16": 2.0 ** -8, "float16": 2.0 ** -11, "fp8_e4m3": 2.0 ** -4}
MIN_SUB = {"bfloat16": 2.0 ** -133, "float16": 2.0 ** -24, "fp8_e4m3": 2.0 ** -9}
MIN_NORMAL = {"bfloat16": 2.0 ** -126, "float16": 2.0 ** -14, "fp8_e4m3": 2.0 ** -6}
DECODE = {"bfloat16": oracle.decode_bf16, "float16": oracle.decode_f16,
          "fp8_e4m3": oracle.decode_e4m3fn}
REPORT = {}


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def handles():
    return {fmt: hm.compile("x[i]", f"float: const {fmt} *x", name=f"prec_{fmt[:4]}")
            for fmt in FORMATS}


@pytest.fixture(scope="module", params=["lognormal", "cancel"])
def values(request):
    return request.param, workloads.precision_values(workloads.N_PRECISION, request.param)


def gates(fmt, q, orig, scale, g_sum, g_norm):
    inv = 1.0 / scale
    o_sum = oracle.exact_sum(q) * inv
    o_norm = oracle.norm2(q) * inv
    abs_q = float(np.sum(np.abs(q))) * inv
    v = orig.astype(np.float64) * inv
    v_sum = oracle.exact_sum(v)
    v_norm = oracle.norm2(v)
    abs_v = float(np.sum(np.abs(v)))
    n_sub = int(np.count_nonzero(np.abs(q) < MIN_NORMAL[fmt]))
    half_sub = MIN_SUB[fmt] / 2 * inv
    gate_i_sum = 1e-6 * abs_q
    gate_i_norm = 1e-6 * o_norm
    err_i_sum, err_i_norm = abs(g_sum - o_sum), abs(g_norm - o_norm)
    err_ii_sum, err_ii_norm = abs(g_sum - v_sum), abs(g_norm - v_norm)
    gate_ii_sum = UQ[fmt] * abs_v + n_sub * half_sub + gate_i_sum
    gate_ii_norm = UQ[fmt] * v_norm + math.sqrt(n_sub) * half_sub + gate_i_norm
    return dict(o_sum=o_sum, o_norm=o_norm, err_i_sum=err_i_sum / abs_q,
                err_i_norm=err_i_norm / o_norm, err_ii_sum=err_ii_sum / abs_v,
                err_ii_norm=err_ii_norm / v_norm, n_sub=n_sub,
                ok=(err_i_sum <= gate_i_sum, err_i_norm <= gate_i_norm,
                    err_ii_sum <= gate_ii_sum, err_ii_norm <= gate_ii_norm))


@pytest.mark.parametrize("fmt", FORMATS)
def test_precision_at_scale(dev, handles, values, fmt):
    case, v64 = values
    qz = workloads.quantize(fmt, v64)
    n = qz.bits.size
    xd = dev_array(qz.bits, fmt)
    k = handles[fmt]
    inv = 1.0 / qz.scale
    g_sum = hm.reduce_compensated(k, n, [xd], post_scale=inv).item()
    g_norm = hm.norm2(k, n, [xd], post_scale=inv, passes=2).item()
    q = DECODE[fmt](qz.bits)
    r = gates(fmt, q, qz.original, qz.scale, g_sum, g_norm)
    REPORT[(fmt, case)] = r
    print(f"{fmt} {case}: sum {g_sum!r} (oracle {r['o_sum']!r}) err(i) {r['err_i_sum']:.2e} "
          f"err(ii) {r['err_ii_sum']:.2e}; norm {g_norm!r} err(i) {r['err_i_norm']:.2e} "
          f"err(ii) {r['err_ii_norm']:.2e}; subnormal/zero {r['n_sub']}")
    assert all(r["ok"]), r
    if fmt != "bfloat16":   # squares of half / FP8 values fit float: one pass is safe
        g1 = hm.norm2(k, n, [xd], post_scale=inv, passes=1).item()
        assert abs(g1 - r["o_norm"]) <= 1e-6 * r["o_norm"]
    # bitwise repeatable
    assert hm.reduce_compensated(k, n, [xd], post_scale=inv).item() == g_sum
    del xd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fmt", FORMATS + ["float32"])
def test_compensated_sweep_ragged_and_misaligned(dev, fmt):
    rng = np.random.default_rng(21)
    v = rng.lognormal(0, 3, 70000) * np.where(rng.random(70000) < 0.5, -1, 1)
    if fmt == "float32":
        bits, scale = v.astype(np.float32), 1.0
        q = bits.astype(np.float64)
    else:
        qz = workloads.quantize(fmt, v)
        bits, scale = qz.bits, qz.scale
        q = DECODE[fmt](bits)
    k = hm.compile("x[i]", f"float: const {'float' if fmt == 'float32' else fmt} *x")
    xd = dev_array(bits, fmt if fmt != "float32" else None)
    for off in (0, 1, 3, 7):
        for n in (0, 1, 2, 15, 16, 17, 63, 64, 65, 1000, 4097, 65537):
            if off + n > bits.size:
                continue
            qs = q[off:off + n]
            g = hm.reduce_compensated(k, n, [xd[off:off + n]], post_scale=1.0 / scale).item()
            o = oracle.exact_sum(qs) / scale
            assert abs(g - o) <= 1e-6 * float(np.sum(np.abs(qs))) / scale + 1e-300, (fmt, off, n)
            gn = hm.norm2(k, n, [xd[off:off + n]], post_scale=1.0 / scale).item()
            on = oracle.norm2(qs) / scale
            assert abs(gn - on) <= 1e-6 * on + 1e-300, (fmt, off, n, gn, on)


def test_compensated_computed_map_and_scalar_fallback(dev):
    rng = np.random.default_rng(22)
    n = 100003
    x = rng.standard_normal(n).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    sig = "float: const float *x, const float *y"
    for expr in ("x[i] * y[i]", "x[n - 1 - i] * y[i]"):
        k = hm.compile(expr, sig)
        g = hm.reduce_compensated(k, n, [dev_array(x), dev_array(y)]).item()
        r = oracle.reduce(sig.replace("float:", "double:"), expr, "a+b", "0", n, [x, y])
        # each product rounds once in float (the map is evaluated in float)
        rf = oracle.reduce(sig, expr, "a+b", "0", n, [x, y])
        assert abs(g - r.value) <= 1e-6 * r.abs_sum + 2 * rf.err_sum, expr


def test_norm_scaling_handles_extreme_magnitudes(dev):
    # float32 values near 1e30: squares overflow float unless scaled
    x = np.array([3e30, -4e30, 1e-30], np.float32)
    k = hm.compile("x[i]", "float: const float *x")
    g = hm.norm2(k, 3, [dev_array(x)], passes=2).item()
    assert abs(g - oracle.norm2(x)) <= 1e-6 * oracle.norm2(x)
    assert math.isinf(hm.norm2(k, 3, [dev_array(x)], passes=1).item())
    # tiny magnitudes: squares underflow float unless scaled
    t = np.array([3e-30, 4e-30], np.float32)
    g = hm.norm2(k, 2, [dev_array(t)], passes=2).item()
    assert abs(g - oracle.norm2(t)) <= 1e-6 * oracle.norm2(t)
    # zeros, NaN, infinity
    z = np.zeros(100, np.float32)
    assert hm.norm2(k, 100, [dev_array(z)]).item() == 0.0
    assert hm.reduce_compensated(k, 0, [dev_array(z)]).item() == 0.0
    assert hm.norm2(k, 0, [dev_array(z)]).item() == 0.0
    nan = np.array([1.0, np.nan, 2.0], np.float32)
    assert math.isnan(hm.norm2(k, 3, [dev_array(nan)]).item())
    assert math.isnan(hm.reduce_compensated(k, 3, [dev_array(nan)]).item())
    inf = np.array([1.0, np.inf], np.float32)
    assert hm.norm2(k, 2, [dev_array(inf)]).item() == math.inf
    assert hm.reduce_compensated(k, 2, [dev_array(inf)]).item() == math.inf
    big = np.full(1000, 3e38, np.float32)            # the float sum overflows
    assert hm.reduce_compensated(k, 1000, [dev_array(big)]).item() == math.inf
    mixed = np.array([np.inf, -np.inf, 1.0], np.float32)
    assert math.isnan(hm.reduce_compensated(k, 3, [dev_array(mixed)]).item())


def test_precision_entry_points_reject_wrong_handles(dev):
    x = torch.zeros(10, device=dev)
    k = hm.compile("x[i]", "double: const float *x")
    with pytest.raises(hm.MismatchError):
        hm.reduce_compensated(k, 10, [x])
    e = hm.compile("z[i] = x[i]", "float *z, const float *x")
    with pytest.raises(hm.MismatchError):
        hm.norm2(e, 10, [x, x])
    k = hm.compile("x[i]", "float: const float *x")
    with pytest.raises(hm.InvalidError):
        hm.norm2(k, 10, [x], passes=3)
