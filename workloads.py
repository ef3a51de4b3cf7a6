"""Seeded synthetic inputs for the tests, the smoke check and the benchmark.

This module only draws and lays out random inputs (numpy ``default_rng``
streams; the 16- and 8-bit float inputs are rounded from float32 by torch's
CPU conversions).  It holds none of the arithmetic of the elementwise or
map-reduce method, and it is shared by both sides of every parity check: the
same bytes go to the GPU library and to the CPU oracle.

Workloads (the paper publishes no data sets; its listings use small random or
``arange`` arrays, which the tests reuse):

* ``dot_1m``: n = 2**20 float32 x, y ~ U[-1, 1], seed 0 -- one map-reduce dot.
* ``plain_at_scale``: n = 2**28; x, y float32 ~ U[-1, 1] (seed 1),
  k int32 ~ U{0 .. 2**20 - 1} (seed 2).
* ``precision``: n = 2**27 values lognormal(0, 3) with random signs, and a
  cancellation case [x; -x (1 + eps)], eps ~ U[-1e-3, 1e-3] (seed 3),
  scaled by a power of two per format, rounded to float32 (the "original"
  tensor) and then to bfloat16, half or FP8-E4M3 (saturating at 448).
* ``segments``: 4096 segment lengths lognormal with median 2**12 and sigma
  sqrt(2 ln 4) (so the mean is 2**14), rounded and clipped to [1, 2**20]
  (seed 4), total 62,032,791; x, y float32 ~ U[-1, 1] drawn after the lengths.
* ``serving``: a resident pool of 2**24 x, y ~ U[-1, 1] and w ~ U[0, 1)
  (float32 and bfloat16, seed 5) and a Poisson schedule per rate (seed
  [5, rate]): sizes floor(2^U), U ~ U[10, 24], one of 8 templates uniformly,
  float32 or bfloat16 with probability 1/2, a random offset into the pool.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

N_DOT = 1 << 20
N_PLAIN = 1 << 28
N_PRECISION = 1 << 27
N_SEGMENTS = 4096

E1 = ("float *z, const float *x, const float *y", "z[i] = 2.5f*x[i] - 0.5f*y[i]")
E2 = ("float *z, const float *x, const float *y", "z[i] = sqrtf(x[i]*x[i] + y[i]*y[i])")
R_COUNT = ("long: const int *k", "k[i] % 7 == 3", "a+b", "0")
R_SUM = ("long: const int *k", "k[i]", "a+b", "0")
R_MAX = ("float: const float *x", "x[i]", "max(a,b)", "-INFINITY")
DOT = ("float: const float *x, const float *y", "x[i]*y[i]", "a+b", "0")


def uniform_f32(rng, n, lo=-1.0, hi=1.0):
    return rng.uniform(lo, hi, n).astype(np.float32)


def dot_1m(n=N_DOT):
    rng = np.random.default_rng(0)
    x = uniform_f32(rng, n)
    y = uniform_f32(rng, n)
    return x, y


def plain_xy(n=N_PLAIN):
    rng = np.random.default_rng(1)
    x = uniform_f32(rng, n)
    y = uniform_f32(rng, n)
    return x, y


def plain_k(n=N_PLAIN):
    rng = np.random.default_rng(2)
    return rng.integers(0, 1 << 20, n, dtype=np.int32)


# -------------------------------------------------------------- complex
N_COMPLEX = 1 << 27
C_AXPBY = ("complex64 *z, complex64 a, const complex64 *x, complex64 b, const complex64 *y",
           "z[i] = a*x[i] + b*y[i]")
C_DOT = ("complex64: const complex64 *x, const complex64 *y", "conj(x[i]) * y[i]", "a+b", "0")
C_SUM = ("complex64: const complex64 *x", "x[i]", "a+b", "0")
C_A, C_B = 0.75 - 1.25j, -0.5 + 0.25j


def complex_xy(n=N_COMPLEX, seed=11):
    """x, y complex64 with real and imaginary parts ~ U[-1, 1] float32."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(2):
        v = np.empty(n, np.complex64)
        v.real = uniform_f32(rng, n)
        v.imag = uniform_f32(rng, n)
        out.append(v)
    return out


# -------------------------------------------------------------- precision
FMAX_SCALE = {"bfloat16": None, "float16": 2.0 ** 15, "fp8_e4m3": 448.0}


def precision_values(n=N_PRECISION, case="lognormal"):
    """float64 values of the precision workload (before any scaling)."""
    rng = np.random.default_rng(3)
    if case == "lognormal":
        mag = rng.lognormal(0.0, 3.0, n)
        sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
        return mag * sign
    if case == "cancel":
        h = n // 2
        mag = rng.lognormal(0.0, 3.0, h)
        sign = np.where(rng.random(h) < 0.5, -1.0, 1.0)
        x = mag * sign
        eps = rng.uniform(-1e-3, 1e-3, h)
        return np.concatenate([x, -x * (1.0 + eps)])
    raise ValueError(case)


@dataclass
class Quantized:
    fmt: str                # 'bfloat16' | 'float16' | 'fp8_e4m3'
    bits: np.ndarray        # raw storage (uint16 or uint8)
    original: np.ndarray    # float32 values before rounding to fmt (already scaled)
    scale: float            # power of two applied before rounding (value = stored / scale)


def power_of_two_scale(fmt, values):
    fmax = FMAX_SCALE[fmt]
    if fmax is None:
        return 1.0
    amax = float(np.max(np.abs(values)))
    if amax == 0.0:
        return 1.0
    return 2.0 ** math.floor(math.log2(fmax / amax))


def quantize(fmt, values64):
    import torch
    scale = power_of_two_scale(fmt, values64)
    original = (values64 * scale).astype(np.float32)
    t = torch.from_numpy(original)
    if fmt == "bfloat16":
        bits = t.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    elif fmt == "float16":
        bits = t.to(torch.float16).view(torch.int16).numpy().view(np.uint16)
    elif fmt == "fp8_e4m3":
        bits = t.clamp(-448.0, 448.0).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    else:
        raise ValueError(fmt)
    return Quantized(fmt, bits.copy(), original, scale)


# -------------------------------------------------------------- segments
SEGMENT_SIGMA = math.sqrt(2.0 * math.log(4.0))


def segments(nseg=N_SEGMENTS, median=4096.0, sigma=SEGMENT_SIGMA, max_len=1 << 20, seed=4):
    rng = np.random.default_rng(seed)
    lengths = np.clip(np.rint(rng.lognormal(math.log(median), sigma, nseg)), 1, max_len)
    lengths = lengths.astype(np.int64)
    offsets = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    x = uniform_f32(rng, total)
    y = uniform_f32(rng, total)
    return offsets, x, y


# -------------------------------------------------------------- serving
N_POOL = 1 << 24
SERVING_RATES = (2000, 10000, 50000)


def serving_pool(n=N_POOL, seed=5):
    """Device-resident input pool: x, y ~ U[-1, 1], w ~ U[0, 1), float32 and
    their bfloat16 roundings (torch's CPU conversion, round to nearest even)."""
    import torch
    rng = np.random.default_rng(seed)
    f32 = {"x": uniform_f32(rng, n), "y": uniform_f32(rng, n),
           "w": rng.uniform(0.0, 1.0, n).astype(np.float32)}
    bf16 = {k: torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
            for k, v in f32.items()}
    return f32, bf16


def serving_schedule(rate, duration_s, seed=5, pool_n=N_POOL, log2_min=10, log2_max=24):
    """Poisson arrivals at `rate` jobs/s for `duration_s`; per job: n = floor(2^U),
    U ~ U[log2_min, log2_max]; template uniform over the 8; dtype float32 or
    bfloat16 with probability 1/2; a random offset into the pool."""
    rng = np.random.default_rng([seed, int(rate)])
    count = int(rate * duration_s * 1.2) + 16
    arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
    arrivals = arrivals[arrivals < duration_s]
    m = arrivals.size
    n = np.floor(2.0 ** rng.uniform(log2_min, log2_max, m)).astype(np.int64)
    n = np.minimum(n, pool_n)
    tmpl = rng.integers(0, 8, m).astype(np.int32)
    bf16 = rng.random(m) < 0.5
    offset = (rng.random(m) * (pool_n - n + 1)).astype(np.int64)
    return {"arrival_ns": (arrivals * 1e9).astype(np.int64), "n": n, "tmpl": tmpl,
            "bf16": bf16, "offset": offset}
