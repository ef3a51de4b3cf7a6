"""The seeded input recipes (no GPU): the batching lengths pinned by their
totals, the serving schedule's ranges, the precision and complex inputs'
shapes and scales, and repeatability."""

import numpy as np

import workloads


def test_segment_lengths_are_pinned():
    # lognormal lengths, median 2^12, sigma = sqrt(2 ln 4) (mean 2^14),
    # rounded and clipped to [1, 2^20], seed 4
    offsets, x, y = workloads.segments()
    lengths = np.diff(offsets)
    assert len(lengths) == 4096 and offsets[0] == 0
    assert int(offsets[-1]) == 62032791 == x.size == y.size
    assert int(lengths.max()) == 1 << 20 and int(lengths.min()) == 5
    assert int(np.median(lengths)) == 4145
    assert abs(workloads.SEGMENT_SIGMA - np.sqrt(2 * np.log(4))) < 1e-12
    assert x.dtype == np.float32 and float(np.abs(x).max()) <= 1.0


def test_serving_schedule_ranges():
    for rate in (2000, 50000):
        s = workloads.serving_schedule(rate, 0.5)
        m = len(s["n"])
        assert abs(m - rate * 0.5) < 5 * np.sqrt(rate * 0.5)
        assert np.all(np.diff(s["arrival_ns"]) >= 0) and s["arrival_ns"][-1] < 0.5e9
        assert s["n"].min() >= 1 << 10 and s["n"].max() < 1 << 24
        assert np.all(s["offset"] >= 0) and np.all(s["offset"] + s["n"] <= workloads.N_POOL)
        assert set(np.unique(s["tmpl"])) == set(range(8))
        assert 0.4 < s["bf16"].mean() < 0.6
        again = workloads.serving_schedule(rate, 0.5)
        assert all(np.array_equal(s[k], again[k]) for k in s)


def test_precision_inputs_and_scales():
    v = workloads.precision_values(1 << 16)
    assert v.dtype == np.float64 and v.size == 1 << 16
    c = workloads.precision_values(1 << 16, "cancel")
    h = c.size // 2
    rel = np.abs(c[:h] + c[h:]) / np.abs(c[:h])
    assert rel.max() <= 1e-3 + 1e-15
    for fmt, fmax in (("fp8_e4m3", 448.0), ("float16", 2.0 ** 15)):
        q = workloads.quantize(fmt, v)
        s = q.scale
        assert s == 2.0 ** np.floor(np.log2(s))                 # a power of two
        assert np.abs(v).max() * s <= fmax < 2 * np.abs(v).max() * s
    assert workloads.quantize("bfloat16", v).scale == 1.0


def test_complex_inputs():
    x, y = workloads.complex_xy(1 << 12)
    assert x.dtype == np.complex64 and y.shape == (1 << 12,)
    assert np.abs(x.real).max() <= 1 and np.abs(x.imag).max() <= 1
    assert not np.array_equal(x, y)
    x2, _ = workloads.complex_xy(1 << 12)
    assert np.array_equal(x, x2)
