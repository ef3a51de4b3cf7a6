"""GPU parity of the lazy expression front end: an operator tree fused into
one generated kernel (and, for comparison, one kernel per operator) against
the oracle's evaluation of the rendered statement; fused reductions against
the oracle's map-reduce."""

import numpy as np
import pytest

from gpu_util import assert_lanes, assert_reduce, need_gpu, torch
import oracle
from paper_1304_5553_amd import lazy as lz
from test_lazy import EXPRS, leaves

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def host_arrays(ts):
    return [t.view(torch.int16).numpy().view(np.uint16) if t.dtype == torch.bfloat16 else t.numpy()
            for t in ts]


@pytest.mark.parametrize("name", list(EXPRS))
@pytest.mark.parametrize("dts", [("float32",) * 3, ("bfloat16", "float32", "int32")])
@pytest.mark.parametrize("fused", [True, False])
def test_lazy_elementwise(dev, name, dts, fused):
    n = 100003
    ts = leaves(n, 11, dts)
    ds = [t.to(dev) for t in ts]
    node = EXPRS[name](*(lz.lazy(t) for t in ds))
    got = node.eval(fused=fused)
    torch.cuda.synchronize()
    dtypes, stmt, lv = lz.elementwise_source(node)
    order = [next(k for k, d in enumerate(ds) if d is t) for t in lv]
    ref = oracle.elementwise(dtypes, stmt, n, [np.zeros(n, np.float32)] + host_arrays([ts[k] for k in order]))
    assert_lanes(got, ref["out"], "float32", what=f"{name} {dts} fused={fused}")


@pytest.mark.parametrize("red", ["sum", "max", "min", "dot"])
def test_lazy_reductions(dev, red):
    n = 200001
    ts = leaves(n, 12)
    ds = [t.to(dev) for t in ts]
    x, y, w = (lz.lazy(t) for t in ds)
    node = x * y - 0.5 * w if red != "dot" else None
    if red == "dot":
        out = lz.dot(x, lz.sqrt(y))
        node, comb, neu = x * lz.sqrt(y), "a+b", "0"
    else:
        out = getattr(node, red)()
        comb, neu = {"sum": ("a+b", "0"), "max": ("max(a,b)", "-INFINITY"),
                     "min": ("min(a,b)", "INFINITY")}[red]
    torch.cuda.synchronize()
    dtypes, expr, lv = lz.reduce_source(node)
    order = [next(k for k, d in enumerate(ds) if d is t) for t in lv]
    r = oracle.reduce(dtypes, expr, comb, neu, n, host_arrays([ts[k] for k in order]))
    assert_reduce(out, r, red)


def test_lazy_shifted_reduction(dev):
    # total variation sum |x[i] - x[i+1]| (x[n] read as x[n-1]'s fill of 0):
    # the map's shifted read takes the reduce kernel's shifted chunk loads
    n = 300007
    ts = leaves(n, 13)
    ds = [t.to(dev) for t in ts]
    x = lz.lazy(ds[0])
    node = lz.abs(x - lz.shift(x, 1))
    out = node.sum()
    torch.cuda.synchronize()
    dtypes, expr, lv = lz.reduce_source(node)
    r = oracle.reduce(dtypes, expr, "a+b", "0", n, host_arrays([ts[0]]))
    assert_reduce(out, r, "total variation")


@pytest.mark.parametrize("fused", [True, False])
def test_lazy_timed_expression_full_size_sampled(dev, fused):
    # the timed fused expression at its measured size: z = 2.5 x y +
    # sqrt(x x + y y) - 0.5 w over 2^26 float32 U[-1, 1] values, checked on
    # both ends and a random sample of lanes
    n = 1 << 26
    rng = np.random.default_rng(9)
    xs = [rng.uniform(-1, 1, n).astype(np.float32) for _ in range(3)]
    ds = [torch.from_numpy(a).to(dev) for a in xs]
    x, y, w = (lz.lazy(t) for t in ds)
    node = 2.5 * x * y + lz.sqrt(x * x + y * y) - 0.5 * w
    got = node.eval(fused=fused)
    torch.cuda.synchronize()
    dtypes, stmt, lv = lz.elementwise_source(node)
    order = [next(k for k, d in enumerate(ds) if d is t) for t in lv]
    lanes = np.unique(np.concatenate([np.arange(4096), np.arange(n - 4096, n),
                                      rng.integers(0, n, 1 << 18)]))
    ref = oracle.elementwise(dtypes, stmt, n, [np.zeros(1, np.float32)] + [xs[k] for k in order],
                             lanes=lanes)["out"]
    assert assert_lanes(got, ref, "float32", what=f"lazy 2^26 fused={fused}") == lanes.size
    del ds, got
    torch.cuda.empty_cache()
