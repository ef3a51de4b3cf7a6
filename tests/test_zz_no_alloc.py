"""The segmented map-reduce's no-allocation entry point, through the C ABI:
on two calls in a row (the second over fewer segments and elements) its
results equal those of hipmr_reduce_segmented with a caller workspace bit
for bit (same kernels, same geometry), and sampled segments match the
oracle; a call before the kernels are on the device, and segments that
need more than the static scratch array, are refused."""

import numpy as np
import pytest

from gpu_util import assert_reduce, dev_array, host_bits, need_gpu, torch
import oracle
import paper_1304_5553_amd as hm
import workloads

pytestmark = pytest.mark.gpu

SIG = "float: const float *x, const float *y"
OPS = {"sum": ("x[i]", "a+b", "0"), "max": ("x[i]", "max(a,b)", "-INFINITY"),
       "dot": ("x[i]*y[i]", "a+b", "0")}


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def inputs(nseg, seed):
    """Lognormal segment lengths as in the batching workload, fewer of them."""
    rng = np.random.default_rng(seed)
    sigma = np.sqrt(2 * np.log(4))
    lens = np.clip(np.rint(rng.lognormal(np.log(2 ** 12), sigma, nseg)), 1, 1 << 20).astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    total = int(offsets[-1])
    x = rng.uniform(-1, 1, total).astype(np.float32)
    y = rng.uniform(-1, 1, total).astype(np.float32)
    return offsets, x, y


@pytest.mark.parametrize("op", list(OPS))
def test_noalloc_equals_workspace_entry_point_twice(dev, op):
    mp, comb, neu = OPS[op]
    k = hm.compile(mp, SIG, name=f"noalloc_{op}")
    runs = [inputs(4096, 4), inputs(600, 41)]      # the second call is smaller
    devs = [(torch.from_numpy(o).to(dev), dev_array(x), dev_array(y), o, x, y) for o, x, y in runs]
    # the allocating entry point once on this device builds and loads the kernels
    for od, xd, yd, o, x, y in devs:
        ref = torch.empty(len(o) - 1, device=dev)
        hm.reduce_segmented(k, comb, neu, od, x.size, [xd, yd], ref)
    torch.cuda.synchronize()
    for call, (od, xd, yd, o, x, y) in enumerate(devs):
        need = hm.segmented_workspace_bytes(k, len(o) - 1, x.size)
        assert need <= hm.hipmr.noalloc_scratch_bytes()
        ref = torch.full((len(o) - 1,), float("nan"), device=dev)
        got = torch.full((len(o) - 1,), float("nan"), device=dev)
        hm.reduce_segmented(k, comb, neu, od, x.size, [xd, yd], ref)
        hm.hipmr.reduce_segmented_noalloc(k, comb, neu, od, x.size, [xd, yd], got)
        torch.cuda.synchronize()
        g, r = host_bits(got), host_bits(ref)
        assert np.array_equal(g.view(np.uint32), r.view(np.uint32)), f"{op} call {call}"
        for s in range(0, len(o) - 1, 37):
            a, b = int(o[s]), int(o[s + 1])
            res = oracle.reduce(SIG, mp, comb, neu, b - a, [x[a:b], y[a:b]])
            assert_reduce(float(g[s]), res, f"{op} call {call} segment {s}")


def test_noalloc_refuses_kernels_not_on_the_device(dev):
    tag = np.random.default_rng().integers(1 << 30)
    k = hm.compile("x[i] * 0.5f", "float: const float *x", name=f"noalloc_cold_{tag}")
    od = torch.tensor([0, 10, 20], dtype=torch.int64, device=dev)
    x = torch.ones(20, device=dev)
    out = torch.empty(2, device=dev)
    with pytest.raises(hm.InvalidError):
        hm.hipmr.reduce_segmented_noalloc(k, "a+b", "0", od, 20, [x], out)
    hm.reduce_segmented(k, "a+b", "0", od, 20, [x], out)
    got = torch.empty(2, device=dev)
    hm.hipmr.reduce_segmented_noalloc(k, "a+b", "0", od, 20, [x], got)
    torch.cuda.synchronize()
    assert host_bits(got).tolist() == [5.0, 5.0]


def test_noalloc_refuses_more_than_its_scratch(dev):
    """Refused on the host before any launch: the array x is never read, so
    the C ABI is called directly (the binding would first check its length)."""
    import ctypes
    k = hm.compile("x[i]", "float: const float *x", name="noalloc_big")
    cap = hm.hipmr.noalloc_scratch_bytes()
    total = cap * 64 // 8                     # about cap / 8 tiles of 64 elements: too many
    assert hm.segmented_workspace_bytes(k, 1, total) > cap
    od = torch.tensor([0, total], dtype=torch.int64, device=dev)
    x = torch.empty(1, device=dev)
    out = torch.empty(1, device=dev)
    keep, ptrs = k.marshal([x])
    st = hm.hipmr.lib().hipmr_reduce_segmented_noalloc(
        k.handle, b"a+b", b"0", 1, ctypes.c_void_p(od.data_ptr()), total, ptrs,
        ctypes.c_void_p(out.data_ptr()), None, None)
    assert st == hm.WorkspaceError.code
    assert b"static scratch array" in hm.hipmr.lib().hipmr_last_error()
