"""Helpers shared by the GPU parity tests: device placement and the
comparison rules (bit-exact for integers and exact float results; the
oracle's per-element bound for computed floats; the map-reduce gates)."""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1304_5553_amd as hm  # noqa: E402

LOWP_TORCH = {"bfloat16": torch.bfloat16, "float16": torch.float16, "fp8_e4m3": torch.float8_e4m3fn}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def dev_array(a, storage=None, device="cuda:0"):
    """Numpy storage array -> device tensor with the same bytes."""
    t = torch.from_numpy(np.ascontiguousarray(a))
    if storage in LOWP_TORCH:
        t = t.view(torch.int16 if t.element_size() == 2 else torch.uint8).view(LOWP_TORCH[storage])
    return t.to(device)


def host_bits(t):
    """Device tensor -> numpy array of its raw storage (low-precision as bits)."""
    t = t.detach().cpu()
    if t.dtype in (torch.bfloat16, torch.float16):
        return t.view(torch.int16).numpy().view(np.uint16)
    if t.dtype == torch.float8_e4m3fn:
        return t.view(torch.uint8).numpy()
    if t.dtype == torch.uint32:
        return t.view(torch.int32).numpy().view(np.uint32)
    return t.numpy()


def decoded(t, storage):
    bits = host_bits(t)
    if storage == "bfloat16":
        return oracle.decode_bf16(bits)
    if storage == "float16":
        return oracle.decode_f16(bits)
    if storage == "fp8_e4m3":
        return oracle.decode_e4m3fn(bits)
    if bits.dtype.kind == "c":
        return bits.astype(np.complex128)
    return bits.astype(np.float64) if bits.dtype.kind == "f" else bits.astype(np.int64)


def assert_lanes(got_t, ref: "oracle.Lanes", storage, lanes=None, what=""):
    """GPU output values at ref.lanes vs the oracle."""
    g = decoded(got_t, storage)
    idx = ref.lanes if lanes is None else lanes
    g = g[idx]
    ok = ~ref.u & ref.written
    if ref.t in ("int", "unsigned", "long"):
        bad = np.nonzero(ok & (g.astype(np.int64) != ref.v))[0]
    else:
        with np.errstate(invalid="ignore"):
            diff = np.abs(g - ref.v)
            same_special = (np.isnan(g) & np.isnan(ref.v)) | (np.isinf(ref.v) & (g == ref.v))
            bad = np.nonzero(ok & ~same_special & ~(diff <= 2 * ref.e))[0]
    if bad.size:
        k = bad[0]
        raise AssertionError(
            f"{what}: {bad.size} mismatches; first at i={idx[k]}: gpu={g[k]!r} oracle={ref.v[k]!r} "
            f"bound={2 * ref.e[k] if ref.e.size else 0!r}")
    return int(np.count_nonzero(ok))


def assert_reduce(got, r: "oracle.ReduceResult", what=""):
    """Map-reduce gates: exact where the result is unique, else
    |g - o| <= 2e-6 * sum|t| + 2 * sum(e) for float sums."""
    if isinstance(got, torch.Tensor):
        got = got.item()
    if r.exact or r.op in ("max", "min") and r.err_sum == 0:
        if isinstance(r.value, float) and math.isnan(r.value):
            assert math.isnan(got), f"{what}: gpu {got} vs oracle NaN"
            return
        assert got == r.value, f"{what}: gpu {got!r} != oracle {r.value!r}"
        if isinstance(r.value, float) and r.value == 0.0:
            assert math.copysign(1, got) == math.copysign(1, r.value), f"{what}: sign of zero"
        return
    if r.op in ("max", "min"):
        assert abs(got - r.value) <= 2 * r.err_sum, f"{what}: gpu {got} vs oracle {r.value}"
        return
    tol = 2e-6 * r.abs_sum + 2 * r.err_sum
    assert abs(got - r.value) <= tol, (
        f"{what}: gpu {got!r} vs oracle {r.value!r}: |diff|={abs(got - r.value):.3e} > tol {tol:.3e}")


def reduce_on_gpu(kernel, combine, neutral, n, args, device="cuda:0", config=None, out=None):
    if out is None:
        out = torch.empty((), dtype=hm.torch_dtype(kernel.result_dtype), device=device)
    hm.reduce(kernel, kernel.expr, combine, neutral, n, args, out, config=config)
    torch.cuda.synchronize()
    return out
