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


NORTH_STAR_REL = 2e-6      # the float sum gate: |g - o| <= 2e-6 * sum |terms|
U24 = 2.0 ** -24


def assert_reduce(got, r: "oracle.ReduceResult", what="", depth=None, bare=False):
    """Map-reduce gates: exact where the result is unique, else for float
    folds |g - o| <= rounds * 2e-6 * sum|t| + 2 * sum(e) + slack (rounds = 1
    for the canonical sum; the oracle's roundings per combination for a
    generic reduce expression).  With `depth` (the longest chain of
    combinations in the kernels' fold tree) the oracle's proved bound
    rounds * u * depth * sum|t| + 2 * sum(e) + slack is asserted as well.
    `bare` asserts the plain 2e-6 * sum|t| with nothing added (the map's own
    rounding, e, counted inside it)."""
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
    diff = abs(got - r.value)
    tol = r.rounds * NORTH_STAR_REL * r.abs_sum + 2 * r.err_sum + r.abs_slack
    assert diff <= tol, (
        f"{what}: gpu {got!r} vs oracle {r.value!r}: |diff|={diff:.3e} > tol {tol:.3e}")
    if bare:
        assert diff <= NORTH_STAR_REL * r.abs_sum, (
            f"{what}: |diff|={diff:.3e} > 2e-6 sum|t| = {NORTH_STAR_REL * r.abs_sum:.3e}")
    if depth is not None:
        proved = r.rounds * U24 * depth * r.abs_sum + 2 * r.err_sum + r.abs_slack
        assert diff <= proved, (
            f"{what}: |diff|={diff:.3e} > proved bound {proved:.3e} at depth {depth}")


def _p2levels(waves):
    """Levels of the LDS stage of the block reduction over `waves` waves."""
    if waves <= 1:
        return 0
    p = 2 if waves <= 2 else 4 if waves <= 4 else 8 if waves <= 8 else 16
    return p.bit_length() - 1


def reduce_depth(n, head=0, vec=4, ipt=4, block=256, blocks_per_cu=2, cus=None):
    """Longest chain of combinations on one map value's path in the plain
    two-stage reduce (vector kernel): a lane folds the head / tail element and
    one chunk of `vec` values per pass into each of its `ipt` accumulators;
    these fold pairwise; the block reduces (6 butterfly steps, then the LDS
    stage); stage 2 folds the G partials, ceil(G/256) per thread, then its
    own block reduction."""
    if cus is None:
        cus = torch.cuda.get_device_properties(0).multi_processor_count
    h = min(head, n)
    nc = (n - h) // vec
    need = max(1, -(-nc // (block * ipt)))
    g = max(1, min(need, blocks_per_cu * cus))
    passes = -(-nc // (g * block * ipt)) if nc else 0
    lane = 2 + passes * vec
    fold = (ipt - 1).bit_length()
    s1 = 6 + _p2levels(block // 64)
    s2 = -(-g // 256) + 6 + _p2levels(256 // 64)
    return lane + fold + s1 + s2


def reduce_on_gpu(kernel, combine, neutral, n, args, device="cuda:0", config=None, out=None):
    if out is None:
        out = torch.empty((), dtype=hm.torch_dtype(kernel.result_dtype), device=device)
    hm.reduce(kernel, kernel.expr, combine, neutral, n, args, out, config=config)
    torch.cuda.synchronize()
    return out
