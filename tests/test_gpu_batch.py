"""GPU parity of the batching extension: segmented map-reduce in one
persistent launch sequence (device planner, tile stage, per-segment fold),
graph capture and replay, and the autotuner.  Workload: 4096 segments with
lognormal lengths (median 2**12, clipped to [1, 2**20], total 62,032,791)
over float32 x, y ~ U[-1, 1]; sum, max and dot per segment."""

import numpy as np
import pytest

from gpu_util import assert_reduce, dev_array, host_bits, need_gpu, torch
import oracle
import paper_1304_5553_amd as hm
import workloads

pytestmark = pytest.mark.gpu

OPS = {
    "sum": ("float: const float *x, const float *y", "x[i]", "a+b", "0"),
    "max": ("float: const float *x, const float *y", "x[i]", "max(a,b)", "-INFINITY"),
    "dot": ("float: const float *x, const float *y", "x[i]*y[i]", "a+b", "0"),
}


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def seg_data(dev):
    offsets, x, y = workloads.segments()
    return offsets, x, y, dev_array(offsets), dev_array(x), dev_array(y)


@pytest.fixture(scope="module")
def handles():
    return {k: hm.compile(v[1], v[0], name=f"seg_{k}") for k, v in OPS.items()}


def run_seg(k, op, offs_d, total, args, dtype=torch.float32, config=None):
    out = torch.empty(offs_d.numel() - 1, dtype=dtype, device=offs_d.device)
    hm.reduce_segmented(k, OPS[op][2], OPS[op][3], offs_d, total, args, out, config=config)
    torch.cuda.synchronize()
    return out


def check_segments(op, got, offsets, x, y, what, stride=1):
    sig, mp, comb, neu = OPS[op]
    g = host_bits(got)
    for s in range(0, len(offsets) - 1, stride):
        a, b = int(offsets[s]), int(offsets[s + 1])
        r = oracle.reduce(sig, mp, comb, neu, b - a, [x[a:b], y[a:b]])
        assert_reduce(float(g[s]), r, f"{what} segment {s} [{a}, {b})", bare=True)


@pytest.mark.parametrize("op", ["sum", "max", "dot"])
def test_segments_config(dev, seg_data, handles, op):
    offsets, x, y, od, xd, yd = seg_data
    assert int(offsets[-1]) == 62032791 and len(offsets) == 4097
    got = run_seg(handles[op], op, od, x.size, [xd, yd])
    check_segments(op, got, offsets, x, y, op)
    again = run_seg(handles[op], op, od, x.size, [xd, yd])
    assert torch.equal(got, again)                      # bitwise repeatable


def test_segment_result_independent_of_other_segments(dev, seg_data, handles):
    offsets, x, y, od, xd, yd = seg_data
    base = host_bits(run_seg(handles["dot"], "dot", od, x.size, [xd, yd]))
    # split every other segment in two and drop the last quarter of segments:
    # the untouched segments must give bit-identical results
    keep = list(range(0, 3072, 2))
    new_off, idx_of = [], {}
    for s in range(3072):
        a, b = int(offsets[s]), int(offsets[s + 1])
        if s % 2 == 0:
            idx_of[s] = len(new_off)
            new_off.append(a)
        else:
            new_off += [a, (a + b) // 2]
    new_off.append(int(offsets[3072]))
    od2 = dev_array(np.array(new_off, np.int64))
    got = host_bits(run_seg(handles["dot"], "dot", od2, x.size, [xd, yd]))
    for s in keep:
        assert got[idx_of[s]] == base[s], s


def test_integer_segments_sum_to_the_whole(dev):
    rng = np.random.default_rng(31)
    k = rng.integers(-1000, 1000, 300001).astype(np.int32)
    cuts = np.sort(rng.integers(0, k.size, 999))
    offsets = np.concatenate([[0], cuts, [k.size]]).astype(np.int64)
    h = hm.compile("k[i]", "long: const int *k")
    out = torch.empty(len(offsets) - 1, dtype=torch.int64, device=dev)
    hm.reduce_segmented(h, "a+b", "0", dev_array(offsets), k.size, [dev_array(k)], out)
    torch.cuda.synchronize()
    g = host_bits(out)
    want = [int(k[a:b].astype(np.int64).sum()) for a, b in zip(offsets[:-1], offsets[1:])]
    assert g.tolist() == want
    assert int(g.sum()) == int(k.astype(np.int64).sum())


@pytest.mark.parametrize("case", ["empty_and_tiny", "misaligned", "clamped", "many_segments",
                                  "single", "all_empty"])
def test_segment_edge_cases(dev, handles, case):
    rng = np.random.default_rng(hash(case) % 1000)
    n = 200003
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    if case == "empty_and_tiny":
        lens = rng.choice([0, 0, 1, 2, 3, 5, 17, 64, 1023, 1024, 1025, 5000], 300)
        offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    elif case == "misaligned":
        offsets = np.array([1, 2, 7, 8, 9, 1000, 1003, 4099, 100001, n - 3, n], np.int64)
    elif case == "clamped":      # out-of-range and decreasing offsets are clamped, never read out of bounds
        offsets = np.array([-5, 10, 5, 100, n + 50, n + 100], np.int64)
    elif case == "many_segments":   # more than the LDS tile table holds
        offsets = np.arange(0, n, 17, dtype=np.int64)
    elif case == "single":
        offsets = np.array([0, n], np.int64)
    else:
        offsets = np.array([5, 5, 5, 5], np.int64)
    xd, yd = dev_array(x), dev_array(y)
    for op in ("dot", "max"):
        got = run_seg(handles[op], op, dev_array(offsets), n, [xd, yd])
        g = host_bits(got)
        for s in range(len(offsets) - 1):
            a = min(max(int(offsets[s]), 0), n)
            b = min(max(int(offsets[s + 1]), a), n)
            sig, mp, comb, neu = OPS[op]
            r = oracle.reduce(sig, mp, comb, neu, b - a, [x[a:b], y[a:b]])
            assert_reduce(float(g[s]), r, f"{case} {op} segment {s}")


def test_zero_segments_is_a_no_op(dev, handles):
    od = torch.zeros(1, dtype=torch.int64, device=dev)
    out = torch.empty(0, device=dev)
    x = torch.zeros(4, device=dev)
    hm.reduce_segmented(handles["sum"], "a+b", "0", od, 4, [x, x], out)
    torch.cuda.synchronize()


def test_graph_capture_and_replay(dev, seg_data, handles):
    offsets, x, y, od, xd, yd = seg_data
    stream = torch.cuda.Stream()
    outs = {op: torch.empty(len(offsets) - 1, dtype=torch.float32, device=dev) for op in OPS}
    ws = {op: torch.empty(hm.segmented_workspace_bytes(handles[op], len(offsets) - 1, x.size),
                          dtype=torch.uint8, device=dev) for op in OPS}
    with torch.cuda.stream(stream):
        def issue():
            for op in OPS:
                hm.reduce_segmented(handles[op], OPS[op][2], OPS[op][3], od, x.size, [xd, yd],
                                    outs[op], workspace_buf=ws[op], stream=stream)
        issue()                                   # warm-up loads the code objects
        stream.synchronize()
        eager = {op: outs[op].clone() for op in OPS}
        graph = hm.Graph()
        with graph.capture(stream):
            issue()
        for rep in range(3):
            for op in OPS:
                outs[op].fill_(float("nan"))
            graph.launch(stream)
            stream.synchronize()
            for op in OPS:
                assert torch.equal(outs[op], eager[op]), (rep, op)
            _ = (xd * 2).sum().item()             # unrelated eager work between replays
        # same graph, new offset values (same count): results follow the offsets
        shifted = offsets.copy()
        shifted[1:-1] += 3
        od.copy_(torch.from_numpy(shifted))
        graph.launch(stream)
        stream.synchronize()
        g = host_bits(outs["max"])
        for s in range(0, len(shifted) - 1, 97):
            a, b = int(shifted[s]), int(shifted[s + 1])
            assert g[s] == np.max(x[a:b]), s
        od.copy_(torch.from_numpy(offsets))
        torch.cuda.synchronize()


def test_concurrent_graph_fork_join(dev, seg_data, handles):
    """The three ops on three streams inside one captured graph (fork / join
    with events), as the benchmark replays them: every replay equals the
    eager results, with eager work and synchronisations in between."""
    offsets, x, y, od, xd, yd = seg_data
    stream = torch.cuda.Stream()
    side = {"max": torch.cuda.Stream(), "dot": torch.cuda.Stream()}
    outs = {op: torch.empty(len(offsets) - 1, dtype=torch.float32, device=dev) for op in OPS}
    ws = {op: torch.empty(hm.segmented_workspace_bytes(handles[op], len(offsets) - 1, x.size),
                          dtype=torch.uint8, device=dev) for op in OPS}

    def one(op, st):
        hm.reduce_segmented(handles[op], OPS[op][2], OPS[op][3], od, x.size, [xd, yd], outs[op],
                            workspace_buf=ws[op], stream=st)

    with torch.cuda.stream(stream):
        def issue():
            fork = torch.cuda.Event()
            fork.record(stream)
            for op, st in side.items():
                st.wait_event(fork)
                one(op, st)
            one("sum", stream)
            for st in side.values():
                join = torch.cuda.Event()
                join.record(st)
                stream.wait_event(join)
        for op in OPS:
            one(op, stream)                       # warm-up loads the code objects
        torch.cuda.synchronize()
        eager = {op: outs[op].clone() for op in OPS}
        graph = hm.Graph()
        with graph.capture(stream):
            issue()
        for rep in range(4):
            for op in OPS:
                outs[op].fill_(float("nan"))
            torch.cuda.synchronize()
            graph.launch(stream)
            stream.synchronize()
            for op in OPS:
                assert torch.equal(outs[op], eager[op]), (rep, op)
            _ = (xd * 2).sum().item()             # unrelated eager work between replays
    torch.cuda.synchronize()


def test_graph_capture_requires_warm_kernels(dev):
    k = hm.compile("x[i] + 1.0f", "float: const float *x", name="cold_capture")
    x = torch.zeros(100, device=dev)
    od = torch.tensor([0, 50, 100], dtype=torch.int64, device=dev)
    out = torch.empty(2, device=dev)
    stream = torch.cuda.Stream()
    graph = hm.Graph()
    with torch.cuda.stream(stream):
        with pytest.raises(hm.InvalidError):
            with graph.capture(stream):
                hm.reduce_segmented(k, "a+b", "0", od, 100, [x], out, stream=stream)
    torch.cuda.synchronize()


def test_autotune_segmented_and_reduce(dev, seg_data, handles):
    offsets, x, y, od, xd, yd = seg_data
    best = hm.autotune_segmented(handles["sum"], "a+b", "0", od, x.size, [xd, yd],
                                 torch.empty(len(offsets) - 1, device=dev), reps=3)
    assert best["block"] in (256, 512) and best["items_per_thread"] in (1, 2, 4, 8)
    got = run_seg(handles["sum"], "sum", od, x.size, [xd, yd], config={"flags": hm.CFG_TUNED})
    check_segments("sum", got, offsets, x, y, "tuned sum", stride=7)
    k = hm.compile("x[i]*y[i]", "float: const float *x, const float *y", name="tuned_dot")
    out = torch.empty((), device=dev)
    default = torch.empty((), device=dev)
    hm.reduce(k, None, "a+b", "0", x.size, [xd, yd], default)
    best = hm.autotune_reduce(k, "a+b", "0", x.size, [xd, yd], out, reps=3)
    assert best["block"] in (256, 512)
    hm.reduce(k, None, "a+b", "0", x.size, [xd, yd], out, config={"flags": hm.CFG_TUNED})
    r = oracle.reduce("float: const float *x, const float *y", "x[i]*y[i]", "a+b", "0", x.size,
                      [x, y])
    assert_reduce(out.item(), r, "tuned dot")
    # without the flag a stored geometry is never applied: the default result is unchanged
    again = torch.empty((), device=dev)
    hm.reduce(k, None, "a+b", "0", x.size, [xd, yd], again)
    torch.cuda.synchronize()
    assert again.item() == default.item()


def test_one_handle_across_tile_table_sizes(dev):
    # regression: a handle first used with a tile table that fits in LDS and
    # then with one that does not must switch to the global-memory table
    rng = np.random.default_rng(33)
    n = 300007
    x = rng.uniform(-1, 1, n).astype(np.float32)
    xd = dev_array(x)
    k = hm.compile("x[i]", "float: const float *x", name="table_sizes")
    for step in (200, 17, 25, 9):
        offsets = np.arange(0, n + 1, step, dtype=np.int64)
        out = torch.empty(len(offsets) - 1, device=dev)
        hm.reduce_segmented(k, "max", "-INFINITY", dev_array(offsets), n, [xd], out)
        torch.cuda.synchronize()
        want = np.array([x[a:b].max() for a, b in zip(offsets[:-1], offsets[1:])], np.float32)
        assert np.array_equal(host_bits(out), want), step


def test_segments_without_common_alignment(dev):
    # x and y misaligned differently: one-element chunks, the most tiles
    rng = np.random.default_rng(34)
    n = 100000
    xb = rng.uniform(-1, 1, n + 8).astype(np.float32)
    yb = rng.uniform(-1, 1, n + 8).astype(np.float32)
    x, y = xb[1:1 + n], yb[2:2 + n]
    xd, yd = dev_array(xb)[1:1 + n], dev_array(yb)[2:2 + n]
    cuts = np.sort(rng.integers(0, n, 300))
    offsets = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    k = hm.compile("x[i]*y[i]", "double: const float *x, const float *y", name="unaligned_dot")
    out = torch.empty(len(offsets) - 1, dtype=torch.float64, device=dev)
    hm.reduce_segmented(k, "a+b", "0", dev_array(offsets), n, [xd, yd], out)
    torch.cuda.synchronize()
    g = host_bits(out)
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        r = oracle.reduce("double: const float *x, const float *y", "x[i]*y[i]", "a+b", "0",
                          b - a, [x[a:b], y[a:b]])
        assert_reduce(float(g[s]), r, f"unaligned segment {s}")


def test_overlapping_offsets_stay_inside_the_workspace(dev):
    """Offsets that are not non-decreasing ([0, N, 0, N, ...]: every other
    segment covers the whole array) describe about nseg/2 * N / T tiles,
    far more than the workspace's capacity nseg + N / 64 + 1.  The planner
    caps the table there: nothing past the workspace is written (a canary
    after it stays intact), and the segments whose tiles all lie below the
    cap are still exact against the oracle."""
    rng = np.random.default_rng(71)
    N, nseg = 1 << 20, 64
    x = rng.uniform(-1, 1, N).astype(np.float32)
    offsets = np.array([0 if s % 2 == 0 else N for s in range(nseg + 1)], dtype=np.int64)
    k = hm.compile("x[i]", "float: const float *x", name="overlap_sum")
    need = hm.segmented_workspace_bytes(k, nseg, N)
    ws = torch.full((need + 65536,), 0x5A, dtype=torch.uint8, device=dev)
    out = torch.full((nseg,), float("nan"), device=dev)
    hm.reduce_segmented(k, "max(a,b)", "-INFINITY", torch.from_numpy(offsets).to(dev), N,
                        [dev_array(x)], out, workspace_buf=ws[:need])
    torch.cuda.synchronize()
    assert bool(torch.all(ws[need:] == 0x5A)), "written past the workspace"
    g = host_bits(out)
    tile = 64 * 4 * 4                      # default geometry: T = 64 lanes x 4 floats x 4 chunks
    cap = nseg + (N + 63) // 64 + 1
    full = cap // (N // tile)             # whole-array segments that fit below the cap
    want = float(np.max(x))
    checked = 0
    for s in range(0, nseg, 2):
        if s // 2 < full:
            assert g[s] == want, s
            checked += 1
    assert checked >= 8
    for s in range(1, nseg, 2):            # decreasing pairs are empty segments
        assert g[s] == -np.inf or s // 2 >= full
