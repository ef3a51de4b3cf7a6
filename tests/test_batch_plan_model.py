"""The segmented reduce's tile capacity, on the CPU: a host model of the
planner's arithmetic (clamp each offset pair into [0, total_n], tiles of the
segment, 64-bit running sum capped at the capacity) shows that for
non-decreasing offsets the capacity nseg + total_n / 64 + 1 always holds
every tile of every geometry, and that for any offsets at all (overlapping,
decreasing, out of range) the capped table stays non-decreasing and inside
the workspace.  The capacity itself is the one the library sizes the
workspace for (hipmr_segmented_workspace_bytes)."""

import numpy as np
import pytest

import paper_1304_5553_amd as hm


def clamp(a0, b0, total, head, v):
    a = min(max(a0, 0), total)
    b = a if b0 < a else min(b0, total)
    r = (head - a) % v
    ab = min(a + r, b)
    return a, b, ab


def tiles(a, b, ab, t):
    if b == a:
        return 0
    return max(1, -(-(b - ab) // t))


def plan(offsets, total, head, v, ipt, cap):
    """tile_start as the planner writes it: exclusive prefix of the tile
    counts, each entry and the final total capped at `cap`."""
    t = 64 * v * ipt
    run, out = 0, []
    for s in range(len(offsets) - 1):
        out.append(min(run, cap))
        run += tiles(*clamp(int(offsets[s]), int(offsets[s + 1]), total, head, v), t)
    out.append(min(run, cap))
    return out, run


def capacity(nseg, total):
    return nseg + (total + 63) // 64 + 1


GEOMETRIES = [(v, ipt, head) for v in (1, 2, 4, 8, 16) for ipt in (1, 2, 4, 8) for head in (0, 1, 3)
              if head < v or head == 0]


@pytest.mark.parametrize("seed", range(6))
def test_capacity_holds_every_tile_of_valid_offsets(seed):
    rng = np.random.default_rng(seed)
    nseg = int(rng.integers(1, 3000))
    kind = seed % 3
    if kind == 0:       # many tiny segments: one (partial) tile each
        lens = rng.integers(0, 3, nseg)
    elif kind == 1:     # lognormal lengths as in the batching workload
        lens = np.clip(np.rint(rng.lognormal(np.log(2 ** 8), 1.665, nseg)), 1, 1 << 16).astype(np.int64)
    else:               # lengths just past a tile boundary
        lens = 64 * rng.integers(0, 4, nseg) + 1
    offsets = np.concatenate([[0], np.cumsum(lens)])
    total = int(offsets[-1])
    cap = capacity(nseg, total)
    for v, ipt, head in GEOMETRIES:
        ts, uncapped = plan(offsets, total, head, v, ipt, cap)
        assert uncapped <= cap, (v, ipt, head)
        assert ts[-1] == uncapped


@pytest.mark.parametrize("seed", range(6))
def test_any_offsets_stay_inside_the_capacity(seed):
    rng = np.random.default_rng(100 + seed)
    nseg = int(rng.integers(1, 500))
    total = int(rng.integers(1, 1 << 22))
    if seed == 0:       # alternating [0, N, 0, N, ...]: every other segment covers everything
        offsets = np.array([0 if s % 2 == 0 else total for s in range(nseg + 1)])
    else:               # arbitrary values, in and out of range
        offsets = rng.integers(-total, 2 * total, nseg + 1)
    cap = capacity(nseg, total)
    for v, ipt, head in GEOMETRIES[::5]:
        ts, uncapped = plan(offsets, total, head, v, ipt, cap)
        assert all(0 <= x <= cap for x in ts)
        assert all(a <= b for a, b in zip(ts, ts[1:]))
        if seed == 0 and nseg >= 4:
            assert uncapped > cap            # the case the cap exists for


def test_library_sizes_the_workspace_for_that_capacity():
    k = hm.compile("x[i]", "float: const float *x", name="plan_model")
    for nseg, total in ((1, 0), (1, 1), (4096, 62032791), (100, 1 << 30), (7, 65)):
        table = -(-((nseg + 1) * 4) // 256) * 256
        assert hm.segmented_workspace_bytes(k, nseg, total) == table + 8 * capacity(nseg, total)
