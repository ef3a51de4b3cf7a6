"""Host logic of the benchmark (no GPU): the one-GPU contract, the CPU leg
(the oracle timed on bounded samples, and as the checker of timed results)
and the lookup of committed HBM counters by kernel symbol."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_leg_baseline_and_accuracy():
    """The CPU leg's worker pool: the oracle timed on one core and on all the
    leg's cores, and the plain results checked against it (a wrong count and
    a wrong lane are reported)."""
    rng = np.random.default_rng(0)
    n = 5000
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    k = rng.integers(0, 1 << 20, n, dtype=np.int32)
    leg = bench.CpuLeg(x, y, k, n)
    try:
        res = leg.baseline(2048, 4096, reps=3)
        assert res["kind"] == "oracle" and res["unit"] == "GB/s" and res["median_of"] == 3
        assert res["value"] > 0 and res["single_core"]["value"] > 0
        assert res["cores"] == min(16, len(os.sched_getaffinity(0))) and res["host_cpus"] >= 1
        assert res["sample"].startswith("first 4096 elements")
        # float32 results computed on the host stand in for the GPU's
        bench._LEG["z"]["E1"][:] = np.float32(2.5) * x - np.float32(0.5) * y
        bench._LEG["z"]["E2"][:] = np.sqrt(x * x + y * y)
        count = int(np.count_nonzero(k % 7 == 3))
        plain = {"R1": count, "R2": int(k.astype(np.int64).sum()), "R3": float(x.max())}
        good = leg.accuracy({"plain": plain})
        assert good["all_ok"], good
        assert good["plain"]["E1"]["lanes_checked"] == n and good["plain"]["R2"]["exact_match"]
        bench._LEG["z"]["E2"][17] += np.float32(1e-3)
        bad = leg.accuracy({"plain": dict(plain, R1=count + 1)})
        assert not bad["all_ok"]
        assert not bad["plain"]["R1"]["exact_match"] and bad["plain"]["E2"]["lanes_outside_bound"] == 1
    finally:
        leg.close()


def test_counter_traffic_by_symbol():
    path = os.path.join(ROOT, bench.COUNTERS_MD)
    rows = [ln for ln in open(path) if ln.startswith("| e1_lincomb_ew_")]
    assert rows
    sym = rows[0].split("|")[1].strip()
    t = bench.counter_traffic(sym)
    assert t is not None and abs(t - 12 * 2 ** 28) <= 0.01 * 12 * 2 ** 28
    assert bench.counter_traffic("e1_lincomb_ew_00000000") is None


def test_profile_commands_are_valid_bench_invocations(monkeypatch):
    # every committed rocprofv3 summary names the command that made it; the
    # program after "--" is this benchmark, with options it still accepts
    import glob
    import shlex
    cmds = []
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if "rocprofv3" in line and " -- " in line:
                cmds.append((os.path.basename(path), line.split(" -- ", 1)[1].strip()))
    assert len(cmds) >= 10
    for name, cmd in cmds:
        argv = shlex.split(cmd)
        assert argv[:2] == ["python", "bench.py"], (name, cmd)
        monkeypatch.setattr(sys, "argv", argv[1:])
        args = bench.parse()
        assert args.gpus == 1, (name, cmd)
