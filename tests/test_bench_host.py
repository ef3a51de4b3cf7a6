"""Host logic of the benchmark (no GPU): the one-GPU contract, the CPU
baseline leg (the oracle on a bounded sample) and the lookup of committed
HBM counters by kernel symbol."""

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


def test_cpu_baseline_leg():
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, 5000).astype(np.float32)
    y = rng.uniform(-1, 1, 5000).astype(np.float32)
    k = rng.integers(0, 1 << 20, 5000, dtype=np.int32)
    res = bench.cpu_baseline(x, y, k, 4096)
    assert res["kind"] == "oracle" and res["unit"] == "GB/s"
    assert res["value"] > 0 and res["cores"] >= 1
    assert res["sample"].startswith("first 4096 elements")


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
