"""GPU parity of the serving loop's resident mode: one kernel stays on the
device and takes jobs from a descriptor ring in mapped host memory.  Its stop
path (no instance, a stopped instance, an instance that stops when idle),
every job against the oracle, results bitwise equal to the launched paths
(batched and one launch pair per job) and to the same job alone, instances
replaced while a stream runs, empty / one-element / misaligned jobs, budget
admission, the full-size stream, the ring's 48-bit fields, a burst of jobs
due at once and the largest jobs taken."""

import math
import time

import numpy as np
import pytest

from gpu_util import need_gpu, torch
import paper_1304_5553_amd as hm
import workloads
from test_gpu_serving import POOL_N, make_jobs, oracle_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def pool(dev):
    f32, bf16 = workloads.serving_pool(POOL_N)
    dev_f32 = {k: torch.from_numpy(v).to(dev) for k, v in f32.items()}
    dev_bf16 = {k: torch.from_numpy(v.view(np.int16)).view(torch.bfloat16).to(dev)
                for k, v in bf16.items()}
    return f32, bf16, dev_f32, dev_bf16


def run(sched, pool, dev, **kw):
    out = torch.full((len(sched["n"]),), float("nan"), dtype=torch.float64, device=dev)
    server = hm.Server(**kw)
    done = server.run_schedule(make_jobs(server, sched, pool, out))
    server.close()
    torch.cuda.synchronize()
    return out.cpu().numpy(), done


def same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def test_resident_stops_cleanly(dev, pool):
    t0 = time.monotonic()
    hm.Server(resident=1).close()                   # never launched
    sched = workloads.serving_schedule(10000, 0.003, pool_n=POOL_N, log2_max=14)
    out = torch.full((len(sched["n"]),), float("nan"), dtype=torch.float64, device=dev)
    server = hm.Server(resident=1)
    jobs = make_jobs(server, sched, pool, out)
    server.submit(jobs[0].copy())
    server.wait_idle()
    server.close()                                  # stops the running instance, waits for it
    torch.cuda.synchronize()
    # an instance stops by itself 10 ms after its last job: a device-wide
    # synchronisation returns while the server stays open
    server = hm.Server(resident=1)
    jobs = make_jobs(server, sched, pool, out)
    for k in (1, 2, 3):
        server.submit(jobs[k].copy())
    server.wait_idle()
    torch.cuda.synchronize()
    server.submit(jobs[4].copy())                   # a new instance starts on demand
    server.wait_idle()
    server.close()
    torch.cuda.synchronize()
    assert time.monotonic() - t0 < 10
    got = out.cpu().numpy()
    for k in range(5):
        oracle_check(k, float(got[k]), sched, pool)


@pytest.fixture(scope="module")
def mix(dev, pool):
    # 100k jobs/s: arrivals overlap on the device
    sched = workloads.serving_schedule(100000, 0.005, pool_n=POOL_N, log2_max=20)
    res = {}
    for mode, kw in (("resident", dict(resident=1)),
                     ("batched", dict(nstreams=2, max_batch_jobs=1024, batch_backlog=1)),
                     ("per_job", dict(nstreams=2, max_batch_jobs=1))):
        got, done = run(sched, pool, dev, **kw)
        assert np.all(done["status"] == 0), mode
        res[mode] = (got, done)
    return sched, res


def test_resident_every_job_matches_the_oracle(pool, mix):
    sched, res = mix
    got, done = res["resident"]
    assert len(got) > 300 and not np.any(np.isnan(got))
    assert np.all(done["done_ns"] >= done["arrival_ns"])
    assert np.max(done["batch_jobs"]) > 1          # jobs were on the device together
    for k in range(len(got)):
        oracle_check(k, float(got[k]), sched, pool)


def test_resident_equals_the_launched_paths(mix):
    _, res = mix
    assert same_bits(res["resident"][0], res["batched"][0])
    assert same_bits(res["resident"][0], res["per_job"][0])


def test_resident_job_alone_equals_mix(dev, pool, mix):
    sched, res = mix
    got = res["resident"][0]
    rng = np.random.default_rng(17)
    pick = rng.choice(len(got), 60, replace=False)
    out = torch.full((len(got),), float("nan"), dtype=torch.float64, device=dev)
    server = hm.Server(resident=1)
    jobs = make_jobs(server, sched, pool, out)
    for k in pick:
        server.submit(jobs[k].copy())
        server.wait_idle()
    server.close()
    torch.cuda.synchronize()
    alone = out.cpu().numpy()
    for k in pick:
        assert same_bits(alone[k], got[k]), (int(k), alone[k], got[k])


def test_resident_instances_replaced_and_edge_jobs(dev, pool):
    # a 0.7 s stream (a new instance every 250 ms) with empty, one-element and
    # misaligned jobs (x one element past y, so the arrays share no 16-byte
    # alignment), against the launched path bit for bit and the oracle
    sched = workloads.serving_schedule(20000, 0.7, pool_n=POOL_N, log2_max=15)
    m = len(sched["n"])
    sched["n"][::97] = 0
    sched["n"][5::89] = 1
    mis = np.zeros(m, bool)
    mis[3::7] = True
    sched["offset"] = np.minimum(sched["offset"], POOL_N - sched["n"] - 1)

    def jobs_for(server, out):
        jobs = make_jobs(server, sched, pool, out)
        es = np.where(sched["bf16"], 2, 4).astype(np.uint64)
        jobs["x"][mis] += es[mis]
        return jobs

    outs, dones = {}, {}
    for mode, kw in (("resident", dict(resident=1)), ("batched", dict(nstreams=4))):
        out = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
        server = hm.Server(**kw)
        dones[mode] = server.run_schedule(jobs_for(server, out))
        server.close()
        torch.cuda.synchronize()
        outs[mode] = out.cpu().numpy()
        assert np.all(dones[mode]["status"] == 0), mode
    assert m > 10000
    assert same_bits(outs["resident"], outs["batched"])
    f32, bf16, _, _ = pool
    rng = np.random.default_rng(23)
    pick = np.unique(np.concatenate([np.nonzero(sched["n"] == 1)[0], np.nonzero(mis)[0][:100],
                                     rng.choice(m, 150, replace=False)]))
    got = outs["resident"]
    for k in pick:
        if mis[k]:
            continue
        oracle_check(int(k), float(got[k]), sched, pool)
    # the misaligned jobs: x starts one element later
    for k in np.nonzero(mis)[0][:100]:
        src = bf16 if sched["bf16"][k] else f32
        one = {key: sched[key][k:k + 1] for key in ("n", "tmpl", "bf16", "offset")}
        view = {"x": src["x"][1:], "y": src["y"], "w": src["w"]}
        oracle_check(0, float(got[k]), one, (view, view, None, None))
    # empty jobs: the neutral result, as on the launched path
    empty = sched["n"] == 0
    assert same_bits(got[empty], outs["batched"][empty])


def test_resident_budget_admission(dev, pool):
    sched = workloads.serving_schedule(50000, 0.01, pool_n=POOL_N, log2_min=16, log2_max=18)
    got, done = run(sched, pool, dev, resident=1, hbm_budget_bytes=4 << 20)
    ref, _ = run(sched, pool, dev, nstreams=4)
    assert np.all(done["status"] == 0)
    assert same_bits(got, ref)


def test_resident_full_size_stream(dev):
    # the measured configuration (2^24-element pool, sizes up to 2^24) at
    # 50k jobs/s: resident == launched batches bit for bit, the 10 largest
    # and 40 more jobs against the oracle
    f32, bf16 = workloads.serving_pool()
    full = (f32, bf16, {k: torch.from_numpy(v).to(dev) for k, v in f32.items()},
            {k: torch.from_numpy(v.view(np.int16)).view(torch.bfloat16).to(dev) for k, v in bf16.items()})
    sched = workloads.serving_schedule(50000, 0.02)
    got, done = run(sched, full, dev, resident=1)
    ref, _ = run(sched, full, dev, hbm_budget_bytes=64 << 30, nstreams=4, max_batch_jobs=1024)
    assert np.all(done["status"] == 0) and same_bits(got, ref)
    assert int(np.max(sched["n"])) > (1 << 23)
    rng = np.random.default_rng(29)
    largest = np.argsort(sched["n"], kind="stable")[-10:]
    pick = np.unique(np.concatenate([largest, rng.choice(len(got), 40, replace=False)]))
    for k in pick:
        oracle_check(int(k), float(got[k]), sched, full)
    del full
    torch.cuda.empty_cache()


def test_resident_ring_refuses_fields_past_48_bits(dev, pool):
    # the resident ring carries addresses and lengths as 48-bit fields: a job
    # beyond them is refused at submission (nothing reaches the device), and
    # the server goes on serving
    sched = workloads.serving_schedule(10000, 0.003, pool_n=POOL_N, log2_max=12)
    out = torch.full((len(sched["n"]),), float("nan"), dtype=torch.float64, device=dev)
    server = hm.Server(resident=1)
    jobs = make_jobs(server, sched, pool, out)
    for field in ("x", "out"):
        bad = jobs[0].copy()
        bad[field] = np.uint64(1 << 48)
        with pytest.raises(hm.UnsupportedError):
            server.submit(bad)
    server.submit(jobs[0].copy())
    server.wait_idle()
    server.close()
    torch.cuda.synchronize()
    oracle_check(0, float(out.cpu().numpy()[0]), sched, pool)


def test_resident_burst_of_jobs_at_once(dev, pool):
    # 300 jobs due at the same instant: the dispatcher takes up to seven
    # complete ring slots per read; every result equals the launched path's
    sched = workloads.serving_schedule(10000, 0.04, pool_n=POOL_N, log2_max=14)
    sched["arrival_ns"][:] = 0
    assert len(sched["n"]) >= 300
    got, done = run(sched, pool, dev, resident=1)
    ref, _ = run(sched, pool, dev, nstreams=4)
    assert np.all(done["status"] == 0)
    assert same_bits(got, ref)


def test_resident_largest_jobs_and_one_past(dev):
    # the largest jobs taken (2^26 float32 elements: 17 passes per tile, 4033
    # tiles), ragged and misaligned ones beside them, float32 and bfloat16, on
    # the resident kernel and on one launch pair per job, bit for bit; one
    # element past the limit is refused at submission
    big = 1 << 26
    f32, bf16 = workloads.serving_pool(big + 8)
    full = (f32, bf16, {k: torch.from_numpy(v).to(dev) for k, v in f32.items()},
            {k: torch.from_numpy(v.view(np.int16)).view(torch.bfloat16).to(dev) for k, v in bf16.items()})
    sched = {"n": np.array([big, big - 3, big - 1000, big, big - 5, big, big - 77, big], np.int64),
             "tmpl": np.array([0, 1, 3, 7, 2, 6, 4, 5], np.int32),
             "bf16": np.array([0, 0, 0, 0, 1, 1, 1, 1], bool),
             "offset": np.array([0, 1, 3, 0, 2, 0, 5, 0], np.int64),
             "arrival_ns": np.arange(8, dtype=np.int64) * 2_000_000}
    got, done = run(sched, full, dev, resident=1, hbm_budget_bytes=64 << 30)
    ref, _ = run(sched, full, dev, hbm_budget_bytes=64 << 30, nstreams=1, max_batch_jobs=1)
    assert np.all(done["status"] == 0) and same_bits(got, ref)
    # the oracle takes 10-20 s per job this long: the float32 sum and the
    # ragged, misaligned dot; the max and the count are exact
    for k in (0, 1):
        oracle_check(k, float(got[k]), sched, full)
    assert got[2] == float(np.max(f32["x"][3:3 + big - 1000]))
    xb = torch.from_numpy(bf16["x"][:big].view(np.int16)).view(torch.bfloat16).float()
    assert got[7] == float(torch.count_nonzero(xb > 0))
    for mode, kw in (("resident", dict(resident=1)), ("per_job", dict(nstreams=1, max_batch_jobs=1))):
        out = torch.zeros(2, dtype=torch.float64, device=dev)
        server = hm.Server(hbm_budget_bytes=64 << 30, **kw)
        jobs = make_jobs(server, {k: v[:2] for k, v in sched.items()}, full, out)
        jobs["n"] = [big + 1, 2 * big + 1]
        jobs["dtype"] = [hm.hipmr.F32, hm.hipmr.BF16]
        for k in range(2):
            with pytest.raises(hm.UnsupportedError):
                server.submit(jobs[k].copy())
        server.close()
    del full
    torch.cuda.empty_cache()
