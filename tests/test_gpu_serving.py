"""GPU parity of the serving extension: a Poisson stream of map-reduce jobs
(8 templates, float32 / bfloat16, sizes log-uniform) replayed open-loop
through the continuous-batching request loop; every job is checked against
the CPU oracle; each job's result is bitwise the same alone and in the mix;
admission by memory budget; rejected jobs are isolated."""

import math

import numpy as np
import pytest

from gpu_util import need_gpu, torch
import oracle
import paper_1304_5553_amd as hm
import workloads

pytestmark = pytest.mark.gpu

POOL_N = 1 << 20
A, B = 2.5, -0.5
MAPS = {0: "x[i]", 1: "x[i]*y[i]", 2: "x[i]*x[i]", 3: "x[i]", 4: "2.5f*x[i] - 0.5f*y[i]",
        5: "x[i] > 0.0f", 6: "x[i]*x[i]", 7: "w[i]*x[i]"}


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


def make_jobs(server, sched, pool, out):
    f32, bf16, dev_f32, dev_bf16 = pool
    jobs = server.jobs(len(sched["n"]))
    for k in range(len(jobs)):
        src = dev_bf16 if sched["bf16"][k] else dev_f32
        off = int(sched["offset"][k])
        es = 2 if sched["bf16"][k] else 4
        jobs[k]["x"] = src["x"].data_ptr() + off * es
        jobs[k]["y"] = src["y"].data_ptr() + off * es
        jobs[k]["w"] = src["w"].data_ptr() + off * es
        jobs[k]["n"] = sched["n"][k]
        jobs[k]["tmpl"] = sched["tmpl"][k]
        jobs[k]["dtype"] = hm.hipmr.BF16 if sched["bf16"][k] else hm.hipmr.F32
        jobs[k]["arrival_ns"] = sched["arrival_ns"][k]
        jobs[k]["out"] = out.data_ptr() + 8 * k
        jobs[k]["a"], jobs[k]["b"] = A, B
    return jobs


def oracle_check(k, got, sched, pool):
    """The job's result against the oracle: exact for max and counts, else the
    map-reduce gate |g - o| <= 2e-6 sum|t| + 2 sum(e) (propagated through
    sqrt and the ratio)."""
    f32, bf16, _, _ = pool
    n, t, off = int(sched["n"][k]), int(sched["tmpl"][k]), int(sched["offset"][k])
    fmt = "bfloat16" if sched["bf16"][k] else "float"
    src = bf16 if sched["bf16"][k] else f32
    arrs = [src[a][off:off + n] for a in ("x", "y", "w")]
    sig = f"double: const {fmt} *x, const {fmt} *y, const {fmt} *w"
    if t == 3:
        r = oracle.reduce(sig.replace("double", "float"), "x[i]", "max", "-INFINITY", n, arrs)
        assert got == r.value, (k, got, r.value)
        return
    if t == 5:
        r = oracle.reduce(sig.replace("double", "long"), "x[i] > 0.0f", "a+b", "0", n, arrs)
        assert got == r.value, (k, got, r.value)
        return
    r = oracle.reduce(sig.replace("double", "float"), MAPS[t], "a+b", "0", n, arrs)
    tol = 2e-6 * r.abs_sum + 2 * r.err_sum
    if t == 2:
        o = math.sqrt(r.value)
        assert abs(got - o) <= tol / max(got + o, 1e-300) + 1e-300, (k, got, o)
    elif t == 7:
        den = oracle.reduce(sig.replace("double", "float"), "w[i]", "a+b", "0", n, arrs)
        tol_d = 2e-6 * den.abs_sum
        o = r.value / den.value
        assert abs(got - o) <= (tol + abs(o) * tol_d) / den.value, (k, got, o)
    else:
        assert abs(got - r.value) <= tol, (k, t, got, r.value, tol)
        # and the bare gate, the map's own rounding counted inside it
        assert abs(got - r.value) <= 2e-6 * r.abs_sum, (k, t, got, r.value)


@pytest.fixture(scope="module")
def mix(dev, pool):
    # 100k jobs/s on two streams: arrivals outpace single-job service, so jobs
    # that arrive while others run are packed into the next free slot (any
    # queue longer than the free slots is packed)
    sched = workloads.serving_schedule(100000, 0.005, pool_n=POOL_N, log2_max=20)
    out = torch.full((len(sched["n"]),), float("nan"), dtype=torch.float64, device=dev)
    server = hm.Server(nstreams=2, max_batch_jobs=1024, batch_backlog=1)
    done = server.run_schedule(make_jobs(server, sched, pool, out))
    torch.cuda.synchronize()
    server.close()
    return sched, out.cpu().numpy(), done


def test_every_job_matches_the_oracle(pool, mix):
    sched, got, done = mix
    assert len(got) > 300
    assert np.all(done["status"] == 0)
    assert np.all(done["done_ns"] >= done["arrival_ns"])
    assert np.max(done["batch_jobs"]) > 1          # jobs were packed together
    for k in range(len(got)):
        oracle_check(k, float(got[k]), sched, pool)


def test_each_job_is_bitwise_the_same_alone(dev, pool, mix):
    sched, got, _ = mix
    rng = np.random.default_rng(7)
    pick = rng.choice(len(got), 60, replace=False)
    for mode in ("batched", "per_job"):
        server = hm.Server(nstreams=2, max_batch_jobs=1 if mode == "per_job" else 64)
        out = torch.full((len(got),), float("nan"), dtype=torch.float64, device=dev)
        jobs = make_jobs(server, sched, pool, out)
        for k in pick:                   # one job at a time: it runs alone
            j = jobs[k].copy()
            server.submit(j)
            server.wait_idle()
        torch.cuda.synchronize()
        alone = out.cpu().numpy()
        server.close()
        for k in pick:
            same = alone[k] == got[k] or (math.isnan(alone[k]) and math.isnan(got[k]))
            assert same, (mode, k, alone[k], got[k])


def test_budget_admission_and_rejection(dev, pool):
    sched = workloads.serving_schedule(50000, 0.01, pool_n=POOL_N, log2_min=16, log2_max=18)
    out = torch.full((len(sched["n"]),), float("nan"), dtype=torch.float64, device=dev)
    budget = 4 << 20                               # a few jobs at a time
    server = hm.Server(hbm_budget_bytes=budget, nstreams=4)
    jobs = make_jobs(server, sched, pool, out)
    big = jobs[0].copy()
    big["n"] = POOL_N                              # 8 MB of float32 x and y: never fits
    big["tmpl"] = hm.hipmr.JOB_DOT
    big["dtype"] = hm.hipmr.F32
    bad = jobs[1].copy()
    bad["x"] = 0                                   # invalid: a NULL input
    jobs = np.concatenate([jobs[:5], [big, bad], jobs[5:]]).astype(jobs.dtype)
    jobs["arrival_ns"] = np.maximum.accumulate(jobs["arrival_ns"])
    done = server.run_schedule(jobs)
    server.close()
    assert done["status"][5] == hm.BudgetError.code
    assert done["status"][6] == hm.InvalidError.code
    ok = np.ones(len(jobs), bool)
    ok[[5, 6]] = False
    assert np.all(done["status"][ok] == 0)
    # in-flight jobs never exceeded the budget: every batch fits it
    sizes = jobs["n"] * np.where(jobs["dtype"] == hm.hipmr.BF16, 2, 4) * \
        np.where(np.isin(jobs["tmpl"], [1, 4, 7]), 2, 1)
    for k in np.nonzero(ok)[0]:
        assert sizes[k] <= budget


def test_submit_and_poll(dev, pool):
    sched = workloads.serving_schedule(10000, 0.01, pool_n=POOL_N, log2_max=16)
    out = torch.full((len(sched["n"]),), float("nan"), dtype=torch.float64, device=dev)
    server = hm.Server()
    jobs = make_jobs(server, sched, pool, out)
    tickets = [server.submit(j) for j in jobs]
    server.wait_idle()
    comps = server.poll()
    server.close()
    assert sorted(int(t) for t in comps["ticket"]) == sorted(tickets)
    assert np.all(comps["status"] == 0)
    got = out.cpu().numpy()
    for k in range(0, len(jobs), 5):
        oracle_check(k, float(got[k]), sched, pool)


@pytest.mark.parametrize("max_jobs", [24, 1024])
def test_burst_packs_large_batches(dev, pool, max_jobs):
    # every job arrives at once on one stream: batches fill up to the cap,
    # which covers both the by-value descriptor path (up to 24 jobs) and the
    # device descriptor table (more)
    sched = workloads.serving_schedule(50000, 0.006, pool_n=POOL_N, log2_max=14)
    sched["arrival_ns"][:] = 0
    out = torch.full((len(sched["n"]),), float("nan"), dtype=torch.float64, device=dev)
    server = hm.Server(nstreams=1, max_batch_jobs=max_jobs)
    done = server.run_schedule(make_jobs(server, sched, pool, out))
    torch.cuda.synchronize()
    server.close()
    assert len(sched["n"]) > 200 and np.all(done["status"] == 0)
    assert int(np.max(done["batch_jobs"])) == min(max_jobs, len(sched["n"]))
    got = out.cpu().numpy()
    for k in range(len(got)):
        oracle_check(k, float(got[k]), sched, pool)


def test_large_jobs_run_alone_and_small_ones_pass_them(dev, pool):
    # a burst on one stream alternating jobs over and under solo_bytes: every
    # large job runs in a batch of its own, the small ones are packed together
    # past them, and every result matches the oracle
    sched = workloads.serving_schedule(50000, 0.004, pool_n=POOL_N, log2_min=10, log2_max=12)
    m = len(sched["n"])
    sched["arrival_ns"][:] = 0
    sched["n"][::3] = POOL_N // 2                  # 1 MiB of bfloat16 / 2 MiB of float32 per array
    sched["offset"][::3] = np.minimum(sched["offset"][::3], POOL_N - POOL_N // 2)
    out = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
    solo = 1 << 20
    server = hm.Server(nstreams=1, max_batch_jobs=1024, solo_bytes=solo)
    jobs = make_jobs(server, sched, pool, out)
    done = server.run_schedule(jobs)
    torch.cuda.synchronize()
    server.close()
    assert m > 100 and np.all(done["status"] == 0)
    large = np.zeros(m, bool)
    large[::3] = True
    assert np.all(done["batch_jobs"][large] == 1)
    assert int(np.max(done["batch_jobs"][~large])) > 10
    # the first small jobs are not held back behind the large ones
    first_small = np.nonzero(~large)[0][:10]
    assert np.all(done["done_ns"][first_small] <= np.sort(done["done_ns"][large])[1])
    got = out.cpu().numpy()
    for k in range(m):
        oracle_check(k, float(got[k]), sched, pool)


def test_short_queue_runs_one_job_per_stream(dev, pool):
    # bursts of 4 jobs on 4 streams wait at most batch_backlog per free stream:
    # each job gets a stream of its own; bursts of 40 are packed
    sched = workloads.serving_schedule(50000, 0.004, pool_n=POOL_N, log2_max=14)
    m = len(sched["n"])
    for burst, packed in ((4, False), (40, True)):
        sched["arrival_ns"] = (np.arange(m) // burst) * 300_000
        out = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
        server = hm.Server(nstreams=4, max_batch_jobs=1024, batch_backlog=8)
        done = server.run_schedule(make_jobs(server, sched, pool, out))
        torch.cuda.synchronize()
        server.close()
        assert np.all(done["status"] == 0)
        assert (int(np.max(done["batch_jobs"])) > 1) == packed, burst
        got = out.cpu().numpy()
        for k in range(0, m, 7):
            oracle_check(k, float(got[k]), sched, pool)


@pytest.fixture(scope="module")
def full_pool(dev):
    f32, bf16 = workloads.serving_pool()
    dev_f32 = {k: torch.from_numpy(v).to(dev) for k, v in f32.items()}
    dev_bf16 = {k: torch.from_numpy(v.view(np.int16)).view(torch.bfloat16).to(dev)
                for k, v in bf16.items()}
    return f32, bf16, dev_f32, dev_bf16


@pytest.mark.parametrize("rate", list(workloads.SERVING_RATES))
def test_full_size_stream(dev, full_pool, rate):
    # the measured serving configuration at each configured rate: a
    # 2^24-element pool per array and dtype, job sizes log-uniform over
    # [2^10, 2^24], a 64 GiB budget, 4 streams, up to 1024 jobs per launch;
    # a window of about 1000 jobs of the stream, of which the 20 largest and
    # 180 others are checked against the oracle and 40 against the same job
    # run alone
    sched = workloads.serving_schedule(rate, 1000 / rate)
    m = len(sched["n"])
    out = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
    server = hm.Server(hbm_budget_bytes=64 << 30, nstreams=4, max_batch_jobs=1024)
    done = server.run_schedule(make_jobs(server, sched, full_pool, out))
    torch.cuda.synchronize()
    server.close()
    got = out.cpu().numpy()
    assert m > 900 and np.all(done["status"] == 0)
    assert not np.any(np.isnan(got))
    assert int(np.max(sched["n"])) > (1 << 23)
    rng = np.random.default_rng(rate)
    largest = np.argsort(sched["n"], kind="stable")[-20:]
    rest = np.setdiff1d(np.arange(m), largest)
    pick = np.unique(np.concatenate([largest, rng.choice(rest, 180, replace=False)]))
    assert pick.size == 200
    for k in pick:
        oracle_check(int(k), float(got[k]), sched, full_pool)
    alone_pick = np.unique(np.concatenate([largest, rng.choice(rest, 20, replace=False)]))
    server = hm.Server(hbm_budget_bytes=64 << 30, nstreams=4, max_batch_jobs=1024)
    alone_out = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
    jobs = make_jobs(server, sched, full_pool, alone_out)
    for k in alone_pick:
        server.submit(jobs[k].copy())
        server.wait_idle()
    torch.cuda.synchronize()
    server.close()
    alone = alone_out.cpu().numpy()
    for k in alone_pick:
        assert alone[k] == got[k], (rate, int(k), alone[k], got[k])
