"""Benchmark of the plain fused elementwise / map-reduce path on one MI355X.

Workload (plain method at scale, n = 2**28, inputs resident in HBM):
  E1  z[i] = 2.5f*x[i] - 0.5f*y[i]          float32, 12 B/element
  E2  z[i] = sqrtf(x[i]*x[i] + y[i]*y[i])   float32, 12 B/element
  R1  count(k[i] % 7 == 3) -> int64         int32,    4 B/element
  R2  sum(k[i])            -> int64         int32,    4 B/element
  R3  max(x[i])            -> float         float32,  4 B/element
x, y ~ U[-1, 1] float32 (seed 1), k ~ U{0 .. 2**20 - 1} int32 (seed 2).

One step = one pass of every op through the C ABI (compile-cache lookup,
launch, two-stage reduce).  ``value`` = algorithmic bytes of a step / step
time (GB/s, 1 GB = 1e9 B).  The roofline entry is for the kernel with the
largest share of the step, timed per launch with HIP events on the stream
the library launches on.  The CPU baseline is the oracle, timed on a bounded
sample of the same workload on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "map-reduce HBM GB/s (% of peak); batched/served vs plain speedup; p99 latency"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=1 << 28)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extensions", action="store_true",
                   help="skip the precision, batching and serving measurements")
    p.add_argument("--extensions", default="compile,dot,precision,batched,served,scan,shifted,cg,lazy,complex",
                   help="comma list of the extension measurements to run "
                        "(compile, dot, precision, batched, served, scan, shifted, cg, lazy, complex)")
    p.add_argument("--batched-eager-only", action="store_true",
                   help="batched leg: the tuned ops eagerly only (no graphs, no per-segment "
                        "baseline), for counter runs")
    p.add_argument("--serving-rates", default="",
                   help="comma list of jobs/s (default: 2000,10000,50000 and the 200000 stress rate)")
    p.add_argument("--serving-duration", type=float, default=4.0,
                   help="measured seconds of each serving rate (after 1 s of warm-up)")
    p.add_argument("--cpu-sample", type=int, default=1 << 28,
                   help="elements per op for the all-core oracle timing")
    p.add_argument("--cpu-sample-one", type=int, default=1 << 25,
                   help="elements per op for the one-core oracle timing")
    p.add_argument("--no-accuracy", action="store_true",
                   help="skip checking the timed results against the oracle")
    p.add_argument("--ops", default="E1,E2,R1,R2,R3",
                   help="comma list of E1,E2,R1,R2,R3 and COPY (z[i] = x[i], the plain copy "
                        "kernel used to calibrate the HBM byte counters)")
    return p.parse_args()


COUNTERS_MD = "profiles/plain_n2e28_hbm_counters.md"


def counter_traffic(symbol):
    """HBM bytes per launch of `symbol` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on the copy kernel), or None
    when that exact kernel (its symbol carries a hash of its source) has not
    been profiled."""
    path = os.path.join(ROOT, COUNTERS_MD)
    if not os.path.exists(path):
        return None
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0] == symbol:
            try:
                return int(float(cells[3]))
            except ValueError:
                return None
    return None


# ---------------------------------------------------------------- CPU leg
# The oracle (test infrastructure) runs only in this leg: timed on this host's
# cores as the CPU baseline, and as the checker of the results the timed GPU
# runs produced.  The leg's worker processes are forked before the GPU is
# touched, so they hold no device state; they share the plain workload's host
# arrays (and two buffers for the GPU's elementwise outputs) copy-on-write and
# regenerate the other workloads from the same seeds, i.e. the same bytes the
# GPU read.

_LEG = {}                   # set in the parent before the fork, read by the workers
MAX_LEG_WORKERS = 16        # the CPU share of one GPU on the measurement hosts
SERVE_MAPS = {0: "x[i]", 1: "x[i]*y[i]", 2: "x[i]*x[i]", 3: "x[i]", 4: "2.5f*x[i] - 0.5f*y[i]",
              5: "x[i] > 0.0f", 6: "x[i]*x[i]", 7: "w[i]*x[i]"}
SEG_OPS = {"sum": ("float: const float *x, const float *y", "x[i]", "a+b", "0"),
           "max": ("float: const float *x, const float *y", "x[i]", "max(a,b)", "-INFINITY"),
           "dot": ("float: const float *x, const float *y", "x[i]*y[i]", "a+b", "0")}
GATE_REL = 2e-6             # float sums: |gpu - oracle| <= 2e-6 * sum |terms|
PREC_UQ = {"bfloat16": 2.0 ** -8, "float16": 2.0 ** -11, "fp8_e4m3": 2.0 ** -4}
PREC_MIN_SUB = {"bfloat16": 2.0 ** -133, "float16": 2.0 ** -24, "fp8_e4m3": 2.0 ** -9}
PREC_MIN_NORMAL = {"bfloat16": 2.0 ** -126, "float16": 2.0 ** -14, "fp8_e4m3": 2.0 ** -6}


def _leg_inputs(key):
    """The seeded inputs of one workload, made once per worker."""
    import workloads
    cache = _LEG.setdefault("cache", {})
    if key not in cache:
        if key == "dot":
            cache[key] = workloads.dot_1m()
        elif key == "segments":
            cache[key] = workloads.segments()
        elif key == "pool":
            cache[key] = workloads.serving_pool()
        elif key[0] == "schedule":
            cache[key] = workloads.serving_schedule(key[1], key[2])
        elif key[0] == "precision":
            for other in [c for c in cache if c[0] == "precision"]:
                del cache[other]                       # one case (1 GiB) at a time
            cache[key] = workloads.precision_values(workloads.N_PRECISION, key[1])
    return cache[key]


def _ratio(err, tol):
    return 0.0 if err == 0 else (err / tol if tol > 0 else float("inf"))


def leg_time_plain(a, b):
    """Seconds the oracle takes for elements [a, b) of every plain op."""
    import oracle
    import workloads
    x, y, k = _LEG["x"][a:b], _LEG["y"][a:b], _LEG["k"][a:b]
    m = b - a
    zero = np.zeros(1, np.float32)
    t0 = time.perf_counter()
    oracle.elementwise(workloads.E1[0], workloads.E1[1], m, [zero, x, y])
    oracle.elementwise(workloads.E2[0], workloads.E2[1], m, [zero, x, y])
    for sig, mp, comb, neu in (workloads.R_COUNT, workloads.R_SUM):
        oracle.reduce(sig, mp, comb, neu, m, [k])
    oracle.reduce(workloads.R_MAX[0], workloads.R_MAX[1], "max(a,b)", "-INFINITY", m, [x])
    return time.perf_counter() - t0


def leg_check_elementwise(name, a, b):
    """GPU output lanes [a, b) of E1 / E2 against the oracle: (lanes checked,
    lanes outside twice the oracle's per-lane bound, largest |gpu - oracle| /
    (2 bound))."""
    import oracle
    import workloads
    sig, stmt = workloads.E1 if name == "E1" else workloads.E2
    g = _LEG["z"][name][a:b].astype(np.float64)
    ref = oracle.elementwise(sig, stmt, _LEG["n"], [np.zeros(1, np.float32), _LEG["x"], _LEG["y"]],
                             lanes=np.arange(a, b))["z"]
    ok = ~ref.u & ref.written
    diff = np.abs(g - ref.v)
    same = (g == ref.v) | (np.isnan(g) & np.isnan(ref.v))
    bound = 2 * ref.e
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(same, 0.0, np.where(bound > 0, diff / bound, np.inf))
    ratio = ratio[ok]
    return int(ok.sum()), int(np.count_nonzero(ratio > 1)), float(ratio.max()) if ratio.size else 0.0


def leg_plain_reduce(a, b):
    """The oracle's count, sum and max over elements [a, b) (exact values)."""
    import oracle
    import workloads
    x, k = _LEG["x"][a:b], _LEG["k"][a:b]
    m = b - a
    vals = [oracle.reduce(sig, mp, comb, neu, m, [k]).value
            for sig, mp, comb, neu in (workloads.R_COUNT, workloads.R_SUM)]
    vals.append(oracle.reduce(workloads.R_MAX[0], workloads.R_MAX[1], "max(a,b)", "-INFINITY",
                              m, [x]).value)
    return vals


def leg_check_dot(g):
    import oracle
    import workloads
    x, y = _leg_inputs("dot")
    r = oracle.reduce(workloads.DOT[0], workloads.DOT[1], "a+b", "0", x.size, [x, y])
    err = abs(g - r.value)
    return {"n": int(x.size), "gpu": g, "oracle": r.value, "abs_err": err,
            "sum_abs_terms": r.abs_sum, "err_over_sum_abs_terms": err / r.abs_sum,
            "gate": GATE_REL, "ok": bool(err <= GATE_REL * r.abs_sum)}


def leg_check_precision(fmt, case, g_sum, g_norm):
    """The compensated sum and two-pass norm of one format and case against
    the oracle: (i) the accumulation error against the exact sum / norm of
    the stored (dequantised) values, relative to sum |q| / the norm, gate
    1e-6; (ii) the total error against the float32 values before rounding to
    the format, relative to sum |v| / |v|, gate u_q (plus the subnormal
    allowance and gate (i))."""
    import oracle
    import workloads
    v64 = _leg_inputs(("precision", case))
    qz = workloads.quantize(fmt, v64)
    decode = {"bfloat16": oracle.decode_bf16, "float16": oracle.decode_f16,
              "fp8_e4m3": oracle.decode_e4m3fn}[fmt]
    q = decode(qz.bits)
    inv = 1.0 / qz.scale
    o_sum, o_norm = oracle.exact_sum(q) * inv, oracle.norm2(q) * inv
    abs_q = float(np.sum(np.abs(q))) * inv
    v = qz.original.astype(np.float64) * inv
    v_sum, v_norm = oracle.exact_sum(v), oracle.norm2(v)
    abs_v = float(np.sum(np.abs(v)))
    n_sub = int(np.count_nonzero(np.abs(q) < PREC_MIN_NORMAL[fmt]))
    half_sub = PREC_MIN_SUB[fmt] / 2 * inv
    gate_i_sum, gate_i_norm = 1e-6 * abs_q, 1e-6 * o_norm
    gate_ii_sum = PREC_UQ[fmt] * abs_v + n_sub * half_sub + gate_i_sum
    gate_ii_norm = PREC_UQ[fmt] * v_norm + math.sqrt(n_sub) * half_sub + gate_i_norm
    e = {"sum_err_i": abs(g_sum - o_sum), "norm_err_i": abs(g_norm - o_norm),
         "sum_err_ii": abs(g_sum - v_sum), "norm_err_ii": abs(g_norm - v_norm)}
    return {"sum": g_sum, "norm2": g_norm, "oracle_sum": o_sum, "oracle_norm2": o_norm,
            "sum_err_i_rel": e["sum_err_i"] / abs_q, "norm_err_i_rel": e["norm_err_i"] / o_norm,
            "sum_err_ii_rel": e["sum_err_ii"] / abs_v, "norm_err_ii_rel": e["norm_err_ii"] / v_norm,
            "gate_i_rel": 1e-6, "gate_ii_rel": PREC_UQ[fmt], "subnormal_or_zero": n_sub,
            "ok": bool(e["sum_err_i"] <= gate_i_sum and e["norm_err_i"] <= gate_i_norm and
                       e["sum_err_ii"] <= gate_ii_sum and e["norm_err_ii"] <= gate_ii_norm)}


def leg_check_segments(op, s0, s1, g):
    """Segments [s0, s1) of one segmented op against the oracle: (largest
    |gpu - oracle| / (2e-6 sum |terms|), results outside the gate; max is
    compared exactly)."""
    import oracle
    offsets, x, y = _leg_inputs("segments")
    sig, mp, comb, neu = SEG_OPS[op]
    worst, bad = 0.0, 0
    for s in range(s0, s1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        r = oracle.reduce(sig, mp, comb, neu, b - a, [x[a:b], y[a:b]])
        gv = float(g[s - s0])
        if r.exact or (r.op in ("max", "min") and r.err_sum == 0):
            bad += int(not (gv == r.value or (math.isnan(gv) and math.isnan(r.value))))
        else:
            q = _ratio(abs(gv - r.value), GATE_REL * r.abs_sum)
            worst = max(worst, q)
            bad += int(q > 1)
    return worst, bad


def leg_check_served(rate, duration_s, idx, got):
    """Served jobs idx (results got) of one rate against the oracle: (largest
    error / gate, jobs outside the gate).  max and count are exact; sums use
    |g - o| <= 2e-6 sum|t| + 2 sum(e), carried through the square root of the
    norm and the ratio of the weighted mean."""
    import oracle
    f32, bf16 = _leg_inputs("pool")
    sched = _leg_inputs(("schedule", rate, duration_s))
    worst, bad = 0.0, 0
    for k, g in zip(idx, got):
        n, t, off = int(sched["n"][k]), int(sched["tmpl"][k]), int(sched["offset"][k])
        fmt = "bfloat16" if sched["bf16"][k] else "float"
        src = bf16 if sched["bf16"][k] else f32
        arrs = [src[a][off:off + n] for a in ("x", "y", "w")]
        sig = f"float: const {fmt} *x, const {fmt} *y, const {fmt} *w"
        if t in (3, 5):
            r = (oracle.reduce(sig, "x[i]", "max", "-INFINITY", n, arrs) if t == 3 else
                 oracle.reduce(sig.replace("float:", "long:"), SERVE_MAPS[5], "a+b", "0", n, arrs))
            bad += int(g != r.value)
            continue
        r = oracle.reduce(sig, SERVE_MAPS[t], "a+b", "0", n, arrs)
        tol = GATE_REL * r.abs_sum + 2 * r.err_sum
        if t == 2:
            o = math.sqrt(r.value)
            tol = tol / max(g + o, 1e-300) + 1e-300
        elif t == 7:
            den = oracle.reduce(sig, "w[i]", "a+b", "0", n, arrs)
            o = r.value / den.value
            tol = (tol + abs(o) * GATE_REL * den.abs_sum) / den.value
        else:
            o = r.value
        q = _ratio(abs(g - o), tol)
        worst = max(worst, q)
        bad += int(q > 1)
    return worst, bad


def _chunks(n, parts):
    step = -(-n // max(1, parts))
    return [(a, min(a + step, n)) for a in range(0, n, step)]


class CpuLeg:
    """The oracle's worker processes (forked at construction, before the
    GPU is touched), the baseline timing and the accuracy checks."""

    def __init__(self, x, y, k, n):
        import mmap
        import multiprocessing
        self.host_cpus = len(os.sched_getaffinity(0))
        self.cores = max(1, min(MAX_LEG_WORKERS, self.host_cpus))
        _LEG.update(x=x, y=y, k=k, n=n, z={})
        self._maps = []
        for name in ("E1", "E2"):
            mm = mmap.mmap(-1, 4 * n)                # anonymous, shared with the workers
            self._maps.append(mm)
            _LEG["z"][name] = np.frombuffer(mm, dtype=np.float32, count=n)
        self.pool = multiprocessing.get_context("fork").Pool(self.cores)

    def close(self):
        self.pool.terminate()
        self.pool.join()

    def baseline(self, sample_one, sample_all, reps=3):
        """Median of `reps` runs of the oracle on one core (the first
        sample_one elements of every plain op) and on all the leg's cores
        (the first sample_all elements, one contiguous chunk per worker)."""
        n = _LEG["n"]
        m1, ma = min(sample_one, n), min(sample_all, n)
        one = [self.pool.apply(leg_time_plain, (0, m1)) for _ in range(reps)]
        chunks = _chunks(ma, self.cores)
        allc = []
        for _ in range(reps):
            t0 = time.perf_counter()
            self.pool.starmap(leg_time_plain, chunks)
            allc.append(time.perf_counter() - t0)
        per = 12 + 12 + 4 + 4 + 4
        t1, ta = float(np.median(one)), float(np.median(allc))
        return {"value": round(ma * per / ta / 1e9, 3), "unit": "GB/s", "cores": self.cores,
                "host_cpus": self.host_cpus, "kind": "oracle", "median_of": reps,
                "sample": f"first {ma} elements of each of E1, E2, R1, R2, R3 "
                          f"({ma * per / 1e6:.0f} MB algorithmic), one chunk per worker process, "
                          f"{ta:.2f} s",
                "single_core": {"value": round(m1 * per / t1 / 1e9, 3), "unit": "GB/s",
                                "sample": f"first {m1} elements of each op, {t1:.2f} s"}}

    def accuracy(self, checks):
        """Every result the timed GPU runs left in `checks`, against the oracle."""
        pool, jobs, out = self.pool, [], {}

        def submit(key, fn, *args):
            jobs.append((key, pool.apply_async(fn, args)))

        for (fmt, case), (gs, gn) in checks.get("precision", {}).items():
            submit(("precision", fmt, case), leg_check_precision, fmt, case, gs, gn)
        for rate, row in checks.get("served", {}).items():
            for part in np.array_split(np.arange(len(row["idx"])), 8):
                submit(("served", rate), leg_check_served, rate, row["duration_s"],
                       row["idx"][part].tolist(), row["got"][part].tolist())
        for op, g in checks.get("batched", {}).items():
            for a, b in _chunks(len(g), 16):
                submit(("batched", op), leg_check_segments, op, a, b, g[a:b])
        if "plain" in checks:
            for name in ("E1", "E2"):
                for a, b in _chunks(_LEG["n"], 64):
                    submit(("plain", name), leg_check_elementwise, name, a, b)
            for a, b in _chunks(_LEG["n"], 32):
                submit(("plain", "R"), leg_plain_reduce, a, b)
        if "dot" in checks:
            submit(("dot",), leg_check_dot, checks["dot"])
        parts = {}
        for key, job in jobs:
            parts.setdefault(key, []).append(job.get())
        ok = True
        if "plain" in checks:
            p = checks["plain"]
            out["plain"] = {}
            for name in ("E1", "E2"):
                rows = parts[("plain", name)]
                lanes, bad = sum(r[0] for r in rows), sum(r[1] for r in rows)
                out["plain"][name] = {"lanes_checked": lanes, "lanes_outside_bound": bad,
                                      "worst_err_over_bound": max(r[2] for r in rows)}
                ok &= bad == 0 and lanes == _LEG["n"]
            rows = parts[("plain", "R")]
            want = {"R1": sum(r[0] for r in rows), "R2": sum(r[1] for r in rows),
                    "R3": max(r[2] for r in rows)}
            for name, w in want.items():
                same = p[name] == w
                out["plain"][name] = {"gpu": p[name], "oracle": w, "exact_match": same}
                ok &= same
        if "dot" in checks:
            out["dot_1m"] = parts[("dot",)][0]
            ok &= out["dot_1m"]["ok"]
        if "precision" in checks:
            out["precision"] = {}
            for (fmt, case) in checks["precision"]:
                r = parts[("precision", fmt, case)][0]
                out["precision"].setdefault(fmt, {})[case] = r
                ok &= r["ok"]
        if "batched" in checks:
            out["batched"] = {}
            for op, g in checks["batched"].items():
                rows = parts[("batched", op)]
                bad = sum(r[1] for r in rows)
                out["batched"][op] = {"segments": len(g), "outside_gate": bad,
                                      "worst_err_over_gate": max(r[0] for r in rows),
                                      "gate": "exact" if op == "max" else "2e-6 sum|terms|"}
                ok &= bad == 0
        if "served" in checks:
            out["served"] = {}
            for rate, row in checks["served"].items():
                rows = parts[("served", rate)]
                bad = sum(r[1] for r in rows)
                out["served"][str(rate)] = {
                    "jobs_checked": len(row["idx"]), "largest_checked": row["largest"],
                    "outside_gate": bad, "worst_err_over_gate": max(r[0] for r in rows),
                    "batched_equals_per_job_bitwise": row["same"], "jobs_compared": row["compared"]}
                ok &= bad == 0 and row["same"]
        out["all_ok"] = bool(ok)
        return out


def _time_ms(torch, fn, reps, stream):
    """Median per-call milliseconds of fn() over reps calls (HIP events on
    the launch stream)."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    fn()
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def bench_compile(torch, hm, workloads, dev, stream, reps=5, launches=2000, hits=2000):
    """The host side of the path (front end, code generation, compile cache,
    launch): the cost of compile(expr, dtypes) when hipRTC runs (cold), when
    the code object comes from the disk cache (after the in-memory caches are
    dropped), when it is in memory but no handle for the text is held (front
    end, code generation with the symbol's SHA-256, and the lookup), and when
    a handle for the same text is still held (the handle cache: one hash
    lookup and a reference), for E1 and for R2's two reduce kernels; then the
    host time of one elementwise call (argument marshalling and the enqueue)
    and the GPU time per launch of a 4096-element E1, back to back.  Each cold
    source is new (its own kernel name) and the disk cache is a fresh
    directory, so nothing is found by accident."""
    import shutil
    import tempfile
    binding = hm.hipmr
    saved = os.environ.get("HIPMR_CACHE_DIR")
    tmp = tempfile.mkdtemp(prefix="hipmr_bench_cache_")
    os.environ["HIPMR_CACHE_DIR"] = tmp
    tag = f"{os.getpid()}_{time.time_ns()}"
    res = {}
    try:
        for label, (sig, expr), combine in (("elementwise_E1", workloads.E1, None),
                                            ("reduce_R2", workloads.R_SUM[:2], workloads.R_SUM[2:])):
            times = {"cold": [], "disk": [], "memory": []}
            handle_us, handle_prep_us = [], []
            before = binding.cache_stats()
            for r in range(reps):
                name = f"cold{r}_{tag}"

                def build():
                    k = hm.compile(expr, sig, name=name)
                    if combine:
                        binding.prepare_reduce(k, *combine)
                    return k

                held = None
                for phase in ("cold", "disk", "memory"):
                    if phase == "disk":
                        binding.cache_drop_memory()
                    held = None                 # no handle for the text is held: not a handle hit
                    t0 = time.perf_counter()
                    held = build()
                    times[phase].append((time.perf_counter() - t0) * 1e3)
                # `held` keeps the memory phase's handle alive: compile() of the
                # same text is now a handle-cache hit
                t0 = time.perf_counter()
                for _ in range(hits):
                    hm.compile(expr, sig, name=name)
                handle_us.append((time.perf_counter() - t0) / hits * 1e6)
                if combine:
                    t0 = time.perf_counter()
                    for _ in range(hits):
                        binding.prepare_reduce(hm.compile(expr, sig, name=name), *combine)
                    handle_prep_us.append((time.perf_counter() - t0) / hits * 1e6)
                del held
            after = binding.cache_stats()
            res[label] = {f"{p}_ms_median": round(float(np.median(v)), 4) for p, v in times.items()}
            res[label]["handle_hit_us_median"] = round(float(np.median(handle_us)), 2)
            if handle_prep_us:
                res[label]["handle_hit_with_prepare_us_median"] = round(float(np.median(handle_prep_us)), 2)
            res[label]["cache_counts"] = {f: after[f] - before[f]
                                          for f in ("compiles", "disk_hits", "memory_hits")}
    finally:
        if saved is None:
            os.environ.pop("HIPMR_CACHE_DIR", None)
        else:
            os.environ["HIPMR_CACHE_DIR"] = saved
        shutil.rmtree(tmp, ignore_errors=True)
    sig, stmt = workloads.E1
    k = hm.compile(stmt, sig, name="e1_lincomb")
    n = 4096
    x = torch.zeros(n, device=dev)
    y = torch.zeros(n, device=dev)
    z = torch.empty(n, device=dev)
    args = [z, x, y]
    hm.elementwise(k, n, args)
    torch.cuda.synchronize()
    host = []
    for _ in range(5):
        t0 = time.perf_counter()
        for _ in range(launches):
            hm.elementwise(k, n, args)
        host.append((time.perf_counter() - t0) / launches * 1e6)
        torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(launches):
        hm.elementwise(k, n, args)
    b.record(stream)
    torch.cuda.synchronize()
    res["launch_E1_4096"] = {"host_us_per_call": round(float(np.median(host)), 2),
                             "gpu_us_per_launch_back_to_back": round(a.elapsed_time(b) * 1e3 / launches, 2)}
    return res


def bench_dot(torch, hm, workloads, dev, stream, checks, reps=200):
    """The small dot product x . y over 2^20 float32 (8.4 MB, about 1 us of
    HBM traffic): a launch-bound call, reported in microseconds.  `async_us`
    is the per-call time of back-to-back calls (HIP events around all of
    them); `synced_us` the median of single calls each followed by a host
    synchronisation (submission + both kernels + the wait); `graph_us` the
    per-call time of ten calls captured in one HIP graph and replayed."""
    x, y = workloads.dot_1m()
    xd, yd = (torch.from_numpy(a).to(dev) for a in (x, y))
    out = torch.empty((), dtype=torch.float32, device=dev)
    k = hm.compile("x[i]*y[i]", "float: const float *x, const float *y", name="dot_1m")
    from paper_1304_5553_amd import hipmr as binding
    ws = binding.workspace(binding.reduce_workspace_bytes(k, x.size), dev, stream.cuda_stream)
    call = lambda: hm.reduce(k, None, "a+b", "0", x.size, [xd, yd], out, workspace_buf=ws)
    for _ in range(20):
        call()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        call()
    b.record(stream)
    torch.cuda.synchronize()
    async_us = a.elapsed_time(b) * 1e3 / reps
    synced = []
    for _ in range(reps):
        t0 = time.perf_counter()
        call()
        torch.cuda.synchronize()
        synced.append((time.perf_counter() - t0) * 1e6)
    gpu_ms = _time_ms(torch, call, reps, stream)
    eager = out.clone()
    # ten calls captured in one HIP graph (on a side stream: the legacy
    # default stream cannot be captured), replayed: the per-call time with
    # the host's launch overhead taken away
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = hm.Graph()
    with graph.capture(side):
        for _ in range(10):
            hm.reduce(k, None, "a+b", "0", x.size, [xd, yd], out, workspace_buf=ws, stream=side)
    out.fill_(float("nan"))
    torch.cuda.synchronize()
    graph.launch(side)
    torch.cuda.synchronize()
    same = bool(torch.equal(out, eager))
    graph_ms = _time_ms(torch, lambda: graph.launch(side), 20, side) / 10
    checks["dot"] = float(eager.item())
    return {"n": int(x.size), "bytes": 8 * int(x.size), "async_us": round(async_us, 2),
            "synced_us_p50": round(float(np.median(synced)), 2),
            "event_us_p50": round(gpu_ms * 1e3, 2),
            "graph_us_per_call": round(graph_ms * 1e3, 2), "graph_equals_eager": same,
            "GB/s_async": round(8 * x.size / async_us / 1e3, 1),
            "note": "launch-bound: 8.4 MB is about 1 us of HBM traffic; GB/s is not a roofline claim"}


def bench_shifted(torch, hm, dev, stream, reps=20):
    """Shifted reads name[i +/- E] on the vector kernels against the
    one-element kernels: the five-point stencil q = A p on a 4096^2 grid
    (8 B per unknown: p read once, q written; the neighbours come from the
    caches) and the lag-1 product sum over 2^28 float32 (4 B per element);
    inputs U[0, 1) from a device generator seeded with 10."""
    from paper_1304_5553_amd import cg as hcg
    res = {}
    gen = torch.Generator(device=dev)
    gen.manual_seed(10)
    nx = 4096
    m = nx * nx
    p = torch.rand(m, device=dev, generator=gen)
    q = torch.empty(m, device=dev)
    k = hm.compile(hcg.SPMV[1], hcg.SPMV[0], name="cg_spmv")
    row = {"n": m, "bytes_per_element": 8}
    for tag, cfg in (("vector", None), ("one_element", {"flags": hm.CFG_FORCE_SCALAR})):
        ms = _time_ms(torch, lambda: hm.elementwise(k, m, [q, p, nx], config=cfg), reps, stream)
        row[tag] = {"us": round(ms * 1e3, 2), "GB/s": round(8 * m / ms / 1e6, 1)}
    row["speedup"] = round(row["one_element"]["us"] / row["vector"]["us"], 2)
    res["stencil_4096x4096"] = row
    del p, q
    n = 1 << 28
    x = torch.rand(n, device=dev, generator=gen)
    out = torch.empty((), device=dev)
    r = hm.compile("(i + 1 < n ? x[i + 1] : 0.0f) * x[i]", "float: const float *x", name="lag1")
    row = {"n": n, "bytes_per_element": 4}
    for tag, cfg in (("vector", None), ("one_element", {"flags": hm.CFG_FORCE_SCALAR})):
        ms = _time_ms(torch, lambda: hm.reduce(r, None, "a+b", "0", n, [x], out, config=cfg), reps, stream)
        row[tag] = {"us": round(ms * 1e3, 2), "GB/s": round(4 * n / ms / 1e6, 1)}
    row["speedup"] = round(row["one_element"]["us"] / row["vector"]["us"], 2)
    res["lag1_sum_2e28"] = row
    del x
    torch.cuda.empty_cache()
    return res


def bench_precision(torch, hm, workloads, dev, stream, checks, reps=10, copies=4):
    """Compensated sum and scaled two-pass L2 norm at n = 2**27 per format,
    for the lognormal values and for the cancellation case.  `copies` rotated
    copies of the input (>= 4 x 134-268 MB) keep the working set out of the
    256 MB last-level cache.  The results of the last timed calls go to the
    accuracy checks."""
    n = workloads.N_PRECISION
    out = {}
    checks["precision"] = {}
    for case in ("lognormal", "cancel"):
        v64 = workloads.precision_values(n, case)
        for fmt in ("bfloat16", "float16", "fp8_e4m3"):
            q = workloads.quantize(fmt, v64)
            tdt = {"bfloat16": torch.bfloat16, "float16": torch.float16,
                   "fp8_e4m3": torch.float8_e4m3fn}[fmt]
            host = torch.from_numpy(q.bits)
            host = host.view(torch.int16 if host.element_size() == 2 else torch.uint8).view(tdt)
            bufs = [host.to(dev) for _ in range(copies)]
            k = hm.compile("x[i]", f"float: const {fmt} *x", name=f"bench_{fmt[:4]}")
            o_sum = torch.empty((), dtype=torch.float64, device=dev)
            o_nrm = torch.empty((), dtype=torch.float64, device=dev)
            ws = hm.hipmr.workspace(hm.reduce_workspace_bytes(k, n), dev, stream.cuda_stream)
            it = [0]

            def nxt():
                it[0] += 1
                return bufs[it[0] % copies]
            inv = 1.0 / q.scale
            t_sum = _time_ms(torch, lambda: hm.reduce_compensated(k, n, [nxt()], inv, o_sum, ws),
                             reps, stream)
            sum_symbols = k.last_symbols()
            t_nrm = _time_ms(torch, lambda: hm.norm2(k, n, [nxt()], inv, 2, o_nrm, ws), reps, stream)
            nbytes = n * host.element_size()
            checks["precision"][(fmt, case)] = (float(o_sum.item()), float(o_nrm.item()))
            out.setdefault(case, {})[fmt] = {
                "sum_ms": round(t_sum, 4), "sum_GB/s": round(nbytes / t_sum / 1e6, 1),
                "sum_frac_of_peak": round(nbytes / t_sum / 1e6 / HBM_PEAK_GBS, 4),
                "norm2_ms": round(t_nrm, 4), "norm2_GB/s": round(2 * nbytes / t_nrm / 1e6, 1),
                "norm2_frac_of_peak": round(2 * nbytes / t_nrm / 1e6 / HBM_PEAK_GBS, 4),
                "sum_symbols": sum_symbols, "norm2_symbols": k.last_symbols()}
            del bufs
            torch.cuda.empty_cache()
        del v64
    return {"n": n, "workload": "lognormal(0,3) x random sign, and the cancellation case "
                                "[x; -x (1 + eps)]; per-tensor power-of-two scale",
            "bytes_note": "sum reads n*size once; the scaled norm reads it twice",
            "inputs": f"{copies} rotated copies (out of the 256 MB last-level cache)",
            "cases": out}


def bench_scan(torch, hm, workloads, dev, stream, reps=10):
    """Prefix scans at n = 2^28 (the plain workload's arrays): inclusive float
    sum of x (4 B read twice + 4 B written = 12 B/element) and inclusive
    int64 sum of the int32 k (4 + 4 + 8 = 16 B/element)."""
    n = workloads.N_PLAIN
    x, _ = workloads.plain_xy(n)
    xd = torch.from_numpy(x).to(dev)
    kd = torch.from_numpy(workloads.plain_k(n)).to(dev)
    res = {"n": n}
    for name, expr, sig, src, out_dt, per in (
            ("sum_f32", "x[i]", "float: const float *x", xd, torch.float32, 12),
            ("sum_i32_to_i64", "k[i]", "long: const int *k", kd, torch.int64, 16)):
        k = hm.compile(expr, sig, name=f"scan_{name}")
        out = torch.empty(n, dtype=out_dt, device=dev)
        ws = hm.hipmr.workspace(hm.scan_workspace_bytes(k, n), dev, stream.cuda_stream)
        ms = _time_ms(torch, lambda: hm.scan(k, "a+b", "0", n, [src], out, workspace_buf=ws), reps, stream)
        gbs = per * n / ms / 1e6
        res[name] = {"ms": round(ms, 4), "bytes_per_element": per, "GB/s": round(gbs, 1),
                     "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                     "elements_per_s": round(n / ms * 1e3, 1), "symbols": k.last_symbols()}
        del out
    del xd, kd
    torch.cuda.empty_cache()
    return res


def bench_cg(torch, hm, dev):
    """Conjugate gradients on the five-point model problem: time per
    iteration, eager (nine launches) and replayed from a HIP graph, on a
    4096 x 4096 grid (bandwidth-bound) and a 256 x 256 grid (launch-bound);
    52 algorithmic bytes per unknown and iteration."""
    from paper_1304_5553_amd import cg as hcg
    res = {"bytes_per_unknown": hcg.BYTES_PER_UNKNOWN}
    for nx in (4096, 256):
        n = nx * nx
        rng = np.random.default_rng(8)
        b = torch.from_numpy(rng.uniform(-1, 1, n).astype(np.float32)).to(dev)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            solver = hcg.PoissonCG(nx, nx, device=dev, stream=stream)
            solver.solve(b, 2)                               # loads every kernel
            graph = solver.capture(10)
            row = {"n": n}
            for mode in ("eager", "graph"):
                solver.start(b)
                stream.synchronize()
                t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0.record(stream)
                for _ in range(5):
                    if mode == "graph":
                        graph.launch(stream)
                    else:
                        for _ in range(10):
                            solver.step()
                t1.record(stream)
                stream.synchronize()
                ms = t0.elapsed_time(t1) / 50
                row[mode] = {"ms_per_iter": round(ms, 5),
                             "GB/s": round(hcg.BYTES_PER_UNKNOWN * n / ms / 1e6, 1)}
            row["graph_speedup"] = round(row["eager"]["ms_per_iter"] / row["graph"]["ms_per_iter"], 2)
            row["rr_after_50"] = float(solver.rr.item())
        res[f"{nx}x{nx}"] = row
        del solver, graph, b
        torch.cuda.empty_cache()
    return res


def bench_lazy(torch, dev, stream, reps=10):
    """The temporaries problem: z = 2.5 x y + sqrt(x x + y y) - 0.5 w over
    n = 2^26 float32, as one fused generated kernel (16 B/element) and as one
    kernel per operator (each writing a temporary)."""
    from paper_1304_5553_amd import lazy as lz
    n = 1 << 26
    rng = np.random.default_rng(9)
    x, y, w = (torch.from_numpy(rng.uniform(-1, 1, n).astype(np.float32)).to(dev) for _ in range(3))
    X, Y, W = lz.lazy(x), lz.lazy(y), lz.lazy(w)
    expr = 2.5 * X * Y + lz.sqrt(X * X + Y * Y) - 0.5 * W
    out = torch.empty(n, device=dev)
    fused_ms = _time_ms(torch, lambda: expr.eval(out=out), reps, stream)
    unfused_ms = _time_ms(torch, lambda: expr.eval(out=out, fused=False), reps, stream)
    # unfused traffic: every operator reads its array operands and writes a temporary
    def count(node):
        if node.op in ("leaf", "const"):
            return 0, 0
        k, b = 0, 0
        for a in node.args:
            kk, bb = count(a)
            k, b = k + kk, b + bb
        return k + 1, b + 4 * (sum(1 for a in node.args if a.op != "const") + 1)
    kernels, per = count(expr)
    del x, y, w, out
    torch.cuda.empty_cache()
    return {"n": n, "expression": "2.5*x*y + sqrt(x*x + y*y) - 0.5*w",
            "fused": {"ms": round(fused_ms, 4), "kernels": 1, "bytes_per_element": 16,
                      "GB/s": round(16 * n / fused_ms / 1e6, 1)},
            "unfused": {"ms": round(unfused_ms, 4), "kernels": kernels, "bytes_per_element": per,
                        "GB/s": round(per * n / unfused_ms / 1e6, 1)},
            "speedup": round(unfused_ms / fused_ms, 2)}


def bench_complex(torch, hm, workloads, dev, stream, reps=10):
    """complex64 at n = 2^27 (1 GiB per array): z = a x + b y with complex
    scalars (24 B/element), the conjugated dot sum conj(x) y (16 B/element)
    and the sum of x (8 B/element)."""
    n = workloads.N_COMPLEX
    x, y = workloads.complex_xy(n)
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    del x, y
    z = torch.empty_like(xd)

    def row(ms, per, k):
        gbs = per * n / ms / 1e6
        return {"ms": round(ms, 4), "bytes_per_element": per, "GB/s": round(gbs, 1),
                "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                "elements_per_s": round(n / ms * 1e3, 1), "symbols": k.last_symbols()}

    res = {"n": n}
    sig, stmt = workloads.C_AXPBY
    k = hm.compile(stmt, sig, name="c_axpby")
    args = [z, workloads.C_A, xd, workloads.C_B, yd]
    res["axpby"] = row(_time_ms(torch, lambda: hm.elementwise(k, n, args), reps, stream), 24, k)
    out = torch.empty((), dtype=torch.complex64, device=dev)
    for name, spec, srcs, per in (("conj_dot", workloads.C_DOT, [xd, yd], 16),
                                  ("sum", workloads.C_SUM, [xd], 8)):
        sig, mp, comb, neu = spec
        k = hm.compile(mp, sig, name=f"c_{name}")
        ws = hm.hipmr.workspace(hm.reduce_workspace_bytes(k, n), dev, stream.cuda_stream)
        call = lambda: hm.reduce(k, None, comb, neu, n, srcs, out, workspace_buf=ws)
        res[name] = row(_time_ms(torch, call, reps, stream), per, k)
    del xd, yd, z
    torch.cuda.empty_cache()
    return res


def bench_batched(torch, hm, workloads, dev, checks, reps=12, baseline_reps=2, copies=3,
                  eager_only=False):
    """4096 lognormal segments (62,032,791 float32): segmented sum, max and dot
    (three persistent launch sequences) replayed from HIP graphs, against one
    plain launch pair per segment (eager, and captured in a graph).  The
    batched graphs run the three ops on three streams (fork / join inside the
    graph, so one op's planner and fold overlap the others' tile kernels) and,
    for reference, one after the other on one stream.  Every op of every
    replay reads arrays of its own: `copies` rotated sets of one x per op and
    one y (12 x 0.25 GB, far beyond the 256 MB last-level cache), one graph
    per set, so no op reads what another just read and the inputs come from
    HBM."""
    offsets, x, y = workloads.segments()
    nseg = len(offsets) - 1
    total = int(offsets[-1])
    od = torch.from_numpy(offsets).to(dev)
    ops = {"sum": ("x[i]", "a+b", "0", 4), "max": ("x[i]", "max(a,b)", "-INFINITY", 4),
           "dot": ("x[i]*y[i]", "a+b", "0", 8)}
    xh, yh = torch.from_numpy(x), torch.from_numpy(y)
    sets = [({op: xh.to(dev) for op in ops}, yh.to(dev)) for _ in range(copies)]
    xd, yd = sets[0][0]["sum"], sets[0][1]
    sig = "float: const float *x, const float *y"
    ks = {op: hm.compile(m, sig, name=f"batch_{op}") for op, (m, _, _, _) in ops.items()}
    stream = torch.cuda.Stream()
    side = {"max": torch.cuda.Stream(), "dot": torch.cuda.Stream()}
    res = {}
    with torch.cuda.stream(stream):
        outs = {op: torch.empty(nseg, device=dev) for op in ops}
        wss = {op: torch.empty(hm.segmented_workspace_bytes(ks[op], nseg, total),
                               dtype=torch.uint8, device=dev) for op in ops}
        tuned = {}
        for op, (m, comb, neu, _) in ops.items():
            tuned[op] = hm.autotune_segmented(ks[op], comb, neu, od, total, [xd, yd], outs[op],
                                              reps=3, workspace_buf=wss[op], stream=stream)

        def one(op, c, st):
            m, comb, neu, _ = ops[op]
            xs, ys = sets[c]
            hm.reduce_segmented(ks[op], comb, neu, od, total, [xs[op], ys], outs[op],
                                workspace_buf=wss[op], stream=st, config={"flags": hm.CFG_TUNED})

        def issue_serial(c=0):
            for op in ops:
                one(op, c, stream)

        def issue_concurrent(c=0):
            fork = torch.cuda.Event()
            fork.record(stream)
            for op, st in side.items():
                st.wait_event(fork)
                one(op, c, st)
            one("sum", c, stream)
            for st in side.values():
                join = torch.cuda.Event()
                join.record(st)
                stream.wait_event(join)
        issue_serial()
        if eager_only:
            for c in range(copies):
                issue_serial(c)
            torch.cuda.synchronize()
            return {"eager_only": True, "symbols": {op: ks[op].last_symbols() for op in ops},
                    "tuned": tuned}
        issue_concurrent()
        torch.cuda.synchronize()
        graphs = {"concurrent": [], "serial": []}
        for c in range(copies):
            for kind, fn in (("concurrent", issue_concurrent), ("serial", issue_serial)):
                g = hm.Graph()
                with g.capture(stream):
                    fn(c)
                graphs[kind].append(g)
        it = [0]

        def replay(kind):
            it[0] += 1
            graphs[kind][it[0] % copies].launch(stream)

        def eager():
            it[0] += 1
            issue_serial(it[0] % copies)
        t_batched = _time_ms(torch, lambda: replay("concurrent"), reps, stream)
        t_serial = _time_ms(torch, lambda: replay("serial"), reps, stream)
        t_eager_batched = _time_ms(torch, eager, reps, stream)
        torch.cuda.synchronize()
        checks["batched"] = {op: outs[op].cpu().numpy().astype(np.float64) for op in ops}
        symbols = {op: ks[op].last_symbols() for op in ops}
        # baseline: one plain map-reduce (two launches) per segment and op
        plain_out = torch.empty(nseg, device=dev)
        ws1 = hm.hipmr.workspace(hm.reduce_workspace_bytes(ks["sum"], 1), dev, stream.cuda_stream)
        views = [(int(a), int(b)) for a, b in zip(offsets[:-1], offsets[1:])]

        def per_segment():
            for op, (m, comb, neu, _) in ops.items():
                k = ks[op]
                for s, (a, b) in enumerate(views):
                    hm.reduce(k, None, comb, neu, b - a, [xd[a:b], yd[a:b]], plain_out[s], ws1,
                              stream=stream)
        t_plain = _time_ms(torch, per_segment, baseline_reps, stream)
        pgraph = hm.Graph()
        with pgraph.capture(stream):
            per_segment()
        t_plain_graph = _time_ms(torch, lambda: pgraph.launch(stream), baseline_reps, stream)
    nbytes = sum(total * b for (_, _, _, b) in ops.values())
    res = {"nseg": nseg, "total_elements": total, "algorithmic_bytes": nbytes,
           "inputs": f"{copies} rotated sets of one x per op and one y (each op reads its own "
                     f"arrays; out of the 256 MB last-level cache)",
           "batched_graph_ms": round(t_batched, 4),
           "batched_graph_GB/s": round(nbytes / t_batched / 1e6, 1),
           "batched_graph_frac_of_peak": round(nbytes / t_batched / 1e6 / HBM_PEAK_GBS, 4),
           "batched_graph_note": "the three ops on three streams inside one graph",
           "serial_graph_ms": round(t_serial, 4),
           "serial_graph_GB/s": round(nbytes / t_serial / 1e6, 1),
           "batched_eager_ms": round(t_eager_batched, 4),
           "per_segment_eager_ms": round(t_plain, 3),
           "per_segment_graph_ms": round(t_plain_graph, 3),
           "speedup_vs_per_segment": round(t_plain / t_batched, 1),
           "speedup_vs_per_segment_graph": round(t_plain_graph / t_batched, 1),
           "launches_batched": sum(len(v) for v in symbols.values()),
           "launches_per_segment": 3 * nseg * 2,
           "symbols": symbols, "tuned": tuned}
    del sets
    torch.cuda.empty_cache()
    return res


SERVE_MODES = (("resident", dict(resident=1)),
               ("batched", dict(nstreams=4, max_batch_jobs=1024)),
               ("per_job", dict(nstreams=4, max_batch_jobs=1)))


def bench_serving(torch, hm, workloads, dev, checks, duration_s=4.0, warmup_s=1.0, rates=None,
                  checked_jobs=200, largest_jobs=20):
    """Poisson streams at 2k, 10k and 50k jobs/s (8 templates, float32 /
    bfloat16 50/50, n log-uniform over [2^10, 2^24], slices of a resident 2^24
    pool), plus a 200k jobs/s stress rate beyond them, replayed open-loop
    through three forms of the serving loop with a 64 GiB budget: the
    resident kernel fed from a descriptor ring (`resident`, the served form),
    batches launched on 4 streams (`batched`), and one launch pair per job on
    the same 4 streams (`per_job`, the baseline); latency = scheduled arrival
    -> the loop sees the job's completion flag (result in device memory).
    Per configured rate, the resident results of `checked_jobs` measured jobs
    (the `largest_jobs` largest among them) go to the accuracy checks, and
    every job's result is compared bit for bit across the three forms."""
    f32, bf16 = workloads.serving_pool()
    dev_f32 = {k: torch.from_numpy(v).to(dev) for k, v in f32.items()}
    dev_bf16 = {k: torch.from_numpy(v.view(np.int16)).view(torch.bfloat16).to(dev)
                for k, v in bf16.items()}
    res = {"pool": workloads.N_POOL, "duration_s": duration_s, "warmup_s": warmup_s,
           "budget_bytes": 64 << 30, "served_form": "resident", "baseline": "per_job",
           "rates": {}}
    for rate in rates or (*workloads.SERVING_RATES, 200000):
        sched = workloads.serving_schedule(rate, warmup_s + duration_s)
        m = len(sched["n"])
        es = np.where(sched["bf16"], 2, 4)
        arrays = np.where(np.isin(sched["tmpl"], [1, 4, 7]), 2, 1)
        job_bytes = sched["n"] * es * arrays
        out = torch.empty(m, dtype=torch.float64, device=dev)
        row = {"jobs": int(m)}
        results = {}
        if rate not in workloads.SERVING_RATES:
            row["note"] = "stress rate beyond the configured ones"
        for mode, kw in SERVE_MODES:
            server = hm.Server(hbm_budget_bytes=64 << 30, **kw)
            jobs = server.jobs(m)
            for key in ("x", "y", "w"):
                base_f = dev_f32[key].data_ptr()
                base_b = dev_bf16[key].data_ptr()
                jobs[key] = np.where(sched["bf16"], base_b + sched["offset"] * 2,
                                     base_f + sched["offset"] * 4).astype(np.uint64)
            jobs["n"] = sched["n"]
            jobs["tmpl"] = sched["tmpl"]
            jobs["dtype"] = np.where(sched["bf16"], hm.hipmr.BF16, hm.hipmr.F32)
            jobs["arrival_ns"] = sched["arrival_ns"]
            jobs["out"] = out.data_ptr() + 8 * np.arange(m, dtype=np.uint64)
            jobs["a"], jobs["b"] = 2.5, -0.5
            out.fill_(float("nan"))
            torch.cuda.synchronize()
            done = server.run_schedule(jobs)
            server.close()
            torch.cuda.synchronize()
            results[mode] = out.cpu().numpy().copy()
            meas = sched["arrival_ns"] >= int(warmup_s * 1e9)
            lat = (done["done_ns"] - done["arrival_ns"])[meas] / 1e3
            first = int(np.min(done["arrival_ns"][meas]))
            last = int(np.max(done["done_ns"][meas]))
            span = (last - first) / 1e9
            queue = (done["launch_ns"] - done["arrival_ns"])[meas] / 1e3
            service = (done["done_ns"] - done["launch_ns"])[meas] / 1e3
            row[mode] = {"p50_us": round(float(np.percentile(lat, 50)), 1),
                         "p99_us": round(float(np.percentile(lat, 99)), 1),
                         "mean_us": round(float(np.mean(lat)), 1),
                         "jobs_per_s": round(int(meas.sum()) / span, 1),
                         "GB/s": round(float(job_bytes[meas].sum()) / span / 1e9, 2),
                         "queue_p50_us": round(float(np.percentile(queue, 50)), 1),
                         "service_p50_us": round(float(np.percentile(service, 50)), 1),
                         "mean_jobs_together": round(float(np.mean(done["batch_jobs"][meas])), 2),
                         "status_ok": bool(np.all(done["status"] == 0))}
        if rate in workloads.SERVING_RATES:
            meas_idx = np.nonzero(sched["arrival_ns"] >= int(warmup_s * 1e9))[0]
            by_size = meas_idx[np.argsort(sched["n"][meas_idx], kind="stable")]
            largest = by_size[-largest_jobs:]
            rng = np.random.default_rng(rate)
            rest = np.setdiff1d(meas_idx, largest)
            idx = np.sort(np.concatenate([largest, rng.choice(rest, checked_jobs - largest_jobs,
                                                              replace=False)]))
            r, b, p = results["resident"], results["batched"], results["per_job"]
            checks.setdefault("served", {})[rate] = {
                "duration_s": warmup_s + duration_s, "idx": idx, "got": r[idx],
                "largest": int(largest.size), "compared": int(m),
                "same": bool(np.array_equal(r.view(np.uint64), p.view(np.uint64)) and
                             np.array_equal(b.view(np.uint64), p.view(np.uint64)))}
        for mode in ("resident", "batched"):
            row[f"{mode}_p99_speedup"] = round(row["per_job"]["p99_us"] / row[mode]["p99_us"], 2)
            row[f"{mode}_p50_speedup"] = round(row["per_job"]["p50_us"] / row[mode]["p50_us"], 2)
        res["rates"][str(rate)] = row
        print(f"serving {rate}/s done", file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (--gpus {args.gpus} requested); how the path "
              "would shard across GPUs is described, not measured", file=sys.stderr)
        sys.exit(2)

    import workloads

    n = args.n
    x, y = workloads.plain_xy(n)
    k = workloads.plain_k(n)
    # the CPU leg's worker processes are forked here, before the GPU is touched
    leg = None if args.no_cpu_baseline else CpuLeg(x, y, k, n)
    checks = {}

    import torch

    import paper_1304_5553_amd as hm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    kd = torch.from_numpy(k).to(dev)
    z = torch.empty_like(xd)
    outs = {"count": torch.empty((), dtype=torch.int64, device=dev),
            "sum": torch.empty((), dtype=torch.int64, device=dev),
            "max": torch.empty((), dtype=torch.float32, device=dev)}

    def kernels():
        # the compile step of the hot path: a memory-cache hit after the first call
        return {
            "E1": hm.compile(workloads.E1[1], workloads.E1[0], name="e1_lincomb"),
            "E2": hm.compile(workloads.E2[1], workloads.E2[0], name="e2_hypot"),
            "R1": hm.compile(workloads.R_COUNT[1], workloads.R_COUNT[0], name="r1_count"),
            "R2": hm.compile(workloads.R_SUM[1], workloads.R_SUM[0], name="r2_sum"),
            "R3": hm.compile(workloads.R_MAX[1], workloads.R_MAX[0], name="r3_max"),
            "COPY": hm.compile("z[i] = x[i]", "float *z, const float *x", name="copy"),
        }

    ks = kernels()
    stream = torch.cuda.current_stream()
    ws = hm.hipmr.workspace(hm.reduce_workspace_bytes(ks["R1"], n), dev, stream.cuda_stream)
    bytes_per = {"E1": 12 * n, "E2": 12 * n, "R1": 4 * n, "R2": 4 * n, "R3": 4 * n, "COPY": 8 * n}
    ops = [o.strip().upper() for o in args.ops.split(",") if o.strip()]
    if any(o not in bytes_per for o in ops):
        print(f"bench.py: unknown op in --ops {args.ops}", file=sys.stderr)
        sys.exit(2)

    def run_op(name, kk):
        if name == "E1":
            hm.elementwise(kk["E1"], n, [z, xd, yd])
        elif name == "E2":
            hm.elementwise(kk["E2"], n, [z, xd, yd])
        elif name == "R1":
            hm.reduce(kk["R1"], workloads.R_COUNT[1], "a+b", "0", n, [kd], outs["count"], ws)
        elif name == "R2":
            hm.reduce(kk["R2"], workloads.R_SUM[1], "a+b", "0", n, [kd], outs["sum"], ws)
        elif name == "COPY":
            hm.elementwise(kk["COPY"], n, [z, xd])
        else:
            hm.reduce(kk["R3"], workloads.R_MAX[1], "max(a,b)", "-INFINITY", n, [xd],
                      outs["max"], ws)

    last = {}

    def step(events=None):
        kk = kernels()
        last.update(kk)
        for name in ops:
            if events is not None:
                events[name][0].record(stream)
            run_op(name, kk)
            if events is not None:
                events[name][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = {name: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(args.steps)] for name in ops}
    per_op_ms = {name: [] for name in ops}
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for s in range(args.steps):
        step({name: ev[name][s] for name in ops})
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    for name in ops:
        per_op_ms[name] = [a.elapsed_time(b) for a, b in ev[name]]

    ms_per_step = total_ms / args.steps
    step_bytes = sum(bytes_per[o] for o in ops)
    value = step_bytes / (ms_per_step / 1e3) / 1e9
    op_stats = {}
    for name in ops:
        avg = float(np.mean(per_op_ms[name]))
        op_stats[name] = {"ms": round(avg, 4), "GB/s": round(bytes_per[name] / avg / 1e6, 1),
                          "frac_of_peak": round(bytes_per[name] / avg / 1e6 / HBM_PEAK_GBS, 4),
                          "elements_per_s": round(n / (avg / 1e3), 1)}
    dominant = max(ops, key=lambda o: np.mean(per_op_ms[o]))
    dom_ms = float(np.mean(per_op_ms[dominant]))
    achieved = bytes_per[dominant] / (dom_ms / 1e3) / 1e9
    dom_symbol = last[dominant].last_symbols()[0]
    traffic = counter_traffic(dom_symbol)

    # results of the last step, and the elementwise outputs of one more pass
    # each, for the accuracy checks
    result = {}
    if "R1" in ops:
        result["R1_count"] = int(outs["count"].item())
    if "R2" in ops:
        result["R2_sum"] = int(outs["sum"].item())
    if "R3" in ops:
        result["R3_max"] = float(outs["max"].item())
    if leg is not None and {"E1", "E2", "R1", "R2", "R3"} <= set(ops):
        for name in ("E1", "E2"):
            run_op(name, last)
            torch.cuda.synchronize()
            torch.from_numpy(_LEG["z"][name]).copy_(z)
        checks["plain"] = {"R1": result["R1_count"], "R2": result["R2_sum"], "R3": result["R3_max"]}

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (E1, E2, R3); i32 loads with i64 accumulation (R1, R2)",
        "data": "synthetic",
        "config": {"workload": "plain fused elementwise + map-reduce at n=2^28: "
                               "E1 z=2.5x-0.5y, E2 z=sqrt(x*x+y*y), R1 count(k%7==3), "
                               "R2 sum(k), R3 max(x)",
                   "n": n, "ops": ops, "step_bytes": step_bytes},
        "frac_of_peak": round(value / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "avg_launch_ms": round(dom_ms, 4), "symbol": dom_symbol,
                     "traffic": traffic,
                     "traffic_source": COUNTERS_MD if traffic is not None else None},
        "ops": op_stats,
        "results": result,
        "wall_s_timed": round(wall, 3),
    }
    ext = set() if args.no_extensions else {e.strip() for e in args.extensions.split(",")}
    if ext:
        del xd, yd, kd, z
        torch.cuda.empty_cache()
    if "compile" in ext:
        line["compile"] = bench_compile(torch, hm, workloads, dev, stream)
        print("compile done", file=sys.stderr, flush=True)
    if "dot" in ext:
        line["dot"] = bench_dot(torch, hm, workloads, dev, stream, checks)
        print("dot done", file=sys.stderr, flush=True)
    if "precision" in ext:
        line["precision"] = bench_precision(torch, hm, workloads, dev, stream, checks)
        print("precision done", file=sys.stderr, flush=True)
    if "batched" in ext:
        line["batched"] = bench_batched(torch, hm, workloads, dev, checks,
                                        eager_only=args.batched_eager_only)
        print("batched done", file=sys.stderr, flush=True)
    if "shifted" in ext:
        line["shifted"] = bench_shifted(torch, hm, dev, stream)
        print("shifted done", file=sys.stderr, flush=True)
    if "scan" in ext:
        line["scan"] = bench_scan(torch, hm, workloads, dev, stream)
        print("scan done", file=sys.stderr, flush=True)
    if "lazy" in ext:
        line["lazy"] = bench_lazy(torch, dev, stream)
        print("lazy done", file=sys.stderr, flush=True)
    if "complex" in ext:
        line["complex"] = bench_complex(torch, hm, workloads, dev, stream)
        print("complex done", file=sys.stderr, flush=True)
    if "cg" in ext:
        line["cg"] = bench_cg(torch, hm, dev)
        print("cg done", file=sys.stderr, flush=True)
    if "served" in ext:
        rates = tuple(int(r) for r in args.serving_rates.split(",") if r.strip()) or None
        line["served"] = bench_serving(torch, hm, workloads, dev, checks,
                                       duration_s=args.serving_duration, rates=rates)
    if leg is not None:
        try:
            line["cpu_baseline"] = leg.baseline(args.cpu_sample_one, args.cpu_sample)
            print("cpu baseline done", file=sys.stderr, flush=True)
            if not args.no_accuracy:
                line["accuracy"] = leg.accuracy(checks)
                print("accuracy done", file=sys.stderr, flush=True)
                if not line["accuracy"]["all_ok"]:
                    print("bench.py: a timed result is outside its gate against the oracle",
                          file=sys.stderr, flush=True)
        finally:
            leg.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
