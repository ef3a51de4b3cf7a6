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
    p.add_argument("--serving-rates", default="",
                   help="comma list of jobs/s (default: 2000,10000,50000 and the 200000 stress rate)")
    p.add_argument("--serving-duration", type=float, default=5.0,
                   help="measured seconds of each serving rate (after 1 s of warm-up)")
    p.add_argument("--cpu-sample", type=int, default=1 << 27,
                   help="elements per op for the oracle timing")
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


def cpu_baseline(x, y, k, sample):
    """The oracle (test infrastructure) timed on the first `sample` elements
    of every op; reported as algorithmic GB/s of that sample."""
    import oracle
    import workloads
    m = min(sample, x.size)
    xs, ys, ks = x[:m], y[:m], k[:m]
    zero = np.zeros(1, np.float32)
    c0 = time.process_time()
    t0 = time.perf_counter()
    oracle.elementwise(workloads.E1[0], workloads.E1[1], m, [zero, xs, ys])
    oracle.elementwise(workloads.E2[0], workloads.E2[1], m, [zero, xs, ys])
    for sig, mp, comb, neu in (workloads.R_COUNT, workloads.R_SUM):
        oracle.reduce(sig, mp, comb, neu, m, [ks])
    oracle.reduce(workloads.R_MAX[0], workloads.R_MAX[1], "max(a,b)", "-INFINITY", m, [xs])
    dt = time.perf_counter() - t0
    busy = (time.process_time() - c0) / dt     # CPU seconds per second: threads in use
    nbytes = m * (12 + 12 + 4 + 4 + 4)
    return {"value": round(nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": max(1, round(busy)),
            "cpu_s_per_s": round(busy, 2), "kind": "oracle",
            "sample": f"first {m} elements of each of E1, E2, R1, R2, R3 "
                      f"({nbytes / 1e6:.0f} MB algorithmic) in {dt:.1f} s"}


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


def bench_compile(torch, hm, workloads, dev, stream, reps=5, launches=2000):
    """The host side of the path (front end, code generation, compile cache,
    launch): the cost of compile(expr, dtypes) when hipRTC
    runs (cold), when the code object comes from the disk cache (after the
    in-memory cache is dropped) and when it is in memory (front end, code
    generation with the symbol's SHA-256, and the lookup), for E1 and for
    R2's two reduce
    kernels; then the host time of one elementwise call (argument marshalling
    and the enqueue) and the GPU time per launch of a 4096-element E1, back to
    back.  Each cold source is new (its own kernel name) and the disk cache is
    a fresh directory, so nothing is found by accident."""
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
            before = binding.cache_stats()
            for r in range(reps):
                name = f"cold{r}_{tag}"

                def build():
                    k = hm.compile(expr, sig, name=name)
                    if combine:
                        binding.prepare_reduce(k, *combine)
                    return k

                for phase in ("cold", "disk", "memory"):
                    if phase == "disk":
                        binding.cache_drop_memory()
                    t0 = time.perf_counter()
                    build()
                    times[phase].append((time.perf_counter() - t0) * 1e3)
            after = binding.cache_stats()
            res[label] = {f"{p}_ms_median": round(float(np.median(v)), 4) for p, v in times.items()}
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


def bench_dot(torch, hm, workloads, dev, stream, reps=200):
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


def bench_precision(torch, hm, workloads, dev, stream, reps=10, copies=4):
    """Compensated sum and scaled two-pass L2 norm at n = 2**27 per format.
    `copies` rotated copies of the input (>= 4 x 134-268 MB) keep the working
    set out of the 256 MB last-level cache."""
    n = workloads.N_PRECISION
    v64 = workloads.precision_values(n, "lognormal")
    out = {}
    for fmt in ("bfloat16", "float16", "fp8_e4m3"):
        q = workloads.quantize(fmt, v64)
        tdt = {"bfloat16": torch.bfloat16, "float16": torch.float16,
               "fp8_e4m3": torch.float8_e4m3fn}[fmt]
        host = torch.from_numpy(q.bits)
        host = host.view(torch.int16 if host.element_size() == 2 else torch.uint8).view(tdt)
        bufs = [host.to(dev) for _ in range(copies)]
        k = hm.compile("x[i]", f"float: const {fmt} *x", name=f"bench_{fmt[:4]}")
        o = torch.empty((), dtype=torch.float64, device=dev)
        ws = hm.hipmr.workspace(hm.reduce_workspace_bytes(k, n), dev, stream.cuda_stream)
        it = [0]

        def nxt():
            it[0] += 1
            return bufs[it[0] % copies]
        inv = 1.0 / q.scale
        t_sum = _time_ms(torch, lambda: hm.reduce_compensated(k, n, [nxt()], inv, o, ws), reps, stream)
        sum_symbols = k.last_symbols()
        t_nrm = _time_ms(torch, lambda: hm.norm2(k, n, [nxt()], inv, 2, o, ws), reps, stream)
        nbytes = n * host.element_size()
        out[fmt] = {"sum_ms": round(t_sum, 4), "sum_GB/s": round(nbytes / t_sum / 1e6, 1),
                    "norm2_ms": round(t_nrm, 4),
                    "norm2_GB/s": round(2 * nbytes / t_nrm / 1e6, 1),
                    "sum_symbols": sum_symbols, "norm2_symbols": k.last_symbols()}
        del bufs
        torch.cuda.empty_cache()
    return {"n": n, "workload": "lognormal(0,3) x random sign, per-tensor power-of-two scale",
            "bytes_note": "sum reads n*size once; the scaled norm reads it twice", "formats": out}


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


def bench_batched(torch, hm, workloads, dev, reps=10, baseline_reps=2):
    """4096 lognormal segments (62,032,791 float32): segmented sum, max and dot
    as one graph replay of the persistent launch sequences, against one plain
    launch pair per segment (eager, and captured in a graph)."""
    offsets, x, y = workloads.segments()
    nseg = len(offsets) - 1
    total = int(offsets[-1])
    od = torch.from_numpy(offsets).to(dev)
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    ops = {"sum": ("x[i]", "a+b", "0", 4), "max": ("x[i]", "max(a,b)", "-INFINITY", 4),
           "dot": ("x[i]*y[i]", "a+b", "0", 8)}
    sig = "float: const float *x, const float *y"
    ks = {op: hm.compile(m, sig, name=f"batch_{op}") for op, (m, _, _, _) in ops.items()}
    stream = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(stream):
        outs = {op: torch.empty(nseg, device=dev) for op in ops}
        wss = {op: torch.empty(hm.segmented_workspace_bytes(ks[op], nseg, total),
                               dtype=torch.uint8, device=dev) for op in ops}
        tuned = {}
        for op, (m, comb, neu, _) in ops.items():
            tuned[op] = hm.autotune_segmented(ks[op], comb, neu, od, total, [xd, yd], outs[op],
                                              reps=3, workspace_buf=wss[op], stream=stream)

        def issue():
            for op, (m, comb, neu, _) in ops.items():
                hm.reduce_segmented(ks[op], comb, neu, od, total, [xd, yd], outs[op],
                                    workspace_buf=wss[op], stream=stream)
        issue()
        stream.synchronize()
        graph = hm.Graph()
        with graph.capture(stream):
            issue()
        t_batched = _time_ms(torch, lambda: graph.launch(stream), reps, stream)
        t_eager_batched = _time_ms(torch, issue, reps, stream)
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
           "batched_graph_ms": round(t_batched, 4),
           "batched_graph_GB/s": round(nbytes / t_batched / 1e6, 1),
           "batched_eager_ms": round(t_eager_batched, 4),
           "per_segment_eager_ms": round(t_plain, 3),
           "per_segment_graph_ms": round(t_plain_graph, 3),
           "speedup_vs_per_segment": round(t_plain / t_batched, 1),
           "speedup_vs_per_segment_graph": round(t_plain_graph / t_batched, 1),
           "launches_batched": 3 * 3, "launches_per_segment": 3 * nseg * 2,
           "tuned": tuned}
    return res


def bench_serving(torch, hm, workloads, dev, duration_s=5.0, warmup_s=1.0, rates=None):
    """Poisson streams at 2k, 10k and 50k jobs/s (8 templates, float32 /
    bfloat16 50/50, n log-uniform over [2^10, 2^24], slices of a resident 2^24
    pool), plus a 200k jobs/s stress rate beyond them, replayed open-loop
    through the continuous-batching loop and through the one-launch-pair-per-
    job baseline on the same 4 streams; latency = scheduled arrival -> the
    loop sees the job's completion flag (result in device memory)."""
    f32, bf16 = workloads.serving_pool()
    dev_f32 = {k: torch.from_numpy(v).to(dev) for k, v in f32.items()}
    dev_bf16 = {k: torch.from_numpy(v.view(np.int16)).view(torch.bfloat16).to(dev)
                for k, v in bf16.items()}
    res = {"pool": workloads.N_POOL, "duration_s": duration_s, "warmup_s": warmup_s,
           "budget_bytes": 64 << 30, "nstreams": 4, "rates": {}}
    for rate in rates or (*workloads.SERVING_RATES, 200000):
        sched = workloads.serving_schedule(rate, warmup_s + duration_s)
        m = len(sched["n"])
        es = np.where(sched["bf16"], 2, 4)
        arrays = np.where(np.isin(sched["tmpl"], [1, 4, 7]), 2, 1)
        job_bytes = sched["n"] * es * arrays
        out = torch.empty(m, dtype=torch.float64, device=dev)
        row = {"jobs": int(m)}
        if rate not in workloads.SERVING_RATES:
            row["note"] = "stress rate beyond the configured ones"
        for mode, max_jobs in (("batched", 1024), ("per_job", 1)):
            server = hm.Server(hbm_budget_bytes=64 << 30, nstreams=4, max_batch_jobs=max_jobs)
            jobs = server.jobs(m)
            for key, src in (("x", None), ("y", None), ("w", None)):
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
            done = server.run_schedule(jobs)
            server.close()
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
                         "mean_batch_jobs": round(float(np.mean(done["batch_jobs"][meas])), 2),
                         "status_ok": bool(np.all(done["status"] == 0))}
        row["p99_speedup"] = round(row["per_job"]["p99_us"] / row["batched"]["p99_us"], 2)
        row["p50_speedup"] = round(row["per_job"]["p50_us"] / row["batched"]["p50_us"], 2)
        res["rates"][str(rate)] = row
        print(f"serving {rate}/s done", file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (--gpus {args.gpus} requested); how the path "
              "would shard across GPUs is described, not measured", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1304_5553_amd as hm
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    x, y = workloads.plain_xy(n)
    k = workloads.plain_k(n)
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

    # results of the last step (sanity: exact integer results are printed)
    result = {}
    if "R1" in ops:
        result["R1_count"] = int(outs["count"].item())
    if "R2" in ops:
        result["R2_sum"] = int(outs["sum"].item())
    if "R3" in ops:
        result["R3_max"] = float(outs["max"].item())

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
        line["dot"] = bench_dot(torch, hm, workloads, dev, stream)
        print("dot done", file=sys.stderr, flush=True)
    if "precision" in ext:
        line["precision"] = bench_precision(torch, hm, workloads, dev, stream)
        print("precision done", file=sys.stderr, flush=True)
    if "batched" in ext:
        line["batched"] = bench_batched(torch, hm, workloads, dev)
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
        line["served"] = bench_serving(torch, hm, workloads, dev, duration_s=args.serving_duration,
                                       rates=rates)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(x, y, k, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
