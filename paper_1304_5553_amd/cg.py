"""Conjugate gradients on the five-point model problem, built from run-time
generated elementwise and map-reduce kernels.

The paper lists a conjugate-gradient Krylov solver for large sparse systems
among the facilities shipped beside the elementwise and map-reduce kernels
(section "Further Facilities").  Here A is the symmetric positive definite
five-point operator on an nx-by-ny grid with zero boundary values (unknown
(j, k) at index j * nx + k), applied matrix-free by an elementwise kernel.
Every step of an iteration runs in the library's kernels; the scalars
(r . r, p . Ap, alpha, beta) stay in a small device array, so an iteration
needs no host synchronisation and can be captured into one HIP graph:

    q = A p                                  elementwise (shifted reads p[i +/- 1], p[i +/- nx])
    s[1] = p . q                             map-reduce
    s[2] = s[0] / s[1]            (alpha)    elementwise over one element
    s[3] = sum (r - alpha q)^2               map-reduce (the next r . r)
    s[4] = s[3] / s[0], s[0] = s[3] (beta)   elementwise over one element
    x += alpha p;  r -= alpha q;  p = r + beta p       one fused elementwise

Per unknown and iteration the kernels move 52 bytes: A p reads p and writes
q (8), the two reductions read two vectors each (16), the update reads x, r,
p, q and writes x, r, p (28).
"""

from __future__ import annotations

from . import hipmr as _hm

SPMV = ("float *q, const float *p, int nx",
        "int c = i % nx; "
        "q[i] = 4.0f*p[i] - (c != 0 ? p[i-1] : 0.0f) - (c != nx - 1 ? p[i+1] : 0.0f)"
        " - (i >= nx ? p[i-nx] : 0.0f) - (i + nx < n ? p[i+nx] : 0.0f)")
DOT = ("float: const float *p, const float *q", "p[i]*q[i]")
ALPHA = ("float *alpha, const float *rr, const float *pq", "alpha[i] = rr[i] / pq[i]")
RR_NEXT = ("float: const float *r, const float *q, const float *s",
           "(r[i] - s[2]*q[i]) * (r[i] - s[2]*q[i])")
BETA = ("float *beta, float *rr, const float *rrn", "beta[i] = rrn[i] / rr[i]; rr[i] = rrn[i]")
UPDATE = ("float *x, float *r, float *p, const float *q, const float *s",
          "x[i] += s[2]*p[i]; r[i] -= s[2]*q[i]; p[i] = r[i] + s[4]*p[i]")
START = ("float *x, float *r, float *p, const float *b", "x[i] = 0.0f; r[i] = b[i]; p[i] = b[i]")

BYTES_PER_UNKNOWN = 52

# The solver rereads its vectors every iteration (x, r, p, q: 256 MB at a
# 4096 x 4096 grid, the size of MI355X's last-level cache).  The reductions
# and the update therefore use temporal loads and stores, which keep the
# vectors cached for the next kernel; the streaming (non-temporal) default
# suits single passes over data larger than the cache.  Measured at 4096^2:
# 136 us per iteration against 165 us with streaming accesses throughout.
CACHED = _hm.LaunchConfig(flags=_hm.CFG_TEMPORAL)


class PoissonCG:
    """Device state and kernels of CG for one grid size.  All calls are
    asynchronous on `stream` (default: torch's current stream)."""

    def __init__(self, nx, ny, device=None, stream=None):
        import torch
        self.nx, self.ny, self.n = int(nx), int(ny), int(nx) * int(ny)
        dev = device or torch.device("cuda")
        self.stream = stream
        f = dict(dtype=torch.float32, device=dev)
        self.x, self.r, self.p, self.q = (torch.empty(self.n, **f) for _ in range(4))
        self.s = torch.zeros(8, **f)          # rr, pq, alpha, rr_next, beta
        self.k = {name: _hm.compile(expr, sig, name=f"cg_{name}") for name, (sig, expr) in
                  dict(spmv=SPMV, dot=DOT, alpha=ALPHA, rrn=RR_NEXT, beta=BETA, update=UPDATE,
                       start=START).items()}
        sp = stream.cuda_stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        self._ws = _hm.workspace(_hm.reduce_workspace_bytes(self.k["dot"], self.n), dev, sp)

    def start(self, b):
        """x = 0, r = p = b, s[0] = b . b."""
        _hm.elementwise(self.k["start"], self.n, [self.x, self.r, self.p, b], stream=self.stream)
        _hm.reduce(self.k["dot"], None, "a+b", "0", self.n, [b, b], self.s[0:1],
                   workspace_buf=self._ws, stream=self.stream)

    def step(self):
        """One CG iteration (six kernels, nine launches, no host sync)."""
        s, n, st = self.s, self.n, self.stream
        _hm.elementwise(self.k["spmv"], n, [self.q, self.p, self.nx], stream=st)
        _hm.reduce(self.k["dot"], None, "a+b", "0", n, [self.p, self.q], s[1:2],
                   workspace_buf=self._ws, stream=st, config=CACHED)
        _hm.elementwise(self.k["alpha"], 1, [s[2:3], s[0:1], s[1:2]], stream=st)
        _hm.reduce(self.k["rrn"], None, "a+b", "0", n, [self.r, self.q, s], s[3:4],
                   workspace_buf=self._ws, stream=st, config=CACHED)
        _hm.elementwise(self.k["beta"], 1, [s[4:5], s[0:1], s[3:4]], stream=st)
        _hm.elementwise(self.k["update"], n, [self.x, self.r, self.p, self.q, s], stream=st,
                        config=CACHED)

    def capture(self, iters):
        """A HIP graph of `iters` iterations (the kernels must have run once;
        the solver's stream must not be the null stream)."""
        if self.stream is None:
            raise _hm.InvalidError("graph capture needs a non-default stream")
        g = _hm.Graph()
        with g.capture(self.stream):
            for _ in range(iters):
                self.step()
        return g

    def solve(self, b, iters):
        self.start(b)
        for _ in range(iters):
            self.step()
        return self.x


__all__ = ["PoissonCG", "SPMV", "DOT", "ALPHA", "RR_NEXT", "BETA", "UPDATE", "START",
           "BYTES_PER_UNKNOWN", "CACHED"]
