"""Conjugate gradients on the five-point model problem, built from run-time
generated elementwise and map-reduce kernels.

The paper lists a conjugate-gradient Krylov solver for large sparse systems
among the facilities shipped beside the elementwise and map-reduce kernels
(section "Further Facilities").  Here A is the symmetric positive definite
five-point operator on an nx-by-ny grid with zero boundary values (unknown
(j, k) at index j * nx + k), applied matrix-free by an elementwise kernel.
Every step of an iteration runs in the library's kernels; the scalars stay
in a small device array, so an iteration needs no host synchronisation and
can be captured into one HIP graph.  The array holds two (r . r, p . Ap)
pairs, c (this iteration's) and d (the next one's), which swap roles every
iteration, so no kernel has to copy r . r forward:

    q = A p                           elementwise (shifted reads p[i +/- 1], p[i +/- nx])
    c[1] = p . q                      map-reduce
    d[0] = sum (r - alpha q)^2        map-reduce (the next r . r), alpha = c[0] / c[1]
    x += alpha p;  r -= alpha q;  p = r + beta p      one fused elementwise,
                                                      beta = d[0] / c[0]

alpha and beta are the same float quotients the textbook iteration forms
once per step; each kernel reads the two scalars as fixed elements.

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
RR_NEXT = ("float: const float *r, const float *q, const float *c",
           "(r[i] - (c[0]/c[1])*q[i]) * (r[i] - (c[0]/c[1])*q[i])")
UPDATE = ("float *x, float *r, float *p, const float *q, const float *c, const float *d",
          "x[i] += (c[0]/c[1])*p[i]; r[i] -= (c[0]/c[1])*q[i]; p[i] = r[i] + (d[0]/c[0])*p[i]")
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
        self.s = torch.zeros(4, **f)          # two (r . r, p . Ap) pairs
        self.parity = 0                       # which pair holds this iteration's r . r
        self.k = {name: _hm.compile(expr, sig, name=f"cg_{name}") for name, (sig, expr) in
                  dict(spmv=SPMV, dot=DOT, rrn=RR_NEXT, update=UPDATE, start=START).items()}
        sp = stream.cuda_stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        self._ws = _hm.workspace(_hm.reduce_workspace_bytes(self.k["dot"], self.n), dev, sp)

    def _pairs(self):
        a, b = self.s[0:2], self.s[2:4]
        return (a, b) if self.parity == 0 else (b, a)

    @property
    def rr(self):
        """This iteration's r . r (a one-element device tensor)."""
        return self._pairs()[0][0:1]

    def start(self, b):
        """x = 0, r = p = b, r . r = b . b."""
        self.parity = 0
        _hm.elementwise(self.k["start"], self.n, [self.x, self.r, self.p, b], stream=self.stream)
        _hm.reduce(self.k["dot"], None, "a+b", "0", self.n, [b, b], self.s[0:1],
                   workspace_buf=self._ws, stream=self.stream)

    def step(self):
        """One CG iteration (four kernels, six launches, no host sync)."""
        c, d = self._pairs()
        n, st = self.n, self.stream
        _hm.elementwise(self.k["spmv"], n, [self.q, self.p, self.nx], stream=st)
        _hm.reduce(self.k["dot"], None, "a+b", "0", n, [self.p, self.q], c[1:2],
                   workspace_buf=self._ws, stream=st, config=CACHED)
        _hm.reduce(self.k["rrn"], None, "a+b", "0", n, [self.r, self.q, c], d[0:1],
                   workspace_buf=self._ws, stream=st, config=CACHED)
        _hm.elementwise(self.k["update"], n, [self.x, self.r, self.p, self.q, c, d], stream=st,
                        config=CACHED)
        self.parity ^= 1

    def capture(self, iters):
        """A HIP graph of `iters` iterations (an even count, so that every
        replay starts and ends with r . r in the first pair, as after start()).
        The kernels must have run once; the solver's stream must not be the
        null stream."""
        if self.stream is None:
            raise _hm.InvalidError("graph capture needs a non-default stream")
        if iters % 2:
            raise _hm.InvalidError("capture an even number of iterations")
        saved, self.parity = self.parity, 0
        g = _hm.Graph()
        try:
            with g.capture(self.stream):
                for _ in range(iters):
                    self.step()
        finally:
            self.parity = saved
        return g

    def solve(self, b, iters):
        self.start(b)
        for _ in range(iters):
            self.step()
        return self.x


__all__ = ["PoissonCG", "SPMV", "DOT", "RR_NEXT", "UPDATE", "START", "BYTES_PER_UNKNOWN", "CACHED"]
