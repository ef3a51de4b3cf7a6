"""The CG solver's generated-kernel statements, run by the oracle on the CPU
(no GPU): one iteration as the solver issues it (A p, p . A p, the next
r . r with alpha folded in, the fused update with alpha and beta folded in,
the scalar pairs swapping roles), with every vector and scalar stored as
float32 between kernels as on the device, tracks the textbook float64
iteration (section "Further Facilities": a CG solver for sparse systems)."""

import numpy as np

import oracle
from paper_1304_5553_amd import cg as hcg


def f32(v):
    return np.asarray(v, np.float64).astype(np.float32)


def test_solver_statements_are_textbook_cg():
    nx, ny = 11, 9
    n = nx * ny
    b = np.random.default_rng(4).uniform(-1, 1, n).astype(np.float32)
    z = np.zeros(n, np.float32)
    st = oracle.elementwise(hcg.START[0], hcg.START[1], n, [z, z.copy(), z.copy(), b])
    x, r, p = f32(st["x"].v), f32(st["r"].v), f32(st["p"].v)
    s = np.zeros(4, np.float32)
    s[0] = oracle.reduce(hcg.DOT[0], hcg.DOT[1], "a+b", "0", n, [b, b]).value
    parity = 0
    iters = 12
    for _ in range(iters):
        ci, di = (0, 2) if parity == 0 else (2, 0)
        q = f32(oracle.elementwise(hcg.SPMV[0], hcg.SPMV[1], n, [z, p, np.int32(nx)])["q"].v)
        s[ci + 1] = oracle.reduce(hcg.DOT[0], hcg.DOT[1], "a+b", "0", n, [p, q]).value
        c = s[ci:ci + 2].copy()
        s[di] = oracle.reduce(hcg.RR_NEXT[0], hcg.RR_NEXT[1], "a+b", "0", n, [r, q, c]).value
        d = s[di:di + 2].copy()
        up = oracle.elementwise(hcg.UPDATE[0], hcg.UPDATE[1], n, [x, r, p, q, c, d])
        x, r, p = f32(up["x"].v), f32(up["r"].v), f32(up["p"].v)
        parity ^= 1
    want, hist = oracle.cg(b.astype(np.float64), nx, iters)
    assert np.linalg.norm(x - want) <= 1e-4 * np.linalg.norm(want)
    rr = s[0] if parity == 0 else s[2]
    assert abs(rr - hist["rr"][-1]) <= 1e-3 * hist["rr"][0]
    # and the statements move the bytes the solver's accounting says
    assert hcg.BYTES_PER_UNKNOWN == 8 + 8 + 8 + 28
