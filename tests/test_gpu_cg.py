"""GPU parity of conjugate gradients on the five-point model problem (section
"Further Facilities": a CG Krylov solver), built from run-time generated
kernels: every kernel of the iteration against the oracle, the GPU solver
against the oracle's float64 CG, and graph replay against eager execution."""

import numpy as np
import pytest

from gpu_util import assert_lanes, assert_reduce, dev_array, host_bits, need_gpu, reduce_on_gpu, torch
import oracle
import paper_1304_5553_amd as hm
from paper_1304_5553_amd import cg as hcg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.mark.parametrize("nx,ny", [(37, 23), (1, 50), (64, 1), (130, 129)])
def test_stencil_kernel(dev, nx, ny):
    n = nx * ny
    rng = np.random.default_rng(nx + ny)
    p = rng.uniform(-1, 1, n).astype(np.float32)
    k = hm.compile(hcg.SPMV[1], hcg.SPMV[0], name="cg_spmv_t")
    q = torch.full((n + 4,), float("nan"), device=dev)
    hm.elementwise(k, n, [q[:n], dev_array(p), nx])
    torch.cuda.synchronize()
    ref = oracle.elementwise(hcg.SPMV[0], hcg.SPMV[1], n, [np.zeros(n, np.float32), p, np.int32(nx)])
    assert_lanes(q[:n], ref["q"], "float32", what=f"A p on {nx}x{ny}")
    assert np.all(np.isnan(host_bits(q[n:])))
    # and the oracle's statement equals the five-point operator
    assert np.allclose(ref["q"].v, oracle.laplace5(p, nx), rtol=0, atol=1e-12)


def test_update_and_scalar_kernels(dev):
    n = 40009
    rng = np.random.default_rng(3)
    x, r, p, q = (rng.uniform(-1, 1, n).astype(np.float32) for _ in range(4))
    c = np.array([2.0, 3.0], np.float32)          # this iteration's (r . r, p . Ap)
    d = np.array([0.5, 7.0], np.float32)          # the next r . r (d[1] unused)
    xd, rd, pd, qd, cd, dd = (dev_array(a) for a in (x, r, p, q, c, d))
    k = hm.compile(hcg.UPDATE[1], hcg.UPDATE[0], name="cg_update_t")
    assert k.vectorizable                          # c[0], c[1], d[0] are fixed elements
    hm.elementwise(k, n, [xd, rd, pd, qd, cd, dd])
    torch.cuda.synchronize()
    ref = oracle.elementwise(hcg.UPDATE[0], hcg.UPDATE[1], n, [x, r, p, q, c, d])
    for name, t in (("x", xd), ("r", rd), ("p", pd)):
        assert_lanes(t, ref[name], "float32", what=f"update {name}")
    rn = hm.compile(hcg.RR_NEXT[1], hcg.RR_NEXT[0], name="cg_rrn_t")
    out = reduce_on_gpu(rn, "a+b", "0", n, [dev_array(r), dev_array(q), cd])
    assert_reduce(out, oracle.reduce(hcg.RR_NEXT[0], hcg.RR_NEXT[1], "a+b", "0", n, [r, q, c]), "rr next")


def make_problem(nx, ny, seed):
    rng = np.random.default_rng(seed)
    x_true = rng.uniform(-1, 1, nx * ny)
    b = oracle.laplace5(x_true, nx).astype(np.float32)
    return x_true, b


def test_cg_converges_and_tracks_the_oracle(dev):
    nx, ny = 48, 40
    x_true, b = make_problem(nx, ny, 5)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        solver = hcg.PoissonCG(nx, ny, device=dev, stream=stream)
        bd = dev_array(b)
        solver.start(bd)
        rr_gpu = [host_bits(solver.rr)[0]]
        for _ in range(12):
            solver.step()
            stream.synchronize()
            rr_gpu.append(host_bits(solver.rr)[0])
        _, hist = oracle.cg(b.astype(np.float64), nx, 12)
        rel = np.abs(np.array(rr_gpu, np.float64) / np.array(hist["rr"]) - 1)
        assert rel.max() < 1e-3, rel
        for _ in range(288):
            solver.step()
        stream.synchronize()
        x = host_bits(solver.x).astype(np.float64)
    err = np.linalg.norm(x - x_true) / np.linalg.norm(x_true)
    assert err < 1e-4, err


def test_graph_replay_equals_eager(dev):
    nx, ny = 256, 192
    _, b = make_problem(nx, ny, 6)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        solver = hcg.PoissonCG(nx, ny, device=dev, stream=stream)
        bd = dev_array(b)
        solver.solve(bd, 20)
        stream.synchronize()
        x_eager, s_eager = solver.x.clone(), solver.s.clone()
        with pytest.raises(hm.InvalidError):
            solver.capture(3)                     # replays must end where they start
        graph = solver.capture(10)
        for rep in range(3):                      # replays after unrelated eager work
            solver.start(bd)
            graph.launch(stream)
            graph.launch(stream)
            stream.synchronize()
            assert torch.equal(solver.x, x_eager) and torch.equal(solver.s, s_eager), rep
            _ = (bd * 2).sum().item()


@pytest.mark.parametrize("nx,ny,iters", [(1024, 768, 40), (4096, 4096, 30)])
def test_cg_at_scale_tracks_the_oracle(dev, nx, ny, iters):
    # the 4096 x 4096 grid is the size the benchmark times
    _, b = make_problem(nx, ny, 7)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        solver = hcg.PoissonCG(nx, ny, device=dev, stream=stream)
        solver.solve(dev_array(b), iters)
        stream.synchronize()
        rr = float(host_bits(solver.rr)[0])
    _, hist = oracle.cg(b.astype(np.float64), nx, iters)
    assert abs(rr / hist["rr"][-1] - 1) < 1e-2, (rr, hist["rr"][-1])
