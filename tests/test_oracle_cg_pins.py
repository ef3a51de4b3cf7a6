"""Pins of the oracle's conjugate-gradient solver on the five-point model
problem (section "Further Facilities": a CG Krylov solver for sparse
systems).  The operator is pinned to SciPy's sparse matrix built from
Kronecker products of the 1-D second difference; the solver to SciPy's
direct sparse solve, to the invariants of exact CG (orthogonal residuals,
A-conjugate directions), and to its finite termination on a problem with
few distinct eigenvalues."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle


def laplace_matrix(nx, ny):
    tx = sp.diags([-np.ones(nx - 1), 2 * np.ones(nx), -np.ones(nx - 1)], [-1, 0, 1])
    ty = sp.diags([-np.ones(ny - 1), 2 * np.ones(ny), -np.ones(ny - 1)], [-1, 0, 1])
    return (sp.kron(sp.identity(ny), tx) + sp.kron(ty, sp.identity(nx))).tocsr()


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 9), (8, 1), (7, 5), (33, 20)])
def test_operator_is_scipys_sparse_laplacian(nx, ny):
    rng = np.random.default_rng(nx * 100 + ny)
    p = rng.standard_normal(nx * ny)
    assert np.allclose(oracle.laplace5(p, nx), laplace_matrix(nx, ny) @ p, rtol=0, atol=1e-13)


def test_cg_reaches_the_direct_solution():
    nx, ny = 24, 17
    rng = np.random.default_rng(1)
    b = rng.uniform(-1, 1, nx * ny)
    x, hist = oracle.cg(b, nx, 200)
    want = spla.spsolve(laplace_matrix(nx, ny).tocsc(), b)
    assert np.linalg.norm(x - want) <= 1e-10 * np.linalg.norm(want)
    assert hist["rr"][-1] <= 1e-24 * hist["rr"][0]


def test_cg_invariants_orthogonal_residuals_conjugate_directions():
    nx, ny = 16, 12
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 1, nx * ny)
    A = laplace_matrix(nx, ny)
    _, hist = oracle.cg(b, nx, 12, keep_directions=True)
    P = np.array(hist["p"])                      # directions p_0 .. p_11
    G = P @ (A @ P.T)                            # p_j . A p_k
    d = np.sqrt(np.outer(np.diag(G), np.diag(G)))
    off = np.abs(G / d - np.eye(len(P)))
    assert off.max() < 1e-9
    assert np.allclose(np.diag(G), hist["pAp"], rtol=1e-12)
    # beta_k = |r_{k+1}|^2 / |r_k|^2
    rr = np.array(hist["rr"])
    assert np.allclose(hist["beta"], rr[1:] / rr[:-1], rtol=1e-14)


def test_cg_terminates_in_as_many_steps_as_distinct_eigenvalues():
    # a one-row grid of 3 unknowns: A = tridiag(-1, 4, -1) has 3 distinct
    # eigenvalues, so exact CG ends after 3 steps
    b = np.array([1.0, -2.0, 0.5])
    x, hist = oracle.cg(b, 3, 3)
    A = laplace_matrix(3, 1).toarray()                   # 4 I - neighbours on a one-row grid
    assert np.allclose(A @ x, b, rtol=0, atol=1e-14)
    assert hist["rr"][-1] < 1e-28


def test_zero_right_hand_side_is_a_fixed_point():
    x, hist = oracle.cg(np.zeros(20), 5, 0)
    assert np.all(x == 0) and hist["rr"] == [0.0]
