"""Conjugate gradients on the five-point model problem.

Oracle (test infrastructure).  The paper names a conjugate-gradient Krylov
solver for large sparse linear systems among the facilities shipped beside
the elementwise and map-reduce kernels (section "Further Facilities").  The
oracle solves A x = b for the symmetric positive definite five-point
operator on an nx-by-ny grid with zero (Dirichlet) boundary values,

    (A p)[j, k] = 4 p[j, k] - p[j, k-1] - p[j, k+1] - p[j-1, k] - p[j+1, k]

(terms outside the grid are zero; unknown (j, k) is index j * nx + k), with
the conjugate-gradient iteration of Hestenes and Stiefel in float64:

    r = b - A x,  p = r
    repeat:  alpha = (r . r) / (p . A p)
             x = x + alpha p,  r' = r - alpha A p
             beta = (r' . r') / (r . r),  p = r' + beta p,  r = r'
"""

from __future__ import annotations

import numpy as np


def laplace5(p, nx: int) -> np.ndarray:
    """A p for the five-point operator on rows of nx unknowns (float64)."""
    p = np.asarray(p, dtype=np.float64)
    if p.size % nx:
        raise ValueError("the vector length must be a multiple of nx")
    g = p.reshape(-1, nx)
    q = 4.0 * g
    q[:, 1:] -= g[:, :-1]
    q[:, :-1] -= g[:, 1:]
    q[1:, :] -= g[:-1, :]
    q[:-1, :] -= g[1:, :]
    return q.ravel()


def cg(b, nx: int, iters: int, x0=None, keep_directions=False):
    """`iters` conjugate-gradient steps from x0 (zero by default).  Returns
    the iterate and the histories of r . r (entry k before step k, so
    iters + 1 values), alpha and beta, the search directions' A-products
    p_k . A p_k, and (with keep_directions) the directions themselves."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r = b - laplace5(x, nx)
    p = r.copy()
    rr = float(r @ r)
    hist = {"rr": [rr], "alpha": [], "beta": [], "pAp": [], "p": []}
    for _ in range(iters):
        q = laplace5(p, nx)
        pq = float(p @ q)
        alpha = rr / pq
        x += alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        beta = rr_new / rr
        if keep_directions:
            hist["p"].append(p.copy())
        p = r + beta * p
        rr = rr_new
        hist["rr"].append(rr)
        hist["alpha"].append(alpha)
        hist["beta"].append(beta)
        hist["pAp"].append(pq)
    return x, hist


__all__ = ["laplace5", "cg"]
