"""Brute-force reference optima for tiny problems (test infrastructure only).

These pin the oracle's ADMM (Algorithm 1) from outside: each finds the exact
optimum of a small problem by enumeration, with no splitting, no proximal
operator and no projection, so an error in the oracle cannot repeat here.

  * lp_vertices    - box-bounded LP, min c^T x s.t. A x <= b, 0 <= x <= 1, by
                     enumerating every vertex (n active constraints).
  * nnls_supports  - min 1/2||A x - b||^2 s.t. x >= 0 over all 2^n supports.
  * lasso_signs    - min 1/2||A x - b||^2 + lam ||x||_1 over all 3^n sign
                     patterns.
  * scalar_min     - argmin of a 1-D convex function by grid search followed
                     by golden-section refinement.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def lp_vertices(A, b, c, tol: float = 1e-9):
    """Optimal value and point of min c^T x s.t. A x <= b, 0 <= x <= 1.

    The feasible set is a polytope (bounded by the box), so the optimum is
    attained at a vertex: a feasible point where n linearly independent
    constraints are active.  Every n-subset of the m + 2n constraints is tried.
    Returns (value, x) or (inf, None) if infeasible.
    """
    A = np.asarray(A, float)
    m, n = A.shape
    G = np.vstack([A, -np.eye(n), np.eye(n)])
    h = np.concatenate([np.asarray(b, float), np.zeros(n), np.ones(n)])
    best, best_x = math.inf, None
    for rows in itertools.combinations(range(m + 2 * n), n):
        M = G[list(rows)]
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        x = np.linalg.solve(M, h[list(rows)])
        if np.all(G @ x <= h + tol):
            v = float(np.dot(c, x))
            if v < best:
                best, best_x = v, x
    return best, best_x


def nnls_supports(A, b):
    """min 1/2 ||A x - b||^2 s.t. x >= 0 by trying every support set.

    For the optimal support S, x_S is the unconstrained least-squares solution
    on the columns S and is non-negative; the best objective among supports
    whose least-squares solution is non-negative is the optimum.
    """
    A = np.asarray(A, float)
    b = np.asarray(b, float)
    m, n = A.shape
    best, best_x = 0.5 * float(b @ b), np.zeros(n)
    for k in range(1, n + 1):
        for S in itertools.combinations(range(n), k):
            S = list(S)
            xs, *_ = np.linalg.lstsq(A[:, S], b, rcond=None)
            if np.all(xs >= -1e-12):
                x = np.zeros(n)
                x[S] = np.maximum(xs, 0.0)
                v = 0.5 * float(np.sum((A @ x - b) ** 2))
                if v < best:
                    best, best_x = v, x
    return best, best_x


def lasso_signs(A, b, lam):
    """min 1/2 ||A x - b||^2 + lam ||x||_1 by trying every sign pattern.

    For a fixed sign vector s (entries -1, 0, +1) the objective restricted to
    {x : sign(x) = s} is the quadratic 1/2||A_S x_S - b||^2 + lam s_S^T x_S,
    minimised by A_S^T A_S x_S = A_S^T b - lam s_S.  A candidate whose signs
    match s is feasible; the best candidate is the global optimum.
    """
    A = np.asarray(A, float)
    b = np.asarray(b, float)
    m, n = A.shape
    best, best_x = 0.5 * float(b @ b), np.zeros(n)
    for s in itertools.product((-1.0, 0.0, 1.0), repeat=n):
        s = np.array(s)
        S = np.flatnonzero(s)
        if S.size == 0:
            continue
        AS = A[:, S]
        M = AS.T @ AS
        if np.linalg.matrix_rank(M) < S.size:
            continue
        xs = np.linalg.solve(M, AS.T @ b - lam * s[S])
        if np.all(np.sign(xs) == s[S]):
            x = np.zeros(n)
            x[S] = xs
            v = 0.5 * float(np.sum((A @ x - b) ** 2)) + lam * float(np.sum(np.abs(x)))
            if v < best:
                best, best_x = v, x
    return best, best_x


def scalar_min(phi, lo: float, hi: float, grid: int = 4001, iters: int = 200) -> float:
    """argmin of a convex scalar function on [lo, hi]: dense grid, then
    golden-section search on the bracket around the best grid point."""
    ts = np.linspace(lo, hi, grid)
    vals = np.array([phi(t) for t in ts])
    i = int(np.argmin(vals))
    a = ts[max(i - 1, 0)]
    bnd = ts[min(i + 1, grid - 1)]
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    c = bnd - gr * (bnd - a)
    d = a + gr * (bnd - a)
    fc, fd = phi(c), phi(d)
    for _ in range(iters):
        if fc <= fd:
            bnd, d, fd = d, c, fc
            c = bnd - gr * (bnd - a)
            fc = phi(c)
        else:
            a, c, fc = c, d, fd
            d = a + gr * (bnd - a)
            fd = phi(d)
        if bnd - a < 1e-13 * max(1.0, abs(a)):
            break
    return 0.5 * (a + bnd)
