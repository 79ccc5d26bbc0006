"""Pins of the oracle's indirect projection (CGLS, Section 3.5) and of the
solver run with it.

CGLS minimises ||x - c||^2 + ||A x - d||^2; its pins are the least-squares
solution by an independent library routine (finite termination in at most n
steps in exact arithmetic), the residual identities the recursion must keep,
the monotone decrease of the quadratic along the CG iterates, and optima of
whole solves against the direct projection and against non-ADMM solvers.
"""
import numpy as np
import pytest
from scipy import optimize

from oracle import pogs_oracle as O
from paper_1503_08366_amd import workloads as W


def _data(m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(m, n)) / np.sqrt(n), rng.normal(size=n), rng.normal(size=m)


@pytest.mark.parametrize("m,n", [(12, 5), (5, 12), (9, 9)])
def test_cgls_terminates_at_least_squares_solution(m, n):
    """With no tolerance and n steps, CGLS returns the projection: the
    least-squares solution of [A; I] x = [d; c] (numpy lstsq, an SVD)."""
    A, c, d = _data(m, n, m * 7 + n)
    x_ls = np.linalg.lstsq(np.vstack([A, np.eye(n)]), np.concatenate([d, c]), rcond=None)[0]
    x, r1, steps = O.cgls_project(A, c, d, np.zeros(n), 0.0, n)
    assert steps == n
    np.testing.assert_allclose(x, x_ls, rtol=0, atol=1e-10)
    np.testing.assert_allclose(r1, d - A @ x_ls, rtol=0, atol=1e-10)


def test_cgls_recursion_keeps_residual_identities():
    """After any number of steps, r1 = d - A x and the quadratic decreases
    monotonically along the iterates; the start point matters only through
    the first residual."""
    A, c, d = _data(40, 25, 3)
    x0 = np.random.default_rng(4).normal(size=25)
    for cap in (0, 1, 3, 7):
        x, r1, steps, xs = O.cgls_project(A, c, d, x0, 0.0, cap, trace=True)
        assert steps == cap
        np.testing.assert_allclose(r1, d - A @ x, rtol=0, atol=1e-12)
        q = [0.5 * np.sum((z - c) ** 2) + 0.5 * np.sum((A @ z - d) ** 2) for z in xs]
        assert all(q[i + 1] <= q[i] + 1e-12 for i in range(len(q) - 1))
        np.testing.assert_array_equal(xs[0], x0)


def test_cgls_tolerance_stops_on_normal_residual():
    A, c, d = _data(60, 20, 5)
    thr = 1e-3
    x, r1, steps = O.cgls_project(A, c, d, np.zeros(20), thr, 100)
    s = A.T @ (d - A @ x) + (c - x)
    assert np.linalg.norm(s) <= thr * (1 + 1e-9)
    # one step fewer would not have met it
    x1, _, _ = O.cgls_project(A, c, d, np.zeros(20), 0.0, steps - 1)
    assert np.linalg.norm(A.T @ (d - A @ x1) + (c - x1)) > thr


def test_cgls_state_is_dual_invariant_up_to_normal_residual():
    """With the CGLS projection, x~ + A^T y~ equals the final normal residual s
    of that projection (zero for the exact projection, Section 3.3), so it stays
    below cg_tol * eps_dual / rho whenever CGLS met its tolerance."""
    p = W.lasso(120, 40, 6, dtype=np.float64)
    prm = O.Params(projection="cgls", cg_max_iter=200)
    r = O.solve(p.A, p.f, p.g, prm, record=True)
    h = r.history
    assert r.converged and max(h["cg"]) < 200
    for inv, eps_dual, rho in zip(h["inv_dual"], h["eps_dual"], h["rho"]):
        # rho recorded before any change made after this iteration
        assert inv <= prm.cg_tol * eps_dual / rho * (1 + 1e-9) + 1e-15
    assert max(h["inv_primal"]) < 1e-10  # y = d - r1 = A^ x up to rounding


@pytest.mark.parametrize("make", [
    lambda: W.lasso(300, 80, 7, dtype=np.float64),
    lambda: W.lasso(60, 150, 8, dtype=np.float64),
    lambda: W.logistic(200, 40, 9, dtype=np.float64),
    lambda: W.lp(60, 25, 10, dtype=np.float64),
    lambda: W.huber_fit(150, 20, 11, dtype=np.float64),
])
def test_cgls_solve_matches_direct_solve(make):
    p = make()
    tight = dict(eps_abs=1e-7, eps_rel=1e-7, max_iter=100000)
    rd = O.solve(p.A, p.f, p.g, O.Params(**tight))
    rc = O.solve(p.A, p.f, p.g, O.Params(projection="cgls", **tight))
    assert rd.converged and rc.converged
    assert abs(rc.optval - rd.optval) <= 1e-5 * max(1.0, abs(rd.optval)), (rc.optval, rd.optval)
    assert rc.cg_steps >= rc.iters  # at least one step per projection at this tolerance


def test_cgls_nnls_matches_scipy_nnls():
    p = W.nnls_from(W.lasso(100, 30, 12, dtype=np.float64))
    x_ref, _ = optimize.nnls(p.A, p.meta["b"])
    ref = 0.5 * np.sum((p.A @ x_ref - p.meta["b"]) ** 2)
    r = O.solve(p.A, p.f, p.g, O.Params(projection="cgls", eps_abs=1e-7, eps_rel=1e-7, max_iter=100000))
    assert r.converged
    assert abs(r.optval - ref) <= 1e-5 * ref
    np.testing.assert_allclose(r.x, x_ref, atol=1e-4)


def test_cgls_default_tolerance_close_to_direct():
    """At the default tolerances (eps_abs 1e-4, eps_rel 1e-3) the CGLS run
    stops within a few iterations of the direct one and at an objective within
    1e-3 relative."""
    p = W.lasso(400, 100, 13, dtype=np.float64)
    rd = O.solve(p.A, p.f, p.g)
    rc = O.solve(p.A, p.f, p.g, O.Params(projection="cgls"))
    assert rc.converged
    assert abs(rc.iters - rd.iters) <= max(3, rd.iters // 10)
    assert abs(rc.optval - rd.optval) <= 1e-3 * max(1.0, abs(rd.optval))
