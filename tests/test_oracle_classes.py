"""Pins of the oracle's solver on the problem classes of Appendix A that use
per-element base functions and the entropy, Huber and quadratic terms
(basis pursuit A.1, entropy maximization A.2, Huber fitting A.3, portfolio
optimization A.8).  Each optimum is found here without ADMM: a closed form,
an LP solver, the smooth dual of the entropy problem, a robust least-squares
solver, or enumeration of the active sets of a small QP.

Tolerance: the oracle runs to eps_abs = eps_rel = 1e-7 (Section 3.4), so the
objective is within about 1e-5 relative of the optimum.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import pogs_oracle as O
from paper_1503_08366_amd import workloads as W

TIGHT = O.Params(eps_abs=1e-7, eps_rel=1e-7, max_iter=100000)


def _solve(p):
    r = O.solve(p.A.astype(np.float64), p.f, p.g, TIGHT)
    assert r.converged, (p.name, r.iters)
    return r


def test_basis_pursuit_tall_recovers_v():
    """m > n (the appendix's shapes): A x = b has the single solution v."""
    p = W.basis_pursuit(60, 25, 1, dtype=np.float64)
    r = _solve(p)
    v = p.meta["v"]
    np.testing.assert_allclose(r.x, v, atol=1e-5)
    assert abs(r.optval - np.abs(v).sum()) <= 1e-5 * np.abs(v).sum()


def test_basis_pursuit_wide_matches_linprog():
    """m < n: min ||x||_1 s.t. A x = b as an LP in (u, w) >= 0, x = u - w."""
    p = W.basis_pursuit(20, 50, 2, dtype=np.float64)
    m, n = p.A.shape
    res = optimize.linprog(np.ones(2 * n), A_eq=np.hstack([p.A, -p.A]), b_eq=p.meta["b"],
                           bounds=[(0, None)] * (2 * n), method="highs")
    assert res.status == 0
    r = _solve(p)
    assert abs(r.optval - res.fun) <= 1e-5 * res.fun, (r.optval, res.fun)
    assert np.linalg.norm(p.A @ r.x - p.meta["b"]) <= 1e-4 * np.linalg.norm(p.meta["b"])


def test_entropy_max_matches_smooth_dual():
    """Dual of min sum x log x s.t. F x <= b, 1^T x = 1: for lam >= 0 the
    minimizing x is softmax(-F^T lam) and the dual function is
    -log sum exp(-F^T lam) - b^T lam; its maximum (L-BFGS-B with lam >= 0)
    equals the primal optimum (Slater holds: v / 1^T v is feasible and
    strictly positive)."""
    p = W.entropy_max(6, 30, 3, dtype=np.float64)
    m = p.A.shape[0] - 1
    F, b = p.A[:m], p.meta["b"]

    def negdual(lam):
        z = -F.T @ lam
        zmax = z.max()
        w = np.exp(z - zmax)
        lse = zmax + math.log(w.sum())
        x = w / w.sum()
        return lse + b @ lam, -F @ x + b

    res = optimize.minimize(negdual, np.zeros(m), jac=True, method="L-BFGS-B",
                            bounds=[(0, None)] * m, options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 10000})
    dual_opt = -res.fun
    z = -F.T @ res.x
    x_star = np.exp(z - z.max())
    x_star /= x_star.sum()
    r = _solve(p)
    assert abs(r.optval - dual_opt) <= 1e-5 * max(1.0, abs(dual_opt)), (r.optval, dual_opt)
    np.testing.assert_allclose(r.x, x_star, atol=1e-4)
    assert abs(r.x.sum() - 1.0) <= 1e-5
    assert np.all(F @ r.x - b <= 1e-4 * np.abs(b).max())


def test_huber_fit_matches_robust_least_squares():
    """scipy's least_squares with loss='huber', f_scale=1 minimizes
    sum 0.5 rho(r_i^2) with rho(z) = z (z <= 1), 2 sqrt(z) - 1 (z > 1), which is
    sum huber(r_i)."""
    p = W.huber_fit(150, 20, 4, dtype=np.float64)
    b = p.meta["b"]
    res = optimize.least_squares(lambda x: b - p.A @ x, np.zeros(p.n), loss="huber", f_scale=1.0,
                                 xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=10000)
    rr = b - p.A @ res.x
    ref = float(np.sum(np.where(np.abs(rr) <= 1, 0.5 * rr * rr, np.abs(rr) - 0.5)))
    r = _solve(p)
    assert abs(r.optval - ref) <= 1e-5 * ref, (r.optval, ref)
    # some residuals beyond the quadratic zone: the outliers exercise the linear branch
    assert np.any(np.abs(b - p.A @ r.x) > 1.5)


def _portfolio_brute_force(F, Dg, mu, gamma):
    """Enumerate supports S of min -mu^T x + gamma x^T Q x, x >= 0, 1^T x = 1
    (Q = F F^T + diag(D)): on S solve the KKT equalities, keep the one whose
    x_S >= 0 and whose multipliers off S are >= 0."""
    n = F.shape[0]
    Q = F @ F.T + np.diag(Dg)
    best = None
    for size in range(1, n + 1):
        for S in itertools.combinations(range(n), size):
            S = list(S)
            K = np.zeros((size + 1, size + 1))
            K[:size, :size] = 2 * gamma * Q[np.ix_(S, S)]
            K[:size, size] = 1.0
            K[size, :size] = 1.0
            rhs = np.append(mu[S], 1.0)
            sol = np.linalg.solve(K, rhs)
            xs, nu = sol[:size], sol[size]
            if np.any(xs < -1e-12):
                continue
            x = np.zeros(n)
            x[S] = xs
            lam = 2 * gamma * Q @ x - mu + nu
            if np.all(lam >= -1e-9):
                val = -mu @ x + gamma * x @ Q @ x
                if best is None or val < best[0]:
                    best = (val, x)
    return best


def test_portfolio_matches_active_set_enumeration():
    p = W.portfolio(3, 10, 5, dtype=np.float64)
    val, x_star = _portfolio_brute_force(p.meta["F"], p.meta["D"], p.meta["mu"], p.meta["gamma"])
    r = _solve(p)
    assert abs(r.optval - val) <= 1e-5 * max(1.0, abs(val)), (r.optval, val)
    np.testing.assert_allclose(r.x, x_star, atol=1e-4)


def test_per_element_functions_split_by_group():
    """A per-element h evaluates, proxes and conjugates each element with its
    own base function: the same as the single-h functions on each part."""
    rng = np.random.default_rng(7)
    names = ["square", "ind_eq0", "abs", "neg_entr", "huber", "ind_le0"]
    n = 60
    h = [names[i % len(names)] for i in range(n)]
    a = rng.uniform(0.5, 2, n)
    b = rng.normal(0, 1, n)
    c = rng.uniform(0.5, 2, n)
    d = rng.normal(0, 1, n)
    F = W.Fn(h, n, a=a, b=b, c=c, d=d)
    v = rng.normal(0, 2, n)
    got = O.prox_param(F, v, 1.7)
    for name in names:
        idx = [i for i in range(n) if h[i] == name]
        Fi = W.Fn(name, len(idx), a=a[idx], b=b[idx], c=c[idx], d=d[idx])
        np.testing.assert_array_equal(got[idx], O.prox_param(Fi, v[idx], 1.7))
    y = got
    tot = sum(O.fn_eval(W.Fn(nm, len(ix), a=a[ix], b=b[ix], c=c[ix], d=d[ix]), y[ix], 1e-9)
              for nm in names for ix in [[i for i in range(n) if h[i] == nm]])
    assert O.fn_eval(F, y, 1e-9) == pytest.approx(tot, rel=1e-14)
    with pytest.raises(ValueError):
        W.Fn(h[:-1], n)
