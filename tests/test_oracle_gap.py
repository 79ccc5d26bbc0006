"""Pins of the gap-based stopping rule (Section 3.4) and of the conjugates of
parametric terms with e > 0 it needs.

The gap eta = f(y) + g(x) + f*(nu) + g*(mu) of a primal and dual feasible
tuple bounds its suboptimality (Section 2.1): f(y) + g(x) - p* <= eta.  The
pins check that bound against optima found without ADMM, check the Fenchel-
Young equality the conjugates must meet at prox outputs, and check that the
gap stays infinite when a constraint is violated (the paper's caveat).
"""
import numpy as np
import pytest

from oracle import pogs_oracle as O
from paper_1503_08366_amd import workloads as W

H_FULL = ["zero", "identity", "abs", "square", "huber", "hinge", "logistic", "ind_ge0", "ind_le0",
          "ind_eq0", "ind_box01", "exp", "neg_entr", "neg_log", "recipr", "max_neg0"]


@pytest.mark.parametrize("h", H_FULL)
def test_conjugate_with_quadratic_term_meets_fenchel_young(h):
    """e > 0: for y = prox_{f,rho}(v), nu = rho (v - y) is a subgradient of f at
    y, so f(y) + f*(nu) = nu y (equality case of Fenchel-Young)."""
    rng = np.random.default_rng(len(h) * 7 + 3)
    N = 40
    a = rng.choice([-1.0, 1.0], N) * rng.uniform(0.5, 2.0, N)
    b = rng.normal(0, 1, N)
    c = rng.uniform(0.2, 2.0, N)
    d = rng.normal(0, 1, N)
    e = rng.uniform(0.1, 2.0, N)
    F = W.Fn(h, N, a=a, b=b, c=c, d=d, e=e)
    v = rng.normal(0, 2, N)
    rho = 1.3
    y = O.prox_param(F, v, rho)
    nu = rho * (v - y)
    fy = np.array([O.fn_eval(W.Fn(h, 1, a=a[i], b=b[i], c=c[i], d=d[i], e=e[i]), y[i:i + 1], 1e-12) for i in range(N)])
    conj = O.fn_conj_terms(F, nu, 1e-12)
    assert np.all(np.isfinite(fy)) and np.all(np.isfinite(conj))
    np.testing.assert_allclose(fy + conj, nu * y, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("h", ["abs", "square", "huber", "logistic", "exp", "ind_box01"])
def test_conjugate_with_quadratic_term_by_grid_supremum(h):
    """f*(s) = sup_y s y - f(y) by a fine grid for a few (a, b, c, d, e, s); the
    grid also holds the points where h has a kink or a domain boundary (u = 0
    and u = 1, i.e. y = b/a and (1 + b)/a), where the supremum often sits."""
    rng = np.random.default_rng(11)
    grid = np.linspace(-12.0, 12.0, 480001)
    for _ in range(4):
        a, b, c, d, e = rng.uniform(0.5, 1.5), rng.normal(), rng.uniform(0.3, 1.5), rng.normal(), rng.uniform(0.3, 1.5)
        s = rng.normal(0, 1.5)
        ys = np.concatenate([grid, [b / a, (1.0 + b) / a]])
        F = W.Fn(h, 1, a=a, b=b, c=c, d=d, e=e)
        with np.errstate(invalid="ignore", over="ignore"):
            hv = O.h_eval(h, a * ys - b)
            fv = c * hv + d * ys + 0.5 * e * ys * ys
        brute = np.max(s * ys - fv)
        got = O.fn_conj(F, np.array([s]))
        assert abs(got - brute) <= 1e-6 * max(1.0, abs(brute)), (h, got, brute)


def test_gap_stop_ridge_certificate():
    """Ridge: f = 1/2 ||y - b||^2, g = (lam/2) ||x||^2 (every domain full).
    At the gap stop, p(x) - p* <= eta < eps_gap with p* in closed form."""
    rng = np.random.default_rng(0)
    m, n, lam = 200, 50, 0.5
    A = rng.normal(size=(m, n)) / np.sqrt(n)
    b = rng.normal(size=m)
    f = W.Fn("square", m, b=b)
    g = W.Fn("square", n, c=lam)
    r = O.solve(A, f, g, O.Params(stop="gap"))
    x_star = np.linalg.solve(A.T @ A + lam * np.eye(n), A.T @ b)
    p_star = 0.5 * np.sum((A @ x_star - b) ** 2) + 0.5 * lam * np.sum(x_star ** 2)
    assert r.converged
    assert 0.0 <= r.optval - p_star <= r.gap + 1e-12
    assert r.gap < r.eps_gap
    # the returned tuple is primal and dual feasible
    np.testing.assert_allclose(r.y, A @ r.x, atol=1e-10)
    np.testing.assert_allclose(r.mu, -A.T @ r.nu, atol=1e-10)


def test_gap_stop_lasso_certificate():
    """Lasso: g*(mu) is the indicator of |mu| <= lam, so the gap is infinite
    until every |mu_j| <= lam; when it stops, the tuple is within eta of the
    optimum of a tight reference solve."""
    p = W.lasso(200, 50, 1, dtype=np.float64)
    r = O.solve(p.A, p.f, p.g, O.Params(stop="gap", max_iter=5000), record=True)
    ref = O.solve(p.A, p.f, p.g, O.Params(eps_abs=1e-10, eps_rel=1e-10, max_iter=100000))
    assert r.converged and np.isfinite(r.gap)
    assert r.optval - ref.optval <= r.gap + 1e-9
    assert np.max(np.abs(r.mu)) <= p.meta["lam"] * (1 + 1e-12)
    assert not np.isfinite(r.history["gap"][0])


def test_gap_infinite_with_violated_constraint():
    """NNLS (g = indicator of x >= 0): the projection's x has negative entries
    early on, so the gap is infinite there (Section 3.4)."""
    p = W.nnls_from(W.lasso(100, 40, 2, dtype=np.float64))
    r = O.solve(p.A, p.f, p.g, O.Params(stop="gap", max_iter=20), record=True)
    assert not np.isfinite(r.history["gap"][0])
