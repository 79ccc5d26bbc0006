"""Pins for the oracle's ADMM solver (Algorithm 1 + Sections 3.2-3.4, 4.3, 5).

The iteration is checked by invariants the paper derives (Section 3.3), and
its results against optima found without ADMM: closed forms, SciPy's NNLS,
HiGHS LP and L-BFGS-B solvers, and brute-force enumeration on tiny problems
(oracle/brute.py).  CPU only.
"""
import math

import numpy as np
import pytest
from scipy.optimize import linprog, minimize, nnls

from oracle import brute
from oracle import pogs_oracle as O
from paper_1503_08366_amd import workloads as W

TIGHT = O.Params(eps_abs=1e-9, eps_rel=1e-9, max_iter=20000, eps_cmp=2.0 ** -52)


# --------------------------------------------------------------------------
# Algorithm 3 as pure logic
# --------------------------------------------------------------------------

def test_adaptive_rho_script():
    """Scripted residual sequence, trajectory worked out by hand from
    Algorithm 3 with delta = 2, tau = 0.5."""
    # (r_pri < eps_pri, r_dual < eps_dual) per iteration k
    seq = [(False, True), (False, True), (False, True), (True, False), (True, False),
           (True, False), (True, False), (False, True), (False, True), (True, True)]
    rho, l, u = 1.0, 0, 0
    traj = []
    for k, (pc, dc) in enumerate(seq):
        rp, ep = (0.5, 1.0) if pc else (2.0, 1.0)
        rd, ed = (0.5, 1.0) if dc else (2.0, 1.0)
        rho, l, u = O.adaptive_rho(rho, l, u, k, rp, ep, rd, ed, delta=2.0, tau=0.5)
        traj.append((rho, l, u))
    # k=0: dual ok but 0.5*0 > 0 false -> no change
    # k=1: 0.5 > l=0 -> rho=2, u=1
    # k=2: 1.0 > 0 -> rho=4, u=2
    # k=3: primal ok, 1.5 > u=2 false -> none
    # k=4: 2.0 > 2 false -> none
    # k=5: 2.5 > 2 -> rho=2, l=5
    # k=6: 3.0 > 2 -> rho=1, l=6
    # k=7: dual ok, 3.5 > l=6 false -> none
    # k=8: 4.0 > 6 false -> none
    # k=9: both ok; dual branch first: 4.5 > 6 false; primal: 4.5 > u=2 -> rho=0.5, l=9
    expect = [(1, 0, 0), (2, 0, 1), (4, 0, 2), (4, 0, 2), (4, 0, 2), (2, 5, 2), (1, 6, 2),
              (1, 6, 2), (1, 6, 2), (0.5, 9, 2)]
    assert traj == [(float(a), b, c) for a, b, c in expect]


# --------------------------------------------------------------------------
# Invariants of the iteration (Section 3.3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(60, 25), (25, 60)])
def test_iteration_invariants(shape):
    p = W.lasso(*shape, seed=3, dtype=np.float64)
    r = O.solve(p.A, p.f, p.g, O.Params(max_iter=300), record=True)
    h = r.history
    ynorm = 1.0
    # y^{k+1} = A^ x^{k+1} after every projection; x~ + A^T y~ = 0 likewise
    # (the dual-feasibility argument of Section 3.3 holds for every k)
    assert max(h["inv_primal"]) < 1e-12 * max(1.0, ynorm) * 100
    assert max(h["inv_dual"]) < 1e-11


def test_half_step_tuple_is_fenchel_feasible():
    """mu_h in dg(x_h) and nu_h in df(y_h) (Section 3.3): the Fenchel equalities
    hold termwise for the returned tuple, in the original variables."""
    for p in [W.lasso(50, 20, seed=1, dtype=np.float64), W.lp(12, 6, seed=2, dtype=np.float64),
              W.svm(40, 10, seed=3, dtype=np.float64), W.logistic(50, 15, seed=4, dtype=np.float64),
              W.basis_pursuit(30, 12, seed=5, dtype=np.float64), W.entropy_max(5, 25, seed=6, dtype=np.float64),
              W.huber_fit(60, 10, seed=7, dtype=np.float64)]:
        r = O.solve(p.A, p.f, p.g, O.Params(max_iter=200))
        if p.f.field("e").any() or p.g.field("e").any():
            continue
        for fn, v, s in [(p.f, r.y, r.nu), (p.g, r.x, r.mu)]:
            P = O.as_param(fn)
            for i in range(fn.size):
                hi = P.h if isinstance(P.h, str) else P.h[i]
                Fi = O.Param(hi, *(getattr(P, k)[i:i + 1] for k in "abcde"))
                lhs = O.fn_eval(Fi, v[i:i + 1], 1e-9) + O.fn_conj(Fi, s[i:i + 1], 1e-9)
                assert math.isfinite(lhs), (p.name, i)
                assert abs(lhs - s[i] * v[i]) < 1e-7 * max(1.0, abs(s[i] * v[i])), (p.name, i)


def test_rho_change_preserves_dual_invariant():
    p = W.lasso(80, 30, seed=5, dtype=np.float64)
    r = O.solve(p.A, p.f, p.g, O.Params(max_iter=500), record=True)
    rhos = r.history["rho"]
    assert len(set(rhos)) > 1  # adaptive rho actually moved
    assert max(r.history["inv_dual"]) < 1e-11


# --------------------------------------------------------------------------
# Results against optima found without ADMM
# --------------------------------------------------------------------------

def test_ridge_closed_form():
    """f = 1/2||y - b||^2, g = (lam/2)||x||^2: x* = (A^T A + lam I)^{-1} A^T b."""
    rng = np.random.default_rng(0)
    for m, n in [(40, 15), (15, 40)]:
        A = rng.normal(size=(m, n))
        b = rng.normal(size=m)
        lam = 0.7
        f = W.Fn("square", m, b=b)
        g = W.Fn("square", n, c=lam)
        r = O.solve(A, f, g, TIGHT)
        xs = np.linalg.solve(A.T @ A + lam * np.eye(n), A.T @ b)
        assert r.converged
        np.testing.assert_allclose(r.x, xs, atol=1e-6)
        np.testing.assert_allclose(r.y, A @ xs, atol=1e-6)


def test_nnls_against_scipy_and_supports():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(14, 7))
    b = rng.normal(size=14)
    f = W.Fn("square", 14, b=b)
    g = W.Fn("ind_ge0", 7)
    r = O.solve(A, f, g, TIGHT)
    x_sp, _ = nnls(A, b)
    v_bf, x_bf = brute.nnls_supports(A, b)
    np.testing.assert_allclose(x_sp, x_bf, atol=1e-10)
    np.testing.assert_allclose(r.x, x_sp, atol=1e-6)
    assert abs(r.optval - v_bf) < 1e-7 * max(1, v_bf)


def test_lasso_against_sign_enumeration():
    rng = np.random.default_rng(2)
    A = rng.normal(size=(12, 6))
    b = rng.normal(size=12)
    lam = 0.3 * np.max(np.abs(A.T @ b))
    f = W.Fn("square", 12, b=b)
    g = W.Fn("abs", 6, c=lam)
    r = O.solve(A, f, g, TIGHT)
    v_bf, x_bf = brute.lasso_signs(A, b, lam)
    np.testing.assert_allclose(r.x, x_bf, atol=1e-6)
    assert abs(r.optval - v_bf) < 1e-8 * max(1, v_bf)
    # KKT: |A^T (b - A x)| <= lam, with equality and matching sign on the support
    gr = A.T @ (b - A @ r.x)
    assert np.all(np.abs(gr) <= lam * (1 + 1e-6))
    sup = np.abs(x_bf) > 1e-8
    np.testing.assert_allclose(gr[sup], lam * np.sign(x_bf[sup]), rtol=1e-5)


def test_lasso_critical_lambda_gives_zero():
    """lam >= ||A^T b||_inf makes x* = 0 exactly (Appendix A.4)."""
    p = W.lasso(60, 30, seed=4, dtype=np.float64)
    lam = 1.0001 * float(np.max(np.abs(p.A.T @ p.meta["b"])))
    g = W.Fn("abs", 30, c=lam)
    r = O.solve(p.A, p.f, g, O.Params(eps_abs=1e-8, eps_rel=1e-8, max_iter=5000))
    assert np.max(np.abs(r.x)) < 1e-6


def test_logistic_critical_lambda_gives_zero():
    """lam >= ||A^T (1/2 - b)||_inf makes x* = 0 (Appendix A.5)."""
    p = W.logistic(80, 20, seed=5, dtype=np.float64)
    lam = 1.0001 * float(np.max(np.abs(p.A.T @ (0.5 - p.meta["labels01"]))))
    g = W.Fn("abs", 20, c=lam)
    r = O.solve(p.A, p.f, g, O.Params(eps_abs=1e-8, eps_rel=1e-8, max_iter=5000))
    assert np.max(np.abs(r.x)) < 1e-6


def test_logistic_against_lbfgs():
    p = W.logistic(60, 10, seed=6, dtype=np.float64)
    A, lab, lam = p.A, p.meta["labels01"], p.meta["lam"]
    n = A.shape[1]

    def obj(z):
        x = z[:n] - z[n:]
        t = A @ x
        val = np.sum(np.logaddexp(0, t) - lab * t) + lam * np.sum(z)
        sig = 1 / (1 + np.exp(-t))
        gx = A.T @ (sig - lab)
        return val, np.concatenate([gx + lam, -gx + lam])

    res = minimize(obj, np.zeros(2 * n), jac=True, method="L-BFGS-B",
                   bounds=[(0, None)] * (2 * n), options={"gtol": 1e-12, "ftol": 1e-15, "maxiter": 10000})
    r = O.solve(A, p.f, p.g, TIGHT)
    assert abs(r.optval - res.fun) < 1e-7 * max(1, abs(res.fun))
    np.testing.assert_allclose(r.x, res.x[:n] - res.x[n:], atol=1e-4)


def test_lp_against_highs_and_vertices():
    for seed in range(3):
        p = W.lp(6, 3, seed=seed, dtype=np.float64)
        A, b, c = p.A, p.meta["b"], p.meta["cost"]
        v_bf, _ = brute.lp_vertices(A, b, c)
        hi = linprog(c, A_ub=A, b_ub=b, bounds=[(0, 1)] * 3, method="highs")
        assert abs(hi.fun - v_bf) < 1e-9
        r = O.solve(A, p.f, p.g, TIGHT)
        assert r.converged
        assert abs(r.optval - v_bf) < 1e-6


def test_dose_against_highs():
    """0.6|y - t| + 0.4 (y - t) with x >= 0 as an LP in (x, s):
    min sum 0.6 s + 0.4 (A x - t) s.t. -s <= A x - t <= s, x >= 0."""
    p = W.dose(40, 8, seed=7, dtype=np.float64)
    A, t = p.A, p.meta["target"]
    m, n = A.shape
    cvec = np.concatenate([0.4 * A.sum(axis=0), 0.6 * np.ones(m)])
    Aub = np.block([[A, -np.eye(m)], [-A, -np.eye(m)]])
    bub = np.concatenate([t, -t])
    hi = linprog(cvec, A_ub=Aub, b_ub=bub, bounds=[(0, None)] * (n + m), method="highs")
    p_star = hi.fun - 0.4 * t.sum()
    r = O.solve(A, p.f, p.g, TIGHT)
    assert abs(r.optval + p.f.const - p_star) < 1e-6 * max(1, abs(p_star))


def test_svm_against_qp():
    p = W.svm(30, 4, seed=8, dtype=np.float64)
    A = p.A
    m, n = A.shape
    # min sum t + lam ||x||^2, t >= 0, t >= 1 - A x  (variables x, t)
    cons = [{"type": "ineq", "fun": lambda z: z[n:] - 1 + A @ z[:n]}]
    res = minimize(lambda z: z[n:].sum() + np.dot(z[:n], z[:n]), np.zeros(n + m),
                   constraints=cons, bounds=[(None, None)] * n + [(0, None)] * m,
                   method="SLSQP", options={"ftol": 1e-14, "maxiter": 1000})
    r = O.solve(A, p.f, p.g, TIGHT)
    assert abs(r.optval - res.fun) < 1e-6 * max(1, res.fun)


def test_duality_gap_bounds_suboptimality():
    """Section 2.1: for a primal and dual feasible tuple eta >= p(x) - p*.
    Lasso, with nu scaled into dom f* ... here f* is finite everywhere and
    g* = lam-box indicator, so nu is scaled to ||A^T nu||_inf <= lam."""
    p = W.lasso(50, 20, seed=9, dtype=np.float64)
    A, b, lam = p.A, p.meta["b"], p.meta["lam"]
    v_ref = O.solve(A, p.f, p.g, TIGHT).optval
    for iters in [5, 20, 80]:
        r = O.solve(A, p.f, p.g, O.Params(max_iter=iters))
        x = r.x
        y = A @ x
        nu = r.nu * min(1.0, lam / np.max(np.abs(A.T @ r.nu)))
        mu = -A.T @ nu
        eta = O.duality_gap(p.f, p.g, x, y, mu, nu, tol=1e-12)
        pval = O.fn_eval(p.f, y) + O.fn_eval(p.g, x)
        assert eta >= -1e-12
        assert pval - v_ref <= eta + 1e-10


def test_equilibration_does_not_change_optimum():
    p = W.lasso(40, 15, seed=10, dtype=np.float64)
    on = O.solve(p.A, p.f, p.g, TIGHT)
    off = O.solve(p.A, p.f, p.g, O.Params(**{**TIGHT.__dict__, "equilibrate": False}))
    assert abs(on.optval - off.optval) < 1e-8 * max(1, abs(on.optval))


def test_small_lasso_config_converges():
    """Lasso 200x100 in float64, eps 1e-4/1e-3, at most 2000 iterations:
    converges, and the objective is within the stated tolerance of p*."""
    p = W.lasso_small_f64()
    r = O.solve(p.A, p.f, p.g, O.Params(max_iter=p.max_iter, eps_cmp=2.0 ** -52))
    ref = O.solve(p.A, p.f, p.g, TIGHT)
    assert r.converged and r.iters < 2000
    assert abs(r.optval - ref.optval) <= 1e-3 * max(abs(ref.optval), 1.0)


def test_two_iterations_by_hand():
    """A = [1], f = 1/2 (y - 2)^2, g = 0.5 |x|, rho = 1, alpha = 1.7, no
    equilibration.  Worked by hand from Algorithm 1 with the Section 3.2
    relaxation and the Section 3.3 half-step duals:
      k=0: x_h = 0, y_h = 1, mu_h = 0, nu_h = -1; x_r = 0, y_r = 1.7;
           projection of (0, 1.7) onto y = x gives x = y = 0.85;
           x~ = -0.85, y~ = 0.85; no rho change at k = 0.
      k=1: x_h = soft(0.85 + 0.85, 0.5) = 1.2, y_h = prox_f(0) = 1,
           mu_h = -(1.2 - 0.85 - 0.85) = 0.5, nu_h = -(1 - 0.85 + 0.85) = -1;
           r_pri = |1.2 - 1| = 0.2, r_dual = |-1 + 0.5| = 0.5."""
    A = np.array([[1.0]])
    f = W.Fn("square", 1, b=2.0)
    g = W.Fn("abs", 1, c=0.5)
    prm = O.Params(max_iter=1, equilibrate=False)
    r = O.solve(A, f, g, prm)
    assert (r.x[0], r.y[0], r.mu[0], r.nu[0]) == (0.0, 1.0, 0.0, -1.0)
    assert (r.r_pri, r.r_dual) == (1.0, 1.0)
    r = O.solve(A, f, g, O.Params(max_iter=2, equilibrate=False))
    np.testing.assert_allclose([r.x[0], r.y[0], r.mu[0], r.nu[0]], [1.2, 1.0, 0.5, -1.0], atol=1e-15)
    np.testing.assert_allclose([r.r_pri, r.r_dual], [0.2, 0.5], atol=1e-15)
    assert not r.converged and r.iters == 2


# --------------------------------------------------------------------------
# Warm start (Section 5: the caller may supply x0 and nu0)
# --------------------------------------------------------------------------
def test_warm_start_from_zero_is_the_cold_start():
    p = W.lasso(60, 25, seed=11, dtype=np.float64)
    prm = O.Params(eps_cmp=2.0 ** -52)
    cold = O.solve(p.A, p.f, p.g, prm)
    warm = O.solve(p.A, p.f, p.g, prm, x0=np.zeros(25), nu0=np.zeros(60))
    assert warm.iters == cold.iters
    assert np.array_equal(warm.x, cold.x) and np.array_equal(warm.nu, cold.nu)


@pytest.mark.parametrize("kind", ["lasso", "nnls", "logistic", "wide_lasso"])
def test_warm_start_from_an_optimum_is_a_fixed_point(kind):
    """From an optimal pair, prox_g(x* + mu*/rho) = x* because mu* is in
    dg(x*), and likewise for y: the warm-start state does not move and the
    stop test passes at the first iteration."""
    if kind == "lasso":
        p = W.lasso(80, 30, seed=12, dtype=np.float64)
    elif kind == "nnls":
        p = W.nnls_from(W.lasso(80, 30, seed=13, dtype=np.float64))
    elif kind == "logistic":
        p = W.logistic(90, 20, seed=14, dtype=np.float64)
    else:
        p = W.lasso(30, 70, seed=15, dtype=np.float64)
    ref = O.solve(p.A, p.f, p.g, TIGHT)
    assert ref.converged
    r = O.solve(p.A, p.f, p.g, O.Params(eps_cmp=2.0 ** -52), x0=ref.x, nu0=ref.nu)
    assert r.converged and r.iters == 1
    scale = max(1.0, float(np.max(np.abs(ref.x))))
    assert np.max(np.abs(r.x - ref.x)) <= 1e-6 * scale


def test_warm_start_along_a_lambda_path_saves_iterations():
    """Continuation: the solution at one lambda is a good start for the next."""
    probs = W.lambda_path(m=300, n=80, R=6, seed=16)
    prm = O.Params(eps_cmp=float(np.finfo(np.float32).eps))
    A = probs[0].A.astype(np.float64)
    prev = O.solve(A, probs[2].f, probs[2].g, prm)
    cold = O.solve(A, probs[3].f, probs[3].g, prm)
    warm = O.solve(A, probs[3].f, probs[3].g, prm, x0=prev.x, nu0=prev.nu)
    assert warm.converged and cold.converged
    assert warm.iters < cold.iters
    assert abs(warm.optval - cold.optval) <= 1e-3 * max(1.0, abs(cold.optval))


# --------------------------------------------------------------------------
# Warm start with one half missing (Section 5: "estimated"; reading: one
# proximal point step from zero, the value the prox step itself returns)
# --------------------------------------------------------------------------
def test_estimated_dual_from_x0_closed_form():
    """f = 1/2 ||y - b||^2 with rho: prox(v) = (b + rho v)/(1 + rho), so the
    estimated scaled dual is y~ = prox(y) - y = (b - y)/(1 + rho) with y = A x0,
    and x~ = -A^T y~ (no pre-conditioning: D = E = 1)."""
    rng = np.random.default_rng(21)
    m, n, rho = 40, 15, 1.7
    A = rng.normal(size=(m, n))
    b = rng.normal(size=m)
    x0 = rng.normal(size=n)
    f = W.Fn("square", m, b=b)
    g = W.Fn("abs", n, c=0.3)
    x, y, xt, yt = O.warm_state(A, O.as_param(f), O.as_param(g), np.ones(m), np.ones(n), rho, x0=x0)
    y_ref = A @ x0
    np.testing.assert_allclose(x, x0, rtol=0, atol=0)
    np.testing.assert_allclose(y, y_ref, rtol=1e-14)
    np.testing.assert_allclose(yt, (b - y_ref) / (1.0 + rho), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(xt, -(A.T @ ((b - y_ref) / (1.0 + rho))), rtol=1e-12, atol=1e-13)


def test_estimated_dual_vanishes_at_a_feasible_point_of_an_indicator():
    """f = indicator(y <= b): at a strictly feasible y = A x0 the prox leaves y
    unchanged, so the estimated dual is zero."""
    rng = np.random.default_rng(22)
    m, n = 30, 10
    A = rng.normal(size=(m, n))
    x0 = rng.normal(size=n)
    b = A @ x0 + rng.uniform(0.1, 1.0, m)
    f = W.Fn("ind_le0", m, b=b)
    g = W.Fn("zero", n)
    _, _, xt, yt = O.warm_state(A, O.as_param(f), O.as_param(g), np.ones(m), np.ones(n), 1.0, x0=x0)
    assert np.array_equal(yt, np.zeros(m)) and np.array_equal(xt, np.zeros(n))


def test_estimated_primal_from_nu0_closed_form():
    """g = 1/2 ||x||^2: prox(v) = rho v/(1 + rho); from nu0 alone, y~ = -nu0/rho,
    x~ = -A^T y~ and x = prox(-x~) = -A^T nu0 / (1 + rho), y = A x."""
    rng = np.random.default_rng(23)
    m, n, rho = 35, 12, 0.6
    A = rng.normal(size=(m, n))
    nu0 = rng.normal(size=m)
    f = W.Fn("square", m, b=rng.normal(size=m))
    g = W.Fn("square", n)
    x, y, xt, yt = O.warm_state(A, O.as_param(f), O.as_param(g), np.ones(m), np.ones(n), rho, nu0=nu0)
    np.testing.assert_allclose(yt, -nu0 / rho, rtol=1e-15)
    np.testing.assert_allclose(x, -(A.T @ nu0) / (1.0 + rho), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(y, A @ x, rtol=1e-12, atol=1e-14)


def test_warm_start_from_x_alone_converges_faster():
    """From x* alone the estimated dual starts the iteration near the optimum:
    the same optimum in fewer iterations than a cold start."""
    p = W.lasso(120, 40, seed=24, dtype=np.float64)
    ref = O.solve(p.A, p.f, p.g, TIGHT)
    assert ref.converged
    prm = O.Params(eps_cmp=2.0 ** -52)
    cold = O.solve(p.A, p.f, p.g, prm)
    warm = O.solve(p.A, p.f, p.g, prm, x0=ref.x)
    assert warm.converged and cold.converged
    assert warm.iters < cold.iters, (warm.iters, cold.iters)
    assert abs(warm.optval - ref.optval) <= 1e-3 * max(1.0, abs(ref.optval))


def test_warm_start_from_nu_alone_reaches_the_optimum():
    """From nu* alone the estimated primal is the x half step the iteration
    takes from x = 0 (zero for l1 terms whose dual lies inside the threshold:
    the dual alone does not locate x there); the solve still reaches the
    optimum."""
    p = W.lasso(120, 40, seed=24, dtype=np.float64)
    ref = O.solve(p.A, p.f, p.g, TIGHT)
    warm = O.solve(p.A, p.f, p.g, O.Params(eps_cmp=2.0 ** -52), nu0=ref.nu)
    assert warm.converged
    assert abs(warm.optval - ref.optval) <= 1e-3 * max(1.0, abs(ref.optval))
