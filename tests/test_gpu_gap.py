"""GPU tests of the gap-based stopping rule (Section 3.4) on the whole-GPU
path, through the C ABI, against the FP64 oracle with the same rule.

Tolerance: objective |p - p_oracle| <= 1e-3 max(|p_oracle|, 1); float64 runs
stop within one iteration of the oracle's; the returned tuple is the feasible
one: y = A x and mu = -A^T nu up to the rounding of float32 vectors
(relative 1e-4 for float32, 1e-9 for float64).
"""
import numpy as np
import pytest

from oracle import pogs_oracle as O
from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = {np.float32: float(np.finfo(np.float32).eps), np.float64: float(np.finfo(np.float64).eps)}


def _ridge(m, n, seed, lam=0.5):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(m, n)) / np.sqrt(n)
    b = rng.normal(size=m)
    return A, W.Fn("square", m, b=b), W.Fn("square", n, c=lam)


def _elastic(m, n, seed):
    """Lasso data with g = lam |x| + (e/2) x^2 (e > 0: the conjugate of g is
    finite everywhere and goes through the prox of the h term)."""
    p = W.lasso(m, n, seed, dtype=np.float64)
    return p.A, p.f, W.Fn("abs", n, c=p.meta["lam"], e=0.3)


def _lasso(m, n, seed):
    p = W.lasso(m, n, seed, dtype=np.float64)
    return p.A, p.f, p.g


CASES = {"ridge": _ridge, "elastic": _elastic, "lasso": _lasso}


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("case,shape", [("ridge", (300, 80)), ("ridge", (80, 300)), ("elastic", (400, 100)),
                                        ("lasso", (300, 60)), ("elastic", (90, 250))])
def test_gap_stop_matches_oracle(case, shape, dt):
    A, f, g = CASES[case](*shape, seed=sum(shape))
    A = A.astype(dt)
    A64 = A.astype(np.float64)
    prm = P.default_params(stop_rule="gap", max_iter=5000)
    with P.Context(A) as ctx:
        r = ctx.solve(f, g, prm)
    ref = O.solve(A64, f, g, O.Params(stop="gap", max_iter=5000, eps_cmp=EPS[dt]))
    assert ref.converged and r.status == P.POGS_CONVERGED, (r, ref.iters)
    assert np.isfinite(r.gap) and r.gap < r.eps_gap
    tol = 1e-3 * max(abs(ref.optval), 1.0)
    assert abs(r.optval - ref.optval) <= tol, (r.optval, ref.optval, r.iters, ref.iters)
    x, y, mu, nu = (v.astype(np.float64) for v in (r.x, r.y, r.mu, r.nu))
    rt = 1e-4 if dt == np.float32 else 1e-9
    assert np.linalg.norm(y - A64 @ x) <= rt * max(1.0, np.linalg.norm(y))
    assert np.linalg.norm(mu + A64.T @ nu) <= rt * max(1.0, np.linalg.norm(mu))
    if dt == np.float64:
        assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
        assert abs(r.gap - ref.gap) <= 1e-6 * max(1.0, abs(ref.gap)) or abs(r.iters - ref.iters) == 1
    print(f"{case} {shape} {np.dtype(dt).name}: iters {r.iters} (oracle {ref.iters}), gap {r.gap:.3e} "
          f"(oracle {ref.gap:.3e}), eps_gap {r.eps_gap:.3e}")


def test_gap_rule_with_constraint_runs_to_cap():
    """NNLS: the projection's x violates x >= 0, the gap stays infinite and
    the solve ends at max_iter, as the oracle does."""
    p = W.nnls_from(W.lasso(200, 60, 31, dtype=np.float64))
    prm = P.default_params(stop_rule="gap", max_iter=40)
    with P.Context(p.A) as ctx:
        r = ctx.solve(p.f, p.g, prm)
    ref = O.solve(p.A, p.f, p.g, O.Params(stop="gap", max_iter=40, eps_cmp=EPS[np.float64]))
    assert r.status == P.POGS_MAXITER and not ref.converged
    assert not np.isfinite(r.gap)


def test_gap_rule_rejections():
    p = W.lasso(200, 60, 32)
    with P.Context(p.A) as ctx:
        with pytest.raises(P.PogsError) as ei:
            ctx.solve(p.f, p.g, P.default_params(stop_rule="gap", projection="cgls"))
        assert ei.value.code == P.POGS_EUNSUPPORTED
        with pytest.raises(P.PogsError) as ei:
            ctx.solve_path([p.f], [p.g], P.default_params(stop_rule="gap"))
        assert ei.value.code == P.POGS_EUNSUPPORTED
        with pytest.raises(P.PogsError) as ei:
            ctx.solve(p.f, p.g, P.default_params(stop_rule=7))
        assert ei.value.code == P.POGS_EINVAL
    with pytest.raises(P.PogsError) as ei:
        P.pogs_solve_batch([p], P.default_params(stop_rule="gap"))
    assert ei.value.code == P.POGS_EUNSUPPORTED
