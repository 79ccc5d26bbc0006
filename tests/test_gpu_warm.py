"""GPU tests of the warm start (Section 5: the caller may supply x0 and nu0)
on the whole-GPU path, against the FP64 oracle's warm start.

Tolerances: objectives |p - p_ref| <= 1e-3 max(|p_ref|, 1); iteration counts
within 2 of the oracle's (float32 iterations against float64: threshold
decisions may branch, parity on counts is not exact).
"""
import numpy as np
import pytest

from oracle import pogs_oracle as O
from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu
FLT_EPS = float(np.finfo(np.float32).eps)
TIGHT = O.Params(eps_abs=1e-9, eps_rel=1e-9, max_iter=20000, eps_cmp=FLT_EPS)


def _tol(v):
    return 1e-3 * max(abs(v), 1.0)


def test_zero_warm_start_is_the_cold_start():
    p = W.lasso(700, 250, 61)
    with P.Context(p.A) as ctx:
        cold = ctx.solve(p.f, p.g)
        warm = ctx.solve(p.f, p.g, x0=np.zeros(p.n), nu0=np.zeros(p.m))
    assert warm.iters == cold.iters
    np.testing.assert_array_equal(warm.x, cold.x)


@pytest.mark.parametrize("kind", ["lasso", "nnls", "wide_lasso", "logistic"])
def test_warm_start_from_an_optimum_stops_at_once(kind):
    if kind == "lasso":
        p = W.lasso(900, 300, 62)
    elif kind == "nnls":
        p = W.nnls_from(W.lasso(900, 300, 63))
    elif kind == "wide_lasso":
        p = W.lasso(250, 700, 64)
    else:
        p = W.logistic(800, 200, 65)
    ref = O.solve(p.A.astype(np.float64), p.f, p.g, TIGHT)
    assert ref.converged
    with P.Context(p.A) as ctx:
        r = ctx.solve(p.f, p.g, x0=ref.x, nu0=ref.nu)
    assert r.converged and r.iters <= 2, r
    assert abs(r.optval - ref.optval) <= _tol(ref.optval)


def test_warm_start_matches_the_oracle():
    probs = W.lambda_path(m=1200, n=300, R=6, seed=66)
    A = probs[0].A
    prm = O.Params(eps_cmp=FLT_EPS)
    start = O.solve(A.astype(np.float64), probs[2].f, probs[2].g, prm)
    ref = O.solve(A.astype(np.float64), probs[3].f, probs[3].g, prm, x0=start.x, nu0=start.nu)
    with P.Context(A) as ctx:
        r = ctx.solve(probs[3].f, probs[3].g, x0=start.x, nu0=start.nu)
    assert r.converged and ref.converged
    assert abs(r.iters - ref.iters) <= 2, (r.iters, ref.iters)
    assert abs(r.optval - ref.optval) <= _tol(ref.optval)


def test_continuation_saves_iterations():
    probs = W.lambda_path(m=2000, n=500, R=8, seed=67)
    fs, gs = [p.f for p in probs], [p.g for p in probs]
    with P.Context(probs[0].A) as ctx:
        cold = [ctx.solve(f, g) for f, g in zip(fs, gs)]
        cont = ctx.solve_continuation(fs, gs)
    for a, b in zip(cold, cont):
        assert a.converged and b.converged
        assert abs(a.optval - b.optval) <= _tol(a.optval)
    assert sum(r.iters for r in cont) < sum(r.iters for r in cold)


def test_warm_start_from_device_tensors():
    import torch
    p = W.lasso(600, 200, 68)
    ref = O.solve(p.A.astype(np.float64), p.f, p.g, TIGHT)
    with P.Context(p.A) as ctx:
        host = ctx.solve(p.f, p.g, x0=ref.x, nu0=ref.nu)
        dev = ctx.solve(p.f, p.g, device_out=True, x0=torch.tensor(ref.x), nu0=torch.tensor(ref.nu))
    assert dev.iters == host.iters
    np.testing.assert_array_equal(np.asarray(dev.x.cpu()) if hasattr(dev.x, "cpu") else dev.x, host.x)


@pytest.mark.parametrize("half", ["x0", "nu0"])
@pytest.mark.parametrize("kind", ["tall_lasso", "wide_lasso", "logistic", "nnls"])
def test_half_warm_start_matches_the_oracle(kind, half):
    """Only one half given: the other is estimated (Section 5) the same way
    on both sides (one proximal point step from zero); iteration counts and
    objectives follow the oracle's warm-started solve."""
    if kind == "tall_lasso":
        p = W.lasso(1500, 400, 71)
    elif kind == "wide_lasso":
        p = W.lasso(300, 900, 72)
    elif kind == "logistic":
        p = W.logistic(1200, 300, 73)
    else:
        p = W.nnls_from(W.lasso(1400, 350, 74))
    prm = O.Params(eps_cmp=FLT_EPS)
    start = O.solve(p.A.astype(np.float64), p.f, p.g, TIGHT)
    kw = {"x0": start.x} if half == "x0" else {"nu0": start.nu}
    ref = O.solve(p.A.astype(np.float64), p.f, p.g, prm, **kw)
    with P.Context(p.A) as ctx:
        r = ctx.solve(p.f, p.g, **kw)
    print(kind, half, "gpu", r.iters, "oracle", ref.iters, flush=True)
    assert r.converged and ref.converged
    assert abs(r.iters - ref.iters) <= 2, (r.iters, ref.iters)
    assert abs(r.optval - ref.optval) <= _tol(ref.optval)


def test_half_warm_start_sparse_matches_the_oracle():
    p = W.sparse_problem("lasso", 3000, 800, 12, seed=75)
    dense = p.A.toarray().astype(np.float64)
    start = O.solve(dense, p.f, p.g, TIGHT)
    prm = P.default_params(projection="cgls")
    ref = O.solve(dense, p.f, p.g, O.Params(eps_cmp=FLT_EPS, projection="cgls", cg_max_iter=prm.cg_max_iter,
                                            cg_tol=prm.cg_tol), x0=start.x)
    with P.SparseContext(p.A) as ctx:
        r = ctx.solve(p.f, p.g, x0=start.x)
    assert r.converged and ref.converged
    assert abs(r.iters - ref.iters) <= 3, (r.iters, ref.iters)
    assert abs(r.optval - ref.optval) <= _tol(ref.optval)
