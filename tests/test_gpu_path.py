"""GPU tests of the lambda path (R Lasso problems sharing one A, iterated
together with stacked right-hand sides on MFMA).

Tolerance: objectives |p - p_ref| <= 1e-3 max(|p_ref|, 1) against the FP64
oracle and against the same problem solved alone on the whole-GPU path;
the critical lambda gives x = 0 (Appendix A.4).
"""
import numpy as np
import pytest

from oracle import pogs_oracle as O
from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu
FLT_EPS = float(np.finfo(np.float32).eps)


def _path(m, n, R, seed):
    return W.lambda_path(m=m, n=n, R=R, seed=seed)


@pytest.mark.parametrize("m,n,R", [(600, 150, 8), (1000, 257, 5), (700, 300, 1), (2000, 500, 70)])
def test_path_matches_alone_and_oracle(m, n, R):
    probs = _path(m, n, R, seed=m + n)
    A = probs[0].A
    with P.Context(A) as ctx:
        res = ctx.solve_path([p.f for p in probs], [p.g for p in probs])
        alone = [ctx.solve(p.f, p.g) for p in probs]
    check = range(R) if R <= 8 else [0, R // 2, R - 1]
    for r in check:
        p = probs[r]
        ref = O.solve(A.astype(np.float64), p.f, p.g, O.Params(eps_cmp=FLT_EPS))
        assert res[r].converged, (r, res[r])
        tol = 1e-3 * max(abs(ref.optval), 1.0)
        assert abs(res[r].optval - ref.optval) <= tol, (r, res[r].optval, ref.optval)
        assert abs(res[r].optval - alone[r].optval) <= tol
    # the largest lambda is the critical one: x* = 0 (Appendix A.4).  At the
    # stopping tolerance the iterate is not exactly 0; it must be as close to 0
    # as the oracle's own iterate and small next to the smallest lambda's x.
    if R > 1:
        ref = O.solve(A.astype(np.float64), probs[-1].f, probs[-1].g, O.Params(eps_cmp=FLT_EPS))
        xmax = float(np.max(np.abs(res[-1].x)))
        assert xmax <= 2.0 * float(np.max(np.abs(ref.x))) + 1e-5, (xmax, float(np.max(np.abs(ref.x))))
        assert xmax <= 1e-2 * float(np.max(np.abs(res[0].x)))


def test_path_rejects_wide_and_bad_R():
    A = np.random.default_rng(0).normal(size=(50, 80)).astype(np.float32)
    f = W.Fn("square", 50, b=np.ones(50))
    g = W.Fn("abs", 80, c=0.1)
    with P.Context(A) as ctx:
        with pytest.raises(P.PogsError) as ei:
            ctx.solve_path([f], [g])
        assert ei.value.code == P.POGS_EUNSUPPORTED
    A = np.random.default_rng(0).normal(size=(80, 50)).astype(np.float32)
    f = W.Fn("square", 80, b=np.ones(80))
    g = W.Fn("abs", 50, c=0.1)
    with P.Context(A) as ctx:
        with pytest.raises(P.PogsError) as ei:
            ctx.solve_path([f] * 257, [g] * 257)
        assert ei.value.code == P.POGS_EINVAL
