"""GPU tests of the lambda path (R Lasso problems sharing one A, iterated
together with stacked right-hand sides on MFMA).

Tolerance: objectives |p - p_ref| <= 1e-3 max(|p_ref|, 1) against the FP64
oracle and against the same problem solved alone on the whole-GPU path;
the critical lambda gives x = 0 (Appendix A.4).
"""
import ctypes as C

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


def test_path_rejects_invalid_functions():
    # every function is validated as it is packed (Section 5: c, e >= 0,
    # finite parameters): a bad entry in any problem fails the whole call
    probs = _path(600, 150, 4, seed=11)
    A = probs[0].A
    bad_g = W.Fn("abs", 150, c=-1.0)
    b = np.array(probs[1].f.b, dtype=np.float64).copy()
    b[17] = np.nan
    bad_f = W.Fn("square", 600, b=b)
    with P.Context(A) as ctx:
        for fs, gs in (([p.f for p in probs], [p.g for p in probs[:2]] + [bad_g, probs[3].g]),
                       ([probs[0].f, bad_f] + [p.f for p in probs[2:]], [p.g for p in probs])):
            with pytest.raises(P.PogsError) as ei:
                ctx.solve_path(fs, gs)
            assert ei.value.code == P.POGS_EINVAL
        ok = ctx.solve_path([p.f for p in probs], [p.g for p in probs])  # the context still works
    assert all(r.converged for r in ok)


class _BroadcastHolder(P._FnHolder):
    """A function with one base function and scalar parameters passed as one
    entry each with stride 0 (broadcast), as include/pogs.h allows."""

    def __init__(self, fn, length):
        super().__init__(fn, length)
        if isinstance(fn.h, str) and all(np.ndim(getattr(fn, k)) == 0 for k in "abcde"):
            self.h1 = self.h[:1].copy()
            self.one = [None if a is None else a[:1].copy() for a in self.arrs]
            dp = C.POINTER(C.c_double)
            self.s = P.pogs_fn(length, 0, self.h1.ctypes.data_as(C.POINTER(C.c_uint8)),
                               *(dp() if a is None else a.ctypes.data_as(dp) for a in self.one))


def test_path_and_solve_take_broadcast_functions(monkeypatch):
    probs = _path(1000, 257, 5, seed=5)
    A = probs[0].A
    with P.Context(A) as ctx:
        ref = ctx.solve_path([p.f for p in probs], [p.g for p in probs])
        ref1 = ctx.solve(probs[2].f, probs[2].g)
        monkeypatch.setattr(P, "_FnHolder", _BroadcastHolder)
        got = ctx.solve_path([p.f for p in probs], [p.g for p in probs])
        got1 = ctx.solve(probs[2].f, probs[2].g)
    for a, b in zip(ref + [ref1], got + [got1]):
        assert a.iters == b.iters
        np.testing.assert_array_equal(a.x, b.x)
        np.testing.assert_array_equal(a.nu, b.nu)
        assert a.optval == b.optval
