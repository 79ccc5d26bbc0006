"""GPU tests of the batched solver (grouped launches: one launch per phase for
all problems of a group) and the serving engine (continuous batching).

Tolerances: objectives |p - p_oracle| <= 1e-3 max(|p_oracle|, 1) against the
FP64 oracle; a problem solved alone, in a mix, in one launch or over many
serving rounds gives bitwise-identical results (its arithmetic does not depend
on co-scheduling), which the tests assert exactly.
"""
import time

import numpy as np
import pytest

from oracle import pogs_oracle as O
from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu
FLT_EPS = float(np.finfo(np.float32).eps)


def _mix(count, seed, m_range=(64, 700), n_range=(32, 300)):
    return W.batch_mix(count=count, seed=seed, m_range=m_range, n_range=n_range)


def _oracle(p):
    return O.solve(p.A.astype(np.float64), p.f, p.g,
                   O.Params(eps_abs=p.eps_abs, eps_rel=p.eps_rel, max_iter=p.max_iter, eps_cmp=FLT_EPS))


def test_batch_matches_oracle():
    probs = _mix(24, seed=11)
    res = P.pogs_solve_batch(probs)
    for p, r in zip(probs, res):
        ref = _oracle(p)
        assert r.converged, (p.name, p.m, p.n, r)
        assert abs(r.optval - ref.optval) <= 1e-3 * max(abs(ref.optval), 1.0), (p.name, p.m, p.n, r.optval, ref.optval)


def test_batch_edge_shapes():
    probs = [W.lasso(1, 1, 1), W.lasso(1, 40, 2), W.lasso(300, 1, 3), W.lasso(64, 64, 4),
             W.logistic(65, 63, 5), W.lasso(129, 257, 6)]
    res = P.pogs_solve_batch(probs)
    for p, r in zip(probs, res):
        ref = _oracle(p)
        assert r.status in (P.POGS_CONVERGED, P.POGS_MAXITER)
        if ref.converged:
            assert abs(r.optval - ref.optval) <= 1e-3 * max(abs(ref.optval), 1.0), (p.m, p.n, r.optval, ref.optval)


def test_batch_alone_equals_mix():
    probs = _mix(12, seed=12)
    mix = P.pogs_solve_batch(probs)
    for i in [0, 3, 7, 11]:
        alone = P.pogs_solve_batch([probs[i]])[0]
        assert alone.iters == mix[i].iters
        np.testing.assert_array_equal(alone.x, mix[i].x)
        np.testing.assert_array_equal(alone.nu, mix[i].nu)


def test_batch_agrees_with_whole_gpu_path():
    probs = _mix(6, seed=13)
    res = P.pogs_solve_batch(probs)
    for p, r in zip(probs, res):
        with P.Context(p.A) as ctx:
            s = ctx.solve(p.f, p.g)
        assert abs(r.optval - s.optval) <= 1e-3 * max(abs(s.optval), 1.0)


def test_batch_routes_large_problem_to_whole_gpu_path():
    big = W.lasso(600, 4500, 21)  # n above the grouped path's limit
    small = W.lasso(300, 100, 22)
    res = P.pogs_solve_batch([small, big])
    for p, r in zip([small, big], res):
        ref = _oracle(p)
        assert r.converged
        assert abs(r.optval - ref.optval) <= 1e-3 * max(abs(ref.optval), 1.0)


def test_serving_engine_same_as_alone():
    probs = _mix(10, seed=14)
    alone = [P.pogs_solve_batch([p])[0] for p in probs]
    eng = P.BatchEngine(chunk_iters=7)
    try:
        tickets = []
        for i, p in enumerate(probs):
            tickets.append(eng.submit(p))
            if i % 3 == 0:
                time.sleep(0.01)  # later requests arrive while earlier ones run
        eng.wait_all()
        for t, a in zip(tickets, alone):
            r = eng.poll(t)
            assert r is not None
            assert r.iters == a.iters and r.status == a.status
            np.testing.assert_array_equal(r.x, a.x)
            np.testing.assert_array_equal(r.y, a.y)
    finally:
        eng.close()


def test_serving_cancel_and_unknown_ticket():
    eng = P.BatchEngine(chunk_iters=5)
    try:
        p = W.lasso(500, 200, 31)
        t = eng.submit(p, P.default_params(max_iter=100000, eps_abs=0.0, eps_rel=0.0))
        eng.cancel(t)
        eng.wait_all()
        r = eng.poll(t)
        assert r.status == P.POGS_CANCELLED
        with pytest.raises(KeyError):
            eng.poll(t)
        with pytest.raises(P.PogsError) as ei:
            eng.cancel(999999)
        assert ei.value.code == P.POGS_ENOTFOUND
    finally:
        eng.close()


def test_serving_budget_refusal():
    # the engine's own descriptor and work-list arrays do not fit 1 MiB: refused
    with pytest.raises(P.PogsError) as ei:
        P.BatchEngine(hbm_budget_bytes=1 << 20)
    assert ei.value.code == P.POGS_EAGAIN
    # a request larger than the whole budget is refused at submit
    eng = P.BatchEngine(hbm_budget_bytes=64 << 20)
    try:
        with pytest.raises(P.PogsError) as ei:
            eng.submit(W.lasso(8000, 2000, 51))
        assert ei.value.code == P.POGS_EAGAIN
        # and a small one is accepted and solved
        t = eng.submit(W.lasso(200, 50, 52))
        eng.wait_all()
        assert eng.poll(t).converged
    finally:
        eng.close()


def test_serving_large_request_overlaps():
    eng = P.BatchEngine(chunk_iters=20)
    try:
        big = W.lasso(4000, 2500, 41)
        small = _mix(4, seed=42)
        tb = eng.submit(big)
        ts = [eng.submit(p) for p in small]
        eng.wait_all()
        rb = eng.poll(tb)
        ref = _oracle(big)
        assert rb.converged and abs(rb.optval - ref.optval) <= 1e-3 * max(abs(ref.optval), 1.0)
        for t in ts:
            assert eng.poll(t).converged
    finally:
        eng.close()


def test_uploads_after_a_serving_engine_is_gone():
    """Host uploads of 64 KB and more go through a pinned ring shared by the
    whole process; after a serving engine that ran grouped and whole-GPU
    requests (its threads and streams now destroyed), new contexts and batches
    from host matrices still upload correctly."""
    big = W.lasso(5000, 4000, 43)  # m n > 16 Mi: the whole-GPU path
    small = _mix(6, seed=44)
    eng = P.BatchEngine(chunk_iters=20)
    try:
        ts = [eng.submit(big)] + [eng.submit(p) for p in small]
        eng.wait_all()
        served = [eng.poll(t) for t in ts]
    finally:
        eng.close()
    assert all(r.converged for r in served)
    with P.Context(big.A) as ctx:
        r = ctx.solve(big.f, big.g)
    assert r.converged and r.iters == served[0].iters and r.optval == served[0].optval
    again = P.pogs_solve_batch(small)
    for a, b in zip(again, served[1:]):
        assert a.iters == b.iters and a.optval == b.optval


def _pad_rows(A, pad):
    big = np.zeros((A.shape[0], A.shape[1] + pad), dtype=A.dtype)
    big[:, :A.shape[1]] = A
    return big[:, :A.shape[1]]


def _pad_cols(A, pad):
    big = np.zeros((A.shape[0] + pad, A.shape[1]), dtype=A.dtype, order="F")
    big[:A.shape[0]] = A
    return big[:A.shape[0]]


def test_serving_submit_copies_layouts_and_rejects_non_finite():
    """pogs_batch_submit keeps its own row-major copy of the request (from
    row-major or column-major input, padded or not; 1.35 M entries take the
    threaded copy) and rejects non-finite entries anywhere."""
    import dataclasses
    p = W.lasso(1500, 900, 45)
    variants = [p, dataclasses.replace(p, A=_pad_rows(p.A, 13)), dataclasses.replace(p, A=np.asfortranarray(p.A)),
                dataclasses.replace(p, A=_pad_cols(p.A, 7))]
    small = W.lasso(50, 20, 46)
    eng = P.BatchEngine(chunk_iters=20)
    try:
        ts = [eng.submit(v) for v in variants]
        eng.wait_all()
        rs = [eng.poll(t) for t in ts]
        for q, at, val in ((p, (0, 0), np.nan), (p, (1499, 899), np.inf), (p, (700, 3), -np.inf),
                           (small, (3, 4), np.nan)):
            for layout in (np.ascontiguousarray, np.asfortranarray):
                A = layout(q.A.copy())
                A[at] = val
                with pytest.raises(P.PogsError) as ei:
                    eng.submit(dataclasses.replace(q, A=A))
                assert ei.value.code == P.POGS_EINVAL
    finally:
        eng.close()
    assert rs[0].converged
    for r in rs[1:]:
        assert r.iters == rs[0].iters and r.optval == rs[0].optval
        np.testing.assert_array_equal(r.x, rs[0].x)


def test_serving_budget_counts_whole_gpu_requests():
    """Whole-GPU requests are charged their device memory while they run: with
    a budget that holds one of them at a time, two such requests (and small
    grouped ones) still all finish, each with the result it has alone."""
    big = [W.lasso(5000, 4000, 71), W.nnls_from(W.lasso(4500, 4000, 72))]  # m n > 16 Mi: whole-GPU path
    small = _mix(3, seed=73)
    alone = []
    for p in big:
        with P.Context(p.A) as ctx:
            alone.append(ctx.solve(p.f, p.g))
    eng = P.BatchEngine(hbm_budget_bytes=600 << 20, chunk_iters=20)
    try:
        ts = [eng.submit(p) for p in big]
        tsmall = [eng.submit(p) for p in small]
        eng.wait_all()
        served = [eng.poll(t) for t in ts]
        rsmall = [eng.poll(t) for t in tsmall]
    finally:
        eng.close()
    for s, a in zip(served, alone):
        assert s.status == a.status == P.POGS_CONVERGED and s.error == 0
        assert s.iters == a.iters and s.optval == a.optval
        np.testing.assert_array_equal(s.x, a.x)
    assert all(r.converged for r in rsmall)
