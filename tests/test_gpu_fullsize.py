"""GPU parity at the full sizes of the benchmark workloads and on the kernel
variants that only large shapes select.

* Grouped (batched / served) kernels with 64 lanes per row: the grouped pass
  over rows, the wide pass 1 and the solve switch from 16 to 64 lanes per row
  when the padded row (n, or min(m, n) for the solve) reaches 512 elements;
  problems with n, min(m, n) >= 449, tall and wide, are compared with the
  FP64 oracle and bitwise with the same problem alone.
* The serving engine on every kind of the mixed request stream (Lasso, NNLS,
  hinge-loss SVM, box LP; Appendix A.4, A.6, A.7, A.9).
* The dose-shaped 100000 x 1000 problem (Section 6.2 shape): equilibration and
  projection against the oracle at full size, and the whole solve against the
  stored FP64-oracle objective (tests/golden/, written by make_golden.py from
  the oracle only).
* The 512-problem batch and the 64-point lambda path at full size against the
  stored oracle objectives; on the path, the solutions x of three lambdas
  against the oracle's and against the same problems solved alone, and the
  critical lambda's x = 0 (Appendix A.4).

Tolerances: objectives |p - p_oracle| <= 1e-3 max(|p_oracle|, 1); projection
||v - v*|| <= 1e-5 ||v*||; equilibration relative 1e-10; alone vs mix bitwise.
Path solutions: ||x - x_ref|| <= 1e-4 ||x_ref|| when both runs take the same
number of iterations: the ADMM map is nonexpansive, so the per-step
difference of the float32 projection (within 5e-7 relative, pinned by the
projection tests) adds up at most linearly over the <= 100 steps.  Runs that
stop at different iterations: 1e-2, since each stops once its residuals are
within eps_rel = 1e-3 (relative), which fixes x to about that accuracy, and
ten times eps_rel leaves room for one iteration's difference.  Entries of
x_ref above 1e-2 max|x_ref| keep their sign (the Lasso solution's support).
"""
import json
import os

import numpy as np
import pytest

from oracle import pogs_oracle as O
from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu
FLT_EPS = float(np.finfo(np.float32).eps)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _oracle(p):
    return O.solve(p.A.astype(np.float64), p.f, p.g,
                   O.Params(eps_abs=p.eps_abs, eps_rel=p.eps_rel, max_iter=p.max_iter, eps_cmp=FLT_EPS))


def _close(got, ref, rtol=1e-3):
    return abs(got - ref) <= rtol * max(abs(ref), 1.0)


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)["results"]


# ---------------------------------------------------------------------------
# grouped kernels with 64 lanes per row
# ---------------------------------------------------------------------------
WIDE_SHAPES = [("lasso", 4096, 1024), ("logistic", 3000, 700), ("lasso", 600, 1000), ("logistic", 700, 900),
               ("lasso", 1024, 1024), ("logistic", 2048, 449), ("lasso", 512, 980), ("logistic", 4000, 512)]


@pytest.fixture(scope="module")
def wide_mix():
    probs = [getattr(W, k)(m, n, seed=m + 7 * n) for k, m, n in WIDE_SHAPES]
    return probs, P.pogs_solve_batch(probs)


def test_grouped_64_lane_variants_match_oracle(wide_mix):
    probs, res = wide_mix
    for p, r in zip(probs, res):
        ref = _oracle(p)
        print(f"{p.name} {p.m}x{p.n}: gpu {r.optval:.8g} ({r.iters} it) oracle {ref.optval:.8g} ({ref.iters} it)")
        assert r.converged and ref.converged, (p.name, p.m, p.n, r)
        assert _close(r.optval, ref.optval), (p.name, p.m, p.n, r.optval, ref.optval)


def test_grouped_64_lane_alone_equals_mix(wide_mix):
    probs, res = wide_mix
    for i in (0, 2, 5, 6):
        alone = P.pogs_solve_batch([probs[i]])[0]
        assert alone.iters == res[i].iters
        np.testing.assert_array_equal(alone.x, res[i].x)
        np.testing.assert_array_equal(alone.nu, res[i].nu)


# ---------------------------------------------------------------------------
# serving engine on every request kind
# ---------------------------------------------------------------------------
def test_serving_every_kind_matches_oracle_and_alone():
    probs = [W.nnls_from(W.lasso(900, 300, 61)), W.svm(1200, 150, 62), W.lp(300, 400, 63),
             W.lasso(2000, 600, 64), W.nnls_from(W.lasso(300, 700, 65)), W.svm(600, 800, 66), W.lp(700, 200, 67)]
    alone = [P.pogs_solve_batch([p])[0] for p in probs]
    eng = P.BatchEngine(chunk_iters=10)
    try:
        tickets = [eng.submit(p) for p in probs]
        eng.wait_all()
        served = [eng.poll(t) for t in tickets]
    finally:
        eng.close()
    for p, s, a in zip(probs, served, alone):
        ref = _oracle(p)
        print(f"{p.name} {p.m}x{p.n}: served {s.optval:.8g} ({s.iters} it) oracle {ref.optval:.8g} ({ref.iters} it)")
        assert s.iters == a.iters and s.status == a.status
        np.testing.assert_array_equal(s.x, a.x)
        np.testing.assert_array_equal(s.nu, a.nu)
        assert ref.converged and s.converged, (p.name, s)
        assert _close(s.optval, ref.optval), (p.name, s.optval, ref.optval)


# ---------------------------------------------------------------------------
# dose-shaped 100000 x 1000 at full size
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def dose():
    return W.dose_100000x1000()


def test_dose_setup_and_projection_full_size(dose):
    import torch
    A = torch.from_numpy(dose.A).cuda()
    rng = np.random.default_rng(2)
    c = rng.normal(size=dose.n).astype(np.float32)
    d = rng.normal(size=dose.m).astype(np.float32)
    with P.Context(A) as ctx:
        D, E = ctx.scaling()
        x, y = ctx.project(c, d)
    Dr, Er = O.equilibrate(dose.A.astype(np.float64), FLT_EPS, 10)
    np.testing.assert_allclose(D, Dr, rtol=1e-10)
    np.testing.assert_allclose(E, Er, rtol=1e-10)
    Ah = (D[:, None] * dose.A.astype(np.float64) * E[None, :]).astype(np.float32).astype(np.float64)
    xr, yr = O.Projector(Ah)(c.astype(np.float64), d.astype(np.float64))
    ex = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    ey = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    # optimality of the returned pair: x - c + A^T (y - d) = 0 with y = A^ x
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    kkt = np.linalg.norm(x64 - c + Ah.T @ (y64 - d)) / np.linalg.norm(c)
    graph = np.linalg.norm(y64 - Ah @ x64) / np.linalg.norm(y64)
    print(f"dose projection: rel err x {ex:.3e} y {ey:.3e}; ||x - c + A^T(y - d)||/||c|| {kkt:.3e}; "
          f"||y - A x||/||y|| {graph:.3e}")
    # float32 accuracy of the Gram over long row splits (1.3e-7 measured)
    assert ex <= 5e-7 and ey <= 5e-7, (ex, ey)


def test_dose_solve_full_size_against_stored_oracle(dose):
    import torch
    (gold,) = _golden("dose_100000x1000.json")
    assert gold["fingerprint"] == W.fingerprint(dose), "stored oracle result is for other inputs"
    A = torch.from_numpy(dose.A).cuda()
    with P.Context(A) as ctx:
        r = ctx.solve(dose.f, dose.g)
    print(f"dose: gpu {r.optval:.8g} ({r.iters} it) oracle {gold['optval']:.8g} ({gold['iters']} it); "
          f"rel err {abs(r.optval - gold['optval']) / abs(gold['optval']):.2e}")
    assert r.converged and gold["converged"]
    assert _close(r.optval, gold["optval"]), (r.optval, gold["optval"])


# ---------------------------------------------------------------------------
# 512-problem batch and 64-point lambda path at full size
# ---------------------------------------------------------------------------
def test_batch_512_against_stored_oracle():
    gold = _golden("batch_mix_512.json")
    probs = W.batch_mix(512)
    for p, g in zip(probs, gold):
        assert g["fingerprint"] == W.fingerprint(p), ("stored oracle result is for other inputs", g["index"])
    res = P.pogs_solve_batch(probs)
    errs = np.array([abs(r.optval - g["optval"]) / max(abs(g["optval"]), 1.0) for r, g in zip(res, gold)])
    print(f"batch 512: max rel objective error {errs.max():.2e} (median {np.median(errs):.2e}); "
          f"converged {sum(r.converged for r in res)}/512")
    assert all(r.converged for r in res)
    assert errs.max() <= 1e-3, (int(errs.argmax()), errs.max())


def test_lambda_path_full_size_against_stored_oracle():
    gold = _golden("lambda_path_8000x1000.json")
    probs = W.lambda_path()
    for p, g in zip(probs, gold):
        assert g["fingerprint"] == W.fingerprint(p)
    with P.Context(probs[0].A) as ctx:
        res = ctx.solve_path([p.f for p in probs], [p.g for p in probs])
    errs = np.array([abs(r.optval - g["optval"]) / max(abs(g["optval"]), 1.0) for r, g in zip(res, gold)])
    print(f"lambda path 64: max rel objective error {errs.max():.2e}; converged {sum(r.converged for r in res)}/64")
    assert all(r.converged for r in res)
    assert errs.max() <= 1e-3, (int(errs.argmax()), errs.max())


def test_lambda_path_full_size_solutions():
    probs = W.lambda_path()
    A = probs[0].A
    pick = (0, 21, 42)
    with P.Context(A) as ctx:
        res = ctx.solve_path([p.f for p in probs], [p.g for p in probs])
        alone = {r: ctx.solve(probs[r].f, probs[r].g) for r in pick}
    A64 = A.astype(np.float64)
    for r in pick:
        ref = O.solve(A64, probs[r].f, probs[r].g, O.Params(eps_cmp=FLT_EPS))
        x, xr, xa = res[r].x.astype(np.float64), ref.x, alone[r].x.astype(np.float64)
        e_or = float(np.linalg.norm(x - xr) / np.linalg.norm(xr))
        e_al = float(np.linalg.norm(x - xa) / np.linalg.norm(xa))
        big = np.abs(xr) > 1e-2 * np.abs(xr).max()
        print(f"lambda {r}: ||x - x_oracle||/||x_oracle|| {e_or:.2e}, vs alone {e_al:.2e}, "
              f"support {int(big.sum())}, iters {res[r].iters}/{ref.iters}")
        assert res[r].converged and res[r].iters <= 100
        assert e_or <= (1e-4 if res[r].iters == ref.iters else 1e-2), (r, e_or)
        assert e_al <= (1e-4 if res[r].iters == alone[r].iters else 1e-2), (r, e_al)
        assert np.all(np.sign(x[big]) == np.sign(xr[big])), r
    # the largest lambda is lambda_max: x* = 0 (Appendix A.4); at the stopping
    # tolerance the iterate is small next to the smallest lambda's
    assert float(np.abs(res[-1].x).max()) <= 1e-2 * float(np.abs(res[0].x).max())
