"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (stated per result):
  * prox, float64: relative 1e-12; float32: |gpu - ref| <= 1e-5 max(1, |ref|),
    with the oracle evaluated on the same float32-rounded inputs.
  * equilibration D, E: relative 1e-10 (both sides accumulate in float64
    from the same matrix; only summation order differs).
  * projection: float64 relative 1e-10; float32 ||v - v*|| <= 1e-5 ||v*||.
  * solves: objective |p - p_oracle| <= 1e-3 max(|p_oracle|, 1); the returned
    tuple's residuals (recomputed in float64 on the host) below the
    tolerances, with slack 1.05 for the float32 rounding of the returned vectors.
"""
import math
import zlib

import numpy as np
import pytest

from oracle import pogs_oracle as O
from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu

FLT_EPS = float(np.finfo(np.float32).eps)
DBL_EPS = float(np.finfo(np.float64).eps)


def _eps_cmp(dt):
    return FLT_EPS if dt == np.float32 else DBL_EPS


def _oracle_params(prob, dt, **kw):
    return O.Params(eps_abs=prob.eps_abs, eps_rel=prob.eps_rel, max_iter=prob.max_iter,
                    eps_cmp=_eps_cmp(dt), **kw)


def _residuals(prob, D, E, r):
    """Residuals of the returned (original-variable) tuple in the scaled space:
    ||D (A x - y)|| and ||E (A^T nu + mu)||, recomputed in float64."""
    A = prob.A.astype(np.float64)
    x, y, mu, nu = (v.astype(np.float64) for v in (r.x, r.y, r.mu, r.nu))
    rp = np.linalg.norm(D * (A @ x - y))
    rd = np.linalg.norm(E * (A.T @ nu + mu))
    return rp, rd


# ---------------------------------------------------------------------------
# prox
# ---------------------------------------------------------------------------
H_ALL = list(P.H_CODES)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("h", H_ALL)
def test_prox_parity(h, dt):
    rng = np.random.default_rng(zlib.crc32(h.encode()))
    N = 1537  # several blocks and a ragged tail
    a = rng.choice([-1.0, 1.0], N) * rng.uniform(0.3, 3.0, N)
    b = rng.normal(0, 1, N)
    c = rng.uniform(0.1, 3.0, N)
    c[::17] = 0.0
    d = rng.normal(0, 1, N)
    e = np.where(rng.random(N) < 0.5, 0.0, rng.uniform(0.1, 2.0, N))
    v = rng.normal(0, 3, N)
    rho = 1.3
    # both sides see the same rounded inputs
    a, b, c, d, e, v = (x.astype(dt).astype(np.float64) for x in (a, b, c, d, e, v))
    F = W.Fn(h, N, a=a, b=b, c=c, d=d, e=e)
    got = P.pogs_prox(F, v.astype(dt), rho).astype(np.float64)
    ref = O.prox_param(F, v, rho)
    if dt == np.float64:
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    else:
        err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
        assert err.max() <= 1e-5, (h, err.max(), int(err.argmax()))


def test_prox_empty_and_single():
    F = W.Fn("abs", 1, c=0.5)
    out = P.pogs_prox(F, np.array([2.0]), 1.0)
    assert abs(out[0] - 1.5) < 1e-15


# ---------------------------------------------------------------------------
# setup: equilibration and projection
# ---------------------------------------------------------------------------
SHAPES = [(300, 70), (70, 300), (257, 129), (1, 1), (513, 1), (1, 600), (128, 128)]


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape", SHAPES)
def test_equilibration_parity(shape, dt):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    A = (rng.normal(size=shape) * rng.uniform(0.1, 10, size=(shape[0], 1))).astype(dt)
    with P.Context(A) as ctx:
        D, E = ctx.scaling()
    Dr, Er = O.equilibrate(A.astype(np.float64), _eps_cmp(dt), 10)
    np.testing.assert_allclose(D, Dr, rtol=1e-10)
    np.testing.assert_allclose(E, Er, rtol=1e-10)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape", SHAPES)
def test_projection_parity(shape, dt):
    rng = np.random.default_rng(shape[0] * 3 + shape[1])
    m, n = shape
    A = rng.normal(size=shape).astype(dt)
    c = rng.normal(size=n).astype(dt)
    d = rng.normal(size=m).astype(dt)
    with P.Context(A) as ctx:
        D, E = ctx.scaling()
        x, y = ctx.project(c, d)
    Ah = D[:, None] * A.astype(np.float64) * E[None, :]
    if dt == np.float32:
        Ah = Ah.astype(np.float32).astype(np.float64)  # the matrix the GPU iterates with
    xr, yr = O.Projector(Ah)(c.astype(np.float64), d.astype(np.float64))
    tol = 1e-10 if dt == np.float64 else 1e-5
    assert np.linalg.norm(x - xr) <= tol * max(np.linalg.norm(xr), 1e-30), (shape, dt)
    assert np.linalg.norm(y - yr) <= tol * max(np.linalg.norm(yr), 1e-30), (shape, dt)


def test_column_major_and_device_input():
    import torch
    rng = np.random.default_rng(8)
    A = rng.normal(size=(200, 90)).astype(np.float32)
    with P.Context(A) as c1:
        D1, E1 = c1.scaling()
    with P.Context(np.asfortranarray(A)) as c2:
        D2, E2 = c2.scaling()
    At = torch.from_numpy(A).cuda()
    with P.Context(At) as c3:
        D3, E3 = c3.scaling()
    np.testing.assert_array_equal(D1, D2)
    np.testing.assert_array_equal(E1, E2)
    np.testing.assert_array_equal(D1, D3)
    np.testing.assert_array_equal(E1, E3)


def test_non_finite_matrix_rejected():
    A = np.ones((10, 5), np.float32)
    A[3, 2] = np.nan
    with pytest.raises(P.PogsError) as ei:
        P.Context(A)
    assert ei.value.code == P.POGS_EINVAL


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

def _check_solve(prob, dt, rtol_obj=1e-3, params=None):
    A = prob.A.astype(dt)
    prm = params or P.default_params(eps_abs=prob.eps_abs, eps_rel=prob.eps_rel, max_iter=prob.max_iter)
    with P.Context(A, prm) as ctx:
        r = ctx.solve(prob.f, prob.g, prm)
        D, E = ctx.scaling()
    ref = O.solve(A.astype(np.float64), prob.f, prob.g, _oracle_params(prob, dt))
    assert r.status == P.POGS_CONVERGED, r
    assert ref.converged
    tol = rtol_obj * max(abs(ref.optval), 1.0)
    assert abs(r.optval - ref.optval) <= tol, (prob.name, r.optval, ref.optval, r.iters, ref.iters)
    rp, rd = _residuals(W.Problem(prob.name, A, prob.f, prob.g), D, E, r)
    assert rp <= 1.05 * r.eps_pri + 1e-6 and rd <= 1.05 * r.eps_dual + 1e-6, (rp, r.eps_pri, rd, r.eps_dual)
    return r, ref


def test_small_lasso_f64_matches_oracle_iteration_for_iteration():
    """Lasso 200 x 100 in float64 (at most 2000 iterations): same stop
    iteration and objective to 1e-9 relative."""
    prob = W.lasso_small_f64()
    r, ref = _check_solve(prob, np.float64)
    assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    assert abs(r.optval - ref.optval) <= 1e-9 * abs(ref.optval)
    np.testing.assert_allclose(r.x, ref.x, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("kind,shape", [
    ("lasso", (300, 120)), ("lasso", (120, 300)), ("nnls", (400, 90)), ("logistic", (500, 60)),
    ("svm", (400, 30)), ("lp", (150, 40)), ("dose", (800, 50)), ("lasso", (257, 257)),
    ("basis_pursuit", (300, 120)), ("basis_pursuit", (120, 300)), ("entropy_max", (40, 300)),
    ("huber_fit", (500, 60)), ("portfolio", (10, 400)),
])
def test_solve_classes(kind, shape, dt):
    m, n = shape
    seed = m + 3 * n
    prob = {
        "lasso": lambda: W.lasso(m, n, seed, dtype=dt),
        "nnls": lambda: W.nnls_from(W.lasso(m, n, seed, dtype=dt)),
        "logistic": lambda: W.logistic(m, n, seed, dtype=dt),
        "svm": lambda: W.svm(m, n, seed, dtype=dt),
        "lp": lambda: W.lp(m, n, seed, dtype=dt),
        "dose": lambda: W.dose(m, n, seed, dtype=dt),
        "basis_pursuit": lambda: W.basis_pursuit(m, n, seed, dtype=dt),
        "entropy_max": lambda: W.entropy_max(m, n, seed, dtype=dt),
        "huber_fit": lambda: W.huber_fit(m, n, seed, dtype=dt),
        "portfolio": lambda: W.portfolio(m, n, seed, dtype=dt),
    }[kind]()
    _check_solve(prob, dt)


@pytest.mark.parametrize("adaptive", [1, 0])
@pytest.mark.parametrize("cap", [7, 8])
def test_maxiter_status_and_repeat_solves(cap, adaptive):
    """The tuple returned at the iteration cap is that iteration's half step,
    for an odd and an even cap (the tall float32 iteration keeps consecutive
    half steps in alternating buffers), with Algorithm 3 on and off."""
    prob = W.lasso(300, 100, 5)
    prm = P.default_params(max_iter=cap, chunk_iters=3, adaptive_rho=adaptive)
    with P.Context(prob.A, prm) as ctx:
        r = ctx.solve(prob.f, prob.g, prm)
        assert r.status == P.POGS_MAXITER and r.iters == cap
        ref = O.solve(prob.A.astype(np.float64), prob.f, prob.g,
                      O.Params(max_iter=cap, eps_cmp=FLT_EPS, adaptive_rho=bool(adaptive)))
        np.testing.assert_allclose(r.x, ref.x, rtol=1e-4, atol=1e-5)
        np.testing.assert_allclose(r.nu, ref.nu, rtol=1e-4, atol=1e-5)
        # a second solve on the same context starts from zero again
        r2 = ctx.solve(prob.f, prob.g, prm)
        np.testing.assert_array_equal(r.x, r2.x)
        full = ctx.solve(prob.f, prob.g, P.default_params())
        assert full.converged


def test_solve_is_deterministic():
    prob = W.lasso(2000, 300, 9)
    with P.Context(prob.A) as ctx:
        r1 = ctx.solve(prob.f, prob.g)
        r2 = ctx.solve(prob.f, prob.g)
    assert r1.iters == r2.iters
    np.testing.assert_array_equal(r1.x, r2.x)
    np.testing.assert_array_equal(r1.nu, r2.nu)


@pytest.mark.parametrize("m,n", [(5000, 700), (1100, 1000)])
def test_tall_gram_float32_accuracy(m, n):
    """The tall float32 Gram (bf16 pieces, six products per float32 product)
    gives the projection float32 accuracy: against the exact FP64 projection of
    the float32 A^ the device holds, within 1e-6 relative -- a Gram that kept
    only five piece products (error 2^-16 of an entry) or lost a piece misses
    this.  Shapes span several 128-wide tiles with ragged edges and several
    row splits."""
    import torch
    rng = np.random.default_rng(m + n)
    A = rng.normal(size=(m, n)).astype(np.float32)
    c = rng.normal(size=n).astype(np.float32)
    d = rng.normal(size=m).astype(np.float32)
    with P.Context(torch.from_numpy(A).cuda()) as ctx:
        D, E = ctx.scaling()
        x, y = ctx.project(c, d)
    Ah = (D[:, None] * A.astype(np.float64) * E[None, :]).astype(np.float32).astype(np.float64)
    xr, yr = O.Projector(Ah)(c.astype(np.float64), d.astype(np.float64))
    ex = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    ey = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    print(f"{m}x{n} projection: rel err x {ex:.3e} y {ey:.3e}")
    assert ex <= 1e-6 and ey <= 1e-6, (ex, ey)


def test_direct_chunks_do_not_change_the_solve():
    """A problem large enough (m n >= 16 Mi) that chunks are launched directly,
    with one iteration of the next chunk queued behind each control read-back:
    the stop test runs on the device, so the chunk length changes neither the
    stopping iteration nor a bit of the result -- whether the solve stops in
    the middle of a chunk or at its end (after which the queued iteration must
    change nothing)."""
    import torch
    prob = W.lasso(8192, 2048, 33)
    A = torch.from_numpy(prob.A).cuda()
    res = {}
    with P.Context(A) as ctx:
        for chunk in (20, 6, 2):
            prm = P.default_params(eps_abs=prob.eps_abs, eps_rel=prob.eps_rel, max_iter=prob.max_iter,
                                   chunk_iters=chunk)
            res[chunk] = ctx.solve(prob.f, prob.g, prm)
    r20 = res[20]
    assert r20.converged
    for chunk in (6, 2):
        r = res[chunk]
        assert r.iters == r20.iters, (chunk, r.iters, r20.iters)
        np.testing.assert_array_equal(r.x, r20.x)
        np.testing.assert_array_equal(r.nu, r20.nu)
        assert r.optval == r20.optval


# ---------------------------------------------------------------------------
# full-size workload (Lasso and NNLS on 20000 x 2000, float32)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def big():
    return W.lasso_20000x2000()


def test_big_setup_and_projection(big):
    import torch
    A = torch.from_numpy(big.A).cuda()
    rng = np.random.default_rng(1)
    c = rng.normal(size=big.n).astype(np.float32)
    d = rng.normal(size=big.m).astype(np.float32)
    with P.Context(A) as ctx:
        D, E = ctx.scaling()
        x, y = ctx.project(c, d)
    Dr, Er = O.equilibrate(big.A.astype(np.float64), FLT_EPS, 10)
    np.testing.assert_allclose(D, Dr, rtol=1e-10)
    np.testing.assert_allclose(E, Er, rtol=1e-10)
    # sampled rows of y = A^ x, recomputed in float64 from the float32 A^ the device holds
    Ah = (D[:, None] * big.A.astype(np.float64) * E[None, :]).astype(np.float32).astype(np.float64)
    rows = rng.choice(big.m, 500, replace=False)
    np.testing.assert_allclose(y[rows], Ah[rows] @ x.astype(np.float64), rtol=1e-5, atol=1e-5)
    # full projection against the oracle
    xr, yr = O.Projector(Ah)(c.astype(np.float64), d.astype(np.float64))
    # optimality of the returned pair: x - c + A^T (y - d) = 0 with y = A^ x
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    kkt = np.linalg.norm(x64 - c + Ah.T @ (y64 - d)) / np.linalg.norm(c)
    print(f"20000x2000 projection: rel err x {np.linalg.norm(x - xr) / np.linalg.norm(xr):.3e} "
          f"y {np.linalg.norm(y - yr) / np.linalg.norm(yr):.3e}; ||x - c + A^T(y - d)||/||c|| {kkt:.3e}")
    # float32 accuracy of the Gram over its row splits (9.7e-8 measured with
    # 2900-row splits; one accumulator for all six bf16 piece products over
    # 4000-row splits gave 1.1e-6)
    assert np.linalg.norm(x - xr) <= 5e-7 * np.linalg.norm(xr)
    assert np.linalg.norm(y - yr) <= 5e-7 * np.linalg.norm(yr)


@pytest.mark.parametrize("kind", ["lasso", "nnls"])
def test_big_solve(big, kind):
    prob = big if kind == "lasso" else W.nnls_from(big)
    _check_solve(prob, np.float32)


@pytest.mark.parametrize("shape", [(3000, 700), (700, 3000)])
def test_autotuned_load_policy_changes_no_bit(shape):
    """The tuner picks only the load policy of the passes (cached or
    non-temporal), so a solve gives the same bits with and without it."""
    prob = W.lasso(*shape, seed=sum(shape))
    out = []
    for tune in (0, 1):
        prm = P.default_params(autotune=tune)
        with P.Context(prob.A, prm) as ctx:
            r = ctx.solve(prob.f, prob.g, prm)
        out.append(r)
    assert out[0].iters == out[1].iters
    np.testing.assert_array_equal(out[0].x, out[1].x)
    np.testing.assert_array_equal(out[0].nu, out[1].nu)
    assert out[0].optval == out[1].optval
