"""GPU tests of sparse A (compressed rows, pogs_init_sparse) with the CGLS
projection, through the C ABI, against the FP64 oracle on the same matrix
(densified: the method does not depend on the storage).

Tolerances: D, E relative 1e-10 (both sides accumulate in float64 from the
same values); objective |p - p_oracle| <= 1e-3 max(|p_oracle|, 1); float64
runs stop within one iteration of the oracle's.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import pogs_oracle as O
from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = {np.float32: float(np.finfo(np.float32).eps), np.float64: float(np.finfo(np.float64).eps)}


def _dense(A):
    return np.asarray(A.toarray(), dtype=np.float64)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape,k,seg", [((500, 120), 6, 0), ((120, 400), 30, 0), ((3000, 700), 40, 0),
                                         ((500, 120), 6, 37), ((3000, 700), 40, 256)])
def test_sparse_equilibration_parity(shape, k, seg, dt):
    """seg > 0: A^T stored in column segments of seg columns (ragged last one)."""
    p = W.sparse_problem("lasso", *shape, k, seed=shape[0] + k, dtype=dt)
    with P.SparseContext(p.A, P.default_params(sparse_segment=seg)) as ctx:
        D, E = ctx.scaling()
    Dr, Er = O.equilibrate(_dense(p.A), EPS[dt], 10)
    np.testing.assert_allclose(D, Dr, rtol=1e-10)
    np.testing.assert_allclose(E, Er, rtol=1e-10)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("kind,shape,k", [
    ("lasso", (600, 150), 10), ("lasso", (150, 500), 40), ("nnls", (500, 100), 8),
    ("logistic", (800, 120), 12), ("lp", (200, 60), 10), ("lasso", (5000, 1200), 3),
])
def test_sparse_solve_matches_oracle(kind, shape, k, dt):
    p = W.sparse_problem(kind, *shape, k, seed=7 * shape[0] + k, dtype=dt)
    with P.SparseContext(p.A) as ctx:
        r = ctx.solve(p.f, p.g)
    ref = O.solve(_dense(p.A), p.f, p.g, O.Params(eps_cmp=EPS[dt], projection="cgls"))
    assert ref.converged and r.status == P.POGS_CONVERGED, (r, ref.iters)
    tol = 1e-3 * max(abs(ref.optval), 1.0)
    assert abs(r.optval - ref.optval) <= tol, (r.optval, ref.optval, r.iters, ref.iters)
    if dt == np.float64:
        assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    print(f"{kind} {shape} k={k} {np.dtype(dt).name}: iters {r.iters} (oracle {ref.iters}), "
          f"CG steps {r.cg_steps} (oracle {ref.cg_steps})")


@pytest.mark.parametrize("seg", [0, 50])
def test_sparse_with_empty_rows_and_columns(seg):
    """Rows and columns without entries (a zero row of A, an unused variable);
    with seg = 50 whole segments of some rows of A^T are empty."""
    rng = np.random.default_rng(3)
    A = W.sparse_matrix(300, 90, 5, rng, np.float64).tolil()
    A[17, :] = 0.0
    A[200:210, :] = 0.0
    A[:, 40] = 0.0
    A = A.tocsr()
    A.eliminate_zeros()
    b = rng.normal(size=300)
    f = W.Fn("square", 300, b=b)
    g = W.Fn("abs", 90, c=0.05)
    with P.SparseContext(A, P.default_params(sparse_segment=seg)) as ctx:
        r = ctx.solve(f, g)
    ref = O.solve(_dense(A), f, g, O.Params(eps_cmp=EPS[np.float64], projection="cgls"))
    assert r.converged and ref.converged
    assert abs(r.optval - ref.optval) <= 1e-3 * max(1.0, abs(ref.optval))
    assert abs(r.x[40]) < 1e-8  # unused variable under an l1 penalty stays at 0


def test_sparse_matches_dense_cgls_on_gpu():
    p = W.sparse_problem("lasso", 2000, 500, 20, seed=11)
    with P.SparseContext(p.A) as ctx:
        rs = ctx.solve(p.f, p.g)
    with P.Context(np.ascontiguousarray(p.A.toarray()), P.default_params(projection="cgls")) as ctx:
        rd = ctx.solve(p.f, p.g, P.default_params(projection="cgls"))
    assert rs.converged and rd.converged
    assert abs(rs.optval - rd.optval) <= 1e-3 * max(1.0, abs(rd.optval))
    assert abs(rs.iters - rd.iters) <= max(2, rd.iters // 20), (rs.iters, rd.iters)


def test_sparse_device_input_and_rejections():
    import torch
    p = W.sparse_problem("lasso", 400, 100, 8, seed=12)
    A = p.A
    At = torch.sparse_csr_tensor(torch.from_numpy(A.indptr.astype(np.int64)), torch.from_numpy(A.indices.astype(np.int32)),
                                 torch.from_numpy(A.data), size=A.shape, device="cuda")
    with P.SparseContext(A) as c_host, P.SparseContext(At) as c_dev:
        r1 = c_host.solve(p.f, p.g)
        r2 = c_dev.solve(p.f, p.g)
        assert r1.converged and r2.converged
        assert r1.iters == r2.iters and abs(r1.optval - r2.optval) <= 1e-12 * max(1.0, abs(r1.optval))
        for call in (lambda: c_host.solve(p.f, p.g, P.default_params(stop_rule="gap")),
                     lambda: c_host.project(np.zeros(100, np.float32), np.zeros(400, np.float32)),
                     lambda: c_host.solve_path([p.f], [p.g])):
            with pytest.raises(P.PogsError) as ei:
                call()
            assert ei.value.code == P.POGS_EUNSUPPORTED


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape,k", [((700, 160), 9), ((160, 600), 40)])
def test_sparse_warm_start_matches_oracle(shape, k, dt):
    """Warm start from a perturbed point (x0, nu0) on the sparse pair against
    the oracle's warm start on the densified matrix."""
    p = W.sparse_problem("lasso", *shape, k, seed=5 * shape[0] + k, dtype=dt)
    m, n = shape
    rng = np.random.default_rng(m + n)
    x0 = (0.1 * rng.normal(size=n)).astype(dt)
    nu0 = (0.1 * rng.normal(size=m)).astype(dt)
    with P.SparseContext(p.A) as ctx:
        r = ctx.solve(p.f, p.g, x0=x0, nu0=nu0)
    ref = O.solve(_dense(p.A), p.f, p.g, O.Params(eps_cmp=EPS[dt], projection="cgls"),
                  x0=x0.astype(np.float64), nu0=nu0.astype(np.float64))
    assert ref.converged and r.status == P.POGS_CONVERGED, (r, ref.iters)
    assert abs(r.optval - ref.optval) <= 1e-3 * max(abs(ref.optval), 1.0), (r.optval, ref.optval)
    if dt == np.float64:
        assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)


def test_sparse_warm_start_from_optimum_and_device_input():
    """From a converged solution the warm state is a fixed point up to the CG
    tolerance; device-resident (x0, nu0) give the same solve as host ones."""
    import torch
    p = W.sparse_problem("lasso", 1200, 300, 12, seed=21, dtype=np.float64)
    prm = P.default_params(eps_abs=1e-6, eps_rel=1e-6)
    with P.SparseContext(p.A, prm) as ctx:
        r0 = ctx.solve(p.f, p.g, prm)
        r1 = ctx.solve(p.f, p.g, x0=r0.x, nu0=r0.nu)
        r2 = ctx.solve(p.f, p.g, device_out=True, x0=torch.from_numpy(r0.x), nu0=torch.from_numpy(r0.nu))
    assert r0.converged and r1.converged
    assert r1.iters <= 3, r1.iters
    assert abs(r1.optval - r0.optval) <= 1e-4 * max(1.0, abs(r0.optval))
    assert r2.iters == r1.iters and abs(r2.optval - r1.optval) <= 1e-12 * max(1.0, abs(r1.optval))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("kind,shape,k,seg", [
    ("lasso", (600, 150), 10, 64), ("lasso", (150, 500), 40, 16), ("logistic", (800, 120), 12, 100),
    ("lp", (200, 60), 10, 7),
])
def test_sparse_segmented_matches_oracle(kind, shape, k, seg, dt):
    """The passes over A^T in column segments (many, ragged last one) follow
    the oracle as the single-segment copy does."""
    p = W.sparse_problem(kind, *shape, k, seed=11 * shape[0] + k, dtype=dt)
    with P.SparseContext(p.A, P.default_params(sparse_segment=seg)) as ctx:
        r = ctx.solve(p.f, p.g)
    ref = O.solve(_dense(p.A), p.f, p.g, O.Params(eps_cmp=EPS[dt], projection="cgls"))
    assert ref.converged and r.status == P.POGS_CONVERGED, (r, ref.iters)
    assert abs(r.optval - ref.optval) <= 1e-3 * max(abs(ref.optval), 1.0), (r.optval, ref.optval)
    if dt == np.float64:
        assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)


def test_sparse_segments_change_only_the_summation_order():
    """float64: one segment against 9 segments on the same matrix: the scaling
    agrees to rounding, the solve takes the same path."""
    p = W.sparse_problem("lasso", 2000, 300, 12, seed=17, dtype=np.float64)
    out = []
    for seg in (2000, 223):
        prm = P.default_params(sparse_segment=seg)
        with P.SparseContext(p.A, prm) as ctx:
            D, E = ctx.scaling()
            r = ctx.solve(p.f, p.g)
            w = ctx.solve(p.f, p.g, x0=r.x, nu0=r.nu)
        out.append((D, E, r, w))
    (D1, E1, r1, w1), (D9, E9, r9, w9) = out
    np.testing.assert_allclose(D9, D1, rtol=1e-13)
    np.testing.assert_allclose(E9, E1, rtol=1e-13)
    assert abs(r9.iters - r1.iters) <= 1 and r9.cg_steps > 0
    assert abs(r9.optval - r1.optval) <= 1e-8 * max(1.0, abs(r1.optval))
    assert w1.iters <= 3 and w9.iters <= 3


def test_sparse_automatic_segments_at_size_match_dense_cgls():
    """float32, m = 300000 (three automatic segments of 131072 columns of A^T)
    against the dense CGLS path on the same matrix."""
    p = W.sparse_problem("lasso", 300_000, 1000, 8, seed=23)
    with P.SparseContext(p.A) as ctx:
        rs = ctx.solve(p.f, p.g)
    prm = P.default_params(projection="cgls")
    with P.Context(np.ascontiguousarray(p.A.toarray()), prm) as ctx:
        rd = ctx.solve(p.f, p.g, prm)
    assert rs.converged and rd.converged
    assert abs(rs.optval - rd.optval) <= 1e-3 * max(1.0, abs(rd.optval))
    assert abs(rs.iters - rd.iters) <= max(2, rd.iters // 20), (rs.iters, rd.iters)
