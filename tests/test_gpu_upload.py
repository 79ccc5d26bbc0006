"""GPU tests of host-matrix uploads of 8 MB and more, which go through the
pinned-ring uploader (chunks of 16 MB, four of them in a ring, so a 75 MB
matrix reuses every chunk and ends on a partial one).  The device copy must
hold the host data bit for bit: solves from a contiguous host matrix, from a
row-major or column-major host matrix with a padded leading dimension, and
from the same matrix already on the device agree bit for bit (same kernels,
same geometry, fixed-order sums)."""
import dataclasses

import numpy as np
import pytest

from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu

M, N = 9000, 2100  # 75.6 MB of float32


@pytest.fixture(scope="module")
def prob():
    return W.lasso(M, N, seed=31)


def _padded_rows(A, pad):
    big = np.zeros((A.shape[0], A.shape[1] + pad), dtype=A.dtype)
    big[:, :A.shape[1]] = A
    return big[:, :A.shape[1]]


def _padded_cols(A, pad):
    big = np.zeros((A.shape[0] + pad, A.shape[1]), dtype=A.dtype, order="F")
    big[:A.shape[0]] = A
    return big[:A.shape[0]]


def _same(r1, r2):
    assert r1.iters == r2.iters and r1.status == r2.status
    assert r1.optval == r2.optval
    for a, b in ((r1.x, r2.x), (r1.y, r2.y), (r1.nu, r2.nu)):
        np.testing.assert_array_equal(np.asarray(a), np.asarray(b))


def test_host_layouts_are_passed_through(prob):
    A = prob.A
    assert P._host_layout(_padded_rows(A, 37))[1:] == (P.POGS_ROW_MAJOR, N + 37)
    assert P._host_layout(_padded_cols(A, 41))[1:] == (P.POGS_COL_MAJOR, M + 41)


def test_init_from_large_host_matrix_matches_device(prob):
    import torch
    out = []
    for A in (prob.A, _padded_rows(prob.A, 37), _padded_cols(prob.A, 41),
              torch.from_numpy(prob.A).cuda()):
        with P.Context(A) as ctx:
            D, E = ctx.scaling()
            r = ctx.solve(prob.f, prob.g)
        out.append((D, E, r))
    D0, E0, r0 = out[0]
    assert r0.converged
    for D, E, r in out[1:]:
        np.testing.assert_array_equal(D, D0)
        np.testing.assert_array_equal(E, E0)
        _same(r, r0)


def test_batch_from_padded_host_matrices(prob):
    probs = [prob, dataclasses.replace(prob, A=_padded_rows(prob.A, 37)),
             dataclasses.replace(prob, A=_padded_cols(prob.A, 41))]
    res = P.pogs_solve_batch(probs)
    assert res[0].converged
    _same(res[1], res[0])
    _same(res[2], res[0])
