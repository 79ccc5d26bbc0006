"""Pins for the oracle's equilibration (Section 4.2, Algorithm 2), Frobenius
normalisation (Section 4.1.2) and graph projection (Sections 3.1, 3.5, 4.1.1).
CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import pogs_oracle as O


def _sk_objective(uv, Ap, gamma):
    """The regularised equilibration objective of Section 4.2 and its gradient."""
    m, n = Ap.shape
    u, v = uv[:m], uv[m:]
    W = Ap * np.exp(u[:, None] + v[None, :])
    obj = W.sum() - n * u.sum() - m * v.sum() + gamma * (np.exp(u).sum() / m + np.exp(v).sum() / n)
    gu = W.sum(axis=1) - n + gamma * np.exp(u) / m
    gv = W.sum(axis=0) - m + gamma * np.exp(v) / n
    return obj, np.concatenate([gu, gv])


@pytest.mark.parametrize("shape", [(7, 4), (4, 9), (12, 12)])
def test_sinkhorn_fixed_point_minimises_objective(shape):
    """Many sweeps of Algorithm 2 reach the minimiser of the convex objective
    it descends (found here by L-BFGS on (u, v), no Sinkhorn step involved)."""
    rng = np.random.default_rng(1)
    A = rng.normal(size=shape)
    m, n = shape
    gamma = 0.3
    d, e = O.sinkhorn_knopp(A, gamma, iters=5000)
    res = minimize(_sk_objective, np.zeros(m + n), args=(A ** 2, gamma), jac=True,
                   method="L-BFGS-B", options={"maxiter": 20000, "gtol": 1e-12, "ftol": 1e-15})
    u, v = res.x[:m], res.x[m:]
    np.testing.assert_allclose(d, np.exp(u), rtol=1e-5)
    np.testing.assert_allclose(e, np.exp(v), rtol=1e-5)
    # Section 4.2: at the optimum the average entries of d and e agree
    assert abs(d.mean() - e.mean()) <= 1e-8 * d.mean()


def test_sinkhorn_large_gamma_limit():
    """gamma -> inf drives both scalings to the constant m n / gamma (Section 4.2)."""
    rng = np.random.default_rng(2)
    A = rng.normal(size=(6, 5))
    gamma = 1e9
    d, e = O.sinkhorn_knopp(A, gamma, iters=3)
    np.testing.assert_allclose(d, 30.0 / gamma, rtol=1e-6)
    np.testing.assert_allclose(e, 30.0 / gamma, rtol=1e-6)


def test_sinkhorn_equilibrates_without_regularisation():
    """gamma ~ 0 on a positive matrix: every row of |D A E|^2 sums to n and
    every column to m (the equilibrated conditions of Section 4.2)."""
    rng = np.random.default_rng(3)
    A = rng.uniform(0.5, 2.0, size=(5, 8))
    d, e = O.sinkhorn_knopp(A, 1e-14, iters=3000)
    S = (d[:, None] * A ** 2 * e[None, :])
    np.testing.assert_allclose(S.sum(axis=1), 8.0, rtol=1e-9)
    np.testing.assert_allclose(S.sum(axis=0), 5.0, rtol=1e-9)


def test_sinkhorn_one_sweep_by_hand():
    A = np.array([[1.0, 2.0], [0.0, 3.0], [4.0, 0.5]])
    gamma = 0.5
    d, e = O.sinkhorn_knopp(A, gamma, iters=1)
    # d_i = n / (sum_j A_ij^2 + gamma/m), with e = 1
    d_ref = 2.0 / (np.array([5.0, 9.0, 16.25]) + 0.5 / 3)
    e_ref = 3.0 / (np.array([d_ref[0] * 1 + d_ref[2] * 16, d_ref[0] * 4 + d_ref[1] * 9 + d_ref[2] * 0.25]) + 0.25)
    np.testing.assert_allclose(d, d_ref, rtol=1e-15)
    np.testing.assert_allclose(e, e_ref, rtol=1e-15)


@pytest.mark.parametrize("shape", [(40, 10), (10, 40), (25, 25)])
def test_frobenius_normalisation(shape):
    rng = np.random.default_rng(4)
    A = rng.normal(size=shape) * rng.uniform(0.01, 100, size=(shape[0], 1))
    D, E = O.equilibrate(A, eps_cmp=2.0 ** -23, iters=10)
    Ah = D[:, None] * A * E[None, :]
    assert abs(np.linalg.norm(Ah) / math.sqrt(min(shape)) - 1.0) < 1e-13
    # equilibration narrows the spread of row norms a lot
    rn = np.linalg.norm(Ah, axis=1)
    assert rn.max() / rn.min() < 1.5
    # D and E are scaled by the same factor: ratio of means as Algorithm 2 left it
    d, e = O.sinkhorn_knopp(A, (sum(shape)) * math.sqrt(2.0 ** -23), 10)
    np.testing.assert_allclose(D / np.sqrt(d), (D / np.sqrt(d))[0], rtol=1e-13)
    np.testing.assert_allclose(E / np.sqrt(e), (D / np.sqrt(d))[0], rtol=1e-13)


@pytest.mark.parametrize("shape", [(30, 12), (12, 30), (16, 16), (1, 5), (5, 1)])
def test_projection_is_least_squares(shape):
    """Pi(c, d) = argmin ||x - c||^2 + ||y - d||^2 s.t. y = A x: solved here by a
    least-squares solve of [I; A] x ~ [c; d] (no Cholesky, no reduced update)."""
    rng = np.random.default_rng(5)
    m, n = shape
    A = rng.normal(size=shape)
    c = rng.normal(size=n)
    d = rng.normal(size=m)
    P = O.Projector(A)
    x, y = P(c, d)
    xr, *_ = np.linalg.lstsq(np.vstack([np.eye(n), A]), np.concatenate([c, d]), rcond=None)
    np.testing.assert_allclose(x, xr, rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(y, A @ xr, rtol=1e-10, atol=1e-11)
    # orthogonality: (c - x, d - y) is orthogonal to the graph
    np.testing.assert_allclose((c - x) + A.T @ (d - y), 0.0, atol=1e-10)
    # idempotent
    x2, y2 = P(x, y)
    np.testing.assert_allclose(x2, x, atol=1e-10)
    np.testing.assert_allclose(y2, y, atol=1e-10)


def test_projection_branches_agree():
    """The m >= n and m < n reduced updates are the same projection: apply the
    wide branch to A and the tall branch to the transposed problem."""
    rng = np.random.default_rng(6)
    A = rng.normal(size=(9, 20))
    c, d = rng.normal(size=20), rng.normal(size=9)
    x, y = O.Projector(A)(c, d)
    # graph of A^T with roles swapped: (y, x) with x = A^T y is not the same set,
    # so compare with the explicit KKT system of Section 3.1 instead
    K = np.block([[np.eye(20), A.T], [A, -np.eye(9)]])
    sol = np.linalg.solve(K, np.concatenate([c + A.T @ d, np.zeros(9)]))
    np.testing.assert_allclose(x, sol[:20], atol=1e-11)
    np.testing.assert_allclose(y, sol[20:], atol=1e-11)
    A2 = rng.normal(size=(20, 9))
    c2, d2 = rng.normal(size=9), rng.normal(size=20)
    x2, y2 = O.Projector(A2)(c2, d2)
    K2 = np.block([[np.eye(9), A2.T], [A2, -np.eye(20)]])
    sol2 = np.linalg.solve(K2, np.concatenate([c2 + A2.T @ d2, np.zeros(20)]))
    np.testing.assert_allclose(x2, sol2[:9], atol=1e-11)
    np.testing.assert_allclose(y2, sol2[9:], atol=1e-11)


@pytest.mark.parametrize("shape", [(6, 4), (4, 6)])
def test_projection_diagonal_closed_form(shape):
    """A = Sigma (rectangular diagonal), Section 4.1.1:
    x_i = (c_i + s_i d_i)/(1 + s_i^2), y_i = s_i x_i for i <= min(m, n);
    x_i = c_i beyond (wide), y_i = 0 beyond (tall); s = 1 averages."""
    m, n = shape
    q = min(m, n)
    s = np.array([0.5, 1.0, 2.0, 3.0])[:q]
    A = np.zeros(shape)
    A[np.arange(q), np.arange(q)] = s
    rng = np.random.default_rng(7)
    c, d = rng.normal(size=n), rng.normal(size=m)
    x, y = O.Projector(A)(c, d)
    xr = c.copy()
    xr[:q] = (c[:q] + s * d[:q]) / (1 + s ** 2)
    yr = np.zeros(m)
    yr[:q] = s * xr[:q]
    np.testing.assert_allclose(x, xr, atol=1e-14)
    np.testing.assert_allclose(y, yr, atol=1e-14)
    # sigma = 1: exact average of the two inputs
    assert abs(x[1] - 0.5 * (c[1] + d[1])) < 1e-15 and abs(y[1] - x[1]) < 1e-15
