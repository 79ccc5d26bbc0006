"""Pins for the oracle's proximal operators and conjugates (CPU only).

Each closed form is checked against brute-force scalar minimisation, each
conjugate against the Fenchel-Young inequality and its equality case, and the
parametric prox formula (Section 5) and the pre-conditioned prox (Section 4.1)
against direct minimisation of the objective they claim to minimise.
"""
import math

import numpy as np
import pytest

from oracle import brute
from oracle import pogs_oracle as O

FINITE_H = ["zero", "identity", "abs", "square", "huber", "hinge", "logistic"]
IND_H = ["ind_ge0", "ind_le0", "ind_eq0", "ind_box01"]


def _h_scalar(h, u):
    return float(O.h_eval(h, np.array([u]))[0])


@pytest.mark.parametrize("h", FINITE_H + IND_H)
def test_prox_h_matches_brute_force(h):
    rng = np.random.default_rng(11)
    for _ in range(25):
        z = float(rng.normal(0.0, 3.0))
        r = float(10.0 ** rng.uniform(-1.5, 1.5))
        got = float(O.prox_h(h, np.array([z]), r)[0])
        lo, hi = min(z, 0.0) - 2.0 / r - 3.0, max(z, 1.0) + 2.0 / r + 3.0

        def phi(u):
            return _h_scalar(h, u) + 0.5 * r * (u - z) ** 2

        if h == "ind_eq0":
            ref = 0.0
        else:
            ref = brute.scalar_min(phi, lo, hi)
        assert abs(got - ref) <= 1e-6 * max(1.0, abs(ref)), (h, z, r, got, ref)
        # The prox value must not be beaten by the brute-force point.
        assert phi(got) <= phi(ref) + 1e-10 * max(1.0, abs(phi(ref)))


@pytest.mark.parametrize("h", ["abs", "square", "ind_ge0", "ind_le0", "ind_box01"])
def test_textbook_closed_forms(h):
    # Hand-written values: soft threshold, shrinkage, clipping.
    z = np.array([-2.0, -0.25, 0.0, 0.3, 0.75, 3.0])
    r = 2.0
    expect = {
        "abs": [-1.5, 0.0, 0.0, 0.0, 0.25, 2.5],
        "square": [-4 / 3, -1 / 6, 0.0, 0.2, 0.5, 2.0],
        "ind_ge0": [0.0, 0.0, 0.0, 0.3, 0.75, 3.0],
        "ind_le0": [-2.0, -0.25, 0.0, 0.0, 0.0, 0.0],
        "ind_box01": [0.0, 0.0, 0.0, 0.3, 0.75, 1.0],
    }[h]
    np.testing.assert_allclose(O.prox_h(h, z, r), expect, rtol=0, atol=1e-15)


def test_logistic_prox_optimality():
    rng = np.random.default_rng(5)
    z = rng.normal(0, 10, 200)
    r = 10.0 ** rng.uniform(-3, 3, 200)
    u = O.prox_h("logistic", z, r)
    sig = 1.0 / (1.0 + np.exp(-u))
    # 0 = sigma(u) + r (u - z) at the minimiser
    assert np.max(np.abs(sig + r * (u - z)) / np.maximum(1.0, r * np.abs(z))) < 1e-12


@pytest.mark.parametrize("h", FINITE_H + IND_H)
def test_fenchel_young_equality_at_prox(h):
    """s = r (z - prox(z)) is a subgradient of h at prox(z), so
    h(u) + h*(s) = s u there (Section 2.2, Fenchel equalities)."""
    rng = np.random.default_rng(3)
    z = rng.normal(0, 2, 300)
    r = 10.0 ** rng.uniform(-1, 1, 300)
    u = O.prox_h(h, z, r)
    s = r * (z - u)
    lhs = O.h_eval(h, u) + O.h_conj(h, s, tol=1e-12)
    assert np.all(np.isfinite(lhs)), h
    np.testing.assert_allclose(lhs, s * u, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("h", FINITE_H + ["ind_box01"])
def test_conjugate_by_grid_sup(h):
    """h*(s) = sup_u s u - h(u) by a dense grid, where finite."""
    us = np.linspace(-60, 60, 240001)
    hv = O.h_eval(h, us)
    half = np.abs(us) <= 30.0
    for s in [-0.7, 0.0, 0.25, 0.5, 0.9, 1.0, 1.4]:
        ref = np.max(s * us - hv)
        got = float(O.h_conj(h, np.array([s]))[0])
        if np.isinf(got):
            # unbounded: the sup keeps growing as the grid widens
            assert ref > np.max(s * us[half] - hv[half]) + 1.0, (h, s, ref)
        else:
            assert abs(got - ref) < 2e-3, (h, s, got, ref)


def test_fenchel_young_inequality_random():
    rng = np.random.default_rng(4)
    for h in FINITE_H + IND_H:
        u = rng.normal(0, 2, 500)
        s = rng.normal(0, 2, 500)
        with np.errstate(invalid="ignore"):
            tot = O.h_eval(h, u) + O.h_conj(h, s)
        ok = np.isinf(tot) | (tot >= s * u - 1e-12)
        assert np.all(ok), h


class _F:
    def __init__(self, h, **kw):
        self.h = h
        self.kw = kw
        self.size = len(next(iter(kw.values())))

    def field(self, k):
        return np.asarray(self.kw[k], float)


@pytest.mark.parametrize("h", FINITE_H + ["ind_ge0", "ind_le0", "ind_box01"])
def test_parametric_prox_formula(h):
    """Section 5 formula vs direct minimisation of
    c h(a y - b) + d y + (e/2) y^2 + (rho/2)(y - v)^2."""
    rng = np.random.default_rng(7)
    N = 12
    a = rng.choice([-1, 1], N) * 10.0 ** rng.uniform(-0.7, 0.7, N)
    b = rng.normal(0, 1, N)
    c = 10.0 ** rng.uniform(-1, 1, N)
    d = rng.normal(0, 1, N)
    e = np.where(rng.random(N) < 0.5, 0.0, 10.0 ** rng.uniform(-1, 1, N))
    v = rng.normal(0, 2, N)
    rho = 10.0 ** rng.uniform(-1, 1, N)
    F = _F(h, a=a, b=b, c=c, d=d, e=e)
    got = O.prox_param(F, v, rho)
    for i in range(N):
        def phi(y, i=i):
            return (c[i] * _h_scalar(h, a[i] * y - b[i]) + d[i] * y + 0.5 * e[i] * y * y
                    + 0.5 * rho[i] * (y - v[i]) ** 2)
        # bracket wide enough for every term's minimiser
        span = 4.0 + abs(v[i]) + (abs(b[i]) + 2.0) / abs(a[i]) + abs(d[i]) / rho[i] + c[i] * abs(a[i]) / rho[i]
        ref = brute.scalar_min(phi, -span, span, grid=8001)
        assert abs(got[i] - ref) <= 1e-6 * max(1.0, abs(ref)), (h, i, got[i], ref)


def test_parametric_prox_c_zero():
    F = _F("abs", a=[2.0], b=[1.0], c=[0.0], d=[0.5], e=[3.0])
    # argmin 0.5 y + 1.5 y^2 + (rho/2)(y - v)^2 = (rho v - d)/(e + rho)
    got = O.prox_param(F, np.array([1.2]), 2.0)[0]
    assert abs(got - (2.0 * 1.2 - 0.5) / (3.0 + 2.0)) < 1e-15


def test_scaled_prox_matches_rho_scaling():
    """Pre-conditioned prox (Section 4.1): with g^(x^) = g(E x^),
    E prox_{g^,rho}(v) = prox_{g, rho/E^2}(E v); with f^(y^) = f(y^/D),
    prox_{f^,rho}(v)/D = prox_{f, rho D^2}(v/D)."""
    rng = np.random.default_rng(9)
    N = 400
    for h in FINITE_H + ["ind_ge0", "ind_box01"]:
        F = _F(h, a=rng.choice([-1, 1], N) * rng.uniform(0.3, 3, N), b=rng.normal(0, 1, N),
               c=rng.uniform(0.1, 3, N), d=rng.normal(0, 1, N),
               e=np.where(rng.random(N) < 0.5, 0.0, rng.uniform(0.1, 2, N)))
        E = rng.uniform(0.2, 5, N)
        D = rng.uniform(0.2, 5, N)
        v = rng.normal(0, 2, N)
        rho = 1.7
        lhs = E * O.prox_param(O.scale_fn(F, E), v, rho)
        rhs = O.prox_param(F, E * v, rho / E ** 2)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-10)
        lhs = O.prox_param(O.scale_fn(F, 1.0 / D), v, rho) / D
        rhs = O.prox_param(F, v / D, rho * D ** 2)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("h", ["abs", "square", "logistic", "hinge", "huber", "ind_ge0", "ind_le0", "ind_box01"])
def test_parametric_conjugate_fenchel_equality(h):
    """nu = rho (v - prox_f(v)) is a subgradient of f at prox_f(v) (Section 3.3),
    so f(y) + f*(nu) = nu y (Section 2.2) for the parametric conjugate."""
    rng = np.random.default_rng(13)
    N = 200
    F = _F(h, a=rng.choice([-1, 1], N) * rng.uniform(0.3, 3, N), b=rng.normal(0, 1, N),
           c=rng.uniform(0.1, 3, N), d=rng.normal(0, 1, N), e=np.zeros(N))
    v = rng.normal(0, 2, N)
    rho = rng.uniform(0.2, 5, N)
    y = O.prox_param(F, v, rho)
    nu = rho * (v - y)
    for i in range(N):
        Fi = _F(h, **{k: F.field(k)[i:i + 1] for k in "abcde"})
        lhs = O.fn_eval(Fi, y[i:i + 1], tol=1e-12) + O.fn_conj(Fi, nu[i:i + 1], tol=1e-12)
        assert math.isfinite(lhs), (h, i)
        assert abs(lhs - nu[i] * y[i]) <= 1e-8 * max(1.0, abs(nu[i] * y[i])), (h, i)


# --------------------------------------------------------------------------
# Base functions with restricted domains or no closed-form prox
# (e^u, u log u, -log u, 1/u, max(0, -u))
# --------------------------------------------------------------------------
MORE_H = ["exp", "neg_entr", "neg_log", "recipr", "max_neg0"]


@pytest.mark.parametrize("h", MORE_H)
def test_more_prox_matches_brute_force(h):
    rng = np.random.default_rng(21)
    for _ in range(25):
        z = float(rng.normal(0.0, 2.0))
        r = float(10.0 ** rng.uniform(-1.0, 1.0))
        got = float(O.prox_h(h, np.array([z]), r)[0])

        def phi(u):
            return _h_scalar(h, u) + 0.5 * r * (u - z) ** 2

        lo = 1e-12 if h in ("neg_entr", "neg_log", "recipr") else min(z, 0.0) - 2.0 / r - 3.0
        hi = max(z, 1.0) + 2.0 / r + 3.0
        ref = brute.scalar_min(phi, lo, hi, grid=20001)
        assert abs(got - ref) <= 1e-6 * max(1.0, abs(ref)), (h, z, r, got, ref)
        assert phi(got) <= phi(ref) + 1e-10 * max(1.0, abs(phi(ref)))


def test_more_prox_optimality_conditions():
    """The stationarity conditions the minimisers satisfy (domains open)."""
    rng = np.random.default_rng(22)
    z = rng.normal(0, 4, 300)
    r = 10.0 ** rng.uniform(-2, 2, 300)
    u = O.prox_h("exp", z, r)
    assert np.max(np.abs(np.exp(u) + r * (u - z)) / np.maximum(1.0, r * np.abs(z) + np.exp(u))) < 1e-12
    u = O.prox_h("neg_entr", z, r)
    pos = u > 1e-300  # exp(r z - 1) below the float64 range rounds to 0
    assert np.all(u >= 0.0) and np.all(r[~pos] * z[~pos] - 1.0 < -600.0)
    assert np.max(np.abs(np.log(u[pos]) + 1.0 + r[pos] * (u[pos] - z[pos])) / np.maximum(1.0, r[pos] * np.abs(z[pos]))) < 1e-10
    u = O.prox_h("neg_log", z, r)
    assert np.all(u > 0.0)
    np.testing.assert_allclose(-1.0 / u + r * (u - z), 0.0, atol=1e-9 * np.max(r * (np.abs(z) + 1)))
    u = O.prox_h("recipr", z, r)
    assert np.all(u > 0.0)
    assert np.max(np.abs(r * (u - z) - 1.0 / u ** 2) / np.maximum(1.0, 1.0 / u ** 2)) < 1e-10


@pytest.mark.parametrize("h", MORE_H)
def test_more_fenchel_young_equality_at_prox(h):
    rng = np.random.default_rng(23)
    z = rng.normal(0, 2, 300)
    r = 10.0 ** rng.uniform(-1, 1, 300)
    u = O.prox_h(h, z, r)
    s = r * (z - u)
    lhs = O.h_eval(h, u) + O.h_conj(h, s, tol=1e-12)
    assert np.all(np.isfinite(lhs)), h
    np.testing.assert_allclose(lhs, s * u, rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("h", MORE_H)
def test_more_conjugate_by_grid_sup(h):
    us = np.linspace(-40, 40, 400001)
    with np.errstate(over="ignore"):
        hv = O.h_eval(h, us)
    for s in [-2.0, -0.7, -0.2, 0.3, 1.0, 2.5]:
        with np.errstate(invalid="ignore", over="ignore"):
            ref = np.max(s * us - hv)
        got = float(O.h_conj(h, np.array([s]))[0])
        if np.isinf(got):
            # unbounded: the supremum grows with the grid
            half = np.abs(us) <= 20.0
            with np.errstate(invalid="ignore", over="ignore"):
                assert ref > np.max(s * us[half] - hv[half]) + 1.0, (h, s, ref)
        else:
            assert abs(got - ref) < 2e-3 * max(1.0, abs(ref)), (h, s, got, ref)


@pytest.mark.parametrize("h", MORE_H)
def test_more_parametric_prox_formula(h):
    rng = np.random.default_rng(24)
    N = 10
    a = rng.choice([-1, 1], N) * 10.0 ** rng.uniform(-0.5, 0.5, N)
    b = rng.normal(0, 1, N)
    c = 10.0 ** rng.uniform(-1, 0.5, N)
    d = rng.normal(0, 1, N)
    e = np.where(rng.random(N) < 0.5, 0.0, 10.0 ** rng.uniform(-1, 1, N))
    v = rng.normal(0, 2, N)
    rho = 10.0 ** rng.uniform(-0.5, 1, N)
    F = _F(h, a=a, b=b, c=c, d=d, e=e)
    got = O.prox_param(F, v, rho)
    for i in range(N):
        def phi(y, i=i):
            return (c[i] * _h_scalar(h, a[i] * y - b[i]) + d[i] * y + 0.5 * e[i] * y * y
                    + 0.5 * rho[i] * (y - v[i]) ** 2)
        span = 6.0 + abs(v[i]) + (abs(b[i]) + 3.0) / abs(a[i]) + abs(d[i]) / rho[i] + 3 * c[i] * abs(a[i]) / rho[i]
        ref = brute.scalar_min(phi, -span, span, grid=40001)
        assert abs(got[i] - ref) <= 1e-6 * max(1.0, abs(ref)), (h, i, got[i], ref)
