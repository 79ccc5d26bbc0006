"""FP64 CPU oracle for graph-form ADMM with equilibration and adaptive rho.

TEST INFRASTRUCTURE ONLY.  This module is a plain, slow, obviously-correct
NumPy implementation of what the GPU solver computes.  Only the test suite,
the package's smoke check and the benchmark's CPU-baseline leg may import it;
the GPU library never calls, links or loads anything here, and nothing here
imports the GPU package.

Problem (Section 1): minimize f(y) + g(x) subject to y = A x, with f and g
separable and each term written in the parametric form of Section 5,
    f_i(y) = c h(a y - b) + d y + (e/2) y^2,   c >= 0, e >= 0.
A function is passed as an object with attributes ``h`` (one base-function
name, or a sequence of ``size`` names, one per element), ``size``, and a method ``field(name)`` returning the float64 array of a, b, c,
d or e (``Fn`` of the workload module has that shape; any duck type does).

Everything here runs in float64.  Readings of passages the paper leaves open
(the fixed Sinkhorn-Knopp iteration count, which machine epsilon, 0-based k in
the adaptive-rho test, strict inequalities, scaled-space residuals, rho0 = 1)
are stated where used.

Pins (tests/test_oracle_*.py) check every function here against closed forms,
brute force, library solvers and invariants that do not reuse this code.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# ---------------------------------------------------------------------------
# Base functions h, their proximal operators and conjugates
# ---------------------------------------------------------------------------

H_NAMES = ("zero", "identity", "abs", "square", "huber", "hinge", "logistic",
           "ind_ge0", "ind_le0", "ind_eq0", "ind_box01",
           "exp", "neg_entr", "neg_log", "recipr", "max_neg0")


def h_eval(h: str, u, tol: float = 0.0):
    """Value of the base function h at u (elementwise, +inf outside its domain).

    ``tol`` widens the domains of the indicator functions by that amount, for
    points that rounding has pushed just outside.
    """
    u = np.asarray(u, dtype=np.float64)
    if h == "zero":
        return np.zeros_like(u)
    if h == "identity":
        return u.copy()
    if h == "abs":
        return np.abs(u)
    if h == "square":
        return 0.5 * u * u
    if h == "huber":
        au = np.abs(u)
        return np.where(au <= 1.0, 0.5 * u * u, au - 0.5)
    if h == "hinge":
        return np.maximum(u, 0.0)
    if h == "logistic":
        return np.logaddexp(0.0, u)
    if h == "ind_ge0":
        return np.where(u >= -tol, 0.0, np.inf)
    if h == "ind_le0":
        return np.where(u <= tol, 0.0, np.inf)
    if h == "ind_eq0":
        return np.where(np.abs(u) <= tol, 0.0, np.inf)
    if h == "ind_box01":
        return np.where((u >= -tol) & (u <= 1.0 + tol), 0.0, np.inf)
    if h == "exp":
        return np.exp(u)
    if h == "neg_entr":  # u log u on u >= 0 (0 at 0)
        with np.errstate(divide="ignore", invalid="ignore"):
            v = np.where(u > 0.0, u * np.log(np.where(u > 0.0, u, 1.0)), 0.0)
        return np.where(u >= -tol, v, np.inf)
    if h == "neg_log":  # -log u on u > 0
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(u > 0.0, -np.log(np.where(u > 0.0, u, 1.0)), np.inf)
    if h == "recipr":  # 1 / u on u > 0
        with np.errstate(divide="ignore"):
            return np.where(u > 0.0, 1.0 / np.where(u > 0.0, u, 1.0), np.inf)
    if h == "max_neg0":
        return np.maximum(-u, 0.0)
    raise ValueError(h)


def h_conj(h: str, s, tol: float = 0.0):
    """Convex conjugate h*(s) = sup_u (s u - h(u)), elementwise (textbook forms).

    ``tol`` widens the closed domain of conjugates that are indicators (or
    finite only on an interval) by that amount, for points that rounding has
    pushed just outside; the value is taken at the nearest domain point.
    """
    s = np.asarray(s, dtype=np.float64)
    inf = np.inf

    def box(lo, hi):
        inside = (s >= lo - tol) & (s <= hi + tol)
        return inside, np.clip(s, lo, hi)

    if h == "zero":
        ok, _ = box(0.0, 0.0)
        return np.where(ok, 0.0, inf)
    if h == "identity":
        ok, _ = box(1.0, 1.0)
        return np.where(ok, 0.0, inf)
    if h == "abs":
        ok, _ = box(-1.0, 1.0)
        return np.where(ok, 0.0, inf)
    if h == "square":
        return 0.5 * s * s
    if h == "huber":
        ok, t = box(-1.0, 1.0)
        return np.where(ok, 0.5 * t * t, inf)
    if h == "hinge":
        ok, _ = box(0.0, 1.0)
        return np.where(ok, 0.0, inf)
    if h == "logistic":
        ok, t = box(0.0, 1.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            ent = np.where(t > 0.0, t * np.log(np.where(t > 0.0, t, 1.0)), 0.0) \
                + np.where(t < 1.0, (1.0 - t) * np.log(np.where(t < 1.0, 1.0 - t, 1.0)), 0.0)
        return np.where(ok, ent, inf)
    if h == "ind_ge0":
        ok, _ = box(-inf, 0.0)
        return np.where(ok, 0.0, inf)
    if h == "ind_le0":
        ok, _ = box(0.0, inf)
        return np.where(ok, 0.0, inf)
    if h == "ind_eq0":
        return np.zeros_like(s)
    if h == "ind_box01":
        return np.maximum(s, 0.0)
    if h == "exp":  # s log s - s on s >= 0
        with np.errstate(divide="ignore", invalid="ignore"):
            v = np.where(s > 0.0, s * np.log(np.where(s > 0.0, s, 1.0)) - s, 0.0)
        return np.where(s >= -tol, v, inf)
    if h == "neg_entr":
        return np.exp(s - 1.0)
    if h == "neg_log":  # -1 - log(-s) on s < 0
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(s < 0.0, -1.0 - np.log(np.where(s < 0.0, -s, 1.0)), inf)
    if h == "recipr":  # -2 sqrt(-s) on s <= 0
        return np.where(s <= tol, -2.0 * np.sqrt(np.maximum(-s, 0.0)), inf)
    if h == "max_neg0":
        ok, _ = box(-1.0, 0.0)
        return np.where(ok, 0.0, inf)
    raise ValueError(h)


def _bisect_increasing(phi, lo, hi, iters=300):
    """Root of an increasing function phi on [lo, hi] with phi(lo) <= 0 <= phi(hi)."""
    lo = np.array(lo, dtype=np.float64)
    hi = np.array(hi, dtype=np.float64)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        pos = phi(mid) > 0.0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
        if np.all(hi - lo <= 4 * np.finfo(float).eps * np.maximum(1.0, np.abs(hi))):
            break
    return 0.5 * (lo + hi)


def _exp_prox(z, r):
    """Root of e^u + r (u - z) = 0: increasing in u, positive at z, negative
    at z - e^z / r."""
    hi = z.copy()
    lo = z - np.exp(np.minimum(z, 700.0)) / r
    return _bisect_increasing(lambda u: np.exp(u) + r * (u - z), lo, hi)


def _neg_entr_prox(z, r):
    """argmin u log u + (r/2)(u - z)^2: with u = e^t the optimality condition
    is t + r e^t - (r z - 1) = 0, increasing in t; it is non-negative at
    t_hi = min(r z - 1, log max(z, 1/e)) and negative at r z - 1 - r e^t_hi."""
    c = r * z - 1.0
    thi = np.minimum(c, np.log(np.maximum(z, math.exp(-1.0))))
    tlo = c - r * np.exp(thi)
    t = _bisect_increasing(lambda t: t + r * np.exp(t) - c, tlo, thi)
    return np.exp(t)


def _recipr_prox(z, r):
    """Root of r (u - z) - 1/u^2 = 0 on u > 0 (increasing in u): non-negative
    at hi = max(z, 0) + r^(-1/3), negative at 1 / sqrt(r (hi - z))."""
    hi = np.maximum(z, 0.0) + r ** (-1.0 / 3.0)
    lo = np.minimum(1.0 / np.sqrt(r * (hi - z)), hi)
    return _bisect_increasing(lambda u: r * (u - z) - 1.0 / (u * u), lo, hi)


def _logistic_prox(z, r):
    """Root of sigma(u) + r (u - z) = 0 by bisection on [z - 1/r, z].

    The left side is increasing in u, negative at z - 1/r (sigma < 1) and
    positive at z (sigma > 0), so the bracket always holds the root.
    """
    lo = z - 1.0 / r
    hi = z.copy()
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        sig = 0.5 * (1.0 + np.tanh(0.5 * mid))
        pos = sig + r * (mid - z) > 0.0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
        if np.all(hi - lo <= 4 * np.finfo(float).eps * np.maximum(1.0, np.abs(hi))):
            break
    return 0.5 * (lo + hi)


def prox_h(h: str, z, r):
    """prox_{h,r}(z) = argmin_u h(u) + (r/2)(u - z)^2 (elementwise; r > 0).

    Closed forms are the textbook ones (soft threshold for |u|, shrinkage
    for u^2/2, clipping for indicators, the positive root of a quadratic for
    -log u); logistic, e^u, u log u and 1/u have none and are solved by
    bisection on a bracket of their monotone optimality condition.
    """
    z = np.asarray(z, dtype=np.float64)
    r = np.broadcast_to(np.asarray(r, dtype=np.float64), z.shape)
    if h == "zero":
        return z.copy()
    if h == "identity":
        return z - 1.0 / r
    if h == "abs":
        return np.sign(z) * np.maximum(np.abs(z) - 1.0 / r, 0.0)
    if h == "square":
        return r * z / (1.0 + r)
    if h == "huber":
        return np.where(np.abs(z) <= 1.0 + 1.0 / r, r * z / (1.0 + r), z - np.sign(z) / r)
    if h == "hinge":
        return np.where(z > 1.0 / r, z - 1.0 / r, np.where(z < 0.0, z, 0.0))
    if h == "logistic":
        return _logistic_prox(z, r)
    if h == "ind_ge0":
        return np.maximum(z, 0.0)
    if h == "ind_le0":
        return np.minimum(z, 0.0)
    if h == "ind_eq0":
        return np.zeros_like(z)
    if h == "ind_box01":
        return np.clip(z, 0.0, 1.0)
    if h == "exp":
        return _exp_prox(z, r)
    if h == "neg_entr":
        return _neg_entr_prox(z, r)
    if h == "neg_log":  # r u^2 - r z u - 1 = 0, positive root
        return 0.5 * (z + np.sqrt(z * z + 4.0 / r))
    if h == "recipr":
        return _recipr_prox(z, r)
    if h == "max_neg0":
        return np.where(z < -1.0 / r, z + 1.0 / r, np.where(z > 0.0, z, 0.0))
    raise ValueError(h)


# ---------------------------------------------------------------------------
# Parametric separable functions (Section 5)
# ---------------------------------------------------------------------------

def _h_groups(h, n: int):
    """Split the elements by base function: yields (name, index array).  ``h``
    is one name for all n elements or a sequence of n names."""
    if isinstance(h, str):
        yield h, np.arange(n)
        return
    names = np.asarray(h, dtype=object)
    if names.shape != (n,):
        raise ValueError(f"h has shape {names.shape}, expected ({n},)")
    for name in sorted(set(names.tolist())):
        yield name, np.flatnonzero(names == name)


def _h_map(fun, h, u, *args):
    """Apply fun(name, u_part, *args_part) group by group (per-element h);
    scalar args are passed unchanged, arrays of u's shape are split."""
    u = np.asarray(u, dtype=np.float64)
    if isinstance(h, str):
        return fun(h, u, *args)
    out = np.empty_like(u)
    for name, idx in _h_groups(h, u.shape[0]):
        part = [a[idx] if isinstance(a, np.ndarray) and a.shape == u.shape else a for a in args]
        out[idx] = fun(name, u[idx], *part)
    return out


@dataclasses.dataclass
class Param:
    """Plain parameter arrays of a separable parametric function (``h`` is one
    name or a per-element sequence of names)."""

    h: object
    a: np.ndarray
    b: np.ndarray
    c: np.ndarray
    d: np.ndarray
    e: np.ndarray

    @property
    def size(self) -> int:
        return self.a.shape[0]

    def field(self, name: str) -> np.ndarray:
        return getattr(self, name)


def as_param(fn) -> Param:
    """Copy a duck-typed function description into float64 arrays."""
    h = fn.h if isinstance(fn.h, str) else tuple(fn.h)
    return Param(h, *(np.array(fn.field(k), dtype=np.float64) for k in "abcde"))


def fn_eval(fn, y, tol: float = 0.0) -> float:
    """Sum of c h(a y - b) + d y + (e/2) y^2 (Section 5), without constant
    offsets.  ``tol`` is passed to h_eval (indicator domains)."""
    p = as_param(fn)
    y = np.asarray(y, dtype=np.float64)
    hv = _h_map(h_eval, p.h, p.a * y - p.b, tol)
    with np.errstate(invalid="ignore"):
        term = np.where(p.c == 0.0, 0.0, p.c * hv)
    return float(np.sum(term + p.d * y + 0.5 * p.e * y * y))


def fn_conj_terms(fn, nu, tol: float = 0.0) -> np.ndarray:
    """Elementwise conjugate of a parametric function (Section 2.1 conjugates of
    the Section 5 form), f*(nu) = sup_y nu y - f(y):

      e = 0, c > 0:  c h*((nu - d)/(a c)) + b (nu - d)/a
      e = 0, c = 0:  indicator of {nu = d}
      e > 0, c = 0:  (nu - d)^2 / (2 e)
      e > 0, c > 0:  (nu - d) y* - (e/2) y*^2 - c h(a y* - b), where the
                     supremum is attained at y* = argmin_y c h(a y - b) +
                     (e/2)(y - (nu - d)/e)^2, the prox of the h term with
                     penalty e at (nu - d)/e.

    ``tol`` is passed to h_conj / h_eval (indicator domains)."""
    p = as_param(fn)
    nu = np.asarray(nu, dtype=np.float64)
    s = nu - p.d
    out = np.empty_like(nu)
    e0, c0 = p.e == 0.0, p.c == 0.0
    k = e0 & c0
    out[k] = np.where(np.abs(s[k]) <= tol, 0.0, np.inf)
    k = e0 & ~c0
    if np.any(k):
        hk = p.h if isinstance(p.h, str) else tuple(np.asarray(p.h, dtype=object)[k])
        out[k] = p.c[k] * _h_map(h_conj, hk, s[k] / (p.a[k] * p.c[k]), tol) + p.b[k] * s[k] / p.a[k]
    k = ~e0 & c0
    out[k] = s[k] * s[k] / (2.0 * p.e[k])
    k = ~e0 & ~c0
    if np.any(k):
        hk = p.h if isinstance(p.h, str) else tuple(np.asarray(p.h, dtype=object)[k])
        a, b, c, e = p.a[k], p.b[k], p.c[k], p.e[k]
        phi = Param(hk, a, b, c, np.zeros_like(a), np.zeros_like(a))
        ys = prox_param(phi, s[k] / e, e)
        out[k] = s[k] * ys - 0.5 * e * ys * ys - c * _h_map(h_eval, hk, a * ys - b, tol)
    return out


def fn_conj(fn, nu, tol: float = 0.0) -> float:
    """Sum of fn_conj_terms."""
    return float(np.sum(fn_conj_terms(fn, nu, tol)))


def fn_eval_strict(fn, y) -> float:
    """f(y) with every indicator taken exactly (+inf outside its domain)."""
    p = as_param(fn)
    y = np.asarray(y, dtype=np.float64)
    hv = _h_map(h_eval, p.h, p.a * y - p.b, 0.0)
    with np.errstate(invalid="ignore"):
        term = np.where(p.c == 0.0, 0.0, p.c * hv)
    return float(np.sum(term + p.d * y + 0.5 * p.e * y * y))


def prox_param(fn, v, rho):
    """prox of a parametric separable function with penalty rho (Section 5):

        argmin_y c h(a y - b) + d y + (e/2) y^2 + (rho/2)(y - v)^2
          = (1/a) (prox_{h, (e+rho)/(c a^2)}(a (rho v - d)/(e + rho) - b) + b).

    ``rho`` may be a scalar or a per-element array.  With c = 0 the h term is
    absent and the result is (rho v - d)/(e + rho).
    """
    p = as_param(fn)
    v = np.asarray(v, dtype=np.float64)
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), v.shape)
    vq = (rho * v - p.d) / (p.e + rho)
    out = vq.copy()
    k = p.c > 0.0
    if np.any(k):
        a, b, c = p.a[k], p.b[k], p.c[k]
        r = (p.e[k] + rho[k]) / (c * a * a)
        hk = p.h if isinstance(p.h, str) else tuple(np.asarray(p.h, dtype=object)[k])
        out[k] = (_h_map(prox_h, hk, a * vq[k] - b, r) + b) / a
    return out


def scale_fn(fn, s) -> Param:
    """The function y -> f(s * y) elementwise, as parametric data:
    c h(a s y - b) + d s y + (e/2) s^2 y^2 (used for the pre-conditioned
    functions of Section 4.1: f^(y^) = f(D^-1 y^), g^(x^) = g(E x^))."""
    p = as_param(fn)
    s = np.asarray(s, dtype=np.float64)
    return Param(p.h, p.a * s, p.b.copy(), p.c.copy(), p.d * s, p.e * s * s)


# ---------------------------------------------------------------------------
# Equilibration (Section 4.2, Algorithm 2) and Frobenius normalisation (4.1.2)
# ---------------------------------------------------------------------------

def sinkhorn_knopp(A, gamma: float, iters: int, p: int = 2):
    """Regularised Sinkhorn-Knopp (Algorithm 2) run for a fixed number of sweeps.

    Starting from e = 1, each sweep sets
        d = n / (|A|^p e + gamma/m),   e = m / (|A^T|^p d + gamma/n),
    and the scalings are D = diag(d)^(1/p), E = diag(e)^(1/p).
    Reading: the algorithm's stopping tolerance is unspecified, so a fixed
    sweep count is used (partial equilibration suffices, Section 4.1.2).
    Returns (d, e) (the p-th powers of the diagonals).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Ap = np.abs(A) ** p
    e = np.ones(n)
    d = np.ones(m)
    for _ in range(iters):
        d = n / (Ap @ e + gamma / m)
        e = m / (Ap.T @ d + gamma / n)
    return d, e


def equilibrate(A, eps_cmp: float, iters: int = 10):
    """Section 5's pre-conditioner: Algorithm 2 with p = 2 and
    gamma = (m + n) sqrt(eps_cmp), then D and E both rescaled by the same
    factor so that ||D A E||_F / sqrt(min(m, n)) = 1 (Section 4.1.2).

    Reading of "rescaled evenly": D <- D / sqrt(s), E <- E / sqrt(s) with
    s = ||D A E||_F / sqrt(min(m, n)).  Returns the diagonals (D, E).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    gamma = (m + n) * math.sqrt(eps_cmp)
    d, e = sinkhorn_knopp(A, gamma, iters, p=2)
    D = np.sqrt(d)
    E = np.sqrt(e)
    s = np.linalg.norm(D[:, None] * A * E[None, :]) / math.sqrt(min(m, n))
    return D / math.sqrt(s), E / math.sqrt(s)


# ---------------------------------------------------------------------------
# Graph projection (Section 3.1 projection formula; Section 3.5 reduced update)
# ---------------------------------------------------------------------------

class Projector:
    """Projection onto {(x, y) : y = A x} through the reduced update of
    Section 3.5 with a cached Cholesky factor:

      m >= n:  x = (I + A^T A)^{-1} (c + A^T d),  y = A x
      m <  n:  y = d + (I + A A^T)^{-1} (A c - d),  x = c + A^T (d - y)

    Reading: the paper prints the last update as c - A^T (d - y).  The
    optimality conditions of the projection (x - c + A^T(y - d) = 0 with
    y = A x, i.e. the K system of Section 3.1) give c + A^T (d - y); the
    printed sign does not return a point of the graph's orthogonal projection.
    """

    def __init__(self, A):
        self.A = np.asarray(A, dtype=np.float64)
        m, n = self.A.shape
        self.tall = m >= n
        K = (self.A.T @ self.A if self.tall else self.A @ self.A.T) + np.eye(min(m, n))
        self.L = np.linalg.cholesky(K)

    def _solve(self, r):
        z = _tri_solve(self.L, r, lower=True)
        return _tri_solve(self.L.T, z, lower=False)

    def __call__(self, c, d):
        A = self.A
        if self.tall:
            x = self._solve(c + A.T @ d)
            y = A @ x
        else:
            y = d + self._solve(A @ c - d)
            x = c + A.T @ (d - y)
        return x, y


def cgls_project(A, c, d, x0, thr: float, cap: int, trace: bool = False):
    """Projection onto {(x, y) : y = A x} by CGLS (Section 3.5, indirect
    methods): x minimises ||x - c||^2 + ||A x - d||^2, the least-squares
    problem [A; I] x ~ [d; c], by conjugate gradients on its normal equations
    (I + A^T A) x = c + A^T d, started from x0.

    Residuals r1 = d - A x (rows), r2 = c - x (columns), normal residual
    s = A^T r1 + r2; direction p, q = A p; step alpha = ||s||^2 / (||q||^2 +
    ||p||^2); then x += alpha p, r1 -= alpha q, s recomputed from the residuals,
    beta = ||s_new||^2 / ||s||^2, p = s_new + beta p.  Stops before a step when
    ||s|| <= thr or after `cap` steps.

    Returns (x, r1, steps) and, with trace, the list of iterates.  y = d - r1
    equals A x up to rounding.
    """
    A = np.asarray(A, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    r1 = d - A @ x
    s = A.T @ r1 + (c - x)
    p = s.copy()
    gamma = float(s @ s)
    steps = 0
    xs = [x.copy()] if trace else None
    while steps < cap and math.sqrt(gamma) > thr:
        q = A @ p
        alpha = gamma / (float(q @ q) + float(p @ p))
        x = x + alpha * p
        r1 = r1 - alpha * q
        s = A.T @ r1 + (c - x)
        gamma_new = float(s @ s)
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        steps += 1
        if trace:
            xs.append(x.copy())
    if trace:
        return x, r1, steps, xs
    return x, r1, steps


def _tri_solve(T, r, lower: bool):
    """Forward or back substitution with a triangular matrix (library primitive)."""
    from scipy.linalg import solve_triangular
    return solve_triangular(T, r, lower=lower)


# ---------------------------------------------------------------------------
# Adaptive penalty (Section 4.3, Algorithm 3)
# ---------------------------------------------------------------------------

def adaptive_rho(rho: float, l: int, u: int, k: int, r_pri: float, eps_pri: float,
                 r_dual: float, eps_dual: float, delta: float, tau: float):
    """One decision of Algorithm 3 after iteration k (0-based).

    If the dual residual has converged and tau k > l: rho *= delta, u = k.
    Else if the primal residual has converged and tau k > u: rho /= delta, l = k.
    Returns (rho, l, u).
    """
    if r_dual < eps_dual and tau * k > l:
        return rho * delta, l, k
    if r_pri < eps_pri and tau * k > u:
        return rho / delta, k, u
    return rho, l, u


# ---------------------------------------------------------------------------
# The solver (Algorithm 1 with the Section 3.2 extensions, Sections 3.3-5)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    eps_abs: float = 1e-4
    eps_rel: float = 1e-3
    max_iter: int = 10000
    rho0: float = 1.0        # reading: unspecified, 1 after the Frobenius normalisation
    alpha: float = 1.7       # Section 5
    delta: float = 1.05      # Section 5
    tau: float = 0.8         # Section 5
    adaptive_rho: bool = True
    equil_iters: int = 10    # reading: fixed sweep count for Algorithm 2
    equilibrate: bool = True
    eps_cmp: float = float(np.finfo(np.float32).eps)  # machine epsilon of the iteration type
    projection: str = "direct"  # "direct" (cached factor) or "cgls" (Section 3.5, indirect)
    cg_max_iter: int = 10       # reading: CGLS step cap per projection
    cg_tol: float = 0.1         # reading: CGLS stops when rho ||s|| <= cg_tol * eps_dual
    stop: str = "residual"      # "residual" or "gap" (Section 3.4)


@dataclasses.dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    mu: np.ndarray
    nu: np.ndarray
    iters: int
    converged: bool
    rho: float
    r_pri: float
    r_dual: float
    eps_pri: float
    eps_dual: float
    optval: float           # f(y) + g(x) at the returned (x, y), without constants
    D: np.ndarray
    E: np.ndarray
    history: Optional[dict] = None
    cg_steps: int = 0       # CGLS steps over all projections (projection = "cgls")
    gap: float = float("nan")      # eta of the returned tuple (stop = "gap")
    eps_gap: float = float("nan")


def warm_state(Ah, fh, gh, D, E, rho0: float, x0=None, nu0=None):
    """Iteration state (x, y, x~, y~) in the scaled variables from a warm start
    (x0, nu0) in the original ones (Section 5; either may be None).

    Reading of the state: x = E^-1 x0 and y = A^ x (a point of the graph);
    y~ = -(D^-1 nu0) / rho0, since nu_h = -rho y~ whenever the prox step leaves y
    unchanged; x~ = -A^T y~, the relation every projection restores.  From an
    optimal pair this state is a fixed point of the iteration; x0 = nu0 = 0 is
    the cold start.

    Reading of the estimate Section 5 promises when only one of them is
    given: one step of the proximal point method from zero for the missing
    half, i.e. the value the prox step of the iteration itself returns.
      x0 only:  nu^ = rho0 (y - prox_f^(y)) (a subgradient of f^ at
                prox_f^(y), the dual of the prox step from (y, y~ = 0)), so
                y~ = prox_f^(y) - y;
      nu0 only: mu^ = -A^T nu^ = -rho0 x~ (dual feasibility, Section 2) and
                x = prox_g^(mu^ / rho0) = prox_g^(-x~) (the x half step from
                (x = 0, x~)), then y = A^ x.
    """
    m, n = Ah.shape
    x = np.zeros(n)
    y = np.zeros(m)
    xt = np.zeros(n)
    yt = np.zeros(m)
    if x0 is not None:
        x = np.asarray(x0, dtype=np.float64) / E
        y = Ah @ x
    if nu0 is not None:
        yt = -(np.asarray(nu0, dtype=np.float64) / D) / rho0
        xt = -(Ah.T @ yt)
    if x0 is not None and nu0 is None:
        yt = prox_param(fh, y, rho0) - y
        xt = -(Ah.T @ yt)
    elif nu0 is not None and x0 is None:
        x = prox_param(gh, -xt, rho0)
        y = Ah @ x
    return x, y, xt, yt


def solve(A, f, g, params: Params = Params(), record: bool = False,
          D: Optional[np.ndarray] = None, E: Optional[np.ndarray] = None,
          x0: Optional[np.ndarray] = None, nu0: Optional[np.ndarray] = None) -> Result:
    """Graph projection splitting (Algorithm 1) on the pre-conditioned problem.

    Per iteration k = 0, 1, ... (all in the scaled variables of Section 4.1,
    A^ = D A E, f^(y) = f(D^-1 y), g^(x) = g(E x)):
      1. x_h = prox_g^(x - x~), y_h = prox_f^(y - y~)                (Alg. 1)
      2. mu_h = -rho (x_h - x + x~), nu_h = -rho (y_h - y + y~)      (Sec. 3.3)
      3. x_r = alpha x_h + (1 - alpha) x, likewise y_r                (Sec. 3.2)
      4. (x, y) = Pi(x_r + x~, y_r + y~)                            (Alg. 1, Sec. 3.5)
      5. x~ += x_r - x, y~ += y_r - y                               (Alg. 1 + Sec. 3.2)
         With projection = "cgls" steps 4-5 are: x = CGLS(c = x_r + x~,
         d = y_r + y~) from x_h, then x~ = c - x, y~ = r1 = d - A^ x and
         y = d - r1 (the same updates with the residual CGLS carries).
      6. r_pri = ||A^ x_h - y_h||, r_dual = ||A^T nu_h + mu_h||,
         eps_pri = eps_abs + eps_rel ||y_h||, eps_dual = eps_abs + eps_rel ||mu_h||
                                                                    (Sec. 3.4)
      7. stop when r_pri < eps_pri and r_dual < eps_dual               (Alg. 3)
         or, with stop = "gap", when the gap of the feasible tuple
         (x, y, -rho x~, -rho y~) after step 5, f(y) + g(x) + f*(-rho y~) +
         g*(-rho x~), is below eps_abs + eps_rel |f(y) + g(x)|; that tuple is
         then the one returned                                       (Sec. 3.4)
      8. Algorithm 3 may change rho; (x~, y~) are then rescaled by
         rho_old / rho_new (Sec. 3.2, varying penalty).
    Readings: residuals and tolerances are taken in the scaled variables the
    iteration runs in; the inequalities are strict as in Algorithm 3; k is the
    0-based iteration index of Algorithm 1.

    The returned tuple is the last half-step tuple (Section 5) mapped back to
    the original variables: x = E x_h, y = D^-1 y_h, mu = E^-1 mu_h, nu = D nu_h.

    Warm start (Section 5: the caller may supply x0 and nu0; with only one
    of them the other is estimated): see warm_state.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if D is None or E is None:
        if params.equilibrate:
            D, E = equilibrate(A, params.eps_cmp, params.equil_iters)
        else:
            D, E = np.ones(m), np.ones(n)
    Ah = D[:, None] * A * E[None, :]
    fh = scale_fn(f, 1.0 / D)
    gh = scale_fn(g, E)
    if params.projection not in ("direct", "cgls"):
        raise ValueError(f"unknown projection {params.projection!r}")
    if params.stop not in ("residual", "gap"):
        raise ValueError(f"unknown stopping rule {params.stop!r}")
    gap_stop = params.stop == "gap"
    gap = eps_gap = float("nan")
    by_gap = False
    cg = params.projection == "cgls"
    proj = None if cg else Projector(Ah)
    cg_steps = 0

    x, y, xt, yt = warm_state(Ah, fh, gh, D, E, params.rho0, x0, nu0)
    rho = params.rho0
    l = u = 0
    hist = {"r_pri": [], "r_dual": [], "eps_pri": [], "eps_dual": [], "rho": [],
            "inv_dual": [], "inv_primal": [], "cg": [], "gap": []} if record else None
    converged = False
    k = 0
    for k in range(params.max_iter):
        xh = prox_param(gh, x - xt, rho)
        yh = prox_param(fh, y - yt, rho)
        mu = -rho * (xh - x + xt)
        nu = -rho * (yh - y + yt)
        xr = params.alpha * xh + (1.0 - params.alpha) * x
        yr = params.alpha * yh + (1.0 - params.alpha) * y
        eps_pri = params.eps_abs + params.eps_rel * float(np.linalg.norm(yh))
        eps_dual = params.eps_abs + params.eps_rel * float(np.linalg.norm(mu))
        if cg:
            # CGLS from the half step (the projection's input converges to its
            # output, Section 3.5); accurate to a fraction of the dual tolerance:
            # the normal residual s is exactly x~ + A^T y~ after the update below,
            # which enters the next dual residual multiplied by rho.
            c_in, d_in = xr + xt, yr + yt
            x_new, r1, steps = cgls_project(Ah, c_in, d_in, xh, params.cg_tol * eps_dual / rho,
                                            params.cg_max_iter)
            cg_steps += steps
            y_new = d_in - r1
            xt = c_in - x_new
            yt = r1
            if record:
                hist["cg"].append(steps)
        else:
            x_new, y_new = proj(xr + xt, yr + yt)
            xt = xt + xr - x_new
            yt = yt + yr - y_new
        x, y = x_new, y_new
        r_pri = float(np.linalg.norm(Ah @ xh - yh))
        r_dual = float(np.linalg.norm(Ah.T @ nu + mu))
        if record:
            hist["r_pri"].append(r_pri)
            hist["r_dual"].append(r_dual)
            hist["eps_pri"].append(eps_pri)
            hist["eps_dual"].append(eps_dual)
            hist["rho"].append(rho)
            hist["inv_dual"].append(float(np.linalg.norm(xt + Ah.T @ yt)))
            hist["inv_primal"].append(float(np.linalg.norm(y - Ah @ x)))
        if gap_stop:
            # gap of the primal and dual feasible tuple (x, y, -rho x~, -rho y~)
            # the projection just produced (Section 3.4, gap based stopping)
            obj = fn_eval_strict(fh, y) + fn_eval_strict(gh, x)
            with np.errstate(invalid="ignore"):
                gap = obj + fn_conj(fh, -rho * yt) + fn_conj(gh, -rho * xt)
            eps_gap = params.eps_abs + params.eps_rel * abs(obj)
            if record:
                hist["gap"].append(gap)
            if gap < eps_gap:
                converged = by_gap = True
                break
        elif r_pri < eps_pri and r_dual < eps_dual:
            converged = True
            break
        if params.adaptive_rho:
            rho_new, l, u = adaptive_rho(rho, l, u, k, r_pri, eps_pri, r_dual, eps_dual,
                                         params.delta, params.tau)
            if rho_new != rho:
                xt = xt * (rho / rho_new)
                yt = yt * (rho / rho_new)
                rho = rho_new
    if by_gap:
        xh, yh, mu, nu = x, y, -rho * xt, -rho * yt
    x_out = E * xh
    y_out = yh / D
    mu_out = mu / E
    nu_out = D * nu
    # indicator domains checked to 1e-9 (prox outputs meet them up to rounding)
    optval = fn_eval(f, y_out, 1e-9) + fn_eval(g, x_out, 1e-9)
    return Result(x_out, y_out, mu_out, nu_out, k + 1, converged, rho, r_pri, r_dual,
                  eps_pri, eps_dual, optval, D, E, hist, cg_steps, gap, eps_gap)


# ---------------------------------------------------------------------------
# Certificates (Section 2)
# ---------------------------------------------------------------------------

def duality_gap(f, g, x, y, mu, nu, tol: float = 0.0) -> float:
    """eta = f(y) + f*(nu) + g(x) + g*(mu) (Section 2.1); >= 0 for feasible tuples."""
    return fn_eval(f, y, tol) + fn_conj(f, nu, tol) + fn_eval(g, x, tol) + fn_conj(g, mu, tol)
