"""Seeded synthetic problem generators for graph-form problems.

minimize f(y) + g(x) subject to y = A x, with separable f and g written in the
parametric form of Section 5:  f_i(y) = c h(a y - b) + d y + (e/2) y^2.

This module only draws inputs (matrices, vectors, function parameters) from a
seeded NumPy generator.  It holds none of the solver's arithmetic: it is shared
by the GPU path's tests and benchmark and by the CPU oracle's tests as the one
source of inputs.

Problem classes follow Appendix A (basis pursuit A.1, entropy maximization
A.2, Huber fitting A.3, Lasso A.4, logistic regression A.5, linear program
A.6, non-negative least squares A.7, portfolio optimization A.8, support vector
machine A.9) and the radiation-treatment shape of Section 6.2; the
sizes, noise levels and lambda rules of the named workloads are the ones the
benchmark configurations fix (documented per generator).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional, Sequence, Union

import numpy as np

ArrayLike = Union[float, np.ndarray]

# Base functions h of the parametric representation (Section 5).
H_NAMES = (
    "zero",       # h(u) = 0
    "identity",   # h(u) = u
    "abs",        # h(u) = |u|
    "square",     # h(u) = u^2 / 2
    "huber",      # h(u) = u^2/2 if |u| <= 1 else |u| - 1/2
    "hinge",      # h(u) = max(0, u)
    "logistic",   # h(u) = log(1 + exp(u))
    "ind_ge0",    # h(u) = 0 if u >= 0 else +inf
    "ind_le0",    # h(u) = 0 if u <= 0 else +inf
    "ind_eq0",    # h(u) = 0 if u == 0 else +inf
    "ind_box01",  # h(u) = 0 if 0 <= u <= 1 else +inf
    "exp",        # h(u) = e^u
    "neg_entr",   # h(u) = u log u on u >= 0
    "neg_log",    # h(u) = -log u on u > 0
    "recipr",     # h(u) = 1/u on u > 0
    "max_neg0",   # h(u) = max(0, -u)
)


@dataclasses.dataclass
class Fn:
    """A separable function sum_i c_i h(a_i y_i - b_i) + d_i y_i + (e_i/2) y_i^2.

    ``h`` is one base-function name for every element or a sequence of
    ``size`` names, one per element.  Each of a..e is a
    scalar (broadcast) or a length-``size`` array.  ``const`` is a constant
    the parametric form cannot carry; it is added back only when objectives
    are reported.
    """

    h: Union[str, Sequence[str]]
    size: int
    a: ArrayLike = 1.0
    b: ArrayLike = 0.0
    c: ArrayLike = 1.0
    d: ArrayLike = 0.0
    e: ArrayLike = 0.0
    const: float = 0.0

    def __post_init__(self):
        names = [self.h] if isinstance(self.h, str) else list(self.h)
        if not isinstance(self.h, str) and len(names) != self.size:
            raise ValueError(f"h has {len(names)} entries, expected {self.size}")
        for h in set(names):
            if h not in H_NAMES:
                raise ValueError(f"unknown base function {h!r}")

    def field(self, name: str) -> np.ndarray:
        """Parameter ``name`` expanded to a float64 array of length ``size``."""
        v = getattr(self, name)
        if np.ndim(v) == 0:
            return np.full(self.size, float(v))
        v = np.asarray(v, dtype=np.float64)
        if v.shape != (self.size,):
            raise ValueError(f"{name} has shape {v.shape}, expected ({self.size},)")
        return v


@dataclasses.dataclass
class Problem:
    name: str
    A: np.ndarray  # m x n, C-contiguous, float32 or float64
    f: Fn          # length m
    g: Fn          # length n
    eps_abs: float = 1e-4
    eps_rel: float = 1e-3
    max_iter: int = 10000
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


_ROW_BLOCK = 2048


def _matvec(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A x in float64 from elementwise products and NumPy's own fixed-order
    sums over row blocks, so that the drawn inputs do not depend on the host's
    BLAS library or its thread count."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(A.shape[0])
    for i in range(0, A.shape[0], _ROW_BLOCK):
        out[i:i + _ROW_BLOCK] = (A[i:i + _ROW_BLOCK].astype(np.float64) * x).sum(axis=1)
    return out


def _rmatvec(A: np.ndarray, v: np.ndarray) -> np.ndarray:
    """A^T v in float64, row blocks accumulated in index order (see _matvec)."""
    v = np.asarray(v, dtype=np.float64)
    acc = np.zeros(A.shape[1])
    for i in range(0, A.shape[0], _ROW_BLOCK):
        acc += (A[i:i + _ROW_BLOCK].astype(np.float64) * v[i:i + _ROW_BLOCK, None]).sum(axis=0)
    return acc


def _sparse_truth(rng: np.random.Generator, n: int, frac: float) -> np.ndarray:
    """x_true with exactly round(frac*n) (at least 1) N(0,1) entries at random positions."""
    k = max(1, int(round(frac * n)))
    x = np.zeros(n)
    idx = rng.choice(n, size=k, replace=False)
    x[idx] = rng.standard_normal(k)
    return x


def lasso(m: int, n: int, seed: int, dtype=np.float32, lam_frac: float = 0.1,
          nnz_frac: float = 0.1, noise: float = 0.01, max_iter: int = 10000,
          rng: Optional[np.random.Generator] = None) -> Problem:
    """Lasso in graph form (Appendix A.4 shape): f = 1/2||y - b||^2, g = lam ||x||_1.

    A_ij ~ N(0, 1/n); x_true has round(nnz_frac*n) N(0,1) nonzeros;
    b = A x_true + N(0, noise^2); lam = lam_frac * ||A^T b||_inf.  The data
    are drawn in float64 and A is rounded to ``dtype``; b and lam are formed
    from the rounded A.
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    A = (rng.standard_normal((m, n)) / math.sqrt(n)).astype(dtype)
    x_true = _sparse_truth(rng, n, nnz_frac)
    b = _matvec(A, x_true) + noise * rng.standard_normal(m)
    lam = lam_frac * float(np.max(np.abs(_rmatvec(A, b))))
    f = Fn("square", m, a=1.0, b=b, c=1.0)
    g = Fn("abs", n, c=lam)
    return Problem("lasso", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"lam": lam, "x_true": x_true, "b": b, "seed": seed})


def nnls_from(p: Problem) -> Problem:
    """Non-negative least squares on the data of a Lasso problem (Appendix A.7 form):
    f = 1/2||y - b||^2, g = indicator(x >= 0)."""
    g = Fn("ind_ge0", p.n)
    return Problem("nnls", p.A, p.f, g, p.eps_abs, p.eps_rel, p.max_iter,
                   meta={"b": p.meta["b"], "seed": p.meta.get("seed")})


def dose(m: int, n: int, seed: int, dtype=np.float32, density: float = 0.3,
         w_over: float = 1.0, w_under: float = 0.2, max_iter: int = 10000) -> Problem:
    """Radiation-dose-shaped problem (Section 6.2 form) on synthetic data.

    A_ij = |N(0,1)| kept with probability ``density`` (stored dense);
    target dose t_i ~ U(0.5, 1.5);
    f_i(y) = w_over max(y - t_i, 0) + w_under max(t_i - y, 0)
           = ((w_over + w_under)/2) |y - t_i| + ((w_over - w_under)/2) (y - t_i);
    g = indicator(x >= 0).
    """
    rng = np.random.default_rng(seed)
    A = np.abs(rng.standard_normal((m, n)))
    A *= rng.random((m, n)) < density
    A = A.astype(dtype)
    t = rng.uniform(0.5, 1.5, m)
    cabs = 0.5 * (w_over + w_under)
    lin = 0.5 * (w_over - w_under)
    f = Fn("abs", m, a=1.0, b=t, c=cabs, d=lin, const=-lin * float(t.sum()))
    g = Fn("ind_ge0", n)
    return Problem("dose", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"target": t, "seed": seed})


def logistic(m: int, n: int, seed: int, dtype=np.float32, lam_frac: float = 0.1,
             nnz_frac: float = 0.1, noise: float = 0.01, max_iter: int = 10000,
             rng: Optional[np.random.Generator] = None) -> Problem:
    """l1-regularised logistic regression in graph form (Appendix A.5 form).

    A_ij ~ N(0, 1/n); labels s = sign(A x_true + N(0, noise^2)) in {-1, +1},
    b01 = (1 + s)/2; f_i(y) = log(1 + e^y) - b01_i y; g = lam ||x||_1 with
    lam = lam_frac * ||A^T (1/2 - b01)||_inf.
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    A = (rng.standard_normal((m, n)) / math.sqrt(n)).astype(dtype)
    x_true = _sparse_truth(rng, n, nnz_frac)
    s = np.sign(_matvec(A, x_true) + noise * rng.standard_normal(m))
    s[s == 0] = 1.0
    b01 = 0.5 * (1.0 + s)
    lam = lam_frac * float(np.max(np.abs(_rmatvec(A, 0.5 - b01))))
    f = Fn("logistic", m, a=1.0, b=0.0, c=1.0, d=-b01)
    g = Fn("abs", n, c=lam)
    return Problem("logistic", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"lam": lam, "labels01": b01, "seed": seed})


def svm(m: int, n: int, seed: int, dtype=np.float32, lam: float = 1.0,
        max_iter: int = 10000, rng: Optional[np.random.Generator] = None) -> Problem:
    """Hinge-loss SVM in graph form (Appendix A.9 data).

    Rows of X are two clusters N(+1/n, 1/n) (first half, label +1) and
    N(-1/n, 1/n) (label -1); the label is folded into the matrix, A = diag(s) X,
    so y_i = s_i x_i^T w.  f_i(y) = max(0, 1 - y) (hinge with a = -1, b = -1),
    g = lam ||x||^2 (square with c = 2 lam).
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    half = m // 2
    s = np.where(np.arange(m) < half, 1.0, -1.0)
    X = rng.standard_normal((m, n)) * math.sqrt(1.0 / n) + (s / n)[:, None]
    A = (s[:, None] * X).astype(dtype)
    f = Fn("hinge", m, a=-1.0, b=-1.0, c=1.0)
    g = Fn("square", n, c=2.0 * lam)
    return Problem("svm", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"lam": lam, "seed": seed})


def lp(m: int, n: int, seed: int, dtype=np.float32, max_iter: int = 10000,
       rng: Optional[np.random.Generator] = None) -> Problem:
    """Box-bounded linear program: minimize c^T x s.t. A x <= b, 0 <= x <= 1.

    A_ij ~ N(0,1); v ~ U[0,1]^n; b = A v + U[0, 0.1] (Appendix A.6 noise), so
    v is strictly feasible; cost c ~ U[0,1]^n (c >= 0).  Graph form:
    f = indicator(y - b <= 0), g_j = indicator(0 <= x_j <= 1) + c_j x_j.
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    A = rng.standard_normal((m, n)).astype(dtype)
    v = rng.random(n)
    b = _matvec(A, v) + rng.uniform(0.0, 0.1, m)
    cost = rng.random(n)
    f = Fn("ind_le0", m, a=1.0, b=b)
    g = Fn("ind_box01", n, d=cost)
    return Problem("lp", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"b": b, "cost": cost, "seed": seed})


def basis_pursuit(m: int, n: int, seed: int, dtype=np.float32, max_iter: int = 10000,
                  rng: Optional[np.random.Generator] = None) -> Problem:
    """Basis pursuit (Appendix A.1): minimize ||x||_1 s.t. A x = b.

    A_ij ~ N(0,1); v_j = 0 with probability 1/2, else N(0, 1/n); b = A v
    (from the rounded A).  Graph form: f = indicator(y = b), g = ||x||_1.
    The appendix draws m > n, where A v = b has the single solution v; any
    shape is accepted.
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    A = rng.standard_normal((m, n)).astype(dtype)
    v = np.where(rng.random(n) < 0.5, 0.0, rng.standard_normal(n) / math.sqrt(n))
    b = _matvec(A, v)
    f = Fn("ind_eq0", m, a=1.0, b=b)
    g = Fn("abs", n)
    return Problem("basis_pursuit", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"b": b, "v": v, "seed": seed})


def entropy_max(m: int, n: int, seed: int, dtype=np.float32, max_iter: int = 10000,
                rng: Optional[np.random.Generator] = None) -> Problem:
    """Entropy maximization (Appendix A.2): maximize -sum x log x s.t.
    1^T x = 1, F x <= b.

    F_ij ~ N(0, n) (variance n); v_j ~ U[0,1]; b = F v / (1^T v), so
    x = v / (1^T v) is feasible.  Graph form on A = [F; 1^T] ((m+1) x n):
    f_i = indicator(y_i <= b_i) for i < m, f_m = indicator(y_m = 1),
    g_j = x_j log x_j.  The appendix draws m < n.
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    F = rng.standard_normal((m, n)) * math.sqrt(n)
    v = rng.random(n)
    A = np.vstack([F, np.ones((1, n))]).astype(dtype)
    b = _matvec(A[:m], v) / v.sum()
    h = ["ind_le0"] * m + ["ind_eq0"]
    f = Fn(h, m + 1, a=1.0, b=np.append(b, 1.0))
    g = Fn("neg_entr", n)
    return Problem("entropy_max", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"b": b, "v": v, "seed": seed})


def huber_fit(m: int, n: int, seed: int, dtype=np.float32, max_iter: int = 10000,
              rng: Optional[np.random.Generator] = None) -> Problem:
    """Huber fitting (Appendix A.3): minimize sum_i huber(b_i - a_i^T x).

    A_ij ~ N(0, n) (variance n); v_j ~ N(0, 1/n); eps_i ~ N(0, 1/4) with
    probability 0.95, else U[0, 10]; b = A v + eps (from the rounded A).
    Graph form: f_i(y) = huber(b_i - y) (h = huber with a = -1, b = -b_i),
    g = 0.  The appendix draws m > n.
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    A = (rng.standard_normal((m, n)) * math.sqrt(n)).astype(dtype)
    v = rng.standard_normal(n) / math.sqrt(n)
    outlier = rng.random(m) >= 0.95
    eps = np.where(outlier, rng.uniform(0.0, 10.0, m), 0.5 * rng.standard_normal(m))
    b = _matvec(A, v) + eps
    f = Fn("huber", m, a=-1.0, b=-b)
    g = Fn("zero", n)
    return Problem("huber_fit", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"b": b, "v": v, "seed": seed})


def portfolio(k: int, n: int, seed: int, dtype=np.float32, gamma: float = 1.0,
              max_iter: int = 10000, rng: Optional[np.random.Generator] = None) -> Problem:
    """Portfolio optimization with a k-factor risk model (Appendix A.8):
    maximize mu^T x - gamma x^T (F F^T + D) x s.t. x >= 0, 1^T x = 1.

    F_ij ~ N(0,1) (n x k); D_jj ~ U[0, sqrt(k)]; mu_j ~ N(0,1).  Graph form
    on A = [F^T; 1^T] ((k+1) x n): f_i = gamma y_i^2 (square with c = 2 gamma)
    for i < k, f_k = indicator(y_k = 1); g_j = -mu_j x_j + gamma D_jj x_j^2 +
    indicator(x_j >= 0) (ind_ge0 with d = -mu_j, e = 2 gamma D_jj).  The
    appendix draws n > k.
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    F = rng.standard_normal((n, k))
    Dg = rng.uniform(0.0, math.sqrt(k), n)
    mu = rng.standard_normal(n)
    A = np.vstack([F.T, np.ones((1, n))]).astype(dtype)
    h = ["square"] * k + ["ind_eq0"]
    c = np.append(np.full(k, 2.0 * gamma), 1.0)
    f = Fn(h, k + 1, a=1.0, b=np.append(np.zeros(k), 1.0), c=c)
    g = Fn("ind_ge0", n, d=-mu, e=2.0 * gamma * Dg)
    return Problem("portfolio", np.ascontiguousarray(A), f, g, max_iter=max_iter,
                   meta={"mu": mu, "D": Dg, "F": A[:k].astype(np.float64).T, "gamma": gamma,
                         "seed": seed})


def sparse_matrix(m: int, n: int, k: int, rng: np.random.Generator, dtype=np.float32):
    """m x n matrix in compressed rows (SciPy CSR): each row draws k column
    indices uniformly with replacement and values N(0, 1/k); repeated columns
    of a row are merged (summed), so a row has at most k entries, sorted."""
    import scipy.sparse as sp
    k = min(k, n)
    cols = rng.integers(0, n, size=(m, k), dtype=np.int64)
    vals = rng.standard_normal((m, k)) / math.sqrt(k)
    indptr = np.arange(0, m * k + 1, k, dtype=np.int64)
    A = sp.csr_matrix((vals.ravel(), cols.ravel(), indptr), shape=(m, n))
    A.sum_duplicates()
    return A.astype(dtype)


def sparse_problem(kind: str, m: int, n: int, k: int, seed: int, dtype=np.float32,
                   max_iter: int = 10000) -> Problem:
    """A problem of the given kind (lasso, nnls, logistic, lp) on a sparse A
    with k entries per row (sparse_matrix); the functions follow the dense
    generators' recipes with A^T b etc. formed from the rounded sparse A.
    ``Problem.A`` is the SciPy CSR matrix."""
    rng = np.random.default_rng(seed)
    A = sparse_matrix(m, n, k, rng, dtype)
    A64 = A.astype(np.float64)
    if kind in ("lasso", "nnls"):
        x_true = _sparse_truth(rng, n, 0.1)
        b = A64 @ x_true + 0.01 * rng.standard_normal(m)
        f = Fn("square", m, a=1.0, b=b, c=1.0)
        if kind == "lasso":
            g = Fn("abs", n, c=0.1 * float(np.max(np.abs(A64.T @ b))))
        else:
            g = Fn("ind_ge0", n)
        meta = {"b": b}
    elif kind == "logistic":
        x_true = _sparse_truth(rng, n, 0.1)
        sgn = np.sign(A64 @ x_true + 0.01 * rng.standard_normal(m))
        sgn[sgn == 0] = 1.0
        b01 = 0.5 * (1.0 + sgn)
        f = Fn("logistic", m, d=-b01)
        g = Fn("abs", n, c=0.1 * float(np.max(np.abs(A64.T @ (0.5 - b01)))))
        meta = {"labels01": b01}
    elif kind == "lp":
        v = rng.random(n)
        b = A64 @ v + rng.uniform(0.0, 0.1, m)
        f = Fn("ind_le0", m, b=b)
        g = Fn("ind_box01", n, d=rng.random(n))
        meta = {"b": b}
    else:
        raise ValueError(kind)
    meta.update({"seed": seed, "nnz_per_row": k})
    return Problem(f"sparse_{kind}", A, f, g, max_iter=max_iter, meta=meta)


# ---------------------------------------------------------------------------
# Named benchmark workloads
# ---------------------------------------------------------------------------

def lasso_small_f64(seed: int = 0) -> Problem:
    """Lasso 200 x 100 in float64, at most 2000 iterations."""
    return lasso(200, 100, seed, dtype=np.float64, max_iter=2000)


def lasso_20000x2000(seed: int = 1) -> Problem:
    return lasso(20000, 2000, seed, dtype=np.float32)


def nnls_20000x2000(seed: int = 1) -> Problem:
    return nnls_from(lasso_20000x2000(seed))


def dose_100000x1000(seed: int = 2) -> Problem:
    return dose(100000, 1000, seed)


def batch_mix(count: int = 512, seed: int = 3, m_range=(64, 4096), n_range=(32, 1024),
              dtype=np.float32) -> List[Problem]:
    """Independent problems of uneven shape: even index Lasso, odd index logistic.

    m ~ U{m_range}, n ~ U{n_range} (inclusive), each problem drawn from its own
    child seed.
    """
    ss = np.random.SeedSequence(seed)
    return [_batch_member(child, i, m_range, n_range, dtype) for i, child in enumerate(ss.spawn(count))]


def batch_member(index: int, count: int = 512, seed: int = 3, m_range=(64, 4096), n_range=(32, 1024),
                 dtype=np.float32) -> Problem:
    """Problem ``index`` of ``batch_mix(count, seed, ...)`` drawn alone (the same data)."""
    child = np.random.SeedSequence(seed).spawn(count)[index]
    return _batch_member(child, index, m_range, n_range, dtype)


def _batch_member(child, i, m_range, n_range, dtype) -> Problem:
    rng = np.random.default_rng(child)
    m = int(rng.integers(m_range[0], m_range[1] + 1))
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    if i % 2 == 0:
        p = lasso(m, n, 0, dtype=dtype, rng=rng)
    else:
        p = logistic(m, n, 0, dtype=dtype, rng=rng)
    p.meta["index"] = i
    return p


def lambda_path(m: int = 8000, n: int = 1000, R: int = 64, seed: int = 33,
                dtype=np.float32, lo: float = 1e-3, hi: float = 1.0) -> List[Problem]:
    """R Lasso problems sharing one A and b, lam_r = lam_max * 10^(log10(lo) + r (log10(hi/lo))/(R-1)).

    lam_max = ||A^T b||_inf, so the last point (lam = lam_max) has x* = 0.
    """
    base = lasso(m, n, seed, dtype=dtype)
    lam_max = float(np.max(np.abs(_rmatvec(base.A, base.meta["b"]))))
    if R == 1:
        lams = np.array([lo * lam_max])
    else:
        lams = lam_max * 10.0 ** np.linspace(math.log10(lo), math.log10(hi), R)
    out = []
    for r, lam in enumerate(lams):
        g = Fn("abs", n, c=float(lam))
        out.append(Problem("lasso_path", base.A, base.f, g, max_iter=base.max_iter,
                           meta={"lam": float(lam), "r": r, "b": base.meta["b"]}))
    return out


def serving_request(rng: np.random.Generator, m_range=(100, 50000), n_range=(50, 5000),
                    kinds: Sequence[str] = ("lasso", "nnls", "svm", "lp"),
                    dtype=np.float32) -> Problem:
    """One request of the mixed serving workload: kind uniform over ``kinds``,
    m = floor(exp U[ln m_lo, ln m_hi]), n likewise."""
    kind = kinds[int(rng.integers(len(kinds)))]
    m = int(math.floor(math.exp(rng.uniform(math.log(m_range[0]), math.log(m_range[1])))))
    n = int(math.floor(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
    if kind == "lasso":
        return lasso(m, n, 0, dtype=dtype, rng=rng)
    if kind == "nnls":
        return nnls_from(lasso(m, n, 0, dtype=dtype, rng=rng))
    if kind == "svm":
        return svm(m, n, 0, dtype=dtype, rng=rng)
    if kind == "lp":
        return lp(m, n, 0, dtype=dtype, rng=rng)
    raise ValueError(kind)


def serving_stream(count: int, qps: float, seed: int = 4, **kw) -> Iterator[tuple]:
    """Yield (arrival_time_s, Problem) with Poisson arrivals at rate ``qps``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    for _ in range(count):
        t += float(rng.exponential(1.0 / qps))
        yield t, serving_request(rng, **kw)


def fingerprint(p: Problem) -> str:
    """Digest of a problem's inputs (shape, storage type, column sums of A in
    float64, every function parameter): a stored result is used only for the
    inputs it was computed on."""
    import hashlib
    h = hashlib.sha256()
    h.update(f"{p.m}x{p.n}:{p.A.dtype.str}:{p.eps_abs}:{p.eps_rel}:{p.max_iter}".encode())
    h.update(np.ascontiguousarray(p.A.sum(axis=0, dtype=np.float64)).tobytes())
    h.update(np.ascontiguousarray(p.A[:, 0], dtype=np.float64).tobytes())
    for fn in (p.f, p.g):
        names = [fn.h] if isinstance(fn.h, str) else list(fn.h)
        h.update(",".join(names).encode())
        for k in "abcde":
            h.update(fn.field(k).tobytes())
    return h.hexdigest()[:24]
