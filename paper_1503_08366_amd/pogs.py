"""ctypes binding to libpogs.so (the C ABI declared in include/pogs.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  Host inputs are NumPy arrays; device inputs/outputs are torch
CUDA (ROCm) tensors, whose data pointers and the current torch stream are
handed to the library.  If libpogs.so is missing, loading raises: there is no
fallback.

Functions carry the C names (``pogs_init``, ``pogs_solve``, ...); ``Context``
wraps a ``pogs_ctx`` handle.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpogs.so")

# --- constants of include/pogs.h ------------------------------------------
POGS_OK, POGS_EINVAL, POGS_ENOMEM, POGS_EDEVICE, POGS_EAGAIN, POGS_ENOTFOUND, POGS_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
POGS_ETOOBIG = -7
POGS_NOALLOC_SCRATCH_BYTES = 64 << 20
POGS_CONVERGED, POGS_MAXITER, POGS_NUMERICAL, POGS_CANCELLED, POGS_FAILED = 0, 1, 2, 3, 4
POGS_F32, POGS_F64 = 0, 1
POGS_ROW_MAJOR, POGS_COL_MAJOR = 0, 1
POGS_HOST, POGS_DEVICE = 0, 1
H_CODES = {"zero": 0, "identity": 1, "abs": 2, "square": 3, "huber": 4, "hinge": 5,
           "logistic": 6, "ind_ge0": 7, "ind_le0": 8, "ind_eq0": 9, "ind_box01": 10,
           "exp": 11, "neg_entr": 12, "neg_log": 13, "recipr": 14, "max_neg0": 15}
STATUS_NAMES = {0: "converged", 1: "maxiter", 2: "numerical", 3: "cancelled", 4: "failed"}


class PogsError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {_lib().pogs_strerror(code).decode()} ({code})")


class pogs_fn(C.Structure):
    _fields_ = [("len", C.c_int64), ("stride", C.c_int64), ("h", C.POINTER(C.c_uint8)),
                ("a", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)),
                ("c", C.POINTER(C.c_double)), ("d", C.POINTER(C.c_double)),
                ("e", C.POINTER(C.c_double))]


class pogs_params(C.Structure):
    _fields_ = [("eps_abs", C.c_double), ("eps_rel", C.c_double), ("max_iter", C.c_int32),
                ("rho0", C.c_double), ("alpha", C.c_double), ("delta", C.c_double),
                ("tau", C.c_double), ("adaptive_rho", C.c_int32), ("equil_iters", C.c_int32),
                ("eps_cmp", C.c_double), ("chunk_iters", C.c_int32), ("verbose", C.c_int32),
                ("projection", C.c_int32), ("cg_max_iter", C.c_int32), ("cg_tol", C.c_double),
                ("stop_rule", C.c_int32), ("autotune", C.c_int32), ("sparse_segment", C.c_int32)]


class pogs_result(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("mu", C.c_void_p), ("nu", C.c_void_p),
                ("mem", C.c_int), ("optval", C.c_double), ("r_pri", C.c_double),
                ("r_dual", C.c_double), ("eps_pri", C.c_double), ("eps_dual", C.c_double),
                ("rho", C.c_double), ("iters", C.c_int32), ("status", C.c_int32),
                ("ms_setup", C.c_double), ("ms_solve", C.c_double), ("cg_steps", C.c_int32),
                ("error", C.c_int32), ("gap", C.c_double), ("eps_gap", C.c_double)]


class pogs_problem(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("A", C.c_void_p), ("dt", C.c_int),
                ("ord", C.c_int), ("lda", C.c_int64), ("f", pogs_fn), ("g", pogs_fn),
                ("params", pogs_params)]


class pogs_batch_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("chunk_iters", C.c_int32), ("stream", C.c_void_p)]


_LIB = None

# every symbol of include/pogs.h with (restype, argtypes)
_SIGS = {
    "pogs_strerror": (C.c_char_p, [C.c_int]),
    "pogs_params_default": (C.c_int, [C.POINTER(pogs_params)]),
    "pogs_init": (C.c_int, [C.POINTER(C.c_void_p), C.c_int64, C.c_int64, C.c_void_p, C.c_int, C.c_int,
                            C.c_int64, C.c_int, C.POINTER(pogs_params), C.c_void_p]),
    "pogs_init_sparse": (C.c_int, [C.POINTER(C.c_void_p), C.c_int64, C.c_int64, C.c_int64, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.POINTER(pogs_params),
                                   C.c_void_p]),
    "pogs_solve": (C.c_int, [C.c_void_p, C.POINTER(pogs_fn), C.POINTER(pogs_fn), C.POINTER(pogs_params),
                             C.c_void_p, C.c_void_p, C.POINTER(pogs_result)]),
    "pogs_solve_path": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(pogs_fn), C.POINTER(pogs_fn),
                                  C.POINTER(pogs_params), C.POINTER(pogs_result)]),
    "pogs_free": (C.c_int, [C.c_void_p]),
    "pogs_get_scaling": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pogs_project": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pogs_prox": (C.c_int, [C.POINTER(pogs_fn), C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_int,
                            C.c_void_p]),
    "pogs_prox_noalloc": (C.c_int, [C.POINTER(pogs_fn), C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "pogs_profile_iteration": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "pogs_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(pogs_batch_cfg)]),
    "pogs_batch_submit": (C.c_int, [C.c_void_p, C.POINTER(pogs_problem), C.POINTER(C.c_uint64)]),
    "pogs_batch_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(pogs_result)]),
    "pogs_batch_wait_all": (C.c_int, [C.c_void_p]),
    "pogs_batch_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "pogs_batch_destroy": (C.c_int, [C.c_void_p]),
    "pogs_solve_batch": (C.c_int, [C.c_int32, C.POINTER(pogs_problem), C.POINTER(pogs_result), C.c_void_p]),
}


def _init_torch_first():
    """torch's ROCm wheel carries its own HIP runtime; it must initialise the
    device before libpogs's runtime does, or torch later reports no GPU."""
    try:
        import torch
    except ImportError:
        return
    try:
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (python -m paper_1503_08366_amd.build)")
        _init_torch_first()
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def load() -> C.CDLL:
    """Load libpogs.so (raises if it is missing) and return the handle."""
    return _lib()


def _check(rc: int, what: str):
    if rc != POGS_OK:
        raise PogsError(rc, what)


# --- marshalling helpers -----------------------------------------------------

PROJECTIONS = {"direct": 0, "cgls": 1}
STOP_RULES = {"residual": 0, "gap": 1}


def default_params(**overrides) -> pogs_params:
    """pogs_params_default with fields overridden by keyword; projection and
    stop_rule may be given by name ("direct", "cgls"; "residual", "gap")."""
    p = pogs_params()
    _check(_lib().pogs_params_default(C.byref(p)), "pogs_params_default")
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k == "projection" and isinstance(v, str):
            v = PROJECTIONS[v]
        if k == "stop_rule" and isinstance(v, str):
            v = STOP_RULES[v]
        setattr(p, k, v)
    return p


class _FnHolder:
    """Keeps the arrays behind a pogs_fn alive for the duration of a call."""

    def __init__(self, fn, length: int):
        if fn.size != length:
            raise ValueError(f"function has length {fn.size}, expected {length}")
        if isinstance(fn.h, str):
            self.h = np.full(length, H_CODES[fn.h], dtype=np.uint8)
        else:
            self.h = np.array([H_CODES[n] for n in fn.h], dtype=np.uint8)
        # a parameter that is its default everywhere goes as NULL (the library
        # fills the default), so no array is built for it
        self.arrs = [None if _is_default(fn, k) else np.ascontiguousarray(fn.field(k), dtype=np.float64)
                     for k in "abcde"]
        dp = C.POINTER(C.c_double)
        self.s = pogs_fn(length, 1, self.h.ctypes.data_as(C.POINTER(C.c_uint8)),
                         *(dp() if a is None else a.ctypes.data_as(dp) for a in self.arrs))


_DEFAULTS = {"a": 1.0, "b": 0.0, "c": 1.0, "d": 0.0, "e": 0.0}

# pogs_fn as a numpy record, for calls that take many descriptors at once
_FN_RECORD = np.dtype([("len", np.int64), ("stride", np.int64), ("h", np.uintp), ("a", np.uintp),
                       ("b", np.uintp), ("c", np.uintp), ("d", np.uintp), ("e", np.uintp)])
assert _FN_RECORD.itemsize == C.sizeof(pogs_fn)


class _FnTable:
    """Descriptors of functions of one length as one record array laid out as
    an array of pogs_fn (stride 1; NULL for default parameters), with the
    arrays behind them kept alive for the duration of a call.  Functions with
    the same single base function share one array of codes."""

    def __init__(self, fns, length: int):
        R = len(fns)
        cols = {k: [0] * R for k in "habcde"}
        self.keep, codes = [], {}
        for i, fn in enumerate(fns):
            if fn.size != length:
                raise ValueError(f"function has length {fn.size}, expected {length}")
            if isinstance(fn.h, str):
                h = codes.get(fn.h)
                if h is None:
                    h = codes[fn.h] = np.full(length, H_CODES[fn.h], dtype=np.uint8)
            else:
                h = np.array([H_CODES[n] for n in fn.h], dtype=np.uint8)
            self.keep.append(h)
            cols["h"][i] = h.ctypes.data
            for k in "abcde":
                if not _is_default(fn, k):
                    arr = np.ascontiguousarray(fn.field(k), dtype=np.float64)
                    self.keep.append(arr)
                    cols[k][i] = arr.ctypes.data
        self.t = np.zeros(R, dtype=_FN_RECORD)
        self.t["len"] = length
        self.t["stride"] = 1
        for k, v in cols.items():
            self.t[k] = v
        self.ptr = self.t.ctypes.data_as(C.POINTER(pogs_fn))


def _is_default(fn, k: str) -> bool:
    v = getattr(fn, k, None)
    if isinstance(v, (float, int, np.generic)):  # the common case, without np.ndim
        return float(v) == _DEFAULTS[k]
    return v is not None and np.ndim(v) == 0 and float(v) == _DEFAULTS[k]


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _dtype_code(x) -> int:
    if _is_torch(x):
        import torch
        if x.dtype == torch.float32:
            return POGS_F32
        if x.dtype == torch.float64:
            return POGS_F64
        raise TypeError(x.dtype)
    if x.dtype == np.float32:
        return POGS_F32
    if x.dtype == np.float64:
        return POGS_F64
    raise TypeError(x.dtype)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _np_dtype(code: int):
    return np.float32 if code == POGS_F32 else np.float64


class Result:
    """Host copy of a pogs_result plus the returned vectors."""

    def __init__(self, r: pogs_result, x, y, mu, nu):
        self.x, self.y, self.mu, self.nu = x, y, mu, nu
        self.optval = r.optval
        self.r_pri, self.r_dual = r.r_pri, r.r_dual
        self.eps_pri, self.eps_dual = r.eps_pri, r.eps_dual
        self.rho = r.rho
        self.iters = r.iters
        self.status = r.status
        self.ms_setup, self.ms_solve = r.ms_setup, r.ms_solve
        self.cg_steps = r.cg_steps
        self.gap, self.eps_gap = r.gap, r.eps_gap
        self.error = r.error

    @property
    def converged(self) -> bool:
        return self.status == POGS_CONVERGED

    def __repr__(self):
        return (f"Result(status={STATUS_NAMES.get(self.status, self.status)}, iters={self.iters}, "
                f"optval={self.optval:.6g}, r_pri={self.r_pri:.3g}/{self.eps_pri:.3g}, "
                f"r_dual={self.r_dual:.3g}/{self.eps_dual:.3g})")


# --- C-named entry points ------------------------------------------------------

def pogs_init(A, params: Optional[pogs_params] = None, stream=None) -> "Context":
    """Create a context for A: a NumPy array (host) or a torch CUDA tensor
    (device), 2-D, float32 or float64, C- or F-contiguous."""
    return Context(A, params, stream)


def pogs_solve(ctx: "Context", f, g, params: Optional[pogs_params] = None, device_out: bool = False):
    return ctx.solve(f, g, params, device_out=device_out)


def pogs_free(ctx: "Context"):
    ctx.free()


def pogs_prox(fn, v, rho: float, stream=None):
    """prox_{fn,rho}(v) evaluated on the device; v NumPy (host) or torch CUDA tensor."""
    holder = _FnHolder(fn, len(v))
    dt = _dtype_code(v)
    if _is_torch(v):
        import torch
        v = v.contiguous()
        out = torch.empty_like(v)
        s = _stream_handle(stream if stream is not None else torch.cuda.current_stream())
        _check(_lib().pogs_prox(C.byref(holder.s), dt, float(rho), C.c_void_p(v.data_ptr()),
                                C.c_void_p(out.data_ptr()), POGS_DEVICE, s), "pogs_prox")
        return out
    v = np.ascontiguousarray(v)
    out = np.empty_like(v)
    _check(_lib().pogs_prox(C.byref(holder.s), dt, float(rho), v.ctypes.data_as(C.c_void_p),
                            out.ctypes.data_as(C.c_void_p), POGS_HOST, _stream_handle(stream)), "pogs_prox")
    return out


def pogs_prox_noalloc(fn, v, rho: float, out, stream=None):
    """prox_{fn,rho}(v) into the caller's tensor ``out`` through the entry point
    that allocates no device memory (v, out: torch CUDA tensors of one dtype,
    contiguous, len(fn) entries).  Returns ``out``."""
    import torch
    if not (_is_torch(v) and _is_torch(out) and v.is_cuda and out.is_cuda):
        raise TypeError("pogs_prox_noalloc takes torch CUDA tensors")
    if v.dtype != out.dtype or v.numel() != out.numel() or not v.is_contiguous() or not out.is_contiguous():
        raise ValueError("v and out must be contiguous tensors of one dtype and length")
    holder = _FnHolder(fn, v.numel())
    s = _stream_handle(stream if stream is not None else torch.cuda.current_stream())
    _check(_lib().pogs_prox_noalloc(C.byref(holder.s), _dtype_code(v), float(rho), C.c_void_p(v.data_ptr()),
                                    C.c_void_p(out.data_ptr()), s), "pogs_prox_noalloc")
    return out


class Context:
    """A pogs_ctx: the scaled matrix, D, E and the cached factor on the device."""

    def __init__(self, A, params: Optional[pogs_params] = None, stream=None):
        lib = _lib()
        if A.ndim != 2:
            raise ValueError("A must be 2-D")
        m, n = int(A.shape[0]), int(A.shape[1])
        self.dtype = _dtype_code(A)
        self.m, self.n = m, n
        if _is_torch(A):
            st = A.stride()
            if st[1] == 1:
                order, lda = POGS_ROW_MAJOR, st[0]
            elif st[0] == 1:
                order, lda = POGS_COL_MAJOR, st[1]
            else:
                A = A.contiguous()
                order, lda = POGS_ROW_MAJOR, n
            ptr, mem = A.data_ptr(), POGS_DEVICE
            if stream is None:
                import torch
                stream = torch.cuda.current_stream()
        else:
            A, order, lda = _host_layout(A)
            ptr, mem = A.ctypes.data, POGS_HOST
        self.stream = stream
        self.projection = int(params.projection) if params is not None else 0
        handle = C.c_void_p()
        rc = lib.pogs_init(C.byref(handle), m, n, C.c_void_p(ptr), self.dtype, order, lda, mem,
                           C.byref(params) if params is not None else None, _stream_handle(stream))
        _check(rc, "pogs_init")
        self.handle = handle

    def _h(self):
        if not self.handle:
            raise RuntimeError("context freed")
        return self.handle

    def free(self):
        if getattr(self, "handle", None):
            _lib().pogs_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    def solve(self, f, g, params: Optional[pogs_params] = None, device_out: bool = False,
              x0=None, nu0=None) -> Result:
        """Solve; x0 (n) and nu0 (m) warm-start the iteration (original
        variables; NumPy arrays, or torch device tensors with device_out)."""
        fh, gh = _FnHolder(f, self.m), _FnHolder(g, self.n)
        r = pogs_result()
        npdt = _np_dtype(self.dtype)
        keep = []

        def _warm(v, k):
            if v is None:
                return None
            if device_out:
                import torch
                tdt = torch.float32 if self.dtype == POGS_F32 else torch.float64
                t = torch.as_tensor(v).to(device="cuda", dtype=tdt).contiguous()
                if t.numel() != k:
                    raise ValueError("warm-start vector has the wrong length")
                keep.append(t)
                return C.c_void_p(t.data_ptr())
            a = np.ascontiguousarray(v, dtype=npdt)
            if a.size != k:
                raise ValueError("warm-start vector has the wrong length")
            keep.append(a)
            return a.ctypes.data_as(C.c_void_p)
        if device_out:
            import torch
            tdt = torch.float32 if self.dtype == POGS_F32 else torch.float64
            outs = [torch.empty(k, dtype=tdt, device="cuda") for k in (self.n, self.m, self.n, self.m)]
            r.x, r.y, r.mu, r.nu = (o.data_ptr() for o in outs)
            r.mem = POGS_DEVICE
        else:
            outs = [np.empty(k, dtype=npdt) for k in (self.n, self.m, self.n, self.m)]
            r.x, r.y, r.mu, r.nu = (o.ctypes.data for o in outs)
            r.mem = POGS_HOST
        wx, wnu = _warm(x0, self.n), _warm(nu0, self.m)
        rc = _lib().pogs_solve(self._h(), C.byref(fh.s), C.byref(gh.s),
                               C.byref(params) if params is not None else None, wx, wnu, C.byref(r))
        _check(rc, "pogs_solve")
        return Result(r, *outs)

    def solve_path(self, fs: Sequence, gs: Sequence, params: Optional[pogs_params] = None) -> List[Result]:
        R = len(fs)
        if len(gs) != R:
            raise ValueError(f"{R} functions f but {len(gs)} functions g")
        ft, gt = _FnTable(fs, self.m), _FnTable(gs, self.n)
        res = (pogs_result * R)()
        m, n = self.m, self.n
        # x, y, mu, nu of every problem in one host block, a row per problem
        blk = np.empty((R, 2 * (m + n)), dtype=_np_dtype(self.dtype))
        base, row, size = blk.ctypes.data, blk.strides[0], blk.itemsize
        offs = (0, n * size, (n + m) * size, (2 * n + m) * size)
        for r in range(R):
            a = base + r * row
            res[r].x, res[r].y, res[r].mu, res[r].nu = (a + o for o in offs)
            res[r].mem = POGS_HOST
        rc = _lib().pogs_solve_path(self._h(), R, ft.ptr, gt.ptr, C.byref(params) if params is not None else None, res)
        _check(rc, "pogs_solve_path")
        return [Result(res[r], blk[r, :n], blk[r, n:n + m], blk[r, n + m:2 * n + m], blk[r, 2 * n + m:])
                for r in range(R)]

    def solve_continuation(self, fs: Sequence, gs: Sequence, params: Optional[pogs_params] = None) -> List[Result]:
        """Solve a sequence of problems on this matrix (e.g. a lambda path),
        each warm-started from the previous one's (x, nu)."""
        out = []
        prev = None
        for f, g in zip(fs, gs):
            r = self.solve(f, g, params, x0=None if prev is None else prev.x,
                           nu0=None if prev is None else prev.nu)
            out.append(r)
            prev = r
        return out

    def profile_iteration(self, reps: int = 50):
        """Average ms of a full iteration and of each part of it (HIP events):
        prox, pass1, solve, pass2 (direct projection) or prox, first (the two
        passes that start a projection), cg_step (a context set up for CGLS)."""
        ms = (C.c_double * 5)()
        _check(_lib().pogs_profile_iteration(self._h(), reps, ms), "pogs_profile_iteration")
        if self.projection == PROJECTIONS["cgls"]:
            return {"iteration": ms[0], "prox": ms[1], "first": ms[2], "cg_step": ms[3]}
        return {"iteration": ms[0], "prox": ms[1], "pass1": ms[2], "solve": ms[3], "pass2": ms[4]}

    def scaling(self):
        D = np.empty(self.m)
        E = np.empty(self.n)
        _check(_lib().pogs_get_scaling(self._h(), D.ctypes.data_as(C.c_void_p), E.ctypes.data_as(C.c_void_p),
                                       POGS_HOST), "pogs_get_scaling")
        return D, E

    def project(self, c, d):
        """Projection onto the graph of the scaled matrix D A E."""
        if _is_torch(c):
            import torch
            x = torch.empty_like(c)
            y = torch.empty_like(d)
            _check(_lib().pogs_project(self._h(), C.c_void_p(c.data_ptr()), C.c_void_p(d.data_ptr()),
                                       C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), POGS_DEVICE),
                   "pogs_project")
            return x, y
        npdt = _np_dtype(self.dtype)
        c = np.ascontiguousarray(c, dtype=npdt)
        d = np.ascontiguousarray(d, dtype=npdt)
        x = np.empty(self.n, dtype=npdt)
        y = np.empty(self.m, dtype=npdt)
        _check(_lib().pogs_project(self._h(), c.ctypes.data_as(C.c_void_p), d.ctypes.data_as(C.c_void_p),
                                   x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p), POGS_HOST),
               "pogs_project")
        return x, y



class SparseContext(Context):
    """A pogs_ctx on a sparse matrix in compressed rows (pogs_init_sparse).

    ``A`` is anything with ``indptr``, ``indices``, ``data`` and ``shape``
    (a SciPy CSR matrix, or a torch sparse CSR tensor on the device for
    device input).  Solves project by CGLS."""

    def __init__(self, A, params: Optional[pogs_params] = None, stream=None):
        lib = _lib()
        if _is_torch(A):
            import torch
            rp = A.crow_indices().to(torch.int64).contiguous()
            ci = A.col_indices().to(torch.int32).contiguous()
            va = A.values().contiguous()
            keep = (rp, ci, va)
            ptrs = (rp.data_ptr(), ci.data_ptr(), va.data_ptr())
            mem = POGS_DEVICE
            dt = _dtype_code(va)
            if stream is None:
                stream = torch.cuda.current_stream()
        else:
            rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
            ci = np.ascontiguousarray(A.indices, dtype=np.int32)
            va = np.ascontiguousarray(A.data)
            if va.dtype not in (np.float32, np.float64):
                va = va.astype(np.float64)
            keep = (rp, ci, va)
            ptrs = (rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
            mem = POGS_HOST
            dt = POGS_F32 if va.dtype == np.float32 else POGS_F64
        m, n = int(A.shape[0]), int(A.shape[1])
        self.dtype = dt
        self.m, self.n = m, n
        self.stream = stream
        self.projection = PROJECTIONS["cgls"]
        self.nnz = int(len(keep[1]))
        handle = C.c_void_p()
        rc = lib.pogs_init_sparse(C.byref(handle), m, n, self.nnz, C.c_void_p(ptrs[0]), C.c_void_p(ptrs[1]),
                                  C.c_void_p(ptrs[2]), dt, mem, C.byref(params) if params is not None else None,
                                  _stream_handle(stream))
        _check(rc, "pogs_init_sparse")
        self.handle = handle


def _host_layout(A):
    """(array, order, lda) of a host matrix: row-major or column-major with a
    padded leading dimension goes as it is (the library packs it on upload),
    any other layout is copied to row-major first."""
    it = A.itemsize
    m, n = A.shape
    s0, s1 = A.strides
    if s1 == it and s0 > 0 and s0 % it == 0 and s0 // it >= n:
        return A, POGS_ROW_MAJOR, s0 // it
    if s0 == it and s1 > 0 and s1 % it == 0 and s1 // it >= m:
        return A, POGS_COL_MAJOR, s1 // it
    return np.ascontiguousarray(A), POGS_ROW_MAJOR, n


def _problem_struct(p, params: Optional[pogs_params], keep: list) -> pogs_problem:
    A = np.asarray(p.A)
    if A.dtype != np.float32:
        raise TypeError("batched problems take float32 matrices")
    A, order, lda = _host_layout(A)
    fh, gh = _FnHolder(p.f, A.shape[0]), _FnHolder(p.g, A.shape[1])
    keep.extend([A, fh, gh])
    prm = params if params is not None else default_params(eps_abs=p.eps_abs, eps_rel=p.eps_rel,
                                                           max_iter=p.max_iter)
    return pogs_problem(A.shape[0], A.shape[1], A.ctypes.data, POGS_F32, order, lda, fh.s, gh.s, prm)


def _host_outputs(m: int, n: int, r: pogs_result, keep: list):
    o = [np.empty(k, dtype=np.float32) for k in (n, m, n, m)]
    r.x, r.y, r.mu, r.nu = (a.ctypes.data for a in o)
    r.mem = POGS_HOST
    keep.append(o)
    return o


def pogs_solve_batch(problems: Sequence, params: Optional[pogs_params] = None, stream=None) -> List[Result]:
    """Solve independent problems (workload ``Problem`` objects) in one batched call."""
    keep: list = []
    N = len(problems)
    arr = (pogs_problem * N)(*(_problem_struct(p, params, keep) for p in problems))
    res = (pogs_result * N)()
    outs = [_host_outputs(p.m, p.n, res[i], keep) for i, p in enumerate(problems)]
    _check(_lib().pogs_solve_batch(N, arr, res, _stream_handle(stream)), "pogs_solve_batch")
    return [Result(res[i], *outs[i]) for i in range(N)]


class BatchEngine:
    """pogs_batch: a serving engine with its own scheduler thread."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 0, chunk_iters: int = 0):
        cfg = pogs_batch_cfg(hbm_budget_bytes, max_slots, chunk_iters, None)
        h = C.c_void_p()
        _check(_lib().pogs_batch_create(C.byref(h), C.byref(cfg)), "pogs_batch_create")
        self.handle = h
        self._pending = {}

    def submit(self, p, params: Optional[pogs_params] = None) -> int:
        keep: list = []
        s = _problem_struct(p, params, keep)
        t = C.c_uint64()
        _check(_lib().pogs_batch_submit(self.handle, C.byref(s), C.byref(t)), "pogs_batch_submit")
        self._pending[t.value] = (p.m, p.n)
        return t.value

    def poll(self, ticket: int) -> Optional[Result]:
        m, n = self._pending[ticket]
        keep: list = []
        r = pogs_result()
        o = _host_outputs(m, n, r, keep)
        rc = _lib().pogs_batch_poll(self.handle, ticket, C.byref(r))
        if rc == 1:
            return None
        _check(rc, "pogs_batch_poll")
        del self._pending[ticket]
        return Result(r, *o)

    def cancel(self, ticket: int):
        _check(_lib().pogs_batch_cancel(self.handle, ticket), "pogs_batch_cancel")

    def wait_all(self):
        _check(_lib().pogs_batch_wait_all(self.handle), "pogs_batch_wait_all")

    def close(self):
        if getattr(self, "handle", None):
            _lib().pogs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
