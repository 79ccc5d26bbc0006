"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/pogs.h, and rejects bad arguments before touching the
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pogs.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pogs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1503_08366_amd import pogs
    if not os.path.exists(pogs.LIB_PATH):
        pytest.skip("libpogs.so not built")
    return pogs.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ["pogs_init", "pogs_solve", "pogs_solve_path", "pogs_free", "pogs_batch_create",
                 "pogs_batch_submit", "pogs_batch_poll", "pogs_batch_destroy", "pogs_strerror",
                 "pogs_params_default", "pogs_project", "pogs_prox", "pogs_get_scaling",
                 "pogs_solve_batch"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1503_08366_amd import pogs
    assert set(_declared_functions()) == set(pogs._SIGS)


def test_params_default_and_strerror(lib):
    from paper_1503_08366_amd import pogs
    p = pogs.default_params()
    assert (p.eps_abs, p.eps_rel, p.max_iter, p.rho0, p.alpha, p.delta, p.tau) == \
        (1e-4, 1e-3, 10000, 1.0, 1.7, 1.05, 0.8)
    assert p.adaptive_rho == 1 and p.equil_iters == 10
    assert lib.pogs_params_default(None) == pogs.POGS_EINVAL
    for code in [0, -1, -2, -3, -4, -5, -6, 99]:
        assert isinstance(lib.pogs_strerror(code), bytes)


def test_init_rejects_bad_arguments_without_device(lib):
    from paper_1503_08366_amd import pogs
    A = np.ones((4, 3), dtype=np.float32)
    h = C.c_void_p()
    ptr = C.c_void_p(A.ctypes.data)
    E = pogs.POGS_EINVAL
    assert lib.pogs_init(None, 4, 3, ptr, 0, 0, 3, 0, None, None) == E
    assert lib.pogs_init(C.byref(h), 0, 3, ptr, 0, 0, 3, 0, None, None) == E
    assert lib.pogs_init(C.byref(h), 4, -1, ptr, 0, 0, 3, 0, None, None) == E
    assert lib.pogs_init(C.byref(h), 4, 3, None, 0, 0, 3, 0, None, None) == E
    assert lib.pogs_init(C.byref(h), 4, 3, ptr, 7, 0, 3, 0, None, None) == E       # dtype
    assert lib.pogs_init(C.byref(h), 4, 3, ptr, 0, 5, 3, 0, None, None) == E       # order
    assert lib.pogs_init(C.byref(h), 4, 3, ptr, 0, 0, 2, 0, None, None) == E       # lda < n
    assert lib.pogs_init(C.byref(h), 4, 3, ptr, 0, 1, 3, 0, None, None) == E       # col-major lda < m
    bad = pogs.default_params(alpha=2.5)
    assert lib.pogs_init(C.byref(h), 4, 3, ptr, 0, 0, 3, 0, C.byref(bad), None) == E
    bad = pogs.default_params(max_iter=0)
    assert lib.pogs_init(C.byref(h), 4, 3, ptr, 0, 0, 3, 0, C.byref(bad), None) == E
    bad = pogs.default_params(sparse_segment=-1)
    assert lib.pogs_init(C.byref(h), 4, 3, ptr, 0, 0, 3, 0, C.byref(bad), None) == E
    assert h.value is None
    p = pogs.default_params()
    assert p.sparse_segment == 0 and p.autotune == 1


def test_solve_and_free_reject_null(lib):
    from paper_1503_08366_amd import pogs
    r = pogs.pogs_result()
    assert lib.pogs_solve(None, None, None, None, None, None, C.byref(r)) == pogs.POGS_EINVAL
    assert lib.pogs_free(None) == pogs.POGS_OK
    assert lib.pogs_project(None, None, None, None, None, 0) == pogs.POGS_EINVAL
    assert lib.pogs_get_scaling(None, None, None, 0) == pogs.POGS_EINVAL


def test_prox_rejects_bad_functions_without_device(lib):
    from paper_1503_08366_amd import pogs
    v = np.zeros(3)
    out = np.zeros(3)
    h = np.array([2], np.uint8)
    neg = np.array([-1.0])
    zero = np.array([0.0])
    dp = C.POINTER(C.c_double)

    def fn(h=h, a=None, c=None, e=None, length=3, stride=0):
        return pogs.pogs_fn(length, stride, h.ctypes.data_as(C.POINTER(C.c_uint8)),
                            a.ctypes.data_as(dp) if a is not None else None, None,
                            c.ctypes.data_as(dp) if c is not None else None, None,
                            e.ctypes.data_as(dp) if e is not None else None)

    call = lambda f, rho=1.0: lib.pogs_prox(C.byref(f), 1, rho, v.ctypes.data, out.ctypes.data, 0, None)
    E = pogs.POGS_EINVAL
    assert call(fn(c=neg)) == E                                    # c < 0: not convex
    assert call(fn(e=neg)) == E                                    # e < 0: not convex
    assert call(fn(a=zero)) == E                                   # a = 0 with c > 0
    assert call(fn(h=np.array([42], np.uint8))) == E               # unknown h
    assert call(fn(a=np.array([np.nan]))) == E                     # non-finite parameter
    assert call(fn(), rho=0.0) == E                                # rho must be > 0
    assert call(fn(stride=3)) == E                                 # stride is 0 or 1


def test_batch_rejects_null(lib):
    from paper_1503_08366_amd import pogs
    assert lib.pogs_batch_submit(None, None, None) in (pogs.POGS_EINVAL, pogs.POGS_EUNSUPPORTED)
    assert lib.pogs_batch_destroy(None) == pogs.POGS_OK


def test_init_sparse_rejects_bad_inputs_without_device(lib):
    """Every check of pogs_init_sparse on host input runs before any device
    call: malformed row pointers, column indices out of range, non-finite
    values, bad sizes and parameters."""
    from paper_1503_08366_amd import pogs
    E = pogs.POGS_EINVAL
    h = C.c_void_p()

    def call(m, n, rp, ci, va, dt=pogs.POGS_F64, prm=None):
        rp = np.ascontiguousarray(rp, dtype=np.int64)
        ci = np.ascontiguousarray(ci, dtype=np.int32)
        va = np.ascontiguousarray(va, dtype=np.float64 if dt == pogs.POGS_F64 else np.float32)
        return lib.pogs_init_sparse(C.byref(h), m, n, len(ci), C.c_void_p(rp.ctypes.data),
                                    C.c_void_p(ci.ctypes.data), C.c_void_p(va.ctypes.data), dt, pogs.POGS_HOST,
                                    C.byref(prm) if prm is not None else None, None)

    good_rp, good_ci, good_va = [0, 2, 3], [0, 2, 1], [1.0, 2.0, 3.0]
    assert call(2, 3, [1, 2, 3], good_ci, good_va) == E           # rowptr[0] != 0
    assert call(2, 3, [0, 2, 2], good_ci, good_va) == E           # rowptr[m] != nnz
    assert call(2, 3, [0, 3, 2], good_ci, good_va) == E           # decreasing
    assert call(2, 3, good_rp, [0, 3, 1], good_va) == E           # column index = n
    assert call(2, 3, good_rp, [0, -1, 1], good_va) == E          # negative column index
    assert call(2, 3, good_rp, good_ci, [1.0, np.nan, 3.0]) == E  # non-finite value
    assert call(2, 3, good_rp, good_ci, [1.0, np.inf, 3.0], dt=pogs.POGS_F32) == E
    assert call(0, 3, [0], [], []) == E                           # m = 0
    assert call(2, 3, good_rp, good_ci, good_va, dt=9) == E       # dtype
    assert call(2, 3, good_rp, good_ci, good_va, prm=pogs.default_params(cg_max_iter=0)) == E
    assert lib.pogs_init_sparse(None, 2, 3, 3, None, None, None, 1, 0, None, None) == E
    assert h.value is None


def test_prox_noalloc_rejects_without_device(lib):
    """Argument checks and the size limit of the allocation-free prox run on
    the host before any device call (the pointers here are never touched)."""
    from paper_1503_08366_amd import pogs
    dp = C.POINTER(C.c_double)
    fake = C.c_void_p(16)
    h1 = np.array([2], np.uint8)
    f = pogs.pogs_fn(3, 0, h1.ctypes.data_as(C.POINTER(C.c_uint8)), None, None, None, None, None)
    assert lib.pogs_prox_noalloc(None, 0, 1.0, fake, fake, None) == pogs.POGS_EINVAL
    assert lib.pogs_prox_noalloc(C.byref(f), 0, 1.0, None, fake, None) == pogs.POGS_EINVAL
    assert lib.pogs_prox_noalloc(C.byref(f), 0, 0.0, fake, fake, None) == pogs.POGS_EINVAL
    assert lib.pogs_prox_noalloc(C.byref(f), 5, 1.0, fake, fake, None) == pogs.POGS_EINVAL
    neg = np.array([-1.0])
    fneg = pogs.pogs_fn(3, 0, h1.ctypes.data_as(C.POINTER(C.c_uint8)), None, None, neg.ctypes.data_as(dp),
                        None, None)
    assert lib.pogs_prox_noalloc(C.byref(fneg), 0, 1.0, fake, fake, None) == pogs.POGS_EINVAL
    # per-element h plus two float64 arrays: 1 + 2 * 8 bytes per entry; 4M
    # entries need 68 MB > 64 MiB
    N = 4 << 20
    hN = np.full(N, 2, np.uint8)
    aN = np.ones(N)
    big = pogs.pogs_fn(N, 1, hN.ctypes.data_as(C.POINTER(C.c_uint8)), aN.ctypes.data_as(dp), None,
                       aN.ctypes.data_as(dp), None, None)
    assert lib.pogs_prox_noalloc(C.byref(big), 0, 1.0, fake, fake, None) == pogs.POGS_ETOOBIG
    assert b"allocation-free" in lib.pogs_strerror(pogs.POGS_ETOOBIG)
