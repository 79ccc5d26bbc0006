"""The allocation-free prox entry point (pogs_prox_noalloc) against the
allocating one (pogs_prox) on the device: bit-identical outputs for every base
function h, float32 and float64, per-element and broadcast parameters, on two
calls in a row whose second input is smaller (the fixed device buffer keeps
the first call's contents and must not leak into the second), then a
function too large for the buffer (POGS_ETOOBIG, nothing launched)."""
import ctypes as C
import zlib

import numpy as np
import pytest

from paper_1503_08366_amd import pogs as P
from paper_1503_08366_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _fn(h, N, seed, broadcast=False):
    rng = np.random.default_rng(seed)
    k = 1 if broadcast else N
    a = rng.choice([-1.0, 1.0], k) * rng.uniform(0.3, 3.0, k)
    b = rng.normal(0, 1, k)
    c = rng.uniform(0.1, 3.0, k)
    d = rng.normal(0, 1, k)
    e = np.where(rng.random(k) < 0.5, 0.0, rng.uniform(0.1, 2.0, k))
    if not broadcast:
        c[::17] = 0.0
        return W.Fn(h, N, a=a, b=b, c=c, d=d, e=e)
    return W.Fn(h, N, a=float(a[0]), b=float(b[0]), c=float(c[0]), d=float(d[0]), e=float(e[0]))


def _pair(F, v, rho):
    """pogs_prox and pogs_prox_noalloc on the same device input."""
    ref = P.pogs_prox(F, v, rho)
    out = torch.full_like(v, float("nan"))
    got = P.pogs_prox_noalloc(F, v, rho, out)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("h", list(P.H_CODES))
def test_noalloc_prox_matches_pogs_prox_two_calls(h, dt):
    print(f"noalloc prox h={h} dt={dt}", flush=True)
    seed = zlib.crc32(h.encode())
    for call, (N, broadcast) in enumerate([(70001, False), (1537, False), (513, True)]):
        F = _fn(h, N, seed + call, broadcast)
        rng = np.random.default_rng(seed + 100 + call)
        v = torch.from_numpy(rng.normal(0, 3, N)).to(dt).cuda()
        ref, got = _pair(F, v, 1.3 + 0.1 * call)
        assert torch.equal(ref, got), (h, call, N, float((ref - got).abs().max()))


def test_noalloc_prox_rejects_oversized_function():
    N = 2_000_000  # 5 float64 arrays of N entries exceed the 64 MiB buffer
    F = W.Fn("abs", N, a=np.ones(N), b=np.zeros(N), c=np.ones(N), d=np.zeros(N), e=np.zeros(N))
    v = torch.zeros(N, dtype=torch.float32, device="cuda")
    out = torch.full_like(v, 7.0)
    with pytest.raises(P.PogsError) as ei:
        P.pogs_prox_noalloc(F, v, 1.0, out)
    assert ei.value.code == P.POGS_ETOOBIG
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing ran
    # the same length with broadcast parameters (stride 0: one entry each) fits
    h1 = np.array([P.H_CODES["abs"]], np.uint8)
    c1 = np.array([0.5])
    f1 = P.pogs_fn(N, 0, h1.ctypes.data_as(C.POINTER(C.c_uint8)), None, None,
                   c1.ctypes.data_as(C.POINTER(C.c_double)), None, None)
    v2 = v + 2.0
    got = torch.full_like(v2, float("nan"))
    rc = P.load().pogs_prox_noalloc(C.byref(f1), P.POGS_F32, 1.0, C.c_void_p(v2.data_ptr()),
                                    C.c_void_p(got.data_ptr()), None)
    assert rc == P.POGS_OK
    ref = P.pogs_prox(W.Fn("abs", N, c=0.5), v2, 1.0)
    torch.cuda.synchronize()
    assert torch.equal(ref, got)
