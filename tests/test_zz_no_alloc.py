"""adc2_sigma_noalloc: the FP64 sigma with its work spaces in the library's
static scratch array, for callers that cannot allocate device memory.

Its output is compared with adc2_sigma's on the same handle and vectors
(bit for bit: the same kernels run with the same split counts, only the work
space addresses differ) and with the oracle's sigma (1e-11 relative, the
FP64 parity bar of the sigma tests), on two calls in a row where the second
has a smaller input, then on a second, smaller system.  The handle is set up
with counting device-memory callbacks, so the test also sees that the
no-allocation call requests no memory through them while adc2_sigma on a
fresh handle does.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import config_system, random_vectors

pytestmark = pytest.mark.gpu

TOL = 1e-11


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


class Counting:
    """Device-memory callbacks on PyTorch's allocator that count requests."""

    def __init__(self):
        self.n = 0
        base = A.torch_allocator()
        self._a, self._r = base.alloc, base.release

        def _alloc(nbytes, ctx):
            self.n += 1
            return self._a(nbytes, ctx)

        self.alloc = A.Alloc(A._ALLOC_FN(_alloc), self._r, None)


def rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def test_noalloc_sigma_equals_sigma_two_calls_then_smaller_system():
    for name, ms in (("c1", (8, 3)), ("tiles", (2,))):
        s = config_system(name)
        print(f"[case] noalloc {name} nc={s.nc} no={s.no} nv={s.nv} naux={s.naux} m={ms}", flush=True)
        cnt = Counting()
        h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux, alloc=cnt.alloc)
        torch.cuda.synchronize()
        o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
        for m in ms:
            x = random_vectors(977 + m, m, h.dim)
            X = dev(x)
            S_na = torch.full_like(X, complex(float("nan"), float("nan")))
            before = cnt.n
            A.adc2_sigma_noalloc(h, X, S_na)
            torch.cuda.synchronize()
            assert cnt.n == before, "adc2_sigma_noalloc requested device memory"
            S_ref = A.adc2_sigma(h, X)
            torch.cuda.synchronize()
            assert torch.equal(S_na, S_ref), f"{name} m={m}: differs from adc2_sigma"
            ref = o.sigma(torch.from_numpy(x))
            err = rel(S_na.cpu(), ref)
            print(f"  m={m}: equal to adc2_sigma; oracle rel err {err:.2e}", flush=True)
            assert err < TOL
        h.close()


def test_noalloc_rejects_what_it_cannot_do():
    s = config_system("mid")
    print(f"[case] noalloc limits mid nc={s.nc} no={s.no} nv={s.nv} naux={s.naux}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    X = dev(random_vectors(5, 8, h.dim))
    S = torch.empty_like(X)
    # eight vectors of this system need more than 128 MiB whatever the K-split: the unpacked
    # doubles (92 MB), the X-build (23 MB) and at least one Y partial (23 MB)
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_sigma_noalloc(h, X, S)
    assert ei.value.status == A.ADC2_ERR_ARG and "maximum" in str(ei.value)
    A.adc2_set_precision(h, A.ADC2_C64)
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_sigma_noalloc(h, X[:1].contiguous(), S[:1].contiguous())
    assert ei.value.status == A.ADC2_ERR_ARG and "FP64" in str(ei.value)
    A.adc2_set_precision(h, A.ADC2_FP64)
    # one vector fits and equals the handle's own sigma of that vector (same split counts)
    A.adc2_sigma_noalloc(h, X[:1].contiguous(), S[:1])
    S2 = A.adc2_sigma(h, X[:1].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(S[:1], S2)
    lib = A.load()
    assert lib.adc2_sigma_noalloc(h.ptr, 0, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                  None) == A.ADC2_ERR_ARG
    assert lib.adc2_sigma_noalloc(h.ptr, 1, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                  None) == A.ADC2_ERR_ARG
    h.close()
