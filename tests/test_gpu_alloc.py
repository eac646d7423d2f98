"""Device-memory callbacks (adc2_alloc): a handle whose every device buffer
comes from PyTorch's caching allocator gives the same results as one on
hipMalloc -- the same kernels on the same data, so sigma, roots, vectors,
transition moments and the adjoint agree bit for bit or to rounding of the
solver's reductions -- its memory shows in torch's statistics while it lives
and goes back when it is destroyed, and an allocator that refuses a request
turns into ADC2_ERR_OOM with nothing launched."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from synth import dipole_integrals, make_system, random_vectors

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_torch_allocator_same_results():
    s = make_system(2, 4, 14, 30, seed=71)
    print("[case] torch allocator (2, 4, 14, 30)", flush=True)
    L, e = dev(s.L), dev(s.eps)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ha = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux)
    ht = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux, alloc="torch")
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - base
    # the handle's integral blocks alone: Lvv, Lvo, Loo
    n_blocks = 16 * s.naux * (s.nv * s.nv + (s.nc + s.no) * s.nv + (s.nc + s.no) ** 2)
    print(f"  torch holds {held} bytes for the handle (blocks {n_blocks})", flush=True)
    assert held >= n_blocks
    x = dev(random_vectors(5, 3, ha.dim))
    Sa, St = A.adc2_sigma(ha, x), A.adc2_sigma(ht, x)
    assert torch.equal(Sa, St)
    for solver in (A.ADC2_SOLVER_FULL, A.ADC2_SOLVER_FOLDED):
        wa, Xa, _ = A.adc2_davidson(ha, 3, tol=1e-9, solver=solver)
        wt, Xt, _ = A.adc2_davidson(ht, 3, tol=1e-9, solver=solver)
        assert np.abs(np.array(wa) - np.array(wt)).max() < 1e-12
    dip = dev(dipole_integrals(3, s.nc + s.no + s.nv))
    Ta, fa = A.adc2_transition(ha, dip, Xa, wa)
    Tt, ft = A.adc2_transition(ht, dip, Xa, wa)
    assert np.array_equal(Ta, Tt)
    g = [1.0, 0.5, 0.25]
    dLa, dea = A.adc2_omega_backward(ha, Xa, g)
    dLt, det = A.adc2_omega_backward(ht, Xa, g)
    assert torch.equal(dLa, dLt) and torch.equal(dea, det)
    ha.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    ht.close()
    torch.cuda.synchronize()
    freed = before - torch.cuda.memory_allocated()
    print(f"  destroying the handle returned {freed} bytes to torch", flush=True)
    assert freed >= n_blocks


def test_refusing_allocator_is_oom():
    s = make_system(1, 2, 5, 12, seed=72)
    calls = []

    def _alloc(nbytes, ctx):
        calls.append(int(nbytes))
        return None

    def _release(ptr, ctx):
        raise AssertionError("nothing was allocated")

    al = A.Alloc(A._ALLOC_FN(_alloc), A._RELEASE_FN(_release), None)
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux, alloc=al)
    assert ei.value.status == A.ADC2_ERR_OOM
    assert len(calls) == 1


def test_torch_allocator_other_entry_points():
    """Natural spinors, the autotuner and the batched setup / solve on
    handles backed by PyTorch's allocator agree with hipMalloc handles."""
    s = make_system(1, 3, 12, 24, seed=73)
    print("[case] torch allocator: fns, autotune, batch", flush=True)
    L, e = dev(s.L), dev(s.eps)
    ha = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux)
    ht = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux, alloc="torch")
    Fa = A.adc2_fns(ha, L, 1e-3)
    Ft = A.adc2_fns(ht, L, 1e-3)
    assert Fa[2] == Ft[2] and torch.equal(Fa[0], Ft[0]) and torch.equal(Fa[1], Ft[1])
    ra, rt = A.adc2_autotune(ha, 2), A.adc2_autotune(ht, 2)
    assert ra["ysplit"] >= 1 and rt["ysplit"] >= 1
    x = dev(random_vectors(9, 2, ha.dim))
    assert torch.equal(A.adc2_sigma(ha, x), A.adc2_sigma(ht, x))
    ha.close()
    ht.close()
    s2 = make_system(1, 2, 9, 18, seed=74)
    systems = [(L, e, s.nc, s.no, s.nv, s.naux), (dev(s2.L), dev(s2.eps), s2.nc, s2.no, s2.nv, s2.naux)]
    hb = A.adc2_setup_batch(systems)
    hbt = A.adc2_setup_batch(systems, alloc="torch")
    wa, _, _ = A.adc2_davidson_batch(hb, 2, tol=1e-9)
    wt, _, _ = A.adc2_davidson_batch(hbt, 2, tol=1e-9)
    for q in range(2):
        assert np.abs(np.array(wa[q]) - np.array(wt[q])).max() < 1e-12
    for hh in hb + hbt:
        hh.close()


def test_torch_allocator_precision_forms_and_two_stage():
    """The complex64 and split-BF16 operand copies and work spaces (built on
    first use) and the two-stage solve (split-BF16 then FP64, nested solver
    calls) on a handle backed by PyTorch's allocator."""
    s = make_system(2, 3, 16, 32, seed=75)
    print("[case] torch allocator: precision forms, two-stage", flush=True)
    L, e = dev(s.L), dev(s.eps)
    ha = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux)
    ht = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux, alloc="torch")
    x = dev(random_vectors(11, 4, ha.dim))
    for prec in (A.ADC2_C64, A.ADC2_BF16X3, A.ADC2_FP64):
        A.adc2_set_precision(ha, prec)
        A.adc2_set_precision(ht, prec)
        assert torch.equal(A.adc2_sigma(ha, x), A.adc2_sigma(ht, x)), prec
    wa, _, _ = A.adc2_davidson(ha, 3, tol=1e-9, mixed_tol=1e-4)
    wt, _, _ = A.adc2_davidson(ht, 3, tol=1e-9, mixed_tol=1e-4)
    assert np.abs(np.array(wa) - np.array(wt)).max() < 1e-12
    ha.close()
    ht.close()
