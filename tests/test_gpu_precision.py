"""GPU precision form: the two heavy sigma contractions on complex64 operands
with the FP32 MFMA, or on split-BF16 operands (hi + lo, three products) with
the BF16 MFMA; FP64 everywhere else.

Tolerances: the sigma of the precision form is compared with the FP64 oracle
at 2e-5 of max|sigma| (FP32 unit roundoff 6e-8 times the sqrt of a
1500-term accumulation, with margin); it must also differ from the FP64 path
(so the FP32 kernels really ran).  Roots of the precision form must be within
1e-3 eV of the FP64 roots before the FP64 Rayleigh polish and within 1e-6 Ha
after it.  The split-BF16 sigma must be within 1e-5 of the oracle (it keeps
~16 bits per operand) and its folded roots, converged to residual 1e-3,
within 1e-4 eV of FP64 before and after the polish.
"""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import config_system, random_vectors

pytestmark = pytest.mark.gpu
EV = O.HARTREE_EV


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def mid():
    s = config_system("mid")
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux, prec=A.ADC2_C64)
    return s, o, h


def test_c64_sigma_mid(mid):
    s, o, h = mid
    x = random_vectors(201, 3, o.dim)
    ref = o.sigma(torch.from_numpy(x)).numpy()
    got = A.adc2_sigma(h, dev(x)).cpu().numpy()
    A.adc2_set_precision(h, A.ADC2_FP64)
    got64 = A.adc2_sigma(h, dev(x)).cpu().numpy()
    A.adc2_set_precision(h, A.ADC2_C64)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    err64 = np.abs(got64 - ref).max() / scale
    print(f"c64 sigma rel err {err:.3e}, fp64 {err64:.3e}")
    assert err < 2e-5
    assert err > 100 * err64          # the FP32 kernels ran
    assert err64 < 1e-11


def test_c64_roots_c1():
    s = config_system("c1")
    L, e = dev(s.L), dev(s.eps)
    h64 = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux)
    w64, X64, info64 = A.adc2_davidson(h64, 4, tol=1e-8)
    h = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux, prec=A.ADC2_C64)
    w32, X32, info32 = A.adc2_davidson(h, 4, tol=1e-5, raise_on_noconv=False)
    wp, rn = A.adc2_rayleigh(h, X32)
    d_raw = np.abs(np.array(w32) - np.array(w64)) * EV
    d_pol = np.abs(np.array(wp) - np.array(w64))
    print("c64 roots eV err", d_raw.tolist(), "polished Ha err", d_pol.tolist(), "iters", info32["iters"],
          "fp64 residuals of c64 vectors", rn)
    assert info64["converged"]
    assert d_raw.max() < 1e-3
    assert d_pol.max() < 1e-6


def test_rayleigh_certifies_fp64_roots():
    s = config_system("tiles")
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    w, X, info = A.adc2_davidson(h, 3, tol=1e-9, max_subspace=40)
    wr, rn = A.adc2_rayleigh(h, X)
    assert np.abs(np.array(wr) - np.array(w)).max() < 1e-10
    assert max(rn) < 1e-8


# ---------------------------------------------------------------- split-BF16
def test_b3_sigma_mid(mid):
    """Split-BF16: each complex64 operand as hi + lo bf16 parts, three
    products per real product on the BF16 MFMA, FP32 accumulation."""
    s, o, h = mid
    x = random_vectors(202, 3, o.dim)
    ref = o.sigma(torch.from_numpy(x)).numpy()
    A.adc2_set_precision(h, A.ADC2_BF16X3)
    got = A.adc2_sigma(h, dev(x)).cpu().numpy()
    A.adc2_set_precision(h, A.ADC2_C64)
    got32 = A.adc2_sigma(h, dev(x)).cpu().numpy()
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    err32 = np.abs(got32 - ref).max() / scale
    print(f"split-bf16 sigma rel err {err:.3e}, c64 {err32:.3e}")
    assert err < 1e-5                 # measured 1.4e-6: hi+lo keeps ~16 bits, lo*lo dropped
    assert err > 3 * err32            # the BF16 kernels ran


def test_b3_roots_c1():
    s = config_system("c1")
    L, e = dev(s.L), dev(s.eps)
    h = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux)
    w64, _, info64 = A.adc2_davidson(h, 4, tol=1e-9, solver=A.ADC2_SOLVER_FOLDED, want_vectors=False)
    A.adc2_set_precision(h, A.ADC2_BF16X3)
    wb, Xb, infob = A.adc2_davidson(h, 4, tol=1e-3, solver=A.ADC2_SOLVER_FOLDED, raise_on_noconv=False)
    A.adc2_set_precision(h, A.ADC2_FP64)
    wp, rn = A.adc2_rayleigh(h, Xb)
    d_raw = np.abs(np.array(wb) - np.array(w64)) * EV
    d_pol = np.abs(np.array(wp) - np.array(w64)) * EV
    print("split-bf16 roots eV err", d_raw.tolist(), "polished eV err", d_pol.tolist(), "iters", infob["iters"],
          "max res", max(infob["resnorm"]), "fp64 residuals", rn)
    assert info64["converged"]
    assert d_raw.max() < 1e-4          # eV; measured 6e-6 (eigenvalue error ~ residual^2)
    assert d_pol.max() < 1e-4


@pytest.fixture(scope="module")
def c1_oracle_roots():
    s = config_system("c1")
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    w, _, inf = o.roots(4, tol=1e-9, max_iter=300)
    assert inf["converged"]
    return s, w.numpy()


@pytest.mark.parametrize("prec,tol", [(A.ADC2_C64, 1e-5), (A.ADC2_BF16X3, 1e-3)])
def test_precision_roots_c1_vs_oracle(c1_oracle_roots, prec, tol):
    """The precision form's roots against the FP64 oracle's own roots (not
    the GPU's FP64 ones): within 1e-3 eV per root raw, and the FP64
    Rayleigh quotients of its vectors within 1e-3 eV as well."""
    s, w_or = c1_oracle_roots
    print(f"[case] precision form {prec} c1 roots vs the oracle", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux, prec=prec)
    w, X, inf = A.adc2_davidson(h, 4, tol=tol, solver=A.ADC2_SOLVER_FOLDED)
    A.adc2_set_precision(h, A.ADC2_FP64)
    wp, rn = A.adc2_rayleigh(h, X)
    d_raw = (np.array(w) - w_or) * EV
    d_pol = (np.array(wp) - w_or) * EV
    print(f"  eV error raw {np.abs(d_raw).max():.2e}, polished {np.abs(d_pol).max():.2e}", flush=True)
    assert inf["converged"]
    assert np.abs(d_raw).max() < 1e-3 and np.abs(d_pol).max() < 1e-3
    h.close()
