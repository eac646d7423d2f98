"""The brute-force pin catches plausible mistakes in the oracle formulas.

Each mutant below is the oracle's expression with one plausible slip (a sign,
a misplaced conjugate, a dropped half of a symmetrised denominator, a
transposed index pair).  The test asserts that every mutant disagrees with the
brute-force intermediate-state construction by far more than the fit error,
so that a pin test passing means the unmutated formula is the right one.
"""
import numpy as np
import torch

from synth import make_system
from oracle import adc2 as O
from oracle.isr_bruteforce import adc2_blocks


def _setup():
    s = make_system(2, 2, 3, 8, seed=17, sigma=0.14, core=(-3.0, -2.5))
    bf = adc2_blocks(s.L, s.eps, s.nc, s.no, s.nv)
    return s, bf, O.as_c128(s.L), O.as_f64(s.eps), O.Spaces(s.nc, s.no, s.nv)


def test_mutants_are_caught():
    s, bf, L, e, sp = _setup()
    ns = sp.n_singles
    t = O.m11_terms(L, e, sp)
    ref = bf["M11_cvs"]
    C, O_, U = sp.C, sp.O, sp.U

    def dev(m):
        return np.abs(m.reshape(ns, ns).numpy() - ref).max()

    base = t["m0"] + t["m1"] + t["m2i"] + t["m2ii"] + t["m2iii"]
    assert dev(base) < 1e-9

    mutants = {}
    mutants["m2iii sign"] = base - 2 * t["m2iii"]
    mutants["m2i sign"] = base - 2 * t["m2i"]
    mutants["m1 transposed (aI|Jb) <-> (aJ|Ib)"] = base - t["m1"] + t["m1"].permute(2, 1, 0, 3)
    # misplaced conjugate in term (ii): <Ik||cd><cd||Jk> instead of <Jk||cd><cd||Ik>
    W_coVV = O.asym(L, C, O_, U, U)
    W_VVco = O.asym(L, U, U, C, O_)
    D_vvco = O.denom(e, sp, U, U, C, O_)
    D_covv = D_vvco.permute(2, 3, 0, 1)
    tii_bad = 0.25 * (torch.einsum("Ikcd,cdJk->IJ", W_coVV, W_VVco / D_vvco)
                      + torch.einsum("Ikcd,cdJk->IJ", W_coVV / D_covv, W_VVco))
    mutants["m2ii conj placement"] = base - t["m2ii"] + torch.einsum(
        "IJ,ab->IaJb", tii_bad, torch.eye(sp.nv, dtype=O.C128))
    # one half of the symmetrised denominator dropped in term (iii)
    W_vvco = W_VVco
    half = -1.0 * torch.einsum("acIk,Jkbc->IaJb", W_vvco / D_vvco, W_coVV)
    mutants["m2iii one denominator"] = base - t["m2iii"] + half
    # core-only k sum in term (i) (a CVS variant, not the projection reading)
    W_vvcc = O.asym(L, U, U, C, C)
    W_ccvv = O.asym(L, C, C, U, U)
    D_vvcc = O.denom(e, sp, U, U, C, C)
    ti_c = 0.25 * (torch.einsum("ackl,klbc->ab", W_vvcc / D_vvcc, W_ccvv)
                   + torch.einsum("ackl,klbc->ab", W_vvcc, W_ccvv / D_vvcc.permute(2, 3, 0, 1)))
    mutants["m2i core-only k,l"] = base - t["m2i"] + torch.einsum(
        "IJ,ab->IaJb", torch.eye(sp.nc, dtype=O.C128), ti_c)
    for name, m in mutants.items():
        assert dev(m) > 1e-6, name

    # coupling: sign of the delta_ac term, and (ab|cj) ordering slip
    M21 = O.m21_dense(L, e, sp).numpy()
    assert np.abs(M21 - bf["M21_cvs"]).max() < 1e-9
    W_vvvV, W_cvcV = O.coupling_integrals(L, sp)
    eyeC = torch.eye(sp.nc, dtype=O.C128)
    eyeU = torch.eye(sp.nv, dtype=O.C128)
    ia, ib = O.pair_index(sp.nv)
    t1 = torch.einsum("IK,abcj->IjabKc", eyeC, W_vvvV)
    t2 = torch.einsum("ac,KbIj->IjabKc", eyeU, W_cvcV)
    t3 = torch.einsum("bc,KaIj->IjabKc", eyeU, W_cvcV)
    for name, full in {"delta_ac sign": t1 + t2 + t3,
                       "conj coupling": t1.conj() - t2 + t3}.items():
        bad = full[:, :, ia, ib].reshape(sp.n_doubles, ns).numpy()
        assert np.abs(bad - bf["M21_cvs"]).max() > 1e-6, name

    # MP2: a factor 1/2 instead of 1/4
    assert abs(2 * float(O.mp2_energy(L, e, sp)) - bf["E_mp2"]) > 1e-6
