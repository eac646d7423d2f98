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


def test_second_order_transition_mutants_are_caught():
    """Plausible slips inside the second-order singles of the transition
    moments (in the second-order amplitudes and in the pair densities) each
    move F2 away from the brute-force lambda^2 coefficient by far more than
    its fit error (5e-9), and so does the CVS-only reading of the
    intermediate states."""
    from oracle.isr_bruteforce import transition_taylor
    s = make_system(2, 2, 3, 6, seed=29, sigma=0.15, core=(-3.0, -2.5))
    L, e, sp = O.as_c128(s.L), O.as_f64(s.eps), O.Spaces(s.nc, s.no, s.nv)
    rng = np.random.default_rng(31)
    d = rng.standard_normal((sp.n, sp.n)) + 1j * rng.standard_normal((sp.n, sp.n))
    d = 0.5 * (d + d.conj().T)
    (F0, F1, F2), resid, singles, _ = transition_taylor(s.L, s.eps, sp.o, d)
    assert resid < 1e-9
    ref = F2[[k for k, (i, a) in enumerate(singles) if i < sp.nc]]
    C, O_, U, V = sp.C, sp.O, sp.U, sp.V
    dd = torch.as_tensor(d).to(O.C128)
    dvv, doo, dov, dvo = dd[U][:, U], dd[O_][:, O_], dd[O_][:, U], dd[U][:, O_]
    tau = O.mp2_amplitudes(L, e, sp)
    eo, ev = e[O_], e[U]
    Dia = ev[None, :] - eo[:, None]
    n1 = torch.einsum("ajbc,bcij->ia", O.asym(L, U, O_, U, U), tau)
    n2 = torch.einsum("jkib,abjk->ia", O.asym(L, O_, O_, O_, U), tau)
    pp = torch.einsum("abcd,cdij->abij", O.asym(L, U, U, U, U), tau)
    hh = torch.einsum("klij,abkl->abij", O.asym(L, O_, O_, O_, O_), tau)
    r = torch.einsum("kbcj,acik->abij", O.asym(L, O_, U, U, O_), tau)
    D = O.denom(e, sp, U, U, O_, O_)
    ring = r - r.permute(1, 0, 2, 3) - r.permute(0, 1, 3, 2) + r.permute(1, 0, 3, 2)
    rho = torch.einsum("abkl,cbkl->ac", tau, tau.conj())
    sig = torch.einsum("cdil,cdkl->ik", tau, tau.conj())
    P = torch.einsum("abil,cbkl->iakc", tau, tau.conj())

    def f2(s_=None, u_=None, rho_=rho, sig_=sig, P_=P, cvs_only=False):
        s_ = 0.5 * (n1 - n2) / Dia if s_ is None else s_
        u_ = (0.5 * pp + 0.5 * hh + ring) / D if u_ is None else u_
        f = (torch.einsum("ab,ib->ia", dvv, s_) - torch.einsum("ji,ja->ia", doo, s_)
             + torch.einsum("jb,abij->ia", dov, u_)
             - 0.25 * torch.einsum("ac,ci->ia", rho_, dvo))
        if cvs_only:
            mc = torch.zeros(sp.o, dtype=O.C128)
            mc[C] = 1.0
            f = f + (-0.5 * torch.einsum("ak,ik->ia", dvo, sig_) + 0.25 * torch.einsum("ak,ik->ia", dvo * mc, sig_)
                     + torch.einsum("iakc,ck->ia", P_, dvo) - 0.5 * torch.einsum("iakc,ck->ia", P_, dvo * mc))
        else:
            f = f - 0.25 * torch.einsum("ak,ik->ia", dvo, sig_) + 0.5 * torch.einsum("iakc,ck->ia", P_, dvo)
        return f[C].reshape(-1).numpy()

    assert np.abs(f2() - ref).max() < 5e-9
    assert np.allclose(f2(), O.second_order_singles(L, e, sp, d).reshape(-1).numpy(), rtol=0, atol=1e-14)
    mutants = {
        "singles: n1 + n2": dict(s_=0.5 * (n1 + n2) / Dia),
        "singles: denominator e_i - e_a": dict(s_=-0.5 * (n1 - n2) / Dia),
        "doubles: hole ladder sign": dict(u_=(0.5 * pp - 0.5 * hh + ring) / D),
        "doubles: full particle ladder (no 1/2)": dict(u_=(pp + 0.5 * hh + ring) / D),
        "doubles: ring without P(ab)": dict(u_=(0.5 * pp + 0.5 * hh + r - r.permute(0, 1, 3, 2)) / D),
        "doubles: ring with tau^{ca}": dict(u_=(0.5 * pp + 0.5 * hh - ring) / D),
        "rho conjugate on the other factor": dict(rho_=torch.einsum("abkl,cbkl->ac", tau.conj(), tau)),
        "sigma indices exchanged": dict(sig_=sig.T.contiguous()),
        "P conjugate on the other factor": dict(P_=torch.einsum("abil,cbkl->iakc", tau.conj(), tau)),
        "CVS-only intermediate states": dict(cvs_only=True),
    }
    for name, kw in mutants.items():
        dev = np.abs(f2(**kw) - ref).max()
        print(f"  {name}: {dev:.2e}")
        assert dev > 1e-6, (name, dev)
