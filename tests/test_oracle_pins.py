"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test would fail on a plausible mistake in the oracle (a dropped term, a
sign, a misplaced conjugate, a transposed operand):

  P1  brute-force intermediate-state construction (paper Eq. 4-12) in a tiny
      Fock space -> E_MP2, singles block through 2nd order, first-order
      coupling, zeroth-order doubles block.
  P2  exact diagonalisation of the explicit matrix vs the oracle Davidson
      and vs the elimination of the diagonal doubles block (roots below
      the doubles threshold); the root-following selection rule.
  P3  Hermiticity, sigma linearity, matrix-free sigma == explicit matrix.
  P4  MP2 closed form vs the textbook closed-shell RMP2 formula.
  P5  nonrelativistic limit: real M, singlet/triplet multiplets, CIS limit
      equal to the textbook RHF singlet and triplet CIS matrices.
  P6  invariances: spinor phases, real rotation of the Cholesky index,
      permutation of spinors inside a block, uniform shift of energies.
  P8  Hellmann-Feynman gradient vs central finite differences and the
      scaling identity.
  TM  transition moments F_I = <Psi~_I|D|Psi0> through first order, and the
      singles through second order, vs the brute-force intermediate states;
      invariance under D -> D + c 1; the spin selection rule (triplets dark)
      in the nonrelativistic limit.
  FNS the MP2 virtual density (Eq. 15) vs the second-order coefficient of
      the exact ground-state density; natural-spinor transform with nothing
      dropped leaves the ADC roots and the MP2 energy unchanged.
"""
import math

import numpy as np
import pytest
import torch

from synth import make_system, make_spin_blocked
from oracle import adc2 as O
from oracle.isr_bruteforce import adc2_blocks, density_taylor, transition_taylor

torch.set_num_threads(min(8, torch.get_num_threads()))


def _tensors(s):
    return O.as_c128(s.L), O.as_f64(s.eps), O.Spaces(s.nc, s.no, s.nv)


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("shape,seed,sigma", [((1, 2, 3), 5, 0.12), ((2, 2, 3), 7, 0.15),
                                              ((1, 3, 3), 11, 0.10)])
def test_p1_bruteforce_isr(shape, seed, sigma):
    nc, no, nv = shape
    s = make_system(nc, no, nv, 8, seed=seed, sigma=sigma, core=(-3.0, -2.5))
    bf = adc2_blocks(s.L, s.eps, nc, no, nv)
    assert bf["fit_resid"] < 1e-11
    L, e, sp = _tensors(s)
    tol = 1e-9
    # ground state: E_MP2 is the lambda^2 coefficient of E0
    assert abs(bf["E_mp2"] - float(O.mp2_energy(L, e, sp))) < tol
    # singles block of CVS-ADC(2) and of full ADC(2) (all occupied as holes)
    m11 = O.m11(L, e, sp).numpy()
    assert np.abs(m11 - bf["M11_cvs"]).max() < tol
    spf = O.Spaces(nc + no, 0, nv)
    assert np.abs(O.m11(L, e, spf).numpy() - bf["M11_full"]).max() < tol
    # first-order coupling and zeroth-order doubles
    assert np.abs(O.m21_dense(L, e, sp).numpy() - bf["M21_cvs"]).max() < tol
    assert np.abs(np.diag(O.m22_diag(e, sp).numpy()) - bf["M22_cvs"]).max() < tol
    # the second-order singles terms are large enough here for the pin to bite
    t = O.m11_terms(L, e, sp)
    for k in ("m2i", "m2ii", "m2iii"):
        assert float(t[k].abs().max()) > 1e3 * tol


def test_p1_orders_separate():
    """The ISR zeroth/first orders alone equal the oracle's m0 and m1."""
    s = make_system(1, 2, 3, 8, seed=3, sigma=0.12, core=(-3.0, -2.5))
    bf = adc2_blocks(s.L, s.eps, 1, 2, 3)
    M0, M1, M2 = bf["orders"]
    L, e, sp = _tensors(s)
    t = O.m11_terms(L, e, O.Spaces(3, 0, 3))
    ns = 9
    assert np.abs(M0[:ns, :ns] - t["m0"].reshape(ns, ns).numpy()).max() < 1e-9
    assert np.abs(M1[:ns, :ns] - t["m1"].reshape(ns, ns).numpy()).max() < 1e-9
    m2 = (t["m2i"] + t["m2ii"] + t["m2iii"]).reshape(ns, ns).numpy()
    assert np.abs(M2[:ns, :ns] - m2).max() < 1e-9


# ---------------------------------------------------------------- P2
def test_p2_davidson_vs_exact():
    s = make_system(2, 4, 14, 24, seed=21)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    assert a.dim == 2 * 14 + 2 * 4 * 91
    w_ex, _ = a.roots_exact(4)
    w_dv, X, info = a.roots(4, tol=1e-9)
    assert info["converged"]
    assert torch.max(torch.abs(w_ex - w_dv)).item() < 1e-10
    # Ritz vectors are orthonormal eigenvectors of the explicit matrix
    M = a.matrix()
    R = X @ M.T - w_dv[:, None] * X
    assert torch.linalg.vector_norm(R, dim=1).max().item() < 1e-8
    assert torch.allclose(X.conj() @ X.T, torch.eye(4, dtype=O.C128), atol=1e-10)


def test_p2_root_following_selection_rule():
    """roots_following picks, per reference, the eigenpair of largest overlap,
    greedily without reuse.  Hand-made 4x4 case: a diagonal matrix, so the
    eigenvectors are the unit vectors (no eigensolver arithmetic involved)."""
    M = torch.diag(torch.tensor([1.0, 2.0, 3.0, 4.0], dtype=O.C128))
    refs = torch.tensor([[0.1, 0.0, 0.9, 0.2],      # -> eigenvalue 3 (overlap 0.81)
                         [0.0, 0.0, 0.8, 0.5],      # wants 3 too (0.64) but loses it -> 4 (0.25)
                         [0.6, 0.5, 0.0, 0.0]], dtype=O.C128)   # -> 1 (0.36)
    w, X = O.roots_following(M, refs)
    assert w.tolist() == [3.0, 4.0, 1.0]
    assert torch.equal(X.abs(), torch.eye(4, dtype=torch.float64)[:, [2, 3, 0]])
    # exact eigenvectors of an ADC matrix as references give those eigenpairs back in reference order
    s = make_system(1, 2, 5, 12, seed=4)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    Mx = a.matrix()
    wn, vn = np.linalg.eigh(Mx.numpy())
    pick = [5, 1, 8]
    w2, _ = O.roots_following(Mx, torch.from_numpy(vn[:, pick].T.copy()))
    assert np.abs(w2.numpy() - wn[pick]).max() < 1e-10


def test_p2_folded_roots_vs_exact():
    # strong coupling pushes the lowest roots below min D
    s = make_system(2, 3, 7, 24, seed=303, sigma=0.25)
    L, e, sp = _tensors(s)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    w_ex, V = a.roots_exact(4)
    assert float(w_ex[3]) < float(O.m22_diag(e, sp).min())
    w, x1 = O.roots_folded(L, e, sp, 4)
    assert np.abs(w - w_ex.numpy()).max() < 1e-10
    # the singles parts are those of the exact eigenvectors up to normalisation and phase
    ns = sp.n_singles
    for j in range(4):
        v = V[:ns, j].numpy()
        v = v / np.linalg.norm(v)
        assert abs(abs(np.vdot(v, x1[j])) - 1.0) < 1e-8
    # here the third root lies just above min D (a doubles state shifted by weak
    # coupling) and the elimination refuses it
    s2 = make_system(1, 2, 3, 5, seed=7)
    L2, e2, sp2 = _tensors(s2)
    w2, _ = O.roots_folded(L2, e2, sp2, 2)
    a2 = O.Adc2(s2.L, s2.eps, s2.nc, s2.no, s2.nv)
    assert np.abs(w2 - a2.roots_exact(2)[0].numpy()).max() < 1e-10
    with pytest.raises(ValueError):
        O.roots_folded(L2, e2, sp2, 3)


# ---------------------------------------------------------------- P3
def test_p3_hermitian_and_sigma():
    s = make_system(2, 3, 7, 16, seed=4)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    M = a.matrix()
    assert torch.linalg.matrix_norm(M - M.conj().T) <= 1e-14 * torch.linalg.matrix_norm(M)
    g = torch.Generator().manual_seed(0)
    x = torch.randn(3, a.dim, dtype=O.C128, generator=g)
    y = torch.randn(3, a.dim, dtype=O.C128, generator=g)
    sx, sy = a.sigma(x), a.sigma(y)
    assert torch.allclose(sx, x @ M.T, atol=1e-11, rtol=0)
    # linearity and x^H sigma(y) = conj(y^H sigma(x))
    assert torch.allclose(a.sigma(2.5 * x - 1j * y), 2.5 * sx - 1j * sy, atol=1e-11)
    lhs = torch.sum(x.conj() * sy, dim=1)
    rhs = torch.sum(y.conj() * sx, dim=1).conj()
    assert torch.allclose(lhs, rhs, atol=1e-10)


# ---------------------------------------------------------------- P4
def test_p4_rmp2_closed_shell():
    sb = make_spin_blocked(1, 2, 4, 12, seed=8, sigma=0.08)
    L, e, sp = _tensors(sb)
    e_so = float(O.mp2_energy(L, e, sp))
    l = sb.extra["l_spatial"]
    es = sb.extra["eps_spatial"]
    ncs, nos, nvs = sb.extra["n_spatial"]
    o = ncs + nos
    ov = np.einsum("Pia,Pjb->iajb", l[:, :o, o:], l[:, :o, o:])
    E = 0.0
    for i in range(o):
        for j in range(o):
            for a in range(nvs):
                for b in range(nvs):
                    d = es[i] + es[j] - es[o + a] - es[o + b]
                    E += ov[i, a, j, b] * (2 * ov[i, a, j, b] - ov[i, b, j, a]) / d
    assert abs(e_so - E) < 1e-12 * max(1.0, abs(E)) + 1e-14
    assert abs(E) > 1e-4


# ---------------------------------------------------------------- P5
def _multiplets(w, tol):
    groups, cur = [], [w[0]]
    for x in w[1:]:
        if x - cur[-1] < tol:
            cur.append(x)
        else:
            groups.append(cur)
            cur = [x]
    groups.append(cur)
    return [len(g) for g in groups]


def test_p5_nonrelativistic_limit():
    sb = make_spin_blocked(1, 2, 4, 12, seed=9, sigma=0.1)
    L, e, sp = _tensors(sb)
    a = O.Adc2(sb.L, sb.eps, sb.nc, sb.no, sb.nv)
    M = a.matrix()
    assert torch.abs(M.imag).max().item() < 1e-14
    w = torch.linalg.eigvalsh(M).numpy()
    dmin = O.m22_diag(e, sp).min().item()
    low = w[w < dmin - 1e-3]
    assert len(low) >= 4
    sizes = _multiplets(low, 1e-9)
    assert all(sz in (1, 3) for sz in sizes), sizes
    assert 3 in sizes
    # CIS limit: spin-orbital CVS-CIS == RHF singlet (x1) and triplet (x3) CIS
    m1 = O.m11(L, e, sp, order=1)
    w_so = np.sort(torch.linalg.eigvalsh(m1).numpy())
    l = sb.extra["l_spatial"]
    es = sb.extra["eps_spatial"]
    ncs, nos, nvs = sb.extra["n_spatial"]
    o = ncs + nos
    C, U = slice(0, ncs), slice(o, o + nvs)
    iajb = np.einsum("Pia,Pjb->iajb", l[:, C, U], l[:, C, U])
    ijab = np.einsum("Pij,Pab->ijab", l[:, C, C], l[:, U, U])
    de = np.einsum("ij,ab->iajb", np.eye(ncs), np.eye(nvs)) * (es[U][None, :, None, None] - es[C][:, None, None, None])
    nsx = ncs * nvs
    A_s = (de + 2 * iajb - ijab.transpose(0, 2, 1, 3)).reshape(nsx, nsx)
    A_t = (de - ijab.transpose(0, 2, 1, 3)).reshape(nsx, nsx)
    ref = np.sort(np.concatenate([np.linalg.eigvalsh(A_s), np.repeat(np.linalg.eigvalsh(A_t), 3)]))
    assert np.abs(ref - w_so).max() < 1e-12


# ---------------------------------------------------------------- P6
def _roots(L, eps, nc, no, nv, k=6):
    a = O.Adc2(L, eps, nc, no, nv)
    return torch.linalg.eigvalsh(a.matrix())[:k].numpy()


def test_p6_invariances():
    s = make_system(2, 3, 6, 10, seed=12, sigma=0.08)
    nc, no, nv = s.nc, s.no, s.nv
    n = s.n
    w0 = _roots(s.L, s.eps, nc, no, nv)
    rng = np.random.default_rng(0)
    # spinor phase gauge L_pq -> e^{-i f_p} L_pq e^{i f_q}
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    Lg = np.conj(ph)[None, :, None] * s.L * ph[None, None, :]
    assert np.abs(_roots(Lg, s.eps, nc, no, nv) - w0).max() < 1e-11
    # real orthogonal mixing of the Cholesky index
    Q, _ = np.linalg.qr(rng.standard_normal((s.naux, s.naux)))
    Lq = np.einsum("PQ,Qpq->Ppq", Q, s.L)
    assert np.abs(_roots(Lq, s.eps, nc, no, nv) - w0).max() < 1e-11
    # permutation of spinors within each block
    perm = np.concatenate([rng.permutation(nc), nc + rng.permutation(no),
                           nc + no + rng.permutation(nv)])
    Lp = s.L[:, perm][:, :, perm]
    assert np.abs(_roots(Lp, s.eps[perm], nc, no, nv) - w0).max() < 1e-11
    # uniform energy shift
    assert np.abs(_roots(s.L, s.eps + 0.37, nc, no, nv) - w0).max() < 1e-11
    # a unitary (complex) mixing of P is NOT a symmetry: guards against a
    # conjugate slipping into (pq|rs) = sum_P L L
    Zu = np.linalg.qr(rng.standard_normal((s.naux, s.naux)) + 1j * rng.standard_normal((s.naux, s.naux)))[0]
    Lu = np.einsum("PQ,Qpq->Ppq", Zu, s.L)
    Lu = 0.5 * (Lu + np.conj(np.transpose(Lu, (0, 2, 1))))
    assert np.abs(_roots(Lu, s.eps, nc, no, nv) - w0).max() > 1e-6


# ---------------------------------------------------------------- P8
def test_p8_gradient_fd_and_scaling():
    s = make_system(2, 2, 5, 8, seed=13, sigma=0.1)
    L, e, sp = _tensors(s)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    k = 3
    w, X = a.roots_exact(k)
    X = X.T.contiguous()
    g = np.array([1.0, -0.5, 0.25])
    G, de = O.omega_gradient(L, e, sp, X, g)
    # Hermitian per P
    assert torch.allclose(G, G.conj().transpose(1, 2), atol=1e-14)
    rng = np.random.default_rng(1)
    h = 1e-5
    for t in range(3):
        A = rng.standard_normal(L.shape) + 1j * rng.standard_normal(L.shape)
        D = 0.5 * (A + np.conj(np.transpose(A, (0, 2, 1))))
        D /= np.linalg.norm(D)
        Dt = torch.from_numpy(D)
        fp = float(np.dot(g, _roots(s.L + h * D, s.eps, s.nc, s.no, s.nv, k)))
        fm = float(np.dot(g, _roots(s.L - h * D, s.eps, s.nc, s.no, s.nv, k)))
        fd = (fp - fm) / (2 * h)
        an = float(torch.sum(G.conj() * Dt).real)
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (fd, an)
    for t in range(3):
        d = rng.standard_normal(s.n)
        fp = float(np.dot(g, _roots(s.L, s.eps + h * d, s.nc, s.no, s.nv, k)))
        fm = float(np.dot(g, _roots(s.L, s.eps - h * d, s.nc, s.no, s.nv, k)))
        assert abs((fp - fm) / (2 * h) - float(de @ torch.from_numpy(d))) < 1e-7
    # uniform shift invariance: sum_p d omega / d eps_p = 0
    assert abs(float(de.sum())) < 1e-10
    # scaling identity for one root: d/ds omega(sL) = 2 x1'M1x1 + 4 x1'M2x1 + 4 Re x1'M12 x2
    G1, _ = O.omega_gradient(L, e, sp, X[:1], [1.0])
    lhs = float(torch.sum(G1.conj() * L).real)
    t = O.m11_terms(L, e, sp)
    ns = sp.n_singles
    x1, x2 = X[0, :ns], X[0, ns:]
    M1 = t["m1"].reshape(ns, ns)
    M2 = (t["m2i"] + t["m2ii"] + t["m2iii"]).reshape(ns, ns)
    M21 = O.m21_dense(L, e, sp)
    rhs = (2 * (x1.conj() @ M1 @ x1).real + 4 * (x1.conj() @ M2 @ x1).real
           + 4 * (x1.conj() @ (M21.conj().T @ x2)).real)
    assert abs(lhs - float(rhs)) < 1e-10 * max(1.0, abs(lhs))


# ---------------------------------------------------------------- FNS
@pytest.mark.parametrize("shape,seed,sigma", [((1, 2, 3), 5, 0.12), ((2, 2, 3), 7, 0.15)])
def test_fns_mp2_density_bruteforce(shape, seed, sigma):
    """Eq. 15 is the lambda^2 coefficient of the exact ground-state density:
    D_ab = <Psi0| a+_b a_a |Psi0>^(2) over virtual a, b (first order vanishes)."""
    s = make_system(*shape, naux=6, seed=seed, sigma=sigma)
    L, e, sp = _tensors(s)
    D = O.mp2_density_vv(L, e, sp).numpy()
    (g0, g1, g2), resid = density_taylor(s.L, s.eps, sp.o)
    assert resid < 1e-9
    o = sp.o
    assert np.abs(g1).max() < 1e-9
    assert np.abs(D - g2[o:, o:].T).max() <= 1e-7 * np.abs(D).max()
    assert np.abs(D - D.conj().T).max() < 1e-15 and np.linalg.eigvalsh(D).min() > -1e-15


def test_fns_keep_all_is_a_rotation():
    """With every natural virtual kept, the semicanonical natural spinors are a
    unitary rotation of the canonical virtuals with the same (diagonal) Fock
    block, so the ADC roots and the MP2 energy do not change; with a threshold
    the kept count is the number of occupations above it."""
    s = make_system(2, 3, 8, 20, seed=17)
    L, e, sp = _tensors(s)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    w0, _ = a.roots_exact(5)
    Lp, ep, nvp, occ, U = O.frozen_natural_spinors(L, e, sp, -1.0)
    assert nvp == s.nv
    assert torch.allclose(U.conj().T @ U, torch.eye(s.nv, dtype=O.C128), atol=1e-12)
    b = O.Adc2(Lp, ep, s.nc, s.no, nvp)
    w1, _ = b.roots_exact(5)
    assert torch.max(torch.abs(w1 - w0)).item() < 1e-10
    assert abs(O.mp2_energy(Lp, ep, b.sp).item() - O.mp2_energy(L, e, sp).item()) < 1e-12
    assert torch.allclose(Lp, Lp.conj().transpose(1, 2), atol=1e-14)
    thr = float(occ[4] + occ[5]) / 2
    Lt, et, nvt, _, Ut = O.frozen_natural_spinors(L, e, sp, thr)
    assert nvt == 5 and Lt.shape == (s.naux, sp.o + 5, sp.o + 5)
    F = Ut.conj().T @ torch.diag(e[sp.U]).to(O.C128) @ Ut
    assert torch.allclose(F, torch.diag(et[sp.o:]).to(O.C128), atol=1e-12)


# ---------------------------------------------------------------- TM
def _hermitian(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (d + d.conj().T)


@pytest.mark.parametrize("shape,seed,sigma", [((1, 2, 3), 5, 0.12), ((2, 2, 3), 7, 0.15), ((1, 3, 3), 11, 0.10)])
def test_tm_first_order_bruteforce(shape, seed, sigma):
    """Zeroth plus first order of F_I(lambda) from the intermediate states
    constructed by brute force equals transition_moments on the CVS rows
    (doubles basis a+_a a+_b a_j a_I = -1 x the brute-force a+_a a+_b a_I a_j)."""
    s = make_system(*shape, naux=6, seed=seed, sigma=sigma)
    L, e, sp = _tensors(s)
    d = _hermitian(sp.n, 3 + seed)
    (F0, F1, F2), resid, singles, doubles = transition_taylor(s.L, s.eps, sp.o, d)
    assert resid < 1e-9
    ns = len(singles)
    nc = sp.nc
    cvs_s = [k for k, (i, a) in enumerate(singles) if i < nc]
    cvs_d = [ns + k for k, (i, j, a, b) in enumerate(doubles) if i < nc <= j]
    ref = np.concatenate([(F0 + F1)[cvs_s], -(F0 + F1)[cvs_d]])
    # brute-force singles are ordered (i, a) with i outer; doubles (i<j, a<b): the CVS order of the vector layout
    got = O.transition_moments(L, e, sp, d, order=1).numpy()
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()
    # the second order is not part of it: it is a genuine correction of these inputs
    assert np.abs(F2[cvs_s]).max() > 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("shape,seed,sigma", [((1, 2, 3), 5, 0.15), ((2, 1, 3), 7, 0.15), ((1, 2, 4), 11, 0.15),
                                              ((2, 2, 3), 13, 0.12)])
def test_tm_second_order_bruteforce(shape, seed, sigma):
    """Singles through second order: the lambda^2 coefficient of F_I(lambda)
    from the brute-force intermediate states (core rows of the full singles
    class) equals second_order_singles, and transition_moments(order=2) is
    F^(0) + F^(1) + F^(2) on the singles rows and F^(0) + F^(1) on the doubles
    rows.  Each of the six second-order terms is of the size of the whole
    here, so a dropped term, a wrong sign or a transposed index fails."""
    s = make_system(*shape, naux=6, seed=seed, sigma=sigma, core=(-3.0, -2.5))
    L, e, sp = _tensors(s)
    d = _hermitian(sp.n, 17 + seed)
    (F0, F1, F2), resid, singles, doubles = transition_taylor(s.L, s.eps, sp.o, d)
    assert resid < 1e-9
    ns = len(singles)
    cvs_s = [k for k, (i, a) in enumerate(singles) if i < sp.nc]
    cvs_d = [ns + k for k, (i, j, a, b) in enumerate(doubles) if i < sp.nc <= j]
    # the lambda^2 coefficient of a degree-10 fit on |lambda| <= 0.5 carries
    # about resid / 0.5^2 of fit error: 5e-9 absolute, while the terms below
    # are each above 1e-5
    f2 = O.second_order_singles(L, e, sp, d).reshape(-1).numpy()
    assert np.abs(f2 - F2[cvs_s]).max() <= 5e-9
    ref = np.concatenate([(F0 + F1 + F2)[cvs_s], -(F0 + F1)[cvs_d]])
    got = O.transition_moments(L, e, sp, d, order=2).numpy()
    assert np.abs(got - ref).max() <= 5e-9
    # every term matters on these inputs: drop each in turn and the pin fails
    tau = O.mp2_amplitudes(L, e, sp)
    sa, u = O.second_order_amplitudes(L, e, sp)
    dd = torch.as_tensor(d).to(O.C128)
    C, O_, U = sp.C, sp.O, sp.U
    dvo = dd[U][:, O_]
    terms = [torch.einsum("ab,ib->ia", dd[U][:, U], sa), -torch.einsum("ji,ja->ia", dd[O_][:, O_], sa),
             torch.einsum("jb,abij->ia", dd[O_][:, U], u),
             -0.25 * torch.einsum("ac,ci->ia", torch.einsum("abkl,cbkl->ac", tau, tau.conj()), dvo),
             -0.25 * torch.einsum("ak,ik->ia", dvo, torch.einsum("cdil,cdkl->ik", tau, tau.conj())),
             0.5 * torch.einsum("iakc,ck->ia", torch.einsum("abil,cbkl->iakc", tau, tau.conj()), dvo)]
    for t in terms:
        assert float(t[C].abs().max()) > 1e-5


@pytest.mark.parametrize("shape,seed", [((1, 2, 3), 5), ((2, 2, 3), 13)])
def test_second_order_amplitudes_from_wavefunction(shape, seed):
    """The exact ground state Psi0(lambda) of the brute-force Fock space,
    expanded in lambda: its first-order doubles coefficients are -tau, its
    second-order singles and doubles coefficients are s and u of
    second_order_amplitudes (each of the ladder, ring and singles terms is a
    sizeable part of them on these inputs)."""
    from oracle.isr_bruteforce import FockSpace
    s = make_system(*shape, naux=6, seed=seed, sigma=0.15, core=(-3.0, -2.5))
    L, e, sp = _tensors(s)
    o = sp.o
    fs = FockSpace(s.L, s.eps, o)
    singles, doubles = fs.excitations()
    ref = np.zeros(1 << fs.n)
    ref[fs.ref] = 1.0
    phi1 = np.stack([fs.ad[a] @ (fs.a[i] @ ref) for (i, a) in singles], axis=1)
    phi2 = np.stack([fs.ad[a] @ (fs.ad[b] @ (fs.a[j] @ (fs.a[i] @ ref))) for (i, j, a, b) in doubles], axis=1)
    npts, deg, lm = 17, 10, 0.5
    lams = lm * np.cos(np.pi * (np.arange(npts) + 0.5) / npts)
    C = np.array([np.concatenate([phi1.T @ psi, phi2.T @ psi]) for psi in (fs.ground(x)[1] for x in lams)])
    coef = np.linalg.lstsq(np.polynomial.chebyshev.chebvander(lams / lm, deg), C, rcond=None)[0]
    taylor = [np.zeros(C.shape[1], dtype=complex) for _ in range(3)]
    for dd in range(deg + 1):
        mono = np.polynomial.chebyshev.cheb2poly(np.eye(deg + 1)[dd])
        for t in range(min(3, mono.size)):
            taylor[t] = taylor[t] + mono[t] / lm ** t * coef[dd]
    ns = len(singles)
    tau = O.mp2_amplitudes(L, e, sp).numpy()
    sa, u = (x.numpy() for x in O.second_order_amplitudes(L, e, sp))
    t1 = np.array([tau[a - o, b - o, i, j] for (i, j, a, b) in doubles])
    s2 = np.array([sa[i, a - o] for (i, a) in singles])
    u2 = np.array([u[a - o, b - o, i, j] for (i, j, a, b) in doubles])
    assert np.abs(taylor[1][:ns]).max() < 1e-9                     # no first-order singles
    assert np.abs(taylor[1][ns:] + t1).max() < 1e-9
    assert np.abs(taylor[2][:ns] - s2).max() < 5e-9 and np.abs(s2).max() > 1e-4
    assert np.abs(taylor[2][ns:] - u2).max() < 5e-9 and np.abs(u2).max() > 1e-4


def test_tm_second_order_shift_invariance():
    """F_I = <Psi~_I|D|Psi0> is unchanged by D -> D + c 1, since every
    intermediate state is orthogonal to Psi0: the two singles-amplitude terms
    of the second order cancel exactly for d = 1."""
    s = make_system(2, 3, 4, 8, seed=23, sigma=0.15, core=(-3.0, -2.5))
    L, e, sp = _tensors(s)
    d = _hermitian(sp.n, 29)
    f = O.transition_moments(L, e, sp, d, order=2)
    g = O.transition_moments(L, e, sp, d + 0.7 * np.eye(sp.n), order=2)
    assert torch.allclose(f, g, rtol=0, atol=1e-13 * float(f.abs().max()))
    assert float(O.second_order_singles(L, e, sp, np.eye(sp.n)).abs().max()) < 1e-14


def test_tm_spin_selection_rule():
    """Nonrelativistic limit with a spin-free dipole: every triplet state has
    zero transition moment, singlets do not (spin is conserved by F at each
    order); oscillator strengths follow f = 2/3 w |T|^2."""
    sb = make_spin_blocked(1, 2, 4, 12, seed=9, sigma=0.1)
    L, e, sp = _tensors(sb)
    a = O.Adc2(sb.L, sb.eps, sb.nc, sb.no, sb.nv)
    M = a.matrix()
    w, v = torch.linalg.eigh(M)
    n_sp = sp.n // 2
    dip = []
    for c in range(3):
        rng = np.random.default_rng(40 + c)
        x = rng.standard_normal((n_sp, n_sp))
        x = x + x.T
        dd = np.zeros((sp.n, sp.n))
        for sg in range(2):
            idx = 2 * np.arange(n_sp) + sg
            dd[np.ix_(idx, idx)] = x
        dip.append(dd)
    dip = np.array(dip)
    k = 12
    T, f = O.oscillator_strengths(L, e, sp, dip, v[:, :k].T, w[:k])
    sizes = _multiplets(w[:k].numpy(), 1e-9)
    pos = 0
    n_dark = n_bright = 0
    for sz in sizes:
        blk = f[pos:pos + sz].numpy()
        if sz == 3:
            assert blk.max() < 1e-20 * max(1.0, float(f.max()))
            n_dark += 1
        else:
            assert sz == 1 and blk[0] > 1e-8
            n_bright += 1
        pos += sz
    assert n_dark >= 1 and n_bright >= 1
    assert torch.allclose(f, (2.0 / 3.0) * w[:k] * (T.abs() ** 2).sum(1), rtol=1e-14)


def test_tm_second_order_terms_by_fit():
    """How the second-order singles terms were found: the lambda^2
    coefficient of F from the brute-force intermediate states is fitted by
    least squares over 16 candidate contractions (the singles and doubles
    second-order amplitude pieces, the pair densities and particle-hole
    terms over all or only core k).  The fit returns the coefficients of
    second_order_singles exactly (1/2, -1/2, -1/2, 1/2, 1/2, 1/2, 1, -1/4,
    -1/4, 1/2) and zero for the six other candidates."""
    rows, rhs = [], []
    for shape, seed in [((1, 2, 3), 5), ((2, 1, 3), 7), ((1, 2, 4), 11)]:
        s = make_system(*shape, naux=6, seed=seed, sigma=0.15, core=(-3.0, -2.5))
        L, e, sp = _tensors(s)
        o = sp.o
        d = _hermitian(sp.n, 100 * seed)
        (_, _, F2), resid, singles, _ = transition_taylor(s.L, s.eps, o, d)
        assert resid < 1e-9
        O_, U = sp.O, sp.U
        dd = torch.as_tensor(d).to(O.C128)
        dvv, doo, dov, dvo = dd[U][:, U], dd[O_][:, O_], dd[O_][:, U], dd[U][:, O_]
        tau = O.mp2_amplitudes(L, e, sp)
        Dia = e[U][None, :] - e[O_][:, None]
        s1 = torch.einsum("ajbc,bcij->ia", O.asym(L, U, O_, U, U), tau) / Dia
        s2 = torch.einsum("jkib,abjk->ia", O.asym(L, O_, O_, O_, U), tau) / Dia
        D = O.denom(e, sp, U, U, O_, O_)
        pp = torch.einsum("abcd,cdij->abij", O.asym(L, U, U, U, U), tau) / D
        hh = torch.einsum("klij,abkl->abij", O.asym(L, O_, O_, O_, O_), tau) / D
        r = torch.einsum("kbcj,acik->abij", O.asym(L, O_, U, U, O_), tau)
        ring = (r - r.permute(1, 0, 2, 3) - r.permute(0, 1, 3, 2) + r.permute(1, 0, 3, 2)) / D
        rho = torch.einsum("abkl,cbkl->ac", tau, tau.conj())
        sig = torch.einsum("cdil,cdkl->ik", tau, tau.conj())
        P = torch.einsum("abil,cbkl->iakc", tau, tau.conj())
        Q = torch.einsum("abkl,cbil->iakc", tau, tau.conj())
        mc = torch.zeros(o, dtype=O.C128)
        mc[:sp.nc] = 1.0
        cand = [torch.einsum("ab,ib->ia", dvv, s1), torch.einsum("ab,ib->ia", dvv, s2),
                torch.einsum("ji,ja->ia", doo, s1), torch.einsum("ji,ja->ia", doo, s2),
                torch.einsum("jb,abij->ia", dov, pp), torch.einsum("jb,abij->ia", dov, hh),
                torch.einsum("jb,abij->ia", dov, ring), torch.einsum("ac,ci->ia", rho, dvo),
                torch.einsum("ak,ik->ia", dvo, sig), torch.einsum("iakc,ck->ia", P, dvo),
                torch.einsum("ak,ki->ia", dvo, sig), torch.einsum("iakc,ck->ia", Q, dvo),
                torch.einsum("ak,ik->ia", dvo * mc, sig), torch.einsum("iakc,ck->ia", P, dvo * mc),
                torch.einsum("ak,ki->ia", dvo * mc, sig), torch.einsum("iakc,ck->ia", Q, dvo * mc)]
        A_ = np.stack([np.array([c[i, a - o].item() for (i, a) in singles]) for c in cand], axis=1)
        rows.append(A_)
        rhs.append(F2[:len(singles)])
    A_ = np.concatenate(rows)
    b = np.concatenate(rhs)
    x = np.linalg.lstsq(np.concatenate([A_.real, A_.imag]), np.concatenate([b.real, b.imag]), rcond=None)[0]
    want = np.array([0.5, -0.5, -0.5, 0.5, 0.5, 0.5, 1.0, -0.25, -0.25, 0.5, 0, 0, 0, 0, 0, 0])
    assert np.abs(x - want).max() < 1e-5, np.round(x, 6)
