"""Brute-force intermediate-state representation in a tiny Fock space.

TEST INFRASTRUCTURE ONLY (used by the oracle's pinning tests).

This follows the paper's own definition of the ADC secular matrix (Theory
section, Eq. 4-11) with no ADC formula in it:

  * H(lambda) = sum_p e_p a+_p a_p + lambda V_N with
    V_N = 1/4 sum <pq||rs> a+_p a+_q a_s a_r - sum_pq u_pq a+_p a_q,
    u_pq = sum_{i occ} <pi||qi>.  The one-body correction makes diag(e) the
    exact Fock matrix of the reference determinant (Moller-Plesset
    partitioning, Brillouin condition), as the normal-ordered Hamiltonians of
    Eq. 1-2 assume.
  * Psi0(lambda), E0(lambda): exact ground state by full diagonalisation.
  * Correlated excited states C_J Psi0 with C_J = a+_a a_i and
    a+_a a+_b a_i a_j (i<j, a<b)  (Eq. 4-5).
  * Precursors: Gram-Schmidt against all lower excitation classes (Eq. 6),
    then symmetric orthonormalisation S^{-1/2} inside each class (Eq. 7-8).
  * M_IJ = <Psi~_I| H - E0 |Psi~_J>  (Eq. 9).
  * The perturbation expansion of M (Eq. 12) is read off as the Taylor
    coefficients of M(lambda) at lambda = 0 by a least-squares polynomial fit
    on Chebyshev points.

Integrals: (pq|rs) = sum_P L^P_pq L^P_rs and <pq||rs> = (pr|qs) - (ps|qr).
"""
from __future__ import annotations

import itertools

import numpy as np


def _annihilators(n):
    """Jordan-Wigner a_p as dense (2^n x 2^n) matrices; bit p = occupation of p."""
    dim = 1 << n
    ops = []
    for p in range(n):
        a = np.zeros((dim, dim))
        for s in range(dim):
            if (s >> p) & 1:
                sign = -1.0 if bin(s & ((1 << p) - 1)).count("1") % 2 else 1.0
                a[s ^ (1 << p), s] = sign
        ops.append(a)
    return ops


class FockSpace:
    def __init__(self, L, eps, nocc):
        self.L = np.asarray(L, dtype=np.complex128)
        self.eps = np.asarray(eps, dtype=np.float64)
        self.n = self.eps.size
        self.nocc = nocc
        n = self.n
        self.a = _annihilators(n)
        self.ad = [x.T.copy() for x in self.a]
        # <pq||rs>
        J = np.einsum("Ppr,Pqs->pqrs", self.L, self.L)       # (pr|qs) at [p,q,r,s]
        K = np.einsum("Pps,Pqr->pqrs", self.L, self.L)       # (ps|qr)
        self.g = J - K
        occ = range(nocc)
        u = np.zeros((n, n), dtype=np.complex128)
        for i in occ:
            u += self.g[:, i, :, i]
        self.u = u
        dim = 1 << n
        H0 = np.zeros((dim, dim), dtype=np.complex128)
        for p in range(n):
            H0 += self.eps[p] * (self.ad[p] @ self.a[p])
        V1 = np.zeros((dim, dim), dtype=np.complex128)
        for p in range(n):
            for q in range(n):
                if self.u[p, q] != 0:
                    V1 -= self.u[p, q] * (self.ad[p] @ self.a[q])
        # two-body: 1/4 sum g_pqrs a+_p a+_q a_s a_r
        pair = {}
        for r in range(n):
            for s in range(n):
                if r != s:
                    pair[(r, s)] = self.a[s] @ self.a[r]
        V2 = np.zeros((dim, dim), dtype=np.complex128)
        for p in range(n):
            for q in range(n):
                if p == q:
                    continue
                B = np.zeros((dim, dim), dtype=np.complex128)
                for (r, s), A in pair.items():
                    gv = self.g[p, q, r, s]
                    if gv != 0:
                        B += gv * A
                V2 += 0.25 * (self.ad[p] @ self.ad[q]) @ B
        self.H0 = H0
        self.V = V1 + V2
        counts = np.array([bin(s).count("1") for s in range(dim)])
        self.sector = np.nonzero(counts == nocc)[0]
        self.ref = (1 << nocc) - 1        # lowest nocc spinors occupied

    def ground(self, lam):
        H = self.H0 + lam * self.V
        idx = self.sector
        Hs = H[np.ix_(idx, idx)]
        w, v = np.linalg.eigh(Hs)
        psi = np.zeros(1 << self.n, dtype=np.complex128)
        psi[idx] = v[:, 0]
        c = psi[self.ref]
        psi *= np.conj(c) / abs(c)
        return w[0], psi, H

    def excitations(self):
        occ = list(range(self.nocc))
        vir = list(range(self.nocc, self.n))
        singles = [(i, a) for i in occ for a in vir]
        doubles = [(i, j, a, b) for i, j in itertools.combinations(occ, 2)
                   for a, b in itertools.combinations(vir, 2)]
        return singles, doubles

    def isr_matrix(self, lam):
        """ISR secular matrix over [singles | doubles] and E0 at coupling lam."""
        E0, psi, H = self.ground(lam)
        singles, doubles = self.excitations()
        P1 = np.stack([self.ad[a] @ (self.a[i] @ psi) for (i, a) in singles], axis=1)
        P2 = np.stack([self.ad[a] @ (self.ad[b] @ (self.a[i] @ (self.a[j] @ psi)))
                       for (i, j, a, b) in doubles], axis=1)
        # class 1: orthogonalise against Psi0, then S^-1/2
        P1 = P1 - np.outer(psi, np.conj(psi) @ P1)
        T1 = _sym_orth(P1)
        # class 2: orthogonalise against Psi0 and class 1, then S^-1/2
        lower = np.concatenate([psi[:, None], T1], axis=1)
        P2 = P2 - lower @ (np.conj(lower.T) @ P2)
        T2 = _sym_orth(P2)
        T = np.concatenate([T1, T2], axis=1)
        Hm = H - E0 * np.eye(H.shape[0])
        M = np.conj(T.T) @ Hm @ T
        return M, E0

    def taylor(self, nterms=3, degree=10, npts=17, lam_max=0.5):
        """Taylor coefficients M^(0..nterms-1) and E0^(0..nterms-1) at lambda=0."""
        k = np.arange(npts)
        lams = lam_max * np.cos(np.pi * (k + 0.5) / npts)
        Ms, Es = [], []
        for lam in lams:
            M, E0 = self.isr_matrix(lam)
            Ms.append(M)
            Es.append(E0)
        Ms = np.array(Ms)
        Es = np.array(Es)
        x = lams / lam_max
        Vm = np.polynomial.chebyshev.chebvander(x, degree)
        coefM = np.linalg.lstsq(Vm, Ms.reshape(npts, -1), rcond=None)[0]
        coefE = np.linalg.lstsq(Vm, Es, rcond=None)[0]
        resid = np.abs(Vm @ coefM - Ms.reshape(npts, -1)).max()
        # Chebyshev -> monomial in x, then x = lam / lam_max
        outM, outE = [], []
        for nidx in range(nterms):
            outM.append(np.zeros(Ms.shape[1:], dtype=np.complex128))
            outE.append(0.0)
        for d in range(degree + 1):
            e = np.zeros(degree + 1)
            e[d] = 1.0
            mono = np.polynomial.chebyshev.cheb2poly(e)
            for nidx in range(min(nterms, mono.size)):
                f = mono[nidx] / lam_max ** nidx
                outM[nidx] = outM[nidx] + f * coefM[d].reshape(Ms.shape[1:])
                outE[nidx] = outE[nidx] + f * coefE[d]
        return outM, np.array(outE), resid


def transition_taylor(L, eps, nocc, d, nterms=3, degree=10, npts=17, lam_max=0.5):
    """Taylor coefficients at lambda = 0 of the modified transition moments
    F_I(lambda) = <Psi~_I| D |Psi0> (Theory section: transition properties)
    of the one-particle operator D = sum_pq d_pq a+_p a_q, over the
    intermediate states [singles | doubles] of isr_matrix.  Returns
    ([F^(0), F^(1), ...], fit residual)."""
    fs = FockSpace(L, eps, nocc)
    n = fs.n
    dim = 1 << n
    Dop = np.zeros((dim, dim), dtype=np.complex128)
    for p in range(n):
        for q in range(n):
            if d[p][q] != 0:
                Dop += d[p][q] * (fs.ad[p] @ fs.a[q])
    singles, doubles = fs.excitations()
    k = np.arange(npts)
    lams = lam_max * np.cos(np.pi * (k + 0.5) / npts)
    Fs = []
    for lam in lams:
        _, psi, _ = fs.ground(lam)
        P1 = np.stack([fs.ad[a] @ (fs.a[i] @ psi) for (i, a) in singles], axis=1)
        P2 = np.stack([fs.ad[a] @ (fs.ad[b] @ (fs.a[i] @ (fs.a[j] @ psi)))
                       for (i, j, a, b) in doubles], axis=1)
        P1 = P1 - np.outer(psi, np.conj(psi) @ P1)
        T1 = _sym_orth(P1)
        lower = np.concatenate([psi[:, None], T1], axis=1)
        P2 = P2 - lower @ (np.conj(lower.T) @ P2)
        T2 = _sym_orth(P2)
        T = np.concatenate([T1, T2], axis=1)
        Fs.append(np.conj(T.T) @ (Dop @ psi))
    Fs = np.array(Fs)
    x = lams / lam_max
    Vm = np.polynomial.chebyshev.chebvander(x, degree)
    coef = np.linalg.lstsq(Vm, Fs, rcond=None)[0]
    resid = np.abs(Vm @ coef - Fs).max()
    out = [np.zeros(Fs.shape[1], dtype=np.complex128) for _ in range(nterms)]
    for dd in range(degree + 1):
        e = np.zeros(degree + 1)
        e[dd] = 1.0
        mono = np.polynomial.chebyshev.cheb2poly(e)
        for t in range(min(nterms, mono.size)):
            out[t] = out[t] + (mono[t] / lam_max ** t) * coef[dd]
    return out, resid, singles, doubles


def density_taylor(L, eps, nocc, nterms=3, degree=10, npts=17, lam_max=0.5):
    """Taylor coefficients at lambda = 0 of the exact ground-state one-particle
    density gamma_pq(lambda) = <Psi0(lambda)| a+_p a_q |Psi0(lambda)> (Psi0
    normalised), read off by the same Chebyshev least-squares fit as the ISR
    matrix.  Returns ([gamma^(0), gamma^(1), ...], fit residual)."""
    fs = FockSpace(L, eps, nocc)
    n = fs.n
    k = np.arange(npts)
    lams = lam_max * np.cos(np.pi * (k + 0.5) / npts)
    G = []
    for lam in lams:
        _, psi, _ = fs.ground(lam)
        g = np.empty((n, n), dtype=np.complex128)
        for p in range(n):
            for q in range(n):
                g[p, q] = np.conj(psi) @ (fs.ad[p] @ (fs.a[q] @ psi))
        G.append(g)
    G = np.array(G)
    x = lams / lam_max
    Vm = np.polynomial.chebyshev.chebvander(x, degree)
    coef = np.linalg.lstsq(Vm, G.reshape(npts, -1), rcond=None)[0]
    resid = np.abs(Vm @ coef - G.reshape(npts, -1)).max()
    out = [np.zeros((n, n), dtype=np.complex128) for _ in range(nterms)]
    for d in range(degree + 1):
        e = np.zeros(degree + 1)
        e[d] = 1.0
        mono = np.polynomial.chebyshev.cheb2poly(e)
        for t in range(min(nterms, mono.size)):
            out[t] = out[t] + (mono[t] / lam_max ** t) * coef[d].reshape(n, n)
    return out, resid


def determinant_doubles_block(L, eps, nc, no, nv):
    """Matrix of the fluctuation potential V_N between the CVS doubly
    excited determinants a+_a a+_b a_j a_I |Phi0> (I core, j valence, a<b),
    minus its reference expectation value <Phi0|V_N|Phi0> (the first-order
    energy, subtracted with E0 in M = H - E0), straight from the Fock-space
    operators: the first-order doubles block with no intermediate-state
    construction and no fit."""
    o = nc + no
    fs = FockSpace(L, eps, o)
    ref = np.zeros(1 << fs.n, dtype=np.complex128)
    ref[fs.ref] = 1.0
    vecs = []
    for I in range(nc):
        for j in range(nc, o):
            for a, b in itertools.combinations(range(o, fs.n), 2):
                vecs.append(fs.ad[a] @ (fs.ad[b] @ (fs.a[j] @ (fs.a[I] @ ref))))
    T = np.stack(vecs, axis=1)
    e1 = np.conj(ref) @ fs.V @ ref
    return np.conj(T.T) @ fs.V @ T - e1 * np.eye(T.shape[1])


def _sym_orth(P):
    S = np.conj(P.T) @ P
    w, U = np.linalg.eigh(S)
    Sih = (U / np.sqrt(w)) @ np.conj(U.T)
    return P @ Sih


def adc2_blocks(L, eps, nc, no, nv, **fit):
    """ADC(2) blocks from the brute-force ISR.

    Returns a dict with
      M11_full : singles block through 2nd order over all occupied i  [(i,a),(j,b)]
      M11_cvs  : its core-core sub-block  [(I,a),(J,b)]
      M21_cvs  : first-order coupling rows (I, j valence, a<b) in the basis
                 a+_a a+_b a_j a_I |Phi0> (= -1 x the a+_a a+_b a_I a_j state)
      M22_cvs  : zeroth-order doubles block on the same rows
      M22x_cvs : first-order doubles block on the same rows (ADC(2)-x)
      E_mp2    : second-order ground-state energy (lambda^2 coefficient)
      fit_resid: max residual of the polynomial fit
    """
    o = nc + no
    fs = FockSpace(L, eps, o)
    singles, doubles = fs.excitations()
    (M0, M1, M2), E, resid = fs.taylor(**fit)
    ns = len(singles)
    adc = M0 + M1 + M2
    M11_full = adc[:ns, :ns]
    cvs_s = [k for k, (i, a) in enumerate(singles) if i < nc]
    cvs_d = [k for k, (i, j, a, b) in enumerate(doubles) if i < nc <= j]
    M11_cvs = M11_full[np.ix_(cvs_s, cvs_s)]
    sign = -1.0
    M21 = (M0 + M1)[ns:, :ns]
    M21_cvs = sign * M21[np.ix_(cvs_d, cvs_s)]
    M22_cvs = M0[ns:, ns:][np.ix_(cvs_d, cvs_d)]
    # first-order doubles block (the extension of ADC(2)-x); the basis sign
    # of the doubles rows cancels between bra and ket
    M22x_cvs = M1[ns:, ns:][np.ix_(cvs_d, cvs_d)]
    return {"M11_full": M11_full, "M11_cvs": M11_cvs, "M21_cvs": M21_cvs,
            "M22_cvs": M22_cvs, "M22x_cvs": M22x_cvs, "E_mp2": E[2], "E1": E[1], "E0": E[0],
            "fit_resid": resid, "orders": (M0, M1, M2), "singles": singles,
            "doubles": doubles}
