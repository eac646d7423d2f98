"""Pins of the oracle's ADC(2)-x doubles block (the extended scheme the
paper's Conclusions name as the next step): the first-order doubles-doubles
block of the intermediate-state matrix.

  X1  the oracle's block equals the first-order Taylor coefficient of the
      brute-force intermediate-state matrix on the CVS doubles (Eq. 6-12,
      the same construction as pin P1), three shapes;
  X2  it equals the matrix of the fluctuation potential between the CVS
      doubly excited determinants, computed from the Fock-space operators
      with no intermediate states and no fit;
  X3  the closed-form diagonal is the diagonal of the block; the explicit
      ADC(2)-x matrix is Hermitian; the matrix-free sigma equals it;
  X4  the oracle Davidson reaches the eigenvalues of the explicit matrix;
  X5  nonrelativistic limit: real matrix, eigenvalues in singlets and
      exact triplets;
  mutants of the block (ring sign, core ring dropped, ladder factor, hole
      ladder transposed) each break X1 by far more than the fit error.
"""
import numpy as np
import pytest
import torch

from synth import make_system, make_spin_blocked, random_vectors
from oracle import adc2 as O
from oracle.isr_bruteforce import adc2_blocks, determinant_doubles_block

CASES = [((1, 2, 3), 5, 0.12), ((2, 2, 3), 7, 0.15), ((1, 3, 3), 11, 0.10)]


def _sys(shape, seed, sigma):
    nc, no, nv = shape
    s = make_system(nc, no, nv, 8, seed=seed, sigma=sigma, core=(-3.0, -2.5))
    return s, O.as_c128(s.L), O.as_f64(s.eps), O.Spaces(nc, no, nv)


@pytest.mark.parametrize("shape,seed,sigma", CASES)
def test_x1_bruteforce_first_order_doubles(shape, seed, sigma):
    s, L, e, sp = _sys(shape, seed, sigma)
    bf = adc2_blocks(s.L, s.eps, *shape)
    assert bf["fit_resid"] < 1e-10
    ours = O.m22x_dense(L, sp).numpy()
    ref = bf["M22x_cvs"]
    assert np.abs(ref).max() > 0.05
    assert np.abs(ours - ref).max() < 1e-9


@pytest.mark.parametrize("shape,seed,sigma", CASES + [((2, 3, 4), 13, 0.2)])
def test_x2_determinant_matrix_elements(shape, seed, sigma):
    s, L, e, sp = _sys(shape, seed, sigma)
    ref = determinant_doubles_block(s.L, s.eps, *shape)
    ours = O.m22x_dense(L, sp).numpy()
    assert np.abs(ours - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("shape,seed,sigma", [((2, 3, 4), 13, 0.2), ((3, 2, 5), 17, 0.1)])
def test_x3_diagonal_hermiticity_sigma(shape, seed, sigma):
    s, L, e, sp = _sys(shape, seed, sigma)
    Mx = O.m22x_dense(L, sp)
    assert torch.allclose(torch.diagonal(Mx).real, O.m22x_diag(L, sp), atol=1e-14, rtol=0)
    assert float(torch.diagonal(Mx).imag.abs().max()) < 1e-15
    M = O.explicit_matrix(L, e, sp, "adc2x")
    assert float((M - M.conj().T).abs().max()) <= 1e-14 * float(M.abs().max())
    x = torch.from_numpy(random_vectors(3, 3, sp.dim))
    got = O.Sigma(L, e, sp, method="adc2x")(x)
    assert float((got - x @ M.T).abs().max()) < 1e-13 * float(got.abs().max())
    d = O.diagonal(L, e, sp, "adc2x")
    assert torch.allclose(d, torch.diagonal(M).real, atol=1e-13, rtol=0)
    # ADC(2)-x differs from ADC(2) only in the doubles block
    M2 = O.explicit_matrix(L, e, sp)
    ns = sp.n_singles
    assert torch.equal(M[:ns], M2[:ns]) and torch.equal(M[:, :ns], M2[:, :ns])


def test_x4_davidson_matches_exact():
    s = make_system(2, 3, 7, 16, seed=101)
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv, method="adc2x")
    w_ex, _ = o.roots_exact(4)
    w, X, info = o.roots(4, tol=1e-10, max_iter=300)
    assert info["converged"]
    assert float((w - w_ex).abs().max()) < 1e-10
    # the extension moves the roots
    w2, _ = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv).roots_exact(4)
    assert float((w - w2).abs().max()) > 1e-4


def test_x5_nonrelativistic_triplets():
    s = make_spin_blocked(1, 2, 3, 6, seed=23, sigma=0.08)
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv, method="adc2x")
    M = o.matrix()
    assert float(M.imag.abs().max()) < 1e-14
    w = np.sort(np.linalg.eigvalsh(M.real.numpy()))
    # group eigenvalues into clusters; every cluster has size 1, 3 or more (singlet/triplet/quintet)
    groups, cur = [], [w[0]]
    for v in w[1:]:
        if v - cur[-1] < 1e-9:
            cur.append(v)
        else:
            groups.append(cur)
            cur = [v]
    groups.append(cur)
    sizes = [len(g) for g in groups]
    assert 3 in sizes
    assert all(sz != 2 for sz in sizes)
    for g in groups:
        assert g[-1] - g[0] < 1e-10


def _sigx_mutant(ints, U, slip):
    t = (1.0 if slip == "ladder factor 1" else 0.5) * torch.einsum("abcd,mIjcd->mIjab", ints["vvvv"], U)
    hl = "IjKk,mKkab->mIjab" if slip == "hole ladder transposed" else "KkIj,mKkab->mIjab"
    t = t + torch.einsum(hl, ints["cvcv"], U)
    r = torch.einsum("kbcj,mIkac->mIjab", ints["VvvV"], U)
    if slip != "core ring dropped":
        r = r + torch.einsum("KbcI,mKjac->mIjab", ints["cvvc"], U)
    if slip == "ring sign":
        r = -r
    return t + r - r.transpose(3, 4)


def test_x_mutants_are_caught():
    shape = (2, 2, 3)
    s, L, e, sp = _sys(shape, 7, 0.15)
    ref = adc2_blocks(s.L, s.eps, *shape)["M22x_cvs"]
    ints = O.adc2x_integrals(L, sp)
    nd = sp.n_doubles
    ia, ib = O.pair_index(sp.nv)
    U = torch.zeros(nd, sp.nc, sp.no, sp.nv, sp.nv, dtype=O.C128)
    U[:, :, :, ia, ib] = torch.eye(nd, dtype=O.C128).reshape(nd, sp.nc, sp.no, sp.n_pairs)
    U = U - U.transpose(3, 4)
    for slip in ["ladder factor 1", "hole ladder transposed", "core ring dropped", "ring sign", None]:
        M = _sigx_mutant(ints, U, slip)[:, :, :, ia, ib].reshape(nd, nd).T.numpy()
        dev = np.abs(M - ref).max()
        if slip is None:
            assert dev < 1e-9
        else:
            assert dev > 1e-4, slip
