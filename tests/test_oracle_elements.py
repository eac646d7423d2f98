"""Pins of the oracle's single-element evaluators against its whole-matrix
forms.

The full-size GPU parity tests compare sampled entries of M11 and of sigma
with `m11_element`, `sigma2_element` and `sigma1_coupling_element`, because
the whole matrices do not fit the CPU there.  Those three functions restate
the singles block (second-order singles terms of ADC(2), pinned by the
brute-force intermediate states) and the first-order coupling one entry at a
time.  Here every entry of small systems is compared with `m11()` and with
the matrix-free `Sigma`, both of which the brute-force construction pins
(tests/test_oracle_pins.py).  The shapes cover nc < no, nc > no, a single
occupied valence spinor and two virtuals, so every index kind (I == J,
I != J, a == b, first and last a and b) is hit.

The mutants at the end restate an evaluator with one plausible slip and
assert that the comparison made here sees it.
"""
import itertools

import numpy as np
import pytest
import torch

from synth import make_system, random_vectors
from oracle import adc2 as O

SHAPES = [
    # (nc, no, nv, naux, seed)
    (2, 3, 4, 7, 101),     # nc < no
    (3, 2, 5, 6, 102),     # nc > no
    (1, 1, 2, 5, 103),     # one core, one valence, two virtuals
    (2, 4, 6, 9, 104),
]


def _system(nc, no, nv, naux, seed):
    s = make_system(nc, no, nv, naux, seed=seed, sigma=0.12)
    return O.as_c128(s.L), O.as_f64(s.eps), O.Spaces(nc, no, nv)


@pytest.mark.parametrize("shape", SHAPES)
def test_m11_element_every_entry(shape):
    L, e, sp = _system(*shape)
    M = O.m11(L, e, sp).reshape(sp.nc, sp.nv, sp.nc, sp.nv)
    scale = float(M.abs().max())
    worst = 0.0
    for I, a, J, b in itertools.product(range(sp.nc), range(sp.nv), range(sp.nc), range(sp.nv)):
        v = O.m11_element(L, e, sp, I, a, J, b)
        worst = max(worst, abs(v - complex(M[I, a, J, b])))
    assert worst < 1e-13 * scale, worst


def _doubles_positions(sp):
    for I, j in itertools.product(range(sp.nc), range(sp.no)):
        for a in range(sp.nv):
            for b in range(a + 1, sp.nv):
                q = a * sp.nv - a * (a + 1) // 2 + (b - a - 1)
                yield I, j, a, b, sp.n_singles + (I * sp.no + j) * sp.n_pairs + q


@pytest.mark.parametrize("shape", SHAPES)
def test_sigma2_element_every_entry(shape):
    L, e, sp = _system(*shape)
    x = torch.from_numpy(random_vectors(shape[-1], 1, sp.dim)[0])
    s = O.Sigma(L, e, sp)(x)
    scale = float(s.abs().max())
    n = 0
    for I, j, a, b, pos in _doubles_positions(sp):
        v = O.sigma2_element(L, e, sp, x, I, j, a, b)
        assert abs(v - complex(s[pos])) < 1e-13 * scale, (I, j, a, b)
        n += 1
    assert n == sp.n_doubles


@pytest.mark.parametrize("shape", SHAPES)
def test_sigma1_coupling_element_every_entry(shape):
    L, e, sp = _system(*shape)
    x = torch.from_numpy(random_vectors(shape[-1] + 7, 1, sp.dim)[0])
    x[:sp.n_singles] = 0          # sigma1 of a doubles-only vector is M12 x2
    s = O.Sigma(L, e, sp)(x)
    scale = float(s[:sp.n_singles].abs().max())
    for K, c in itertools.product(range(sp.nc), range(sp.nv)):
        v = O.sigma1_coupling_element(L, sp, x, K, c)
        assert abs(v - complex(s[K * sp.nv + c])) < 1e-13 * scale, (K, c)


# ---------------------------------------------------------------- mutants
def _m11_element_mutant(L, eps, sp, I, a, J, b, slip):
    """m11_element restated with one slip."""
    o, C, O_, U = sp.o, sp.C, sp.O, sp.U
    A_, B_ = O._one(o + a), O._one(o + b)
    I_, J_ = O._one(I), O._one(J)
    val = complex(O.asym(L, A_, J_, I_, B_).reshape(()))
    if I == J and a == b:
        val += float(eps[o + a] - eps[I])
    eU, eO = eps[U], eps[O_]
    if I == J:
        W_a = O.asym(L, A_, U, O_, O_)[0]
        W_b = O.asym(L, O_, O_, B_, U)[:, :, 0]
        Da = eps[o + a] + eU[:, None, None] - eO[None, :, None] - eO[None, None, :]
        Db = eps[o + b] + eU[:, None, None] - eO[None, :, None] - eO[None, None, :]
        Wb = W_b.permute(2, 0, 1)
        inv = (1 / Da + 1 / Da) if slip == "term i: 1/Da twice" else (1 / Da + 1 / Db)
        val += complex(0.25 * torch.sum(W_a * Wb * inv))
    if a == b:
        W_J = O.asym(L, J_, O_, U, U)[0]
        W_I = O.asym(L, U, U, I_, O_)[:, :, 0]
        DI = eU[:, None, None] + eU[None, :, None] - eps[I] - eO[None, None, :]
        DJ = eU[:, None, None] + eU[None, :, None] - eps[J] - eO[None, None, :]
        if slip == "term ii: no transpose of <Jk||cd>":
            val += complex(0.25 * torch.sum(W_J.permute(2, 1, 0) * W_I * (1 / DI + 1 / DJ)))
        else:
            val += complex(0.25 * torch.sum(W_J.permute(1, 2, 0) * W_I * (1 / DI + 1 / DJ)))
    W_aI = O.asym(L, A_, U, I_, O_)[0, :, 0]
    W_Jb = O.asym(L, J_, O_, B_, U)[0, :, 0]
    D1 = eps[o + a] + eU[:, None] - eps[I] - eO[None, :]
    D2 = eps[o + b] + eU[:, None] - eps[J] - eO[None, :]
    sign = 0.5 if slip == "term iii: sign" else -0.5
    val += complex(sign * torch.sum(W_aI * W_Jb.T * (1 / D1 + 1 / D2)))
    return val


def _sigma2_element_mutant(L, eps, sp, x, I, j, a, b, slip):
    o, nc, nv = sp.o, sp.nc, sp.nv
    x1 = x[:sp.n_singles].reshape(nc, nv)
    q = a * nv - a * (a + 1) // 2 + (b - a - 1)
    x2 = x[sp.n_singles + (I * sp.no + j) * sp.n_pairs + q]
    D = eps[o + a] + eps[o + b] - eps[I] - eps[nc + j]
    jj = O._one(nc + j)
    Wc = O.asym(L, O._one(o + a), O._one(o + b), sp.U, jj)[0, 0, :, 0]
    Gb = O.asym(L, sp.C, O._one(o + b), O._one(I), jj)[:, 0, 0, 0]
    Ga = O.asym(L, sp.C, O._one(o + a), O._one(I), jj)[:, 0, 0, 0]
    ga = -1.0 if slip == "Ga sign" else 1.0
    wc = Wc.conj() if slip == "conj <ab||cj>" else Wc
    val = D * x2 + torch.sum(wc * x1[I]) - torch.sum(Gb * x1[:, a]) + ga * torch.sum(Ga * x1[:, b])
    return complex(val)


def _sigma1_coupling_mutant(L, sp, x, K, c, slip):
    nc, no, nv = sp.nc, sp.no, sp.nv
    ia, ib = O.pair_index(nv)
    U = torch.zeros(nc, no, nv, nv, dtype=O.C128)
    U[:, :, ia, ib] = x[sp.n_singles:].reshape(nc, no, sp.n_pairs)
    W = O.asym(L, sp.U, sp.U, O._one(sp.o + c), sp.V)[:, :, 0, :]
    G = O.asym(L, O._one(K), sp.U, sp.C, sp.V)[0]
    Gc = G if slip == "no conj on <Kb||Ij>" else G.conj()
    t1 = torch.einsum("abj,jab->", W.conj(), U[K])
    t2 = torch.einsum("bIj,Ijb->", Gc, U[:, :, c, :])
    t3 = torch.einsum("aIj,Ija->", Gc, U[:, :, :, c])
    if slip == "t3 sign":
        t3 = -t3
    return complex(t1 - t2 + t3)


def test_element_mutants_are_caught():
    L, e, sp = _system(*SHAPES[0])
    M = O.m11(L, e, sp).reshape(sp.nc, sp.nv, sp.nc, sp.nv)
    scale = float(M.abs().max())
    entries = list(itertools.product(range(sp.nc), range(sp.nv), range(sp.nc), range(sp.nv)))
    for slip in ["term i: 1/Da twice", "term ii: no transpose of <Jk||cd>", "term iii: sign"]:
        worst = max(abs(_m11_element_mutant(L, e, sp, I, a, J, b, slip) - complex(M[I, a, J, b]))
                    for I, a, J, b in entries)
        assert worst > 1e-6 * scale, slip

    x = torch.from_numpy(random_vectors(SHAPES[0][-1], 1, sp.dim)[0])
    s = O.Sigma(L, e, sp)(x)
    for slip in ["Ga sign", "conj <ab||cj>"]:
        worst = max(abs(_sigma2_element_mutant(L, e, sp, x, I, j, a, b, slip) - complex(s[pos]))
                    for I, j, a, b, pos in _doubles_positions(sp))
        assert worst > 1e-6 * float(s.abs().max()), slip

    x0 = x.clone()
    x0[:sp.n_singles] = 0
    s0 = O.Sigma(L, e, sp)(x0)
    for slip in ["no conj on <Kb||Ij>", "t3 sign"]:
        worst = max(abs(_sigma1_coupling_mutant(L, sp, x0, K, c, slip) - complex(s0[K * sp.nv + c]))
                    for K, c in itertools.product(range(sp.nc), range(sp.nv)))
        assert worst > 1e-6 * float(s0[:sp.n_singles].abs().max()), slip

    # the unmutated restatements agree (the mutants differ only by the slip)
    for I, a, J, b in entries[:20]:
        assert abs(_m11_element_mutant(L, e, sp, I, a, J, b, None) - complex(M[I, a, J, b])) < 1e-13 * scale


@pytest.mark.parametrize("shape", SHAPES)
def test_m11_row_every_row(shape):
    """m11_row (the row evaluator the full-size GPU tests compare whole rows
    of M11 with) equals m11() on every row; without term (i) it differs only
    on the J == I block, and there by term (i) itself (nonzero)."""
    L, e, sp = _system(*shape)
    M = O.m11(L, e, sp).reshape(sp.nc, sp.nv, sp.nc, sp.nv)
    ti = O.m11_terms(L, e, sp)["m2i"]
    scale = float(M.abs().max())
    for I, a in itertools.product(range(sp.nc), range(sp.nv)):
        r = O.m11_row(L, e, sp, I, a)
        assert float((r - M[I, a]).abs().max()) < 1e-13 * scale
        r0 = O.m11_row(L, e, sp, I, a, with_term_i=False)
        d = r0 - M[I, a]
        assert float((d + ti[I, a]).abs().max()) < 1e-13 * scale
    assert float(ti.abs().max()) > 1e3 * 1e-13 * scale     # far above the comparison tolerance
