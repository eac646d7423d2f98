"""GPU parity of the transition moments and oscillator strengths
(adc2_transition) against the oracle's transition_moments /
oscillator_strengths (Theory section), singles of F through second order
(the default) and through first order.

T = X^H F is linear in X, so random vectors as well as eigenvectors probe F
element by element in projection: 8 random directions x 3 Cartesian
components, and the 4 lowest eigenvectors with their oscillator strengths.
In the nonrelativistic limit with a spin-free dipole every triplet root is
dark on the GPU as well.

Tolerance: both sides are FP64; the second-order terms are sums over up to
naux nv (ladder) or o nv (ring, densities) products of O(1e-2) values, whose
rounding differs between the GEMMs and the oracle's einsum.  Relative
1e-11 of max |T| covers a random-walk error of sqrt(K) 1.1e-16 with a wide
margin and is far below the second-order part itself (checked to be above
1e-4 of max |T|).
"""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import dipole_integrals, make_spin_blocked, make_system, random_vectors

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("shape,seed", [((2, 4, 14, 30), 51), ((1, 3, 17, 24), 52), ((3, 2, 11, 20), 53)])
def test_transition_parity(shape, seed):
    s = make_system(*shape, seed=seed)
    sp = O.Spaces(s.nc, s.no, s.nv)
    dip = dipole_integrals(seed, sp.n)
    print(f"[case] transition moments {shape}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    L, e = O.as_c128(s.L), O.as_f64(s.eps)
    Xr = random_vectors(seed, 8, h.dim)
    for order, tol in ((1, 1e-12), (2, 1e-11)):
        Fo = O.transition_moments(L, e, sp, dip, order=order).numpy()   # [3][dim]
        T, f = A.adc2_transition(h, dev(dip), dev(Xr), [1.0] * 8, order=order)
        Tref = Xr.conj() @ Fo.T
        err = np.abs(T - Tref).max() / np.abs(Tref).max()
        print(f"  order {order} random directions: max rel err {err:.2e}", flush=True)
        assert err < tol
    # the second order is a real part of these T
    F1 = O.transition_moments(L, e, sp, dip, order=1).numpy()
    assert np.abs(Tref - Xr.conj() @ F1.T).max() > 1e-4 * np.abs(Tref).max()
    # eigenvectors and oscillator strengths
    w, X, inf = A.adc2_davidson(h, 4, tol=1e-10)
    T, f = A.adc2_transition(h, dev(dip), X, w)
    Tr, fr = O.oscillator_strengths(L, e, sp, dip, X.cpu(), w)
    ef = np.abs(f - fr.numpy()).max() / np.abs(fr.numpy()).max()
    print(f"  roots {np.round(w, 6)} f {np.round(f, 6)}  rel err {ef:.2e}", flush=True)
    assert np.abs(T - Tr.numpy()).max() < 1e-11 * np.abs(Tr.numpy()).max()
    assert ef < 1e-11
    h.close()


@pytest.mark.parametrize("shape,seed", [((1, 1, 3, 5), 61), ((2, 1, 5, 9), 62), ((3, 1, 2, 6), 63)])
def test_transition_tiny_shapes(shape, seed):
    """Edge shapes of the second-order path: a single occupied pair
    (o = 2), more core than valence spinors, two virtuals (one virtual
    pair); random directions only."""
    s = make_system(*shape, seed=seed)
    sp = O.Spaces(s.nc, s.no, s.nv)
    dip = dipole_integrals(seed, sp.n)
    print(f"[case] transition tiny {shape}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    Xr = random_vectors(seed, 3, h.dim)
    for order in (1, 2):
        Fo = O.transition_moments(O.as_c128(s.L), O.as_f64(s.eps), sp, dip, order=order).numpy()
        T, _ = A.adc2_transition(h, dev(dip), dev(Xr), [1.0] * 3, order=order)
        Tref = Xr.conj() @ Fo.T
        err = np.abs(T - Tref).max() / np.abs(Tref).max()
        print(f"  order {order}: max rel err {err:.2e}", flush=True)
        assert err < 1e-11
    h.close()


def test_transition_with_folded_eigenvectors_c1():
    """Eigenvectors of the folded solver (doubles rebuilt from the singles) at
    nc=6, no=10, nv=40, naux=150: GPU transition moments against the oracle's
    with the same vectors."""
    from synth import config_system
    s = config_system("c1")
    sp = O.Spaces(s.nc, s.no, s.nv)
    dip = dipole_integrals(7, sp.n)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    w, X, inf = A.adc2_davidson(h, 4, tol=1e-9, solver=A.ADC2_SOLVER_FOLDED)
    T, f = A.adc2_transition(h, dev(dip), X, w)
    Tr, fr = O.oscillator_strengths(O.as_c128(s.L), O.as_f64(s.eps), sp, dip, X.cpu(), w)
    err = np.abs(T - Tr.numpy()).max() / np.abs(Tr.numpy()).max()
    print(f"[case] folded c1: f {np.round(f, 5)} rel err {err:.2e}", flush=True)
    assert err < 1e-11
    assert np.abs(f - fr.numpy()).max() < 1e-11 * np.abs(fr.numpy()).max()
    h.close()


def test_transition_spin_selection_rule():
    sb = make_spin_blocked(1, 2, 4, 12, seed=9, sigma=0.1)
    sp = O.Spaces(sb.nc, sb.no, sb.nv)
    n_sp = sp.n // 2
    rng = np.random.default_rng(44)
    dip = np.zeros((3, sp.n, sp.n), dtype=np.complex128)
    for c in range(3):
        x = rng.standard_normal((n_sp, n_sp))
        x = x + x.T
        for sg in range(2):
            idx = 2 * np.arange(n_sp) + sg
            dip[c][np.ix_(idx, idx)] = x
    h = A.adc2_setup(dev(sb.L), dev(sb.eps), sb.nc, sb.no, sb.nv, sb.naux)
    w, X, inf = A.adc2_davidson(h, 8, tol=1e-10)
    T, f = A.adc2_transition(h, dev(dip), X, w)
    h.close()
    w = np.array(w)
    groups, cur = [], [0]
    for i in range(1, len(w)):
        if w[i] - w[cur[-1]] < 1e-7:
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    print(f"[case] spin selection: roots {np.round(w, 6)} f {f}", flush=True)
    dark = [g for g in groups if len(g) == 3]
    bright = [g for g in groups if len(g) == 1 and g[0] < len(w) - 1]
    assert dark and bright
    for g in dark:
        assert f[g].max() < 1e-18 * max(1.0, f.max())
    assert max(f[g[0]] for g in bright) > 1e-6


def test_transition_argument_errors():
    s = make_system(1, 2, 5, 12, seed=4)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    dip = dev(dipole_integrals(1, s.nc + s.no + s.nv))
    X = torch.zeros(33, h.dim, dtype=torch.complex128, device="cuda")
    with pytest.raises(A.Adc2Error):
        A.adc2_transition(h, dip, X, [1.0] * 33)
    with pytest.raises(A.Adc2Error):
        A.adc2_transition(h, dip, X[:2], [1.0] * 2, order=3)
    h.close()


def test_transition_c2_shift_invariance():
    """nc=6, no=60, nv=300, naux=1500, second order, 4 random directions.
    Every intermediate state is orthogonal to Psi0, so T is unchanged by
    d -> d + c 1 at any size: at second order this needs the two
    singles-amplitude terms to cancel to rounding across the whole
    occupied space, and the remaining terms to see no diagonal of d.  The
    second-order part itself is checked to be present."""
    from synth import config_system
    s = config_system("c2")
    n = s.nc + s.no + s.nv
    print(f"[case] transition c2 shift invariance", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    dip = dipole_integrals(11, n)
    X = dev(random_vectors(12, 4, h.dim))
    T1, _ = A.adc2_transition(h, dev(dip), X, [1.0] * 4, order=1)
    T2, _ = A.adc2_transition(h, dev(dip), X, [1.0] * 4, order=2)
    Ts, _ = A.adc2_transition(h, dev(dip + 0.7 * np.eye(n)[None]), X, [1.0] * 4, order=2)
    h.close()
    err = np.abs(Ts - T2).max() / np.abs(T2).max()
    print(f"  shift: rel change {err:.2e}; second-order part {np.abs(T2 - T1).max() / np.abs(T2).max():.2e}",
          flush=True)
    assert err < 1e-12
    assert np.abs(T2 - T1).max() > 1e-3 * np.abs(T2).max()


def test_transition_spin_selection_rule_larger():
    """The selection rule at order 2 on a nonrelativistic system whose GEMMs
    span ragged tiles (nc=6, no=20, nv=160 spinors, naux=160): every triplet
    root is dark to rounding, the singlets are not."""
    sb = make_spin_blocked(3, 10, 80, 160, seed=19, sigma=0.05)
    sp = O.Spaces(sb.nc, sb.no, sb.nv)
    n_sp = sp.n // 2
    rng = np.random.default_rng(45)
    dip = np.zeros((3, sp.n, sp.n), dtype=np.complex128)
    for c in range(3):
        x = rng.standard_normal((n_sp, n_sp))
        x = x + x.T
        for sg in range(2):
            idx = 2 * np.arange(n_sp) + sg
            dip[c][np.ix_(idx, idx)] = x
    print("[case] spin selection rule, nc=6 no=20 nv=160", flush=True)
    h = A.adc2_setup(dev(sb.L), dev(sb.eps), sb.nc, sb.no, sb.nv, sb.naux)
    w, X, inf = A.adc2_davidson(h, 8, tol=1e-9, solver=A.ADC2_SOLVER_FOLDED)
    T, f = A.adc2_transition(h, dev(dip), X, w, order=2)
    h.close()
    w = np.array(w)
    groups, cur = [], [0]
    for i in range(1, len(w)):
        if w[i] - w[cur[-1]] < 1e-7:
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    print(f"  roots {np.round(w, 6)} f {f}", flush=True)
    dark = [g for g in groups if len(g) == 3]
    bright = [g for g in groups if len(g) == 1 and g[0] < len(w) - 1]
    assert dark and bright
    for g in dark:
        assert f[g].max() < 1e-18 * max(1.0, f.max())     # measured <= 3e-21
    assert max(f[g[0]] for g in bright) > 1e-6


@pytest.mark.parametrize("shape,seed", [((1, 2, 5, 9), 61), ((2, 3, 6, 12), 62)])
def test_transition_F_element_by_element(shape, seed):
    """F itself, entry by entry: with unit vectors e_i as X (groups of at most
    32, the entry point's limit) T_i = e_i^H F = F_i for each Cartesian
    component; compared with the oracle's F through first and second order
    (singles and doubles, every entry)."""
    s = make_system(*shape, seed=seed)
    sp = O.Spaces(s.nc, s.no, s.nv)
    dip = dipole_integrals(seed, sp.n)
    print(f"[case] transition F element by element {shape} dim={sp.dim}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    L, e = O.as_c128(s.L), O.as_f64(s.eps)
    dd = dev(dip)
    for order, tol in ((1, 1e-12), (2, 1e-11)):
        Fo = O.transition_moments(L, e, sp, dip, order=order).numpy()   # [3][dim]
        Fg = np.zeros((3, sp.dim), dtype=np.complex128)
        for i0 in range(0, sp.dim, 32):
            k = min(32, sp.dim - i0)
            E = torch.zeros((k, sp.dim), dtype=torch.complex128)
            E[torch.arange(k), i0 + torch.arange(k)] = 1.0
            T, _ = A.adc2_transition(h, dd, E.cuda(), [1.0] * k, order=order)
            Fg[:, i0:i0 + k] = T.T
        err = np.abs(Fg - Fo).max() / np.abs(Fo).max()
        print(f"  order {order}: F max rel err {err:.2e} over {3 * sp.dim} entries", flush=True)
        assert err < tol
        assert np.abs(Fo[:, sp.n_singles:]).max() > 1e-3 * np.abs(Fo).max()   # the doubles of F are compared too
    h.close()
