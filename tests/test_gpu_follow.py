"""GPU parity of root following (adc2_davidson with follow=1, the
root-specific Davidson): each root converges to the eigenpair of M whose
eigenvector overlaps most with its guess vector, in guess order, as the
oracle's roots_following selects it from the exact eigendecomposition of
the explicit matrix.

Two kinds of guesses: exact eigenvectors of chosen non-lowest states plus a
random perturbation (the follower must home in on those states, not on the
lowest ones), and singles-only CVS-CIS eigenvectors (the paper's guesses),
for which the followed ADC(2) states are those of largest CIS character.
"""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import make_system

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(s, refs, tol=1e-9):
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    g = dev(refs.numpy())
    w, X, inf = A.adc2_davidson(h, refs.shape[0], tol=tol, guess=g, nguess=refs.shape[0], follow=True)
    h.close()
    return np.array(w), X.cpu(), inf


def margin(M, refs, w_sel):
    """smallest gap between the chosen overlap and the next best, per reference"""
    w, v = torch.linalg.eigh(M)
    ov = (refs.conj() @ v).abs() ** 2
    out = []
    for j in range(refs.shape[0]):
        l = int(torch.argmin((w - w_sel[j]).abs()))
        others = torch.cat([ov[j, :l], ov[j, l + 1:]])
        out.append(float(ov[j, l] - others.max()))
    return min(out)


def test_follow_perturbed_eigenvectors():
    s = make_system(1, 3, 8, 20, seed=12)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    M = a.matrix()
    w_all, v_all = torch.linalg.eigh(M)
    pick = [4, 1, 9]
    rng = np.random.default_rng(3)
    noise = torch.from_numpy(rng.standard_normal((3, a.dim)) + 1j * rng.standard_normal((3, a.dim)))
    noise = noise / torch.linalg.vector_norm(noise, dim=1, keepdim=True)
    refs = v_all[:, pick].T + 0.25 * noise
    print(f"[case] follow perturbed eigenvectors {pick} dim {a.dim}", flush=True)
    w_ref, X_ref = O.roots_following(M, refs)
    assert np.abs(w_ref.numpy() - w_all[pick].numpy()).max() < 1e-12   # the perturbed guesses still pick the targets
    w, X, inf = run(s, refs)
    print(f"  gpu {w}  oracle {w_ref.numpy()}  its {inf['iters']}", flush=True)
    assert inf["converged"]
    assert np.abs(w - w_ref.numpy()).max() < 1e-9
    # the returned vectors are those eigenvectors (up to phase)
    ovl = (X.conj() @ X_ref).abs().diagonal()
    assert (ovl - 1).abs().max().item() < 1e-8


def test_follow_cis_guesses():
    s = make_system(2, 3, 9, 24, seed=8)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    sp = a.sp
    M = a.matrix()
    M1 = O.m11(a.L, a.eps, sp, order=1)
    wc, vc = torch.linalg.eigh(M1)
    pick = [0, 2, 5]
    refs = torch.zeros(3, a.dim, dtype=O.C128)
    refs[:, :sp.n_singles] = vc[:, pick].T
    w_ref, X_ref = O.roots_following(M, refs)
    mg = margin(M, refs, w_ref)
    print(f"[case] follow CIS states {pick}: oracle {w_ref.numpy()} overlap margin {mg:.3f}", flush=True)
    assert mg > 0.05
    w, X, inf = run(s, refs)
    print(f"  gpu {w}  its {inf['iters']}", flush=True)
    assert inf["converged"]
    assert np.abs(w - w_ref.numpy()).max() < 1e-9


def test_follow_argument_errors():
    s = make_system(1, 2, 5, 12, seed=4)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    with pytest.raises(A.Adc2Error):
        A.adc2_davidson(h, 2, follow=True)                       # no guess
    g = torch.zeros(2, h.dim, dtype=torch.complex128, device="cuda")
    g[0, 0] = 1
    g[1, 1] = 1
    with pytest.raises(A.Adc2Error):
        A.adc2_davidson(h, 2, follow=True, solver=A.ADC2_SOLVER_FOLDED)     # no guess
    with pytest.raises(A.Adc2Error):
        A.adc2_davidson(h, 2, guess=g, nguess=1, follow=True, solver=A.ADC2_SOLVER_FOLDED)   # fewer than roots
    h.close()


# ---------------------------------------------------------------- folded solver
FOLD = A.ADC2_SOLVER_FOLDED


def strong_system():
    """A system whose lowest 16 roots lie below min D (coupling sigma 0.3)."""
    return make_system(2, 3, 8, 24, seed=305, sigma=0.3)


def run_folded(s, refs, tol=1e-9):
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    g = dev(refs.numpy())
    w, X, inf = A.adc2_davidson(h, refs.shape[0], tol=tol, guess=g, nguess=refs.shape[0], follow=True,
                                solver=FOLD)
    h.close()
    return np.array(w), X.cpu(), inf


def test_follow_folded_perturbed_eigenvectors():
    """The folded solver follows roots by the overlap of its Ritz singles with
    the guesses' singles (the doubles of a Ritz vector are a function of its
    singles); targets are non-lowest states below min D."""
    s = strong_system()
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    M = a.matrix()
    w_all, v_all = torch.linalg.eigh(M)
    Dmin = float(O.m22_diag(a.eps, a.sp).min())
    pick = [4, 1, 9]
    assert float(w_all[max(pick)]) < Dmin - 0.5
    rng = np.random.default_rng(3)
    noise = torch.from_numpy(rng.standard_normal((3, a.dim)) + 1j * rng.standard_normal((3, a.dim)))
    noise = noise / torch.linalg.vector_norm(noise, dim=1, keepdim=True)
    refs = v_all[:, pick].T + 0.25 * noise
    w_ref, X_ref = O.roots_following(M, refs)
    assert np.abs(w_ref.numpy() - w_all[pick].numpy()).max() < 1e-12
    print(f"[case] folded follow perturbed eigenvectors {pick}", flush=True)
    w, X, inf = run_folded(s, refs)
    print(f"  gpu {w}  oracle {w_ref.numpy()}  its {inf['iters']}", flush=True)
    assert inf["converged"]
    assert np.abs(w - w_ref.numpy()).max() < 1e-9
    ovl = (X.conj() @ X_ref).abs().diagonal()
    assert (ovl - 1).abs().max().item() < 1e-8


def test_follow_folded_cis_guesses():
    s = strong_system()
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    sp = a.sp
    M = a.matrix()
    M1 = O.m11(a.L, a.eps, sp, order=1)
    wc, vc = torch.linalg.eigh(M1)
    pick = [0, 2, 5]
    refs = torch.zeros(3, a.dim, dtype=O.C128)
    refs[:, :sp.n_singles] = vc[:, pick].T
    w_ref, _ = O.roots_following(M, refs)
    print(f"[case] folded follow CIS states {pick}: oracle {w_ref.numpy()} margin {margin(M, refs, w_ref):.3f}",
          flush=True)
    assert not np.all(np.diff(w_ref.numpy()) > 0)      # not simply the lowest roots in order
    w, X, inf = run_folded(s, refs)
    print(f"  gpu {w}  its {inf['iters']}", flush=True)
    assert inf["converged"]
    assert np.abs(w - w_ref.numpy()).max() < 1e-9


def test_follow_folded_equals_full_space_c1():
    """At c1 (no explicit matrix on the host) the folded and the full-space
    solvers follow the same CIS guesses to the same roots, each certified by
    its FP64 residual."""
    from synth import config_system
    s = config_system("c1")
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    M1 = O.m11(a.L, a.eps, a.sp, order=1)
    wc, vc = torch.linalg.eigh(M1)
    pick = [0, 2, 5, 3]
    refs = torch.zeros(len(pick), a.dim, dtype=O.C128)
    refs[:, :a.sp.n_singles] = vc[:, pick].T
    print(f"[case] follow c1 folded vs full space, CIS states {pick}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    g = dev(refs.numpy())
    wf, Xf, inf_f = A.adc2_davidson(h, len(pick), tol=1e-9, guess=g, nguess=len(pick), follow=True, solver=FOLD)
    wa, Xa, inf_a = A.adc2_davidson(h, len(pick), tol=1e-9, guess=g, nguess=len(pick), follow=True,
                                    max_iter=400)
    print(f"  folded {np.round(wf, 9)} ({inf_f['iters']} it)  full {np.round(wa, 9)} ({inf_a['iters']} it)",
          flush=True)
    assert inf_f["converged"] and inf_a["converged"]
    assert np.abs(np.array(wf) - np.array(wa)).max() < 1e-8
    for X in (Xf, Xa):
        wr, rn = A.adc2_rayleigh(h, X)
        assert max(rn) < 1e-8
    h.close()
