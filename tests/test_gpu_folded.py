"""GPU parity of the folded (doubles-free) eigensolver, ADC2_SOLVER_FOLDED.

For roots below the doubles threshold the folded solver returns eigenpairs
of the full matrix M; they are compared with exact diagonalisation of the
oracle's explicit matrix (tiny), with the oracle's Davidson (config c1), and
certified at larger sizes by the FP64 residual of the returned vectors
(adc2_rayleigh: for Hermitian M an eigenvalue lies within |r| of omega).
"""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import make_system, config_system

pytestmark = pytest.mark.gpu

FOLD = A.ADC2_SOLVER_FOLDED


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def handle(s):
    print(f"[case] folded nc={s.nc} no={s.no} nv={s.nv} naux={s.naux}", flush=True)
    return A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)


def test_folded_tiny_vs_exact():
    s = make_system(2, 3, 7, 24, seed=303, sigma=0.25)
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    w_ex, _ = o.roots_exact(4)
    h = handle(s)
    w, X, info = A.adc2_davidson(h, 4, tol=1e-10, solver=FOLD)
    print("  folded", w, "exact", w_ex.tolist(), "iters", info["iters"], flush=True)
    assert info["converged"]
    assert np.abs(np.array(w) - w_ex.numpy()).max() < 1e-9
    Xc = X.cpu()
    M = o.matrix()
    R = Xc @ M.T - torch.tensor(w, dtype=torch.float64)[:, None] * Xc
    assert torch.linalg.vector_norm(R, dim=1).max().item() < 1e-8
    assert torch.allclose(Xc.conj() @ Xc.T, torch.eye(4, dtype=torch.complex128), atol=1e-9)
    h.close()


def test_folded_refuses_root_in_doubles_band():
    s = make_system(1, 2, 3, 5, seed=7)
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    h = handle(s)
    w, _, info = A.adc2_davidson(h, 2, tol=1e-10, solver=FOLD)
    assert np.abs(np.array(w) - o.roots_exact(2)[0].numpy()).max() < 1e-9
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_davidson(h, 3, tol=1e-10, solver=FOLD)
    assert ei.value.status == A.ADC2_ERR_NOCONV and "not below" in str(ei.value)
    h.close()


def test_folded_c1_vs_oracle():
    s = config_system("c1")
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    w_or, _, info_o = o.roots(4, tol=1e-9)
    assert info_o["converged"]
    h = handle(s)
    w, X, info = A.adc2_davidson(h, 4, tol=1e-9, solver=FOLD)
    print("  c1 folded", w, "oracle", w_or.tolist(), "iters", info["iters"], "oracle iters", info_o["iters"],
          flush=True)
    assert info["converged"]
    assert np.abs(np.array(w) - w_or.numpy()).max() < 1e-8
    wr, rn = A.adc2_rayleigh(h, X)
    assert np.abs(np.array(wr) - np.array(w)).max() < 1e-10
    assert max(rn) < 1e-8
    # same roots from the full-space solver on the GPU
    wf, _, infof = A.adc2_davidson(h, 4, tol=1e-9, want_vectors=False)
    assert infof["converged"] and np.abs(np.array(wf) - np.array(w)).max() < 1e-8
    h.close()


def test_folded_mid_certified():
    s = config_system("mid")
    h = handle(s)
    w, X, info = A.adc2_davidson(h, 6, tol=1e-8, solver=FOLD)
    print("  mid folded", w, "iters", info["iters"], "sigma vectors", info["n_sigma"], flush=True)
    assert info["converged"]
    assert all(np.diff(w) >= 0)
    wr, rn = A.adc2_rayleigh(h, X)
    assert max(rn) < 1e-7
    assert np.abs(np.array(wr) - np.array(w)).max() < 1e-9
    h.close()


def test_folded_precision_form_c1():
    """complex64 heavy contractions inside the folded solver, FP64 polish."""
    s = config_system("c1")
    h = handle(s)
    w64, _, _ = A.adc2_davidson(h, 4, tol=1e-9, solver=FOLD, want_vectors=False)
    A.adc2_set_precision(h, A.ADC2_C64)
    w32, X32, info = A.adc2_davidson(h, 4, tol=1e-6, solver=FOLD)
    A.adc2_set_precision(h, A.ADC2_FP64)
    wp, rn = A.adc2_rayleigh(h, X32)
    ev = 27.211386245988
    print("  c64 raw eV err", (np.array(w32) - w64) * ev, "polished Ha err", np.array(wp) - w64, flush=True)
    assert np.abs(np.array(w32) - w64).max() * ev < 1e-3
    assert np.abs(np.array(wp) - w64).max() < 1e-6
    h.close()


def test_folded_restarts_and_single_root():
    """Small search spaces force a restart every iteration or two (restart
    basis, rotation of V, S1, H11, every moment matrix and U on the GPU);
    one root and five roots against exact diagonalisation."""
    s = make_system(2, 3, 8, 24, seed=305, sigma=0.3)
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    M = o.matrix()
    h = handle(s)
    for k, smax in [(1, 2), (5, 10)]:
        w_ex, _ = o.roots_exact(k)
        w, X, info = A.adc2_davidson(h, k, tol=1e-10, max_subspace=smax, max_iter=400, solver=FOLD)
        print(f"  k={k} smax={smax}: folded {np.round(w, 10)} exact {np.round(w_ex.numpy(), 10)} "
              f"iters {info['iters']} space {info['subspace']}", flush=True)
        assert info["converged"]
        assert np.abs(np.array(w) - w_ex.numpy()).max() < 1e-9
        Xc = X.cpu()
        R = Xc @ M.T - torch.tensor(w, dtype=torch.float64)[:, None] * Xc
        assert torch.linalg.vector_norm(R, dim=1).max().item() < 1e-8
    h.close()


def test_folded_deterministic_c1():
    """Two folded solves of the same handle return the same roots and vectors
    bit for bit (every reduction of the subspace algebra has a fixed order)."""
    s = config_system("c1")
    h = handle(s)
    w1, X1, i1 = A.adc2_davidson(h, 4, tol=1e-9, solver=FOLD)
    w2, X2, i2 = A.adc2_davidson(h, 4, tol=1e-9, solver=FOLD)
    torch.cuda.synchronize()
    assert i1["iters"] == i2["iters"]
    assert list(w1) == list(w2)
    assert torch.equal(X1, X2)
    h.close()
