"""GPU parity of CVS-ADC(2)-x (adc2_set_method(h, ADC2_METHOD_ADC2X)): the
ADC(2) matrix with the first-order doubles-doubles block, against the
oracle's ADC(2)-x (pinned by the brute-force intermediate states and by the
determinant matrix elements, tests/test_oracle_adc2x.py).

Parity: sigma element by element (1e-11 relative, FP64) at an edge shape,
tiny, ragged tiles, c1 and mid; the diagonal; roots against exact
diagonalisation (tiny) and the oracle Davidson (c1); switching back to
ADC(2) restores its sigma bit for bit; the folded solver, the adjoint and the
no-allocation sigma refuse ADC(2)-x.
"""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import make_system, config_system, random_vectors

pytestmark = pytest.mark.gpu

TOL = 1e-11


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def system(name):
    if name == "edge":
        return make_system(1, 1, 2, 3, seed=7)
    if name == "tiny":
        return make_system(2, 3, 7, 16, seed=101)
    if name == "ragged":
        return make_system(3, 2, 65, 70, seed=8)
    return config_system(name)


def handle_x(s):
    print(f"[case] adc2x nc={s.nc} no={s.no} nv={s.nv} naux={s.naux}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    A.adc2_set_method(h, A.ADC2_METHOD_ADC2X)
    return h


@pytest.mark.parametrize("name,m", [("edge", 2), ("tiny", 3), ("ragged", 2), ("tiles", 2), ("c1", 3), ("mid", 2)])
def test_adc2x_sigma_matches_oracle(name, m):
    s = system(name)
    h = handle_x(s)
    x = random_vectors(41, m, h.dim)
    S = A.adc2_sigma(h, dev(x)).cpu()
    ref = O.Sigma(O.as_c128(s.L), O.as_f64(s.eps), O.Spaces(s.nc, s.no, s.nv), method="adc2x")(torch.from_numpy(x))
    err = float((S - ref).abs().max() / ref.abs().max())
    print(f"  sigma rel err {err:.2e}", flush=True)
    assert err < TOL
    d = A.adc2_get_diag(h).cpu()
    dref = O.diagonal(O.as_c128(s.L), O.as_f64(s.eps), O.Spaces(s.nc, s.no, s.nv), "adc2x")
    assert float((d - dref).abs().max() / dref.abs().max()) < TOL
    # back to ADC(2): the sigma of a fresh ADC(2) handle, bit for bit
    A.adc2_set_method(h, A.ADC2_METHOD_ADC2)
    S2 = A.adc2_sigma(h, dev(x))
    h2 = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    S3 = A.adc2_sigma(h2, dev(x))
    torch.cuda.synchronize()
    assert torch.equal(S2, S3)
    assert torch.equal(A.adc2_get_diag(h), A.adc2_get_diag(h2))
    h.close()
    h2.close()


def test_adc2x_roots_tiny_exact():
    s = system("tiny")
    h = handle_x(s)
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv, method="adc2x")
    w_ex, V = o.roots_exact(4)
    w, X, info = A.adc2_davidson(h, 4, tol=1e-10, max_iter=300)
    print("  roots", w, "exact", w_ex.tolist(), flush=True)
    assert info["converged"]
    assert np.abs(np.array(w) - w_ex.numpy()).max() < 1e-9
    Xc = X.cpu()
    R = Xc @ o.matrix().T - torch.tensor(w, dtype=torch.float64)[:, None] * Xc
    assert float(torch.linalg.vector_norm(R, dim=1).max()) < 1e-8
    h.close()


def test_adc2x_roots_c1_vs_oracle():
    s = system("c1")
    h = handle_x(s)
    w, X, info = A.adc2_davidson(h, 4, tol=1e-9, max_iter=400)
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv, method="adc2x")
    w_or, _, inf = o.roots(4, tol=1e-9, max_iter=300)
    print("  gpu", w, "oracle", w_or.tolist(), "iters", info["iters"], inf["iters"], flush=True)
    assert info["converged"] and inf["converged"]
    assert np.abs(np.array(w) - w_or.numpy()).max() < 1e-8
    # the FP64 Rayleigh quotients of the returned vectors under ADC(2)-x
    wr, rn = A.adc2_rayleigh(h, X)
    assert np.abs(np.array(wr) - np.array(w)).max() < 1e-10 and max(rn) < 1e-8
    # ADC(2)-x moves the roots away from ADC(2)'s
    w2, _ = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv).roots(4, tol=1e-9, max_iter=300)[:2]
    assert np.abs(np.array(w) - w2.numpy()).min() > 1e-3
    h.close()


def test_adc2x_refusals_and_precision_form():
    s = system("tiny")
    h = handle_x(s)
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_davidson(h, 2, tol=1e-8, solver=A.ADC2_SOLVER_FOLDED)
    assert ei.value.status == A.ADC2_ERR_ARG and "folded" in str(ei.value)
    X = dev(random_vectors(3, 2, h.dim))
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_omega_backward(h, X, [1.0, 1.0])
    assert ei.value.status == A.ADC2_ERR_ARG
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_sigma_noalloc(h, X, torch.empty_like(X))
    assert ei.value.status == A.ADC2_ERR_ARG
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_set_method(h, 7)
    assert ei.value.status == A.ADC2_ERR_ARG
    # complex64 heavy contractions beside the FP64 first-order doubles block
    A.adc2_set_precision(h, A.ADC2_C64)
    S = A.adc2_sigma(h, X).cpu()
    ref = O.Sigma(O.as_c128(s.L), O.as_f64(s.eps), O.Spaces(s.nc, s.no, s.nv), method="adc2x")(X.cpu())
    err = float((S - ref).abs().max() / ref.abs().max())
    print(f"  complex64 sigma rel err {err:.2e}", flush=True)
    assert err < 2e-6
    h.close()
