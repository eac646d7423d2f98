"""GPU parity of the adjoint adc2_omega_backward (Hellmann-Feynman gradient
of the eigenvalues with respect to the Cholesky vectors and the energies).

Parity: for fixed vectors X and weights g the library returns the gradient of
f = sum_k g_k x_k^H M x_k / x_k^H x_k; the oracle's omega_gradient returns the
same quantity by automatic differentiation of its own M (vectors normalised
first).  Both are compared element by element, |gpu - oracle| <= 1e-10 *
max|oracle| (FP64 sums of the same products in different orders; the
gradient has up to four factors of L, so its rounding spread is a few 1e-15
relative).

At the full size the oracle cannot differentiate the whole matrix, so the
test uses a property that holds at any size: with X fixed, f(L + t Delta) is
a polynomial of degree four in real t (M is at most quartic in L), so the
five-point central difference of f is exact up to rounding, and must equal
Re sum conj(G) Delta.  f itself comes from the library's sigma.

At converged eigenvectors the gradient is d omega; it is checked against
central finite differences of the eigenvalues (h = 1e-5).
"""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import make_system, config_system, random_vectors

pytestmark = pytest.mark.gpu

GTOL = 1e-10


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(1e-300, np.abs(b).max()))


def system(name):
    if name == "tiny":
        return make_system(2, 3, 7, 16, seed=101)
    if name == "edge":
        return make_system(1, 1, 2, 3, seed=7)
    if name == "ragged":
        return make_system(3, 2, 65, 70, seed=8)
    return config_system(name)


def oracle_grad(s, X, g):
    sp = O.Spaces(s.nc, s.no, s.nv)
    Xn = X / np.linalg.norm(X, axis=1, keepdims=True)
    G, de = O.omega_gradient(torch.from_numpy(s.L), torch.from_numpy(s.eps), sp, torch.from_numpy(Xn), g)
    return G.numpy(), de.numpy()


@pytest.mark.parametrize("name,m", [("edge", 1), ("tiny", 3), ("ragged", 2), ("tiles", 3), ("c1", 4),
                                    ("mid", 3)])
def test_backward_matches_oracle(name, m):
    s = system(name)
    print(f"[case] backward {name} nc={s.nc} no={s.no} nv={s.nv} naux={s.naux} m={m}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    X = random_vectors(31, m, h.dim)
    g = np.random.default_rng(5).normal(size=m).tolist()
    dL, de = A.adc2_omega_backward(h, dev(X), g)
    torch.cuda.synchronize()
    G, dref = oracle_grad(s, X, g)
    eL = rel(dL.cpu().numpy(), G)
    ee = rel(de.cpu().numpy(), dref)
    print(f"  dL rel err {eL:.2e}  deps rel err {ee:.2e}", flush=True)
    assert eL < GTOL
    assert ee < GTOL
    # the gradient is Hermitian per Cholesky vector and uniform shifts of eps leave M - shift invariant
    d = dL.cpu().numpy()
    assert np.abs(d - np.conj(d.transpose(0, 2, 1))).max() <= 1e-14 * np.abs(d).max()
    h.close()


def test_backward_repeatable_and_linear_in_weights():
    s = system("tiles")
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    X = dev(random_vectors(3, 2, h.dim))
    a1, e1 = A.adc2_omega_backward(h, X, [1.0, 0.0])
    a2, e2 = A.adc2_omega_backward(h, X, [0.0, 1.0])
    b, eb = A.adc2_omega_backward(h, X, [2.0, -3.0])
    c, ec = A.adc2_omega_backward(h, X, [2.0, -3.0])
    assert torch.equal(b, c) and torch.equal(eb, ec)
    assert float((b - (2 * a1 - 3 * a2)).abs().max()) <= 1e-12 * float(b.abs().max())
    assert float((eb - (2 * e1 - 3 * e2)).abs().max()) <= 1e-12 * float(eb.abs().max())
    h.close()


def test_backward_argument_errors():
    s = system("tiny")
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    X = torch.zeros((1, h.dim), dtype=torch.complex128, device="cuda")
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_omega_backward(h, X, [1.0])
    assert ei.value.status == A.ADC2_ERR_ARG and "norm" in str(ei.value)
    X[0, 0] = 1.0
    with pytest.raises(A.Adc2Error) as ei:
        A.adc2_omega_backward(h, X, [float("nan")])
    assert ei.value.status == A.ADC2_ERR_ARG
    h.close()


def _hermitian_direction(shape, seed, device="cuda"):
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    naux, n, _ = shape
    re = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    im = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    D = torch.complex(re, im)
    D = 0.5 * (D + D.conj().transpose(1, 2))
    return D.contiguous()


def _f(L, eps, s, X, g):
    h = A.adc2_setup(L, eps, s.nc, s.no, s.nv, s.naux)
    S = A.adc2_sigma(h, X)
    num = (X.conj() * S).sum(dim=1).real
    den = (X.conj() * X).sum(dim=1).real
    val = float((torch.tensor(g, dtype=torch.float64, device=X.device) * num / den).sum())
    h.close()
    return val


@pytest.mark.parametrize("name", ["mid", "c2"])
def test_backward_directional_identity(name):
    """Full size: five-point stencil of the quartic f(L + t Delta) and a
    fourth-order stencil in eps against the returned gradient."""
    s = system(name)
    print(f"[case] directional identity {name} nc={s.nc} no={s.no} nv={s.nv} naux={s.naux}", flush=True)
    L = dev(s.L)
    eps = dev(s.eps)
    m = 2
    dim = s.nc * s.nv + s.nc * s.no * s.nv * (s.nv - 1) // 2
    X = dev(random_vectors(41, m, dim))
    g = [0.8, -1.1]
    h = A.adc2_setup(L, eps, s.nc, s.no, s.nv, s.naux)
    dL, de = A.adc2_omega_backward(h, X, g)
    h.close()
    Dl = _hermitian_direction(tuple(L.shape), 1234) * 0.05
    lin = float((dL.conj() * Dl).sum().real)
    # f is exactly quartic in t, so a large step costs no truncation error and
    # keeps the rounding of f (relative 1e-14) far below the derivative
    t = 5e-2
    f = {k: _f((L + k * t * Dl).contiguous(), eps, s, X, g) for k in (-2, -1, 1, 2)}
    fd = (f[-2] - 8 * f[-1] + 8 * f[1] - f[2]) / (12 * t)
    print(f"  L: stencil {fd:.12e} gradient {lin:.12e}", flush=True)
    assert abs(fd - lin) <= 1e-8 * abs(lin)
    del Dl
    de_dir = torch.from_numpy(np.random.default_rng(9).normal(size=s.eps.shape[0])).cuda()
    lin_e = float((de * de_dir).sum())
    te = 1e-4
    fe = {k: _f(L, (eps + k * te * de_dir).contiguous(), s, X, g) for k in (-2, -1, 1, 2)}
    fde = (fe[-2] - 8 * fe[-1] + 8 * fe[1] - fe[2]) / (12 * te)
    print(f"  eps: stencil {fde:.12e} gradient {lin_e:.12e}", flush=True)
    assert abs(fde - lin_e) <= 1e-7 * max(1.0, abs(lin_e))


def test_gradient_at_eigenvectors_vs_finite_differences():
    """d omega_k along random Hermitian directions: central differences of
    the GPU eigenvalues (h = 1e-5) against the adjoint."""
    s = system("tiny")
    k = 3
    L = dev(s.L)
    eps = dev(s.eps)
    h = A.adc2_setup(L, eps, s.nc, s.no, s.nv, s.naux)
    w, X, info = A.adc2_davidson(h, k, tol=1e-11, max_iter=400)
    assert info["converged"]
    grads = [A.adc2_omega_backward(h, X, [1.0 if r == q else 0.0 for r in range(k)]) for q in range(k)]
    h.close()
    hstep = 1e-5
    for seed in (1, 2, 3):
        Dl = _hermitian_direction(tuple(L.shape), seed)
        Dl = Dl / float(torch.linalg.vector_norm(Dl))
        ws = []
        for sgn in (1, -1):
            hh = A.adc2_setup((L + sgn * hstep * Dl).contiguous(), eps, s.nc, s.no, s.nv, s.naux)
            wk, _, inf = A.adc2_davidson(hh, k, tol=1e-11, max_iter=400, want_vectors=False)
            assert inf["converged"]
            ws.append(np.array(wk))
            hh.close()
        fd = (ws[0] - ws[1]) / (2 * hstep)
        lin = np.array([float((gq[0].conj() * Dl).sum().real) for gq in grads])
        print(f"  direction {seed}: fd {fd} adjoint {lin}", flush=True)
        assert np.abs(fd - lin).max() <= 1e-6 * max(1.0, np.abs(lin).max())
    # energies: shifting every eps together changes nothing, so the gradient sums to zero
    for gq in grads:
        assert abs(float(gq[1].sum())) <= 1e-9 * float(gq[1].abs().max())


def test_gradient_from_complex64_eigenvectors():
    """The differentiation form with complex64 contractions: eigenvectors from
    a complex64 solve (the adjoint itself is FP64 arithmetic) give gradients
    within 1e-4 of the FP64-eigenvector gradient, itself checked against the
    oracle to 1e-10."""
    s = system("c1")
    k = 3
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    w, X, info = A.adc2_davidson(h, k, tol=1e-10, max_iter=400)
    g64 = [A.adc2_omega_backward(h, X, [1.0 if r == q else 0.0 for r in range(k)]) for q in range(k)]
    Go, deo = oracle_grad(s, X.cpu().numpy(), [1.0, 0.0, 0.0])
    assert rel(g64[0][0].cpu().numpy(), Go) < GTOL
    A.adc2_set_precision(h, A.ADC2_C64)
    wc, Xc, infc = A.adc2_davidson(h, k, tol=1e-6, max_iter=400)
    assert infc["converged"]
    A.adc2_set_precision(h, A.ADC2_FP64)
    for q in range(k):
        gc = A.adc2_omega_backward(h, Xc, [1.0 if r == q else 0.0 for r in range(k)])
        dl = float(torch.linalg.vector_norm(gc[0] - g64[q][0]) / torch.linalg.vector_norm(g64[q][0]))
        de = float(torch.linalg.vector_norm(gc[1] - g64[q][1]) / torch.linalg.vector_norm(g64[q][1]))
        print(f"  root {q}: complex64-eigenvector gradient rel. dev. L {dl:.2e} eps {de:.2e}", flush=True)
        assert dl < 1e-4 and de < 1e-4
    h.close()


def test_autograd_function_matches_oracle():
    s = system("tiny")
    k = 3
    L = dev(s.L).requires_grad_(True)
    eps = dev(s.eps).requires_grad_(True)
    w = A.adc2_omega(L, eps, s.nc, s.no, s.nv, k, tol=1e-11, solver=A.ADC2_SOLVER_FULL)
    coef = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    (w * coef).sum().backward()
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    w_ex, V = o.roots_exact(k)
    assert np.abs(w.detach().cpu().numpy() - w_ex.numpy()).max() < 1e-9
    G, de = O.omega_gradient(torch.from_numpy(s.L), torch.from_numpy(s.eps), O.Spaces(s.nc, s.no, s.nv),
                             V.T.contiguous(), coef.cpu().tolist())
    assert rel(L.grad.cpu().numpy(), G.numpy()) < 1e-8
    assert rel(eps.grad.cpu().numpy(), de.numpy()) < 1e-8


def test_autograd_function_folded_c1():
    """adc2_omega with its default solver (the folded one) at c1: roots
    against the oracle Davidson, gradients against the oracle's autograd
    gradient at the oracle's own eigenvectors, and a second backward through
    the same graph (retain_graph) giving the same gradient."""
    s = system("c1")
    k = 4
    print(f"[case] autograd folded c1 nc={s.nc} no={s.no} nv={s.nv} naux={s.naux} k={k}", flush=True)
    L = dev(s.L).requires_grad_(True)
    eps = dev(s.eps).requires_grad_(True)
    w = A.adc2_omega(L, eps, s.nc, s.no, s.nv, k, tol=1e-10)
    coef = torch.tensor([1.0, -0.5, 0.25, 2.0], dtype=torch.float64, device="cuda")
    (w * coef).sum().backward(retain_graph=True)
    gL1, ge1 = L.grad.clone(), eps.grad.clone()
    L.grad = None
    eps.grad = None
    (w * coef).sum().backward()
    assert torch.equal(L.grad, gL1) and torch.equal(eps.grad, ge1)
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    w_or, X_or, inf = o.roots(k, tol=1e-9, max_iter=400)   # the oracle's Davidson stalls near 3e-10 here
    assert inf["converged"]
    assert np.abs(w.detach().cpu().numpy() - w_or.numpy()).max() < 1e-9
    G, de = O.omega_gradient(torch.from_numpy(s.L), torch.from_numpy(s.eps), O.Spaces(s.nc, s.no, s.nv),
                             X_or / torch.linalg.vector_norm(X_or, dim=1, keepdim=True), coef.cpu().tolist())
    # the two solvers' eigenvectors differ by about residual / gap = 1e-9 / 0.03, and so do the gradients
    assert rel(gL1.cpu().numpy(), G.numpy()) < 1e-6
    assert rel(ge1.cpu().numpy(), de.numpy()) < 1e-6
