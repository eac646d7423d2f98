"""Host algebra of the folded eigensolver (paper_2604_27451_amd/csrc/hostla.h),
compiled on the CPU with g++ and checked against numpy.

herm_eig (Householder tridiagonalisation + implicit QL) must return the
eigenvalues of numpy.linalg.eigvalsh and orthonormal eigenvectors with
A Z = Z diag(w), for random, diagonal, degenerate and zero Hermitian
matrices of orders 1..64 (the projected problems are at most 64 x 64).
cheb_resolvent must reproduce 1/(x - t) and 1/(x - t)^2 from its Chebyshev
coefficients on [-1, 1].  ResolventMap's coefficients, summed against
T_m(tau(D)), must give (omega - D)^-1 and (omega - D)^-2 evaluated directly
(the definition of the folded resolvent and of the Newton slope) for both
the linear and the shifted-inverse variable, and its reach must be the
omega whose pole sits at |x| = 1.05.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2604_27451_amd", "csrc")

SHIM = r'''
#include "hostla.h"
extern "C" void heig(int n, const double* A, double* w, double* Z) {
  adc2::hostla::herm_eig(n, (const adc2::hostla::cplx*)A, w, (adc2::hostla::cplx*)Z);
}
extern "C" int cheb(double x, int mmax, double* b, double* e) {
  return adc2::hostla::cheb_resolvent(x, mmax, b, e);
}
static adc2::hostla::ResolventMap mk(int inv, double Dmin, double Dmax, double w0) {
  return inv ? adc2::hostla::ResolventMap::shifted_inverse(Dmin, Dmax, w0)
             : adc2::hostla::ResolventMap::linear(Dmin, Dmax);
}
extern "C" int rmap_coeffs(int inv, double Dmin, double Dmax, double w0, double omega, int mmax, double* g,
                           double* h) {
  double b[512], e[512];
  return mk(inv, Dmin, Dmax, w0).coeffs(omega, mmax, b, e, g, h);
}
extern "C" double rmap_tau(int inv, double Dmin, double Dmax, double w0, double D) {
  return mk(inv, Dmin, Dmax, w0).tau(D);
}
extern "C" double rmap_reach(int inv, double Dmin, double Dmax, double w0, double xmin) {
  return mk(inv, Dmin, Dmax, w0).reach(xmin);
}
'''


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.fail("g++ not found")
    d = tmp_path_factory.mktemp("hostla")
    src = d / "shim.cpp"
    src.write_text(SHIM)
    so = d / "libhostla.so"
    subprocess.run([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, str(src), "-o", str(so)], check=True)
    return ctypes.CDLL(str(so))


def eig(lib, A):
    n = A.shape[0]
    A = np.ascontiguousarray(A, dtype=np.complex128)
    w = np.zeros(n)
    Z = np.zeros((n, n), dtype=np.complex128)
    lib.heig(n, A.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
             Z.ctypes.data_as(ctypes.c_void_p))
    return w, Z


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 33, 64])
def test_herm_eig_matches_numpy(lib, n):
    rng = np.random.default_rng(100 + n)
    cases = []
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    cases.append(A + A.conj().T)
    cases.append(np.diag(rng.standard_normal(n)).astype(complex))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    cases.append(Q @ np.diag(np.round(rng.standard_normal(n))) @ Q.conj().T)   # repeated eigenvalues
    cases.append(np.zeros((n, n), dtype=complex))
    cases.append(1e6 * np.eye(n) + (cases[0] * 1e-3))                             # clustered, large shift
    for A in cases:
        w, Z = eig(lib, A)
        ref = np.linalg.eigvalsh(A)
        scale = max(1.0, np.abs(ref).max())
        assert np.all(np.diff(w) >= -1e-12 * scale)
        assert np.abs(w - ref).max() <= 1e-13 * scale
        assert np.abs(A @ Z - Z * w).max() <= 1e-12 * scale
        assert np.abs(Z.conj().T @ Z - np.eye(n)).max() <= 1e-12


def test_cheb_resolvent(lib):
    t = np.cos(np.linspace(0, np.pi, 257))
    for x in (1.3, -1.7, 4.0, -12.5):
        b = np.zeros(128)
        e = np.zeros(128)
        m = lib.cheb(ctypes.c_double(x), 128, b.ctypes.data_as(ctypes.c_void_p), e.ctypes.data_as(ctypes.c_void_p))
        assert 2 <= m <= 128
        T = np.cos(np.outer(np.arange(m), np.arccos(t)))
        assert np.abs(b[:m] @ T - 1.0 / (x - t)).max() < 1e-13 * np.abs(1.0 / (x - t)).max()
        assert np.abs(e[:m] @ T - 1.0 / (x - t) ** 2).max() < 1e-12 * np.abs(1.0 / (x - t) ** 2).max()
    assert lib.cheb(ctypes.c_double(1.0), 128, np.zeros(128).ctypes.data_as(ctypes.c_void_p),
                    np.zeros(128).ctypes.data_as(ctypes.c_void_p)) == -1


def _rmap(lib):
    lib.rmap_coeffs.restype = ctypes.c_int
    lib.rmap_coeffs.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.rmap_tau.restype = ctypes.c_double
    lib.rmap_tau.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4
    lib.rmap_reach.restype = ctypes.c_double
    lib.rmap_reach.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4
    return lib


@pytest.mark.parametrize("inv,w0,omega", [(0, 0.0, 14.9), (0, 0.0, 28.0), (1, 8.78, 14.9), (1, 8.78, 28.5),
                                          (1, 27.47, 28.44), (1, 27.47, 29.2)])
def test_resolvent_map_reproduces_resolvent(lib, inv, w0, omega):
    lib = _rmap(lib)
    Dmin, Dmax = 29.255, 40.87
    g = np.zeros(128)
    h = np.zeros(128)
    M = lib.rmap_coeffs(inv, Dmin, Dmax, w0, omega, 128, g.ctypes.data_as(ctypes.c_void_p),
                        h.ctypes.data_as(ctypes.c_void_p))
    assert 0 < M <= 128
    D = np.concatenate([[Dmin, Dmax], np.random.default_rng(5).uniform(Dmin, Dmax, 200)])
    tau = np.array([lib.rmap_tau(inv, Dmin, Dmax, w0, d) for d in D])
    assert np.all(np.abs(tau) <= 1.0 + 1e-12)
    T = np.polynomial.chebyshev.chebvander(np.clip(tau, -1.0, 1.0), M - 1)
    r1 = T @ g[:M]
    r2 = T @ h[:M]
    ex1 = 1.0 / (omega - D)
    ex2 = ex1 ** 2
    assert np.abs(r1 - ex1).max() <= 1e-13 * np.abs(ex1).max()
    assert np.abs(r2 - ex2).max() <= 1e-12 * np.abs(ex2).max()


def test_resolvent_map_term_counts_and_reach(lib):
    """The shifted inverse needs far fewer terms for a root well below min D,
    and its reach is the omega with pole at x = -1.05 (linear) or +1.05 in the
    inverse variable."""
    lib = _rmap(lib)
    Dmin, Dmax = 29.255, 40.87
    g = np.zeros(128)
    h = np.zeros(128)
    args = (g.ctypes.data_as(ctypes.c_void_p), h.ctypes.data_as(ctypes.c_void_p))
    m_lin = lib.rmap_coeffs(0, Dmin, Dmax, 0.0, 14.9, 128, *args)
    m_inv = lib.rmap_coeffs(1, Dmin, Dmax, 8.78, 14.9, 128, *args)
    assert m_inv < 0.7 * m_lin
    c, hw = 0.5 * (Dmin + Dmax), 0.5 * (Dmax - Dmin)
    assert abs(lib.rmap_reach(0, Dmin, Dmax, 0.0, 1.05) - (c - 1.05 * hw)) < 1e-12
    w0 = 27.47
    lo, hi = 1.0 / (Dmax - w0), 1.0 / (Dmin - w0)
    reach = lib.rmap_reach(1, Dmin, Dmax, w0, 1.05)
    x = (1.0 / (reach - w0) - 0.5 * (lo + hi)) / (0.5 * (hi - lo))
    assert abs(x - 1.05) < 1e-10
    assert Dmin - reach < 0.03 * (Dmin - w0)
    # omega at or above min D, or at or below w0, has no expansion
    assert lib.rmap_coeffs(1, Dmin, Dmax, w0, Dmin, 128, *args) < 0
    assert lib.rmap_coeffs(1, Dmin, Dmax, w0, w0, 128, *args) < 0
