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
extern "C" int heig_it(int n, const double* A, double* w, double* Z, int max_iter) {
  return adc2::hostla::herm_eig(n, (const adc2::hostla::cplx*)A, w, (adc2::hostla::cplx*)Z, max_iter);
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


def test_herm_eig_reports_unconverged_eigenvalues(lib):
    """herm_eig returns the number of eigenvalues whose QL iteration did not
    finish within max_iter sweeps: 0 with the default limit, nonzero when the
    limit is forced to zero sweeps on a matrix that needs them (the callers
    turn a nonzero count into ADC2_ERR_NOCONV)."""
    lib.heig_it.restype = ctypes.c_int
    n = 12
    rng = np.random.default_rng(3)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = np.ascontiguousarray(A + A.conj().T)
    w = np.zeros(n)
    Z = np.zeros((n, n), dtype=np.complex128)
    args = (A.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p), Z.ctypes.data_as(ctypes.c_void_p))
    assert lib.heig_it(n, *args, 60) == 0
    assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12 * np.abs(w).max()
    bad = lib.heig_it(n, *args, 0)
    assert 1 <= bad <= n
    # a diagonal matrix needs no sweep at all
    D = np.ascontiguousarray(np.diag(np.arange(n, dtype=float)).astype(complex))
    assert lib.heig_it(n, D.ctypes.data_as(ctypes.c_void_p), args[1], args[2], 0) == 0


SAN_MAIN = r'''
#include "hostla.h"
#include <cstdio>
#include <random>
using adc2::hostla::cplx;
int main() {
  std::mt19937_64 g(11);
  std::normal_distribution<double> nd;
  int fails = 0;
  for (int n : {1, 2, 5, 17, 64}) {
    std::vector<cplx> A((size_t)n * n), Z((size_t)n * n);
    std::vector<double> w(n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) {
        const cplx v(nd(g), i == j ? 0.0 : nd(g));
        A[(size_t)i * n + j] = v;
        A[(size_t)j * n + i] = std::conj(v);
      }
    if (adc2::hostla::herm_eig(n, A.data(), w.data(), Z.data()) != 0) ++fails;
    double r = 0.0;
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < n; ++c) {
        cplx acc = 0.0;
        for (int k = 0; k < n; ++k) acc += A[(size_t)i * n + k] * Z[(size_t)k * n + c];
        r = std::max(r, std::abs(acc - w[c] * Z[(size_t)i * n + c]));
      }
    if (r > 1e-10 * (1.0 + std::fabs(w[0]) + std::fabs(w[n - 1]))) ++fails;
    double b[256], e[256], gg[256], hh[256];
    if (adc2::hostla::cheb_resolvent(1.5 + n, 256, b, e) < 1) ++fails;
    auto rm = adc2::hostla::ResolventMap::shifted_inverse(2.0, 9.0, -1.0);
    if (rm.coeffs(0.5, 256, b, e, gg, hh) < 1) ++fails;
  }
  std::printf("fails=%d\n", fails);
  return fails;
}
'''


def test_host_algebra_under_address_and_undefined_sanitizers(tmp_path):
    """The host algebra of the folded solver, built as a host program with
    AddressSanitizer and UndefinedBehaviorSanitizer (g++, no GPU code), runs
    its eigensolver and resolvent coefficients without a report."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.fail("g++ not found")
    src = tmp_path / "san.cpp"
    src.write_text(SAN_MAIN)
    exe = tmp_path / "san"
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:verify_asan_link_order=0"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "fails=0" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
