"""Host algebra of the folded eigensolver (paper_2604_27451_amd/csrc/hostla.h),
compiled on the CPU with g++ and checked against numpy.

herm_eig (Householder tridiagonalisation + implicit QL) must return the
eigenvalues of numpy.linalg.eigvalsh and orthonormal eigenvectors with
A Z = Z diag(w), for random, diagonal, degenerate and zero Hermitian
matrices of orders 1..64 (the projected problems are at most 64 x 64).
cheb_resolvent must reproduce 1/(x - t) and 1/(x - t)^2 from its Chebyshev
coefficients on [-1, 1].
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
