"""The C-ABI library loads and exports every symbol include/adc2.h declares.

Runs without a GPU: only argument-validation paths that return before any
HIP call are exercised here.
"""
import ctypes
import os

import pytest

import paper_2604_27451_amd as A

LIB = A.LIB_PATH


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (run __graft_entry__.build())")
    return A.load()


def test_header_declares_expected_entry_points():
    names = A.header_exports()
    assert names == sorted(A.EXPORTS), names


def test_library_exports_every_declared_symbol(lib):
    for name in A.header_exports():
        assert hasattr(lib, name), name
        assert getattr(lib, name) is not None


def test_exports_visible_in_dynamic_table():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for name in A.header_exports():
        assert f" T {name}\n" in out or out.endswith(f" T {name}"), name


def test_argument_errors_without_gpu(lib):
    out = ctypes.c_void_p(123)
    st = lib.adc2_setup(None, None, 1, 1, 2, 1, 0, None, ctypes.byref(out))
    assert st == A.ADC2_ERR_ARG
    assert out.value is None
    assert "NULL" in A.adc2_last_error()
    st = lib.adc2_setup(ctypes.c_void_p(8), ctypes.c_void_p(8), 0, 1, 2, 1, 0, None, ctypes.byref(out))
    assert st == A.ADC2_ERR_ARG
    st = lib.adc2_setup(ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 1, 2, 1, 7, None, ctypes.byref(out))
    assert st == A.ADC2_ERR_ARG and "precision" in A.adc2_last_error()
    assert lib.adc2_setup(ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 1, 2, 1, 0, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_dim(None) == 0
    assert lib.adc2_destroy(None) == A.ADC2_OK
    assert lib.adc2_sigma(None, 1, None, None, None) == A.ADC2_ERR_ARG
    om = (ctypes.c_double * 1)()
    assert lib.adc2_davidson(None, 1, None, None, om, None, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_get_m11(None, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_get_diag(None, None, None) == A.ADC2_ERR_ARG
    e = ctypes.c_double()
    assert lib.adc2_mp2_energy(None, ctypes.byref(e)) == A.ADC2_ERR_ARG
    assert lib.adc2_set_precision(None, 0) == A.ADC2_ERR_ARG
    assert lib.adc2_rayleigh(None, 1, None, om, None, None) == A.ADC2_ERR_ARG
    g = (ctypes.c_double * 1)(1.0)
    assert lib.adc2_omega_backward(None, 1, None, g, None, None, None) == A.ADC2_ERR_ARG
    assert "NULL" in A.adc2_last_error()


def test_binding_has_no_cpu_fallback(tmp_path):
    with pytest.raises(ImportError):
        A._lib_backup = A._lib
        try:
            A._lib = None
            A.load(str(tmp_path / "missing.so"))
        finally:
            A._lib = A._lib_backup
