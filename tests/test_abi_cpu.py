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
    st = lib.adc2_setup(None, None, 1, 1, 2, 1, 0, None, None, ctypes.byref(out))
    assert st == A.ADC2_ERR_ARG
    assert out.value is None
    assert "NULL" in A.adc2_last_error()
    st = lib.adc2_setup(ctypes.c_void_p(8), ctypes.c_void_p(8), 0, 1, 2, 1, 0, None, None, ctypes.byref(out))
    assert st == A.ADC2_ERR_ARG
    st = lib.adc2_setup(ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 1, 2, 1, 7, None, None, ctypes.byref(out))
    assert st == A.ADC2_ERR_ARG and "precision" in A.adc2_last_error()
    assert lib.adc2_setup(ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 1, 2, 1, 0, None, None, None) == A.ADC2_ERR_ARG
    # allocator callbacks need both functions (checked before any HIP call)
    half = A.Alloc(A._ALLOC_FN(lambda n, c: None), A._RELEASE_FN(), None)
    assert lib.adc2_setup(ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 1, 2, 1, 0, ctypes.byref(half), None,
                          ctypes.byref(out)) == A.ADC2_ERR_ARG
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
    assert lib.adc2_autotune(None, 1, None, None) == A.ADC2_ERR_ARG and "NULL" in A.adc2_last_error()
    assert lib.adc2_transition(None, None, 1, None, None, 2, None, None, None) == A.ADC2_ERR_ARG
    nvo = ctypes.c_int(5)
    assert lib.adc2_fns(None, None, 1e-4, ctypes.byref(nvo), None, None, None, None) == A.ADC2_ERR_ARG
    assert "NULL" in A.adc2_last_error()
    # peak probes: argument checks come before any device call
    r = ctypes.c_double(7.0)
    assert lib.adc2_peak_probe(0, 0, 1, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_peak_probe(9, 0, 1, ctypes.byref(r), None) == A.ADC2_ERR_ARG and r.value == 0.0
    assert "unknown kind" in A.adc2_last_error()
    assert lib.adc2_peak_probe(A.ADC2_PEAK_MFMA_F64, 0, 0, ctypes.byref(r), None) == A.ADC2_ERR_ARG
    assert lib.adc2_peak_probe(A.ADC2_PEAK_HBM_READ, 1 << 20, 1, ctypes.byref(r), None) == A.ADC2_ERR_ARG
    assert "64 MiB" in A.adc2_last_error()


def test_binding_has_no_cpu_fallback(tmp_path):
    with pytest.raises(ImportError):
        A._lib_backup = A._lib
        try:
            A._lib = None
            A.load(str(tmp_path / "missing.so"))
        finally:
            A._lib = A._lib_backup


def test_batch_argument_errors_without_gpu(lib):
    vp = ctypes.c_void_p
    out = (vp * 2)(vp(5).value, vp(6).value)
    mols = (A.Mol * 2)()
    # sizes and NULLs are refused before any HIP call; out[] is cleared
    assert lib.adc2_setup_batch(0, mols, 0, None, None, out) == A.ADC2_ERR_ARG
    assert lib.adc2_setup_batch(65, mols, 0, None, None, out) == A.ADC2_ERR_ARG
    assert lib.adc2_setup_batch(2, None, 0, None, None, out) == A.ADC2_ERR_ARG
    assert out[0] is None and out[1] is None
    assert lib.adc2_setup_batch(2, mols, 0, None, None, None) == A.ADC2_ERR_ARG
    # a NULL system (L = eps = NULL) fails in adc2_setup and is named
    assert lib.adc2_setup_batch(2, mols, 0, None, None, out) == A.ADC2_ERR_ARG
    assert "system 0" in A.adc2_last_error()
    hs = (vp * 2)(None, None)
    ms = (ctypes.c_int * 2)(1, 1)
    xs = (vp * 2)(vp(8).value, vp(16).value)
    ss = (vp * 2)(vp(24).value, vp(32).value)
    assert lib.adc2_sigma_batch(0, hs, ms, xs, ss, None) == A.ADC2_ERR_ARG
    assert lib.adc2_sigma_batch(2, hs, ms, xs, ss, None) == A.ADC2_ERR_ARG
    assert "system 0" in A.adc2_last_error()
    hs2 = (vp * 2)(vp(64).value, vp(64).value)   # never dereferenced: the repeat is refused first
    assert lib.adc2_sigma_batch(2, hs2, ms, xs, ss, None) == A.ADC2_ERR_ARG
    assert "twice" in A.adc2_last_error()
    ms0 = (ctypes.c_int * 2)(1, 0)
    hs3 = (vp * 2)(vp(64).value, vp(128).value)
    assert lib.adc2_sigma_batch(2, hs3, ms0, xs, ss, None) == A.ADC2_ERR_ARG
    om = (ctypes.c_double * 4)()
    assert lib.adc2_davidson_batch(0, hs3, 2, None, 0, om, None, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_davidson_batch(2, hs, 2, None, 0, om, None, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_davidson_batch(2, hs2, 2, None, 0, om, None, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_davidson_batch(2, hs3, 2, None, 0, None, None, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_davidson_batch(2, hs3, 2, None, 7, om, None, None, None) == A.ADC2_ERR_ARG
    assert "mode" in A.adc2_last_error()
    # graph capture of a batched sigma: the same checks, out[] cleared; NULL graphs
    g = vp(72)
    assert lib.adc2_graph_sigma_batch(2, hs3, ms, xs, ss, None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_graph_sigma_batch(2, hs, ms, xs, ss, None, ctypes.byref(g)) == A.ADC2_ERR_ARG
    assert g.value is None
    assert lib.adc2_graph_sigma_batch(2, hs2, ms, xs, ss, None, ctypes.byref(g)) == A.ADC2_ERR_ARG
    assert "twice" in A.adc2_last_error()
    assert lib.adc2_graph_sigma_batch(2, hs3, ms0, xs, ss, None, ctypes.byref(g)) == A.ADC2_ERR_ARG
    assert lib.adc2_graph_launch(None, None) == A.ADC2_ERR_ARG
    assert lib.adc2_graph_destroy(None) == A.ADC2_OK


def test_one_hip_runtime_in_the_process():
    """load() binds the library to torch's HIP runtime even when nothing else
    imported torch first: a second runtime in the process (the library's
    dependency resolved to another copy) sees no device."""
    import subprocess
    import sys
    code = ("import paper_2604_27451_amd as A; A.load(); "
            "m = open('/proc/self/maps').read().splitlines(); "
            "print(len({l.split()[-1] for l in m if 'libamdhip64' in l}))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"


def test_binding_rejects_wrong_shapes_before_any_call(monkeypatch):
    """The library sees only pointers, so the binding checks every tensor
    shape first: a wrong shape raises ValueError before any library call (the
    library is replaced by an object that fails on any attribute access)."""
    import torch

    class NoCalls:
        def __getattr__(self, name):
            raise AssertionError(f"library call {name} reached with a wrong shape")

    monkeypatch.setattr(A, "_lib", NoCalls())
    h = A.Handle.__new__(A.Handle)
    h.ptr, h.alloc = None, None
    h.nc, h.no, h.nv, h.naux = 2, 3, 4, 5
    h.ns = 8
    h.dim = 8 + 2 * 3 * 6
    n = 9
    c = torch.complex128
    good = torch.zeros((2, h.dim), dtype=c)
    with pytest.raises(ValueError):                      # X too short
        A.adc2_sigma(h, torch.zeros((2, h.dim - 1), dtype=c))
    with pytest.raises(ValueError):                      # S with fewer rows than X
        A.adc2_sigma(h, good, torch.zeros((1, h.dim), dtype=c))
    with pytest.raises(ValueError):                      # S too short
        A.adc2_sigma(h, good, torch.zeros((2, h.dim - 3), dtype=c))
    with pytest.raises(ValueError):                      # guess too short
        A.adc2_davidson(h, 2, guess=torch.zeros((2, h.dim - 1), dtype=c))
    with pytest.raises(ValueError):                      # nguess beyond the guess rows
        A.adc2_davidson(h, 2, nguess=3, guess=good)
    with pytest.raises(ValueError):
        A.adc2_rayleigh(h, torch.zeros((2, h.dim + 1), dtype=c))
    with pytest.raises(ValueError):
        A.adc2_omega_backward(h, torch.zeros((2, 7), dtype=c), [1.0, 1.0])
    dip = torch.zeros((3, n, n), dtype=c)
    with pytest.raises(ValueError):                      # dip of the wrong size
        A.adc2_transition(h, torch.zeros((3, n - 1, n - 1), dtype=c), good, [0.1, 0.2])
    with pytest.raises(ValueError):                      # X of the wrong length
        A.adc2_transition(h, dip, torch.zeros((2, h.dim - 1), dtype=c), [0.1, 0.2])
    with pytest.raises(ValueError):                      # omega shorter than X
        A.adc2_transition(h, dip, good, [0.1])
    with pytest.raises(ValueError):
        A.adc2_fns(h, torch.zeros((h.naux, n, n - 1), dtype=c), 1e-4)
    with pytest.raises(ValueError):
        A.adc2_setup(torch.zeros((5, n, n), dtype=c), torch.zeros(n - 1, dtype=torch.float64), 2, 3, 4, 5)
    # right shapes on host memory get past the shape checks and stop at the device check
    with pytest.raises(TypeError):
        A.adc2_sigma(h, good)
    with pytest.raises(TypeError):
        A.adc2_transition(h, dip, good, [0.1, 0.2])


def test_graph_wrapper_refuses_closed_handles_and_graphs():
    """SigmaGraph.launch refuses, before any library call, a graph whose
    handle was closed or that was itself closed."""
    class Closed:
        ptr = None
    g = A.SigmaGraph(ctypes.c_void_p(4096), [Closed()], [], [])
    with pytest.raises(A.Adc2Error, match="handle of the graph was closed"):
        g.launch()
    g.ptr = None   # never handed to the library: nothing to destroy
    with pytest.raises(A.Adc2Error, match="graph is closed"):
        g.launch()
