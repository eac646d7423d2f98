"""Python binding of the gfx950 CVS-ADC(2) library (libadc2.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/adc2.h.  Torch tensors provide
device memory and streams.  There is no CPU fallback: if the shared library
is missing the import of the binding functions fails loudly.

Functions mirror the C ABI names:
    adc2_setup(L, eps, nc, no, nv, naux, prec=0) -> Handle
    adc2_dim(h)
    adc2_sigma(h, X, S=None) -> S
    adc2_sigma_noalloc(h, X, S) -> S
    adc2_davidson(h, nroots, tol=1e-8, max_iter=0, max_subspace=0, nguess=0,
                  guess=None, want_vectors=True, verbose=0) -> (omega, X, info)
    adc2_set_precision(h, prec)
    adc2_set_method(h, method)
    adc2_rayleigh(h, X) -> (omega, resnorm)
    adc2_omega_backward(h, X, g_omega, dL=None, deps=None) -> (dL, deps)
    adc2_get_m11(h) -> complex128 tensor
    adc2_get_diag(h) -> float64 tensor
    adc2_mp2_energy(h) -> float
    adc2_destroy(h)
    adc2_last_error() -> str
and the autograd wrapper
    adc2_omega(L, eps, nc, no, nv, nroots, tol=1e-10, max_iter=0, solver=FOLDED) -> omega (float64 tensor)
whose backward is adc2_omega_backward.
"""
from __future__ import annotations

import ctypes
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadc2.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "adc2.h")

ADC2_OK = 0
ADC2_ERR_ARG = 1
ADC2_ERR_NOT_HERMITIAN = 2
ADC2_ERR_OOM = 3
ADC2_ERR_HIP = 4
ADC2_ERR_NOCONV = 5
ADC2_ERR_NONFINITE = 6
ADC2_FP64 = 0
ADC2_C64 = 1
ADC2_BF16X3 = 2
ADC2_MAX_ROOTS = 32
ADC2_METHOD_ADC2 = 0
ADC2_METHOD_ADC2X = 1
ADC2_SOLVER_FULL = 0
ADC2_SOLVER_FOLDED = 1
ADC2_BATCH_ROUNDS = 0
ADC2_BATCH_STREAMS = 1
ADC2_PEAK_MFMA_F64 = 0
ADC2_PEAK_MFMA_F32 = 1
ADC2_PEAK_MFMA_BF16 = 2
ADC2_PEAK_VALU_F64 = 3
ADC2_PEAK_HBM_READ = 4
ADC2_PEAK_HBM_COPY = 5
ADC2_PEAK_MFMA_F64_RAND = 6
ADC2_PEAK_MFMA_BF16_RAND = 7

STATUS_NAMES = {0: "ADC2_OK", 1: "ADC2_ERR_ARG", 2: "ADC2_ERR_NOT_HERMITIAN", 3: "ADC2_ERR_OOM",
                4: "ADC2_ERR_HIP", 5: "ADC2_ERR_NOCONV", 6: "ADC2_ERR_NONFINITE"}

EXPORTS = ["adc2_setup", "adc2_dim", "adc2_sigma", "adc2_davidson", "adc2_set_precision",
           "adc2_rayleigh", "adc2_omega_backward", "adc2_get_m11", "adc2_get_diag", "adc2_mp2_energy", "adc2_profile",
           "adc2_kernel_stats", "adc2_destroy", "adc2_last_error", "adc2_setup_batch", "adc2_sigma_batch",
           "adc2_davidson_batch", "adc2_peak_probe", "adc2_autotune", "adc2_fns", "adc2_transition",
           "adc2_sigma_noalloc", "adc2_set_method", "adc2_graph_sigma_batch", "adc2_graph_launch",
           "adc2_graph_destroy"]


class DavOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("max_subspace", ctypes.c_int), ("nguess", ctypes.c_int),
                ("verbose", ctypes.c_int), ("solver", ctypes.c_int), ("follow", ctypes.c_int),
                ("mixed_tol", ctypes.c_double)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("ysplit", ctypes.c_int), ("ncand", ctypes.c_int), ("cand", ctypes.c_int * 8),
                ("ms", ctypes.c_double * 8), ("from_cache", ctypes.c_int), ("zgemm", ctypes.c_int),
                ("nengine", ctypes.c_int), ("engine", ctypes.c_int * 4), ("engine_ms", ctypes.c_double * 4)]


ZGEMM_NAMES = {0: "128x128 four waves", 1: "128x64 three-multiplication", 2: "128x64 two per CU",
               3: "128x128 eight waves"}


class Mol(ctypes.Structure):
    """adc2_mol: one system of a batch."""
    _fields_ = [("L", ctypes.c_void_p), ("eps", ctypes.c_void_p), ("nc", ctypes.c_int), ("no", ctypes.c_int),
                ("nv", ctypes.c_int), ("naux", ctypes.c_int)]


class DavInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("n_sigma", ctypes.c_int),
                ("converged", ctypes.c_int), ("subspace", ctypes.c_int),
                ("resnorm", ctypes.c_double * ADC2_MAX_ROOTS),
                ("ms_sigma", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("sigma_flops", ctypes.c_double)]

    def as_dict(self, nroots):
        return {"iters": self.iters, "n_sigma": self.n_sigma, "converged": bool(self.converged),
                "subspace": self.subspace, "resnorm": list(self.resnorm[:nroots]),
                "ms_sigma": self.ms_sigma, "ms_total": self.ms_total,
                "sigma_flops": self.sigma_flops}


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_long),
                ("ms", ctypes.c_double), ("flops", ctypes.c_double)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Alloc(ctypes.Structure):
    """adc2_alloc: device-memory callbacks of a handle."""
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("ctx", ctypes.c_void_p)]


def torch_allocator():
    """Device-memory callbacks backed by PyTorch's caching allocator (on the
    current device and stream): pass as alloc= to adc2_setup /
    adc2_setup_batch.  A request the allocator cannot serve returns NULL,
    which the library reports as ADC2_ERR_OOM."""
    import torch

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None

    def _release(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    return Alloc(_ALLOC_FN(_alloc), _RELEASE_FN(_release), None)


class Adc2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libadc2.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2604_27451_amd.build` "
                          "(there is no CPU fallback)")
    # torch first: its HIP runtime (libamdhip64.so.7) is then the one the
    # library's dependency of that name resolves to.  Loaded the other way
    # round, the process holds two HIP and HSA runtimes and the library's
    # own finds no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.adc2_setup.argtypes = [vp, vp, i, i, i, i, i, ctypes.POINTER(Alloc), vp, ctypes.POINTER(vp)]
    lib.adc2_setup.restype = i
    lib.adc2_dim.argtypes = [vp]
    lib.adc2_dim.restype = ctypes.c_size_t
    lib.adc2_sigma.argtypes = [vp, i, vp, vp, vp]
    lib.adc2_sigma.restype = i
    lib.adc2_sigma_noalloc.argtypes = [vp, i, vp, vp, vp]
    lib.adc2_sigma_noalloc.restype = i
    lib.adc2_davidson.argtypes = [vp, i, ctypes.POINTER(DavOpts), vp, ctypes.POINTER(d), vp,
                                  ctypes.POINTER(DavInfo), vp]
    lib.adc2_davidson.restype = i
    lib.adc2_set_method.argtypes = [vp, i, vp]
    lib.adc2_set_method.restype = i
    lib.adc2_set_precision.argtypes = [vp, i]
    lib.adc2_set_precision.restype = i
    lib.adc2_rayleigh.argtypes = [vp, i, vp, ctypes.POINTER(d), ctypes.POINTER(d), vp]
    lib.adc2_rayleigh.restype = i
    lib.adc2_omega_backward.argtypes = [vp, i, vp, ctypes.POINTER(d), vp, vp, vp]
    lib.adc2_omega_backward.restype = i
    lib.adc2_get_m11.argtypes = [vp, vp, vp]
    lib.adc2_get_m11.restype = i
    lib.adc2_get_diag.argtypes = [vp, vp, vp]
    lib.adc2_get_diag.restype = i
    lib.adc2_mp2_energy.argtypes = [vp, ctypes.POINTER(d)]
    lib.adc2_mp2_energy.restype = i
    lib.adc2_profile.argtypes = [vp, i]
    lib.adc2_profile.restype = i
    lib.adc2_kernel_stats.argtypes = [vp, ctypes.POINTER(KStat), i]
    lib.adc2_kernel_stats.restype = i
    lib.adc2_setup_batch.argtypes = [i, ctypes.POINTER(Mol), i, ctypes.POINTER(Alloc), vp, ctypes.POINTER(vp)]
    lib.adc2_setup_batch.restype = i
    lib.adc2_sigma_batch.argtypes = [i, ctypes.POINTER(vp), ctypes.POINTER(i), ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), vp]
    lib.adc2_sigma_batch.restype = i
    lib.adc2_graph_sigma_batch.argtypes = [i, ctypes.POINTER(vp), ctypes.POINTER(i), ctypes.POINTER(vp),
                                           ctypes.POINTER(vp), vp, ctypes.POINTER(vp)]
    lib.adc2_graph_sigma_batch.restype = i
    lib.adc2_graph_launch.argtypes = [vp, vp]
    lib.adc2_graph_launch.restype = i
    lib.adc2_graph_destroy.argtypes = [vp]
    lib.adc2_graph_destroy.restype = i
    lib.adc2_davidson_batch.argtypes = [i, ctypes.POINTER(vp), i, ctypes.POINTER(DavOpts), i, ctypes.POINTER(d),
                                        ctypes.POINTER(vp), ctypes.POINTER(DavInfo), vp]
    lib.adc2_davidson_batch.restype = i
    lib.adc2_transition.argtypes = [vp, vp, i, vp, ctypes.POINTER(d), i, vp, ctypes.POINTER(d), vp]
    lib.adc2_transition.restype = i
    lib.adc2_fns.argtypes = [vp, vp, d, ctypes.POINTER(i), ctypes.POINTER(d), vp, vp, vp]
    lib.adc2_fns.restype = i
    lib.adc2_autotune.argtypes = [vp, i, ctypes.POINTER(TuneInfo), vp]
    lib.adc2_autotune.restype = i
    lib.adc2_peak_probe.argtypes = [i, ctypes.c_size_t, i, ctypes.POINTER(d), vp]
    lib.adc2_peak_probe.restype = i
    lib.adc2_destroy.argtypes = [vp]
    lib.adc2_destroy.restype = i
    lib.adc2_last_error.argtypes = []
    lib.adc2_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def adc2_last_error() -> str:
    return load().adc2_last_error().decode()


def _check(status, what):
    if status != ADC2_OK:
        raise Adc2Error(status, f"{what}: {adc2_last_error()}")


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def _rows(t, dim, what, rows=None):
    """Shape check of a block of ADC vectors [k][dim] before any pointer is
    handed to the library (which cannot see tensor shapes): wrong shapes would
    otherwise mean reads or writes past the end of a device buffer."""
    if t.dim() != 2 or t.shape[1] != dim:
        raise ValueError(f"{what} must be [k][{dim}], got {list(t.shape)}")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{what} must have {rows} rows, got {t.shape[0]}")


class Handle:
    def __init__(self, ptr, nc, no, nv, naux, alloc=None):
        self.ptr = ptr
        self.alloc = alloc          # keeps the callbacks alive while the handle lives
        self.nc, self.no, self.nv, self.naux = nc, no, nv, naux
        self.dim = int(load().adc2_dim(ptr))
        self.ns = nc * nv

    def close(self):
        if self.ptr:
            load().adc2_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        # at interpreter shutdown a handle whose memory belongs to PyTorch's
        # allocator is left to the process exit: its release callbacks would
        # call into a torch that may already be torn down
        if self.alloc is not None and sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def adc2_setup(L, eps, nc, no, nv, naux, prec=ADC2_FP64, stream=None, alloc=None) -> Handle:
    """Handle of one system.  alloc: None (hipMalloc), "torch" (PyTorch's
    caching allocator) or an Alloc of one's own."""
    import torch
    n = nc + no + nv
    if tuple(L.shape) != (naux, n, n) or tuple(eps.shape) != (n,):
        raise ValueError("L must be [naux][n][n] and eps [n]")
    _need(L, torch.complex128, "L")
    _need(eps, torch.float64, "eps")
    out = ctypes.c_void_p()
    al = torch_allocator() if alloc == "torch" else alloc
    st = load().adc2_setup(ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(eps.data_ptr()),
                           nc, no, nv, naux, prec, ctypes.byref(al) if al is not None else None,
                           _stream_ptr(stream), ctypes.byref(out))
    _check(st, "adc2_setup")
    return Handle(out, nc, no, nv, naux, al)


def adc2_dim(h: Handle) -> int:
    return int(load().adc2_dim(h.ptr))


def adc2_sigma(h: Handle, X, S=None, stream=None):
    import torch
    if X.dim() == 1:
        X = X[None]
    _rows(X, h.dim, "X")
    m = X.shape[0]
    if S is not None:
        if S.dim() == 1:
            S = S[None]
        if tuple(S.shape) != tuple(X.shape):
            raise ValueError(f"S must have the shape of X {list(X.shape)}, got {list(S.shape)}")
    _need(X, torch.complex128, "X")
    if S is None:
        S = torch.empty_like(X)
    _need(S, torch.complex128, "S")
    st = load().adc2_sigma(h.ptr, m, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                           _stream_ptr(stream))
    _check(st, "adc2_sigma")
    return S


def adc2_sigma_noalloc(h: Handle, X, S, stream=None):
    """S = M X (FP64 form) with the library's static scratch array for the
    work spaces: no device allocation inside the call (S must be given)."""
    import torch
    if X.dim() == 1:
        X = X[None]
    if S.dim() == 1:
        S = S[None]
    _rows(X, h.dim, "X")
    if tuple(S.shape) != tuple(X.shape):
        raise ValueError(f"S must have the shape of X {list(X.shape)}, got {list(S.shape)}")
    _need(X, torch.complex128, "X")
    _need(S, torch.complex128, "S")
    st = load().adc2_sigma_noalloc(h.ptr, X.shape[0], ctypes.c_void_p(X.data_ptr()),
                                   ctypes.c_void_p(S.data_ptr()), _stream_ptr(stream))
    _check(st, "adc2_sigma_noalloc")
    return S


def adc2_davidson(h: Handle, nroots, tol=1e-8, max_iter=0, max_subspace=0, nguess=0, guess=None,
                  want_vectors=True, verbose=0, stream=None, raise_on_noconv=True, solver=ADC2_SOLVER_FULL,
                  follow=False, mixed_tol=0.0):
    """Eigenpairs of M.  follow=True: root j follows guess vector j (root-specific
    Davidson; either solver; results in guess order).  mixed_tol > 0: solve
    with split-BF16 sigma builds to mixed_tol first, then in FP64 to tol."""
    import torch
    opts = DavOpts(tol, max_iter, max_subspace, nguess, verbose, solver, 1 if follow else 0, float(mixed_tol))
    info = DavInfo()
    omega = (ctypes.c_double * nroots)()
    gp = ctypes.c_void_p(0)
    if guess is not None:
        _rows(guess, h.dim, "guess")
        if opts.nguess == 0:
            opts.nguess = guess.shape[0]
        if opts.nguess > guess.shape[0]:
            raise ValueError(f"nguess={opts.nguess} exceeds the {guess.shape[0]} rows of guess")
        _need(guess, torch.complex128, "guess")
        gp = ctypes.c_void_p(guess.data_ptr())
    X = torch.empty((nroots, h.dim), dtype=torch.complex128, device="cuda") if want_vectors else None
    st = load().adc2_davidson(h.ptr, nroots, ctypes.byref(opts), gp, omega,
                              ctypes.c_void_p(X.data_ptr()) if X is not None else ctypes.c_void_p(0),
                              ctypes.byref(info), _stream_ptr(stream))
    res = (list(omega), X, info.as_dict(nroots))
    if st == ADC2_ERR_NOCONV and not raise_on_noconv:
        return res
    _check(st, "adc2_davidson")
    return res


def adc2_setup_batch(systems, prec=ADC2_FP64, stream=None, alloc=None):
    """Handles for a batch of systems; systems is a list of (L, eps, nc, no, nv, naux);
    alloc as in adc2_setup."""
    import torch
    n = len(systems)
    mols = (Mol * n)()
    for q, (L, eps, nc, no, nv, naux) in enumerate(systems):
        _need(L, torch.complex128, f"L[{q}]")
        _need(eps, torch.float64, f"eps[{q}]")
        nn = nc + no + nv
        if tuple(L.shape) != (naux, nn, nn) or tuple(eps.shape) != (nn,):
            raise ValueError(f"system {q}: L must be [naux][n][n] and eps [n]")
        mols[q] = Mol(L.data_ptr(), eps.data_ptr(), nc, no, nv, naux)
    out = (ctypes.c_void_p * n)()
    al = torch_allocator() if alloc == "torch" else alloc
    _check(load().adc2_setup_batch(n, mols, prec, ctypes.byref(al) if al is not None else None,
                                   _stream_ptr(stream), out), "adc2_setup_batch")
    return [Handle(ctypes.c_void_p(out[q]), *systems[q][2:6], alloc=al) for q in range(n)]


def _batch_args(hs, Xs, Ss):
    import torch
    n = len(hs)
    Xs = [X[None] if X.dim() == 1 else X for X in Xs]
    if Ss is None:
        Ss = [torch.empty_like(X) for X in Xs]
    hp = (ctypes.c_void_p * n)(*[h.ptr.value if isinstance(h.ptr, ctypes.c_void_p) else h.ptr for h in hs])
    ms = (ctypes.c_int * n)()
    xp = (ctypes.c_void_p * n)()
    sp = (ctypes.c_void_p * n)()
    for q in range(n):
        _need(Xs[q], torch.complex128, f"X[{q}]")
        _need(Ss[q], torch.complex128, f"S[{q}]")
        if Xs[q].shape[1] != hs[q].dim or Ss[q].shape != Xs[q].shape:
            raise ValueError(f"system {q}: X and S must be [m][dim]")
        ms[q] = Xs[q].shape[0]
        xp[q] = Xs[q].data_ptr()
        sp[q] = Ss[q].data_ptr()
    return n, hp, ms, xp, sp, Xs, Ss


def adc2_sigma_batch(hs, Xs, Ss=None, stream=None):
    """S_i = M_i X_i for every system of a batch in one batched launch sequence."""
    n, hp, ms, xp, sp, Xs, Ss = _batch_args(hs, Xs, Ss)
    _check(load().adc2_sigma_batch(n, hp, ms, xp, sp, _stream_ptr(stream)), "adc2_sigma_batch")
    return Ss


class SigmaGraph:
    """A batched sigma captured as a HIP graph (adc2_graph_sigma_batch).
    launch() replays it: it reads the X tensors and writes the S tensors it
    was captured with (refill X in place between launches).  The tensors and
    handles are kept alive as long as the graph."""

    def __init__(self, ptr, hs, Xs, Ss):
        self.ptr, self.hs, self.X, self.S = ptr, list(hs), Xs, Ss

    def launch(self, stream=None):
        if self.ptr is None:
            raise Adc2Error(ADC2_ERR_ARG, "adc2_graph_launch: graph is closed")
        if not all(h.ptr for h in self.hs):
            raise Adc2Error(ADC2_ERR_ARG, "adc2_graph_launch: a handle of the graph was closed")
        _check(load().adc2_graph_launch(self.ptr, _stream_ptr(stream)), "adc2_graph_launch")
        return self.S

    def close(self):
        if self.ptr is not None:
            load().adc2_graph_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def adc2_graph_sigma_batch(hs, Xs, Ss=None, stream=None):
    """Capture the batched sigma S_i = M_i X_i as a HIP graph; S holds the
    eager result on return.  Returns a SigmaGraph."""
    n, hp, ms, xp, sp, Xs, Ss = _batch_args(hs, Xs, Ss)
    out = ctypes.c_void_p()
    _check(load().adc2_graph_sigma_batch(n, hp, ms, xp, sp, _stream_ptr(stream), ctypes.byref(out)),
           "adc2_graph_sigma_batch")
    return SigmaGraph(out, hs, Xs, Ss)


def adc2_davidson_batch(hs, nroots, tol=1e-8, max_iter=0, max_subspace=0, nguess=0, want_vectors=True,
                        verbose=0, stream=None, solver=ADC2_SOLVER_FOLDED, mode=None):
    """Lowest nroots eigenpairs of every system of a batch, solved concurrently.
    Returns (omega [nmol][nroots] as lists, list of X or None, list of info dicts)."""
    import torch
    n = len(hs)
    opts = DavOpts(tol, max_iter, max_subspace, nguess, verbose, solver)
    infos = (DavInfo * n)()
    omega = (ctypes.c_double * (n * nroots))()
    Xs = [torch.empty((nroots, h.dim), dtype=torch.complex128, device="cuda") for h in hs] if want_vectors else None
    hp = (ctypes.c_void_p * n)(*[h.ptr.value if isinstance(h.ptr, ctypes.c_void_p) else h.ptr for h in hs])
    xp = (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs]) if want_vectors else None
    if mode is None:   # the faster of the two on the eight-system batch workload
        mode = ADC2_BATCH_ROUNDS
    st = load().adc2_davidson_batch(n, hp, nroots, ctypes.byref(opts), mode, omega, xp, infos, _stream_ptr(stream))
    _check(st, "adc2_davidson_batch")
    om = [list(omega[q * nroots:(q + 1) * nroots]) for q in range(n)]
    return om, Xs, [infos[q].as_dict(nroots) for q in range(n)]


def adc2_set_precision(h: Handle, prec: int):
    _check(load().adc2_set_precision(h.ptr, prec), "adc2_set_precision")


def adc2_set_method(h: Handle, method: int, stream=None):
    """ADC2_METHOD_ADC2 (default) or ADC2_METHOD_ADC2X (first-order doubles
    block; its integrals are formed on first selection)."""
    _check(load().adc2_set_method(h.ptr, int(method), _stream_ptr(stream)), "adc2_set_method")


def adc2_rayleigh(h: Handle, X, stream=None):
    """FP64 Rayleigh quotients and residual norms of the rows of X."""
    import torch
    _rows(X, h.dim, "X")
    _need(X, torch.complex128, "X")
    k = X.shape[0]
    om = (ctypes.c_double * k)()
    rn = (ctypes.c_double * k)()
    _check(load().adc2_rayleigh(h.ptr, k, ctypes.c_void_p(X.data_ptr()), om, rn, _stream_ptr(stream)),
           "adc2_rayleigh")
    return list(om), list(rn)


def adc2_omega_backward(h: Handle, X, g_omega, dL=None, deps=None, stream=None):
    """Gradient of sum_k g_k x_k^H M x_k / x_k^H x_k with respect to L
    (Hermitian-projected, complex128 [naux][n][n]) and eps (float64 [n])."""
    import torch
    if X.dim() == 1:
        X = X[None]
    _rows(X, h.dim, "X")
    _need(X, torch.complex128, "X")
    k = X.shape[0]
    g = [float(v) for v in (g_omega.tolist() if isinstance(g_omega, torch.Tensor) else g_omega)]
    if len(g) != k:
        raise ValueError("g_omega must have one entry per vector")
    n = h.nc + h.no + h.nv
    if dL is None:
        dL = torch.empty((h.naux, n, n), dtype=torch.complex128, device=X.device)
    if deps is None:
        deps = torch.empty((n,), dtype=torch.float64, device=X.device)
    _need(dL, torch.complex128, "dL")
    _need(deps, torch.float64, "deps")
    if tuple(dL.shape) != (h.naux, n, n) or tuple(deps.shape) != (n,):
        raise ValueError("dL must be [naux][n][n] and deps [n]")
    ga = (ctypes.c_double * k)(*g)
    _check(load().adc2_omega_backward(h.ptr, k, ctypes.c_void_p(X.data_ptr()), ga,
                                      ctypes.c_void_p(dL.data_ptr()), ctypes.c_void_p(deps.data_ptr()),
                                      _stream_ptr(stream)), "adc2_omega_backward")
    return dL, deps


_omega_fn = None


def _omega_function():
    global _omega_fn
    if _omega_fn is not None:
        return _omega_fn
    import torch

    class Adc2Omega(torch.autograd.Function):
        """omega = lowest eigenvalues of M(L, eps); backward by adc2_omega_backward."""

        @staticmethod
        def forward(ctx, L, eps, nc, no, nv, nroots, tol, max_iter, solver):
            naux = L.shape[0]
            h = adc2_setup(L.detach().contiguous(), eps.detach().contiguous(), nc, no, nv, naux)
            w, X, _ = adc2_davidson(h, nroots, tol=tol, max_iter=max_iter, solver=solver)
            # the handle lives as long as the graph node: it is destroyed when
            # ctx is released (Handle.__del__), so backward may run again
            # under retain_graph=True
            ctx.h, ctx.X = h, X
            return torch.tensor(w, dtype=torch.float64, device=L.device)

        @staticmethod
        def backward(ctx, g):
            dL, de = adc2_omega_backward(ctx.h, ctx.X, g.detach().cpu())
            return dL, de, None, None, None, None, None, None, None

    _omega_fn = Adc2Omega
    return _omega_fn


def adc2_omega(L, eps, nc, no, nv, nroots, tol=1e-10, max_iter=0, solver=ADC2_SOLVER_FOLDED):
    """Lowest nroots eigenvalues as a differentiable function of (L, eps).
    solver: ADC2_SOLVER_FOLDED (default; roots below the doubles threshold,
    the case of every benchmark system) or ADC2_SOLVER_FULL."""
    return _omega_function().apply(L, eps, nc, no, nv, nroots, tol, max_iter, solver)


def adc2_get_m11(h: Handle, stream=None):
    import torch
    out = torch.empty((h.ns, h.ns), dtype=torch.complex128, device="cuda")
    _check(load().adc2_get_m11(h.ptr, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "adc2_get_m11")
    return out


def adc2_get_diag(h: Handle, stream=None):
    import torch
    out = torch.empty((h.dim,), dtype=torch.float64, device="cuda")
    _check(load().adc2_get_diag(h.ptr, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "adc2_get_diag")
    return out


def adc2_mp2_energy(h: Handle) -> float:
    e = ctypes.c_double()
    _check(load().adc2_mp2_energy(h.ptr, ctypes.byref(e)), "adc2_mp2_energy")
    return e.value


def adc2_profile(h: Handle, enable: bool = True):
    _check(load().adc2_profile(h.ptr, 1 if enable else 0), "adc2_profile")


def adc2_kernel_stats(h: Handle):
    arr = (KStat * 16)()
    n = load().adc2_kernel_stats(h.ptr, arr, 16)
    if n < 0:
        raise Adc2Error(ADC2_ERR_ARG, "adc2_kernel_stats: NULL handle")
    return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms, "flops": arr[i].flops}
            for i in range(n)}


def adc2_transition(h: Handle, dip, X, omega, order: int = 2, stream=None):
    """Transition dipole moments T [k][3] (complex) and oscillator strengths
    f [k] of the eigenpairs (X, omega); dip: [3][n][n] complex128 on the GPU;
    order: the singles of F through first (1) or second (2) order."""
    import numpy as np
    import torch
    n = h.nc + h.no + h.nv
    if tuple(dip.shape) != (3, n, n):
        raise ValueError(f"dip must be [3][{n}][{n}], got {list(dip.shape)}")
    _rows(X, h.dim, "X")
    k = X.shape[0]
    omega = [float(w) for w in (omega.tolist() if isinstance(omega, torch.Tensor) else omega)]
    if len(omega) != k:
        raise ValueError(f"omega must have one entry per row of X ({k}), got {len(omega)}")
    _need(dip, torch.complex128, "dip")
    _need(X, torch.complex128, "X")
    om = (ctypes.c_double * k)(*omega)
    T = np.zeros((k, 3), dtype=np.complex128)
    f = (ctypes.c_double * k)()
    _check(load().adc2_transition(h.ptr, ctypes.c_void_p(dip.data_ptr()), k, ctypes.c_void_p(X.data_ptr()), om,
                                  int(order), ctypes.c_void_p(T.ctypes.data), f, _stream_ptr(stream)),
           "adc2_transition")
    return T, np.array(f[:])


def adc2_fns(h: Handle, L, threshold: float, stream=None):
    """Frozen natural virtual spinors from the MP2 density of h's system.
    Returns (L', eps', nv', occupations): the rotated Cholesky vectors and
    energies of the truncated problem (nc, no, nv', naux)."""
    import torch
    n = h.nc + h.no + h.nv
    if tuple(L.shape) != (h.naux, n, n):
        raise ValueError(f"L must be [{h.naux}][{n}][{n}], got {list(L.shape)}")
    _need(L, torch.complex128, "L")
    occ = (ctypes.c_double * h.nv)()
    nvp = ctypes.c_int()
    Lout = torch.empty((h.naux * n * n,), dtype=torch.complex128, device="cuda")
    eout = torch.empty((n,), dtype=torch.float64, device="cuda")
    _check(load().adc2_fns(h.ptr, ctypes.c_void_p(L.data_ptr()), float(threshold), ctypes.byref(nvp), occ,
                           ctypes.c_void_p(Lout.data_ptr()), ctypes.c_void_p(eout.data_ptr()), _stream_ptr(stream)),
           "adc2_fns")
    np_ = h.nc + h.no + nvp.value
    Lp = Lout[:h.naux * np_ * np_].view(h.naux, np_, np_).clone()
    return Lp, eout[:np_].clone(), nvp.value, list(occ)


def adc2_autotune(h: Handle, m: int, stream=None) -> dict:
    """Times the Y-build candidates of h at block size m (in the FP64 form its
    engines, then the K-splits of the fastest) and fixes the fastest; returns
    {"ysplit", "zgemm", "from_cache", "ms": {split: ms}, "engines": {zgemm: ms}}."""
    info = TuneInfo()
    _check(load().adc2_autotune(h.ptr, m, ctypes.byref(info), _stream_ptr(stream)), "adc2_autotune")
    return {"ysplit": info.ysplit, "zgemm": info.zgemm, "from_cache": bool(info.from_cache),
            "ms": {info.cand[c]: info.ms[c] for c in range(info.ncand)},
            "engines": {info.engine[e]: info.engine_ms[e] for e in range(info.nengine)}}


def adc2_peak_probe(kind: int, nbytes: int = 0, reps: int = 5, stream=None) -> float:
    """Measured device rate for one of the ADC2_PEAK_* kinds: TFLOP/s for the
    MFMA and FMA probes, GB/s for the HBM probes."""
    r = ctypes.c_double()
    _check(load().adc2_peak_probe(kind, nbytes, reps, ctypes.byref(r), _stream_ptr(stream)), "adc2_peak_probe")
    return r.value


def adc2_destroy(h: Handle):
    h.close()


def header_exports(path: str = HEADER):
    """Names of the functions include/adc2.h declares."""
    import re
    txt = open(path).read()
    return sorted(set(re.findall(r"ADC2_API\s+[\w\s\*]+?\b(adc2_\w+)\s*\(", txt)))
