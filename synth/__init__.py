"""Seeded synthetic inputs for two-component CVS-ADC(2).

This module only draws random numbers; it holds none of the method's
arithmetic.  Both the CPU oracle and the GPU path take their inputs from here.

A system is a set of complex MO Cholesky vectors L[P, p, q] (each L[P] is
Hermitian: L[P, q, p] = conj(L[P, p, q])) and spinor energies eps[p], with the
spinors ordered [core | valence | virtual].

Recipe (all draws FP64):
  * eps: one generator seeded with SeedSequence([seed, 0]); core, valence and
    virtual energies are drawn uniform in their ranges, in that order, and each
    block is sorted ascending.
  * L[P]: one generator per Cholesky index P, seeded SeedSequence([seed, 1, P]).
    It draws the strict upper triangle (row-major p < q) as CN(0, sigma^2)
    (real and imaginary parts N(0, sigma^2/2)), then the real diagonal as
    N(0, sigma^2); the lower triangle is the conjugate mirror.
The per-P generators make generation chunkable and reproducible at any size.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EPS_CORE = (-30.0, -28.0)
EPS_VAL = (-1.0, -0.3)
EPS_VIRT = (0.1, 5.0)


@dataclass
class System:
    nc: int
    no: int
    nv: int
    naux: int
    L: np.ndarray          # complex128 [naux][n][n]
    eps: np.ndarray        # float64 [n]
    seed: int = 0
    label: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nc + self.no + self.nv


def draw_eps(seed: int, nc: int, no: int, nv: int,
             core=EPS_CORE, val=EPS_VAL, virt=EPS_VIRT) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0]))
    e_c = np.sort(rng.uniform(core[0], core[1], nc))
    e_o = np.sort(rng.uniform(val[0], val[1], no))
    e_v = np.sort(rng.uniform(virt[0], virt[1], nv))
    return np.concatenate([e_c, e_o, e_v]).astype(np.float64)


def draw_cholesky_P(seed: int, P: int, n: int, sigma: float) -> np.ndarray:
    """One Hermitian n x n Cholesky slice L[P]."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 1, P]))
    iu = np.triu_indices(n, 1)
    m = iu[0].size
    s = sigma / math.sqrt(2.0)
    re = rng.standard_normal(m)
    im = rng.standard_normal(m)
    d = rng.standard_normal(n) * sigma
    out = np.zeros((n, n), dtype=np.complex128)
    out[iu] = (re + 1j * im) * s
    out[(iu[1], iu[0])] = np.conj(out[iu])
    out[np.arange(n), np.arange(n)] = d
    return out


def draw_cholesky(seed: int, naux: int, n: int, sigma: float,
                  out: np.ndarray | None = None, threads: int = 16) -> np.ndarray:
    """All slices L[P]; large draws are spread over a pool of host threads
    (each slice has its own generator, so the values do not depend on it)."""
    if out is None:
        out = np.empty((naux, n, n), dtype=np.complex128)

    def one(P):
        out[P] = draw_cholesky_P(seed, P, n, sigma)
    if threads > 1 and naux * n * n > (1 << 22):
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(naux)))
    else:
        for P in range(naux):
            one(P)
    return out


def draw_cholesky_device(seed: int, naux: int, n: int, sigma: float, device="cuda", threads: int = 16,
                         chunk: int = 64):
    """draw_cholesky straight into a device tensor [naux][n][n] (complex128):
    the same per-P draws, made by a pool of host threads chunk by chunk and
    copied to the device, so that no host array of the whole size is held."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    out = torch.empty((naux, n, n), dtype=torch.complex128, device=device)
    host = torch.empty((chunk, n, n), dtype=torch.complex128).pin_memory()
    hv = host.numpy()
    with ThreadPoolExecutor(max(1, threads)) as ex:
        for p0 in range(0, naux, chunk):
            p1 = min(naux, p0 + chunk)

            def one(P, p0=p0):
                hv[P - p0] = draw_cholesky_P(seed, P, n, sigma)
            list(ex.map(one, range(p0, p1)))
            out[p0:p1].copy_(host[:p1 - p0])
    torch.cuda.synchronize(device)
    return out


def config_inputs_device(name: str, device="cuda", threads: int = 16):
    """(L, eps) of a configuration on the device, drawn as config_system draws
    them (same values)."""
    import torch
    c = CONFIGS[name]
    n = c["nc"] + c["no"] + c["nv"]
    eps = torch.from_numpy(draw_eps(c["seed"], c["nc"], c["no"], c["nv"])).to(device)
    return draw_cholesky_device(c["seed"], c["naux"], n, 0.05, device, threads), eps


def make_system(nc: int, no: int, nv: int, naux: int, seed: int,
                sigma: float = 0.05, core=EPS_CORE, val=EPS_VAL,
                virt=EPS_VIRT, label: str = "") -> System:
    n = nc + no + nv
    eps = draw_eps(seed, nc, no, nv, core, val, virt)
    L = draw_cholesky(seed, naux, n, sigma)
    return System(nc, no, nv, naux, L, eps, seed, label)


def make_spin_blocked(nc_sp: int, no_sp: int, nv_sp: int, naux: int, seed: int,
                      sigma: float = 0.05, core=(-3.0, -2.5), val=EPS_VAL,
                      virt=EPS_VIRT) -> System:
    """Nonrelativistic-limit input: real symmetric spatial Cholesky vectors
    l[P, p, q] copied onto both spin blocks, spin-degenerate energies.

    Spatial orbital i of a block becomes spinors 2i (alpha) and 2i+1 (beta)
    of that block; L[P, (p,s), (q,s')] = delta_{s s'} l[P, p, q].
    """
    n_sp = nc_sp + no_sp + nv_sp
    rng_e = np.random.default_rng(np.random.SeedSequence([seed, 0]))
    e_c = np.sort(rng_e.uniform(core[0], core[1], nc_sp))
    e_o = np.sort(rng_e.uniform(val[0], val[1], no_sp))
    e_v = np.sort(rng_e.uniform(virt[0], virt[1], nv_sp))
    e_sp = np.concatenate([e_c, e_o, e_v])
    l = np.empty((naux, n_sp, n_sp))
    for P in range(naux):
        rng = np.random.default_rng(np.random.SeedSequence([seed, 2, P]))
        a = rng.standard_normal((n_sp, n_sp)) * sigma
        l[P] = (a + a.T) / math.sqrt(2.0)
    n = 2 * n_sp
    L = np.zeros((naux, n, n), dtype=np.complex128)
    for s in range(2):
        idx = 2 * np.arange(n_sp) + s
        L[:, idx[:, None], idx[None, :]] = l
    eps = np.repeat(e_sp, 2)
    sysm = System(2 * nc_sp, 2 * no_sp, 2 * nv_sp, naux, L, eps, seed, "spin-blocked")
    sysm.extra["l_spatial"] = l
    sysm.extra["eps_spatial"] = e_sp
    sysm.extra["n_spatial"] = (nc_sp, no_sp, nv_sp)
    return sysm


def random_vectors(seed: int, m: int, dim: int) -> np.ndarray:
    """m complex128 vectors of length dim, entries CN(0, 1)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 3]))
    v = rng.standard_normal((m, dim)) + 1j * rng.standard_normal((m, dim))
    return (v / math.sqrt(2.0)).astype(np.complex128)


def dipole_integrals(seed: int, n: int, scale: float = 0.5) -> np.ndarray:
    """Stand-in spinor dipole integrals d^x, d^y, d^z: [3][n][n] complex
    Hermitian, entries of size ~scale (atomic units)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 5]))
    a = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    return np.ascontiguousarray(0.5 * scale * (a + np.conj(np.transpose(a, (0, 2, 1)))), dtype=np.complex128)


def random_hermitian_direction(seed: int, naux: int, n: int) -> np.ndarray:
    """A Hermitian-per-P direction dL of unit Frobenius norm."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4]))
    a = rng.standard_normal((naux, n, n)) + 1j * rng.standard_normal((naux, n, n))
    h = 0.5 * (a + np.conj(np.transpose(a, (0, 2, 1))))
    return h / np.linalg.norm(h)


# Configurations of the workloads (sizes, energy ranges, Cholesky spread).
CONFIGS = {
    # small case: oracle Davidson finishes in seconds
    "c1": dict(nc=6, no=10, nv=40, naux=150, nroots=4, seed=27451 + 1),
    # 3d-transition-metal-compound-like size after virtual truncation
    "c2": dict(nc=6, no=60, nv=300, naux=1500, nroots=10, seed=27451 + 2),
    # heavy-element-complex shape (precision form)
    "c3": dict(nc=6, no=120, nv=600, naux=3000, nroots=10, seed=27451 + 3),
    # several tiles with ragged tails; oracle still finishes in seconds
    "mid": dict(nc=6, no=12, nv=100, naux=300, nroots=6, seed=27451 + 11),
    # ragged tiles in every dimension; the oracle Davidson converges in seconds
    "tiles": dict(nc=3, no=6, nv=80, naux=60, nroots=4, seed=27451 + 12),
}


def config_system(name: str) -> System:
    c = CONFIGS[name]
    return make_system(c["nc"], c["no"], c["nv"], c["naux"], c["seed"], label=name)


# Batching form: eight systems of uneven size, nc = 6, naux = 4 nv, 16 roots
# each; system m drawn with seed 274510 + m.
BATCH_C4 = [(20, 100), (80, 400), (35, 250), (60, 150), (25, 380), (70, 220), (45, 310), (55, 120)]


def batch_systems(scale: float = 1.0, nc: int = 6) -> list:
    """The batching workload; scale < 1 shrinks no and nv (naux = 4 nv kept)
    for parity tests the oracle can follow."""
    out = []
    for m, (no, nv) in enumerate(BATCH_C4):
        no_s = max(1, int(round(no * scale)))
        nv_s = max(2, int(round(nv * scale)))
        out.append(make_system(nc, no_s, nv_s, 4 * nv_s, 274510 + m, label=f"c4[{m}]"))
    return out


def random_hermitian_direction_device(seed: int, naux: int, n: int, device="cuda"):
    """A Hermitian-per-P direction dL of unit Frobenius norm drawn on the
    device (torch generator seeded with seed): for directions at sizes where a
    host draw would dominate the run time."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    re = torch.randn((naux, n, n), generator=g, device=device, dtype=torch.float64)
    im = torch.randn((naux, n, n), generator=g, device=device, dtype=torch.float64)
    a = torch.complex(re, im)
    del re, im
    h = 0.5 * (a + a.transpose(1, 2).conj())
    del a
    return h / torch.linalg.vector_norm(h)
