"""GPU parity at the benchmark sizes, on sampled outputs the oracle computes
one by one (oracle/adc2.py: m11_element, sigma2_element,
sigma1_coupling_element).

c2 (nc=6, no=60, nv=300, naux=1500) and c3 (nc=6, no=120, nv=600,
naux=3000) with m = 10 vectors, the block size of the benchmark's sigma
builds, in every precision form.  Sampled entries include the first and last
pair (a, b) and the last core/valence indices, so that the ragged tails of
every GEMM tile dimension are hit.  Whole rows of M11 are compared with the
oracle's row evaluator (m11_row): at c2 complete rows, at c3 the columns
J != I of a row (the delta_IJ term would need every <kl||bc>, 5.7e9
integrals, on the host).

Singles entries of sigma are split into the singles block and the
doubles-to-singles coupling: M11 is checked entry by entry against
m11_element, and (S - M11 x)_singles against sigma1_coupling_element with
the GPU's M11 (already checked) applied on the host.
Tolerances: FP64 |gpu - oracle| <= 1e-10 max|oracle| over the sampled
entries of the same kind; complex64 3e-5; split-BF16 1e-4 (measured
relative sigma errors 1e-7 and 1.5e-6).
"""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import config_system, random_vectors

pytestmark = pytest.mark.gpu

TOL = {A.ADC2_FP64: 1e-10, A.ADC2_C64: 3e-5, A.ADC2_BF16X3: 1e-4}


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def doubles_samples(nc, no, nv, rng, n):
    pts = [(0, 0, 0, 1), (nc - 1, no - 1, nv - 2, nv - 1), (0, no - 1, 0, nv - 1), (nc - 1, 0, nv // 2, nv // 2 + 1)]
    while len(pts) < n:
        I, j = int(rng.integers(nc)), int(rng.integers(no))
        a, b = sorted(int(v) for v in rng.choice(nv, 2, replace=False))
        pts.append((I, j, a, b))
    return pts


def doubles_offset(nc, no, nv, I, j, a, b):
    q = a * nv - a * (a + 1) // 2 + (b - a - 1)
    return nc * nv + (I * no + j) * (nv * (nv - 1) // 2) + q


def run_case(name, precs, m, n_d, n_s, n_m11, s_vecs=None, rows=(), rows_offdiag=()):
    s = config_system(name)
    nc, no, nv = s.nc, s.no, s.nv
    sp = O.Spaces(nc, no, nv)
    Lt, et = torch.from_numpy(s.L), torch.from_numpy(s.eps)
    print(f"[case] full size {name} m={m} precs={precs}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), nc, no, nv, s.naux)
    x = dev(random_vectors(4242, m, h.dim))
    xc = x.cpu()
    rng = np.random.default_rng(27451)
    # singles block, entry by entry
    M11 = A.adc2_get_m11(h).cpu()
    ns = nc * nv
    m_pts = [(0, 0, 0, 0), (nc - 1, nv - 1, 0, 0), (0, 1, 0, 1)][:n_m11]
    while len(m_pts) < n_m11:
        m_pts.append((int(rng.integers(nc)), int(rng.integers(nv)), int(rng.integers(nc)), int(rng.integers(nv))))
    ref = np.array([O.m11_element(Lt, et, sp, I, a, J, b) for I, a, J, b in m_pts])
    got = np.array([complex(M11[I * nv + a, J * nv + b]) for I, a, J, b in m_pts])
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  M11 sampled rel err {err:.2e}", flush=True)
    assert err < 1e-10
    Mr = M11.reshape(nc, nv, nc, nv)
    for I, a in rows:
        ref_r = O.m11_row(Lt, et, sp, I, a)
        err = float((Mr[I, a] - ref_r).abs().max() / ref_r.abs().max())
        print(f"  M11 row ({I},{a}) rel err {err:.2e}", flush=True)
        assert err < 1e-10
    for I, a in rows_offdiag:
        ref_r = O.m11_row(Lt, et, sp, I, a, with_term_i=False)
        keep = [J for J in range(nc) if J != I]
        err = float((Mr[I, a, keep] - ref_r[keep]).abs().max() / ref_r[keep].abs().max())
        print(f"  M11 row ({I},{a}), columns J != I, rel err {err:.2e}", flush=True)
        assert err < 1e-10
    d_pts = doubles_samples(nc, no, nv, rng, n_d)
    s_pts = ([(0, 0), (nc - 1, nv - 1)] + [(int(rng.integers(nc)), int(rng.integers(nv))) for _ in range(n_s)])[:n_s]
    vecs = [0, m - 1]
    s_vecs = vecs if s_vecs is None else s_vecs
    d_ref = {(v, p): O.sigma2_element(Lt, et, sp, xc[v], *p) for v in vecs for p in d_pts}
    s_ref = {(v, p): O.sigma1_coupling_element(Lt, sp, xc[v], *p) for v in s_vecs for p in s_pts}
    print(f"  oracle samples ready", flush=True)
    for prec in precs:
        A.adc2_set_precision(h, prec)
        S = A.adc2_sigma(h, x).cpu()
        # doubles entries
        gd = np.array([complex(S[v, doubles_offset(nc, no, nv, *p)]) for v in vecs for p in d_pts])
        rd = np.array([d_ref[(v, p)] for v in vecs for p in d_pts])
        ed = np.abs(gd - rd).max() / np.abs(rd).max()
        # singles: coupling part = S1 - M11 x1
        x1 = xc[:, :ns]
        c1 = S[:, :ns] - x1 @ M11.T
        gs = np.array([complex(c1[v, K * nv + c]) for v in s_vecs for K, c in s_pts])
        rs = np.array([s_ref[(v, p)] for v in s_vecs for p in s_pts])
        es = np.abs(gs - rs).max() / np.abs(rs).max()
        print(f"  prec {prec}: doubles rel err {ed:.2e}, coupling rel err {es:.2e}", flush=True)
        assert ed < TOL[prec] and es < TOL[prec]
    h.close()


def test_c2_sampled_sigma_all_precisions():
    run_case("c2", [A.ADC2_FP64, A.ADC2_C64, A.ADC2_BF16X3], 10, 12, 4, 5, rows=[(5, 299)],
             rows_offdiag=[(0, 0), (3, 150)])


def test_c3_sampled_sigma_all_precisions():
    # the c3 evaluators are costly on the host (one coupling entry contracts
    # nv^2 no naux = 1.3e11 terms): fewer coupling samples, same kinds
    run_case("c3", [A.ADC2_FP64, A.ADC2_C64, A.ADC2_BF16X3], 10, 16, 2, 3, s_vecs=[9],
             rows_offdiag=[(5, 599)])
