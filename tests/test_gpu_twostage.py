"""GPU check of the two-stage solve (adc2_dav_opts.mixed_tol): split-BF16
sigma builds to mixed_tol, then the FP64 solver from those vectors.  The
roots must be the FP64 roots (same tolerance as a plain FP64 solve), with the
full-space and the folded solver, and they must match the oracle."""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import config_system, make_system

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("solver", [A.ADC2_SOLVER_FULL, A.ADC2_SOLVER_FOLDED])
def test_two_stage_equals_fp64(solver):
    s = config_system("c1")
    print(f"[case] two-stage solve, solver {solver}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    w64, X64, i64 = A.adc2_davidson(h, 4, tol=1e-9, solver=solver, max_iter=400)
    w2, X2, i2 = A.adc2_davidson(h, 4, tol=1e-9, solver=solver, max_iter=400, mixed_tol=1e-4)
    print(f"  plain {i64['iters']} it, two-stage {i2['iters']} it, max|dw| {np.abs(np.array(w2) - np.array(w64)).max():.1e}",
          flush=True)
    assert i2["converged"] and max(i2["resnorm"]) <= 1e-9
    assert np.abs(np.array(w2) - np.array(w64)).max() < 1e-10
    ov = (X2.conj() @ X64.T).abs().diagonal().cpu().numpy()
    assert np.abs(ov - 1).max() < 1e-8
    h.close()


def test_two_stage_vs_oracle_and_errors():
    s = make_system(2, 4, 14, 30, seed=61)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    w2, _, _ = A.adc2_davidson(h, 3, tol=1e-10, mixed_tol=1e-3)
    a = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    w0, _ = a.roots_exact(3)
    assert np.abs(np.array(w2) - w0.numpy()).max() < 1e-9
    with pytest.raises(A.Adc2Error):
        A.adc2_davidson(h, 3, tol=1e-6, mixed_tol=1e-7)          # mixed_tol must exceed tol
    A.adc2_set_precision(h, A.ADC2_C64)
    with pytest.raises(A.Adc2Error):
        A.adc2_davidson(h, 3, tol=1e-8, mixed_tol=1e-4)          # needs an FP64 handle
    h.close()
