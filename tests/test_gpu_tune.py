"""GPU checks of the autotuner (adc2_autotune).

The tuner times every Y-build K-split candidate of a handle and fixes the
fastest; a sigma build after tuning must still match the oracle (the K-split
only changes the summation order), a second handle of the same shape must
take the choice from the cache without timing, and the choice must be
written to the cache file named by ADC2_TUNE_CACHE.
"""
import os
import re
import tempfile

import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import make_system, random_vectors

pytestmark = pytest.mark.gpu

CACHE = os.path.join(tempfile.mkdtemp(prefix="adc2tune"), "tune.txt")
os.environ["ADC2_TUNE_CACHE"] = CACHE


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("prec", [A.ADC2_FP64, A.ADC2_C64, A.ADC2_BF16X3])
def test_autotune_choice_keeps_sigma_and_is_cached(prec):
    s = make_system(2, 8, 40, 120, seed=31 + prec)
    print(f"[case] autotune prec={prec} shape {(s.nc, s.no, s.nv, s.naux)}", flush=True)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux, prec=prec)
    x = dev(random_vectors(77, 3, h.dim))
    r = A.adc2_autotune(h, 3)
    print(f"  choice {r['ysplit']} from {r['ms']}", flush=True)
    assert not r["from_cache"]
    assert r["ysplit"] in r["ms"] and len(r["ms"]) >= 2
    assert r["ms"][r["ysplit"]] == min(r["ms"].values())
    S = A.adc2_sigma(h, x).cpu()
    o = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv)
    ref = o.sigma(x.cpu())
    err = ((S - ref).abs().max() / ref.abs().max()).item()
    tol = {A.ADC2_FP64: 1e-11, A.ADC2_C64: 3e-5, A.ADC2_BF16X3: 1e-4}[prec]
    print(f"  sigma after tuning vs oracle {err:.2e}", flush=True)
    assert err < tol
    # same shape, same block size and form: the cached choice, no timing
    h2 = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux, prec=prec)
    r2 = A.adc2_autotune(h2, 3)
    assert r2["from_cache"] and r2["ysplit"] == r["ysplit"] and r2["ms"] == {}
    assert torch.equal(A.adc2_sigma(h2, x).cpu(), S)
    lines = open(CACHE).read().splitlines()
    key = re.compile(rf"prec={prec} zgemm=\d+ ysplit={r['ysplit']}$")
    assert any(key.search(l) and "nv=40" in l for l in lines), lines
    h.close()
    h2.close()


def test_autotune_rejects_bad_arguments():
    s = make_system(1, 2, 6, 20, seed=5)
    h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
    with pytest.raises(A.Adc2Error):
        A.adc2_autotune(h, 0)
    h.close()
