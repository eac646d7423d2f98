"""GPU checks of the autotuner (adc2_autotune) and of the FP64 GEMM engines
it chooses between.

The tuner times the FP64 engines (tile shapes) at their size-rule K-splits,
then every Y-build K-split candidate of the fastest (or of the form's only
engine), and fixes the fastest; a sigma build after tuning must still match
the oracle (engine and K-split only change the summation order), a second
handle of the same shape must take the choice from the cache without timing,
and the choice must be written to the cache file named by ADC2_TUNE_CACHE.
The four-multiplication engines must give identical products at equal
K-splits; every engine must match the oracle.
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
    print(f"  choice {r['ysplit']} from {r['ms']}; engine {r['zgemm']} from {r['engines']}", flush=True)
    assert not r["from_cache"]
    assert r["ysplit"] in r["ms"] and len(r["ms"]) >= 2
    assert r["ms"][r["ysplit"]] == min(r["ms"].values())
    if prec == A.ADC2_FP64:
        assert sorted(r["engines"]) == [0, 1, 2, 3]
        assert r["engines"][r["zgemm"]] == min(r["engines"].values())
    else:
        assert r["engines"] == {}
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
    assert r2["from_cache"] and r2["ysplit"] == r["ysplit"] and r2["ms"] == {} and r2["zgemm"] == r["zgemm"]
    assert torch.equal(A.adc2_sigma(h2, x).cpu(), S)
    lines = open(CACHE).read().splitlines()
    if prec == A.ADC2_FP64:
        key = re.compile(rf"prec=0 zgemm=search engine={r['zgemm']} ysplit={r['ysplit']}$")
    else:
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


def test_fp64_engines_equal_and_match_oracle(monkeypatch):
    """Equal K-splits (forced): the four-multiplication engines (128 x 128 on
    four and on eight waves, 128 x 64 two per CU) give the same product bit
    for bit (same MFMAs in the same k order per output), and every engine,
    the three-multiplication one included, matches the oracle."""
    s = make_system(2, 7, 37, 110, seed=41)
    x = dev(random_vectors(78, 3, s.nc * s.nv + s.nc * s.no * s.nv * (s.nv - 1) // 2))
    ref = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv).sigma(x.cpu())
    out = {}
    monkeypatch.setenv("ADC2_YSPLIT", "3")
    for eng in ("big", "mid", "wide", "3m"):
        monkeypatch.setenv("ADC2_ZGEMM", eng)
        print(f"[case] engine {eng} shape {(s.nc, s.no, s.nv, s.naux)} K-split 3", flush=True)
        h = A.adc2_setup(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux)
        out[eng] = A.adc2_sigma(h, x).cpu()
        h.close()
        err = ((out[eng] - ref).abs().max() / ref.abs().max()).item()
        print(f"  vs oracle {err:.2e}", flush=True)
        assert err < 1e-11
    assert torch.equal(out["big"], out["mid"]) and torch.equal(out["big"], out["wide"])
