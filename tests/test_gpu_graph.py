"""GPU tests of the graph-captured batched sigma (adc2_graph_sigma_batch,
adc2_graph_launch, adc2_graph_destroy).

The graph records the launch sequence of one adc2_sigma_batch call, so every
replay must equal an eager adc2_sigma_batch on the same inputs bit for bit.
Each test replays several times, refills X in place between replays, puts
unrelated eager GPU work and host synchronisations between them, and checks
every replay.  The FP64 member is also checked against the oracle's sigma.
"""
import numpy as np
import pytest
import torch

import paper_2604_27451_amd as A
from oracle import adc2 as O
from synth import batch_systems, random_vectors

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def mixed_batch(scale, precs):
    systems = batch_systems(scale)[:len(precs)]
    print(f"[case] graph batch precs={precs} sizes={[(s.no, s.nv, s.naux) for s in systems]}", flush=True)
    data = [(dev(s.L), dev(s.eps), s.nc, s.no, s.nv, s.naux) for s in systems]
    hs = A.adc2_setup_batch(data, A.ADC2_FP64)
    for h, p in zip(hs, precs):
        if p != A.ADC2_FP64:
            A.adc2_set_precision(h, p)
    return systems, hs


def refill(xs, seed):
    for q, x in enumerate(xs):
        x.copy_(dev(random_vectors(seed + q, x.shape[0], x.shape[1])))


def test_graph_replays_equal_eager_mixed_precisions():
    precs = [A.ADC2_FP64, A.ADC2_C64, A.ADC2_BF16X3, A.ADC2_C64]
    systems, hs = mixed_batch(0.1, precs)
    xs = [dev(random_vectors(1200 + q, 1 + q % 3, h.dim)) for q, h in enumerate(hs)]
    eager0 = [s.clone() for s in A.adc2_sigma_batch(hs, xs)]
    g = A.adc2_graph_sigma_batch(hs, xs)
    torch.cuda.synchronize()
    for q in range(len(hs)):     # the capture call's own eager run
        assert torch.equal(g.S[q], eager0[q]), q
    s0 = systems[0]
    ref = O.Adc2(s0.L, s0.eps, s0.nc, s0.no, s0.nv).sigma(xs[0].cpu())
    for rep in range(4):
        if rep > 0:
            refill(xs, 1300 + 10 * rep)
        for S in g.S:
            S.fill_(float("nan"))
        # unrelated eager work on the same stream and a host synchronisation
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        eager = A.adc2_sigma_batch(hs, xs)
        torch.cuda.synchronize()
        for q in range(len(hs)):
            assert torch.equal(g.S[q], eager[q]), (rep, q)
        if rep == 0:
            err = ((g.S[0].cpu() - ref).abs().max() / ref.abs().max()).item()
            print(f"  replay 0: fp64 member vs oracle {err:.2e}", flush=True)
            assert err < 1e-11
        print(f"  replay {rep} equals eager ({float(junk[0, 0]):.1f})", flush=True)
    g.close()
    for h in hs:
        h.close()


def test_graph_replays_interleaved_with_other_sigma():
    """Between replays the handles serve other work (a smaller sigma, an
    eager batched sigma into other buffers); the graph keeps replaying the
    captured sequence."""
    systems, hs = mixed_batch(0.1, [A.ADC2_C64, A.ADC2_C64, A.ADC2_BF16X3])
    xs = [dev(random_vectors(1400 + q, 2, h.dim)) for q, h in enumerate(hs)]
    g = A.adc2_graph_sigma_batch(hs, xs)
    for rep in range(3):
        refill(xs, 1500 + 10 * rep)
        small = A.adc2_sigma(hs[1], xs[1][:1].clone())     # m = 1 fits the captured work spaces
        g.launch()
        other = A.adc2_sigma_batch(hs, [x.clone() for x in xs])
        torch.cuda.synchronize()
        for q in range(len(hs)):
            assert torch.equal(g.S[q], other[q]), (rep, q)
        # the m = 1 product agrees with the first row of the m = 2 one to complex64 rounding
        assert ((small[0] - other[1][0]).abs().max() / other[1][0].abs().max()).item() < 1e-5
    g.close()
    for h in hs:
        h.close()


def test_graph_refuses_changed_workspaces_and_recaptures():
    systems, hs = mixed_batch(0.1, [A.ADC2_FP64, A.ADC2_C64])
    xs = [dev(random_vectors(1600 + q, 1, h.dim)) for q, h in enumerate(hs)]
    g = A.adc2_graph_sigma_batch(hs, xs)
    g.launch()
    torch.cuda.synchronize()
    # a larger block re-sizes system 1's work spaces: the graph must not replay
    A.adc2_sigma(hs[1], dev(random_vectors(1700, 3, hs[1].dim)))
    torch.cuda.synchronize()
    with pytest.raises(A.Adc2Error, match="capture the batch again"):
        g.launch()
    g.close()
    with pytest.raises(A.Adc2Error, match="closed"):
        g.launch()
    # a change of precision form is refused too; a new capture replays again
    g2 = A.adc2_graph_sigma_batch(hs, xs)
    A.adc2_set_precision(hs[0], A.ADC2_BF16X3)
    with pytest.raises(A.Adc2Error, match="capture the batch again"):
        g2.launch()
    A.adc2_set_precision(hs[0], A.ADC2_FP64)
    g2.launch()
    eager = A.adc2_sigma_batch(hs, xs)
    torch.cuda.synchronize()
    for q in range(2):
        assert torch.equal(g2.S[q], eager[q]), q
    g2.close()
    # the autotuner re-sizes the work spaces for a smaller block (they may come back at the
    # same addresses): the graph of the larger block must not replay into them
    g3 = A.adc2_graph_sigma_batch(hs, [dev(random_vectors(1800 + q, 3, h.dim)) for q, h in enumerate(hs)])
    A.adc2_autotune(hs[1], 1)
    with pytest.raises(A.Adc2Error, match="capture the batch again"):
        g3.launch()
    g3.close()
    # the ADC(2)-x method is not captured
    A.adc2_set_method(hs[0], A.ADC2_METHOD_ADC2X)
    with pytest.raises(A.Adc2Error, match="ADC\\(2\\)-x"):
        A.adc2_graph_sigma_batch(hs, xs)
    for h in hs:
        h.close()
