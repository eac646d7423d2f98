#!/usr/bin/env python3
"""Benchmark: sigma-build complex TFLOP/s and time-to-N-roots of the CVS-ADC(2)
hot path on one MI355X, FP64 and mixed precision side by side.

Default (`--workload headline`): the heavy-element-complex-sized system
nc=6, no=120, nv=600, naux=3000 (complex128, 10 roots, dim 129,387,600),
drawn on the device and resident in HBM before anything is timed.

One step = one sigma build of 10 vectors in each of FP64, complex64 (FP32
MFMA) and split-BF16 (BF16 MFMA, hi + lo operands, three products), every
kernel timed with HIP events on the stream it is launched on.  Once per
invocation, outside the timed steps:
  time_to_roots  from a fresh adc2_setup each (the input L released after
                 it): FP64 roots through split-BF16 (adc2_davidson with
                 mixed_tol = 1e-4, then FP64 to residual 1e-8), and
                 split-BF16 roots to residual 1e-3 followed by their FP64
                 Rayleigh quotients, with the eV error per root
  roots_vs_oracle_c1  both forms against the CPU oracle's roots at
                 nc=6, no=10, nv=40, naux=150
  c2             the whole path at nc=6, no=60, nv=300, naux=1500: setup,
                 FP64 folded solve, adjoint, two-stage solve, split-BF16 and
                 complex64 solves with FP64 Rayleigh quotients
  cpu_baseline   the CPU oracle timed on a bounded sample of the workload

Printed JSON line:
  value          FP64 sigma-build complex TFLOP/s over the timed steps
                 (algorithmic flops, 8 per complex multiply-add, / HIP-event
                 time of the sigma builds)
  ms_per_step    wall time of one step (three sigma builds)
  roofline       the dominant FP64 sigma kernel (the Y-build): algorithmic
                 flops per launch / mean launch time, against the FP64 matrix
                 peak, with its hardware-counter HBM traffic per launch
  sigma          per form: time, complex TFLOP/s, roofline record, per-kernel
                 times
Other workloads: pipeline (the whole path at one configuration), batch,
fd, peaks, transition.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sigma-build complex TFLOP/s and time-to-N-roots, mixed vs FP64, 1 MI355X"
PEAK_FP64_MFMA = 78.6      # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32_MFMA = 157.3     # TFLOP/s, MI355X dense FP32 matrix
# split-BF16: 2.5 PFLOP/s dense BF16, 3 real products per split real product -> 8/24 of it in
# algorithmic complex flops (8 per complex multiply-add)
PEAK_BF16X3 = 2500.0 * 8.0 / 24.0
HARTREE_EV = 27.211386245988
# hardware-counter traffic of the heavy sigma kernels, per configuration profiled
TRAFFIC_FILES = {"c3": os.path.join(ROOT, "profiles", "traffic_c3.json")}
CSRC = "paper_2604_27451_amd/csrc"
# sources that define each heavy sigma kernel: its GEMM engine header(s) and its own definition
KERNEL_DEFS = {("fp64", "ybuild"): (["zgemm.h", "tile.h"], "k_ygemm_wide("),
               ("fp64", "sigma2"): (["zgemm.h", "tile.h"], "k_zsig2_wide("),
               ("c64", "ybuild"): (["zgemm32.h", "zgemm.h"], "k_ygemm_c64("),
               ("c64", "sigma2"): (["zgemm32.h", "zgemm.h"], "k_zsig2_c64("),
               ("bf16x3", "ybuild"): (["zgemmb.h", "zgemm.h"], "k_ygemm_b3("),
               ("bf16x3", "sigma2"): (["zgemmb.h", "zgemm.h"], "k_zsig2_b3(")}


def _definition(text: str, name: str) -> str:
    """Source text of the kernel whose declarator contains `name`: from the
    line that starts its declaration (with a template line above it) to the
    closing brace in column 0."""
    i = text.index("void " + name)
    start = text.rfind("\n", 0, i) + 1
    prev = text.rfind("\n", 0, start - 1) + 1
    if text[prev:start].startswith("template"):
        start = prev
    end = text.index("\n}\n", i) + 3
    return text[start:end]


def kernel_hash(prec: str, kernel: str) -> str:
    """Hash of the sources of one heavy sigma kernel: hardware counters taken
    on it stay valid exactly while this is unchanged."""
    files, name = KERNEL_DEFS[(prec, kernel)]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, CSRC, "k_sigma.hip")) as fh:
        h.update(_definition(fh.read(), name).encode())
    return h.hexdigest()[:16]


def f_sigma(nc, no, nv, naux):
    """Algorithmic flops of one sigma vector (8 per complex multiply-add)."""
    return 8.0 * (2.0 * nc * no * nv * nv * naux + 2.0 * nc * nv * nv * naux + (nc * nv) ** 2)


def host_info():
    """The host the CPU baseline runs on: core count, CPU model, BLAS of the
    libraries the oracle calls (torch for its contractions, numpy beside it)."""
    import platform
    import subprocess
    import numpy as np
    import torch
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    torch_blas = None
    for tok in torch.__config__.show().replace(",", " ").split():
        if tok.startswith("BLAS_INFO="):
            torch_blas = tok.split("=", 1)[1]
    np_blas = None
    try:
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        np_blas = f"{b.get('name')} {b.get('version', '')}".strip()
    except Exception:
        pass
    return {"os_cpu_count": os.cpu_count(), "cpu_model": model or platform.processor(),
            "torch_threads": torch.get_num_threads(), "torch_blas": torch_blas, "numpy_blas": np_blas}


def cpu_baseline(L, eps, nc, no, nv, naux, nj: int, nvs: int):
    """The CPU oracle, as it stands, on a bounded sample of the same workload:
    the sigma build (integral blocks + product) for one vector of the system
    restricted to its first nj valence and first nvs virtual spinors (every
    Cholesky vector kept).  L, eps may be host arrays or device tensors."""
    import numpy as np
    import torch
    from oracle import adc2 as O
    from synth import random_vectors
    idx = np.r_[0:nc, nc:nc + nj, nc + no:nc + no + nvs]
    if isinstance(L, torch.Tensor):
        it = torch.as_tensor(idx, device=L.device)
        Ls = np.concatenate([L[p0:p0 + 250][:, it][:, :, it].cpu().numpy() for p0 in range(0, naux, 250)])
        es = eps[it.to(eps.device)].cpu().numpy()
    else:
        Ls = np.ascontiguousarray(L[:, idx][:, :, idx])
        es = eps[idx]
    t0 = time.perf_counter()
    a = O.Adc2(Ls, es, nc, nj, nvs)
    a.sigma_op()
    t1 = time.perf_counter()
    x = torch.from_numpy(random_vectors(11, 1, a.dim))
    a.sigma(x)
    t2 = time.perf_counter()
    dt = t2 - t0
    fl = f_sigma(nc, nj, nvs, naux)
    hi = host_info()
    # value: a sigma build from the Cholesky vectors, as the GPU path does it on every call (it keeps
    # no three-virtual integrals); product_only: the same flops over the product with the oracle's
    # stored integral blocks alone (their construction amortised over many vectors)
    return {"value": fl / dt / 1e12, "unit": "complex TFLOP/s", "cores": hi["torch_threads"],
            "kind": "oracle",
            "sample": f"oracle sigma (integral blocks {t1 - t0:.2f} s + product {t2 - t1:.2f} s) for 1 vector of "
                      f"the same system restricted to its first {nj} valence and first {nvs} virtual spinors "
                      f"(nc={nc}, no={nj}, nv={nvs}, naux={naux}); {dt:.2f} s for {fl:.3e} algorithmic flops",
            "seconds": dt, "integral_seconds": t1 - t0, "product_seconds": t2 - t1,
            "product_only_value": fl / max(1e-9, t2 - t1) / 1e12, "host": hi}


def load_traffic(prec, config="c2"):
    """Calibrated HBM bytes per launch of the heavy sigma kernels (m = 10
    vectors) from the committed hardware-counter profile of the
    configuration, for the kernels whose sources are unchanged since."""
    if config not in TRAFFIC_FILES:
        return {}
    try:
        tr = json.load(open(TRAFFIC_FILES[config]))
    except (OSError, ValueError):
        return {}
    out = {}
    for kern, rec in tr.get("kernels", {}).get(prec, {}).items():
        if (prec, kern) in KERNEL_DEFS and rec.get("hash") == kernel_hash(prec, kern):
            out[kern] = rec["bytes_per_launch"]
    return out


def roofline_of(stats, peak, traffic, every_launch_m10=False):
    dom = max(stats, key=lambda k: stats[k]["ms"])
    d = stats[dom]
    # the counter profile is per launch of m = 10 vectors; in the folded solver every Y-build
    # launch has m = nroots = 10, the sigma2 launches have as many vectors as new directions
    tb = traffic.get(dom) if (dom == "ybuild" or every_launch_m10) else None
    per_flops = d["flops"] / max(1, d["launches"])
    per_ms = d["ms"] / max(1, d["launches"])
    achieved = per_flops / (per_ms * 1e-3) / 1e12 if per_ms > 0 else 0.0
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": tb,
            "kernel": dom, "launches": d["launches"], "ms_per_launch": round(per_ms, 3),
            "flops_per_launch": per_flops}


# published MI355X figures next to which the probes are reported
DATASHEET = {"mfma_f64": (78.6, "TFLOP/s"), "mfma_f32": (157.3, "TFLOP/s"), "mfma_bf16": (2500.0, "TFLOP/s"),
             "valu_f64": (78.6, "TFLOP/s"), "hbm_read": (8000.0, "GB/s"), "hbm_copy": (8000.0, "GB/s"),
             "mfma_f64_rand": (78.6, "TFLOP/s"), "mfma_bf16_rand": (2500.0, "TFLOP/s")}


def measure_peaks(A, names, reps=5, nbytes=8 << 30):
    """Rates of the adc2_peak_probe microbenchmarks, with the datasheet value."""
    kinds = {"mfma_f64": A.ADC2_PEAK_MFMA_F64, "mfma_f32": A.ADC2_PEAK_MFMA_F32,
             "mfma_bf16": A.ADC2_PEAK_MFMA_BF16, "valu_f64": A.ADC2_PEAK_VALU_F64,
             "hbm_read": A.ADC2_PEAK_HBM_READ, "hbm_copy": A.ADC2_PEAK_HBM_COPY,
             "mfma_f64_rand": A.ADC2_PEAK_MFMA_F64_RAND, "mfma_bf16_rand": A.ADC2_PEAK_MFMA_BF16_RAND}
    out = {}
    for n in names:
        v = A.adc2_peak_probe(kinds[n], nbytes if n.startswith("hbm") else 0, reps)
        ds, unit = DATASHEET[n]
        out[n] = {"measured": round(v, 2), "datasheet": ds, "unit": unit, "frac_of_datasheet": round(v / ds, 4)}
        print(f"[bench] peak {n}: {v:.1f} {unit} (datasheet {ds:g})", file=sys.stderr, flush=True)
    return out


def with_measured_peak(roof, measured):
    """Adds the probe-measured peak (and the fraction of it) to a roofline record."""
    roof = dict(roof)
    roof["peak_measured"] = round(measured, 2)
    roof["frac_of_measured"] = round(roof["achieved"] / measured, 4) if measured > 0 else None
    return roof


def run_transition(args, A, np, torch):
    """Transition dipole moments and oscillator strengths of the FP64 roots of
    the configuration, with synthetic dipole integrals: F through first order
    and the singles through second order, each timed after a warm-up."""
    from synth import CONFIGS, config_system, dipole_integrals
    s = config_system(args.config)
    nroots = args.nroots or CONFIGS[args.config]["nroots"]
    L, e = torch.from_numpy(s.L).cuda(), torch.from_numpy(s.eps).cuda()
    dip = torch.from_numpy(dipole_integrals(27451, s.nc + s.no + s.nv)).cuda()
    h = A.adc2_setup(L, e, s.nc, s.no, s.nv, s.naux)
    w, X, inf = A.adc2_davidson(h, nroots, tol=args.tol, solver=A.ADC2_SOLVER_FOLDED)
    A.adc2_transition(h, dip, X[:1], w[:1], order=1)          # warm-up (first-call costs)
    out = {}
    for order in (1, 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T, f = A.adc2_transition(h, dip, X, w, order=order)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[order] = (dt, T, f)
        print(f"[bench] transition moments of {nroots} roots, order {order}: {dt:.3f}s", file=sys.stderr,
              flush=True)
    dt, T, f = out[2]
    print(json.dumps({"metric": "transition moments and oscillator strengths, time", "value": round(dt, 4),
                      "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"CVS-ADC(2) {args.config}: nc={s.nc} no={s.no} nv={s.nv} "
                                             f"naux={s.naux}, {nroots} FP64 roots, singles of F through second "
                                             "order, 3 dipole components"},
                      "first_order_s": round(out[1][0], 4),
                      "omega_ha": list(w), "oscillator_strengths": [float(x) for x in f],
                      "oscillator_strengths_first_order": [float(x) for x in out[1][2]],
                      "abs_T": [[float(abs(t)) for t in row] for row in T]}), flush=True)
    h.close()


def run_peaks(args, A):
    """Microbenchmarks of the rates the rooflines are quoted against."""
    names = ["mfma_f64", "mfma_f32", "mfma_bf16", "valu_f64", "hbm_read", "hbm_copy", "mfma_f64_rand",
             "mfma_bf16_rand"]
    peaks = measure_peaks(A, names, reps=10)
    print(json.dumps({"metric": "measured device peaks (adc2_peak_probe), 1 MI355X", "n_gpus": 1,
                      "data": "synthetic", "config": {"workload": "peak microbenchmarks: dense MFMA "
                                                      "(FP64 16x16x4, FP32 16x16x4, BF16 16x16x32), FP64 FMA, "
                                                      "HBM read and copy over 8 GiB"},
                      "peaks": peaks}), flush=True)


def heuristic_ysplit(s, m):
    """The library's size rule for the Y-build K-split of a complex64 handle
    (used when no tuned choice is set): the count 1..8 whose 128x128 tiles
    fill whole rounds of the 512 workgroup slots best (two per CU), each
    further split charged 0.2%."""
    ytiles = -(-s.naux // 128) * -(-(m * s.nc * s.nv) // 128)
    best, ys = None, 1
    for c in range(1, 9):
        rounds = ytiles * c / 512
        cost = math.ceil(rounds) / rounds * (1.0 + 0.002 * (c - 1))
        if best is None or cost < best:
            best, ys = cost, c
    return ys


def run_batch(args, A, np, torch):
    """Batching form: the eight systems of the batch workload, 16 roots each,
    complex64 heavy contractions with the folded solver and an FP64 Rayleigh
    polish; batched (adc2_setup_batch + adc2_davidson_batch in both modes)
    and, for comparison, one system after the other."""
    from synth import batch_systems
    fold = A.ADC2_SOLVER_FOLDED
    nroots = args.nroots or 16
    tol = args.tol_batch
    verbose = 1 if args.verbose else 0
    t = time.time()
    systems = batch_systems(1.0)
    if args.batch_systems:
        systems = [systems[int(i)] for i in args.batch_systems.split(",")]
    data = [(torch.from_numpy(s.L).cuda(), torch.from_numpy(s.eps).cuda(), s.nc, s.no, s.nv, s.naux)
            for s in systems]
    torch.cuda.synchronize()
    print(f"[bench] generated batch of {len(systems)} in {time.time() - t:.1f}s", file=sys.stderr, flush=True)

    def polish(h, X):
        A.adc2_set_precision(h, A.ADC2_FP64)
        wp, rn = A.adc2_rayleigh(h, X)
        A.adc2_set_precision(h, A.ADC2_C64)
        return wp, rn

    # autotuner (untimed, one-time per shape): Y-build K-split of every system at m = nroots; later
    # calls on a handle of the same shape take the choice from the in-process cache
    tune = []
    if not args.no_autotune:
        for q, d in enumerate(data):
            h = A.adc2_setup(*d, prec=A.ADC2_C64)
            ta = time.perf_counter()
            r = A.adc2_autotune(h, nroots)
            r["s"] = round(time.perf_counter() - ta, 3)
            r["heuristic_ysplit"] = h_ysplit = heuristic_ysplit(systems[q], nroots)
            tune.append(r)
            h.close()
            print(f"[bench] tune system {q}: K-split {r['ysplit']} (heuristic {h_ysplit}), "
                  + ", ".join(f"{k}: {v:.2f} ms" for k, v in r["ms"].items()), file=sys.stderr, flush=True)

    def tuned(h):
        if not args.no_autotune:
            A.adc2_autotune(h, nroots)
        return h

    sig = batch_sigma_leg(A, torch, data, nroots, tuned, reps=args.batch_sigma_reps)
    if args.batch_sigma_only:
        print(json.dumps({"metric": "batched sigma of every system of the batch (m = " + str(nroots) + " each)",
                          "value": sig["graph_ms"], "unit": "ms", "n_gpus": 1, "higher_is_better": False,
                          "dtype": "c64 contractions", "data": "synthetic",
                          "config": {"workload": "batching form: " + str(len(systems)) + " systems, nc=6, "
                                     "(no, nv) = " + ", ".join(f"({s.no},{s.nv})" for s in systems) +
                                     ", naux = 4 nv"},
                          "sigma_launch": sig}), flush=True)
        return
    # warm-up (untimed): one solve of the smallest system, so that no timed leg pays first-call costs
    qmin = min(range(len(data)), key=lambda q: systems[q].no * systems[q].nv ** 2)
    h = tuned(A.adc2_setup(*data[qmin], prec=A.ADC2_C64))
    A.adc2_davidson(h, nroots, tol=tol, solver=fold)
    torch.cuda.synchronize()
    h.close()
    # one after the other
    seq = []
    t4 = time.perf_counter()
    for q, d in enumerate(data):
        ta = time.perf_counter()
        h = tuned(A.adc2_setup(*d, prec=A.ADC2_C64))
        w, X, inf = A.adc2_davidson(h, nroots, tol=tol, solver=fold, verbose=verbose)
        wp, rn = polish(h, X)
        torch.cuda.synchronize()
        seq.append(dict(w=w, wp=wp, rn=rn, info=inf, s=time.perf_counter() - ta))
        h.close()
        del X
        print(f"[bench] system {q} alone: {seq[-1]['s']:.2f}s ({inf['iters']} it)", file=sys.stderr, flush=True)
    t5 = time.perf_counter()
    sequential_s = t5 - t4
    modes = {}
    for name, mode in (("rounds", A.ADC2_BATCH_ROUNDS), ("streams", A.ADC2_BATCH_STREAMS)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hs = [tuned(h) for h in A.adc2_setup_batch(data, A.ADC2_C64)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        print(f"[bench] {name}: setup {t1 - t0:.2f}s", file=sys.stderr, flush=True)
        wb, Xb, infb = A.adc2_davidson_batch(hs, nroots, tol=tol, solver=fold, verbose=verbose, mode=mode)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        pol = [polish(h, X) for h, X in zip(hs, Xb)]
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        print(f"[bench] {name}: solve {t2 - t1:.2f}s polish {t3 - t2:.2f}s", file=sys.stderr, flush=True)
        modes[name] = {
            "total_s": round(t3 - t0, 3), "setup_s": round(t1 - t0, 3), "solve_s": round(t2 - t1, 3),
            "polish_s": round(t3 - t2, 3), "iterations": [i["iters"] for i in infb],
            "speedup_vs_sequential": round(sequential_s / max(1e-9, t3 - t0), 3),
            "roots_equal_sequential": bool(all(wb[q] == seq[q]["w"] for q in range(len(data)))),
            "max_polished_resnorm": max(max(rn) for _, rn in pol),
            "max_polish_shift_ev": max(float(np.abs(np.array(wp) - np.array(w)).max()) * HARTREE_EV
                                       for (wp, _), w in zip(pol, wb)),
        }
        for h in hs:
            h.close()
        del Xb
    best = min(modes, key=lambda k: modes[k]["total_s"])
    out = {
        "metric": "time to 16 roots of every system of the batch (batching form)",
        "value": modes[best]["total_s"],
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "c64 contractions, f64 subspace",
        "data": "synthetic",
        "config": {"workload": "batching form: " + str(len(systems)) + " systems, nc=6, (no, nv) = " +
                               ", ".join(f"({s.no},{s.nv})" for s in systems) + ", naux = 4 nv, "
                               f"{nroots} roots each, folded solver, complex64 tolerance {tol:g}, FP64 polish"},
        "best_mode": best,
        "modes": modes,
        "sequential_s": round(sequential_s, 3),
        "sequential_per_system_s": [round(r["s"], 3) for r in seq],
        "sequential_iterations": [r["info"]["iters"] for r in seq],
        "omega_ha_polished": [list(r["wp"]) for r in seq],
        "sigma_launch": sig,
        "autotune": ({"m": nroots, "tune_s": round(sum(r["s"] for r in tune), 3),
                      "systems": [{"ysplit": r["ysplit"], "heuristic_ysplit": r["heuristic_ysplit"],
                                   "ms": {str(k): round(v, 3) for k, v in r["ms"].items()}} for r in tune]}
                     if tune else None),
    }
    print(json.dumps(out), flush=True)


def batch_sigma_leg(A, torch, data, m, tuned, reps=20):
    """One sigma product of m vectors for every system of the batch, timed
    three ways on torch's current stream (HIP events, mean over reps): one
    adc2_sigma per system, one adc2_sigma_batch (grouped heavy GEMMs), and the
    replay of that batched launch sequence captured as a HIP graph
    (adc2_graph_sigma_batch / adc2_graph_launch).  The replay's output is
    checked against the eager batched product."""
    hs = [tuned(h) for h in A.adc2_setup_batch(data, A.ADC2_C64)]
    g = torch.Generator(device="cpu").manual_seed(77)
    xs = [torch.randn(m, h.dim, dtype=torch.complex128, generator=g).cuda() for h in hs]
    ss = [torch.empty_like(x) for x in xs]
    graph = A.adc2_graph_sigma_batch(hs, xs)     # also the eager warm-up of every work space
    for h, x, s_ in zip(hs, xs, ss):
        A.adc2_sigma(h, x, s_)
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    sep = timed(lambda: [A.adc2_sigma(h, x, s_) for h, x, s_ in zip(hs, xs, ss)])
    bat = timed(lambda: A.adc2_sigma_batch(hs, xs, ss))
    rep = timed(graph.launch)
    eager = A.adc2_sigma_batch(hs, xs)
    graph.launch()
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(graph.S, eager))
    graph.close()
    for h in hs:
        h.close()
    out = {"m": m, "reps": reps, "separate_ms": round(sep, 3), "batched_ms": round(bat, 3),
           "graph_ms": round(rep, 3), "graph_equals_batched": bool(same)}
    print(f"[bench] batched sigma m={m}: separate {sep:.2f} ms, batched {bat:.2f} ms, graph replay {rep:.2f} ms "
          f"(equal {same})", file=sys.stderr, flush=True)
    return out


def run_fd(args, A, np, torch):
    """Differentiation form at the c2 shape: d omega_k / dL and d omega_k / d eps
    of the 10 lowest roots from the adjoint (adc2_omega_backward, one call per
    root) against central finite differences of the eigenvalues, h = 1e-5, on
    50 random Hermitian directions of L (unit Frobenius norm) and 10 random
    directions of eps.  Each perturbed solve is the FP64 folded solver warm-
    started from the unperturbed eigenvectors."""
    from synth import config_system, random_hermitian_direction_device
    fold = A.ADC2_SOLVER_FOLDED
    ndir, nedir, hstep = 50, 10, 1e-5
    sysm = config_system(args.config)
    nc, no, nv, naux = sysm.nc, sysm.no, sysm.nv, sysm.naux
    n = nc + no + nv
    L = torch.from_numpy(sysm.L).cuda()
    eps = torch.from_numpy(sysm.eps).cuda()
    nroots = args.nroots or 10
    tol = 1e-10
    t0 = time.perf_counter()
    h = A.adc2_setup(L, eps, nc, no, nv, naux)
    w0, X0, inf0 = A.adc2_davidson(h, nroots, tol=tol, solver=fold)
    print(f"[bench] fd: reference roots in {inf0['iters']} iterations", file=sys.stderr, flush=True)
    G, GE = [], []
    tb = time.perf_counter()
    for k in range(nroots):
        g = [0.0] * nroots
        g[k] = 1.0
        dL, de = A.adc2_omega_backward(h, X0, g)
        G.append(dL)
        GE.append(de)
    torch.cuda.synchronize()
    t_adj = (time.perf_counter() - tb) / nroots
    # complex64 leg: eigenvectors from the complex64 solve (tolerance 1e-5), the
    # same adjoint (FP64 arithmetic) on them, against the FP64 gradient
    A.adc2_set_precision(h, A.ADC2_C64)
    wc, Xc, infc = A.adc2_davidson(h, nroots, tol=1e-5, solver=fold)
    A.adc2_set_precision(h, A.ADC2_FP64)
    Gc, GEc = [], []
    for k in range(nroots):
        g = [0.0] * nroots
        g[k] = 1.0
        dL, de = A.adc2_omega_backward(h, Xc, g)
        Gc.append(dL)
        GEc.append(de)
    c64_rel = [float(torch.linalg.vector_norm(Gc[k] - G[k]) / torch.linalg.vector_norm(G[k])) for k in range(nroots)]
    c64_rel_e = [float(torch.linalg.vector_norm(GEc[k] - GE[k]) / torch.linalg.vector_norm(GE[k]))
                 for k in range(nroots)]
    print(f"[bench] fd: complex64 eigenvectors ({infc['iters']} it): gradient rel. dev. vs FP64 "
          f"L {max(c64_rel):.2e}, eps {max(c64_rel_e):.2e}", file=sys.stderr, flush=True)
    del Xc
    h.close()

    def roots_at(Lp, ep):
        hp = A.adc2_setup(Lp, ep, nc, no, nv, naux)
        w, _, inf = A.adc2_davidson(hp, nroots, tol=tol, solver=fold, guess=X0, nguess=nroots, want_vectors=False)
        hp.close()
        return np.array(w), inf["iters"]

    rows, rows_c, iters = [], [], []
    for d in range(ndir + nedir):
        if d < ndir:
            dL = random_hermitian_direction_device(27451 + 5000 + d, naux, n)
            wp, ip = roots_at(L + hstep * dL, eps)
            wm, im_ = roots_at(L - hstep * dL, eps)
            ad = np.array([float(torch.sum(torch.conj(G[k]) * dL).real) for k in range(nroots)])
            adc = np.array([float(torch.sum(torch.conj(Gc[k]) * dL).real) for k in range(nroots)])
            del dL
        else:
            gen = torch.Generator(device="cuda")
            gen.manual_seed(27451 + 6000 + d)
            de = torch.randn(n, generator=gen, device="cuda", dtype=torch.float64)
            de = de / torch.linalg.vector_norm(de)
            wp, ip = roots_at(L, eps + hstep * de)
            wm, im_ = roots_at(L, eps - hstep * de)
            ad = np.array([float(torch.dot(GE[k], de)) for k in range(nroots)])
            adc = np.array([float(torch.dot(GEc[k], de)) for k in range(nroots)])
        fd = (wp - wm) / (2 * hstep)
        rows.append((d < ndir, fd, ad))
        rows_c.append((d < ndir, fd, adc))
        iters += [ip, im_]
        err = np.abs(fd - ad).max() / max(1e-300, np.abs(ad).max())
        print(f"[bench] fd direction {d} ({'L' if d < ndir else 'eps'}): max rel dev {err:.2e} "
              f"(|d omega| max {np.abs(ad).max():.3e})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    def stats(is_l, rows=rows):
        sel = [(fd, ad) for l, fd, ad in rows if l == is_l]
        dev = [float(np.abs(fd - ad).max() / np.abs(ad).max()) for fd, ad in sel]
        absd = [float(np.abs(fd - ad).max()) for fd, ad in sel]
        return {"directions": len(sel), "max_rel_dev": max(dev), "median_rel_dev": float(np.median(dev)),
                "max_abs_dev_ha": max(absd)}

    out = {
        "metric": "adjoint d omega/dL, d omega/d eps vs central finite differences (differentiation form)",
        "value": stats(True)["max_rel_dev"],
        "unit": "max relative deviation",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"CVS-ADC(2) {args.config}: nc={nc} no={no} nv={nv} naux={naux}, {nroots} roots, "
                               f"{ndir} Hermitian L directions + {nedir} eps directions (unit norm), h = {hstep:g}, "
                               "FP64 folded solves warm-started, tolerance 1e-10"},
        "L_directions": stats(True),
        "eps_directions": stats(False),
        "adjoint_s_per_root": round(t_adj, 3),
        "perturbed_solve_iterations": {"min": int(min(iters)), "max": int(max(iters))},
        "complex64": {"eigenvectors": "complex64 folded solve, tolerance 1e-5; adjoint in FP64 arithmetic",
                      "iterations": infc["iters"],
                      "max_rel_dev_vs_fp64_gradient_L": max(c64_rel),
                      "max_rel_dev_vs_fp64_gradient_eps": max(c64_rel_e),
                      "L_directions": stats(True, rows_c), "eps_directions": stats(False, rows_c)},
        "wall_s": round(time.perf_counter() - t0, 1),
    }
    print(json.dumps(out), flush=True)


def run_pipeline(args, A, np, torch, config=None, peaks=True, with_cpu=True):
    """The whole hot path of one configuration as one step: setup, FP64
    folded solve, adjoint, two-stage FP64 solve through split-BF16, split-BF16
    and complex64 solves with FP64 polish.  Returns the JSON record."""
    from synth import CONFIGS, config_inputs_device
    config = config or args.config
    cfg = CONFIGS[config]
    nroots = args.nroots or cfg["nroots"]
    solver = A.ADC2_SOLVER_FOLDED if args.solver == "folded" else A.ADC2_SOLVER_FULL
    t = time.time()
    L, eps = config_inputs_device(config)
    print(f"[bench] generated {config} on the device in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    nc, no, nv, naux = cfg["nc"], cfg["no"], cfg["nv"], cfg["naux"]

    if args.sigma_probe:
        from synth import random_vectors
        h = A.adc2_setup(L, eps, nc, no, nv, naux)
        x = torch.from_numpy(random_vectors(1, 10, h.dim)).cuda()
        S = torch.empty_like(x)
        for prec in (A.ADC2_FP64, A.ADC2_C64, A.ADC2_BF16X3):
            A.adc2_set_precision(h, prec)
            for _ in range(3):
                A.adc2_sigma(h, x, S)
        torch.cuda.synchronize()
        src = torch.ones(2 ** 31 // 8, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        dst = src + 1.0          # calibration: reads 2 GiB, writes 2 GiB
        torch.cuda.synchronize()
        print(f"[bench] sigma probe done ({float(dst[5]):.1f})", file=sys.stderr, flush=True)
        return

    def solve(h, tol):
        A.adc2_profile(h, True)
        w, X, info = A.adc2_davidson(h, nroots, tol=tol, max_iter=args.max_iter, solver=solver,
                                     max_subspace=args.max_subspace, nguess=args.nguess,
                                     verbose=1 if args.verbose else 0, raise_on_noconv=False)
        torch.cuda.synchronize()
        return w, X, info, A.adc2_kernel_stats(h)

    def step(i, timed):
        r = {}
        t0 = time.perf_counter()
        h = A.adc2_setup(L, eps, nc, no, nv, naux)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        w64, X64, info64, ks64 = solve(h, args.tol)
        t2 = time.perf_counter()
        r.update(setup_s=t1 - t0, fp64_solve_s=t2 - t1, w64=w64, info64=info64, ks64=ks64,
                 emp2=A.adc2_mp2_energy(h))
        if not args.no_adjoint:
            dL, de = A.adc2_omega_backward(h, X64, [1.0] * nroots)
            torch.cuda.synchronize()
            r["adjoint_s"] = time.perf_counter() - t2
            r["adjoint_norm"] = float(torch.linalg.vector_norm(dL))
            del dL, de
        del X64
        if not args.no_mixed:
            legs = [("b3", A.ADC2_BF16X3, args.tol_mixed)] + ([] if args.no_c64 else [("c64", A.ADC2_C64, args.tol_c64)])
            for tag, prec, tol in legs:
                t3 = time.perf_counter()
                A.adc2_set_precision(h, prec)
                wm, Xm, infom, ksm = solve(h, tol)
                t4 = time.perf_counter()
                A.adc2_set_precision(h, A.ADC2_FP64)
                wp, rn = A.adc2_rayleigh(h, Xm)
                torch.cuda.synchronize()
                t5 = time.perf_counter()
                r[tag] = dict(solve_s=t4 - t3, polish_s=t5 - t4, w=wm, wp=wp, rn_polish=rn, info=infom, ks=ksm)
                del Xm
            if not args.no_refined:
                # FP64 roots through the precision form: split-BF16 solve to tol_refine, then the
                # FP64 folded solve to the FP64 tolerance started from those vectors
                # (the library's two-stage solve: adc2_dav_opts.mixed_tol)
                A.adc2_set_precision(h, A.ADC2_FP64)
                t6 = time.perf_counter()
                wr, Xr, infr = A.adc2_davidson(h, nroots, tol=args.tol, max_iter=args.max_iter, solver=solver,
                                               max_subspace=args.max_subspace, nguess=args.nguess,
                                               mixed_tol=args.tol_refine, raise_on_noconv=False)
                torch.cuda.synchronize()
                t8 = time.perf_counter()
                r["refined"] = dict(solve_s=t8 - t6, w=wr, iters=infr["iters"], converged=infr["converged"],
                                    max_resnorm=max(infr["resnorm"]), ms_sigma=infr["ms_sigma"])
                del Xr
        h.close()
        r["wall_s"] = time.perf_counter() - t0
        msg = (f"[bench] step {i} ({'timed' if timed else 'warmup'}): setup {r['setup_s']:.3f}s "
               f"fp64 {r['fp64_solve_s']:.2f}s ({info64['iters']} it, max|r| {max(info64['resnorm']):.1e})")
        if "adjoint_s" in r:
            msg += f" adjoint {r['adjoint_s']:.2f}s"
        if "refined" in r:
            m = r["refined"]
            msg += (f" fp64-via-b3 {m['solve_s']:.2f}s ({m['iters']} it, max|dw| "
                    f"{np.abs(np.array(m['w']) - np.array(w64)).max():.1e} Ha)")
        for tag in ("b3", "c64"):
            if tag in r:
                m = r[tag]
                msg += (f" {tag} {m['solve_s']:.2f}s ({m['info']['iters']} it) polish {m['polish_s']:.2f}s "
                        f"max|dw| {np.abs(np.array(m['w']) - np.array(w64)).max() * HARTREE_EV:.1e} eV")
        print(msg, file=sys.stderr, flush=True)
        return r

    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    res = [step(i, True) for i in range(args.steps)]
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start

    def agg_stats(key):
        agg = {}
        for r in res:
            for k, v in r[key].items():
                if v["launches"] == 0:
                    continue
                a = agg.setdefault(k, {"launches": 0, "ms": 0.0, "flops": 0.0})
                for f in a:
                    a[f] += v[f]
        return agg

    def tflops(infos):
        fl = sum(i["sigma_flops"] for i in infos)
        ms = sum(i["ms_sigma"] for i in infos)
        return fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0

    agg64 = agg_stats("ks64")
    value = tflops([r["info64"] for r in res])
    roofline = roofline_of(agg64, PEAK_FP64_MFMA, load_traffic("fp64", config))
    last = res[-1]
    w64 = np.array(last["w64"])
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "complex TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_total / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"CVS-ADC(2) {config}: nc={nc} no={no} nv={nv} naux={naux} complex128, "
                               f"{nroots} roots, {args.solver} solver, FP64 tol {args.tol:g}",
                   "nc": nc, "no": no, "nv": nv, "naux": naux, "nroots": nroots,
                   "dim": nc * nv + nc * no * nv * (nv - 1) // 2, "solver": args.solver},
        "time_to_roots_s": round(float(np.mean([r["setup_s"] + r["fp64_solve_s"] for r in res])), 3),
        "setup_s": round(float(np.mean([r["setup_s"] for r in res])), 4),
        "iterations": last["info64"]["iters"],
        "sigma_vectors": last["info64"]["n_sigma"],
        "converged": last["info64"]["converged"],
        "max_resnorm": max(last["info64"]["resnorm"]),
        "omega_ha": last["w64"],
        "e_mp2_ha": last["emp2"],
        "sigma_ms_share": round(sum(r["info64"]["ms_sigma"] for r in res) /
                                (1e3 * sum(r["fp64_solve_s"] for r in res)), 4),
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 2),
                        "tflops": round(v["flops"] / max(1e-9, v["ms"] * 1e-3) / 1e12, 3)}
                    for k, v in agg64.items()},
        "roofline": roofline,
    }
    if "adjoint_s" in last:
        out["adjoint_s"] = round(float(np.mean([r["adjoint_s"] for r in res])), 3)
    def mixed_block(tag, dtype, peak):
        agg = {}
        for r in res:
            for k, v in r[tag]["ks"].items():
                if v["launches"] == 0:
                    continue
                a = agg.setdefault(k, {"launches": 0, "ms": 0.0, "flops": 0.0})
                for f in a:
                    a[f] += v[f]
        m = last[tag]
        wm, wp = np.array(m["w"]), np.array(m["wp"])
        return {
            "dtype": dtype,
            "sigma_tflops": round(tflops([r[tag]["info"] for r in res]), 4),
            "time_to_roots_s": round(float(np.mean([r["setup_s"] + r[tag]["solve_s"] + r[tag]["polish_s"]
                                                    for r in res])), 3),
            "solve_s": round(float(np.mean([r[tag]["solve_s"] for r in res])), 3),
            "polish_s": round(float(np.mean([r[tag]["polish_s"] for r in res])), 3),
            "iterations": m["info"]["iters"],
            "converged": m["info"]["converged"],
            "max_resnorm": max(m["info"]["resnorm"]),
            "ev_err_raw": [float(x) for x in (wm - w64) * HARTREE_EV],
            "ev_err_polished": [float(x) for x in (wp - w64) * HARTREE_EV],
            "polished_resnorm": [float(x) for x in m["rn_polish"]],
            "roofline": roofline_of(agg, peak, load_traffic({"b3": "bf16x3"}.get(tag, tag), config)),
            "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 2),
                            "tflops": round(v["flops"] / max(1e-9, v["ms"] * 1e-3) / 1e12, 3)}
                        for k, v in agg.items()},
        }

    if "b3" in last:
        out["mixed"] = mixed_block("b3", "split-BF16 operands (hi + lo), BF16 MFMA, FP32 accumulation; "
                                         "FP64 setup, denominators and subspace; tolerance "
                                         f"{args.tol_mixed:g}", PEAK_BF16X3)
        out["mixed"]["tol"] = args.tol_mixed
    if "refined" in last:
        m = last["refined"]
        t_ref = float(np.mean([r["setup_s"] + r["refined"]["solve_s"] for r in res]))
        out["fp64_via_mixed"] = {
            "what": f"two-stage solve (adc2_dav_opts.mixed_tol = {args.tol_refine:g}): split-BF16 folded solve to "
                    f"{args.tol_refine:g}, then the FP64 folded solve to {args.tol:g} started from its vectors",
            "time_to_roots_s": round(t_ref, 3),
            "solve_s": round(float(np.mean([r["refined"]["solve_s"] for r in res])), 3),
            "iterations": m["iters"], "converged": m["converged"], "max_resnorm": m["max_resnorm"],
            "max_abs_dev_from_fp64_roots_ha": float(np.abs(np.array(m["w"]) - w64).max()),
            "speedup_vs_fp64": round(out["time_to_roots_s"] / max(1e-9, t_ref), 3),
        }
    if "c64" in last:
        out["mixed_c64"] = mixed_block("c64", "complex64 operands, FP32 MFMA accumulation; FP64 setup, "
                                              f"denominators and subspace; tolerance {args.tol_c64:g}",
                                       PEAK_FP32_MFMA)
        out["mixed_c64"]["tol"] = args.tol_c64
    # measured MFMA rates beside the published peaks (outside the timed steps)
    if not peaks:
        out["cpu_baseline"] = None
        return out
    pk = measure_peaks(A, ["mfma_f64", "mfma_f64_rand"] +
                       (["mfma_bf16", "mfma_bf16_rand"] if "mixed" in out else []) +
                       (["mfma_f32"] if "mixed_c64" in out else []))
    out["roofline"] = with_measured_peak(out["roofline"], pk["mfma_f64"]["measured"])
    out["roofline"]["peak_measured_random_operands"] = pk["mfma_f64_rand"]["measured"]
    if "mixed" in out:
        out["mixed"]["roofline"] = with_measured_peak(out["mixed"]["roofline"],
                                                      pk["mfma_bf16"]["measured"] * 8.0 / 24.0)
        # the same instruction on data-like operands: the rate the power limit allows
        rnd = pk["mfma_bf16_rand"]["measured"] * 8.0 / 24.0
        out["mixed"]["roofline"]["peak_measured_random_operands"] = round(rnd, 2)
        out["mixed"]["roofline"]["frac_of_random_operands"] = round(out["mixed"]["roofline"]["achieved"] / rnd, 4)
    if "mixed_c64" in out:
        out["mixed_c64"]["roofline"] = with_measured_peak(out["mixed_c64"]["roofline"], pk["mfma_f32"]["measured"])
    cpu = None
    if with_cpu and not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(L, eps, nc, no, nv, naux, 8, nv)
    out["cpu_baseline"] = cpu
    return out


FORMS = (("fp64", "ADC2_FP64", PEAK_FP64_MFMA, "complex128 operands, FP64 MFMA"),
         ("c64", "ADC2_C64", PEAK_FP32_MFMA, "complex64 operands, FP32 MFMA, FP32 accumulation"),
         ("bf16x3", "ADC2_BF16X3", PEAK_BF16X3,
          "split-BF16 operands (hi + lo of each complex64 part), BF16 MFMA, FP32 accumulation"))


def agg_kernel_stats(records):
    agg = {}
    for ks in records:
        for k, v in ks.items():
            if v["launches"] == 0:
                continue
            a = agg.setdefault(k, {"launches": 0, "ms": 0.0, "flops": 0.0})
            for f in a:
                a[f] += v[f]
    return agg


def oracle_leg_c1(A, np, torch, tol_mixed):
    """Roots at c1 against the oracle itself: the oracle's Davidson (FP64,
    CPU) beside the GPU's FP64 and split-BF16 folded solves."""
    from oracle import adc2 as O
    from synth import CONFIGS, config_system
    c = CONFIGS["c1"]
    s = config_system("c1")
    k = c["nroots"]
    t0 = time.perf_counter()
    w_or, _, inf = O.Adc2(s.L, s.eps, s.nc, s.no, s.nv).roots(k, tol=1e-9, max_iter=400)
    t_or = time.perf_counter() - t0
    h = A.adc2_setup(torch.from_numpy(s.L).cuda(), torch.from_numpy(s.eps).cuda(), s.nc, s.no, s.nv, s.naux)
    w64, _, _ = A.adc2_davidson(h, k, tol=1e-9, solver=A.ADC2_SOLVER_FOLDED)
    A.adc2_set_precision(h, A.ADC2_BF16X3)
    wb, Xb, infb = A.adc2_davidson(h, k, tol=tol_mixed, solver=A.ADC2_SOLVER_FOLDED)
    A.adc2_set_precision(h, A.ADC2_FP64)
    wp, _ = A.adc2_rayleigh(h, Xb)
    h.close()
    wo = w_or.numpy()
    return {"workload": f"c1: nc={s.nc} no={s.no} nv={s.nv} naux={s.naux}, {k} roots; oracle Davidson to 1e-9 "
                        f"(converged {inf['converged']}, {t_or:.1f} s on the host)",
            "fp64_abs_err_ha": [float(x) for x in np.array(w64) - wo],
            "bf16x3_ev_err_raw": [float(x) for x in (np.array(wb) - wo) * HARTREE_EV],
            "bf16x3_ev_err_polished": [float(x) for x in (np.array(wp) - wo) * HARTREE_EV],
            "bf16x3_tol": tol_mixed}


def run_headline(args, A, np, torch):
    """The benchmark line: on the heavy-element-complex configuration (c3:
    nc=6, no=120, nv=600, naux=3000, inputs resident in HBM) one step is one
    sigma build of a block of 10 vectors in each of the three forms (FP64,
    complex64, split-BF16), timed with HIP events on the launch stream; setup
    (blocks, MP2, singles block, operand copies of both precision forms) is
    outside the steps.  After the timed steps, once each: FP64 roots through
    the precision form (two-stage solve) and split-BF16 roots with the FP64
    polish, each from a fresh setup, with the per-root eV error; the roots at
    c1 against the oracle itself; the whole path at c2; the CPU baseline."""
    import argparse as _ap
    from synth import CONFIGS, config_inputs_device
    cfg = CONFIGS[args.config]
    nc, no, nv, naux = cfg["nc"], cfg["no"], cfg["nv"], cfg["naux"]
    nroots = args.nroots or cfg["nroots"]
    m = nroots
    fold = A.ADC2_SOLVER_FOLDED
    t = time.time()
    L, eps = config_inputs_device(args.config)
    print(f"[bench] generated {args.config} on the device in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    dim = nc * nv + nc * no * nv * (nv - 1) // 2
    if args.sigma_probe:
        h = A.adc2_setup(L, eps, nc, no, nv, naux)
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        X = torch.complex(torch.randn((m, dim), generator=g, device="cuda", dtype=torch.float64),
                          torch.randn((m, dim), generator=g, device="cuda", dtype=torch.float64))
        S = torch.empty_like(X)
        for prec in (A.ADC2_FP64, A.ADC2_C64, A.ADC2_BF16X3):
            A.adc2_set_precision(h, prec)
            for _ in range(3):
                A.adc2_sigma(h, X, S)
        torch.cuda.synchronize()
        src = torch.ones(2 ** 31 // 8, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        dst = src + 1.0          # calibration: reads 2 GiB, writes 2 GiB
        torch.cuda.synchronize()
        print(f"[bench] sigma probe done ({float(dst[5]):.1f})", file=sys.stderr, flush=True)
        return
    t0 = time.perf_counter()
    h = A.adc2_setup(L, eps, nc, no, nv, naux)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    g = torch.Generator(device="cuda")
    g.manual_seed(27451)
    X = torch.complex(torch.randn((m, dim), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((m, dim), generator=g, device="cuda", dtype=torch.float64)) * (0.5 ** 0.5)
    S = torch.empty_like(X)
    for _, prec, _, _ in FORMS:          # operand copies and work spaces of every form (setup, untimed)
        A.adc2_set_precision(h, getattr(A, prec))
        A.adc2_sigma(h, X, S)
    torch.cuda.synchronize()
    print(f"[bench] setup {setup_s:.2f}s, operand copies built", file=sys.stderr, flush=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    rec = {f[0]: {"ms": [], "ks": []} for f in FORMS}

    def step(i, timed):
        line = []
        for tag, prec, _, _ in FORMS:
            A.adc2_set_precision(h, getattr(A, prec))
            A.adc2_profile(h, True)
            e0.record()
            A.adc2_sigma(h, X, S)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            ks = A.adc2_kernel_stats(h)
            A.adc2_profile(h, False)
            if timed:
                rec[tag]["ms"].append(ms)
                rec[tag]["ks"].append(ks)
            line.append(f"{tag} {ms:.1f} ms")
        print(f"[bench] step {i} ({'timed' if timed else 'warmup'}): " + ", ".join(line), file=sys.stderr,
              flush=True)

    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(i, True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    A.adc2_set_precision(h, A.ADC2_FP64)
    del X, S
    h.close()
    torch.cuda.empty_cache()

    fl = f_sigma(nc, no, nv, naux) * m
    sig = {}
    for tag, prec, peak, what in FORMS:
        ms = float(np.mean(rec[tag]["ms"]))
        agg = agg_kernel_stats(rec[tag]["ks"])
        sig[tag] = {"what": what, "ms_per_sigma": round(ms, 3), "tflops": round(fl / (ms * 1e-3) / 1e12, 3),
                    "frac_of_peak": round(fl / (ms * 1e-3) / 1e12 / peak, 4),
                    "roofline": roofline_of(agg, peak, load_traffic(tag, args.config), every_launch_m10=True),
                    "kernels": {k: {"launches": v["launches"], "ms_per_launch": round(v["ms"] / v["launches"], 3),
                                    "tflops": round(v["flops"] / max(1e-9, v["ms"] * 1e-3) / 1e12, 3)}
                                for k, v in agg.items()}}
    pk = measure_peaks(A, ["mfma_f64", "mfma_f64_rand", "mfma_f32", "mfma_bf16", "mfma_bf16_rand"])
    sig["fp64"]["roofline"] = with_measured_peak(sig["fp64"]["roofline"], pk["mfma_f64"]["measured"])
    sig["c64"]["roofline"] = with_measured_peak(sig["c64"]["roofline"], pk["mfma_f32"]["measured"])
    sig["bf16x3"]["roofline"] = with_measured_peak(sig["bf16x3"]["roofline"], pk["mfma_bf16"]["measured"] * 8 / 24)
    rnd = pk["mfma_bf16_rand"]["measured"] * 8.0 / 24.0
    sig["bf16x3"]["roofline"]["peak_measured_random_operands"] = round(rnd, 2)
    sig["bf16x3"]["roofline"]["frac_of_random_operands"] = round(sig["bf16x3"]["roofline"]["achieved"] / rnd, 4)

    # ---- time to roots (outside the timed steps), each from a fresh setup ----
    # The handle keeps its own blocks of L, so the input is released after
    # each setup (the solve's search space needs the room) and uploaded again
    # from a pinned host copy, untimed, before the next leg.
    kw = dict(max_iter=args.max_iter, solver=fold, max_subspace=args.max_subspace,
              nguess=args.nguess or nroots, raise_on_noconv=False, verbose=1 if args.verbose else 0)
    Lhost = torch.empty(L.shape, dtype=L.dtype, pin_memory=True)
    Lhost.copy_(L)
    torch.cuda.synchronize()
    state = {"L": L}
    del L

    def setup_then_release(prec=A.ADC2_FP64):
        h_ = A.adc2_setup(state["L"], eps, nc, no, nv, naux, prec=prec)
        state["L"] = None
        torch.cuda.empty_cache()
        return h_

    def reload():
        if state["L"] is None:
            state["L"] = Lhost.cuda()
            torch.cuda.synchronize()

    roots = {}
    if not args.no_refined:
        reload()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = setup_then_release()
        wr, Xr, infr = A.adc2_davidson(h, nroots, tol=args.tol, mixed_tol=args.tol_refine, **kw)
        torch.cuda.synchronize()
        roots["fp64_via_bf16x3"] = {
            "what": f"FP64 roots through the precision form: adc2_davidson with mixed_tol = {args.tol_refine:g} "
                    f"(split-BF16 folded solve to {args.tol_refine:g}, then the FP64 folded solve to {args.tol:g} "
                    "from its vectors), from adc2_setup to the roots on the host",
            "time_to_roots_s": round(time.perf_counter() - t0, 3), "iterations": infr["iters"],
            "converged": infr["converged"], "max_resnorm": max(infr["resnorm"]), "omega_ha": list(wr)}
        print(f"[bench] FP64 roots through split-BF16: {roots['fp64_via_bf16x3']['time_to_roots_s']:.1f}s "
              f"({infr['iters']} it, max|r| {max(infr['resnorm']):.1e})", file=sys.stderr, flush=True)
        del Xr
        h.close()
    if not args.no_mixed:
        reload()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = setup_then_release(A.ADC2_BF16X3)
        wb, Xb, infb = A.adc2_davidson(h, nroots, tol=args.tol_mixed, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        A.adc2_set_precision(h, A.ADC2_FP64)
        wp, rn = A.adc2_rayleigh(h, Xb)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r = {"what": f"split-BF16 folded solve to residual {args.tol_mixed:g} and the FP64 Rayleigh quotients of "
                     "its vectors (adc2_rayleigh), from adc2_setup to the roots on the host",
             "time_to_roots_s": round(t1 - t0, 3), "time_to_polished_roots_s": round(t2 - t0, 3),
             "iterations": infb["iters"], "converged": infb["converged"], "max_resnorm": max(infb["resnorm"]),
             "polished_resnorm_max": max(rn), "omega_ha": list(wb)}
        if "fp64_via_bf16x3" in roots:
            wref = np.array(roots["fp64_via_bf16x3"]["omega_ha"])
            r["ev_err_raw"] = [float(x) for x in (np.array(wb) - wref) * HARTREE_EV]
            r["ev_err_polished"] = [float(x) for x in (np.array(wp) - wref) * HARTREE_EV]
            r["error_reference"] = "the FP64 roots above (GPU, residual <= tol; the oracle check is at c1)"
        roots["bf16x3"] = r
        print(f"[bench] split-BF16 roots: {t1 - t0:.1f}s ({infb['iters']} it), polish {t2 - t1:.1f}s",
              file=sys.stderr, flush=True)
        del Xb
        h.close()
    torch.cuda.empty_cache()
    c1 = oracle_leg_c1(A, np, torch, args.tol_mixed)
    print("[bench] c1 roots against the oracle: FP64 max |dw| "
          f"{max(abs(x) for x in c1['fp64_abs_err_ha']):.1e} Ha, split-BF16 polished max "
          f"{max(abs(x) for x in c1['bf16x3_ev_err_polished']):.1e} eV", file=sys.stderr, flush=True)
    c2 = None
    if not args.no_c2:
        a2 = _ap.Namespace(**vars(args))
        a2.steps, a2.warmup, a2.max_subspace, a2.nguess, a2.nroots = 1, 0, 0, 0, 0
        c2 = run_pipeline(a2, A, np, torch, config="c2", peaks=False, with_cpu=False)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(Lhost, eps, nc, no, nv, naux, 4, 300)
    out = {
        "metric": METRIC,
        "value": sig["fp64"]["tflops"],
        "unit": "complex TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_total / max(1, args.steps) * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"CVS-ADC(2) {args.config}: nc={nc} no={no} nv={nv} naux={naux}; one step = one "
                               f"sigma build of {m} vectors in each of FP64, complex64 and split-BF16 "
                               "(value: the FP64 one)",
                   "nc": nc, "no": no, "nv": nv, "naux": naux, "m": m, "dim": dim},
        "roofline": sig["fp64"]["roofline"],
        "sigma": sig,
        "setup_s": round(setup_s, 3),
        "time_to_roots": roots,
        "roots_vs_oracle_c1": c1,
        "c2": c2,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--nroots", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--tol-mixed", type=float, default=1e-3)
    ap.add_argument("--tol-c64", type=float, default=1e-5)
    ap.add_argument("--max-iter", type=int, default=400)
    ap.add_argument("--max-subspace", type=int, default=0, help="search-space limit (0: the solver's default)")
    ap.add_argument("--nguess", type=int, default=0, help="guess vectors (0: the solver's default)")
    ap.add_argument("--solver", choices=["folded", "full"], default="folded")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-c64", action="store_true", help="skip the complex64 leg of the precision form")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the FP64 solve started from split-BF16 vectors (FP64 roots through the precision form)")
    ap.add_argument("--tol-refine", type=float, default=1e-4,
                    help="split-BF16 tolerance before the FP64 continuation")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="headline: skip the whole-path leg at c2")
    ap.add_argument("--workload", choices=["headline", "pipeline", "batch", "fd", "peaks", "transition"],
                    default="headline",
                    help="headline (default): sigma builds of the configuration in the three forms as the "
                         "steps, then the time-to-roots legs; pipeline: the whole path of one configuration "
                         "(setup, solves in every form, adjoint) as one step.  batch: the batching form (eight systems of uneven size, 16 roots each, complex64 "
                         "contractions, FP64 subspace) solved with adc2_davidson_batch and, for comparison, "
                         "one after the other; prints its own JSON line.  peaks: the device-rate "
                         "microbenchmarks the rooflines are quoted against")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch workload: keep the size rule for the Y-build K-split instead of adc2_autotune")
    ap.add_argument("--tol-batch", type=float, default=5e-5,
                    help="complex64 residual tolerance of the batch workload (its largest system's noise floor "
                         "is ~2e-5)")
    ap.add_argument("--batch-systems", default="",
                    help="comma-separated indices of the batch systems to run (default: all eight)")
    ap.add_argument("--batch-sigma-only", action="store_true",
                    help="batch workload: time only the batched sigma (separate, batched, graph replay)")
    ap.add_argument("--batch-sigma-reps", type=int, default=20,
                    help="batch workload: repetitions of each timed batched-sigma variant")
    ap.add_argument("--sigma-probe", action="store_true",
                    help="short run for hardware counters: 3 FP64, 3 complex64 and 3 split-BF16 sigma "
                         "builds (m=10) and a 2 GiB read+write calibration kernel; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over the valence index is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2604_27451_amd as A
    from synth import CONFIGS, config_system

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    A.load()
    if args.workload == "batch":
        run_batch(args, A, np, torch)
        return
    if args.workload == "fd":
        run_fd(args, A, np, torch)
        return
    if args.workload == "peaks":
        run_peaks(args, A)
        return
    if args.workload == "transition":
        run_transition(args, A, np, torch)
        return
    if args.workload == "pipeline":
        print(json.dumps(run_pipeline(args, A, np, torch, config=args.config)), flush=True)
        return
    run_headline(args, A, np, torch)


if __name__ == "__main__":
    main()
