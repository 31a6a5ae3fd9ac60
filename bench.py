"""Throughput of the periodic hot path on one MI355X: k-point blocks per second.

One step is one full pass of the hot path over every lattice of the plan:
assemble the generator blocks (factors, lattice sums, 1D Grams, combination),
block DFT over the lattice index, and the generalized eigensolve of every
Fourier block (with FP64 refinement on the mixed path).  Inputs (the lattice
descriptions) live in the plan; all buffers are resident in HBM before timing
starts.  Each plan is autotuned first, then one step is captured into a
hipGraph and the timed steps are graph replays.

Prints one JSON line.  ``value`` is the mixed-precision path's blocks/s; the
FP64 path is timed the same way and reported beside it.  Both are gated on
accuracy against the CPU oracle (run once, untimed for the GPU; for the
64-lattice mix, on one lattice of each basis size).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-point blocks/s (assemble+FFT+eig), mixed vs FP64 GPU at ≤1e-8 Ha eig error"
WORKLOADS = {
    "c1": "periodic 8x1x1 chain, m0=4 s, n=128^3, R=20",
    "c2": "periodic 256x1x1 tube, m0=16 (4 s + 4 p shells), n=2048x256x256, R=30",
    "c3": "periodic 32x32x32 lattice, m0=8 s, n=512^3, R=24",
    "c4": "64 periodic lattices in one grouped plan, L1 in [16,512], L2,L3 in {1,2,4}, m0 in {4,8,16,32}, "
          "n=16 L (128 across one-cell dims), R=24",
}
# lattices of the 64-lattice mix checked against the oracle: the cheapest of each basis size
C4_CHECK = (28, 41, 52, 2)
HBM_PEAK_GBS = 8000.0
# HBM bytes per call (FETCH_SIZE + WRITE_SIZE, KiB, scaled by a plain 512 MiB copy) of the mixed path's
# eigensolve call, block DFT and separable Fourier-block formation, from two rocprofv3 --pmc runs of
# `bench.py --probe-traffic` (profiles/traffic_per_dispatch.md).  The eigensolve's kernels depend on the
# tuned route, so its entry is keyed by the mixed plan's heev_fp64 and heev_wide masks.  Valid for the
# kernels as they were when counted; absent (reported as null) where not counted.
TRAFFIC_KIB = {"c2": {"eig": {"fp64=4,wide=4": 655.2}, "dft": 2357.1},
               "c3": {"eig": {"fp64=2,wide=0": 19202.8}, "sep": 69268.3},
               "c4": {"eig": {"fp64=15,wide=1": 310894.4}, "sep": 1344444.3}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the Dirichlet-chain (c5) measurement")
    ap.add_argument("--probe-traffic", action="store_true",
                    help="for hardware-counter runs: a device copy of 512 MiB (the counters' scale), then three "
                         "eager steps of each path; prints nothing else")
    ap.add_argument("--mixed-tuning", default="",
                    help="with --probe-traffic or --probe-mfma: JSON object of tuning fields for the mixed plans")
    ap.add_argument("--probe-mfma", action="store_true",
                    help="for MFMA counter runs: three eager mixed steps with each Gram arithmetic (FP64, FP32, "
                         "bf16 hi+lo); prints nothing else")
    return ap.parse_args()


def time_graph(graph, steps, torch):
    """Wall time per step of `steps` graph replays, bracketed by device
    synchronisations."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.lhf_graph_launch()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def event_ms(fn, steps, torch):
    """Average duration of fn()'s launches, timed with events recorded on the
    torch current stream (the stream the library launches on)."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / steps


def dft_bytes(pipe, insts, kind="plan"):
    """Algorithmic HBM bytes of one block-DFT call: every Fourier block written
    once (H and S, complex) plus every band generator read once (H and S,
    real).  kind "plan": in the plan's precision; "fp64": complex128 from FP64
    stacks (the mixed path's transform); "dual": complex128 and complex64."""
    from paper_1702_00339_amd import lhf
    cbytes = 16 if pipe.prec == lhf.LHF_PREC_FP64 else 8
    rbytes = cbytes // 2
    if kind == "fp64":
        cbytes, rbytes = 16, 8
    elif kind == "dual":
        cbytes, rbytes = 16 + 8, 8
    total = 0
    for i, inst in enumerate(insts):
        m2 = inst.m0 * inst.m0
        nshift, _, _ = pipe.plan.lhf_plan_band(i)
        band = 1
        for d in range(3):
            band *= nshift[d] if inst.L[d] > 1 else 1
        total += 2 * inst.ncells * m2 * cbytes + 2 * band * m2 * rbytes
    return total


def sep_bytes(pipe, insts):
    """Algorithmic HBM bytes of one lhf_fourier_blocks call: every Fourier
    block written once (H and S, complex128), every FP64 1D Gram read once,
    and the 1D-transformed Grams of dimensions 2 and 3 (complex128) written
    once and read once."""
    total = 0
    for i, inst in enumerate(insts):
        m2 = inst.m0 * inst.m0
        T = 2 + inst.M0 * inst.R
        nshift, _, _ = pipe.plan.lhf_plan_band(i)
        total += 2 * inst.ncells * m2 * 16
        total += sum(T * nshift[d] * m2 * 8 for d in range(3))
        total += 2 * sum(T * inst.L[d] * m2 * 16 for d in (1, 2))
    return total


def canonical_blocks(L):
    """Blocks solved once per conjugate pair j, -j."""
    self_conj = 1
    for x in L:
        self_conj *= 2 if x % 2 == 0 else 1
    n = L[0] * L[1] * L[2]
    return (n + self_conj) // 2


def heev_class(m0):
    """Eigensolver size class of a basis size: M = 4, 8, 16, 32 -> 0..3."""
    return 0 if m0 <= 4 else 1 if m0 <= 8 else 2 if m0 <= 16 else 3


def heev_flops(insts, prec, R, fp64_mask=0):
    """Algorithmic flops of one eigenvalues-only lhf_heev_batched call, per
    distinct block (8 flops per complex multiply-add).  FP64 solve: reduction
    to standard form (overlap elimination m0^3 / 3 and two m0^3 products,
    complex) and Householder tridiagonalisation (4/3 m0^3 complex), 29.3 m0^3,
    plus bisection, m0 eigenvalues x 53 halvings x m0 rows x 4 flops.  A mixed
    plan's FP32 classes: 150 m0^3 (reduction and 6-10 Jacobi sweeps) plus the
    FP64 refinement, (R + 4) m0^2 8 + 36 m0^3; its FP64 classes (bits of
    fp64_mask) count as the FP64 solve."""
    from paper_1702_00339_amd import lhf
    total = 0.0
    for inst in insts:
        m = inst.m0
        if prec == lhf.LHF_PREC_MIXED and not (fp64_mask >> heev_class(m)) & 1:
            per = 150.0 * m ** 3 + (R + 4) * m * m * 8 + 36.0 * m ** 3
        else:
            per = (8.0 / 3.0 + 16.0 + 32.0 / 3.0) * m ** 3 + 4.0 * 53.0 * m * m
        total += canonical_blocks(inst.L) * per
    return total


def eig_route(m0s, mask):
    """The eigensolver route of the tuned mixed plan, per size class (bits of
    mask: the FP64 solve alone)."""
    f64 = sorted({4 << heev_class(m) for m in m0s if (mask >> heev_class(m)) & 1})
    mix = sorted({4 << heev_class(m) for m in m0s if not (mask >> heev_class(m)) & 1})
    def which(sizes):
        return " (M = " + ", ".join(str(x) for x in sizes) + ")" if f64 and mix else ""
    parts = []
    if mix:
        parts.append("FP32 Jacobi on the rounded blocks + FP64 Rayleigh-Ritz refinement" + which(mix))
    if f64:
        parts.append("FP64 Householder tridiagonalisation + bisection" + which(f64))
    return "; ".join(parts)


def bench_c5(torch, np, lhf, steps):
    """Dirichlet 512-cell chain with 26 defect cells: time to the 32 lowest
    eigenpairs (operator assembly, then block LOBPCG), their error against the
    stored oracle values, and the event-timed matvec of a full LOBPCG basis
    (120 vectors, H and S) with its algorithmic HBM bytes: x read once, y_H and
    y_S written once (FP64), the two per-frequency operators and the cross
    corrections read once."""
    from synth import make_config
    inst = make_config("c5")
    gold = np.loadtxt(os.path.join(ROOT, "tests", "golden", "c5_lowest32.txt"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = lhf.Toeplitz(inst)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    w = torch.empty(32, dtype=torch.float64, device="cuda")
    ws = op.eigs_workspace(32)
    op.lhf_toeplitz_eigs(32, w, None, maxit=150, tol=1e-5, seed=1, ws=ws)     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, res = op.lhf_toeplitz_eigs(32, w, None, maxit=150, tol=1e-5, seed=1, ws=ws)
    torch.cuda.synchronize()
    t_eigs = time.perf_counter() - t0
    err = float(np.abs(w.cpu().numpy() - gold).max())
    info = op.info
    N, m0, P = info.N, info.m0, info.P
    ncols = 120
    x = torch.randn((N, ncols), dtype=torch.float64, device="cuda")
    yH, yS = torch.empty_like(x), torch.empty_like(x)
    mws = op.matvec_workspace(ncols)
    mv = {}
    nent = 2 * info.ncross_blocks - info.ncross   # correction entries: both orientations, diagonal once
    for name, prec, csz in (("fp32", lhf.LHF_PREC_MIXED, 8), ("fp64", lhf.LHF_PREC_FP64, 16)):
        ms = event_ms(lambda: op.lhf_toeplitz_matvec(prec, x, yH, yS, mws), steps, torch)
        nbytes = 3 * N * ncols * 8 + 2 * P * m0 * m0 * csz + 2 * nent * m0 * m0 * 8
        mv[name] = {"avg_launch_ms": ms, "bytes": nbytes, "GB/s": nbytes / (ms * 1e-3) / 1e9}
    return {"workload": "c5: Dirichlet 512x1x1 chain, m0=16, n=4096x256x256, R=30, 26 defect cells",
            "metric": "time to the 32 lowest eigenpairs", "create_ms": t_create * 1e3, "eigs_ms": t_eigs * 1e3,
            "unit": "ms", "lobpcg_iterations": it, "residual": res, "max_abs_eig_err_ha": err,
            "L0": info.L0, "cross_cells": info.ncross, "embedding": P, "matvec_120_vectors": mv}


def apply_tuning(pipe, spec):
    """Set the tuning fields of a JSON object (--mixed-tuning) on a pipeline's plan."""
    if not spec:
        return
    t = pipe.plan.lhf_plan_get_tuning()
    for k, v in json.loads(spec).items():
        setattr(t, k, int(v))
    pipe.plan.lhf_plan_set_tuning(t)


def probe_traffic(args, torch, lhf, Pipeline, make_config, config_c4_lattices):
    """Kernels for a FETCH_SIZE / WRITE_SIZE counter run: a plain copy of
    512 MiB (reads and writes exactly that many bytes: the scale of the
    counters), then three eager steps of the mixed and the FP64 paths; the
    mixed plan takes the tuning fields given by --mixed-tuning (a JSON object,
    e.g. the autotuned route of a timed run), the FP64 plan its defaults."""
    src = torch.ones(512 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    insts = config_c4_lattices() if args.config == "c4" else [make_config(args.config)]
    for prec in (lhf.LHF_PREC_MIXED, lhf.LHF_PREC_FP64):
        kw = {"gram": lhf.LHF_GRAM_FP64} if prec == lhf.LHF_PREC_MIXED else {}
        pipe = Pipeline(insts, prec=prec, **kw)
        if prec == lhf.LHF_PREC_MIXED:
            apply_tuning(pipe, args.mixed_tuning)
        for _ in range(3):
            pipe.step_native()
    torch.cuda.synchronize()


def probe_mfma(args, torch, lhf, Pipeline, make_config, config_c4_lattices):
    """Kernels for an MFMA counter run: three eager steps of the mixed path
    with each Gram arithmetic (the assembly's MFMA kernels), with the tuning
    fields of --mixed-tuning (e.g. the Gram tile of a timed run)."""
    insts = config_c4_lattices() if args.config == "c4" else [make_config(args.config)]
    for gram, src in ((lhf.LHF_GRAM_FP64, "dual"), (lhf.LHF_GRAM_FP32, "bar64"), (lhf.LHF_GRAM_BF16X3, "bar64")):
        pipe = Pipeline(insts, prec=lhf.LHF_PREC_MIXED, gram=gram, refine_src=src)
        apply_tuning(pipe, args.mixed_tuning)
        for _ in range(3):
            pipe.step()
    torch.cuda.synchronize()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is designed but not built)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1702_00339_amd import lhf
    from paper_1702_00339_amd.pipeline import Pipeline
    from synth import config_c4_lattices, make_config

    torch.cuda.set_device(0)
    if args.probe_traffic:
        probe_traffic(args, torch, lhf, Pipeline, make_config, config_c4_lattices)
        return
    if args.probe_mfma:
        probe_mfma(args, torch, lhf, Pipeline, make_config, config_c4_lattices)
        return
    if args.config == "c4":
        insts = config_c4_lattices()
        checked = [insts[i] for i in C4_CHECK]
    else:
        insts = [make_config(args.config)]
        checked = insts
    # mixed: FP64 MFMA Grams (which the FP64 refinement needs anyway), FP64
    # stacks, one FP64 block DFT writing complex128 blocks, which the FP32
    # solve reads and rounds; mixed_bf16x3: FP32 stacks from separate bf16
    # hi+lo split Grams and a complex64 DFT, reported beside it
    pipes = {"mixed": Pipeline(insts, prec=lhf.LHF_PREC_MIXED, gram=lhf.LHF_GRAM_FP64),
             "fp64": Pipeline(insts, prec=lhf.LHF_PREC_FP64),
             "mixed_bf16x3": Pipeline(insts, prec=lhf.LHF_PREC_MIXED, gram=lhf.LHF_GRAM_BF16X3,
                                      refine_src="band" if all(i.L[1] == 1 and i.L[2] == 1 for i in insts)
                                      else "bar64")}
    tuning = {name: p.autotune().as_dict() for name, p in pipes.items()}
    graphs = {name: p.capture() for name, p in pipes.items()}
    for g in graphs.values():
        for _ in range(args.warmup):
            g.lhf_graph_launch()
    torch.cuda.synchronize()

    # accuracy gate against the CPU oracle (also the CPU baseline's first run)
    from oracle import separable
    t0 = time.perf_counter()
    refs = [np.sort(separable.solve(inst)["eig"], axis=-1) for inst in checked]
    t_oracle_first = time.perf_counter() - t0
    errs = {}
    for name, p in pipes.items():
        graphs[name].lhf_graph_launch()
        torch.cuda.synchronize()
        all_w = p.eigenvalues()
        got = {inst.name: w for inst, w in zip(insts, all_w)}
        ea, er = 0.0, 0.0
        for inst, ref in zip(checked, refs):
            w = got[inst.name]
            ea = max(ea, float(np.abs(w - ref).max()))
            er = max(er, float((np.abs(w - ref) / np.maximum(np.abs(ref), 1.0)).max()))
        errs[name] = (ea, er, bool((p.info.cpu().numpy() == 0).all()))

    # timed region: graph replays
    sec = {name: time_graph(graphs[name], args.steps, torch) for name in pipes}
    nblk = sum(inst.ncells for inst in insts)
    value = nblk / sec["mixed"]

    # rooflines, event-timed on the stream the kernels run on
    pm = pipes["mixed"]
    sep = pm.separable()   # the Fourier-block route the tuned step takes
    if sep:
        ms_dft = event_ms(lambda: pm.plan.lhf_fourier_blocks(pm.grams64, pm.H_bar64, pm.S_bar64, pm.ws),
                          args.steps, torch)
        bytes_alg = sep_bytes(pm, insts)
    else:
        ms_dft = event_ms(lambda: pm.plan.lhf_block_fft(lhf.LHF_PREC_FP64, pm.H_gen64, pm.S_gen64, pm.H_bar64,
                                                         pm.S_bar64, pm.ws), args.steps, torch)
        bytes_alg = dft_bytes(pm, insts, kind="fp64")
    achieved = bytes_alg / (ms_dft * 1e-3) / 1e9
    flags = lhf.LHF_HEEV_REFINE_FP64
    ms_heev = event_ms(lambda: pm.plan.lhf_heev_batched(flags, None, None, pm.w, pm.info, pm.ws,
                                                         H_bar64=pm.H_bar64, S_bar64=pm.S_bar64,
                                                         H_gen64=pm.H_gen64, S_gen64=pm.S_gen64),
                       args.steps, torch)
    R = insts[0].R
    fp64_mask = pm.plan.lhf_plan_get_tuning().heev_fp64
    flops = heev_flops(insts, pm.prec, R, fp64_mask)
    tflops = flops / (ms_heev * 1e-3) / 1e12

    c5 = None if args.no_c5 else bench_c5(torch, np, lhf, args.steps)

    cpu = None
    if not args.no_cpu_baseline:
        runs = [t_oracle_first]
        while sum(runs) < 10.0 and len(runs) < 8:
            t0 = time.perf_counter()
            for inst in checked:
                separable.solve(inst)
            runs.append(time.perf_counter() - t0)
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        tmed = float(np.median(runs))
        nchk = sum(inst.ncells for inst in checked)
        what = (f"the whole {args.config} lattice" if len(checked) == len(insts) else
                f"{len(checked)} of the {len(insts)} lattices (one per basis size)")
        cpu = {"value": nchk / tmed, "unit": "blocks/s", "cores": int(cores), "kind": "oracle",
               "sample": f"{what} ({nchk} blocks) through the oracle's separable route (1D Grams for every "
                         f"shift, combination, FFT, batched LAPACK eigensolves), median of {len(runs)} runs "
                         f"of {tmed:.2f} s"}

    tuned = pm.plan.lhf_plan_get_tuning()

    def traffic(kind):
        t = TRAFFIC_KIB.get(args.config, {}).get(kind)
        if kind == "eig":
            t = (t or {}).get(f"fp64={tuned.heev_fp64},wide={tuned.heev_wide}")
        return None if t is None else t * 1024.0

    m0s = sorted({inst.m0 for inst in insts})
    line = {
        "metric": METRIC, "value": value, "unit": "blocks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec["mixed"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64", "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "lattices": len(insts),
                   "k_point_blocks": nblk, "m0": m0s if len(m0s) > 1 else m0s[0],
                   "path": ("mixed: FP64 MFMA Grams, " +
                            ("Fourier blocks formed separably from the Grams (complex128, no generator stacks)"
                             if sep else "FP64 stacks, one block DFT writing complex128 blocks") +
                            "; " + eig_route(m0s, fp64_mask) + "; one hipGraph replay per step")},
        "fp64_path": {"value": nblk / sec["fp64"], "ms_per_step": sec["fp64"] * 1e3, "dtype": "f64"},
        "mixed_bf16x3_path": {"value": nblk / sec["mixed_bf16x3"], "ms_per_step": sec["mixed_bf16x3"] * 1e3,
                              "max_abs_eig_err_ha": errs["mixed_bf16x3"][0], "info_ok": errs["mixed_bf16x3"][2]},
        "accuracy": {"lattices_checked": len(checked),
                     "mixed_max_abs_eig_err_ha": errs["mixed"][0], "mixed_info_ok": errs["mixed"][2],
                     "fp64_max_rel_eig_err": errs["fp64"][1], "fp64_info_ok": errs["fp64"][2]},
        "roofline": {"bound": "alu", "kernel": "eigensolve (lhf_heev_batched: " + eig_route(m0s, fp64_mask) + ")",
                     "achieved": tflops, "peak": 157.3, "unit": "TFLOP/s", "frac": tflops / 157.3,
                     "traffic": traffic("eig"), "flops_per_launch": flops, "avg_launch_ms": ms_heev},
        "roofline_dft": {"bound": "hbm",
                         "kernel": ("separable Fourier blocks (lhf_fourier_blocks: gram_dft + sep_fused, FP64 Grams "
                                    "to complex128)" if sep else "block DFT (lhf_block_fft, FP64 stacks to complex128)"),
                         "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic("sep" if sep else "dft"),
                         "bytes_per_launch": bytes_alg, "avg_launch_ms": ms_dft},
        "tuning": tuning,
        "dirichlet_c5": c5,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
