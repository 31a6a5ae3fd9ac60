"""Throughput of the periodic hot path on one MI355X: k-point blocks per second.

One step is one full pass of the hot path over every lattice of a plan:
assemble the generator blocks (factors, lattice sums, 1D Grams, combination),
form the Fourier blocks (block DFT over the lattice index, or separably from
the 1D Grams), and solve the generalized eigenproblem of every Fourier block.
Inputs (the lattice descriptions) live in the plan; every buffer is resident
in HBM before timing starts.  Each plan is autotuned, one step is captured
into a hipGraph, and the timed steps are graph replays.

Every workload is run on three routes, each gated on accuracy against the CPU
oracle (run untimed, in the same process):
  * "tuned"  the mixed-precision plan with every choice left to its autotuner,
             which may give a size class to the FP64 solve alone; its route
             and dtype are reported as taken;
  * "fp64"   the plain all-FP64 plan;
  * "fp32"   the reduced-precision route: bf16 hi+lo split Grams on the
             matrix cores, FP32 stacks, complex64 block DFT, FP32 Jacobi, and
             FP64 refinement of every eigenpair (no class goes to the FP64
             solve alone).
``value`` is the tuned route on the headline workload (the 256-cell tube);
the other two and the cube and the 64-lattice mix are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2] [--legs c3,c4]
"""

from __future__ import annotations

import argparse
import hashlib
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
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}     # MI355X vector peaks
HEEV_FLOPS_PER_M3 = 150.0                    # algorithmic eigensolve work per block: 150 m0^3

# HBM bytes per call (FETCH_SIZE + WRITE_SIZE, KiB, each scaled by what the counter reads for a plain
# 512 MiB device copy) of the headline kernels, from two rocprofv3 --pmc runs of `bench.py
# --probe-traffic` (profiles/traffic_per_dispatch.md).  Each entry names the source files of its kernels
# and their SHA-1 (first 16 hex digits) when counted, and the route it was counted on (a list holds one
# entry per route); an entry whose sources have changed since, or whose route is not the one timed, is
# reported as null.
TRAFFIC_KIB = {
    "c2": {
        "eigensolve": {"kib": 1233.2, "route": "fp64=4,wide=4", "src": ["heev.hip", "sturm.h", "dpp.h"], "sha": "2d52cf7efc8892d1"},
        "fourier": {"kib": 4123.2, "route": "sep", "src": ["blockdft.hip"], "sha": "550f7bca970db033"},
    },
    "c3": {
        "eigensolve": {"kib": 35988.9, "route": "fp64=2,wide=0", "src": ["heev.hip", "sturm.h", "dpp.h"], "sha": "2d52cf7efc8892d1"},
        "fourier": {"kib": 71354.8, "route": "sep", "src": ["blockdft.hip"], "sha": "550f7bca970db033"},
    },
    "c4": {
        "eigensolve": [
            {"kib": 606495.2, "route": "fp64=15,wide=0", "src": ["heev.hip", "sturm.h", "dpp.h"], "sha": "2d52cf7efc8892d1"},
            # the same run's dispatches with the M = 4 class in the wide layout
            {"kib": 606646.6, "route": "fp64=15,wide=1", "src": ["heev.hip", "sturm.h", "dpp.h"], "sha": "2d52cf7efc8892d1"},
        ],
        "fourier": {"kib": 1471752.7, "route": "sep", "src": ["blockdft.hip"], "sha": "550f7bca970db033"},
    },
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--legs", default="c3,c4", help="further workloads reported in the same line ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the Dirichlet-chain (c5) measurement")
    ap.add_argument("--no-box", action="store_true", help="skip the exact box-case measurements")
    ap.add_argument("--probe-traffic", action="store_true",
                    help="for hardware-counter runs: a device copy of 512 MiB (the counters' scale), then three "
                         "eager steps of the tuned and the FP64 paths; prints nothing else")
    ap.add_argument("--mixed-tuning", default="",
                    help="with --probe-traffic or --probe-mfma: JSON object of tuning fields for the mixed plans")
    ap.add_argument("--probe-mfma", action="store_true",
                    help="for MFMA counter runs: three eager mixed steps with each Gram arithmetic (FP64, FP32, FP16 hi+lo, "
                         "bf16 hi+lo); prints nothing else")
    return ap.parse_args()


def src_sha(files):
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, "paper_1702_00339_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(cfg, kernel, route):
    ents = TRAFFIC_KIB.get(cfg, {}).get(kernel) or []
    for e in ents if isinstance(ents, list) else [ents]:
        if e["route"] == route and src_sha(e["src"]) == e["sha"]:
            return e["kib"] * 1024.0
    return None


def time_graph(graph, steps, torch):
    """Wall time per step of `steps` graph replays, bracketed by device
    synchronisations."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.lhf_graph_launch()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def event_ms(fn, reps, torch):
    """Average duration of one call of fn, from `reps` calls issued back to
    back between two events on torch's current stream (the stream the library
    launches on), after one untimed call."""
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


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


def heev_flops_kernel(insts, fp64_classes, R):
    """The kernels' own operation count per call (8 flops per complex
    multiply-add), per distinct block.  FP64 solve: reduction to standard
    form (elimination m0^3 / 3 and two m0^3 products, complex) and Householder
    tridiagonalisation (4/3 m0^3 complex), 29.3 m0^3, plus bisection, m0
    eigenvalues x 53 halvings x m0 rows x 4.  FP32 solve: 150 m0^3 (reduction
    and 6-10 Jacobi sweeps) plus the FP64 refinement, (R + 4) m0^2 8 + 36 m0^3."""
    total = 0.0
    for inst in insts:
        m = inst.m0
        if heev_class(m) in fp64_classes:
            per = (8.0 / 3.0 + 16.0 + 32.0 / 3.0) * m ** 3 + 4.0 * 53.0 * m * m
        else:
            per = 150.0 * m ** 3 + (R + 4) * m * m * 8 + 36.0 * m ** 3
        total += canonical_blocks(inst.L) * per
    return total


def dft_bytes(pipe, insts, cbytes):
    """Algorithmic HBM bytes of one block-DFT call: every Fourier block written
    once (H and S, complex of cbytes) plus every band generator read once (H
    and S, real of cbytes / 2)."""
    total = 0
    for i, inst in enumerate(insts):
        m2 = inst.m0 * inst.m0
        nshift, _, _ = pipe.plan.lhf_plan_band(i)
        band = 1
        for d in range(3):
            band *= nshift[d] if inst.L[d] > 1 else 1
        total += 2 * inst.ncells * m2 * cbytes + 2 * band * m2 * (cbytes // 2)
    return total


def is_chain(inst):
    return inst.L[1] == 1 and inst.L[2] == 1


def sep_bytes(pipe, insts):
    """Algorithmic HBM bytes of one lhf_fourier_blocks call: every Fourier
    block written once (H and S, complex128), every FP64 1D Gram read once,
    and for lattices other than chains the 1D-transformed Grams of dimensions
    2 and 3 (complex128) written once and read once."""
    total = 0
    for i, inst in enumerate(insts):
        m2 = inst.m0 * inst.m0
        T = 2 + inst.M0 * inst.R
        nshift, _, _ = pipe.plan.lhf_plan_band(i)
        total += 2 * inst.ncells * m2 * 16
        total += sum(T * nshift[d] * m2 * 8 for d in range(3))
        if not is_chain(inst):
            total += 2 * sum(T * inst.L[d] * m2 * 16 for d in (1, 2))
    return total


def sep_kernels(insts):
    """The kernels of the separable route for these lattices."""
    names = []
    if any(is_chain(i) for i in insts):
        names.append("sep_chain")
    if not all(is_chain(i) for i in insts):
        names.append("gram_dft + sep_fused")
    return ", ".join(names)


def route_of(pipe, insts):
    """(description, dtype, FP64-solve classes) of the route a pipeline's step takes."""
    from paper_1702_00339_amd import lhf
    t = pipe.plan.lhf_plan_get_tuning()
    classes = sorted({heev_class(i.m0) for i in insts})
    sep = pipe.separable()
    if pipe.prec == lhf.LHF_PREC_FP64:
        f64 = set(classes)
        parts = ["FP64 MFMA Grams",
                 "complex128 Fourier blocks " + ("formed separably from the Grams" if sep else "by block DFT"),
                 "FP64 Householder tridiagonalisation + bisection"]
        return "; ".join(parts), "f64", f64
    f64 = set() if pipe.fp32_solve else {c for c in classes if (t.heev_fp64 >> c) & 1}
    gram = {lhf.LHF_GRAM_FP64: "FP64 MFMA Grams", lhf.LHF_GRAM_FP32: "FP32 MFMA Grams + FP64 Grams",
            lhf.LHF_GRAM_BF16X3: "bf16 hi+lo split MFMA Grams (FP32 stacks) + FP64 Grams for refinement",
            lhf.LHF_GRAM_FP16X3: "FP16 hi+lo split MFMA Grams (FP32 stacks) + FP64 Grams for refinement"}
    parts = [gram[pipe.plan.gram] if pipe.refine_src in ("bar64", "band") else "FP64 MFMA Grams"]
    if pipe.refine_src == "direct":
        parts.append("complex128 Fourier blocks " + ("formed separably" if sep else "by block DFT"))
    elif pipe.refine_src == "dual":
        parts.append("one FP64 block DFT writing complex128 + complex64 blocks")
    else:
        parts.append("complex64 block DFT of the FP32 stacks" +
                     (" + complex128 block DFT of the FP64 stacks" if pipe.refine_src == "bar64" else ""))
    size = lambda cs: ", ".join(f"M={4 << c}" for c in sorted(cs))
    f32 = [c for c in classes if c not in f64]
    if f32:
        src = {"direct": "rounded complex128 blocks", "dual": "complex64 blocks", "bar64": "complex64 blocks",
               "band": "complex64 blocks"}[pipe.refine_src]
        ref = "regenerated from the FP64 generator band" if pipe.refine_src == "band" else "complex128 blocks"
        parts.append(f"FP32 Jacobi on the {src} + FP64 Rayleigh-Ritz refinement with {ref}" +
                     (f" ({size(f32)})" if f64 else ""))
    if f64:
        parts.append("FP64 Householder tridiagonalisation + bisection" + (f" ({size(f64)})" if f32 else ""))
    only64 = not f32 and pipe.refine_src == "direct"
    return "; ".join(parts), ("f64" if only64 else "fp32+fp64"), f64


def block_errors(pipe, which, insts, checked_idx, refs):
    """Largest absolute entry errors (Ha) of the Fourier blocks a route's
    solve reads, against the oracle's, and relative to the largest entry."""
    import numpy as np
    out = {}
    for name, key in (("H", which[0]), ("S", which[1])):
        got = pipe.stacks(key)
        ea, er = 0.0, 0.0
        for i, ref in zip(checked_idx, refs):
            want = ref[name + "_bar"]
            d = float(np.abs(got[i].astype(np.complex128) - want).max())
            ea = max(ea, d)
            er = max(er, d / float(np.abs(want).max()))
        out[f"max_abs_d{name}bar_ha"] = ea
        out[f"max_rel_d{name}bar"] = er
    return out


def leg(cfg, args, torch, np, lhf, Pipeline, headline):
    from synth import config_c4_lattices, make_config
    from oracle import separable
    if cfg == "c4":
        insts = config_c4_lattices()
        checked_idx = list(C4_CHECK)
    else:
        insts = [make_config(cfg)]
        checked_idx = [0]
    checked = [insts[i] for i in checked_idx]
    chain = all(i.L[1] == 1 and i.L[2] == 1 for i in insts)
    pipes = {"tuned": Pipeline(insts, prec=lhf.LHF_PREC_MIXED, gram=lhf.LHF_GRAM_FP64),
             "fp64": Pipeline(insts, prec=lhf.LHF_PREC_FP64),
             "fp32": Pipeline(insts, prec=lhf.LHF_PREC_MIXED, gram=lhf.LHF_GRAM_BF16X3,
                              refine_src="band" if chain else "bar64", fp32_solve=True)}
    tuning = {name: p.autotune().as_dict() for name, p in pipes.items()}
    graphs = {name: p.capture() for name, p in pipes.items()}
    for g in graphs.values():
        for _ in range(args.warmup):
            g.lhf_graph_launch()
    torch.cuda.synchronize()

    # accuracy against the oracle (its first run is also the CPU baseline's first run)
    t0 = time.perf_counter()
    refs = [separable.solve(inst) for inst in checked]
    t_oracle = time.perf_counter() - t0
    ref_eigs = [np.sort(r["eig"], axis=-1) for r in refs]
    # condition numbers of the overlap blocks (they bound how the block errors reach the eigenvalues)
    kappas = []
    for r in refs:
        ev = np.linalg.eigvalsh(r["S_bar"].reshape(-1, r["S_bar"].shape[-1], r["S_bar"].shape[-1]))
        kappas.append(ev[:, -1] / ev[:, 0])
    kap = np.concatenate(kappas)
    acc = {}
    for name, p in pipes.items():
        graphs[name].lhf_graph_launch()
        torch.cuda.synchronize()
        all_w = p.eigenvalues()
        ea, er, per_m0 = 0.0, 0.0, {}
        for i, ref in zip(checked_idx, ref_eigs):
            d = np.abs(all_w[i] - ref)
            ea = max(ea, float(d.max()))
            er = max(er, float((d / np.maximum(np.abs(ref), 1.0)).max()))
            m0 = insts[i].m0
            per_m0[m0] = max(per_m0.get(m0, 0.0), float(d.max()))
        a = {"max_abs_eig_err_ha": ea, "max_rel_eig_err": er, "info_ok": bool((p.info.cpu().numpy() == 0).all())}
        if len(per_m0) > 1:
            a["max_abs_eig_err_ha_by_m0"] = {str(k): v for k, v in sorted(per_m0.items())}
        # the Fourier blocks the route's solve reads
        if p.prec == lhf.LHF_PREC_FP64:
            a.update(block_errors(p, ("H_bar", "S_bar"), insts, checked_idx, refs))
        elif p.refine_src == "direct":
            a.update(block_errors(p, ("H_bar64", "S_bar64"), insts, checked_idx, refs))
        else:
            a.update({k + "_c64": v for k, v in block_errors(p, ("H_bar", "S_bar"), insts, checked_idx, refs).items()})
        acc[name] = a

    steps = args.steps if cfg != "c4" else max(5, min(args.steps, 10))
    sec = {name: time_graph(graphs[name], steps, torch) for name in pipes}
    nblk = sum(inst.ncells for inst in insts)
    # stage times: each call of the step issued back to back between two events
    stage_ms = {name: {st: event_ms(fn, steps, torch) for st, fn in p.stages()} for name, p in pipes.items()}

    routes = {name: route_of(p, insts) for name, p in pipes.items()}
    R = insts[0].R
    pt = pipes["tuned"]
    desc, dtype, f64 = routes["tuned"]
    classes = sorted({heev_class(i.m0) for i in insts})
    solve_dtype = "f64" if all(c in f64 for c in classes) else "f32"
    ms_heev = stage_ms["tuned"]["eigensolve"]
    flops = sum(canonical_blocks(i.L) * HEEV_FLOPS_PER_M3 * i.m0 ** 3 for i in insts)
    flops_kernel = heev_flops_kernel(insts, f64, R)
    achieved = flops / (ms_heev * 1e-3) / 1e12
    tuned_t = pt.plan.lhf_plan_get_tuning()
    eig_route = f"fp64={tuned_t.heev_fp64},wide={tuned_t.heev_wide}"
    sep = pt.separable()
    fourier_bytes = sep_bytes(pt, insts) if sep else dft_bytes(pt, insts, 16)
    ms_fourier = stage_ms["tuned"]["fourier"]
    fourier_gbs = fourier_bytes / (ms_fourier * 1e-3) / 1e9
    out = {
        "workload": f"{cfg}: {WORKLOADS[cfg]}", "lattices": len(insts), "k_point_blocks": nblk,
        "m0": sorted({i.m0 for i in insts}),
        "value": nblk / sec["tuned"], "ms_per_step": sec["tuned"] * 1e3, "dtype": dtype, "path": desc,
        "fp64_path": {"value": nblk / sec["fp64"], "ms_per_step": sec["fp64"] * 1e3, "dtype": "f64",
                      "path": routes["fp64"][0]},
        "fp32_path": {"value": nblk / sec["fp32"], "ms_per_step": sec["fp32"] * 1e3, "dtype": routes["fp32"][1],
                      "path": routes["fp32"][0], "vs_fp64": sec["fp64"] / sec["fp32"]},
        "tuned_vs_fp64": sec["fp64"] / sec["tuned"],
        "stage_ms": stage_ms,
        "accuracy": {"lattices_checked": len(checked), "oracle_s": t_oracle,
                     "kappa_Sbar": {"max": float(kap.max()), "median": float(np.median(kap))}, **acc},
        "roofline": {"bound": "alu", "kernel": f"eigensolve (lhf_heev_batched: {desc.split('; ')[-1]})",
                     "dtype": solve_dtype, "achieved": achieved, "peak": PEAK_TFLOPS[solve_dtype],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[solve_dtype],
                     "traffic": traffic_bytes(cfg, "eigensolve", eig_route),
                     "flops_per_launch": flops, "work_per_block": "150 m0^3 (distinct blocks)",
                     "kernel_flops_per_launch": flops_kernel,
                     "kernel_tflops": flops_kernel / (ms_heev * 1e-3) / 1e12, "avg_launch_ms": ms_heev},
        "roofline_fourier": {"bound": "hbm",
                             "kernel": (f"separable Fourier blocks (lhf_fourier_blocks: {sep_kernels(insts)}, FP64 "
                                        "Grams to complex128)" if sep else
                                        "block DFT (lhf_block_fft, FP64 stacks to complex128)"),
                             "achieved": fourier_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": fourier_gbs / HBM_PEAK_GBS,
                             "traffic": traffic_bytes(cfg, "fourier", "sep" if sep else "dft"),
                             "bytes_per_launch": fourier_bytes, "avg_launch_ms": ms_fourier},
        "tuning": tuning,
    }
    if headline and not args.no_cpu_baseline:
        runs = [t_oracle]
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
        what = (f"the whole {cfg} lattice" if len(checked) == len(insts) else
                f"{len(checked)} of the {len(insts)} lattices (one per basis size)")
        out["cpu_baseline"] = {
            "value": nchk / tmed, "unit": "blocks/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{what} ({nchk} blocks) through the oracle's separable route (1D Grams for every shift, "
                      f"combination, FFT, batched LAPACK eigensolves), median of {len(runs)} runs of {tmed:.2f} s"}
    for g in graphs.values():
        g.close()
    return out


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
    # the FP32 route with FP32 vectors (lhf_toeplitz_matvec_f32): x and y in 4 bytes
    x32 = x.float()
    yH32, yS32 = torch.empty_like(x32), torch.empty_like(x32)
    ms = event_ms(lambda: op.lhf_toeplitz_matvec_f32(x32, yH32, yS32, mws), steps, torch)
    nbytes = 3 * N * ncols * 4 + 2 * P * m0 * m0 * 8 + 2 * nent * m0 * m0 * 8
    mv["fp32_io"] = {"avg_launch_ms": ms, "bytes": nbytes, "GB/s": nbytes / (ms * 1e-3) / 1e9}
    return {"workload": "c5: Dirichlet 512x1x1 chain, m0=16, n=4096x256x256, R=30, 26 defect cells",
            "metric": "time to the 32 lowest eigenpairs", "create_ms": t_create * 1e3, "eigs_ms": t_eigs * 1e3,
            "unit": "ms", "lobpcg_iterations": it, "residual": res, "max_abs_eig_err_ha": err,
            "L0": info.L0, "cross_cells": info.ncross, "embedding": P, "matvec_120_vectors": mv}


def bench_box(torch, np, lhf, Pipeline, steps):
    """The exact box operator (case (B): finite-lattice potential, every band
    block) beside the block-Toeplitz model: time to the 32 lowest eigenpairs of
    the 512-cell chain with 26 defect cells, and the largest difference of the
    two spectra.  Then two qualitative comparisons of a chain in a box with the
    periodic chain, on the 8-cell chain's cell (4 s functions, Z = 1; the
    paper's hydrogen-chain workloads, stood in for), same grid spacing and
    sinc rule in both: the 32 lowest eigenvalues at L = 128 and 256 (box by
    LOBPCG, periodic from every Fourier block), and the mean energy of the
    lowest band (L states) per cell against L (box: LOBPCG with nev = L, so
    L <= 32; periodic up to 512)."""
    from synth import make_config, make_instance
    inst = make_config("c5")
    out = {}
    for name, exact in (("exact", True), ("model", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = lhf.Toeplitz(inst, exact=exact)
        torch.cuda.synchronize()
        t_create = time.perf_counter() - t0
        w = torch.empty(32, dtype=torch.float64, device="cuda")
        ws = op.eigs_workspace(32)
        op.lhf_toeplitz_eigs(32, w, None, maxit=150, tol=1e-5, seed=1, ws=ws)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, res = op.lhf_toeplitz_eigs(32, w, None, maxit=150, tol=1e-5, seed=1, ws=ws)
        torch.cuda.synchronize()
        out[name] = {"create_ms": t_create * 1e3, "eigs_ms": (time.perf_counter() - t0) * 1e3,
                     "lobpcg_iterations": it, "residual": res, "w": w.cpu().numpy()}
        op.close()
    d = np.abs(out["exact"]["w"] - out["model"]["w"])
    res = {"workload": "c5 chain as the exact box operator (finite-lattice potential, every band block)",
           "exact": {k: v for k, v in out["exact"].items() if k != "w"},
           "model": {k: v for k, v in out["model"].items() if k != "w"},
           "max_abs_diff_lowest32_ha": float(d.max()), "lowest_exact_ha": float(out["exact"]["w"][0]),
           "lowest_model_ha": float(out["model"]["w"][0])}

    def chain(L, bc):
        pad = (6.0, 6.0, 6.0) if bc == "periodic" else (5.0 / 32, 6.0, 6.0)
        i = make_instance(name=f"hchain_{bc}_{L}", L=(L, 1, 1), n=(16 * L, 128, 128), a=5.0, pad=pad, bc=bc,
                          n_s=4, n_p=0, exp_range=(0.2, 8.0), Z=1, R=20, seed=1)
        return i

    def periodic_eigs(L):
        pi = chain(L, "periodic")
        pipe = Pipeline([pi], prec=lhf.LHF_PREC_FP64)
        pipe.step()
        torch.cuda.synchronize()
        return pi, np.sort(pipe.eigenvalues()[0].ravel())

    def box_eigs(L, nev, like):
        bi = chain(L, "dirichlet")
        bi.sinc_u0, bi.sinc_step = like.sinc_u0, like.sinc_step
        op = lhf.Toeplitz(bi, exact=True)
        w = torch.empty(nev, dtype=torch.float64, device="cuda")
        op.lhf_toeplitz_eigs(nev, w, None, maxit=300, tol=1e-7, seed=2)
        torch.cuda.synchronize()
        op.close()
        return w.cpu().numpy()

    spectra = {}
    for L in (128, 256):
        pi, wp = periodic_eigs(L)
        wb = box_eigs(L, 32, pi)
        spectra[str(L)] = {"periodic_lowest": wp[:4].tolist(), "box_lowest": wb[:4].tolist(),
                           "mean_shift_lowest32_ha": float(np.mean(wb - wp[:32])),
                           "max_abs_shift_lowest32_ha": float(np.max(np.abs(wb - wp[:32])))}
    per_cell = {"L": [], "periodic": [], "box": []}
    for L in (4, 8, 16, 32, 64, 128, 256, 512):
        pi, wp = periodic_eigs(L)
        per_cell["L"].append(L)
        per_cell["periodic"].append(float(np.mean(wp[:L])))
        per_cell["box"].append(float(np.mean(box_eigs(L, L, pi))) if L <= 32 else None)
    res["box_vs_periodic_spectrum"] = spectra
    res["lowest_band_energy_per_cell"] = per_cell
    return res


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
    counters), then three eager steps of the tuned mixed plan (with the tuning
    fields given by --mixed-tuning, e.g. the route of a timed run) and of the
    FP64 plan with its defaults."""
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
    """Kernels for an MFMA counter run: three eager mixed steps with each Gram
    arithmetic (FP64, FP32, bf16 and FP16 hi+lo), with the tuning fields of
    --mixed-tuning (e.g. the Gram tile of a timed run)."""
    insts = config_c4_lattices() if args.config == "c4" else [make_config(args.config)]
    for gram, src in ((lhf.LHF_GRAM_FP64, "dual"), (lhf.LHF_GRAM_FP32, "bar64"), (lhf.LHF_GRAM_BF16X3, "bar64"),
                      (lhf.LHF_GRAM_FP16X3, "bar64")):
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
    head = leg(args.config, args, torch, np, lhf, Pipeline, headline=True)
    print(f"[bench] {args.config}: tuned {head['ms_per_step']:.4f} ms/step, fp64 {head['fp64_path']['ms_per_step']:.4f}, "
          f"fp32 {head['fp32_path']['ms_per_step']:.4f}", file=sys.stderr, flush=True)
    legs = {}
    for cfg in [c for c in args.legs.split(",") if c and c != args.config]:
        legs[cfg] = leg(cfg, args, torch, np, lhf, Pipeline, headline=False)
        print(f"[bench] {cfg}: tuned {legs[cfg]['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    c5 = None if args.no_c5 else bench_c5(torch, np, lhf, args.steps)
    box = None if args.no_box else bench_box(torch, np, lhf, Pipeline, args.steps)
    cpu = head.pop("cpu_baseline", None)
    line = {
        "metric": METRIC, "value": head["value"], "unit": "blocks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head["dtype"], "data": "synthetic",
        "config": {"workload": head["workload"], "lattices": head["lattices"], "k_point_blocks": head["k_point_blocks"],
                   "m0": head["m0"], "path": head["path"] + "; one hipGraph replay per step"},
        "fp64_path": head["fp64_path"], "fp32_path": head["fp32_path"], "tuned_vs_fp64": head["tuned_vs_fp64"],
        "accuracy": head["accuracy"], "stage_ms": head["stage_ms"],
        "roofline": head["roofline"], "roofline_fourier": head["roofline_fourier"], "tuning": head["tuning"],
        "legs": legs, "dirichlet_c5": c5, "box_case": box, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
