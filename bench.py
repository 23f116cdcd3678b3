#!/usr/bin/env python3
"""Benchmark of the APD hot path on one MI355X.

One step = one pass of the hot path on the 3D workload (256^3 voxels,
N = 10 000 seeds, Haar-random anisotropy with log-normal semi-axes of
determinant 1, log-normal volumes): seed preparation, the fused
single-precision assignment with the per-cell moment reduction, the double
re-check of near-tie voxels, and the double-precision finalize (objective
(2.7), gradient (2.8), max relative volume error), at weights fitted to 1 %
and moved through 5 generalised Lloyd steps (Algorithm 3).  The metric is
pixel-seed pairs per second, N J / (time per pass), with the inputs resident
in HBM, every pair evaluated.  Beside it: the same pass with per-tile
candidate lists (same result, less work), the bf16 tier, the time to fit
from W_0 = 0 to 1 % (Algorithm 2, library defaults) over runs 0..9, and the
same figures for the 2D workload (1024^2 pixels, N = 1000).

The roofline is the vector ALU's issue rate: the kernels are bound by it,
not by HBM.  Per pair the method needs two fused multiply-adds (the
quadratic form in the axis-0 offset by Horner's rule) and one update of the
running minimum: 3 lane operations.  The peak is 256 compute units x 4 SIMDs
x 32 lanes per clock x 2.4 GHz = 78.6e12 lane operations/s (the published
FP32 vector rate, 157.3 TFLOP/s, is this many fused multiply-adds of 2 flops
each); apd_measure_valu_rate checks it on the device.

Prints one JSON line.  ``--gpus`` above 1 is refused: the library runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_FP32_PEAK = 157.3e12  # FLOP/s, vector FP32 (published)
MI355X_HBM_PEAK = 8.0e12     # B/s
# vector-ALU issue rate: 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz
MI355X_VALU_PEAK = 256 * 4 * 32 * 2.4e9  # lane operations/s
# algorithmic lane operations per pixel-seed pair: two fused multiply-adds
# (Horner's rule in the axis-0 offset) and one running-minimum update.  The
# count is the algorithm's, the peak the vector ALU's; the hybrid kernel
# forms the per-position coefficients on the matrix cores and shares one
# multiply-add between the two rows of a symmetric pair, so it issues fewer.
OPS_PER_PAIR = 3

# HBM bytes per launch of a kernel, from two rocprofv3 --pmc runs of this
# script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by what the
# same counters read for a 1 GiB device copy in the same session
# (--copy-calibration: the factors below are 1 GiB over the counter's
# reading).  A figure holds for the kernel sources it was measured on (their
# SHA-256); after any change to them it is reported as null until measured
# again.
KERNEL_SOURCES = ("paper_2403_03571_amd/csrc/apd_device.h", "paper_2403_03571_amd/csrc/apd_internal.h",
                  "paper_2403_03571_amd/csrc/apd_kernels.hip")
MEASURED_TRAFFIC = {
    ("k_assign_hyb<3>", "c3"): {
        "fetch_kib": 5692.0, "write_kib": 20526.7, "fetch_factor": 1048576 / 524302.5, "write_factor": 1.0,
        "sources_sha256": "d6e1432f3ee2cf41122062e0506e6c059bd5ca704adf47dfbddb357b20ae9a4e"},
    ("k_assign_vec<2, false, 4>", "c2"): {
        "fetch_kib": 366.0, "write_kib": 715.9, "fetch_factor": 1048576 / 524302.5, "write_factor": 1.0,
        "sources_sha256": "d6e1432f3ee2cf41122062e0506e6c059bd5ca704adf47dfbddb357b20ae9a4e"},
}


def kernel_sources_digest() -> str:
    """SHA-256 of the kernel sources without their // comments and blank
    lines: the code the traffic was measured on."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None or rec["sources_sha256"] != kernel_sources_digest():
        return None
    return 1024.0 * (rec["fetch_factor"] * rec["fetch_kib"] + rec["write_factor"] * rec["write_kib"])


WORKLOADS = {
    "c1": "2D unit square, 256x256 pixels, N=16 seeds, aspect U[1,3], equal volumes",
    "c2": "2D unit square, 1024x1024 pixels, N=1000 seeds, det-1 aspect U[1,4], "
          "log-normal(0.35) volumes, weights fitted to 1%",
    "c3": "3D unit cube, 256^3 voxels, N=10000 seeds, Haar rotations, log a ~ N(0,0.3^2) det 1, "
          "log-normal(0.3) volumes, weights fitted to 1%",
}


def hyb_by_default(inst) -> bool:
    """The library's default kernel choice over every seed: the hybrid kernel
    from 1536 seeds on grids of at least 128 of its tiles (16 x 16 x 8 in 3D,
    32 x 32 in 2D)."""
    g = inst.grid
    tiles = (-(-g[0] // 16) * -(-g[1] // 16) * -(-g[2] // 8)) if inst.dim == 3 else (-(-g[0] // 32) * -(-g[1] // 32))
    return inst.n >= 1536 and tiles >= 128


def kernel_name(args, inst, cull=False) -> str:
    """The assignment kernel a pass of this configuration launches."""
    d = inst.dim
    if args.prec == "fp64":
        return f"k_assign_fp64<{d}>"
    if args.prec == "bf16":
        p = getattr(args, "pixels_per_lane", 0)
        rows = p // 2 if p in (4, 8) else (4 if d == 2 else 2)
        chunk = 1024 if d == 2 and not cull else 256
        return f"k_assign_bf16<{d}, {rows}, {chunk}, {'true' if cull else 'false'}>"
    if args.variant == 0:
        return f"k_assign_mfma<{d}>"
    if not cull and (args.variant == 3 or (args.variant == 2 and hyb_by_default(inst))):
        return f"k_assign_hyb<{d}>"
    p = getattr(args, "pixels_per_lane", 0)
    if p not in (4, 8):
        p = 4 if cull else (8 if inst.J >= 1024 * 2048 else 4)
    return f"k_assign_vec<{d}, {'true' if cull else 'false'}, {p}>"


def cpu_baseline(inst, w, budget_s: float = 15.0):
    """The CPU oracle (FP64 brute force) timed on this host on a bounded
    sample: whole passes of the same workload until about budget_s, or for
    workloads whose single pass exceeds the budget, Algorithm 1 on a random
    sample of pixels sized to the budget."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    if inst.pairs > 2e10:
        rng = np.random.default_rng(0)
        m = 20000
        t0 = time.perf_counter()
        oracle.assign_pixels(inst, w, rng.choice(inst.J, m, replace=False))
        probe = time.perf_counter() - t0
        m = int(min(inst.J, m * max(1.0, budget_s / max(probe, 1e-3))))
        idx = rng.choice(inst.J, m, replace=False)
        t0 = time.perf_counter()
        oracle.assign_pixels(inst, w, idx)
        el = time.perf_counter() - t0
        return {
            "value": m * inst.n / el,
            "unit": "pairs/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"Algorithm 1 (FP64 brute force) at {m} random pixels of the same workload "
                      f"and weights, {el:.1f} s",
        }
    n_pass = 0
    t0 = time.perf_counter()
    while True:
        oracle.evaluate(inst, w)
        n_pass += 1
        el = time.perf_counter() - t0
        if el > budget_s or n_pass >= 20:
            break
    return {
        "value": inst.pairs * n_pass / el,
        "unit": "pairs/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{n_pass} full passes (evaluate: assignment + objective + gradient) of the "
                  f"same workload at the same weights, FP64, {el:.1f} s",
    }


def bench_batched(args):
    """512 independent 2D instances (N ~ U{50..2000}, grids 256^2..1024^2):
    the batched solver (one persistent pass per evaluation of every active
    instance, device L-BFGS, graph replays) against the plain per-instance
    GPU solve on the same instances, both from W_0 = 0 to 1 %."""
    import numpy as np
    import torch

    import apd_synth as S
    import paper_2403_03571_amd as apd
    insts = S.make_c4_batch(args.batch)
    probs = [apd.Problem.from_instance(i, "cuda:0") for i in insts]
    ctx = apd.Context(0)
    ctx.apd_set_variant(args.variant)
    ctx.apd_set_pixels_per_lane(args.pixels_per_lane)
    prec = "bf16" if args.prec == "bf16" else "fp32"
    out = {"metric": "wall time to fit 1% volume error (batched, all instances)", "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"{args.batch} independent 2D APDs, N~U{{50..2000}}, "
                                  "grids clamp(roundup64(20 sqrt N),256,1024)^2, aspect U[1,3], "
                                  "equal volumes",
                      "instances": args.batch, "pixels": int(sum(i.J for i in insts)),
                      "pairs_per_pass": int(sum(i.pairs for i in insts))},
           "dtype": {"fp32": "f32", "bf16": "bf16"}[prec]}
    # warm-up (module load, first launch, graph instantiation paths)
    ctx.apd_fit_weights_batched(probs[:4], prec=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ws, reps, status = ctx.apd_fit_weights_batched(probs, prec=prec)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    evals = np.array([r.evals for r in reps])
    pairs = float(sum(e * i.pairs for e, i in zip(evals, insts)))
    out.update({"value": tb, "status": status,
                "converged": int(sum(r.converged for r in reps)),
                "evals_mean": float(evals.mean()), "evals_max": int(evals.max()),
                "graph_replays": int(evals.max()),
                "pairs_evaluated": pairs, "pairs_per_s": pairs / tb})
    print(f"# batched: {tb:.3f} s, {status}", file=sys.stderr, flush=True)
    # the plain per-instance solve of the same instances
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv = 0
    ev1 = []
    for p in probs:
        w, r = ctx.apd_fit_weights(p, prec=prec)
        conv += r.converged
        ev1.append(r.evals)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out["per_instance"] = {"seconds": ts, "converged": conv, "evals_mean": float(np.mean(ev1))}
    out["speedup_vs_per_instance"] = ts / tb
    print(f"# per instance: {ts:.3f} s", file=sys.stderr, flush=True)
    return out


def bench_microstructure(args):
    """Algorithm 3 at the scale of the paper's synthetic microstructure
    (Section 3.4): N = 4587 grains with areas spanning a factor of ~196,
    seeds X^0 uniform, fit to 2 % from W = 0, then 5 Lloyd steps each
    followed by a warm refit, on the grid of eq. (2.10) for 2 %; then the
    grain-map fit at 1 % (eq. (2.10) grid for 1 %) with the final seeds
    (grain centroids) from W = 0, the analogue of the paper's EBSD fit."""
    import numpy as np
    import torch

    import apd_synth as S
    import paper_2403_03571_amd as apd
    ctx = apd.Context(0)
    ctx.apd_set_variant(args.variant)
    probe = S.make_microstructure(6000, M=64)
    M2 = apd.apd_choose_resolution(2, 0.02, float(probe.v.min()), 1.0)
    M1 = apd.apd_choose_resolution(2, 0.01, float(probe.v.min()), 1.0)
    inst = S.make_microstructure(6000, M=M2)
    prob = apd.Problem.from_instance(inst, "cuda:0")
    out = {"metric": "wall time of Algorithm 3 (fit to 2 % + 5 Lloyd steps with refits)", "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "2D polycrystal-like APD: N=4587, areas log-normal max/min ~196, "
                                  "aspect ratios up to ~5 (small grains more elongated), uniform X^0",
                      "grid_2pct": M2, "grid_1pct": M1, "pairs_per_pass": int(inst.n) * M2 * M2},
           "dtype": "f32"}
    # warm-up on a small grid (module load, first launches)
    small = apd.Problem.from_instance(S.make_microstructure(6000, M=512), "cuda:0")
    ctx.apd_fit_weights(small, eps=0.05, max_evals=20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, rep = ctx.apd_fit_weights(prob, eps=0.02)
    steps = [{"fit_evals": rep.evals, "converged": rep.converged}]
    x = prob.x.clone()
    for k in range(5):
        x, w, r = ctx.apd_lloyd_step(prob, x, w, eps=0.02)
        steps.append({"lloyd": k, "evals": r.evals, "converged": r.converged})
    final = apd.Problem(prob.dim, prob.grid, prob.lo, prob.hi, x, prob.A, prob.v)
    w, r = ctx.apd_fit_weights(final, w=w, eps=0.02)
    torch.cuda.synchronize()
    t_alg3 = time.perf_counter() - t0
    steps.append({"final_fit_evals": r.evals, "converged": r.converged, "max_rel_err": r.max_rel_err})
    out.update({"value": t_alg3, "steps": steps,
                "evals_total": int(sum(st.get("fit_evals", 0) + st.get("evals", 0) +
                                       st.get("final_fit_evals", 0) for st in steps))})
    print(f"# Algorithm 3: {t_alg3:.2f} s", file=sys.stderr, flush=True)
    # the grain-map fit: seeds = the final centroids, 1 %, from W = 0
    grains = apd.Problem(2, (M1, M1), prob.lo, prob.hi, x, prob.A, prob.v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wg, rg = ctx.apd_fit_weights(grains, eps=0.01)
    torch.cuda.synchronize()
    out["grain_map_fit"] = {"seconds": time.perf_counter() - t0, "evals": rg.evals,
                            "converged": rg.converged, "max_rel_err": rg.max_rel_err,
                            "pairs_per_pass": int(inst.n) * M1 * M1,
                            "paper": "50.5 s on one A100 in FP64 for its EBSD grain map (N = 4587, "
                                     "1 %); 266 s for its Algorithm 3 run (2 %, 5 Lloyd steps)"}
    if args.coarse_eps > 0:
        # the first fit of Algorithm 3 (uniform seeds, 2 %) plain and with the
        # coarse-to-fine start
        cs = {"coarse_eps": args.coarse_eps}
        for key, ce in (("plain", 0.0), ("coarse_start", args.coarse_eps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rf = ctx.apd_fit_weights(prob, eps=0.02, coarse_eps=ce)
            torch.cuda.synchronize()
            cs[key] = {"seconds": time.perf_counter() - t0, "evals": rf.evals,
                       "coarse_evals": rf.coarse_evals, "converged": rf.converged}
        out["first_fit"] = cs
    return out


def bench_pass(args, workload: str, steps: int, warmup: int, fit_runs: int, lloyd: int,
               with_cpu: bool, extras: bool = True):
    """Fits (Algorithm 2 from W_0 = 0 on runs 0..fit_runs-1, then `lloyd`
    steps of Algorithm 3 on run 0), then `steps` timed passes over every
    pair at the resulting weights; with `extras` the culled, bf16, W = 0 and
    labelled passes as well."""
    import numpy as np
    import torch

    import apd_synth as S
    import paper_2403_03571_amd as apd

    inst = S.make(workload)
    prob = apd.Problem.from_instance(inst, "cuda:0")
    ctx = apd.Context(0)
    ctx.apd_set_variant(args.variant)
    ctx.apd_set_pixels_per_lane(args.pixels_per_lane)

    # Algorithm 2 from W_0 = 0 (metric 2) on runs 0..R-1 of the workload; run
    # 0 also gives the realistic weights the passes are timed at.  Module load
    # and first launches are excluded by one untimed fit of run 0.
    ctx.apd_fit_weights(prob, eps=0.01, prec=args.prec)
    fits = []
    w = None
    for run in range(max(1, fit_runs)):
        inst_r = inst if run == 0 else S.make(workload, run)
        prob_r = prob if run == 0 else apd.Problem.from_instance(inst_r, "cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w_r, rep = ctx.apd_fit_weights(prob_r, eps=0.01, prec=args.prec)
        torch.cuda.synchronize()
        fits.append({"run": run, "seconds": time.perf_counter() - t0, "converged": rep.converged,
                     "iters": rep.iters, "evals": rep.evals, "max_rel_err": rep.max_rel_err})
        if run == 0:
            w = w_r
        print(f"# {workload} fit: {fits[-1]}", file=sys.stderr, flush=True)
    fs = np.array([f["seconds"] for f in fits])
    fit_stats = {"runs": len(fits), "seconds_mean": float(fs.mean()), "seconds_min": float(fs.min()),
                 "seconds_max": float(fs.max()),
                 "evals_mean": float(np.mean([f["evals"] for f in fits])),
                 "iters_mean": float(np.mean([f["iters"] for f in fits])),
                 "all_converged": bool(all(f["converged"] for f in fits))}
    out = {"fit": dict(fits[0]), "fit_runs": fit_stats}
    if args.coarse_eps > 0:
        # the same runs with the coarse-to-fine start (apd_fit_opts.coarse_eps)
        fc = []
        for run in range(max(1, fit_runs)):
            prob_r = prob if run == 0 else apd.Problem.from_instance(S.make(workload, run), "cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rep = ctx.apd_fit_weights(prob_r, eps=0.01, prec=args.prec, coarse_eps=args.coarse_eps)
            torch.cuda.synchronize()
            fc.append((time.perf_counter() - t0, rep))
        tc = np.array([t for t, _ in fc])
        out["fit_runs_coarse_start"] = {
            "coarse_eps": args.coarse_eps, "runs": len(fc), "seconds_mean": float(tc.mean()),
            "seconds_min": float(tc.min()), "seconds_max": float(tc.max()),
            "evals_mean": float(np.mean([r.evals for _, r in fc])),
            "coarse_evals_mean": float(np.mean([r.coarse_evals for _, r in fc])),
            "all_converged": bool(all(r.converged for _, r in fc))}
        print(f"# {workload} coarse-start fits: {out['fit_runs_coarse_start']}", file=sys.stderr, flush=True)
    if lloyd:
        steps_l = []
        x = prob.x.clone()
        t0 = time.perf_counter()
        for k in range(lloyd):
            x, w, r = ctx.apd_lloyd_step(prob, x, w, eps=0.01, prec=args.prec)
            steps_l.append({"iters": r.iters, "evals": r.evals, "converged": r.converged})
            print(f"# {workload} lloyd {k}: {steps_l[-1]}", file=sys.stderr, flush=True)
        prob_final = apd.Problem(prob.dim, prob.grid, prob.lo, prob.hi, x, prob.A, prob.v)
        w, r = ctx.apd_fit_weights(prob_final, w=w, eps=0.01, prec=args.prec)
        torch.cuda.synchronize()
        steps_l.append({"final_fit_iters": r.iters, "evals": r.evals, "converged": r.converged,
                        "seconds_total": time.perf_counter() - t0})
        prob = prob_final
        out["lloyd"] = steps_l

    def timed_passes(prec, reps):
        """(kernel ms, pass ms, rechecked) lists over reps passes with HIP events."""
        ctx.apd_set_profiling(True)
        cms, pms, rch = [], [], []
        for _ in range(reps):
            ctx.apd_dual_objective_grad(prob, w, prec=prec)
            st = ctx.apd_last_pass_stats()
            cms.append(st["assign_ms"])
            pms.append(st["pass_ms"])
            rch.append(st["rechecked"])
        ctx.apd_set_profiling(False)
        return cms, pms, rch

    if extras and args.prec == "fp32" and args.variant >= 1:
        # the per-tile candidate lists: the same result with less work
        ctx.apd_set_culling(True)
        for _ in range(warmup):
            ctx.apd_dual_objective_grad(prob, w, prec=args.prec)
        cms, pms, _ = timed_passes(args.prec, steps)
        labels = ctx.apd_assign(prob, w, prec=args.prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.apd_assign(prob, w, labels=labels, prec=args.prec)
        torch.cuda.synchronize()
        assign_culled_ms = (time.perf_counter() - t0) / steps * 1e3
        del labels
        out["culled_pass"] = {"kernel": kernel_name(args, inst, cull=True),
                              "kernel_ms": float(np.mean(cms)), "pass_ms": float(np.mean(pms)),
                              "effective_pairs_per_s": inst.pairs / (float(np.mean(pms)) * 1e-3),
                              "assign_with_labels_ms": assign_culled_ms}
        # the bf16 tier (matrix-core costs, FP32 re-evaluation of each
        # pixel's winning group, double re-check of the uncertified pixels)
        bf_args = argparse.Namespace(**{**vars(args), "prec": "bf16"})
        ctx.apd_set_culling(False)
        for _ in range(warmup):
            ctx.apd_dual_objective_grad(prob, w, prec="bf16")
        cms, pms, rch = timed_passes("bf16", steps)
        bf16 = {"kernel": kernel_name(bf_args, inst),
                "kernel_ms": float(np.mean(cms)), "pass_ms": float(np.mean(pms)),
                "pairs_per_s": inst.pairs / (float(np.mean(pms)) * 1e-3),
                "rechecked_pixels": int(rch[-1])}
        ctx.apd_set_culling(True)
        for _ in range(warmup):
            ctx.apd_dual_objective_grad(prob, w, prec="bf16")
        cms, pms, rch = timed_passes("bf16", steps)
        bf16["culled"] = {"kernel": kernel_name(bf_args, inst, cull=True),
                          "kernel_ms": float(np.mean(cms)), "pass_ms": float(np.mean(pms)),
                          "effective_pairs_per_s": inst.pairs / (float(np.mean(pms)) * 1e-3),
                          "rechecked_pixels": int(rch[-1])}
        out["bf16_pass"] = bf16
    # every pass below evaluates every pixel-seed pair
    ctx.apd_set_culling(False)
    if extras:
        # the paper's test (a) setting: the same pass at W = 0; and Algorithm
        # 1 alone with the labels written (apd_assign)
        w0 = torch.zeros_like(w)
        extra_reps = max(3, steps // 5)
        ctx.apd_dual_objective_grad(prob, w0, prec=args.prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(extra_reps):
            ctx.apd_dual_objective_grad(prob, w0, prec=args.prec)
        torch.cuda.synchronize()
        pass_w0_ms = (time.perf_counter() - t0) / extra_reps * 1e3
        labels = ctx.apd_assign(prob, w, prec=args.prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(extra_reps):
            ctx.apd_assign(prob, w, labels=labels, prec=args.prec)
        torch.cuda.synchronize()
        assign_labels_ms = (time.perf_counter() - t0) / extra_reps * 1e3
        del labels
        out["pass_at_w0"] = {"ms": pass_w0_ms, "pairs_per_s": inst.pairs / (pass_w0_ms * 1e-3)}
        out["assign_with_labels"] = {"ms": assign_labels_ms,
                                     "pairs_per_s": inst.pairs / (assign_labels_ms * 1e-3)}

    # (one output buffer for all passes)
    gbuf = torch.empty(inst.n, dtype=torch.float64, device="cuda:0")
    for _ in range(warmup):
        ctx.apd_dual_objective_grad(prob, w, prec=args.prec, grad=gbuf)
    # the timed region: K passes, nothing else
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.apd_dual_objective_grad(prob, w, prec=args.prec, grad=gbuf)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the same passes again with HIP events around the assignment kernel and
    # the whole pass, on the library's stream (the roofline's kernel time)
    assign_ms, pass_ms, rch = timed_passes(args.prec, steps)
    ctx.apd_set_culling(True)

    pairs = inst.pairs
    a_ms = float(np.mean(assign_ms))
    achieved = OPS_PER_PAIR * pairs / (a_ms * 1e-3)
    kname = kernel_name(args, inst)
    out.update({
        "value": pairs * steps / el,
        "ms_per_step": el / steps * 1e3,
        "pixels": inst.J, "seeds": inst.n, "pairs_per_pass": pairs,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": MI355X_VALU_PEAK / 1e12,
                     "unit": "Tops/s", "frac": achieved / MI355X_VALU_PEAK,
                     "traffic": measured_traffic(kname, workload),
                     "kernel": kname, "kernel_ms": a_ms, "ops_per_pair": OPS_PER_PAIR,
                     "op": "algorithmic lane operations per pair (2 fused multiply-adds, 1 minimum)"},
        "pass_ms_events": float(np.mean(pass_ms)),
        "pass_ms_events_median_min_max": [float(np.median(pass_ms)), float(np.min(pass_ms)),
                                          float(np.max(pass_ms))],
        "kernel_ms_median_min_max": [float(np.median(assign_ms)), float(np.min(assign_ms)),
                                     float(np.max(assign_ms))],
        "rechecked_pixels": int(rch[-1]),
        "time_to_1pct_s": fit_stats["seconds_mean"],
    })
    if "fit_runs_coarse_start" in out:
        out["time_to_1pct_coarse_start_s"] = out["fit_runs_coarse_start"]["seconds_mean"]
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, w.cpu().numpy())
        # the oracle's fit, extrapolated from its pass rate and the number
        # of evaluations the fits above took (labelled as such)
        out["cpu_fit_extrapolated_s"] = {
            "seconds": pairs * fit_stats["evals_mean"] / out["cpu_baseline"]["value"],
            "how": "oracle pass rate x mean evaluations of the GPU fits (an extrapolation, not a run)"}
    ctx.close()
    return out


def bench_adaptive(args, M: int = 4096, steps: int = 20):
    """The boundary-aware refinement on the 2D workload at a fine grid
    (M x M, N = 1000, weights fitted there): the pass over the candidate
    lists with tiles inside one cell credited whole, the same pass pixel by
    pixel, and the pass over every pair -- all with identical results."""
    import numpy as np
    import torch

    import apd_synth as S
    import paper_2403_03571_amd as apd
    inst = S.make_c2(M=M)
    prob = apd.Problem.from_instance(inst, "cuda:0")
    ctx = apd.Context(0)
    w, rep = ctx.apd_fit_weights(prob, eps=0.01)
    out = {"workload": f"2D unit square, {M}x{M} pixels, N=1000 (the 2D workload's seeds), "
                       "weights fitted to 1% on this grid",
           "fit": {"seconds": rep.seconds, "evals": rep.evals, "converged": rep.converged}}

    def timed(reps):
        for _ in range(3):
            ctx.apd_dual_objective_grad(prob, w)
        ctx.apd_set_profiling(True)
        cms, pms = [], []
        for _ in range(reps):
            ctx.apd_dual_objective_grad(prob, w)
            st = ctx.apd_last_pass_stats()
            cms.append(st["assign_ms"])
            pms.append(st["pass_ms"])
        ctx.apd_set_profiling(False)
        return float(np.mean(cms)), float(np.mean(pms)), st

    for name, cull, adapt in (("adaptive", True, True), ("lists", True, False), ("every_pair", False, True)):
        ctx.apd_set_culling(cull)
        ctx.apd_set_adaptive(adapt)
        k, p_, st = timed(steps if cull else max(3, steps // 4))
        out[name] = {"kernel_ms": k, "pass_ms": p_, "tiles_credited": st["tiles_credited"],
                     "rechecked": st["rechecked"]}
    ctx.apd_set_culling(True)
    ctx.apd_set_adaptive(True)
    tiles = ((M + 31) // 32) ** 2
    out["tiles"] = tiles
    out["speedup_vs_lists"] = out["lists"]["pass_ms"] / out["adaptive"]["pass_ms"]
    ctx.close()
    torch.cuda.synchronize()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "microstructure"])
    ap.add_argument("--no-c2", action="store_true",
                    help="with the default 3D workload, skip the 2D figures reported beside it")
    ap.add_argument("--batch", type=int, default=512, help="instances of the batched workload")
    ap.add_argument("--variant", type=int, default=2,
                    help="single-precision kernel over every seed: 0 matrix cores, 1 vector ALU, "
                         "2 hybrid from 1536 seeds on 128 hybrid tiles, else vector (default), 3 hybrid")
    ap.add_argument("--pixels-per-lane", type=int, default=0,
                    help="tile shape of the vector kernel: 4, 8 or 0 (automatic)")
    ap.add_argument("--lloyd", type=int, default=None,
                    help="generalised Lloyd steps after the fit (Algorithm 3); default 5 for c3, "
                         "else 0")
    ap.add_argument("--fit-runs", type=int, default=10,
                    help="instances (runs 0..R-1 of the workload) fitted from W_0 = 0 for the "
                         "time-to-1%% statistics")
    ap.add_argument("--coarse-eps", type=float, default=0.05,
                    help="tolerance of the coarse-to-fine start (fit on the grid halved per axis "
                         "first) timed beside the plain fits; 0: not timed")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4,
                          "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_2403_03571_amd as apd

    torch.cuda.set_device(0)
    if args.workload == "c4":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.workload == "microstructure":
        print(json.dumps(bench_microstructure(args)), flush=True)
        return
    if args.lloyd is None:
        args.lloyd = 5 if args.workload == "c3" else 0
    r = bench_pass(args, args.workload, args.steps, args.warmup, args.fit_runs, args.lloyd,
                   with_cpu=not args.no_cpu_baseline)
    out = {
        "metric": "pixel-seed pairs/s in assign+reduce pass",
        "value": r.pop("value"),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16"}[args.prec],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "pixels": r.pop("pixels"),
                   "seeds": r.pop("seeds"), "pairs_per_pass": r.pop("pairs_per_pass")},
    }
    out["roofline"] = r.pop("roofline")
    # the ALU's issue rate measured on this device beside the derived peak
    try:
        fma = apd.apd_measure_valu_rate(0, "fma")
        add = apd.apd_measure_valu_rate(0, "add")
        out["roofline"]["peak_probe"] = {
            "fma_lane_ops_per_s": fma, "add_lane_ops_per_s": add,
            "fma_frac_of_peak": fma / MI355X_VALU_PEAK, "add_frac_of_peak": add / MI355X_VALU_PEAK,
            "how": "apd_measure_valu_rate: 8 independent register chains per thread, 8 waves per SIMD"}
    except Exception as e:  # the headline does not depend on it
        out["roofline"]["peak_probe"] = {"error": str(e)}
    if "cpu_baseline" in r:
        out["cpu_baseline"] = r.pop("cpu_baseline")
    out.update(r)
    if args.workload == "c3" and not args.no_c2:
        # the 2D workload beside the 3D headline (1024^2 pixels, N = 1000)
        c2 = bench_pass(args, "c2", args.steps, args.warmup, args.fit_runs, 0, with_cpu=False)
        c2["workload"] = WORKLOADS["c2"]
        out["c2"] = c2
        # the boundary-aware refinement, reported apart from the headline
        out["adaptive_refinement"] = bench_adaptive(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
