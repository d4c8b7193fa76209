#!/usr/bin/env python3
"""Benchmark of the FOT hot path on one MI355X.

A step is one full fot_solve of the 1024 x 1024 two-Gaussian -> ellipses-and-rings workload
(FP32 operands, eps 5e-3, 200 iterations of Algorithm 1, then the phase read-out of Eq. 9-10
and the final reductions), with inputs resident in HBM.  The value is whole-job throughput in
Mpixel.iterations/s = n^2 * iterations * steps / elapsed.

Also reported:
  roofline      the dominant kernel, pass 2 of the fused half-step: 2 n^3 flop per launch over
                its HIP-event-timed average launch duration on the solve's stream, against the
                FP32 MFMA peak (157.3 TFLOP/s); pass 1 and the two-pass mean beside it, and the
                committed rocprofv3 trace's figures for the same kernels.
  cpu_baseline  the FP64 oracle (separable form) timed on the host cores on a bounded sample
                of the same workload (first `--cpu-iters` iterations).
  variants      the same workload with BF16 and FP16 operands, and the BF16/FP32 speed ratio
                at equal marginal L1 error (first iteration reaching the common error level).
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel·iter/s at 1024²; %MFMA/HBM peak; BF16 vs FP32 at equal marginal L1"
# BF16x3 executes three BF16 matrix-core products per algorithmic product: its peak in
# algorithmic FLOP/s is a third of BF16's
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "f64": 78.6, "bf16x3": 2500.0 / 3}
HBM_PEAK_GBS = 8000.0
# operand bytes per element of each precision (BF16x3: a hi and a lo half)
OPERAND_BYTES = {"f32": 4, "bf16": 2, "f16": 2, "f64": 8, "bf16x3": 4}


def alg_bytes_per_launch(n, prec):
    """Algorithmic HBM bytes of one fused launch, the mean of the two passes of a half-step:
    pass 1 reads the operand and writes the transposed intermediate (2 s bytes per pixel), pass 2
    reads the intermediate, ln m and the potential, writes the potential and the next operand
    (24 + 2 s).  Lambda (n^2 s) is shared by every launch and stays in the caches."""
    s = OPERAND_BYTES[prec]
    return n * n * (12 + 2 * s)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_fused_twogauss_1024.md")
TRACE_FILE = os.path.join(ROOT, "profiles", "k_fused_{prec}_twogauss_1024.md")


# the sources the fused half-step kernels are compiled from (their launch code in fot_api.hip
# passes only sizes and pointers)
FUSED_SOURCES = ("fot_fused.hpp", "fot_kernels.hpp")


def kernel_source_hash():
    """sha256 over the fused kernels' sources (file name and bytes)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2512_19072_amd", "csrc")
    for f in FUSED_SOURCES:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(prec):
    """HBM-side bytes per fused-kernel launch (mean of the two passes) from the committed
    FETCH_SIZE / WRITE_SIZE summary, scaled by the copy calibration; None when the summary
    is missing or was taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != kernel_source_hash() or prec not in blob:
        return None
    return round(float(blob[prec]["bytes_per_launch"]))


def traced_passes(prec):
    """Per-pass average launch times of the fused kernels from the committed rocprofv3 kernel-trace
    summary of this workload (its json block), or None when it is missing or was taken on other
    kernel sources."""
    try:
        with open(TRACE_FILE.format(prec=prec)) as fh:
            text = fh.read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != kernel_source_hash():
        return None
    return float(blob["pass1_avg_us"]), float(blob["pass2_avg_us"])


def pass_times(reps):
    """Mean HIP-event time (ms) of pass-1 and pass-2 launches over profiled solves: the launches
    alternate pass 1, pass 2 (two per half-step)."""
    import numpy as np
    l1, l2 = [], []
    for r in reps:
        ms = np.asarray(r.ms_launches[:r.n_contract])
        l1.append(ms[0::2])
        l2.append(ms[1::2])
    return float(np.mean(np.concatenate(l1))), float(np.mean(np.concatenate(l2)))


def run_variant(F, W, torch, precision, g, G, eps, iters, steps, warmup, profile=True, graph=True, history=True,
                cfot=False, keep=None, tail=None, tail_iters=0, check=True, small_tiles=False):
    """Time `steps` solves after `warmup`; returns (elapsed s, reports).  With a dict `keep`, the last
    solve's potentials and phase of target 0 are copied into it (after the timed region)."""
    n = g.shape[-1]
    dev = torch.device("cuda", 0)
    gd = torch.tensor(g, dtype=torch.float64, device=dev)
    Gd = torch.tensor(G, dtype=torch.float64, device=dev)
    plan = F.Plan(n, G.shape[0], precision, max_iters=iters, profile=profile, graph=graph, history=history,
                  cfot=cfot, tail_precision=tail, tail_iters=tail_iters, small_tiles=small_tiles)
    phase = torch.empty((G.shape[0], n, n), dtype=torch.float64, device=dev)
    try:
        for _ in range(warmup):
            plan.solve(gd, Gd, eps, iters, out=phase, check=check)
    except Exception:
        plan.close()
        raise
    torch.cuda.synchronize()
    # no allocations and no garbage collection inside the timed region
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        reps = []
        for _ in range(steps):
            _, rep, st = plan.solve(gd, Gd, eps, iters, out=phase, check=check)
            rep.status = st
            reps.append(rep)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        if keep is not None:
            f_, psi_ = plan.potentials()
            keep.update(f=f_[0].cpu().numpy(), psi=psi_[0].cpu().numpy(), phase=phase[0].cpu().numpy(),
                        dual=float(reps[-1].dual[0]), cost=float(reps[-1].transport_cost[0]))
    finally:
        gc.enable()
        plan.close()
    return elapsed, reps


def gauge_rel(x, ref, w):
    """max |x - ref| / (max ref - min ref) over finite entries after removing each one's w-weighted
    mean (potentials are defined up to (f + k, psi - k)); inf if the finite sets differ."""
    import numpy as np
    m = np.isfinite(ref)
    if not np.array_equal(np.isfinite(x), m):
        return float("inf")
    xs = x[m] - np.sum(w[m] * x[m]) / np.sum(w[m])
    rs = ref[m] - np.sum(w[m] * ref[m]) / np.sum(w[m])
    return float(np.max(np.abs(xs - rs)) / np.ptp(rs))


def errors_vs_oracle(out, ref, a, b):
    """Range-normalised, gauge-fixed errors of one solve's outputs against the oracle's."""
    import numpy as np
    return {"f": gauge_rel(out["f"], ref.f, a), "psi": gauge_rel(out["psi"], ref.psi, b),
            "phase": float(np.max(np.abs(out["phase"] - ref.phase)) / np.ptp(ref.phase)),
            "dual": abs(out["dual"] - ref.dual) / abs(ref.dual),
            "transport_cost": abs(out["cost"] - ref.cost) / abs(ref.cost)}


def adjoint_steps(F, W, torch, np, steps, warmup, checkpoint_every=None):
    """The reverse-mode workload (workload 4: 512^2, 8 targets, FP32 operands, 100 iterations,
    checkpoints every 10, or every `checkpoint_every`): `warmup` then `steps` forward solves with
    tape and fot_backward of L = D + 1/2 sum_p a_p phi_p^2, each timed wall-clock between stream
    synchronisations; returns the summed forward and backward seconds."""
    wl4 = W.workload(4)
    g4, G4 = wl4.images()
    dev = torch.device("cuda", 0)
    g4d = torch.tensor(g4, dtype=torch.float64, device=dev)
    G4d = torch.tensor(G4, dtype=torch.float64, device=dev)
    a4 = torch.tensor(g4 ** 2 / np.sum(g4 ** 2), dtype=torch.float64, device=dev)
    B4, n4, T4 = G4.shape[0], wl4.n, wl4.iters
    plan = F.Plan(n4, B4, "f32", max_iters=T4, checkpoint_every=checkpoint_every or wl4.checkpoint_every)
    ph4 = torch.empty((B4, n4, n4), dtype=torch.float64, device=dev)
    dD = np.ones(B4)
    try:
        for _ in range(warmup):
            plan.solve(g4d, G4d, float(wl4.eps[0]), T4, out=ph4)
            plan.backward(dD, (a4[None] * ph4).contiguous())
        torch.cuda.synchronize()
        tf = tb = 0.0
        for _ in range(steps):
            t0 = time.perf_counter()
            plan.solve(g4d, G4d, float(wl4.eps[0]), T4, out=ph4)
            dphi = (a4[None] * ph4).contiguous()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            plan.backward(dD, dphi)
            torch.cuda.synchronize()
            tf += t1 - t0
            tb += time.perf_counter() - t1
    finally:
        plan.close()
    return tf, tb


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-iters", type=int, default=200, help="oracle iterations in the CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch the iteration loop kernel by kernel")
    ap.add_argument("--precision", default="f32", choices=["f64", "f32", "bf16", "f16", "bf16x3"],
                    help="operand precision of the headline run (profiling aid; the headline is f32)")
    ap.add_argument("--cfot-run", action="store_true",
                    help="profiling aid: only the headline workload's solves with cFOT (FP64 FFT convolutions), "
                         "graph-replayed and then kernel by kernel, and one JSON line of their rates")
    ap.add_argument("--eps", type=float, default=None,
                    help="profiling aid: run the headline workload at this eps instead of its own (the "
                         "config then names it); e.g. the paper's 2e-4")
    ap.add_argument("--adjoint-run", action="store_true",
                    help="profiling aid: only the reverse-mode workload (gauss_to_ellipses 512x512, 8 targets, "
                         "100 iterations, checkpoints every 10, FP32): --warmup then --steps forward solves with "
                         "their backward passes, and one JSON line of the times")
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for hardware-counter passes: two solves launched kernel by kernel "
                         "and one 256 MiB device-to-device copy whose bytes calibrate the counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: one GPU only: the FOT solve is measured on one MI355X (sharding across "
              "GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2512_19072_amd import fot as F
    from paper_2512_19072_amd import workloads as W

    wl = W.workload(1)
    n, iters, eps = wl.n, wl.iters, float(wl.eps[0])
    if args.eps is not None:
        eps = float(args.eps)
    g, G = wl.images()
    if args.pmc_run:
        run_variant(F, W, torch, args.precision, g, G, eps, iters, 1, 1, profile=False, graph=False)
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_run": True, "precision": args.precision, "solves": 2, "iters": iters,
                          "copy_bytes": nbytes}), flush=True)
        return
    if args.adjoint_run:
        tf, tb = adjoint_steps(F, W, torch, np, args.steps, args.warmup)
        print(json.dumps({"adjoint_run": True, "steps": args.steps, "ms_forward": round(1e3 * tf / args.steps, 3),
                          "ms_backward": round(1e3 * tb / args.steps, 3)}), flush=True)
        return
    if args.cfot_run:
        el, rp = run_variant(F, W, torch, "f64", g, G, eps, iters, args.steps, args.warmup, profile=False,
                             graph=not args.no_graph, cfot=True)
        _, rpp = run_variant(F, W, torch, "f64", g, G, eps, iters, args.steps, args.warmup, profile=True,
                             graph=False, cfot=True)
        pass_us = 1e3 * sum(r.ms_contract for r in rpp) / max(1, sum(r.n_contract for r in rpp))
        print(json.dumps({"cfot_run": True, "value": round(n * n * iters * args.steps / el / 1e6, 3),
                          "unit": "Mpixel·iter/s", "steps": args.steps, "pass_avg_us": round(pass_us, 3)}),
              flush=True)
        return
    prec0 = args.precision
    log(f"bench: workload {wl.name} n={n} iters={iters} eps={eps} {prec0}, steps={args.steps} warmup={args.warmup}")
    graph = not args.no_graph
    # (a profiling run at another eps keeps going past a reported loss of range: its status is
    # printed, and the kernels are what it is for)
    check = args.eps is None
    # timed region 1: the production launch path (graph replay of the iteration loop)
    finals = {prec0: {}}
    elapsed, reps = run_variant(F, W, torch, args.precision, g, G, eps, iters, args.steps, args.warmup,
                                profile=False, graph=graph, keep=finals[prec0], check=check)
    if not check:
        log(f"bench: status {F.STATUS_NAMES.get(reps[-1].status, reps[-1].status)} at eps {eps}")
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * n * iters * args.steps / elapsed / 1e6
    # timed region 2: the same steps launched kernel by kernel with HIP events around every
    # contraction GEMM on the solve's stream (events cannot be timed inside a graph)
    el_prof, reps_prof = run_variant(F, W, torch, args.precision, g, G, eps, iters, args.steps, args.warmup,
                                     profile=True, graph=False, check=check)
    ms_gemm = sum(r.ms_contract for r in reps_prof) / max(1, sum(r.n_contract for r in reps_prof))
    ms_p1, ms_p2 = pass_times(reps_prof)
    flop = 2.0 * n ** 3
    # the dominant kernel is pass 2 (the longer of the two launches of every half-step)
    achieved = flop / (ms_p2 * 1e-3) / 1e12
    achieved_mean = flop / (ms_gemm * 1e-3) / 1e12
    traced = traced_passes(prec0)
    ms_iter0 = float(np.median([r.ms_iterations for r in reps])) / iters
    # device memory of one plan of the headline solve (its O(n^2) workspace: FP64 state, the
    # operands, the FP64 read-out buffers), measured as the drop in free device memory
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    mplan = F.Plan(n, 1, prec0, max_iters=iters)
    torch.cuda.synchronize()
    plan_mib = (free0 - torch.cuda.mem_get_info()[0]) / 2 ** 20
    mplan.close()
    log(f"bench: {prec0} {value:.1f} Mpx.it/s, {ms_per_step:.2f} ms/step, fused kernel pass 1 {ms_p1 * 1e3:.2f} us, "
        f"pass 2 {ms_p2 * 1e3:.2f} us ({achieved:.1f} TFLOP/s), iteration loop {ms_iter0 * 1e3:.1f} us/it, "
        f"final err_a {reps[-1].err_a[0]:.3e}; trace {traced}")

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpixel·iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec0,
        "data": "synthetic",
        "config": {"workload": "twogauss_to_shapes", "n": n, "iters": iters, "eps": eps, "batch": 1,
                   "precision": prec0, "seed": 0, "graph": bool(reps[-1].graph)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[prec0],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[prec0], 4),
                     "traffic": measured_traffic(prec0),
                     "kernel": "fot::k_fused pass 2 (Lambda . Bt^T with the fused potential update, marginal-"
                               "error partial and next operand; 2 n_p^3 flop per launch): the longer of the "
                               "two launches of every half-step",
                     "avg_launch_us": round(ms_p2 * 1e3, 3),
                     "pass1_avg_launch_us": round(ms_p1 * 1e3, 3),
                     "pass1_frac": round(flop / (ms_p1 * 1e-3) / 1e12 / PEAK_TFLOPS[prec0], 4),
                     "two_pass_mean_frac": round(achieved_mean / PEAK_TFLOPS[prec0], 4),
                     "trace": (None if traced is None else {
                         "pass1_avg_us": traced[0], "pass2_avg_us": traced[1],
                         "frac": round(flop / (traced[1] * 1e-6) / 1e12 / PEAK_TFLOPS[prec0], 4),
                         "two_pass_mean_frac": round(flop / (0.5 * (traced[0] + traced[1]) * 1e-6) / 1e12
                                                     / PEAK_TFLOPS[prec0], 4),
                         "source": f"profiles/k_fused_{prec0}_twogauss_1024.md (rocprofv3 kernel trace of the "
                                   "same command, on the current kernel sources)"}),
                     # the same launches against HBM: algorithmic bytes (n^2 (12 + 2 s) per launch,
                     # Lambda cache-resident) and, when counted, the HBM-side bytes
                     "hbm_frac_algorithmic": round(alg_bytes_per_launch(n, prec0) / (ms_gemm * 1e-3) / 1e9
                                                   / HBM_PEAK_GBS, 4),
                     "hbm_frac_counted": (round(measured_traffic(prec0) / (ms_gemm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                          if measured_traffic(prec0) else None),
                     "hbm_note": "the HBM fractions and traffic are per launch over both passes (mean)",
                     "traffic_note": "HBM-side bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated, "
                                     "mean of the two passes) from profiles/traffic_k_fused_twogauss_1024.md",
                     "timing": "HIP events around every fused-kernel launch over a second timed region of "
                               f"{args.steps} steps launched kernel by kernel "
                               f"({1e3 * el_prof / args.steps:.2f} ms/step)"},
        "final_err_a": float(reps[-1].err_a[0]),
        "plan_device_mib": round(plan_mib, 1),
    }

    if not args.no_variants:
        # Operand precisions compared with FP32 at equal marginal L1 error.  The error of a solve
        # of T iterations is the FP64 read-out's row-marginal L1 of the final plan (err_a), which
        # for 16-bit operands plateaus at the precision floor.  For each precision, fresh solves of
        # T = 1, ..., 60 and then every 5th T up to iters give err(T).  Each precision p is compared
        # with FP32 at E_p = 1.1 max(floor of p, FP32's error at T = iters), the level both reach
        # (the margin keeps E_p off the noise of p's plateau); each one's time to E_p is its first
        # such T times its graph-replayed iteration time.
        grid = list(range(1, min(60, iters) + 1)) + list(range(65, iters + 1, 5))

        def err_curve(prec):
            dev = torch.device("cuda", 0)
            gd = torch.tensor(g, dtype=torch.float64, device=dev)
            Gd = torch.tensor(G, dtype=torch.float64, device=dev)
            plan = F.Plan(n, G.shape[0], prec, max_iters=iters)
            errs = [float(plan.solve(gd, Gd, eps, T, phase=False)[1].err_a[0]) for T in grid]
            plan.close()
            return np.array(errs)

        per_prec = {prec0: {"ms_it": ms_iter0, "value": value, "ms_per_step": ms_per_step, "gemm_us": ms_gemm}}
        for prec in ("f32", "bf16", "f16", "bf16x3"):
            if prec in per_prec:
                continue
            finals[prec] = {}
            el, rp = run_variant(F, W, torch, prec, g, G, eps, iters, args.steps, args.warmup,
                                 profile=False, graph=graph, keep=finals[prec])
            _, rpp = run_variant(F, W, torch, prec, g, G, eps, iters, max(1, args.steps // 2), 1,
                                 profile=True, graph=False)
            per_prec[prec] = {"ms_it": float(np.median([r.ms_iterations for r in rp])) / iters,
                              "value": n * n * iters * args.steps / el / 1e6,
                              "ms_per_step": 1e3 * el / args.steps,
                              "gemm_us": 1e3 * sum(r.ms_contract for r in rpp) / max(1, sum(r.n_contract for r in rpp)),
                              "final_err_a": float(rp[-1].err_a[0])}
        curves = {prec: err_curve(prec) for prec in per_prec}

        def reach(c, lev):
            hit = np.nonzero(c <= lev)[0]
            return grid[int(hit[0])] if hit.size else None

        levels, t_reach, t_f32 = {}, {}, {}
        for prec, c in curves.items():
            if prec == "f32":
                continue
            lev = 1.1 * max(float(np.min(c)), float(curves["f32"][-1]))
            levels[prec] = lev
            t_reach[prec] = reach(c, lev)
            t_f32[prec] = reach(curves["f32"], lev)
        variants = {}
        base = per_prec["f32"]
        for prec, d in per_prec.items():
            if prec == "f32":
                continue
            sp = None
            if t_reach.get(prec) and t_f32.get(prec):
                sp = round((t_f32[prec] * base["ms_it"]) / (t_reach[prec] * d["ms_it"]), 3)
            ach = flop / (d["gemm_us"] * 1e-6) / 1e12
            hbm = alg_bytes_per_launch(n, prec) / (d["gemm_us"] * 1e-6) / 1e9
            # the same comparison at coarser levels (multiples of the level's floor term), where the
            # iteration counts meet and the ratio tends to the per-iteration one
            by_level = {}
            for mult in (1.5, 2.0, 3.0):
                lv = levels[prec] / 1.1 * mult
                ta, tb = reach(curves["f32"], lv), reach(curves[prec], lv)
                by_level[f"{mult:g}x"] = (round((ta * base["ms_it"]) / (tb * d["ms_it"]), 3)
                                          if ta and tb else None)
            variants[prec] = {"value": round(d["value"], 3), "ms_per_step": round(d["ms_per_step"], 4),
                              "speedup_vs_f32_per_iteration": round(base["ms_it"] / d["ms_it"], 3),
                              "equal_marginal_l1": {"err_level": levels[prec], "iters_f32": t_f32.get(prec),
                                                    "iters": t_reach.get(prec), "speedup_vs_f32": sp,
                                                    "speedup_at_floor_multiples": by_level},
                              "lowest_err_a": float(np.min(curves[prec])),
                              "final_err_a": d.get("final_err_a", float(reps[-1].err_a[0])),
                              "kernel_avg_launch_us": round(d["gemm_us"], 3),
                              "kernel_tflops": round(ach, 2),
                              "kernel_frac_of_peak": round(ach / PEAK_TFLOPS[prec], 4),
                              "kernel_hbm_gbs": round(hbm, 1),
                              "kernel_hbm_frac": round(hbm / HBM_PEAK_GBS, 4)}
            log(f"bench: {prec} {d['value']:.1f} Mpx.it/s, kernel {d['gemm_us']:.1f} us, "
                f"per-iteration speedup {base['ms_it'] / d['ms_it']:.2f}, equal-L1 speedup {sp} "
                f"(E = {levels[prec]:.2e}: f32 {t_f32.get(prec)} its, {prec} {t_reach.get(prec)} its)")
        out["variants"] = variants
        # Algorithm 1 as the paper times it: a fixed number of iterations without evaluating a
        # loss per iteration (FOT_FLAG_NO_HISTORY); final errors still come from the read-out.
        nh = {}
        for prec in ("f32", "bf16", "bf16x3"):
            el, rp = run_variant(F, W, torch, prec, g, G, eps, iters, args.steps, args.warmup,
                                 profile=False, graph=graph, history=False)
            nh[prec] = {"value": round(n * n * iters * args.steps / el / 1e6, 3),
                        "ms_per_step": round(1e3 * el / args.steps, 4),
                        "us_per_iteration": round(1e3 * float(np.median([r.ms_iterations for r in rp])) / iters, 2),
                        "final_err_a": float(rp[-1].err_a[0])}
            log(f"bench: {prec} without per-iteration errors {nh[prec]['value']:.1f} Mpx.it/s, "
                f"{nh[prec]['us_per_iteration']:.1f} us/it")
        out["no_history"] = nh
        # the equal-L1 comparison again with these iteration times: err(T) above is the read-out's,
        # which a solve without the per-iteration history reports just the same
        for prec in ("bf16", "bf16x3"):
            eq = variants.get(prec, {}).get("equal_marginal_l1")
            if eq and eq["iters"] and eq["iters_f32"]:
                eq["speedup_vs_f32_no_history"] = round(
                    (eq["iters_f32"] * nh["f32"]["us_per_iteration"]) / (eq["iters"] * nh[prec]["us_per_iteration"]), 3)
                log(f"bench: {prec} equal-L1 speedup without per-iteration errors "
                    f"{eq['speedup_vs_f32_no_history']}")
        # The precision schedule inside one solve (fot_plan_desc.tail_precision / tail_iters): T - k
        # BF16 iterations, then k FP32 ones.  For each level E the smallest (T, k) whose read-out
        # err_a reaches E is timed end to end as real solves, against FP32 solves of the iteration
        # count FP32 needs for E; both without the per-iteration history (the read-out's err_a is
        # what the comparison uses).  Times are the medians of the iteration loop's HIP-event time
        # (and of the whole solve, read-out included) over repeated graph-replayed solves.
        def timed(prec, T, tail=None, k=0, reps_=7):
            el_, rp_ = run_variant(F, W, torch, prec, g, G, eps, T, reps_, 2, profile=False, graph=graph,
                                   history=False, tail=tail, tail_iters=k)
            return (float(np.median([r.ms_iterations for r in rp_])), float(np.median([r.ms_total for r in rp_])),
                    float(rp_[-1].err_a[0]))

        dev = torch.device("cuda", 0)
        gd = torch.tensor(g, dtype=torch.float64, device=dev)
        Gd = torch.tensor(G, dtype=torch.float64, device=dev)
        sched = {}
        for name, lev in (("1.1x_bf16_floor", levels.get("bf16")),
                          ("f32_err_at_T40", float(curves["f32"][grid.index(40)]) if 40 in grid else None)):
            T32 = reach(curves["f32"], lev) if lev else None
            if not T32:
                continue
            best = None
            for k in (1, 2, 3):
                ps = F.Plan(n, G.shape[0], "bf16", max_iters=iters, tail_precision="f32", tail_iters=k)
                found = None
                for T in range(max(k + 1, T32 - 4), T32 + 6):
                    if float(ps.solve(gd, Gd, eps, T, phase=False)[1].err_a[0]) <= lev:
                        found = T
                        break
                ps.close()
                if found is None:
                    continue
                ms_it, ms_tot, e_ = timed("bf16", found, tail="f32", k=k)
                if best is None or ms_it < best["ms_iterations"]:
                    best = {"T": found, "k_f32": k, "err_a": e_, "ms_iterations": round(ms_it, 4),
                            "ms_solve": round(ms_tot, 4)}
            if best:
                ms32, ms32_tot, e32 = timed("f32", T32)
                best.update({"err_level": lev, "iters_f32": T32, "f32_ms_iterations": round(ms32, 4),
                             "f32_ms_solve": round(ms32_tot, 4), "f32_err_a": e32,
                             "speedup_vs_f32": round(ms32 / best["ms_iterations"], 3),
                             "speedup_vs_f32_whole_solve": round(ms32_tot / best["ms_solve"], 3)})
                sched[name] = best
                log(f"bench: bf16 then f32 in one solve at E = {lev:.2e}: {best['T'] - best['k_f32']} + "
                    f"{best['k_f32']} iterations in {best['ms_iterations']:.3f} ms against f32 alone {T32} in "
                    f"{ms32:.3f} ms: {best['speedup_vs_f32']}x (whole solves {best['speedup_vs_f32_whole_solve']}x)")
        out["precision_schedule_bf16_f32"] = sched
        out["equal_l1_protocol"] = ("err(T) = FP64 read-out row-marginal L1 after fresh solves of T = 1..60, "
                                    "then every 5th T up to iters; for each operand type p, E_p = 1.1 x "
                                    "max(lowest err of p, err of f32 at T = iters); speedup = "
                                    "T_f32(E_p) t_it,f32 / (T_p(E_p) t_it,p), t_it from graph-replayed solves "
                                    "with per-iteration errors")

    if not args.no_variants:
        # A10: the reverse mode on its own workload (512^2, 8 targets, FP32 operands, 100
        # iterations, checkpoints every 10): forward solve with tape, then fot_backward of
        # L = D + 1/2 sum_p a_p phi_p^2, each timed over the same steps.
        wl4 = W.workload(4)
        B4, n4, T4 = wl4.batch, wl4.n, wl4.iters
        tf, tb = adjoint_steps(F, W, torch, np, args.steps, args.warmup)
        out["adjoint"] = {"workload": f"{wl4.name} {n4}x{n4}, {B4} targets, eps {float(wl4.eps[0])}, {T4} iterations, "
                                      f"checkpoints every {wl4.checkpoint_every}, FP32 operands (FP32 reverse sweep)",
                          "ms_forward": round(1e3 * tf / args.steps, 3), "ms_backward": round(1e3 * tb / args.steps, 3),
                          "backward_over_forward": round(tb / tf, 3),
                          "value_forward": round(B4 * n4 * n4 * T4 * args.steps / tf / 1e6, 3),
                          "unit": "Mpixel·iter/s (targets x pixels x iterations)"}
        log(f"bench: adjoint {out['adjoint']['ms_forward']:.2f} ms forward + {out['adjoint']['ms_backward']:.2f} ms "
            f"backward per step ({B4} x {n4}^2, {T4} its)")
        # the same with every iterate kept by the forward solve (one checkpoint segment of T
        # iterations, the plan's segment buffers holding f, psi, ln S, ln S' of each: the backward
        # pass replays nothing), the memory-for-time end of the checkpoint trade-off
        tfk, tbk = adjoint_steps(F, W, torch, np, args.steps, args.warmup, checkpoint_every=T4)
        out["adjoint"]["every_iterate_kept"] = {
            "checkpoint_every": T4, "ms_forward": round(1e3 * tfk / args.steps, 3),
            "ms_backward": round(1e3 * tbk / args.steps, 3), "backward_over_forward": round(tbk / tfk, 3),
            "segment_buffers_gib": round(4 * T4 * B4 * n4 * n4 * 8 / 2 ** 30, 2)}
        log(f"bench: adjoint with every iterate kept: {1e3 * tfk / args.steps:.2f} ms forward + "
            f"{1e3 * tbk / args.steps:.2f} ms backward per step")

        # output beam and L1 intensity loss of the FP32 phase of the headline workload, and
        # Gerchberg-Saxton rounds from it (FP64 transforms on the matrix cores)
        dev = torch.device("cuda", 0)
        gd = torch.tensor(g, dtype=torch.float64, device=dev)
        Gd = torch.tensor(G, dtype=torch.float64, device=dev)
        plan = F.Plan(n, G.shape[0], "f32", max_iters=iters)
        ph, _, _ = plan.solve(gd, Gd, eps, iters)
        _, l_fot = plan.output_beam(gd, ph, Gd, intensity=False)
        torch.cuda.synchronize()
        reps_b = max(1, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(reps_b):
            plan.output_beam(gd, ph, Gd, intensity=False)
        t_beam = (time.perf_counter() - t0) / reps_b
        gs_rounds = 10
        ph_gs = ph.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.polish_gs(gd, Gd, ph_gs, gs_rounds)
        t_gs = (time.perf_counter() - t0) / gs_rounds
        _, l_gs = plan.output_beam(gd, ph_gs, Gd, intensity=False)
        _, l_flat = plan.output_beam(gd, torch.zeros_like(ph), Gd, intensity=False)
        plan.close()
        tflop = 16.0 * n ** 3 / t_beam / 1e12
        out["output_beam"] = {"workload": f"{wl.name} {n}x{n}: FP32 FOT phase after {iters} iterations",
                              "ms_output_beam": round(1e3 * t_beam, 3), "ms_per_gs_round": round(1e3 * t_gs, 3),
                              "transform_tflops_fp64": round(tflop, 2),
                              "l1_flat_phase": float(l_flat[0]), "l1_fot": float(l_fot[0]),
                              f"l1_fot_plus_{gs_rounds}_gs": float(l_gs[0])}
        log(f"bench: output beam {1e3 * t_beam:.2f} ms ({tflop:.1f} TFLOP/s FP64), GS round {1e3 * t_gs:.2f} ms; "
            f"L1 flat {l_flat[0]:.4f}, FOT {l_fot[0]:.4f}, FOT + {gs_rounds} GS {l_gs[0]:.4f}")

        # cFOT (Eq. 11): the same solve with FP64 FFT convolutions instead of the matrix products,
        # against the FP64 and FP32 matrix-product paths (speed, and accuracy against FP64)
        conv = {}
        for name, prec, cf in (("cfot_f64_fft", "f64", True), ("gemm_f64", "f64", False)):
            el, rp = run_variant(F, W, torch, prec, g, G, eps, iters, max(2, args.steps // 2), 1,
                                 profile=False, graph=graph, cfot=cf)
            _, rpp = run_variant(F, W, torch, prec, g, G, eps, iters, 1, 1, profile=True, graph=False, cfot=cf)
            steps_c = max(2, args.steps // 2)
            conv[name] = {"value": round(n * n * iters * steps_c / el / 1e6, 3),
                          "us_per_iteration": round(1e3 * float(np.median([r.ms_iterations for r in rp])) / iters, 2),
                          "pass_avg_us": round(1e3 * sum(r.ms_contract for r in rpp)
                                               / max(1, sum(r.n_contract for r in rpp)), 3),
                          "final_err_a": float(rp[-1].err_a[0])}
        conv["gemm_" + prec0] = {"value": round(value, 3), "us_per_iteration": round(1e3 * ms_iter0, 2),
                                 "pass_avg_us": round(1e3 * ms_gemm, 3), "final_err_a": float(reps[-1].err_a[0])}
        pots = {}
        for name, prec, cf in (("cfot_f64_fft", "f64", True), ("gemm_f64", "f64", False)):
            plan = F.Plan(n, G.shape[0], prec, max_iters=iters, cfot=cf)
            plan.solve(gd, Gd, eps, iters, phase=False)
            pots[name] = plan.potentials()[0].cpu().numpy()[0]
            plan.close()
        fin = np.isfinite(pots["gemm_f64"])
        dv = pots["cfot_f64_fft"][fin] - pots["gemm_f64"][fin]
        conv["cfot_f_err_vs_f64_gemm"] = float(np.max(np.abs(dv - dv.mean())) / np.ptp(pots["gemm_f64"][fin]))
        # per-iteration cost at 2048^2 (the lattice workload's size), constant eps 5e-3, 20 iterations
        n2 = 2048
        g2_, G2_ = W.speckle_to_lattice(n2)
        G2_ = G2_ if G2_.ndim == 3 else G2_[None]
        big = {}
        for name, prec, cf in (("cfot_f64_fft", "f64", True), ("gemm_f32", "f32", False), ("gemm_bf16", "bf16", False)):
            try:
                el, rp = run_variant(F, W, torch, prec, g2_, G2_, 5e-3, 20, 3, 1, profile=False, graph=graph, cfot=cf)
                big[name] = round(1e3 * float(np.median([r.ms_iterations for r in rp])) / 20, 2)
            except F.FOTError as exc:   # (cFOT can lose the small values on this target)
                big[name] = f"failed: {exc}"[:160]
        conv["us_per_iteration_2048"] = big
        out["contraction_by_fft"] = conv

        # the lattice workload at its own configuration: 2048^2, eps annealed 5e-2 -> 2e-3 over 400
        # iterations (Lambda regenerated at every eps, held block-normalised once its entries leave
        # the 32- and 16-bit range), FP32 and BF16 operands; each against its roofline: FP32 against
        # the FP32 matrix cores (8 n^3 flop per iteration), BF16 against HBM (four launches of
        # n^2 (12 + 2 s) algorithmic bytes per iteration) and its matrix cores
        wl3 = W.workload(3)
        g3, G3 = wl3.images()
        n3, T3 = wl3.n, wl3.iters
        lattice = {"workload": f"{wl3.name} {n3}x{n3}, eps annealed {wl3.eps[0]:g} -> {wl3.eps[-1]:g} over {T3} "
                               "iterations, read-out included"}
        for pp in ("f32", "bf16"):
            el, rp = run_variant(F, W, torch, pp, g3, G3, wl3.eps, T3, 2, 1, profile=False, graph=graph, check=False)
            ms_it = float(np.median([r.ms_iterations for r in rp])) / T3
            tflops = 8.0 * n3 ** 3 / (ms_it * 1e-3) / 1e12
            gbs = 4 * alg_bytes_per_launch(n3, pp) / (ms_it * 1e-3) / 1e9
            lattice[pp] = {"value": round(n3 * n3 * T3 * 2 / el / 1e6, 3), "ms_per_solve": round(1e3 * el / 2, 3),
                           "us_per_iteration": round(1e3 * ms_it, 2), "tflops": round(tflops, 2),
                           "frac_mfma": round(tflops / PEAK_TFLOPS[pp], 4),
                           "frac_hbm_algorithmic": round(gbs / HBM_PEAK_GBS, 4),
                           "status": F.STATUS_NAMES.get(rp[-1].status, str(rp[-1].status)),
                           "final_err_a": float(rp[-1].err_a[0]), "final_err_b": float(rp[-1].err_b[0])}
        out["lattice_2048_annealed"] = lattice
        log(f"bench: lattice 2048^2 annealed, 400 its: " + ", ".join(
            f"{pp} {lattice[pp]['value']:.1f} Mpx.it/s ({lattice[pp]['ms_per_solve']:.1f} ms/solve, "
            f"MFMA {lattice[pp]['frac_mfma']:.3f}, HBM {lattice[pp]['frac_hbm_algorithmic']:.3f}, "
            f"{lattice[pp]['status']})" for pp in ("f32", "bf16")))
        log(f"bench: cFOT (FP64 FFT) {conv['cfot_f64_fft']['value']:.1f} Mpx.it/s "
            f"({conv['cfot_f64_fft']['us_per_iteration']:.1f} us/it, pass {conv['cfot_f64_fft']['pass_avg_us']:.1f} us), "
            f"FP64 GEMM {conv['gemm_f64']['value']:.1f}, {prec0} GEMM {conv['gemm_' + prec0]['value']:.1f}; "
            f"cFOT f error vs FP64 GEMM {conv['cfot_f_err_vs_f64_gemm']:.1e}; at 2048^2 (us/it): {big}")

        # the paper's regime (eps = 2e-4, Sec. 4): FP64 operands, where Lambda's band (the |i - k| at
        # which it is nonzero in FP64) is about 0.55 n and the fused kernels skip the zero K stages;
        # the 32- and 16-bit forms with Lambda block-normalised (its entries span more than their
        # range there) and the same band
        paper = {"eps": 2e-4, "workload": f"twogauss_to_shapes {n}x{n}, {iters} iterations"}
        for pp in ("f64", "f32", "bf16", "f32_small_tiles"):
            ks = max(2, args.steps // 2)
            el, rp = run_variant(F, W, torch, pp.split("_")[0], g, G, 2e-4, iters, ks, 1, profile=False, graph=graph,
                                 check=False, small_tiles=pp.endswith("small_tiles"))
            paper[pp] = {"value": round(n * n * iters * ks / el / 1e6, 3),
                         "us_per_iteration": round(1e3 * float(np.median([r.ms_iterations for r in rp])) / iters, 2),
                         "final_err_a": float(rp[-1].err_a[0]), "final_err_b": float(rp[-1].err_b[0]),
                         "status": F.STATUS_NAMES.get(rp[-1].status, str(rp[-1].status)),
                         "range_loss": float(rp[-1].range_loss[0]), "range_iter": int(rp[-1].range_iter[0])}
        out["paper_eps"] = paper
        log("bench: eps 2e-4 (1024^2): " + ", ".join(
            f"{pp} {paper[pp]['value']:.1f} Mpx.it/s ({paper[pp]['us_per_iteration']:.1f} us/it, "
            f"err_b {paper[pp]['final_err_b']:.1e}, {paper[pp]['status']})" for pp in paper if pp not in ("eps", "workload")))

        # synthetic re-run of the eps sweep of Fig. 3: the L1 intensity loss of the output beam of
        # 200 iterations at 512^2, for matrix products (FP64 operands, valid down to the paper's
        # 2e-4) and for cFOT (FP64 FFT convolutions), on the two-Gaussian -> shapes stand-in
        n5 = 512
        g5, G5 = W.twogauss_to_shapes(n5)
        G5 = G5 if G5.ndim == 3 else G5[None]
        g5d = torch.tensor(g5, dtype=torch.float64, device=dev)
        G5d = torch.tensor(G5, dtype=torch.float64, device=dev)
        sweep = {"eps": [5e-2, 2e-2, 1e-2, 5e-3, 2e-3, 1e-3, 5e-4, 2e-4], "fot_f64": [], "fot_f32": [],
                 "cfot_f64": []}
        for key, pp, cf in (("fot_f64", "f64", False), ("fot_f32", "f32", False), ("cfot_f64", "f64", True)):
            plan = F.Plan(n5, 1, pp, max_iters=200, cfot=cf)
            for e5 in sweep["eps"]:
                ph5, _, st5 = plan.solve(g5d, G5d, e5, 200, check=False)
                if st5 == F.FOT_OK:
                    _, l5 = plan.output_beam(g5d, ph5, G5d, intensity=False)
                    sweep[key].append(round(float(l5[0]), 5))
                else:
                    sweep[key].append(F.STATUS_NAMES.get(st5, str(st5)))
            plan.close()
        sweep["workload"] = "twogauss_to_shapes 512x512, 200 iterations, L1 intensity loss of the output beam"
        out["eps_sweep_512"] = sweep
        log(f"bench: eps sweep 512^2 (L1 loss): eps {sweep['eps']}; FOT {sweep['fot_f64']}; "
            f"FOT (FP32 operands) {sweep['fot_f32']}; cFOT {sweep['cfot_f64']}")

        # small-grid latency (the paper's 128^2, 200 iterations): one whole solve per call,
        # inputs resident, timed wall-clock around the call
        ns = 128
        gs_, Gs_ = W.twogauss_to_shapes(ns)
        Gs_ = Gs_ if Gs_.ndim == 3 else Gs_[None]
        gsd = torch.tensor(gs_, dtype=torch.float64, device=dev)
        Gsd = torch.tensor(Gs_, dtype=torch.float64, device=dev)
        small = {}
        for prec in ("f32", "bf16"):
            plan = F.Plan(ns, 1, prec, max_iters=200)
            phs = torch.empty((1, ns, ns), dtype=torch.float64, device=dev)
            for _ in range(2):
                plan.solve(gsd, Gsd, 5e-3, 200, out=phs)
            torch.cuda.synchronize()
            ts = []
            for _ in range(5):
                t0 = time.perf_counter()
                plan.solve(gsd, Gsd, 5e-3, 200, out=phs)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            plan.close()
            small[prec] = round(1e3 * float(np.median(ts)), 3)
        out["small_grid"] = {"workload": f"twogauss_to_shapes {ns}x{ns}, eps 5e-3, 200 iterations + read-out",
                             "ms_per_solve": small}
        log(f"bench: {ns}^2 x 200 iterations: {small} ms per solve")

    if not args.no_cpu_baseline:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count()
        k = args.cpu_iters
        t0 = time.perf_counter()
        ref_cpu = oracle.solve_sep(g, G[0], eps, k)
        t_cpu = time.perf_counter() - t0
        cpu_model = "unknown CPU"
        try:
            with open("/proc/cpuinfo") as fh:
                cpu_model = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
        except (OSError, StopIteration):
            pass
        affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        out["cpu_baseline"] = {"value": round(n * n * k / t_cpu / 1e6, 3), "unit": "Mpixel·iter/s",
                               "cores": cores, "kind": "oracle",
                               "sample": f"{wl.name} {n}x{n}, eps {eps}: first {k} of {iters} iterations plus "
                                         f"read-out, FP64 separable oracle (numpy/OpenBLAS), {t_cpu:.1f} s; "
                                         f"{cpu_model}, {affinity} CPUs in this process's affinity"}
        # the same oracle restricted to one thread, on a shorter sample
        try:
            from threadpoolctl import threadpool_limits
            k1 = max(2, k // 10)
            with threadpool_limits(limits=1):
                t0 = time.perf_counter()
                oracle.solve_sep(g, G[0], eps, k1)
                t1 = time.perf_counter() - t0
            out["cpu_baseline"]["single_thread"] = {"value": round(n * n * k1 / t1 / 1e6, 3),
                                                    "sample": f"first {k1} iterations plus read-out, {t1:.1f} s"}
        except ImportError:
            pass
        log(f"bench: cpu oracle {out['cpu_baseline']['value']} Mpx.it/s on {cores} threads ({t_cpu:.1f} s)")
        # every operand type's final outputs against the oracle's (outside any timed region)
        ref = ref_cpu if k == iters else oracle.solve_sep(g, G[0], eps, iters)
        a_, b_ = oracle.normalise(g), oracle.normalise(G[0])
        for prec, fin in finals.items():
            if not fin:
                continue
            ev = {key: float(f"{val:.3e}") for key, val in errors_vs_oracle(fin, ref, a_, b_).items()}
            if prec == prec0:
                out["err_vs_oracle"] = ev
            elif prec in out.get("variants", {}):
                out["variants"][prec]["err_vs_oracle"] = ev
            log(f"bench: {prec} against the oracle: {ev}")
        out["err_vs_oracle_note"] = ("range-normalised, gauge-fixed max errors of f, psi and the phase, and relative "
                                     "errors of the dual and transport cost, against the FP64 oracle's solve of the "
                                     "same workload")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
