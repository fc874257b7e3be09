"""Benchmark of the SWF hot path on one MI355X.

One bench "step" is the whole job of the (2+1)D Schwinger workload: 64
U_out(s=+1) solves with momenta uniform in |p| < 1 on a 512 x 512 grid over
[-80, 80)^2, field A_1 = exp(-t^2/100 - (x^2+y^2)/400), stepped from
t_out = 60 to t_in = -60 with dt = 0.02 (6000 RK4 steps), then the electron
marginal P(s,p) of every solve at t_in.  The timed path is the batched mixed
precision solver (complex64 state and FFTs, FP64 phases/times/reductions).

Both the mixed-precision and the FP64 batched solvers are timed on the full
job.  The headline ("value") is the mixed path when every marginal matches the
FP64 path to P_TOL, else the FP64 path; both are reported under "paths", with
the plain FP64 per-instance solver and the CPU oracle's rate on a bounded
sample beside them.  The roofline is that of the headline path's dominant
kernel: algorithmic bytes / average launch time from HIP events recorded on
the solver's stream during the timed region.
"""
from __future__ import annotations

import argparse
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# a speedup of the mixed-precision path is only claimed when every marginal
# matches the FP64 path to this relative tolerance
P_TOL = 1e-4


def workload(name, time_steps=None):
    import swf_workloads as W
    if name == "2d":
        prob = W.config_2d(steps=time_steps)
        desc = "(2+1)D Schwinger, A_1 Gaussian (a0=1, tau=10, w=20), 512x512 over [-80,80)^2, " \
               "64 U_out solves |p|<1, dt=0.02"
    elif name == "3d":
        prob = W.config_3d(steps=time_steps)
        desc = "(3+1)D Schwinger, A_3 = 0.8 sech^2(t/8) exp(-r^2/225), 256^3 over [-60,60)^3, 8 solves, dt=0.025"
    elif name == "ragged":
        prob = W.config_ragged_2d(steps=time_steps)
        desc = "(2+1)D ragged batch: 256 solves, n in {256,384,512,768,1024}, Gaussian fields from seed 0"
    elif name == "1d":
        prob = W.config_1d(steps=time_steps)
        desc = "(1+1)D Schwinger, A_1 = 1.5 sech^2(0.2 t) sech^2(0.1 x), n=1024 over [-100,100), dt=0.02"
    elif name == "bw3d":
        prob = W.config_bw_3d(steps=time_steps)
        desc = "(3+1)D Breit-Wheeler, focused pulse, 320^3, 16 U + 16 V solves, 32 vertices"
    else:
        raise SystemExit(f"unknown workload {name}")
    return prob, desc


def chosen_row_variant(report):
    """The row-pass tile variant the autotuner kept: the fastest one it timed."""
    times = {int(m.group(1)): float(m.group(2)) for m in re.finditer(r"row v(\d+) ([0-9.eE+-]+) ms", report)}
    return min(times, key=times.get) if times else None


def stored_traffic(precision, n, variant):
    """HBM bytes per launch of the row stage pass (the mean over its four RK4
    stages) from the committed counter summary, or None when the kernel
    sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if variant is None or not os.path.exists(path):
        return None
    from paper_2512_16889_amd.build import source_hash
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != source_hash():
        return None
    real = "double" if precision == "fp64" else "float"
    per_stage = []
    for stage in range(4):
        k = t["kernels"].get(f"void swf::row_kernel<{real}, {n}, {variant}, 1, {stage}>(swf::PassArgs)")
        if k is None:
            return None
        per_stage.append(k["fetch_bytes"] + k["write_bytes"])
    return sum(per_stage) / 4


def run_job(ctx, prob, progress=0, bw_partial=False):
    if progress > 0:
        # chunks of `progress` steps, each synchronised and reported (long jobs)
        left = prob.window.steps
        while left > 0:
            left = ctx.step(min(progress, left))
            ctx.sync()
            print(f"[bench]   {prob.window.steps - left}/{prob.window.steps} steps", file=sys.stderr, flush=True)
    else:
        ctx.step()
    out = []
    for i, s in enumerate(prob.solves):
        out.append(ctx.marginal(i))
    for v in range(len(prob.vertices)):
        out.append(abs(ctx.bw(v)) ** 2)
    if bw_partial:
        # |M|^2 by the partial-integration route, kept apart from the P check
        ctx.last_bw_partial = [abs(ctx.bw_partial(v)) ** 2 for v in range(len(prob.vertices))]
    return out


def timed_jobs(S, torch, prob, precision, K, W, batched=True, graph=False, profile=True, tune=True, chunk=0,
               variant=None, progress=0, bw_partial=False):
    ctx = S.Context(prob, precision=precision, batched=batched, use_graph=graph, profile=profile, tune=tune,
                    chunk=chunk, variant=variant, bw_partial=bw_partial)
    report = ctx.tune_report()
    results = None
    for _ in range(W):
        ctx.reset()
        run_job(ctx, prob, progress, bw_partial)
    ctx.sync()
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        ctx.reset()
        results = run_job(ctx, prob, progress, bw_partial)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = {k: ctx.kernel_stats(k) for k in range(6)} if profile else {}
    norms = [ctx.diagnostics(i)[0] for i in range(len(prob.solves))]
    if bw_partial:
        nb = len(prob.vertices)
        m1 = results[len(results) - nb:]
        m2 = ctx.last_bw_partial
        stats["bw_routes_max_rel_diff"] = max(abs(a - b) / abs(b) for a, b in zip(m2, m1) if b != 0)
    ctx.close()
    return wall, results, stats, report, norms


def partial_rate(S, torch, prob, precision, nsteps, batched, tune=False):
    """Site-updates/s of a shorter run (work is linear in the step count)."""
    ctx = S.Context(prob, precision=precision, batched=batched, tune=tune, persistent=batched)
    ctx.step(min(20, nsteps))
    ctx.sync()
    ctx.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(nsteps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    return prob.site_updates(nsteps) / wall


def cpu_baseline(prob, target_s=15.0):
    """The oracle, as it stands, on one solve of the same workload."""
    import numpy as np
    from oracle.swf import SWFSolve
    sv = SWFSolve(prob, 0)
    y = sv.zero_state()
    # start near the field maximum so the sample does representative work
    start = prob.window.steps // 2
    t0 = time.perf_counter()
    n = 0
    while True:
        y = sv.step(start + n, y)
        n += 1
        el = time.perf_counter() - t0
        if el > target_s or n >= 200:
            break
    sites = int(np.prod([prob.grids[0].n[j] for j in range(prob.grids[0].dim)]))
    return {"value": sites * n / el, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} RK4 steps of one {prob.grids[0].dim}D solve ({sites} sites) of the same workload, "
                      f"numpy/pocketfft FP64, single thread, {el:.1f} s"}


def pair_matrix_bench(S, torch, n_each, form=1):
    """All N x N pair amplitudes of eq. (Nmn) at once (swf_pair_matrix) on the
    2D 512^2 lattice, against the per-pair path on a sample of pairs."""
    import numpy as np
    import swf_workloads as W
    g = W.Grid(2, [512, 512, 1], [160.0, 160.0, 1.0])
    rng = np.random.default_rng(0)
    solves = [W.Solve(0, 1, [float(x) for x in rng.uniform(-0.8, 0.8, 2)] + [0.0]) for _ in range(n_each)]
    solves += [W.Solve(1, 1, [float(x) for x in rng.uniform(-0.8, 0.8, 2)] + [0.0]) for _ in range(n_each)]
    prob = W.Problem("pairs", [g], [W.field_gauss_2d()], solves, W.Window(-0.2, 0.2, 0.02))
    us, vs = list(range(n_each)), list(range(n_each, 2 * n_each))
    sample = [(0, 0), (n_each // 3, n_each - 1), (n_each - 1, n_each // 2)]
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        ctx.sync()
        M = ctx.pair_matrix(us, vs, form)              # warm-up (allocates the scratch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = ctx.pair_matrix(us, vs, form)
        torch.cuda.synchronize()
        t_matrix = time.perf_counter() - t0
        t0 = time.perf_counter()
        ref = [ctx.pair(us[i], vs[j], form) for i, j in sample]
        t_pair = (time.perf_counter() - t0) / len(sample)
    err = max(abs(M[i, j] - r) for (i, j), r in zip(sample, ref)) / float(np.abs(M).max())
    n_amp = n_each * n_each
    sites = 512 * 512
    flops = 2 * 8.0 * n_amp * 4 * sites              # two complex contractions over sites x components
    return {"metric": "pair amplitudes/s", "value": n_amp / t_matrix, "unit": "amplitudes/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": t_matrix * 1e3, "higher_is_better": True, "scaling": "strong",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"pair-amplitude matrix, {n_each} U x {n_each} V solves, 2D 512^2, form {form}"},
            "per_pair_path_ms": t_pair * 1e3, "speedup_vs_per_pair": t_pair * n_amp / t_matrix,
            "matrix_flop": flops, "sample_rel_err_vs_per_pair": err}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed jobs (each = the full workload)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="2d")
    ap.add_argument("--time-steps", type=int, default=None, help="override RK4 steps per job (default: full window)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=300)
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 per-instance leg")
    ap.add_argument("--chunk", type=int, default=0, help="solves per launch group (0 = all)")
    ap.add_argument("--no-tune", action="store_true", help="use the default tile variants")
    ap.add_argument("--variant", type=int, default=None, help="force tile variant 0..3 for every pass")
    ap.add_argument("--progress", type=int, default=0, metavar="STEPS",
                    help="step in synchronised chunks of STEPS and report each (long jobs)")
    ap.add_argument("--bw-partial", action="store_true",
                    help="also integrate the BW vertices by the partial-integration route (timed with the job)")
    ap.add_argument("--pair-matrix", type=int, default=0, metavar="N",
                    help="only time the N x N pair-amplitude matrix on the 2D 512^2 lattice")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU only: every solve of a job is independent and "
                          "the multi-GPU sharding is described, not built; run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2512_16889_amd import swf as S

    if args.pair_matrix:
        print(json.dumps(pair_matrix_bench(S, torch, args.pair_matrix)), flush=True)
        return

    prob, desc = workload(args.workload, args.time_steps)
    steps = prob.window.steps
    su = prob.site_updates()
    print(f"[bench] workload {desc}; {len(prob.solves)} solves, {steps} RK4 steps, {su:.3e} site-updates per job",
          file=sys.stderr, flush=True)

    names = {0: "row pass (x FFTs + RK4 stage epilogue)", 1: "column pass y (stepping)",
             2: "column pass z (stepping)", 3: "BW vertex reduction", 4: "other passes (t_in transforms, BW partial-integration route)",
             5: "1D whole-loop kernel (all steps on chip)"}

    def summarize(wall, stats):
        routes = stats.pop("bw_routes_max_rel_diff", None)
        dom = max((k for k in stats if k != 4), key=lambda k: stats[k][1])
        n_l, ms, by = stats[dom]
        achieved = by / (ms * 1e-3) / 1e9
        kern = {names.get(k, str(k)): {"launches": stats[k][0], "avg_ms": stats[k][1] / max(stats[k][0], 1),
                                       "GB_per_s": stats[k][2] / max(stats[k][1], 1e-30) / 1e6}
                for k in stats if stats[k][0] > 0}
        roof = {"bound": "hbm", "kernel": names.get(dom, str(dom)), "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_launch_ms": ms / max(n_l, 1),
                "algorithmic_bytes_per_launch": by / max(n_l, 1)}
        res = {"value": su * args.steps / wall, "ms_per_step": wall / args.steps * 1e3, "roofline": roof,
               "kernels": kern}
        if routes is not None:
            res["bw_partial_route"] = {"timed_with_job": True, "max_rel_diff_of_M2_vs_first_route": routes}
        return res

    paths = {}
    if args.bw_partial and not prob.vertices:
        raise SystemExit("--bw-partial needs a workload with BW vertices (bw3d)")
    wall, P_mixed, stats, tune_rep, norms_m = timed_jobs(S, torch, prob, "mixed", args.steps, args.warmup,
                                                        chunk=args.chunk, tune=not args.no_tune,
                                                        variant=args.variant, progress=args.progress,
                                                        bw_partial=args.bw_partial)
    paths["mixed_batched"] = summarize(wall, stats)
    paths["mixed_batched"]["autotune"] = tune_rep
    print(f"[bench] mixed batched: {wall:.2f} s for {args.steps} job(s) -> {paths['mixed_batched']['value']:.4e} "
          f"site-updates/s", file=sys.stderr, flush=True)
    headline = "mixed_batched"
    if not args.no_fp64:
        wall64, P64, stats64, tune64, norms64 = timed_jobs(S, torch, prob, "fp64", args.steps, args.warmup,
                                                           chunk=args.chunk, tune=not args.no_tune,
                                                           variant=args.variant, progress=args.progress,
                                                           bw_partial=args.bw_partial)
        paths["fp64_batched"] = summarize(wall64, stats64)
        paths["fp64_batched"]["autotune"] = tune64
        rel = [abs(a - b) / abs(b) for a, b in zip(P_mixed, P64) if b != 0]
        ok = max(rel) <= P_TOL
        paths["mixed_batched"]["p_rel_err_vs_fp64"] = {"max": max(rel), "median": float(np.median(rel)),
                                                       "within_tolerance": ok}
        ratio = [p / n for p, n in zip(P64, norms64) if n > 0]
        print(f"[bench] fp64 batched: {wall64:.2f} s; max rel P err mixed vs fp64 {max(rel):.3e}; "
              f"P/(psi|psi) in [{min(ratio):.2e}, {max(ratio):.2e}]", file=sys.stderr, flush=True)
        paths["fp64_batched"]["P_range"] = [min(P64), max(P64)]
        paths["fp64_batched"]["P_over_norm_range"] = [min(ratio), max(ratio)]
        if not args.no_plain:
            plain = partial_rate(S, torch, prob, "fp64", min(args.plain_steps, steps), batched=False)
            paths["fp64_plain_per_instance"] = {"value": plain, "steps_timed": min(args.plain_steps, steps)}
            print(f"[bench] fp64 plain per-instance: {plain:.4e} site-updates/s", file=sys.stderr, flush=True)
        if not ok:
            headline = "fp64_batched"
    H = paths[headline]
    out = {
        "metric": "spinor site-updates/s",
        "value": H["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if headline.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "solves": len(prob.solves), "grid": prob.grids[0].n[:prob.grids[0].dim],
                   "rk4_steps": steps, "timed_path": headline, "p_tolerance": P_TOL,
                   "parallelism": "single GPU, batched solves", "chunk": args.chunk,
                   "bw_partial": bool(args.bw_partial)},
        "roofline": H["roofline"],
        "kernels": H["kernels"],
        "paths": paths,
    }
    if H["roofline"]["kernel"].startswith("row pass"):
        H["roofline"]["traffic"] = stored_traffic("fp64" if headline.startswith("fp64") else "mixed",
                                                  prob.grids[0].n[0],
                                                  chosen_row_variant(H.get("autotune") or "")
                                                  if args.variant is None else args.variant)
    if "fp64_plain_per_instance" in paths:
        out["speedup_vs_fp64_plain"] = H["value"] / paths["fp64_plain_per_instance"]["value"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
