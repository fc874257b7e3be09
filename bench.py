"""Benchmark of the SWF hot path on one MI355X.

Default workload: the (3+1)D nonlinear Breit-Wheeler batch, the largest
configuration of the method on one GPU: 16 U_out + 16 V_out solves on a 320^3
lattice over [-60, 60)^3, the focused pulse A_1 = exp(-t^2/36 - |x|^2/100)
cos(t/2), dt = 0.025 (3000 RK4 steps over [-37.5, 37.5]), and 32 photon
vertices whose finite-time overlap is integrated at every RK4 stage.

One bench step is one RK4 step of the whole batch: the four stages of every
solve (transforms along x, y, z, the -i H0 multiply, the source term, the
RK4 update) and the vertex overlaps at each stage.  ``--warmup W`` steps run
untimed, then ``--steps K`` steps are timed between device synchronisations.
The W + K steps are the central W + K steps of the workload's window (where
the pulse is on), started from psi_s = 0; the work of a step does not depend
on the data, so the rate is that of the full 3000-step job.  At the end of
the W + K steps the amplitudes |M|^2 of every vertex are formed (timed apart
from the steps), and the mixed-precision path's |M|^2 are compared with the
FP64 path's over the same steps.

Paths (each its own context, freed before the next):
  * FP64 batched, autotuned tiles ("fp64_batched");
  * FP64 plain: one launch per solve and pass, default tiles ("fp64_plain");
  * mixed precision batched, autotuned ("mixed_batched": complex64 state and
    transforms, FP64 phases, times and reductions).
When the FP64 batch does not fit the free device memory in one context it
runs as sub-batches of whole vertices (a U and a V solve of a vertex stay
together); the timed steps are then the sum over the sub-batches.

The headline ("value") is the mixed path when every probability matches the
FP64 path to P_TOL, else the FP64 batched path.  The roofline is that of the
headline path's dominant kernel class: algorithmic bytes per launch over the
average launch time from HIP events recorded on the solver's stream during
the timed steps.  The CPU baseline runs the oracle (plain numpy FP64) on a
bounded sample of the same workload, one process per core.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# a speedup of the mixed-precision path is only claimed when every probability
# matches the FP64 path to this relative tolerance
P_TOL = 1e-4
# device memory kept free beside a context (runtime, torch, reductions)
MEM_MARGIN = 2 << 30

KIND_NAMES = {0: "row pass (x transforms + RK4 stage epilogue)", 1: "column pass y (stepping)",
              2: "column pass z (stepping)", 3: "BW vertex reduction",
              4: "other passes (t_in transforms, BW partial-integration route)",
              5: "1D whole-loop kernel (all steps on chip)"}


def workload(name):
    import swf_workloads as W
    if name == "bw3d":
        return W.config_bw_3d(), ("(3+1)D nonlinear Breit-Wheeler: focused pulse a0=1, w=10, tau=6, omega0=0.5; "
                                  "photon k=(0,0,2), eps_par; 320^3 over [-60,60)^3, dt=0.025, 3000-step window; "
                                  "16 U_out + 16 V_out solves, 32 vertices (P in linspace(-0.7,0.7,8) x 4 spin pairs)")
    if name == "2d":
        return W.config_2d(), ("(2+1)D Schwinger: A_1 = exp(-t^2/100 - (x^2+y^2)/400), 512^2 over [-80,80)^2, "
                               "dt=0.02, 6000-step window, 64 U_out solves |p|<1")
    if name == "3d":
        return W.config_3d(), ("(3+1)D Schwinger: A_3 = 0.8 sech^2(t/8) exp(-|x|^2/225), 256^3 over [-60,60)^3, "
                               "dt=0.025, 4000-step window, 8 solves")
    if name == "ragged":
        return W.config_ragged_2d(), ("(2+1)D ragged batch: 256 solves, n in {256,384,512,768,1024}, "
                                      "Gaussian fields from seed 0, dt=0.02, 8000-step window")
    if name == "1d":
        return W.config_1d(), ("(1+1)D Schwinger: A_1 = 1.5 sech^2(0.2 t) sech^2(0.1 x), n=1024 over [-100,100), "
                               "dt=0.02, 6000-step window, one solve")
    if name == "2d-small":
        import dataclasses
        p = W.config_2d()
        g = dataclasses.replace(p.grids[0], n=[128, 128, 1])
        return dataclasses.replace(p, grids=[g], solves=p.solves[:8]), (
            "(2+1)D Schwinger field of the 2D workload on a 128^2 lattice over [-80,80)^2, 8 of its solves, "
            "dt=0.02 (launch-bound: microsecond passes)")
    raise SystemExit(f"unknown workload {name}")


def central_window(prob, count):
    """The problem restricted to the central `count` steps of its window."""
    import dataclasses
    import swf_workloads as W
    w = prob.window
    first = (w.steps - count) // 2
    t_out = w.t_out - first * w.dt
    return dataclasses.replace(prob, window=W.Window(t_out - count * w.dt, t_out, w.dt, w.scheme))


def components(prob):
    """Solve sets that must share a context: the U and V solve of every vertex."""
    parent = list(range(len(prob.solves)))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i
    for v in prob.vertices:
        parent[find(v.u_solve)] = find(v.v_solve)
    comp = {}
    for i in range(len(prob.solves)):
        comp.setdefault(find(i), []).append(i)
    return sorted(comp.values(), key=lambda c: c[0])


def sub_problem(prob, solve_ids):
    """The problem restricted to the given solves and the vertices among them."""
    import dataclasses
    remap = {s: i for i, s in enumerate(solve_ids)}
    verts = [dataclasses.replace(v, u_solve=remap[v.u_solve], v_solve=remap[v.v_solve])
             for v in prob.vertices if v.u_solve in remap and v.v_solve in remap]
    return dataclasses.replace(prob, solves=[prob.solves[s] for s in solve_ids], vertices=verts)


def split_to_fit(S, prob, precision, free_bytes, bw_partial, max_solves=0):
    """Sub-batches of whole components, each fitting in free_bytes (one if possible)."""
    comps = components(prob)
    batches, cur = [], []
    for c in comps:
        trial = cur + c
        too_many = max_solves and len(trial) > max_solves
        if cur and (too_many or S.workspace_size(sub_problem(prob, trial), precision, bw_partial) > free_bytes):
            batches.append(cur)
            cur = list(c)
        else:
            cur = trial
    if cur:
        batches.append(cur)
    for b in batches:
        if S.workspace_size(sub_problem(prob, b), precision, bw_partial) > free_bytes:
            raise SystemExit(f"a vertex component needs more than the {free_bytes / 1e9:.1f} GB free")
    return batches


def observables(ctx, prob):
    """|M|^2 of every vertex, else the marginal of every solve (at t_in)."""
    if prob.vertices:
        return [abs(ctx.bw(v)) ** 2 for v in range(len(prob.vertices))]
    return [ctx.marginal(i) for i in range(len(prob.solves))]


def run_path(S, torch, prob, precision, K, Wm, batched=True, tune=True, variant=None, chunk=0, graph=False,
             bw_partial=False, max_solves=0, label="", reset_after_warmup=False, tune_cache=None, graph_steps=0,
             profile=None):
    """Time K RK4 steps (after Wm untimed ones) of every solve of prob.
    With reset_after_warmup the context is returned to t_out after the Wm
    steps, so the K timed steps can span the whole window.

    Returns wall seconds of the timed steps (summed over sub-batches), the
    observables at the end of the window, per-kind kernel statistics, the
    tune reports and the sub-batch sizes."""
    free, _total = torch.cuda.mem_get_info()
    batches = split_to_fit(S, prob, precision, free - MEM_MARGIN, bw_partial, max_solves)
    wall, t_obs, obs = 0.0, 0.0, [None] * (len(prob.vertices) if prob.vertices else len(prob.solves))
    stats = {k: [0, 0.0, 0.0] for k in range(6)}
    reports, extra = [], {}
    for b in batches:
        sub = sub_problem(prob, b)
        print(f"[bench] {label}: context of {len(b)} solves, {len(sub.vertices)} vertices, "
              f"{S.workspace_size(sub, precision, bw_partial) / 1e9:.1f} GB", file=sys.stderr, flush=True)
        prof = (not graph) if profile is None else profile
        ctx = S.Context(sub, precision=precision, batched=batched, use_graph=graph, profile=prof, tune=tune,
                        chunk=chunk, variant=variant, bw_partial=bw_partial, tune_cache=tune_cache,
                        graph_steps=graph_steps)
        reports.append(ctx.tune_report())
        if Wm:
            ctx.step(Wm)
            if reset_after_warmup:
                ctx.reset()
        ctx.sync()
        ctx.reset_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(K)
        ctx.sync()
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        if prof:
            for k in range(6):
                n, ms, by = ctx.kernel_stats(k)
                stats[k][0] += n
                stats[k][1] += ms
                stats[k][2] += by
        t0 = time.perf_counter()
        vals = observables(ctx, sub)
        torch.cuda.synchronize()
        t_obs += time.perf_counter() - t0
        if sub.vertices:
            # vertex indices of the sub-problem follow the order of prob.vertices
            idx = [i for i, v in enumerate(prob.vertices) if v.u_solve in b and v.v_solve in b]
        else:
            idx = b
        for i, val in zip(idx, vals):
            obs[i] = val
        if bw_partial:
            m1 = vals
            m2 = [abs(ctx.bw_partial(v)) ** 2 for v in range(len(sub.vertices))]
            extra["bw_routes_max_rel_diff"] = max(extra.get("bw_routes_max_rel_diff", 0.0),
                                                  max(abs(a - c) / abs(c) for a, c in zip(m2, m1) if c != 0))
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    return wall, t_obs, obs, stats, reports, [len(b) for b in batches], extra


def summarize(prob, K, wall, t_obs, stats, sub_batches):
    su = prob.site_updates(K)
    dom = max((k for k in stats if k != 4 and stats[k][0] > 0), key=lambda k: stats[k][1], default=None)
    kern = {KIND_NAMES[k]: {"launches": stats[k][0], "avg_ms": stats[k][1] / stats[k][0],
                            "GB_per_s": stats[k][2] / max(stats[k][1], 1e-30) / 1e6}
            for k in stats if stats[k][0] > 0}
    res = {"value": su / wall, "ms_per_step": wall / K * 1e3, "wall_s": wall, "t_in_observables_s": t_obs,
           "sub_batches": sub_batches, "kernels": kern}
    if dom is not None:
        n_l, ms, by = stats[dom]
        achieved = by / (ms * 1e-3) / 1e9
        res["roofline"] = {"bound": "hbm", "kernel": KIND_NAMES[dom], "kind": dom, "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "avg_launch_ms": ms / n_l, "algorithmic_bytes_per_launch": by / n_l,
                           "kernel_time_share": ms / sum(s[1] for s in stats.values())}
    return res


def stored_traffic(kind, precision, n, report, variant):
    """Measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the
    copy-kernel calibration) of the kernel class `kind` from the committed
    counter summary, or None when the kernel sources changed since it was
    taken or the class's kernels were not measured."""
    import re
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    from paper_2512_16889_amd.build import source_hash
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != source_hash():
        return None
    real = "double" if precision == "fp64" else "float"
    tag = {0: "row", 1: "col1", 2: "col2", 3: "bw"}.get(kind)
    if tag is None:
        return None
    if variant is None and kind != 3:
        # the variant the autotuner kept: the fastest one it timed, or the cached choice
        cached = re.search(r"cached (\d+) (\d+) (\d+)", report)
        if cached:
            variant = int(cached.group(1 + kind))
        else:
            times = {}
            for m in re.finditer(rf"{tag} v(\d+) ([0-9.eE+-]+) ms", report):
                v, ms = int(m.group(1)), float(m.group(2))
                times[v] = min(ms, times.get(v, ms))
            if not times:
                return None
            variant = min(times, key=times.get)
    if kind == 0:
        names = [f"void swf::row_d_kernel<{real}, {n}, {variant}, {s}>(swf::PassArgs)" for s in range(4)]
    elif kind == 1:
        names = [f"void swf::col_d_kernel<{real}, {n}, {variant}, 1, 0>(swf::PassArgs)"]
    elif kind == 2:
        names = [f"void swf::col_d_kernel<{real}, {n}, {variant}, 2, 1>(swf::PassArgs)"]
    else:
        names = [f"void swf::bw_stage_kernel<{real}, 2, 2>(swf::BwArgs)"]
    vals = []
    for nm in names:
        k = t["kernels"].get(nm)
        if k is None:
            return None
        vals.append(k["fetch_bytes"] + k["write_bytes"])
    return sum(vals) / len(vals)


# ------------------------------------------------------------------ CPU baseline
def cpu_sample_problem(name, n_cpu):
    """The workload on the lattice the CPU sample uses (3D: n_cpu^3 points over
    the same box; 2D and 1D: the workload's own lattice)."""
    import dataclasses
    import swf_workloads as W
    prob, _ = workload(name)
    if name in ("bw3d", "3d"):
        g = dataclasses.replace(prob.grids[0], n=[n_cpu, n_cpu, n_cpu])
        prob = dataclasses.replace(prob, grids=[g])
    return prob


def _cpu_worker(name, n_cpu, solve_ids, vert_ids, steps, barrier, out_q):
    """One process of the CPU baseline: `steps` RK4 steps of its solves (with
    the finite-time overlap of its vertices at every stage), after setup."""
    from oracle.bw import Vertex
    from oracle.swf import SWFSolve
    prob = cpu_sample_problem(name, n_cpu)
    svs = {i: SWFSolve(prob, i) for i in solve_ids}
    verts = [Vertex(prob, v) for v in vert_ids]
    ys = {i: s.zero_state() for i, s in svs.items()}
    start = prob.window.steps // 2
    barrier.wait()
    t0 = time.monotonic()
    sites = 0
    for n in range(start, start + steps):
        stages = {}
        for i, s in svs.items():
            ys[i], st, tt, _ = s.step_stages(n, ys[i])
            stages[i] = (st, tt)
            sites += s.lat.N
        for vx in verts:
            su, tt = stages[vx.vx.u_solve]
            sv, _ = stages[vx.vx.v_solve]
            for j in range(len(tt)):
                vx.mdot(tt[j], su[j], sv[j])
    out_q.put((t0, time.monotonic(), sites))


def cpu_units(prob):
    """Independent pieces of CPU work: disjoint vertices (their U and V solve
    with the vertex overlap), then every remaining solve on its own."""
    units, used = [], set()
    for v, vx in enumerate(prob.vertices):
        if vx.u_solve not in used and vx.v_solve not in used:
            units.append(([vx.u_solve, vx.v_solve], [v]))
            used.update((vx.u_solve, vx.v_solve))
    units += [([i], []) for i in range(len(prob.solves)) if i not in used]
    return units


def cpu_baseline(name, workers, n_cpu):
    """The oracle, as it stands, on a bounded sample of the workload: one
    process per core, each stepping its own solves (with the overlap of a
    vertex whose U and V solve it holds); rate = all site-updates / wall of
    the parallel run."""
    import multiprocessing as mp
    import platform
    prob = cpu_sample_problem(name, n_cpu)
    units = cpu_units(prob)
    if name == "1d":
        steps = 200
    elif name == "2d" or name == "ragged":
        steps = 3
    else:
        steps = 1
    workers = max(1, min(workers, len(units)))
    plan = units[:workers]
    env_threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_threads:
        os.environ[k] = "1"
    ctxm = mp.get_context("spawn")
    barrier = ctxm.Barrier(workers)
    q = ctxm.Queue()
    procs = []
    for sids, vids in plan:
        pr = ctxm.Process(target=_cpu_worker, args=(name, n_cpu, sids, vids, steps, barrier, q))
        pr.start()
        procs.append(pr)
    res = [q.get() for _ in procs]
    for pr in procs:
        pr.join()
    for k, v in env_threads.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    t0 = min(r[0] for r in res)
    t1 = max(r[1] for r in res)
    sites = sum(r[2] for r in res)
    cpu_model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    g = prob.grids[0]
    lattice = "x".join(str(g.n[j]) for j in range(g.dim)) if name != "ragged" else "the batch's own lattices"
    n_solves = sum(len(p[0]) for p in plan)
    n_verts = sum(len(p[1]) for p in plan)
    with_v = f" with the overlaps of their {n_verts} vertices" if n_verts else ""
    return {"value": sites / (t1 - t0), "unit": "site-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"{steps} RK4 step(s) of {n_solves} solves{with_v} from the middle of the window, on the "
                      f"{lattice} lattice over the workload's box, one single-threaded numpy FP64 process per "
                      f"core ({workers} processes), {t1 - t0:.1f} s wall",
            "host": {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": cpu_model}}


# ------------------------------------------------------------------ full-window accuracy
def accuracy_problem(name, n_acc):
    """The workload over its whole window on a coarser lattice over the same
    box (3D: n_acc^3, 2D: n_acc^2), or None where no such copy is defined."""
    import dataclasses
    prob, _ = workload(name)
    g = prob.grids[0]
    if name in ("bw3d", "3d"):
        n = [n_acc, n_acc, n_acc]
    elif name == "2d":
        n = [n_acc, n_acc, 1]
    else:
        return None
    return dataclasses.replace(prob, grids=[dataclasses.replace(g, n=n)])


def accuracy_check(S, torch, name, n_acc):
    """Mixed against FP64 probabilities over the workload's whole window on
    the coarser lattice: the FP32 rounding noise of the mixed path accumulates
    over every step of the window, which the short timed window does not show."""
    import numpy as np
    prob = accuracy_problem(name, n_acc)
    if prob is None:
        return None
    vals, secs = {}, {}
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        with S.Context(prob, precision=prec) as ctx:
            ctx.step()
            vals[prec] = observables(ctx, prob)
        secs[prec] = time.perf_counter() - t0
        torch.cuda.empty_cache()
    rel = [abs(a - b) / abs(b) for a, b in zip(vals["mixed"], vals["fp64"]) if b != 0]
    g = prob.grids[0]
    return {"lattice": g.n[:g.dim], "window_steps": prob.window.steps,
            "observable": "|M|^2 per vertex" if prob.vertices else "marginal P per solve",
            "max_rel_err": max(rel), "median_rel_err": float(np.median(rel)), "tolerance": P_TOL,
            "within_tolerance": max(rel) <= P_TOL, "fp64_range": [min(vals["fp64"]), max(vals["fp64"])],
            "seconds": secs}


# ------------------------------------------------------------------ pair matrix mode
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


def matched_error_bench(S, torch, name, n_solves=8):
    """The steppers at matched P error (FP64, whole window): marginals of the
    workload's first solves from RK4 at the window's dt and at 2 dt, from the
    fixed-step Dormand-Prince tableau at 1, 2, 2.5 and 4 dt, and from the
    interaction-picture RK4 at 1, 2, 4 and 8 dt, each against Dormand-Prince
    at dt/4; wall time of each whole window."""
    import dataclasses
    import numpy as np
    import swf_workloads as W
    full, desc = workload(name)
    base = dataclasses.replace(full, solves=full.solves[:n_solves], vertices=[])
    w = base.window

    def run(scheme, f):
        dt = w.dt * f
        prob = dataclasses.replace(base, window=W.Window(w.t_in, w.t_out, dt, scheme))
        with S.Context(prob, precision="fp64", tune=True, persistent=False) as ctx:
            ctx.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.step()
            ctx.sync()
            wall = time.perf_counter() - t0
            P = np.array([ctx.marginal(i) for i in range(len(prob.solves))])
        print(f"[bench] {scheme} dt={dt:g}: {prob.window.steps} steps in {wall:.2f} s", file=sys.stderr, flush=True)
        return P, wall, prob.window.steps

    ref, _, _ = run("dp5", 0.25)
    runs = {}
    for scheme, fs in (("rk4", (1.0, 2.0)), ("dp5", (1.0, 2.0, 2.5, 4.0)), ("iprk4", (1.0, 2.0, 4.0, 8.0))):
        for f in fs:
            P, wall, steps = run(scheme, f)
            runs[f"{scheme} dt x{f:g}"] = {"dt": w.dt * f, "steps": steps, "wall_s": wall,
                                           "ms_per_step": wall / steps * 1e3,
                                           "max_rel_P_err": float(np.max(np.abs(P - ref) / np.abs(ref)))}
    target = runs["rk4 dt x1"]["max_rel_P_err"]
    speedup, matched = {}, {}
    for scheme in ("dp5", "iprk4"):
        ok = [k for k, v in runs.items() if k.startswith(scheme + " ") and v["max_rel_P_err"] <= target]
        if ok:
            matched[scheme] = min(ok, key=lambda k: runs[k]["wall_s"])
            speedup[scheme] = runs["rk4 dt x1"]["wall_s"] / runs[matched[scheme]]["wall_s"]
    best = max(speedup, key=speedup.get) if speedup else None
    return {"metric": "whole-window time at matched P error (variant steppers vs RK4, FP64)",
            "value": speedup[best] if best else None,
            "unit": "RK4 time / variant time", "n_gpus": 1, "steps": runs["rk4 dt x1"]["steps"], "warmup": 0,
            "ms_per_step": runs["rk4 dt x1"]["ms_per_step"], "higher_is_better": True, "scaling": "strong",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{desc}; first {len(base.solves)} solves",
                       "reference": "Dormand-Prince at dt/4", "rk4_error": target,
                       "matched_by": matched.get(best), "speedup": speedup, "matched": matched},
            "runs": runs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed RK4 steps of the whole batch")
    ap.add_argument("--warmup", type=int, default=5, help="untimed RK4 steps before the timed ones")
    ap.add_argument("--workload", default="bw3d", choices=["bw3d", "2d", "3d", "ragged", "1d", "2d-small"])
    ap.add_argument("--full-window", action="store_true",
                    help="time the workload's whole window (--steps is ignored; the warmup steps run first "
                         "and the context is reset)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 plain per-instance path")
    ap.add_argument("--no-graph", action="store_true", help="skip the hipGraph replay leg of the FP64 batched path")
    ap.add_argument("--graph-steps", type=int, default=16, help="time steps captured per graph of the replay leg")
    ap.add_argument("--graph-compare", action="store_true",
                    help="only compare eager launches (no event timing), one-step and multi-step graph replay")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16, help="CPU baseline processes (capped by the cores)")
    ap.add_argument("--cpu-n", type=int, default=80, help="3D lattice points per axis of the CPU sample")
    ap.add_argument("--accuracy-n", type=int, default=64,
                    help="lattice points per axis of the full-window mixed-vs-FP64 check (0: skip)")
    ap.add_argument("--max-solves", type=int, default=0, help="at most this many solves per context (0: fit memory)")
    ap.add_argument("--chunk", type=int, default=0, help="solves per launch group (0 = all)")
    ap.add_argument("--no-tune", action="store_true", help="use the default tile variants")
    ap.add_argument("--variant", type=int, default=None, help="force tile variant 0..3 for every pass")
    ap.add_argument("--tune-cache", default=None, metavar="FILE",
                    help="autotuner cache: tile choices are read from FILE and new ones appended")
    ap.add_argument("--bw-partial", action="store_true",
                    help="also integrate the BW vertices by the partial-integration route (timed with the steps)")
    ap.add_argument("--pair-matrix", type=int, default=0, metavar="N",
                    help="only time the N x N pair-amplitude matrix on the 2D 512^2 lattice")
    ap.add_argument("--stepper", default="rk4", choices=["rk4", "dp5", "iprk4"],
                    help="time stepper of every path (dp5: the fixed-step Dormand-Prince tableau; iprk4: the "
                         "interaction-picture RK4)")
    ap.add_argument("--matched-error", action="store_true",
                    help="only compare the steppers at matched P error over whole windows "
                         "(workloads 1d, 2d, 3d; first 8 solves, FP64)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU: every solve of a batch is independent and the "
                          "sharding over several GPUs is described, not built; run with --gpus 1"}), flush=True)
        sys.exit(2)
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
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("need --steps >= 1 and --warmup >= 0")

    full, desc = workload(args.workload)
    if args.stepper != "rk4":
        import dataclasses
        import swf_workloads as W
        w = full.window
        full = dataclasses.replace(full, window=W.Window(w.t_in, w.t_out, w.dt, args.stepper))
        desc += f"; stepper {args.stepper}"
    K, Wm = args.steps, args.warmup
    if args.full_window:
        K = full.window.steps
        prob = full
    else:
        if Wm + K > full.window.steps:
            raise SystemExit(f"--warmup + --steps exceeds the window's {full.window.steps} steps")
        prob = central_window(full, Wm + K)

    # the CPU leg first: its worker processes start before this process touches the GPU
    cpu = None
    if not args.no_cpu and not args.pair_matrix and not args.matched_error:
        cores = len(os.sched_getaffinity(0))
        print(f"[bench] CPU baseline: oracle on up to {min(args.cpu_workers, cores)} processes", file=sys.stderr,
              flush=True)
        cpu = cpu_baseline(args.workload, min(args.cpu_workers, cores), args.cpu_n)
        print(f"[bench] CPU baseline: {cpu['value']:.4e} site-updates/s ({cpu['sample']})", file=sys.stderr,
              flush=True)

    import numpy as np
    import torch
    from paper_2512_16889_amd import swf as S

    if args.pair_matrix:
        print(json.dumps(pair_matrix_bench(S, torch, args.pair_matrix)), flush=True)
        return
    if args.graph_compare:
        res = {}
        for name, kw in (("eager", {}), ("graph, 1 step", {"graph": True}),
                         (f"graph, {args.graph_steps} steps", {"graph": True, "graph_steps": args.graph_steps})):
            wall, *_ = run_path(S, torch, prob, "fp64", K, Wm, tune_cache=args.tune_cache, profile=False, label=name,
                                **kw)
            res[name] = {"ms_per_step": wall / K * 1e3}
            print(f"[bench] {name}: {wall / K * 1e3:.4f} ms/step", file=sys.stderr, flush=True)
        print(json.dumps({"workload": desc, "steps": K, "warmup": Wm, "paths": res}), flush=True)
        return
    if args.matched_error:
        if args.workload not in ("1d", "2d", "3d"):
            raise SystemExit("--matched-error takes the 1d, 2d or 3d workload")
        print(json.dumps(matched_error_bench(S, torch, args.workload)), flush=True)
        return

    free, total = torch.cuda.mem_get_info()
    print(f"[bench] workload {desc}; {len(prob.solves)} solves, {len(prob.vertices)} vertices; timing {K} RK4 "
          f"steps after {Wm}; {prob.site_updates(K):.3e} site-updates timed; device memory {free / 1e9:.1f} of "
          f"{total / 1e9:.1f} GB free", file=sys.stderr, flush=True)

    def leg(name, precision, **kw):
        wall, t_obs, obs, stats, reps, subs, extra = run_path(
            S, torch, prob, precision, K, Wm, reset_after_warmup=args.full_window, tune_cache=args.tune_cache,
            tune=kw.pop("tune", not args.no_tune),
            variant=kw.pop("variant", args.variant), chunk=args.chunk, bw_partial=args.bw_partial,
            max_solves=args.max_solves, label=name, **kw)
        res = summarize(prob, K, wall, t_obs, stats, subs)
        res["autotune"] = "".join(reps)
        res.update(extra)
        print(f"[bench] {name}: {wall:.2f} s for {K} steps -> {res['value']:.4e} site-updates/s "
              f"({res['ms_per_step']:.1f} ms/step; sub-batches {subs})", file=sys.stderr, flush=True)
        return res, obs

    paths, obs = {}, {}
    if not args.no_fp64:
        paths["fp64_batched"], obs["fp64"] = leg("fp64 batched", "fp64")
        if not args.no_graph:
            paths["fp64_batched_graph"], _ = leg(f"fp64 batched, graph replay ({args.graph_steps} steps per graph)",
                                                 "fp64", graph=True, graph_steps=args.graph_steps)
        if not args.no_plain:
            paths["fp64_plain"], _ = leg("fp64 plain per-instance", "fp64", batched=False, tune=False, variant=None)
    if not args.no_mixed:
        paths["mixed_batched"], obs["mixed"] = leg("mixed batched", "mixed")
    if not paths:
        raise SystemExit("no path selected")

    headline = "fp64_batched" if "fp64_batched" in paths else "mixed_batched"
    kind_obs = "|M|^2 per vertex" if prob.vertices else "marginal P per solve"
    if "fp64" in obs and "mixed" in obs:
        rel = [abs(a - b) / abs(b) for a, b in zip(obs["mixed"], obs["fp64"]) if b != 0]
        ok = bool(rel) and max(rel) <= P_TOL
        paths["mixed_batched"]["p_rel_err_vs_fp64"] = {"observable": kind_obs, "max": max(rel) if rel else None,
                                                       "median": float(np.median(rel)) if rel else None,
                                                       "tolerance": P_TOL, "within_tolerance": ok,
                                                       "over": "the same steps as the timed run"}
        print(f"[bench] mixed vs fp64 ({kind_obs}) over the timed window: max rel err "
              f"{max(rel) if rel else float('nan'):.3e}", file=sys.stderr, flush=True)
        acc = accuracy_check(S, torch, args.workload, args.accuracy_n) if args.accuracy_n else None
        if acc is not None:
            paths["mixed_batched"]["p_rel_err_vs_fp64_full_window"] = acc
            print(f"[bench] mixed vs fp64 over the whole window on {acc['lattice']}: max rel err "
                  f"{acc['max_rel_err']:.3e}", file=sys.stderr, flush=True)
        # the mixed path is the headline only when it matches FP64 over the
        # timed steps and over a whole window
        if ok and acc is not None and acc["within_tolerance"]:
            headline = "mixed_batched"
    if "fp64" in obs:
        paths["fp64_batched"]["observables_range"] = [min(obs["fp64"]), max(obs["fp64"])]
    H = paths[headline]
    if "roofline" in H:
        H["roofline"]["traffic"] = stored_traffic(H["roofline"]["kind"], "fp64" if headline.startswith("fp64")
                                                  else "mixed", prob.grids[0].n[0], H["autotune"], args.variant)
    g = prob.grids[0]
    out = {
        "metric": "spinor site-updates/s",
        "value": H["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": H["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if headline.startswith("fp64") else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "solves": len(prob.solves), "vertices": len(prob.vertices),
                   "grid": g.n[:g.dim], "window_steps": full.window.steps,
                   "timed_steps": f"{'the whole window' if args.full_window else f'the central {Wm + K} steps of the window, the last {K} timed'}",
                   "timed_path": headline, "sub_batches": H["sub_batches"], "p_tolerance": P_TOL,
                   "parallelism": "single GPU, batched solves", "bw_partial": bool(args.bw_partial)},
        "roofline": H.get("roofline"),
        "paths": paths,
    }
    if "fp64_plain" in paths:
        out["speedup_vs_fp64_plain"] = H["value"] / paths["fp64_plain"]["value"]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
