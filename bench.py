"""Benchmark: active voxel-steps/s and launches/step, optimized vs eager
pipeline, on one GPU.

Default workload (band512): sparse Jacobi on a 512^3 domain, a narrow band
around 4 seeded spheres, 8^3 fp32 leaves under a bitmasked root.  A step is
one Jacobi iteration of the whole program -- listgen, jacobi (xn = (sum of 6
neighbours of x + b) / 6), copy (x = xn) -- over every active voxel.  The
optimized pipeline runs the same task list through the inter-kernel
optimizer (list generation removal, activation demotion, task fusion, dead
store elimination).  Inputs are resident in HBM before timing; the timed
region is K steps submitted as one engine window (plan lookup and launch
included) bracketed by device synchronisation.

Other workloads (--workload): shell (64^3 activate/lap_update/axpy),
particles (2M-particle PIC), serving (256 Poisson-arriving 128^3 Jacobi
requests, continuous batching), diffusion (128^3 forward + adjoint) and
multigrid (V-cycles over a 256^3 band and its coarse levels), advection
(three scalar fields on a 256^3 tube) and mpm (the MLS-MPM falling cube,
16.7M particles on a 256^3 grid).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3      # MI355X dense fp32 vector peak

# Algorithmic fp32 operations of one MLS-MPM particle-substep (gather of v
# and C over 27 nodes, advection, F update, polar decomposition by two Newton
# iterations, fixed-corotated stress, scatter of mass and APIC momentum over
# 27 nodes); the count is derived term by term in the design notes.
MPM_FLOPS_PER_PARTICLE = 2034

# HBM bytes per launch of the Jacobi stencil on band512 (seed 0), from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE), each scaled by the reading
# for a plain 256 MiB copy in the same run.  Valid only for the kernel
# source the counters were taken on; any change to it reports null.
JACOBI_TRAFFIC = {"kernels_sha256": "11365eaf2afa2c621385c717f524a0962c2d0f848257d1f4f2934948910f1bf9",
                  "bytes_per_launch": 83327291, "profile": "profiles/band512_jacobi_traffic.md"}


def _jacobi_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2012_08141_amd", "csrc", "kernels.hip")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if JACOBI_TRAFFIC["kernels_sha256"] != h:
        return None
    return JACOBI_TRAFFIC["bytes_per_launch"]
METRIC = "active voxel-steps/s + launches/step, optimized vs eager pipeline, 1 GPU"


def _base(K, W, value, ms, config):
    return {"metric": METRIC, "value": value, "unit": "voxel-steps/s", "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": config}


def _ablations():
    from paper_2012_08141_amd import engine as E
    return [("no_lgr", E.OPT_ALL & ~E.OPT_LGR), ("no_ad", E.OPT_ALL & ~E.OPT_AD),
            ("no_fusion", E.OPT_ALL & ~E.OPT_FUSE), ("no_dse", E.OPT_ALL & ~E.OPT_DSE)]


def settle_host():
    """Collect once and freeze the survivors (torch's import graph, ~170k
    objects), so a generation-2 collection inside a timed region scans only
    new objects instead of taking ~50 ms."""
    import gc
    gc.collect()
    gc.freeze()


def _host_cpu():
    try:
        return subprocess.run(["bash", "-c", "lscpu | grep 'Model name' | head -1"], capture_output=True,
                              text=True).stdout.split(":", 1)[-1].strip()
    except Exception:
        return "unknown"


def roofline(achieved_gbs, kernel, alg_bytes, traffic=None, bound="hbm"):
    """The roofline object of a bench line: algorithmic GB/s of the dominant
    launch against MI355X's 8 TB/s HBM peak."""
    return {"bound": bound, "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "algorithmic_bytes_per_launch": alg_bytes,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)"}


def cpu_leg(step, min_s, max_calls):
    """Run one oracle step repeatedly, pinned to a single core of this host,
    until ``min_s`` seconds have passed (at most ``max_calls`` calls).
    Returns (calls, seconds, core)."""
    prev = os.sched_getaffinity(0)
    core = min(prev)
    os.sched_setaffinity(0, {core})
    try:
        calls, t0 = 0, time.perf_counter()
        while calls < max_calls:
            step(calls)
            calls += 1
            if time.perf_counter() - t0 >= min_s:
                break
        return calls, time.perf_counter() - t0, core
    finally:
        os.sched_setaffinity(0, prev)


def cpu_baseline(value, unit, sample, seconds, core):
    return {"value": value, "unit": unit, "cores": 1, "kind": "oracle",
            "sample": "%s; single-threaded C oracle (-O2, no contraction) pinned to core %d, %.1f s"
                      % (sample, core, seconds),
            "host_cpu": _host_cpu(), "host_nproc": os.cpu_count()}


def window_kernel_means(E, tasks, opt, reps):
    """Per launched kind of a window (task kind, op, fused members): mean
    duration in us between HIP events recorded around each launch on its
    stream, over ``reps`` runs of the window (its plan already cached)."""
    E.timing_enable(True)
    try:
        for _ in range(reps):
            E.run_sequence(tasks, opt)
        res = E.timing_collect()
    finally:
        E.timing_enable(False)
    return res


def time_group(torch, E, group_fn, reps, opt, windows=3):
    """Like time_kernel, for a group of tasks that the optimizer turns into
    one launch: a window of ``reps`` groups (``group_fn(r)`` for r = 0 ..
    reps - 1, built so that consecutive groups cannot fuse) planned with
    ``opt``.  Returns (seconds per group, launches per group)."""
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tasks = E.prepare(sum((group_fn(r) for r in range(reps)), []))
    E.run_sequence(tasks, opt)
    st = E.run_sequence(tasks, opt)
    torch.cuda.synchronize()
    per = []
    for _ in range(windows):
        ev0.record(stream)
        E.run_sequence(tasks, opt)
        ev1.record(stream)
        torch.cuda.synchronize()
        per.append(ev0.elapsed_time(ev1) / reps * 1e-3)
    return sorted(per)[len(per) // 2], st["dispatches"] / reps


def time_kernel(torch, E, task_fn, reps, windows=3):
    """Average duration of back-to-back launches of one task, from HIP events
    on the stream the launches go to: the median over `windows` windows of
    `reps` launches.  Untimed runs of the same window first put its plan in
    the engine's plan cache (and its HIP graph in the graph cache, when graph
    replay is on), so no host planning or capture falls between the events."""
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tasks = E.prepare([task_fn() for _ in range(reps)])
    E.run_sequence(tasks, E.OPT_AD)
    E.run_sequence(tasks, E.OPT_AD)
    torch.cuda.synchronize()
    per = []
    for _ in range(windows):
        ev0.record(stream)
        E.run_sequence(tasks, E.OPT_AD)
        ev1.record(stream)
        torch.cuda.synchronize()
        per.append(ev0.elapsed_time(ev1) / reps * 1e-3)
    return sorted(per)[len(per) // 2]


# --------------------------------------------------------------------- band512
def bench_band(args, torch):
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import inputs, programs as PR
    w = inputs.band(args.seed, n=args.n)
    voxels = w.active_voxels
    K, W = args.steps, args.warmup

    def run_pipeline(opt):
        g = PR.load_workload(w, PR.JACOBI, 3)
        E.run_sequence([E.listgen(g)], opt)               # setup list (outside timing)
        # windows packed once, as an application re-running a window does
        warm = E.prepare(sum((PR.jacobi_step(g) for _ in range(W)), []))
        timed = E.prepare(sum((PR.jacobi_step(g) for _ in range(K)), []))
        if W:
            E.run_sequence(warm, opt)
        # whatever --warmup says, one untimed window of the timed shape: its
        # plan is then in the engine's plan cache when the timed window runs
        cold = E.run_sequence(timed, opt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = E.run_sequence(timed, opt)
        torch.cuda.synchronize()
        st["cold_optimizer_us"] = cold["optimizer_us"]
        return g, st, time.perf_counter() - t0

    g_opt, st_opt, t_opt = run_pipeline(E.OPT_ALL)
    x_opt = g_opt.channel(0).clone()
    # the same timed window once more with every launch bracketed by HIP
    # events on its stream (the brackets add about 1.5-2 us per launch, so
    # the roofline takes back-to-back launches between two events instead)
    E.timing_enable(True)
    try:
        E.run_sequence(sum((PR.jacobi_step(g_opt) for _ in range(K)), []), E.OPT_ALL)
        torch.cuda.synchronize()
        timed = {e["name"]: e for e in E.timing_collect()}
    finally:
        E.timing_enable(False)
    g_eag, st_eag, t_eag = run_pipeline(0)
    same = bool(torch.equal(x_opt, g_eag.channel(0)))
    del g_eag
    ablations = {}
    if not args.profile:
        for name, flags in _ablations():
            g_ab, st_ab, t_ab = run_pipeline(flags)
            ablations[name] = {"launches_per_step": st_ab["dispatches"] / K, "ms_per_step": t_ab / K * 1e3,
                               "equals_eager": bool(torch.equal(g_ab.channel(0), x_opt))}
            del g_ab
    reps = max(20, K)
    t_jac = time_kernel(torch, E, lambda: E.jacobi(g_opt, PR.JACOBI["x"], PR.JACOBI["b"], PR.JACOBI["xn"]), reps)
    t_copy = time_kernel(torch, E, lambda: E.copy(g_opt, PR.JACOBI["x"], PR.JACOBI["xn"]), reps)
    t_list = time_kernel(torch, E, lambda: E.listgen(g_opt), reps)
    t_jac_window = timed["jacobi"]["mean_us"] * 1e-6
    t_copy_window = timed["copy"]["mean_us"] * 1e-6
    achieved = 12.0 * voxels / t_jac / 1e9
    out = _base(K, W, voxels * K / t_opt, t_opt / K * 1e3,
                {"workload": "band512: sparse Jacobi, %d^3 domain, narrow band (|sdf| <= 1.5 blocks) around "
                             "4 seeded spheres, 8^3 fp32 leaves, bitmasked root" % args.n,
                 "seed": args.seed, "active_blocks": w.nblocks, "active_voxels": voxels,
                 "program_per_step": "listgen, jacobi, copy", "parallelism": "single GPU"})
    out.update({
        "launches_per_step": {"optimized": st_opt["dispatches"] / K, "eager": st_eag["dispatches"] / K},
        "eager": {"value": voxels * K / t_eag, "ms_per_step": t_eag / K * 1e3},
        "speedup_vs_eager": t_eag / t_opt,
        "optimized_equals_eager": same,
        "ablations": ablations,
        "optimizer_us_per_window": st_opt["optimizer_us"],
        "optimizer_us_first_window_of_timed_shape": st_opt["cold_optimizer_us"],
        "plan_cache_hits": st_opt["plan_cache_hits"],
        "timed_window_plan_cached": st_opt["plan_cache_hits"] > 0,
        "kernels": {"back_to_back": {"jacobi_us": t_jac * 1e6, "copy_us": t_copy * 1e6, "listgen_us": t_list * 1e6,
                                     "jacobi_GBs": achieved, "copy_GBs": 8.0 * voxels / t_copy / 1e9},
                    "timed_window_bracketed": {"jacobi_us": t_jac_window * 1e6, "copy_us": t_copy_window * 1e6,
                                               "launches": timed["jacobi"]["launches"] + timed["copy"]["launches"],
                                               "note": "each launch between its own pair of HIP events"},
                    "step_GBs_algorithmic": 20.0 * voxels / (t_opt / K) / 1e9},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": _jacobi_traffic() if args.seed == 0 else None,
                     "kernel": "k_stencil_lds<JACOBI> (12 B per active voxel: x, b read; xn written); mean of "
                               "%d back-to-back launches over the workload's list between two HIP events on the "
                               "launch stream, median of 3 such windows (plan cached)" % reps,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "algorithmic_bytes_per_launch": 12 * voxels},
    })
    if not args.no_cpu_baseline and not args.profile:
        from oracle import OracleGrid
        og = OracleGrid(w.n, 3, "f32")
        og.load(w.blocks, {"b": w.channels["b"]}, {"x": 0, "xn": 1, "b": 2})

        def it(_):
            og.listgen()
            og.jacobi(0, 2, 1)
            og.copy(0, 1)
        calls, dt, core = cpu_leg(it, 1e9, args.cpu_iters)
        out["cpu_baseline"] = cpu_baseline(voxels * calls / dt, "voxel-steps/s",
                                           "%d iterations (listgen, jacobi, copy) of the full band512 workload, "
                                           "seed %d" % (calls, args.seed), dt, core)
    return out


# ----------------------------------------------------------------------- shell
def bench_shell(args, torch):
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import inputs, programs as PR
    w = inputs.shell(args.seed)
    K, W = args.steps, args.warmup
    coords = torch.as_tensor(w.blocks, device="cuda")
    res = {}
    for name, opt in (("optimized", E.OPT_ALL), ("eager", 0)):
        g = PR.load_workload(w, PR.SHELL, 2)
        E.run_sequence(PR.shell_setup(g, coords), opt)
        if W:
            E.run_sequence(sum((PR.shell_step(g, coords) for _ in range(W)), []), opt)
        timed = E.prepare(sum((PR.shell_step(g, coords) for _ in range(K)), []))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = E.run_sequence(timed, opt)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0, st)
    t, st = res["optimized"]
    out = _base(K, W, w.active_voxels * K / t, t / K * 1e3,
                {"workload": "shell64: 64^3 spherical shell (%d blocks), per step activate, listgen, lap_update, "
                             "listgen, axpy" % w.nblocks, "seed": args.seed})
    out.update({"launches_per_step": {"optimized": st["dispatches"] / K, "eager": res["eager"][1]["dispatches"] / K},
                "eager": {"value": w.active_voxels * K / res["eager"][0], "ms_per_step": res["eager"][0] / K * 1e3},
                "speedup_vs_eager": res["eager"][0] / t, "plan_cache_hits": st["plan_cache_hits"]})
    # the optimized step launches lap_update (a read, out written: 8 B per
    # voxel) and axpy (a, out read, a written: 12 B); the longer is the
    # dominant launch.  The working set (a few hundred KiB) stays in L2, so
    # the HBM fraction is context only: this workload is bound by launches.
    g = PR.load_workload(w, PR.SHELL, 2)
    E.run_sequence(PR.shell_setup(g, coords), E.OPT_ALL)
    t_lap = time_kernel(torch, E, lambda: E.lap_update(g, PR.SHELL["a"], PR.SHELL["out"], 0.1), 100)
    t_axpy = time_kernel(torch, E, lambda: E.axpy(g, PR.SHELL["a"], PR.SHELL["out"], 0.5), 100)
    name, tk, per = max((("k_stencil_lds<LAP_UPDATE>", t_lap, 8), ("k_elem<AXPY>", t_axpy, 12)), key=lambda e: e[1])
    out["kernels"] = {"lap_update_us": t_lap * 1e6, "axpy_us": t_axpy * 1e6}
    out["roofline"] = roofline(per * w.active_voxels / tk / 1e9,
                               "%s (%d B per active voxel), mean of 100 back-to-back launches between two HIP events "
                               "on the launch stream, median of 3 windows; L2-resident working set" % (name, per),
                               per * w.active_voxels)
    if not args.no_cpu_baseline and not args.profile:
        from oracle import programs as OP
        calls, dt, core = cpu_leg(lambda _: OP.shell_program(w.n, w.blocks, w.channels["a"], 100), 5.0, 100)
        out["cpu_baseline"] = cpu_baseline(w.active_voxels * 100 * calls / dt, "voxel-steps/s",
                                           "%d runs of the 100-step shell64 program (setup included), seed %d"
                                           % (calls, args.seed), dt, core)
    return out


# ------------------------------------------------------------------- particles
def bench_particles(args, torch):
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import inputs, programs as PR
    from paper_2012_08141_amd.grid import SparseGrid
    p = inputs.particles(args.seed)
    K, W = args.steps, args.warmup
    W += W % 2          # keep the grid alternation in phase, so the timed window's plan is cached
    res = {}
    runs = [("optimized", E.OPT_ALL), ("eager", 0)] + ([] if args.profile else _ablations())
    for name, opt in runs:
        grids = [SparseGrid(p.n, 7, "pointer", (p.n // 8) ** 3, particle_capacity=p.nparticles) for _ in range(2)]
        x, v, m = PR.device_particles(p)
        step = lambda t: PR.particle_step(grids, t, x, v, m, p.params["dt"], 1.0 / p.n)
        # warm-up in windows of the timed shape: the first plans from the
        # cold engine state, the next from the steady state the timed window sees
        for t0 in range(0, W, K):
            E.run_sequence(sum((step(t) for t in range(t0, min(t0 + K, W))), []), opt)
        tasks = E.prepare(sum((step(t) for t in range(W, W + K)), []))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = E.run_sequence(tasks, opt)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0, st, grids, (x, v, m))
    t, st, grids, _ = res["optimized"]
    vox = sum(len(g.active_cells()) for g in grids) * 512 // 2
    out = _base(K, W, vox * K / t, t / K * 1e3,
                {"workload": "particles256: 2M particles in 3 boxes, 256^3 grid, PIC P2G/normalise/G2P, two "
                             "alternating pointer-rooted grids", "seed": args.seed, "particles": p.nparticles})
    out.update({"particle_steps_per_s": p.nparticles * K / t,
                "launches_per_step": {"optimized": st["dispatches"] / K, "eager": res["eager"][1]["dispatches"] / K},
                "tasks_per_step": {"optimized": st["tasks_launched"] / K, "eager": res["eager"][1]["tasks_launched"] / K},
                "scatter": "binned: keys, LDS-histogram ranks, scan, place, LDS tile per bin (5 dispatches); a fused "
                           "gather-advect-scatter node reuses the previous binning for up to %d scatters (gather "
                           "rewriting the records, advection, tiles: 3 dispatches)" % E.get_option(L.AT_OPTION_BIN_REUSE),
                "gather": "through the previous scatter's bins (LDS velocity tile per quarter bin)",
                "eager": {"value": vox * K / res["eager"][0], "ms_per_step": res["eager"][0] / K * 1e3,
                          "particle_steps_per_s": p.nparticles * K / res["eager"][0]},
                "speedup_vs_eager": res["eager"][0] / t, "fusions": st["fusions"],
                "stores_eliminated": st["stores_eliminated"], "optimizer_us_per_window": st["optimizer_us"],
                "plan_cache_hits": st["plan_cache_hits"],
                "ablations": {name: {"tasks_per_step": res[name][1]["tasks_launched"] / K,
                                     "launches_per_step": res[name][1]["dispatches"] / K,
                                     "ms_per_step": res[name][0] / K * 1e3}
                              for name, _ in runs[2:]}})
    # dominant launch: the fused gather-advect-scatter node (G2P from the
    # previous grid, x += dt v, P2G into this one; three or five dispatches
    # depending on bin reuse), timed between HIP events around each launch
    # over two more windows of the timed shape (plan cached)
    x, v, m = res["optimized"][3]
    tasks = E.prepare(sum((PR.particle_step(grids, t_, x, v, m, p.params["dt"], 1.0 / p.n)
                           for t_ in range(W + K, W + 2 * K)), []))
    E.run_sequence(tasks, E.OPT_ALL)
    ents = window_kernel_means(E, tasks, E.OPT_ALL, 2)
    dom = max(ents, key=lambda e: e["launches"] * e["mean_us"])
    out["kernels"] = {"%s/%d" % (e["name"], e["members"]): {"launches": e["launches"], "mean_us": e["mean_us"]}
                      for e in ents}
    # 48 B per particle (x and v read and written) + the gathered grid
    # velocity (12 B per active voxel) + the scattered mass and momentum
    # (16 B per active voxel)
    alg = 48 * p.nparticles + 28 * vox
    if dom["kind"] == L.AT_TASK_G2P and dom["members"] == 3:
        out["roofline"] = roofline(alg / (dom["mean_us"] * 1e-6) / 1e9,
                                   "fused G2P2G node (gather, advect, binned scatter): 48 B per particle + 28 B per "
                                   "active voxel; mean over %d launches, each between its own HIP events (adds "
                                   "about 2 us); HBM fraction is context: the node is bound by the tile sums and "
                                   "atomics" % dom["launches"], alg)
    if not args.no_cpu_baseline and not args.profile:
        from oracle import programs as OP
        steps = 2
        rr = {}

        def run(_):
            rr["r"] = OP.particle_program(p.n, p.x, p.v, p.m, steps, p.params["dt"], "f32")
        calls, dt, core = cpu_leg(run, 1e9, 1)
        cvox = (len(rr["r"]["cells0"]) + len(rr["r"]["cells1"])) * 512 // 2
        out["cpu_baseline"] = cpu_baseline(cvox * steps / dt, "voxel-steps/s",
                                           "the first %d steps of the full particles256 workload (2M particles), "
                                           "seed %d" % (steps, args.seed), dt, core)
        out["cpu_baseline"]["particle_steps_per_s"] = p.nparticles * steps / dt
    return out


# ------------------------------------------------------------------------ mpm
def bench_mpm(args, torch):
    """The paper's MLS-MPM falling cube (256^3 grid, 16,777,216 particles):
    a step is one substep (listgen, fill, p2g_mls, listgen, mpm_grid,
    g2p_apic, advect; optimized: the G2P2G node with the stores of v and C
    dropped)."""
    import gc
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import inputs, programs as PR
    mp = inputs.mpm_cube(args.seed, 256, side=0.5)
    prm = mp.params
    K, W = args.steps, args.warmup
    W += W % 2          # keep the grid alternation in phase, so the timed window's plan is cached
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    runs = [("optimized", E.OPT_ALL), ("eager", 0)] + ([] if args.profile else _ablations())
    for name, opt in runs:
        E.reset()
        grids = PR.mpm_grids(mp)
        x, v, C, F = PR.device_mpm(mp)
        step = lambda t: PR.mpm_step(grids, t, x, v, C, F, prm)
        for t0 in range(0, W, K):
            E.run_sequence(sum((step(t) for t in range(t0, min(t0 + K, W))), []), opt)
        tasks = E.prepare(sum((step(t) for t in range(W, W + K)), []))
        torch.cuda.synchronize()
        ev0.record(stream)
        st = E.run_sequence(tasks, opt)
        ev1.record(stream)
        torch.cuda.synchronize()
        vox = sum(len(g.active_cells()) for g in grids) * 512 // 2
        res[name] = (ev0.elapsed_time(ev1) * 1e-3, st, vox)
        if name == "optimized":
            keep = (grids, x, v, C, F)
        else:
            del grids, x, v, C, F
        gc.collect()
        torch.cuda.empty_cache()
    t, st, vox = res["optimized"]
    npart = mp.nparticles
    out = _base(K, W, vox * K / t, t / K * 1e3,
                {"workload": "mpm256: MLS-MPM falling cube, 16,777,216 fixed-corotated particles (2 per cell per "
                             "axis, block-ordered lattice), 256^3 grid, two alternating bitmask-rooted grids, "
                             "dt 1e-4", "seed": args.seed, "particles": npart})
    out.update({"particle_steps_per_s": npart * K / t,
                "launches_per_step": {"optimized": st["dispatches"] / K, "eager": res["eager"][1]["dispatches"] / K},
                "eager": {"value": res["eager"][2] * K / res["eager"][0], "ms_per_step": res["eager"][0] / K * 1e3,
                          "particle_steps_per_s": npart * K / res["eager"][0]},
                "speedup_vs_eager": res["eager"][0] / t, "fusions": st["fusions"],
                "stores_eliminated": st["stores_eliminated"], "plan_cache_hits": st["plan_cache_hits"],
                "optimizer_us_per_window": st["optimizer_us"],
                "ablations": {name: {"launches_per_step": res[name][1]["dispatches"] / K,
                                     "ms_per_step": res[name][0] / K * 1e3,
                                     "stores_eliminated": res[name][1]["stores_eliminated"]}
                              for name, _ in runs[2:]}})
    # dominant launch: the fused G2P2G node, timed between HIP events around
    # each launch over two more windows of the timed shape (plan cached)
    grids, x, v, C, F = keep
    tasks = E.prepare(sum((PR.mpm_step(grids, t_, x, v, C, F, prm) for t_ in range(W + K, W + 2 * K)), []))
    E.run_sequence(tasks, E.OPT_ALL)
    ents = window_kernel_means(E, tasks, E.OPT_ALL, 2)
    out["kernels"] = {"%s/%d" % (e["name"], e["members"]): {"launches": e["launches"], "mean_us": e["mean_us"]}
                      for e in ents}
    dom = max(ents, key=lambda e: e["launches"] * e["mean_us"])
    if dom["kind"] == L.AT_TASK_G2P_APIC and dom["members"] == 3:
        tf = MPM_FLOPS_PER_PARTICLE * npart / (dom["mean_us"] * 1e-6) / 1e12
        out["roofline"] = {"bound": "alu", "achieved": tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": tf / FP32_PEAK_TFLOPS, "traffic": None,
                           "kernel": "k_mpm<G2P|ADVECT|P2G> (fused G2P2G node): %d algorithmic fp32 operations "
                                     "per particle; mean over %d launches, each between its own HIP events"
                                     % (MPM_FLOPS_PER_PARTICLE, dom["launches"]),
                           "algorithmic_flops_per_launch": MPM_FLOPS_PER_PARTICLE * npart,
                           "hbm_GBs_algorithmic": 96.0 * npart / (dom["mean_us"] * 1e-6) / 1e9,
                           "hbm_note": "96 B per particle (x and F read and written)"}
    del keep, grids, x, v, C, F
    if not args.no_cpu_baseline and not args.profile:
        from oracle import programs as OP
        sample = 1 << 18     # the first 262,144 particles: 512 whole blocks of the lattice
        sx, sv, sC, sF = (a[:, :sample].copy() for a in (mp.x, mp.v, mp.C, mp.F))
        calls, dt, core = cpu_leg(lambda _: OP.mpm_program(256, sx, sv, sC, sF, 1, prm["dt"], prm["mass"],
                                                            prm["vol"], prm["mu"], prm["lam"], prm["gravity"],
                                                            prm["bound"], "f64"), 10.0, 200)
        out["cpu_baseline"] = cpu_baseline(sample * calls / dt, "particle-steps/s",
                                           "%d substeps of the first %d particles of the mpm256 cube (fp64 oracle), "
                                           "seed %d" % (calls, sample, args.seed), dt, core)
    return out


# --------------------------------------------------------------------- serving
def bench_serving(args, torch):
    import numpy as np
    from paper_2012_08141_amd import autotune, inputs
    from paper_2012_08141_amd.batching import BatchArena
    from paper_2012_08141_amd.serving import JacobiServer, make_requests, serve_eager_fifo
    count = args.requests
    reqs0 = make_requests(args.seed, count, np.zeros(count))
    # tune the batched launch on the full closed batch (long windows)
    scratch = BatchArena(128, count, sum(r.nblocks for r in reqs0))
    for r in reqs0:
        scratch.admit(r.cells_dev, r.b_dev, (1 << 31) - 1)     # active for good
    tune = autotune.tune_batch(scratch, "batch128x%d" % count)
    del scratch
    # closed-batch capacity: the second of two runs (the first warms the
    # allocator, the graph and the clocks)
    for _ in range(2):
        srv = JacobiServer(128, args.budget_mib << 20, 64, tune["iters_per_replay"], tune["workgroups"],
                           waves=tune["waves"])
        closed = srv.serve(make_requests(args.seed, count, np.zeros(count)), realtime=False)
        del srv
    cap_rps = count / closed.makespan
    rate = args.load * cap_rps
    arr = inputs.poisson_arrivals(args.seed, count, rate)
    reqs = make_requests(args.seed, count, arr)
    srv2 = JacobiServer(128, args.budget_mib << 20, 64, tune["iters_per_replay"], tune["workgroups"],
                        waves=tune["waves"])
    st = srv2.serve(reqs, realtime=True)
    base = serve_eager_fifo(make_requests(args.seed, count, arr), realtime=True)
    s, b = st.summary(), base.summary()
    out = _base(count, 0, s["voxel_steps_per_s"], s["makespan_s"] * 1e3 / count,
                {"workload": "serving: %d Jacobi requests (128^3, 32-4096 blocks log-uniform, 50 iterations), "
                             "Poisson arrivals at %.2f x batched capacity, HBM budget %d MiB" %
                             (count, args.load, args.budget_mib), "seed": args.seed})
    out.update({"latency_ms": {"p50": s["p50_ms"], "p99": s["p99_ms"], "mean": s["mean_ms"]},
                "closed_batch_voxel_steps_per_s": closed.voxel_iters / closed.makespan,
                "arrival_rate_per_s": rate, "max_resident": s["max_resident"], "replays": s["replays"],
                "autotune": {k: v for k, v in tune.items() if k != "candidates"},
                "eager_fifo": {"value": b["voxel_steps_per_s"], "latency_ms": {"p50": b["p50_ms"], "p99": b["p99_ms"]}},
                "speedup_vs_eager": s["voxel_steps_per_s"] / b["voxel_steps_per_s"]})
    # dominant launches: one batched iteration (the Jacobi and the copy
    # launch over the whole work list, 20 B per voxel) over the resident set
    # the budget admits (the first requests of the stream that fit it), timed
    # between HIP events around replays of the server's captured graph
    budget_blocks = (args.budget_mib << 20) // BatchArena.footprint(1)
    first, nb = [], 0
    for r in reqs0:
        if nb + r.nblocks > budget_blocks or len(first) == 64:
            break
        first.append(r)
        nb += r.nblocks
    arena = BatchArena(128, 64, budget_blocks)
    for r in first:
        arena.admit(r.cells_dev, r.b_dev, (1 << 31) - 1)
    K = tune["iters_per_replay"]
    g = arena.capture(K, tune["workgroups"], tune["waves"])
    g.replay()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(20):
        g.replay()
    ev1.record()
    torch.cuda.synchronize()
    s_iter = ev0.elapsed_time(ev1) * 1e-3 / (20 * K)
    del g, arena
    vox = nb * 512
    out["closed_batch_iteration_all_resident_s"] = tune["s_per_iter"]
    out["roofline"] = roofline(20.0 * vox / s_iter / 1e9,
                               "one batched Jacobi iteration (k_batch_lds jacobi + k_batch copy launches, 20 B per active voxel) "
                               "over the %d requests (%d blocks) the %d MiB budget admits first; mean per iteration "
                               "over 20 replays of the captured %d-iteration graph between two HIP events; the "
                               "working set is near the 256 MiB last-level cache" % (len(first), nb, args.budget_mib, K),
                               20 * vox)
    if not args.no_cpu_baseline and not args.profile:
        from oracle import programs as OP
        done = []

        def one(i):
            r = reqs0[i]
            blocks = np.stack(np.unravel_index(r.cells, (16, 16, 16)), axis=1).astype(np.int32)
            OP.jacobi_program(128, blocks, r.b, r.iters)
            done.append(r.voxel_iters)
        calls, dt, core = cpu_leg(one, 10.0, count)
        out["cpu_baseline"] = cpu_baseline(sum(done) / dt, "voxel-steps/s",
                                           "the first %d requests of the stream solved one at a time (50 iterations "
                                           "of listgen, jacobi, copy each), seed %d" % (calls, args.seed), dt, core)
    return out


# ------------------------------------------------------------------- diffusion
def bench_diffusion(args, torch):
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import inputs
    from paper_2012_08141_amd.autodiff import DiffusionProblem, diffusion_loss
    w = inputs.diffusion(args.seed)
    a0 = torch.as_tensor(w.channels["a"], device="cuda")
    k = torch.as_tensor(w.channels["k"], device="cuda")
    tgt = torch.as_tensor(w.channels["target"], device="cuda")
    # the two forms alternate repetition by repetition, so clock ramps and
    # host noise fall on both alike
    forms = (("optimized", E.OPT_ALL), ("eager", 0))
    probs = {name: DiffusionProblem(w.n, w.blocks, 0.1, 20, 5, opt_flags=opt) for name, opt in forms}
    times = {name: [] for name, _ in forms}
    disp, grads = {}, {}
    for _ in range(args.warmup + args.steps):
        for name, _ in forms:
            a = a0.clone().requires_grad_(True)
            kk = k.clone().requires_grad_(True)
            torch.cuda.synchronize()
            d0 = E.dispatch_count()
            t0 = time.perf_counter()
            loss = diffusion_loss(a, kk, tgt, probs[name])
            loss.backward()
            torch.cuda.synchronize()
            times[name].append(time.perf_counter() - t0)
            disp[name] = E.dispatch_count() - d0
            grads[name] = (a.grad.clone(), kk.grad.clone())
    res = {}
    for name, _ in forms:
        tt = sorted(times[name][args.warmup:])
        res[name] = (tt[len(tt) // 2], disp[name], grads[name][0], grads[name][1])
    del probs
    t, d, ga, gk = res["optimized"]
    te, de, gae, gke = res["eager"]
    out = _base(args.steps, args.warmup, w.active_voxels * 20 / t, t * 1e3,
                {"workload": "diffusion128: 20 diffusion steps + adjoint (checkpoints every 5) on a 128^3 shell "
                             "(%d blocks)" % w.nblocks, "seed": args.seed})
    out.update({"note": "value counts forward steps only; one step = forward and backward of the whole 20-step "
                        "loss; ms_per_step is the median over the timed repetitions",
                "launches_per_step": {"optimized": d, "eager": de},
                "eager": {"value": w.active_voxels * 20 / te, "ms_per_step": te * 1e3},
                "speedup_vs_eager": te / t,
                "gradients_equal_eager": bool(torch.equal(ga, gae) and torch.equal(gk, gke))})
    # dominant launch: the adjoint step (a, k, lam', gk read; lam, gk
    # written: 24 B per active voxel); the forward step moves 12 B
    pr = DiffusionProblem(w.n, w.blocks, 0.1, 20, 5, opt_flags=E.OPT_ALL)
    G = pr.grid
    t_adj = time_kernel(torch, E, lambda: E.diffuse_adj(G, pr.ck[0], pr.K, pr.LA, pr.LB, pr.GK, 0.1), 100)
    t_fwd = time_kernel(torch, E, lambda: E.diffuse(G, pr.ck[0], pr.K, pr.seg[1], 0.1), 100)
    out["kernels"] = {"diffuse_adj_us": t_adj * 1e6, "diffuse_us": t_fwd * 1e6}
    out["roofline"] = roofline(24.0 * w.active_voxels / t_adj / 1e9,
                               "k_stencil_pipe<DIFFUSE_ADJ> (24 B per active voxel), mean of 100 back-to-back "
                               "launches between two HIP events on the launch stream, median of 3 windows; the "
                               "working set (under 8 MiB) stays in cache, so the HBM fraction is context",
                               24 * w.active_voxels)
    del pr
    if not args.no_cpu_baseline and not args.profile:
        from oracle import programs as OP
        calls, dt, core = cpu_leg(lambda _: OP.diffusion_grad(w.n, w.blocks, w.channels["a"], w.channels["k"],
                                                              w.channels["target"], 0.1, 20, "f32"), 5.0, 50)
        out["cpu_baseline"] = cpu_baseline(w.active_voxels * 20 * calls / dt, "voxel-steps/s",
                                           "%d forward + adjoint passes of the full diffusion128 loss (20 steps, "
                                           "all states stored), seed %d; value counts forward steps" % (calls, args.seed),
                                           dt, core)
    return out


# ------------------------------------------------------------------- advection
def bench_advection(args, torch, mac=False):
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import inputs, programs as PR
    w = inputs.tube(args.seed)
    dt = w.params["dt"]
    K, W = args.steps, args.warmup
    names = {"q0": 0, "q1": 1, "q2": 2, "v0": 3, "v1": 4, "v2": 5}
    # the MacCormack workload back-traces with RK3, as the paper's benchmark does
    step_fn, nch = ((lambda g_, dt_: PR.maccormack_step(g_, dt_, rk3=True)), 15) if mac else (PR.advection_step, 9)
    res = {}
    for name, opt in (("optimized", E.OPT_ALL), ("eager", 0)):
        E.reset()
        g = PR.load_workload(w, names, nch)
        step = E.prepare(step_fn(g, dt))               # one engine window per step
        for _ in range(max(W, 2)):
            E.run_sequence(step, opt)
        torch.cuda.synchronize()
        d0 = E.dispatch_count()
        t0 = time.perf_counter()
        for _ in range(K):
            E.run_sequence(step, opt)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0, E.dispatch_count() - d0, E.plan_sequence(step_fn(g, dt), opt)[0])
        del step, g
    t, d, plan = res["optimized"]
    te, de, plane = res["eager"]
    out = _base(K, W, w.active_voxels * K / t, t / K * 1e3,
                {"workload": ("maccormack256: MacCormack advection (forward and backward semi-Lagrangian steps "
                              "with RK3 back-traces, clamped correction, copy back; each after a listgen)" if mac else
                              "advection256: semi-Lagrangian advection (listgen, advect, listgen, copy)") +
                             " of 3 scalar fields by a swirling velocity on a 256^3 tube (r 0.32-0.45, %d blocks), "
                             "one engine window per step" % w.nblocks, "seed": args.seed})
    # per-pass ablations of the step's plan (launches per step, as in the
    # paper's ablation tables), planned from the steady state
    abl = {}
    E.reset()
    ga = PR.load_workload(w, names, nch)
    sa = step_fn(ga, dt)
    E.run_sequence(sa, E.OPT_ALL)
    for key, fl in (("no_lgr", E.OPT_ALL & ~E.OPT_LGR), ("no_ad", E.OPT_ALL & ~E.OPT_AD),
                    ("no_fusion", E.OPT_ALL & ~E.OPT_FUSE), ("no_dse", E.OPT_ALL & ~E.OPT_DSE)):
        pl = E.plan_sequence(sa, fl)[0]
        abl[key] = {"launches_per_step": len(pl), "paper_task_count": E.paper_task_count(pl)}
    del sa, ga
    out.update({"launches_per_step": {"optimized": d / K, "eager": de / K},
                "ablations": abl,
                "paper_task_count_per_step": {"optimized": E.paper_task_count(plan),
                                              "eager": E.paper_task_count(plane)},
                "eager": {"value": w.active_voxels * K / te, "ms_per_step": te / K * 1e3},
                "speedup_vs_eager": te / t})
    # dominant launch of the optimized step, timed between HIP events around
    # each launch over further windows (plan cached).  Algorithmic bytes per
    # active voxel of a fused node: each field's q read and output written
    # (advection: 8 B; MacCormack correction: q, fwd, bwd read, out written,
    # 16 B; copy 8 B), plus the shared velocity (12 B) when the node samples it
    E.reset()
    g = PR.load_workload(w, names, nch)
    step = E.prepare(step_fn(g, dt))
    for _ in range(2):
        E.run_sequence(step, E.OPT_ALL)
    ents = window_kernel_means(E, step, E.OPT_ALL, 5)
    dom = max(ents, key=lambda e: e["launches"] * e["mean_us"])
    per_field = {L.AT_OP_ADVECT: 8, L.AT_OP_MACCORMACK: 16, L.AT_OP_COPY: 8}
    out["kernels"] = {"%s/%d" % (e["name"], e["members"]): {"launches": e["launches"], "mean_us": e["mean_us"]}
                      for e in ents}
    if dom["kind"] == L.AT_TASK_STENCIL and dom["op"] in per_field:
        per = per_field[dom["op"]] * dom["members"] + (12 if dom["op"] != L.AT_OP_COPY else 0)
        out["roofline"] = roofline(per * w.active_voxels / (dom["mean_us"] * 1e-6) / 1e9,
                                   "%s node fusing %d fields (%d B per active voxel); mean over %d launches, each "
                                   "between its own HIP events (adds about 2 us per launch)"
                                   % (dom["name"], dom["members"], per, dom["launches"]), per * w.active_voxels)
    del step, g
    if not args.no_cpu_baseline and not args.profile:
        from oracle import programs as OP
        fn = ((lambda: OP.maccormack_program(w.n, w.blocks, w.channels, dt, 1, rk3=True)) if mac else
              (lambda: OP.advection_program(w.n, w.blocks, w.channels, dt, 1)))
        calls, dt_cpu, core = cpu_leg(lambda _: fn(), 5.0, 10)
        out["cpu_baseline"] = cpu_baseline(w.active_voxels * calls / dt_cpu, "voxel-steps/s",
                                           "%d one-step runs of the full %s program (3 fields, setup included), "
                                           "seed %d" % (calls, "maccormack256" if mac else "advection256", args.seed),
                                           dt_cpu, core)
    return out


# ------------------------------------------------------------------- multigrid
def bench_multigrid(args, torch):
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import inputs, programs as PR
    w = inputs.band(args.seed, n=256)
    K, W = args.steps, args.warmup
    nl = 4

    def timed_run(window, opt):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = E.run_sequence(window, opt)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    res = {}
    for name, opt in (("optimized", E.OPT_ALL), ("eager", 0)):
        E.reset()
        lv = PR.mg_levels(w, nl)
        # the first window builds the coarse levels; windows of the timed
        # window's shape then leave its plan in the engine's plan cache
        if W:
            E.run_sequence(sum((PR.mg_vcycle(lv) for _ in range(W)), []), opt)
        steps = sum((PR.mg_vcycle(lv) for _ in range(K)), [])
        timed = E.prepare(steps)
        cold = E.run_sequence(timed, opt)["optimizer_us"]
        plan, _ = E.plan_sequence(steps, opt)
        E.run_sequence(timed, opt)
        t, st = timed_run(timed, opt)
        wg = None
        if opt:
            E.set_option(L.AT_OPTION_GRAPHS, 1)
            E.run_sequence(timed, opt)                     # captures the window's graph
            wg = timed_run(timed, opt)[0]
            E.set_option(L.AT_OPTION_GRAPHS, 0)
        res[name] = (t, st, plan, cold, wg)
        del lv
    t, st, plan, cold, wg = res["optimized"]
    te, ste, plane, _, _ = res["eager"]
    lists = {k: sum(1 for e in p if e["kind"] == 2) for k, p in (("optimized", plan), ("eager", plane))}
    out = _base(K, W, w.active_voxels * K / t, t / K * 1e3,
                {"workload": "multigrid256: V-cycles on a 256^3 narrow band (%d blocks; %d levels down to 32^3), "
                             "per cycle 2+2 damped-Jacobi sweeps per level, 8 on the coarsest, residual "
                             "restriction and injection prolongation; a step is one V-cycle" % (w.nblocks, nl),
                 "seed": args.seed})
    out.update({"launches_per_step": {"optimized": st["dispatches"] / K, "eager": ste["dispatches"] / K},
                "list_generations_per_step": {"optimized": lists["optimized"] / K, "eager": lists["eager"] / K},
                "paper_task_count_per_step": {"optimized": E.paper_task_count(plan) / K,
                                              "eager": E.paper_task_count(plane) / K},
                "activations_demoted": st["activations_demoted"],
                "optimizer_us": {"timed_window": st["optimizer_us"], "cold_plan": cold,
                                 "plan_cache_hits": st["plan_cache_hits"]},
                "eager": {"value": w.active_voxels * K / te, "ms_per_step": te / K * 1e3},
                "optimized_with_graph_replay": {"value": w.active_voxels * K / wg, "ms_per_step": wg / K * 1e3},
                "speedup_vs_eager": te / t})
    # dominant launch: the fine level's smoothing stencil, which the
    # optimizer fuses with the update after it (t = J(x); t -= x) into one
    # k_stencil_tail launch: x, b read, t written (12 B per fine voxel).
    # Consecutive groups swap x and t, so each reads the previous group's
    # output at neighbours and the groups cannot fuse with one another.
    E.reset()
    lv = PR.mg_levels(w, nl)
    g0 = lv[0]

    def group(r):
        x, t = (PR.MG["x"], PR.MG["t"]) if r % 2 == 0 else (PR.MG["t"], PR.MG["x"])
        return [E.listgen(g0), E.jacobi(g0, x, PR.MG["b"], t), E.listgen(g0), E.axpy(g0, t, x, -1.0)]

    t_fused, lpg = time_group(torch, E, group, 100, E.OPT_ALL & ~E.OPT_DSE)    # (DSE would drop stores)
    out["kernels"] = {"fine_jacobi_tail_us": t_fused * 1e6, "launches_per_group": lpg}
    if lpg == 1:
        out["roofline"] = roofline(12.0 * w.active_voxels / t_fused / 1e9,
                                   "k_stencil_tail_lds (fine-level jacobi fused with t -= x; 12 B per fine active voxel), "
                                   "mean of 100 back-to-back launches between two HIP events on the launch stream, "
                                   "median of 3 windows", 12 * w.active_voxels)
    del lv, g0
    if not args.no_cpu_baseline and not args.profile:
        from oracle import programs as OP
        calls, dt, core = cpu_leg(lambda _: OP.multigrid_program(w.n, w.blocks, w.channels["b"], 2, levels=nl),
                                  5.0, 10)
        out["cpu_baseline"] = cpu_baseline(w.active_voxels * 2 * calls / dt, "voxel-steps/s",
                                           "%d solves of 2 V-cycles (%d levels) of the full multigrid256 workload, "
                                           "seed %d; value counts fine voxel-cycles" % (calls, nl, args.seed), dt, core)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--workload", default="band512", choices=["band512", "shell", "particles", "serving", "diffusion",
                                                           "multigrid", "advection", "maccormack", "mpm"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=90)
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--budget-mib", type=int, default=256)
    ap.add_argument("--no-variants", action="store_true",
                    help="run fused element-wise nodes in the interpreter, not their compiled variants")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3 (no CPU baseline)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, one plain torch copy of this many MiB (the known-size kernel that "
                         "scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the sharding design is documented, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    # warm-up windows have the timed window's shape, so the timed window
    # finds its plan in the engine's plan cache (the cold planning time is
    # reported beside the result)
    defaults = {"band512": (100, 100), "shell": (100, 100), "particles": (20, 40), "serving": (256, 0),
                "diffusion": (40, 5), "multigrid": (20, 5), "advection": (50, 5),
                "maccormack": (30, 5), "mpm": (16, 32)}
    d = defaults[args.workload]
    args.steps = d[0] if args.steps is None else args.steps
    args.warmup = d[1] if args.warmup is None else args.warmup

    import torch
    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    # fused element-wise struct-fors run their compiled variants, built at
    # first use (inside the untimed warm-up windows); unfused (eager) tasks
    # never use them
    if not args.no_variants:
        E.set_option(L.AT_OPTION_VARIANTS, 2)
    settle_host()
    fn = {"band512": bench_band, "shell": bench_shell, "particles": bench_particles, "serving": bench_serving,
          "diffusion": bench_diffusion, "multigrid": bench_multigrid,
          "advection": bench_advection,
          "maccormack": lambda a, t: bench_advection(a, t, mac=True), "mpm": bench_mpm}[args.workload]
    out = fn(args, torch)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 18
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 4 * n
    out["compiled_variants"] = E.get_option(L.AT_OPTION_VARIANTS_LOADED)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
