"""Benchmark: active voxel-steps/s and launches/step of the sparse Jacobi
pipeline (512^3 domain, narrow band around 4 random spheres, 8^3 fp32
leaves under a bitmasked root), optimized vs eager, on one GPU.

A step is one Jacobi iteration of the whole program -- listgen, jacobi
(xn = (sum of 6 neighbours of x + b) / 6), copy (x = xn) -- over every
active voxel.  The optimized pipeline runs the same task list through the
inter-kernel optimizer (list generation removal, activation demotion, task
fusion, dead store elimination).  Inputs are resident in HBM before timing;
the timed region is K steps submitted as one engine window (plan lookup and
launch included) bracketed by device synchronisation.

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=30)
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3 (no baseline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharding design is documented, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import inputs, programs as PR

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    w = inputs.band(args.seed, n=args.n)
    voxels = w.active_voxels
    K, W = args.steps, args.warmup

    def run_pipeline(opt):
        g = PR.load_workload(w, PR.JACOBI, 3)
        E.run_sequence([E.listgen(g)], opt)               # setup list (outside timing)
        warm = sum((PR.jacobi_step(g) for _ in range(W)), [])
        timed = sum((PR.jacobi_step(g) for _ in range(K)), [])
        if W:
            E.run_sequence(warm, opt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = E.run_sequence(timed, opt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return g, st, t1 - t0

    g_opt, st_opt, t_opt = run_pipeline(E.OPT_ALL)
    g_eag, st_eag, t_eag = run_pipeline(0)
    same = bool(torch.equal(g_opt.channel(0), g_eag.channel(0)))

    # dominant kernel: the Jacobi stencil, timed alone with HIP events on the
    # stream it is launched on (the copy kernel is timed the same way)
    stream = torch.cuda.current_stream()

    def time_kernel(task_fn, reps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tasks = [task_fn() for _ in range(reps)]
        E.run_sequence(tasks[:2], E.OPT_AD)
        torch.cuda.synchronize()
        ev0.record(stream)
        E.run_sequence(tasks, E.OPT_AD)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps * 1e-3   # seconds per launch

    reps = max(20, K)
    t_jac = time_kernel(lambda: E.jacobi(g_opt, PR.JACOBI["x"], PR.JACOBI["b"], PR.JACOBI["xn"]), reps)
    t_copy = time_kernel(lambda: E.copy(g_opt, PR.JACOBI["x"], PR.JACOBI["xn"]), reps)
    jac_bytes = 12.0 * voxels        # read x, read b, write xn
    copy_bytes = 8.0 * voxels        # read xn, write x
    achieved = jac_bytes / t_jac / 1e9

    value = voxels * K / t_opt
    out = {
        "metric": "active voxel-steps/s + launches/step, optimized vs eager pipeline, 1 GPU",
        "value": value,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": t_opt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "band512: sparse Jacobi, %d^3 domain, narrow band (|sdf| <= 1.5 blocks) around "
                               "4 seeded spheres, 8^3 fp32 leaves, bitmasked root" % args.n,
                   "seed": args.seed, "active_blocks": w.nblocks, "active_voxels": voxels,
                   "program_per_step": "listgen, jacobi, copy", "parallelism": "single GPU"},
        "launches_per_step": {"optimized": st_opt["dispatches"] / K, "eager": st_eag["dispatches"] / K},
        "eager": {"value": voxels * K / t_eag, "ms_per_step": t_eag / K * 1e3},
        "speedup_vs_eager": t_eag / t_opt,
        "optimized_equals_eager": same,
        "optimizer_us_per_window": st_opt["optimizer_us"],
        "plan_cache_hits": st_opt["plan_cache_hits"],
        "kernels": {"jacobi_us": t_jac * 1e6, "copy_us": t_copy * 1e6,
                    "jacobi_GBs": achieved, "copy_GBs": copy_bytes / t_copy / 1e9,
                    "step_GBs_algorithmic": 20.0 * voxels / (t_opt / K) / 1e9},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_stencil<JACOBI> (12 B per active voxel: x, b read; xn written)"},
    }

    if not args.no_cpu_baseline and not args.profile:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_iters)
    print(json.dumps(out), flush=True)


def cpu_baseline(w, iters):
    """The oracle (single-threaded C) on a bounded sample of the same
    workload: `iters` Jacobi iterations of the full 512^3 band."""
    from oracle import OracleGrid
    g = OracleGrid(w.n, 3, "f32")
    g.load(w.blocks, {"b": w.channels["b"]}, {"x": 0, "xn": 1, "b": 2})
    t0 = time.perf_counter()
    for _ in range(iters):
        g.listgen()
        g.jacobi(0, 2, 1)
        g.copy(0, 1)
    dt = time.perf_counter() - t0
    try:
        model = subprocess.run(["bash", "-c", "lscpu | grep 'Model name' | head -1"], capture_output=True,
                               text=True).stdout.split(":", 1)[-1].strip()
    except Exception:
        model = "unknown"
    return {"value": w.active_voxels * iters / dt, "unit": "voxel-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d iterations (listgen, jacobi, copy) of the full band512 workload, seed 0, "
                      "single-threaded C oracle (-O2, no contraction), %.1f s" % (iters, dt),
            "host_cpu": model, "host_nproc": os.cpu_count()}


if __name__ == "__main__":
    main()
