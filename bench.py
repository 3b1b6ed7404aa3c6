"""Benchmark of the MIUGKS hot path on one MI355X.

Workload: lid-driven cavity, 64x64 tanh-clustered cells (first cell 0.005),
28x28 Gauss-Hermite velocities, Kn 0.075, lid Mach 0.16, 4-level V-cycles,
FP32 distribution with FP64 moments / macroscopic prediction / norms.  A step
is one outer MIUGKS cycle (Steps 1-8: UGKS flux and residuals, FAS
prediction, micro residual, CS correction, update and moments).  The input
is synthetic (no dataset); every array lives in HBM before timing starts.

Prints one JSON line:
  value      cell-velocity updates per second per MG cycle
             (fluid cells x velocities / seconds per cycle)
  roofline   dominant kernel: algorithmic bytes per launch / mean launch time
             (HIP events on the library's stream) against 8 TB/s
  cpu_baseline  the FP64 CPU oracle timed on this host on a bounded sample
plus the wall time and cycle count to an RMS residual of 1e-6 for the
FP32-f form and the FP64 form.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell·velocity updates/s per MG cycle; wall time to residual 1e-6; HBM GB/s"
HBM_PEAK_GBS = 8000.0
# HBM-side traffic of the dominant kernel, bytes per launch (mean over its
# launches in one profiled run): rocprofv3 FETCH_SIZE and WRITE_SIZE, each
# scaled by the ratio of known bytes to counted bytes of a plain copy in the
# same run (--copy-calibration).  Keyed by (workload, precision, kernel); an
# entry is dropped whenever that kernel changes.
MEASURED_TRAFFIC = {
    # profiles/sweep_wave_cavity64_fp32f_hbm_traffic.md: 77 dispatches of the
    # sweep (every level, G-only and G+H forms), scaled FETCH_SIZE + WRITE_SIZE
    ("cavity64_kn0.075", "fp32f", "sweep"): 12.19e6,
}

# what each workload recipe is (the sizes are printed from the case itself)
RECIPES = {
    1: "lid-driven cavity, uniform cells, lid Mach 0.16",
    2: "lid-driven cavity, two-sided tanh cells (first cell 0.005), lid Mach 0.16",
    3: "zero-thickness flat plate in a 40x30 farfield box, cells clustered at the plate, Mach 0.1",
    4: "Mach-5 flow over a square cylinder (32x32 solid cells), farfield and outflow boundaries",
    5: "lid-driven cavity as config 2 with seeded bottom-wall temperatures",
}


def cpu_baseline(case, cycles):
    """The oracle (numpy FP64) on the same case: setup untimed, then `cycles`
    full outer cycles timed, single thread."""
    from threadpoolctl import threadpool_limits

    from oracle.solver import Oracle
    with threadpool_limits(limits=1):
        o = Oracle(case.with_(precision="fp64"))
        t0 = time.perf_counter()
        for _ in range(cycles):
            o.step1()
            o.advance()
        dt = (time.perf_counter() - t0) / cycles
    return {"value": case.n_fluid * case.n_vel / dt, "unit": "cell*velocity updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{cycles} full outer cycle(s) of the same {case.nx}x{case.ny}x{case.n_vel} cavity, "
                      f"numpy FP64 oracle, one thread, {dt:.2f} s per cycle"}


def explicit_bench(args, case, solver, pts):
    """Explicit time-accurate UGKS steps: K timed after W warm-up steps, then
    the per-kernel pass; the roofline is that of the interface-flux kernel."""
    import torch
    solver.explicit(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dt, res = solver.explicit(args.steps)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    print(f"[bench] {args.steps} explicit steps (dt {dt:.3e}): {sec * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    solver.set_timing(True)
    solver.explicit(args.steps)
    stats = solver.timing()
    solver.set_timing(False)
    n_l, ms, by = stats["flux_div"]
    achieved = by / n_l / (ms / n_l * 1e-3) / 1e9
    line = {
        "metric": "cell·velocity updates/s per explicit UGKS step",
        "value": pts / sec, "unit": "cell*velocity updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == "fp32f" else "f64", "data": "synthetic",
        "config": {"workload": f"{case.name}: {RECIPES.get(args.config, 'synthetic case')}, explicit steps of "
                               f"{dt:.3e}", "cells": case.n_cells, "velocities": case.n_vel,
                   "precision": args.precision},
        "roofline": {"bound": "hbm", "kernel": "flux_div", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": by / n_l, "mean_launch_ms": ms / n_l},
        "kernel_ms_per_step": {k: v[1] / args.steps for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])},
        "residual": [float(x) for x in res],
    }
    print(json.dumps(line), flush=True)


def adjoint_bench(args, case, solver):
    """Wall-temperature gradients of the lid shear on a converged FP64 steady
    state: W untimed and K timed adjoint solves (each with its two
    mass-perturbed steady states), then one with per-kernel timing."""
    import numpy as np
    import torch
    rc, n, res = solver.iterate(1000, tol=1e-12)
    print(f"[bench] steady state: {n} cycles, residual {res.max():.2e} (status {rc})", file=sys.stderr, flush=True)
    cell, side = solver.wall_list()
    lid = [int(j) for j in np.nonzero(side == 3)[0]]
    nfx = (case.nx + 1) * case.ny
    faces = [nfx + i for i in range(case.nx)]
    tol = 1e-8
    for _ in range(args.warmup):
        solver.adjoint(1, lid, faces, tol=tol, max_iter=5000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, g, iters, rel = solver.adjoint(1, lid, faces, tol=tol, max_iter=5000)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    print(f"[bench] {args.steps} adjoint solves: {sec:.3f} s each, {iters} corrections, residual {rel:.2e}",
          file=sys.stderr, flush=True)
    solver.set_timing(True)
    solver.adjoint(1, lid, faces, tol=tol, max_iter=5000)
    stats = solver.timing()
    solver.set_timing(False)
    adj = {k: v for k, v in stats.items() if k.startswith("adj_")}
    dom = max(adj, key=lambda k: adj[k][1])
    n_l, ms, by = adj[dom]
    achieved = by / n_l / (ms / n_l * 1e-3) / 1e9
    pts = case.n_fluid * case.n_vel
    line = {
        "metric": "wall-temperature gradients/s (adjoint solves of the steady lid shear)",
        "value": 1.0 / sec, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{case.name}: {RECIPES.get(args.config, 'synthetic case')}; lid shear, "
                               f"{len(faces)} bottom-face temperatures, adjoint to a 1e-8 residual drop",
                   "cells": case.n_cells, "velocities": case.n_vel, "precision": "fp64"},
        "corrections": iters, "relative_residual": rel,
        "ms_per_correction": sec * 1e3 / max(iters, 1),
        "transposed_products_per_s": pts * max(iters, 1) / sec,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": by / n_l,
                     "mean_launch_ms": ms / n_l},
        "kernel_ms_per_solve": {k: v[1] for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])[:12]},
        "gradient_max": float(np.max(np.abs(g))),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32f", choices=["fp32f", "fp64"])
    ap.add_argument("--config", type=int, default=2, help="workload recipe (2 = the headline cavity)")
    ap.add_argument("--explicit", action="store_true",
                    help="time explicit time-accurate UGKS steps instead of MG cycles (the interface flux, the "
                         "collision update and the moments, once per step)")
    ap.add_argument("--adjoint", action="store_true",
                    help="time adjoint solves (wall-temperature gradients of the lid shear) on a converged FP64 "
                         "steady state of the adjoint cavity (config 5 unless --config is given)")
    ap.add_argument("--dtn-growth", type=float, default=None,
                    help="override the workload's pseudo-step growth a (dt_n = a^n dt_p; 0: off)")
    ap.add_argument("--cpu-cycles", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true", help="skip the time-to-1e-6 runs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="end with one plain device-to-device copy of MIB MiB, the reference launch "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters of a profiled run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design notes describe how it would shard over velocities).", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as wl
    from paper_1704_03151_amd import Solver

    torch.cuda.set_device(0)
    if args.adjoint:
        if "--config" not in sys.argv:
            args.config = 5
        args.precision = "fp64"
    case = wl.CONFIGS[args.config]()
    if args.dtn_growth is not None:
        case = case.with_(dtn_growth=args.dtn_growth)
    solver = Solver(case, precision=args.precision)
    pts = case.n_fluid * case.n_vel
    print(f"[bench] {case.name}: {case.nx}x{case.ny} cells ({case.n_fluid} fluid) x {case.n_vel} velocities, "
          f"{case.n_levels} levels, {args.precision}", file=sys.stderr, flush=True)

    if args.explicit:
        return explicit_bench(args, case, solver, pts)
    if args.adjoint:
        return adjoint_bench(args, case, solver)
    # warm-up, then exactly K timed cycles
    solver.iterate(args.warmup, tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, n, res = solver.iterate(args.steps, tol=0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if n != args.steps:
        sys.exit(f"bench: the timed cycles stopped after {n} of {args.steps} (status {rc}: "
                 f"{'diverged' if rc == 4 else 'error'}); residuals {res}")
    sec = (t1 - t0) / args.steps
    value = pts / sec
    print(f"[bench] {args.steps} cycles: {sec * 1e3:.3f} ms/cycle", file=sys.stderr, flush=True)

    # per-kernel timing over K more cycles (HIP events on the library stream)
    solver.set_timing(True)
    solver.iterate(args.steps, tol=0.0)
    stats = solver.timing()
    solver.set_timing(False)
    total_ms = sum(v[1] for v in stats.values())
    # labels "kernel/level" are one kernel launched on several levels: the
    # roofline takes the kernel with the largest total time over all levels
    per_kernel = {}
    for k, (n_l, ms_l, by_l) in stats.items():
        a = per_kernel.setdefault(k.split("/")[0], [0, 0.0, 0.0])
        a[0] += n_l
        a[1] += ms_l
        a[2] += by_l
    dom = max(per_kernel, key=lambda k: per_kernel[k][1])
    launches, ms, by = per_kernel[dom]
    achieved = by / launches / (ms / launches * 1e-3) / 1e9
    cycle_bytes = sum(v[2] for v in stats.values()) / args.steps
    kernels = {k: {"launches": v[0], "ms_per_cycle": v[1] / args.steps,
                   "gbs": (v[2] / (v[1] * 1e-3) / 1e9 if v[1] > 0 else None)}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}
    traffic = MEASURED_TRAFFIC.get((case.name, args.precision, dom))
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "bytes_per_launch": by / launches, "mean_launch_ms": ms / launches,
                "traffic_over_algorithmic": (traffic / (by / launches)) if traffic else None}
    print(f"[bench] dominant kernel {dom}: {ms / launches * 1e3:.1f} us/launch, {achieved:.0f} GB/s",
          file=sys.stderr, flush=True)

    extra = {}
    if not args.no_converge:
        for prec in (args.precision, "fp64" if args.precision != "fp64" else None):
            if prec is None:
                continue
            s = solver if prec == args.precision else Solver(case, precision=prec)
            s.init_macro(case.init)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, cyc, res = s.iterate(1000, tol=1e-6)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            extra[prec] = {"converged": rc == 0, "cycles": cyc, "wall_s": wall,
                           "final_residual": [float(x) for x in res]}
            print(f"[bench] {prec}: residual 1e-6 after {cyc} cycles, {wall:.3f} s", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "cell*velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32f" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{case.name}: {RECIPES.get(args.config, 'synthetic case')}, "
                               f"{case.nx}x{case.ny} cells x {case.nu}x{case.nv} {case.quad} velocities, "
                               f"Kn {case.Kn}, {case.n_levels}-level V-cycles",
                   "cells": case.n_cells, "fluid_cells": case.n_fluid, "velocities": case.n_vel,
                   "levels": case.n_levels, "precision": args.precision},
        "roofline": roofline,
        "cycle_algorithmic_gbs": cycle_bytes / (total_ms / args.steps * 1e-3) / 1e9,
        "kernel_ms_per_cycle": {k: v["ms_per_cycle"] for k, v in kernels.items()},
        "kernel_us_per_launch": {k: 1e3 * v[1] / v[0] for k, v in
                                 sorted(stats.items(), key=lambda kv: -kv[1][1])},
        "to_residual_1e-6": extra,
    }
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = n * 4
        del src, dst
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_cycles)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
