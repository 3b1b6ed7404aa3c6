"""Benchmark of the MIUGKS hot path on one MI355X.

Workload (default): Mach-5 argon past a square cylinder, 160x160 stretched
cells (24 576 fluid), 100x100 trapezoid velocities on [-15, 15]^2, Kn 0.1,
5-level V-cycles (FAS prediction on the two finest), pseudo step 3^n dt_p
capped at 300 dt_p, FP32 distribution with FP64 moments / macroscopic
prediction / norms.  A step is one outer MIUGKS cycle (Steps 1-8: UGKS flux
and residuals, FAS prediction, micro residual, CS correction, update and
moments).  The input is synthetic (no dataset); every array lives in HBM
before timing starts.

Prints one JSON line:
  value      cell-velocity updates per second per MG cycle
             (fluid cells x velocities / seconds per cycle)
  roofline   dominant kernel: algorithmic bytes per launch / mean launch time
             (HIP events on the library's stream) against 8 TB/s; the flux
             and smoother kernels under roofline_kernels
  cpu_baseline  the FP64 CPU oracle timed on this host on a bounded sample
plus the other precision form's cycle time, and the wall time and cycle
count to an RMS residual of 1e-6 for the FP32-f and FP64 forms (and, where
the FP32-f form stalls at the resolution of its storage, FP32-f cycles
followed by FP64 cycles from their state).
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
    # profiles/square160x160_kernel_trace_and_hbm_traffic.md: the flux, the
    # ordered sweep over all its launches (bands on the 160- and 80-row
    # levels, the whole-tile wavefront sweep below), the band launches of the
    # 160-row level (those of the last sweep also add df to f)
    ("square160x160", "fp32f", "flux_div"): 7.6077e9,
    ("square160x160", "fp32f", "sweep"): 3.9865e8,
    ("square160x160", "fp32f", "sweep/l0"): 7.0812e8,
    ("square160x160", "fp64", "flux_div"): 1.7050e10,
    ("square160x160", "fp64", "sweep"): 4.6305e8,
    ("square160x160", "fp64", "sweep/l0"): 5.5761e8,
    # profiles/plate128x96_kernel_trace_and_hbm_traffic.md (bands on the
    # 96-row level only)
    ("plate128x96", "fp32f", "flux_div"): 5.1537e8,
    ("plate128x96", "fp32f", "sweep"): 5.6823e7,
    ("plate128x96", "fp32f", "sweep/l0"): 8.9933e7,
    ("plate128x96", "fp64", "flux_div"): 1.3118e9,
    ("plate128x96", "fp64", "sweep"): 1.1317e8,
    ("plate128x96", "fp64", "sweep/l0"): 1.7939e8,
    # profiles/cavity64_kn0.075_kernel_trace_and_hbm_traffic.md (FP64: bands
    # on the 64-row level; in FP32-f that level's whole-tile sweeps share
    # their kernels with the coarser levels, so no level-0 figure)
    ("cavity64_kn0.075", "fp32f", "flux_div"): 8.0200e7,
    ("cavity64_kn0.075", "fp32f", "sweep"): 1.2199e7,
    ("cavity64_kn0.075", "fp64", "flux_div"): 1.9380e8,
    ("cavity64_kn0.075", "fp64", "sweep"): 2.3247e7,
    ("cavity64_kn0.075", "fp64", "sweep/l0"): 4.5385e7,
}

# what each workload recipe is (the sizes are printed from the case itself)
RECIPES = {
    1: "lid-driven cavity, uniform cells, lid Mach 0.16",
    2: "lid-driven cavity, two-sided tanh cells (first cell 0.005), lid Mach 0.16",
    3: "zero-thickness flat plate in a 40x30 farfield box, cells clustered at the plate, Mach 0.1",
    4: "Mach-5 flow over a square cylinder (32x32 solid cells), farfield and outflow boundaries",
    5: "lid-driven cavity as config 2 with seeded bottom-wall temperatures",
}


def host_cpu():
    """(model string, logical CPUs) of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(case, cycles, nvel=None):
    """The oracle (numpy FP64) on a bounded sample of the same case: the same
    mesh, levels, boundaries and flow, with the velocity grid cut to nvel x
    nvel nodes on the same range when it is larger (the oracle's work per
    cycle is proportional to the number of velocities, so the rate per
    cell-velocity update carries over); setup untimed, then `cycles` full
    outer cycles timed on one thread."""
    from threadpoolctl import threadpool_limits

    from oracle.solver import Oracle
    sample = case.with_(precision="fp64")
    cut = nvel is not None and case.nu * case.nv > nvel * nvel
    if cut:
        sample = sample.with_(nu=nvel, nv=nvel)
    with threadpool_limits(limits=1):
        o = Oracle(sample)
        t0 = time.perf_counter()
        for _ in range(cycles):
            o.step1()
            o.advance()
        dt = (time.perf_counter() - t0) / cycles
    model, ncpu = host_cpu()
    what = (f"the same {case.nx}x{case.ny} mesh and {case.n_levels}-level cycle with {sample.nu}x{sample.nv} of "
            f"the {case.nu}x{case.nv} velocity nodes (same range)" if cut else
            f"the same {case.nx}x{case.ny}x{case.n_vel} case")
    return {"value": sample.n_fluid * sample.n_vel / dt, "unit": "cell*velocity updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{cycles} full outer cycle(s) of {what}, numpy FP64 oracle, one thread, "
                      f"{dt:.2f} s per cycle",
            "host_cpu": model, "host_logical_cpus": ncpu}


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
    # the same solve with the Krylov basis in FP32 (miugks_adjoint_ex)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st32, g32, iters32, rel32 = solver.adjoint(1, lid, faces, tol=tol, max_iter=5000, krylov_precision="fp32")
    torch.cuda.synchronize()
    sec32 = (time.perf_counter() - t0) / args.steps
    dev32 = float(np.max(np.abs(g32 - g)) / np.max(np.abs(g)))
    print(f"[bench] with an FP32 Krylov basis: {sec32:.3f} s each, {iters32} corrections, residual {rel32:.2e}, "
          f"gradient within {dev32:.1e} of the FP64 one", file=sys.stderr, flush=True)
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
        "fp32_krylov": {"ms_per_step": sec32 * 1e3, "corrections": iters32, "relative_residual": rel32,
                        "gradient_deviation": dev32},
    }
    print(json.dumps(line), flush=True)


def kernel_roofline(stats, kernel):
    """Roofline entry of one kernel (all its labels kernel or kernel/level):
    algorithmic bytes per launch over the mean HIP-event launch time."""
    n_l, ms, by = 0, 0.0, 0.0
    for k, (a, b, c) in stats.items():
        if k == kernel or k.startswith(kernel + "/"):
            n_l, ms, by = n_l + a, ms + b, by + c
    if n_l == 0 or ms <= 0:
        return None
    achieved = by / n_l / (ms / n_l * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "launches": n_l, "bytes_per_launch": by / n_l,
            "mean_launch_ms": ms / n_l}


def time_cycles(solver, steps, warmup):
    """Seconds per outer cycle over `steps` cycles after `warmup` (tol 0: every
    cycle runs)."""
    import torch
    solver.iterate(warmup, tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, n, res = solver.iterate(steps, tol=0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if n != steps:
        sys.exit(f"bench: the timed cycles stopped after {n} of {steps} (status {rc}: "
                 f"{'diverged' if rc == 4 else 'error'}); residuals {res}")
    return (t1 - t0) / steps


def to_tolerance(case, solver, prec, tol=1e-6, max_cycles=600, chunk=10):
    """Wall time and cycles from the initial state to every RMS residual below
    tol.  Runs in chunks of `chunk` cycles (one host check per chunk) and
    stops early when the residual stalls: no halving over 20 cycles once
    below 1e-3 (the FP32-f form meets the resolution of its storage there;
    its cycles advance the state at FP64's pace even so, so the FP64 cycles
    that follow are few).
    Returns the record and the solver left at the last state."""
    import numpy as np
    import torch
    solver.init_macro(case.init)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, hist, rc, res = 0, [], 5, None
    while done < max_cycles:
        rc, n, res = solver.iterate(chunk, tol=tol)
        done += n
        hist.append(float(np.max(res)))
        if rc != 5:
            break
        if len(hist) > 2 and hist[-1] < 1e-3 and hist[-1] > 0.5 * hist[-3]:
            rc = "stalled"
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rec = {"converged": rc == 0, "cycles": done, "wall_s": wall, "final_residual": [float(x) for x in res]}
    if rc == "stalled":
        rec["stalled_at"] = float(np.max(res))
    print(f"[bench] {prec}: {'residual 1e-6' if rc == 0 else 'stopped'} after {done} cycles, {wall:.3f} s, "
          f"max residual {np.max(res):.2e}", file=sys.stderr, flush=True)
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32f", choices=["fp32f", "fp64"])
    ap.add_argument("--config", type=int, default=4,
                    help="workload recipe (4 = the Mach-5 square cylinder, the largest one-GPU case)")
    ap.add_argument("--explicit", action="store_true",
                    help="time explicit time-accurate UGKS steps instead of MG cycles (the interface flux, the "
                         "collision update and the moments, once per step)")
    ap.add_argument("--adjoint", action="store_true",
                    help="time adjoint solves (wall-temperature gradients of the lid shear) on a converged FP64 "
                         "steady state of the adjoint cavity (config 5 unless --config is given)")
    ap.add_argument("--dtn-growth", type=float, default=None,
                    help="override the workload's pseudo-step growth a (dt_n = a^n dt_p; 0: off)")
    ap.add_argument("--cpu-cycles", type=int, default=1)
    ap.add_argument("--cpu-velocities", type=int, default=16,
                    help="velocity nodes per axis of the oracle's sample (the case's own grid when smaller)")
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

    import numpy as np
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
    sec = time_cycles(solver, args.steps, args.warmup)
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
    roofline = kernel_roofline(stats, dom)
    traffic = MEASURED_TRAFFIC.get((case.name, args.precision, dom))
    roofline["traffic"] = traffic
    roofline["traffic_over_algorithmic"] = (traffic / roofline["bytes_per_launch"]) if traffic else None
    print(f"[bench] dominant kernel {dom}: {roofline['mean_launch_ms'] * 1e3:.1f} us/launch, "
          f"{roofline['achieved']:.0f} GB/s", file=sys.stderr, flush=True)
    # the flux and the smoother, each against the HBM roofline (and the
    # smoother's finest level alone)
    others = {}
    for kname in ("flux_div", "sweep", "sweep/l0"):
        r = kernel_roofline(stats, kname) if "/" not in kname else (
            None if kname not in stats else kernel_roofline({kname: stats[kname]}, kname))
        if r is not None:
            t = MEASURED_TRAFFIC.get((case.name, args.precision, kname))
            r["traffic"] = t
            others[kname] = r
    cycle_bytes = sum(v[2] for v in stats.values()) / args.steps
    kernels = {k: {"launches": v[0], "ms_per_cycle": v[1] / args.steps}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}

    # the other precision form's cycle time on the same workload
    other_prec = "fp64" if args.precision != "fp64" else "fp32f"
    s_other = Solver(case, precision=other_prec)
    sec_other = time_cycles(s_other, args.steps, args.warmup)
    print(f"[bench] {other_prec}: {sec_other * 1e3:.3f} ms/cycle", file=sys.stderr, flush=True)

    extra = {}
    if not args.no_converge:
        solvers = {args.precision: solver, other_prec: s_other}
        s32, s64 = solvers["fp32f"], solvers["fp64"]
        extra["fp32f"] = to_tolerance(case, s32, "fp32f")
        # where the FP32-f form stalls at the resolution of FP32 storage: FP64
        # cycles from the state it reached (the distribution converted on the
        # device), the wall time counted from the initial state
        if not extra["fp32f"]["converged"]:
            t0 = time.perf_counter()
            f64 = torch.empty(s64.fshape, dtype=torch.float64, device="cuda")
            s32.get_f(out=f64)
            s64.set_f(f64)
            del f64
            rc, n64, res = s64.iterate(600, tol=1e-6)
            torch.cuda.synchronize()
            wall = extra["fp32f"]["wall_s"] + time.perf_counter() - t0
            extra["fp32f_then_fp64"] = {"converged": rc == 0, "cycles_fp32f": extra["fp32f"]["cycles"],
                                        "cycles_fp64": n64, "wall_s": wall,
                                        "final_residual": [float(x) for x in res]}
            print(f"[bench] fp32f then fp64: {extra['fp32f']['cycles']} + {n64} cycles, {wall:.3f} s",
                  file=sys.stderr, flush=True)
        extra["fp64"] = to_tolerance(case, s64, "fp64")
    s_other.close()

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
        "roofline_kernels": others,
        f"{other_prec}_ms_per_step": sec_other * 1e3,
        f"{other_prec}_value": pts / sec_other,
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
    solver.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_cycles, args.cpu_velocities)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
