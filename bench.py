#!/usr/bin/env python3
"""Benchmark: DG S_N sweep throughput inside the SMM outer iteration on one
MI355X.

Workload: the two-material channel problem on [0,10]^2, 128 x 128 quads,
p = 2, S12 (84 directions), FP32 sweep and moments, FP64 CG and residual,
delta sweeps (synthetic seeded inputs; see workloads.config_channel).

A step is one full outer iteration X -> G(X): scattering source, sweep,
angular moments on the matrix cores, SMM closures, IP right-hand side, FP64
PCG moment solve, residual.  value = elem*angle*DOF per second of whole
steps.  Extra fields report the sweep kernel alone (HIP events on the
library's stream), its roofline, and the time to a 1e-8 outer residual.

The CPU baseline is the FP64 oracle's sweep on a bounded sample of the same
workload (a few directions), single thread.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def cpu_baseline(wl, n_dirs: int = 6):
    """Time the oracle sweep for n_dirs directions of the workload (one
    thread).  Returns units/s and a description of the sample."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import numpy as np
    from oracle import smm as osmm, transport

    pr = osmm.make_problem(wl)
    S = np.ones((pr.ne, pr.n))
    dirs = np.linspace(0, len(pr.w) - 1, n_dirs).astype(int)
    ctx = threadpool_limits(1) if threadpool_limits else None
    t0 = time.perf_counter()
    transport.sweep(pr.mesh, pr.omega[dirs], pr.sigma_t, S, None)
    dt = time.perf_counter() - t0
    if ctx is not None:
        ctx.unregister() if hasattr(ctx, "unregister") else None
    units = pr.ne * len(dirs) * pr.n
    return units / dt, f"oracle FP64 sweep of {len(dirs)} of {len(pr.w)} directions on the full " \
                       f"{wl.nx}x{wl.ny} p={wl.p} mesh ({units} units, {dt:.1f} s)"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweep-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1e-8 solve")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2304_07386_amd as L
    from workloads import config_channel

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = L.smm_ctx_create(0, stream)
    wl = config_channel()
    prob = L.problem_from_workload(ctx, wl)
    units = wl.units_per_sweep
    print(f"[bench] workload channel 128x128 p=2 S12: {units} units per sweep", file=sys.stderr, flush=True)

    opts = L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=0.0,
                              inner_tol=1e-10, max_inner=20000)
    # warmup (also builds the device tables)
    opts.max_outer = max(args.warmup, 1)
    L.smm_solve(prob, opts, raise_on_noconv=False)
    torch.cuda.synchronize()
    # timed steps
    opts.max_outer = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, info = L.smm_solve(prob, opts, raise_on_noconv=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = units * args.steps / wall
    print(f"[bench] {args.steps} outer iterations: {ms_per_step:.3f} ms/step, "
          f"CG iterations total {info['cg_iterations_total']}", file=sys.stderr, flush=True)

    # sweep kernel alone: HIP events around back-to-back sweeps on the library stream
    sweep_ms = L.smm_time_sweep(prob, L.SMM_FP32_SWEEP, args.sweep_reps)
    sweep_rate = units / (sweep_ms * 1e-3)
    nd, n = prob.n_dir, prob.n_node
    bytes_per_unit = 4.0 + 4.0 / nd      # psi written once (FP32) + S read once per element
    achieved = units * bytes_per_unit / (sweep_ms * 1e-3) / 1e9
    print(f"[bench] sweep {sweep_ms * 1e3:.1f} us -> {sweep_rate:.3e} units/s", file=sys.stderr, flush=True)

    solve = None
    if not args.no_solve:
        o2 = L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-8,
                                inner_tol=1e-10, max_inner=20000, max_outer=200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc2, inf2 = L.smm_solve(prob, o2, raise_on_noconv=False)
        torch.cuda.synchronize()
        solve = {"ms": 1e3 * (time.perf_counter() - t0), "outer_iterations": inf2["iterations"],
                 "cg_iterations_total": inf2["cg_iterations_total"], "residual": inf2["residual"],
                 "converged": rc2 == L.SMM_OK, "start": "zero"}
        print(f"[bench] time to 1e-8: {solve}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        rate, sample = cpu_baseline(wl)
        cpu = {"value": rate, "unit": "elem*angle*DOF/s", "cores": 1, "kind": "oracle", "sample": sample,
               "cpu": platform.processor() or platform.machine()}

    out = {
        "metric": "sweep elem*angle*DOF/s (whole SMM outer iteration) + time-to-1e-8 SMM solve",
        "value": value,
        "unit": "elem*angle*DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_detail": "sweep and moments f32; CG, closures, residual f64",
        "data": "synthetic",
        "config": {"workload": "channel two-material [0,10]^2 128x128 p=2 S12, seed 0",
                   "units_per_sweep": units, "parallelism": "single GPU"},
        "sweep_only": {"ms": sweep_ms, "units_per_s": sweep_rate},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sweep_cart_kernel<float,3>",
                     "bytes_per_unit": bytes_per_unit},
        "time_to_1e-8": solve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
