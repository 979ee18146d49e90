#!/usr/bin/env python3
"""Benchmark: the batched SMM hot path on one MI355X.

Workload (value): 256 independent problems solved as one batch, seeds 0-255
of the seeded generator (uniform Cartesian [0,1]^2 meshes of 16^2 to 128^2
elements, orders p = 1-4, S4-S12, homogeneous sigma_t log-uniform in
[0.1, 100], scattering ratio uniform in [0.5, 0.999], unit isotropic
source, vacuum), FP32 sweeps and moments with delta sweeps, FP64 closures,
PCG and residual.  Inputs are synthetic and resident on the GPU before the
timed region.

A step is one full outer iteration X -> G(X) of every problem: scattering
source, sweep (persistent per-order launches), angular moments on the matrix
cores, SMM closures, right-hand side, FP64 block-Jacobi PCG, residual.
value = elem*angle*DOF units swept per second of whole steps.

Also reported:
  * the time of each phase inside the steps and the roofline of the kernel of
    the dominant phase (and of the sweep), from HIP events on the stream each
    kernel runs on;
  * time to a 1e-8 outer residual on held-out warm-start layouts (64 x 64,
    p = 2, S8 blob layouts): the plain method (problems solved one after the
    other from the zero start) against the batched solve with the learned
    start, on identical inputs;
  * the IP and the continuous (CG) moment systems on the multi-material
    channel problem: time to a 1e-8 outer residual, and the roofline of the
    CG product kernel;
  * the parallel block Jacobi sweep on the same problem: sweep time and
    outer iterations per tile size;
  * the sweep on curved meshes (per-element assembly and elimination) at
    p = 2, 3, 4;
  * the CPU oracle's sweep on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64, matrix cores and vector units alike
METRIC = "sweep elem*angle*DOF/s + time-to-1e-8 SMM solve, plain vs batched+warm"
# The paper's own figures (CPU runs), as context only: derived sweep rate of
# the weak-scaling study on one processor (crooked pipe, p = 2, S12: scalar
# DOF x 84 directions / average sweep time per outer iteration, Table
# tab:weak_time) and its outer iterations with the parallel block Jacobi sweep
# (Table tab:weak_itr).
PAPER_CONTEXT = {
    "sweep_units_per_s": 3.57e5,
    "sweep_units_per_s_1024_procs": 2.31e8,
    "hardware": "Intel Xeon E5-2695 nodes (LLNL rztopaz), one processor / 1024 processors; precision not stated",
    "workload": "crooked pipe, p = 2, S12, parallel block Jacobi sweep, 4032 DOF per processor",
    "block_jacobi_outer_iterations_1_to_1024_procs": [32, 55, 80, 135, 277, 592],
    "source": "Tables tab:weak_time and tab:weak_itr (Sec. 6.5)",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(workloads, max_dirs: int = 12, budget_s: float = 12.0):
    """The oracle's sweep (FP64, one thread) over up to max_dirs directions of
    the given problems in order, until about budget_s seconds of sweeping.
    Returns (units/s, description)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import smm as osmm, transport

    units, dt, parts = 0, 0.0, []
    with threadpool_limits(1):
        for wl in workloads:
            pr = osmm.make_problem(wl)
            nd = min(max_dirs, len(pr.w))
            S = np.ones((pr.ne, pr.n))
            t0 = time.perf_counter()
            transport.sweep(pr.mesh, pr.omega[:nd], pr.sigma_t, S, None)
            dt += time.perf_counter() - t0
            units += pr.ne * nd * pr.n
            parts.append(f"{wl.nx}^2 p={wl.p} S{wl.sn} {nd} dirs")
            if dt >= budget_s:
                break
    return units / dt, (f"oracle FP64 sweep, first {len(parts)} problems of the batch ({'; '.join(parts)}): "
                        f"{units} units in {dt:.1f} s")


def cpu_model() -> str:
    """The host CPU's model name (Linux), else the machine type."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def traffic_for(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    ent = tab.get(kernel)
    if not ent:
        return None
    src = os.path.join(ROOT, "paper_2304_07386_amd", "csrc", ent["source"])
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha != ent["sha256"]:
        return None
    return ent["bytes_per_launch"]


def issued_for(kernel: str, ms: float):
    """Issued floating-point rate from the committed counter table (taken on
    the current kernel source), or None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if traffic_for(kernel) is None or not os.path.exists(path):
        return None
    with open(path) as f:
        ent = json.load(f).get(kernel, {})
    if "issued_flops_per_launch" not in ent:
        return None
    return {"issued_tflops": ent["issued_flops_per_launch"] / (ms * 1e-3) / 1e12, "kind": ent["kind"]}


def roofline(kernel: str, what: str, bytes_per_launch: float, ms: float):
    """`kernel` is the name prefix of the launches timed together as one
    operation (`what`): one sweep, or one q = A p, runs one launch per order
    present in the batch."""
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    tr = traffic_for(kernel)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": tr, "kernel": kernel, "operation": what,
            "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": ms,
            "counted": issued_for(kernel, ms)}


def roofline_flops(kernel: str, what: str, flops_per_launch: float, bytes_per_launch: float, ms: float):
    """FP64 compute roofline (the binding one for q = A p, whose ridge point
    9.8 flop/B is below its 11.5 flop/B), with the HBM figures beside it."""
    achieved = flops_per_launch / (ms * 1e-3) / 1e12
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic_for(kernel), "kernel": kernel,
            "operation": what, "algorithmic_flops_per_launch": flops_per_launch,
            "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": ms,
            "hbm_achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS, "counted": issued_for(kernel, ms)}


def time_to_solution(L, ctx, n: int, log):
    """Plain (one problem at a time, zero start) vs batched + learned start on
    the held-out layouts 20000..20000+n-1; wall time to a 1e-8 residual."""
    import numpy as np
    import torch
    from paper_2304_07386_amd import warmstart as W
    from workloads import config_blobs

    if not os.path.exists(W.DEFAULT_WEIGHTS):
        log("no trained warm-start weights: skipping the time-to-solution comparison")
        return None
    wls = [config_blobs(20000 + k) for k in range(n)]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    opts = W.solve_opts(1e-8, start=L.SMM_START_ZERO)
    # plain: the single-problem solve, zero start, one problem after the other
    warm = W.solve_opts(1e-8, start=L.SMM_START_ZERO)
    warm.max_outer = 1
    for p in probs:                                              # one-time device set-up outside the timing
        L.smm_solve(p, warm, raise_on_noconv=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_its = []
    for p in probs:
        rc, info = L.smm_solve(p, opts, raise_on_noconv=False)
        plain_its.append(info["iterations"])
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log(f"plain: {n} problems in {t_plain:.2f} s, outer its mean {np.mean(plain_its):.2f}")
    batch = L.smm_batch_create(ctx, probs)
    net, meta = W.load(ctx, max_batch=32)
    L.smm_batch_set_warmstart(batch, net)
    res = {"n_problems": n, "workload": "blobs 64x64 p=2 S8, held-out seeds 20000..%d" % (20000 + n - 1),
           "plain_s": t_plain, "plain_outer_mean": float(np.mean(plain_its))}
    L.smm_batch_solve(batch, W.solve_opts(1e-8, start=L.SMM_START_ZERO), raise_on_noconv=False)  # autotune
    for name, start in (("batched_zero", L.SMM_START_ZERO), ("batched_diffusion", L.SMM_START_DIFFUSION),
                        ("batched_warm", L.SMM_START_LEARNED)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, infos = L.smm_batch_solve(batch, W.solve_opts(1e-8, start=start), raise_on_noconv=False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res[name + "_s"] = t
        res[name + "_outer_mean"] = float(np.mean([i["iterations"] for i in infos]))
        res[name + "_converged"] = rc == L.SMM_OK
        log(f"{name}: {t:.2f} s, outer its mean {res[name + '_outer_mean']:.2f}")
    res["learned_start_kept"] = int(L.smm_batch_warmstart_used(batch).sum())
    res["speedup_batched_warm_vs_plain"] = t_plain / res["batched_warm_s"]
    L.smm_batch_set_warmstart(batch, None)
    L.smm_batch_destroy(batch)
    L.smm_cnn_destroy(net)
    return res


def moment_discretisations(L, ctx, log):
    """IP versus CG moment system (Sec. 5.1) on the multi-material channel
    problem (128 x 128, p = 2, S12, FP32 sweep): wall time to a 1e-8 outer
    residual from the zero start, and the roofline of the CG product kernel
    (FP64 CSR, HBM-bound: 12 B per stored entry, the row pointers, x read
    once and y written once)."""
    import torch
    from workloads import config_channel

    wl = config_channel(n=128, p=2, sn=12)
    common = dict(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-8, inner_tol=1e-10, inner_adapt=1e-2,
                  max_inner=20000, max_outer=60, use_graph=1)
    variants = (("ip_two_level", dict(precond=1), "IP, typed path, two-level PCG"),
                ("ip_block_jacobi", dict(moment_path=1), "IP, per-element path, block-Jacobi PCG"),
                ("cg_jacobi", dict(discretization=L.SMM_DISC_CG), "CG, per-element path, Jacobi PCG"))
    res = {"workload": "channel 128x128 p=2 S12 (two materials), FP32 sweep, zero start, outer 1e-8"}
    for name, kw, what in variants:
        p = L.problem_from_workload(ctx, wl)
        L.smm_solve(p, L.smm_default_opts(**{**common, **kw, "max_outer": 1}), raise_on_noconv=False)  # set-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = L.smm_solve(p, L.smm_default_opts(**common, **kw), raise_on_noconv=False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res[name] = {"what": what, "s": t, "converged": rc == L.SMM_OK, "outer": info["iterations"],
                     "inner_total": info["cg_iterations_total"]}
        log(f"{what}: {t * 1e3:.1f} ms, {info['iterations']} outer, {info['cg_iterations_total']} inner")
        if name == "cg_jacobi":
            rowptr, col, _, _ = L.smm_debug_cg_system(p)
            nc, nnz = len(rowptr) - 1, len(col)
            res["cg_unknowns"], res["ip_unknowns"] = nc, wl.n_elem * (wl.p + 1) ** 2
            ms = L.smm_time_cg_spmv(p, 200)
            by = 12.0 * nnz + 4.0 * (nc + 1) + 16.0 * nc
            res["roofline_cg_spmv"] = roofline("cgs_spmv_kernel", "y = A_c x, continuous moment system "
                                               f"({nc} rows, {nnz} entries)", by, ms)
            log(f"CG product: {ms * 1e3:.2f} us, {res['roofline_cg_spmv']['achieved']:.0f} GB/s")
        L.smm_problem_destroy(p)
    return res


def block_jacobi_sweeps(L, ctx, log):
    """Parallel block Jacobi sweep (Sec. 6.5) on the channel problem (128 x
    128, p = 2, S12): time of one FP32 sweep of the per-element kernel (one
    workgroup per direction and tile, one lane per element) for several tile sizes, outer
    iterations and wall time to a 1e-8 outer residual (CG moment system,
    FP32 delta sweeps), beside the tabulated Cartesian sweep, which has no
    tiled form.  The per-element kernel assembles and eliminates every
    element and direction: 165 flops per elem*angle*DOF at p = 2, on the FP32
    vector units."""
    import torch
    from workloads import config_channel

    wl = config_channel(n=128, p=2, sn=12)
    common = dict(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-8, inner_tol=1e-10, inner_adapt=1e-2,
                  max_inner=20000, max_outer=400, use_graph=1, discretization=L.SMM_DISC_CG)
    units = float(wl.n_elem * (wl.p + 1) ** 2 * 84)
    res = {"workload": "channel 128x128 p=2 S12, FP32 delta sweeps, CG moment system, outer 1e-8",
           "units_per_sweep": units, "runs": []}
    for tiles in ((0, 0), (128, 128), (32, 32), (16, 16), (8, 8)):
        p = L.problem_from_workload(ctx, wl)
        if tiles != (0, 0):
            L.smm_set_sweep_tiles(p, *tiles)
        ms = L.smm_time_sweep(p, L.SMM_FP32_SWEEP, 5)
        L.smm_solve(p, L.smm_default_opts(**{**common, "max_outer": 1}), raise_on_noconv=False)  # set-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = L.smm_solve(p, L.smm_default_opts(**common), raise_on_noconv=False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        kind = "tabulated Cartesian sweep (full)" if tiles == (0, 0) else \
            f"per-element sweep, tiles {tiles[0]}x{tiles[1]}"
        run = {"kernel": kind, "tiles": list(tiles), "sweep_ms": ms, "units_per_s": units / (ms * 1e-3),
               "solve_s": t, "converged": rc == L.SMM_OK, "outer": info["iterations"]}
        if tiles != (0, 0):
            tf = 165.0 * units / (ms * 1e-3) / 1e12
            run["roofline"] = {"bound": "alu", "achieved": tf, "peak": 157.3, "unit": "TFLOP/s", "frac": tf / 157.3,
                               "traffic": None, "kernel": "sweep_lane_general_kernel"}
        res["runs"].append(run)
        log(f"{kind}: sweep {ms:.3f} ms, solve {t * 1e3:.1f} ms, {info['iterations']} outer")
        L.smm_problem_destroy(p)
    return res


def curved_sweeps(L, ctx, log):
    """The sweep on curved meshes (the manufactured problem: 32 x 32 elements
    with an order-p map, S8), where every element and direction is assembled
    and eliminated by the per-element kernel (one lane per element at p = 2,
    one wave per element at p = 3, 4): time per sweep, units/s, and
    the rate against the FP32 vector peak at the assembly and elimination
    work per DOF (165 / 344 / 664 flops for p = 2 / 3 / 4)."""
    from workloads import config_curved_mms

    flops = {2: 165.0, 3: 344.0, 4: 664.0}
    res = {"workload": "curved manufactured problem, 32x32 elements, order-p map, S8 (40 directions)", "runs": []}
    for p in (2, 3, 4):
        wl = config_curved_mms(32, p, 8)
        prob = L.problem_from_workload(ctx, wl)
        units = float(wl.n_elem * (p + 1) ** 2 * 40)
        run = {"p": p, "units_per_sweep": units}
        for name, prec in (("fp32", L.SMM_FP32_SWEEP), ("fp64", L.SMM_FP64)):
            ms = L.smm_time_sweep(prob, prec, 5)
            run[name + "_ms"] = ms
            run[name + "_units_per_s"] = units / (ms * 1e-3)
        tf = flops[p] * units / (run["fp32_ms"] * 1e-3) / 1e12
        run["roofline_fp32"] = {"bound": "alu", "achieved": tf, "peak": 157.3, "unit": "TFLOP/s", "frac": tf / 157.3,
                                "traffic": None,
                                "kernel": "sweep_lane_general_kernel" if p <= 2 else "sweep_general_kernel"}
        log(f"curved 32^2 p={p} S8: FP32 sweep {run['fp32_ms']:.3f} ms, FP64 {run['fp64_ms']:.3f} ms")
        res["runs"].append(run)
        L.smm_problem_destroy(prob)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--problems", type=int, default=256)
    ap.add_argument("--tts-problems", type=int, default=24, help="held-out problems for the time-to-solution run")
    ap.add_argument("--precond", type=int, default=1, help="0 block-Jacobi, 1 two-level PCG")
    ap.add_argument("--anderson", type=int, default=2, help="Anderson mixing depth of the outer iteration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1e-8 comparisons")
    ap.add_argument("--disc-only", action="store_true",
                    help="run only the IP versus CG moment-system comparison and print its JSON")
    ap.add_argument("--tiles-only", action="store_true",
                    help="run only the block Jacobi sweep comparison and print its JSON")
    ap.add_argument("--curved-only", action="store_true",
                    help="run only the curved-mesh sweep timings and print their JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the problems of a batch are "
              "independent and would be split across GPUs by the caller)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2304_07386_amd as L
    from workloads import config_batched_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = L.smm_ctx_create(0, torch.cuda.current_stream())
    if args.disc_only:
        print(json.dumps(moment_discretisations(L, ctx, log)))
        return
    if args.tiles_only:
        print(json.dumps(block_jacobi_sweeps(L, ctx, log)))
        return
    if args.curved_only:
        print(json.dumps(curved_sweeps(L, ctx, log)))
        return
    t0 = time.time()
    wls = [config_batched_problem(s) for s in range(args.problems)]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    units = L.smm_batch_units(batch)
    dofs = float(sum(p.n_elem * p.n_node for p in probs))
    log(f"batch of {args.problems} problems: {units:.4g} units per sweep, {dofs:.4g} DOF, "
        f"set-up {time.time() - t0:.1f} s")

    opts = L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=0.0,
                              inner_tol=1e-10, max_inner=20000, max_outer=max(args.warmup, 1),
                              precond=args.precond, use_graph=1, anderson=args.anderson)
    L.smm_batch_solve(batch, opts, raise_on_noconv=False)       # warm-up (also autotunes the sweep grids)
    torch.cuda.synchronize()
    opts.max_outer = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, infos = L.smm_batch_solve(batch, opts, raise_on_noconv=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert all(i["iterations"] == args.steps for i in infos)
    ms_per_step = 1e3 * wall / args.steps
    value = units * args.steps / wall
    phases, cg_its = L.smm_batch_phase_times(batch)
    names = ["source+sweep", "moments+closures+rhs", "pcg", "residual"]
    phase = {n: ms / args.steps for n, ms in zip(names, phases)}
    log(f"{args.steps} steps: {ms_per_step:.1f} ms/step; per step " +
        ", ".join(f"{n} {v:.2f} ms" for n, v in phase.items()) + f"; batched PCG iterations {cg_its}")

    sweep_ms = L.smm_batch_time_kernel(batch, L.SMM_KERNEL_SWEEP_FP32, 5)
    # sweep: psi written once in FP32 (4 B/unit) + the FP32 source read once per
    # element and direction set (4/N_dir B/unit, N_dir per problem)
    sweep_bytes = float(sum(p.n_elem * p.n_node * (4.0 * p.n_dir + 4.0) for p in probs))
    rl_sweep = roofline("b_sweep_kernel", "one batched sweep (the per-order launches b_sweep_kernel<T, NB, ...>)",
                        sweep_bytes, sweep_ms)
    # the same sweep against the unit-rate roofline of the method: 8 B per
    # elem*angle*DOF in FP32 (psi written by the sweep and read back by the
    # moment contraction) at 8 TB/s is 1.0e12 units/s
    rl_sweep["units_per_s"] = units / (sweep_ms * 1e-3)
    rl_sweep["units_roofline"] = HBM_PEAK_GBS * 1e9 / 8.0
    rl_sweep["units_frac"] = rl_sweep["units_per_s"] / rl_sweep["units_roofline"]
    spmv_ms = L.smm_batch_time_kernel(batch, L.SMM_KERNEL_CG_SPMV, 50)
    # q = A p: p read once and q written once, FP64 (16 B/DOF)
    # q = A p: p read once and q written once, FP64 (16 B/DOF); 2 N^2 flops per
    # nonzero block (the element's own block and one per interior face)
    spmv_flops = float(sum(2.0 * (wl.p + 1) ** 4 * (wl.nx * wl.ny + 2 * (2 * wl.nx * wl.ny - wl.nx - wl.ny))
                           for wl in wls))
    rl_spmv = roofline_flops("b_cg_k1", "one q = A p over the batch (the per-order launches b_cg_k1<NB>)",
                             spmv_flops, 16.0 * dofs, spmv_ms)
    log(f"sweep {sweep_ms:.3f} ms -> {units / sweep_ms / 1e-3:.3e} units/s, {rl_sweep['achieved']:.0f} GB/s; "
        f"PCG q=Ap {spmv_ms * 1e3:.1f} us, {rl_spmv['achieved']:.2f} TFLOP/s, {rl_spmv['hbm_achieved_gbs']:.0f} GB/s")
    dominant = rl_spmv if phase["pcg"] > phase["source+sweep"] else rl_sweep

    tts = None
    disc = None
    tiles = None
    curved = None
    if not args.no_solve:
        tts = time_to_solution(L, ctx, args.tts_problems, log)
        disc = moment_discretisations(L, ctx, log)
        tiles = block_jacobi_sweeps(L, ctx, log)
        curved = curved_sweeps(L, ctx, log)

    cpu = None
    if not args.no_cpu_baseline:
        rate, sample = cpu_baseline(wls[:32])
        cpu = {"value": rate, "unit": "elem*angle*DOF/s", "cores": 1, "kind": "oracle", "sample": sample,
               "cpu": cpu_model(), "host_cpus": os.cpu_count()}
        log(f"cpu baseline {rate:.3e} units/s")

    out = {
        "metric": METRIC,
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
        "dtype_detail": "sweep and moments f32; closures, PCG, residual f64; warm-start network bf16/f32",
        "data": "synthetic",
        "config": {"workload": f"batch of {args.problems} problems, seeds 0..{args.problems - 1}: "
                               "[0,1]^2 16^2..128^2, p 1..4, S4..S12, sigma_t 10^U(-1,2), c U(0.5,0.999)",
                   "units_per_sweep": units, "dof": dofs, "parallelism": "single GPU"},
        "phase_ms_per_step": phase,
        "sweep_only": {"ms": sweep_ms, "units_per_s": units / (sweep_ms * 1e-3)},
        "roofline": dominant,
        "roofline_sweep": rl_sweep,
        "roofline_pcg_spmv": rl_spmv,
        "paper_context": PAPER_CONTEXT,
        "time_to_1e-8": tts,
        "moment_discretisations": disc,
        "block_jacobi_sweeps": tiles,
        "curved_sweeps": curved,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
