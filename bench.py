#!/usr/bin/env python3
"""Benchmark: the batched SMM hot path on one MI355X.

Workload (value): 256 independent problems solved as one batch, seeds 0-255
of the seeded generator (uniform Cartesian [0,1]^2 meshes of 16^2 to 128^2
elements, orders p = 1-4, S4-S12, homogeneous sigma_t log-uniform in
[0.1, 100], scattering ratio uniform in [0.5, 0.999], unit isotropic
source, vacuum), FP32 sweeps and moments with delta sweeps, FP64 closures,
PCG and residual.  Inputs are synthetic and resident on the GPU before the
timed region.

A step is one whole batched solve of every problem from the zero start to a
1e-8 outer residual (relative max-norm of successive iterates): scattering
source, sweep (persistent per-order launches), angular moments on the matrix
cores, SMM closures, right-hand side, FP64 two-level PCG, residual, Anderson
mixing; problems that have converged drop out of later launches.
value = elem*angle*DOF units swept (units per sweep x outer iterations, per
problem) per second of whole steps, so no step sweeps past convergence.

Also reported:
  * the time of each phase inside the steps; the roofline of the sweep kernel
    (the hot loop) against the method's 8 B per unit (psi written by the
    sweep and read back by the moment contraction), with the kernel's own
    bytes beside it, and that of the PCG product;
  * the FP32 error: the batch's FP32-sweep flux against its all-FP64 solve
    (every problem) and against the oracle (three members it solves in
    seconds);
  * the wavefront critical path: levels x per-level time of single sweeps;
  * time to a 1e-8 outer residual on held-out warm-start layouts (64 x 64,
    p = 2, S8 blob layouts): the plain method (problems solved one after the
    other from the zero start) against the batched solve with the learned
    start, on identical inputs;
  * the IP and the continuous (CG) moment systems on the multi-material
    channel problem: time to a 1e-8 outer residual, and the roofline of the
    CG product kernel;
  * the parallel block Jacobi sweep on the same problem: sweep time and
    outer iterations per tile size;
  * the sweep on curved meshes (stored element operators, and the
    assembling form for comparison) at p = 2, 3, 4;
  * the CPU oracle on bounded samples of the workloads, one thread and all
    host cores, minimum of three runs.
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


def _oracle_worker(conn, tasks):
    """Child process: build the oracle problems named in `tasks` (pairs of
    batch seed and direction index) once, then sweep those directions on
    every "go", one thread."""
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import smm as osmm, transport
    from workloads import config_batched_problem

    with threadpool_limits(1):
        probs = {s: osmm.make_problem(config_batched_problem(s)) for s in sorted({s for s, _ in tasks})}
        conn.send(sum(probs[s].ne * probs[s].n for s, _ in tasks))
        while conn.recv() == "go":
            t0 = time.perf_counter()
            for s, d in tasks:
                pr = probs[s]
                transport.sweep(pr.mesh, pr.omega[d:d + 1], pr.sigma_t, np.ones((pr.ne, pr.n)), None)
            conn.send(time.perf_counter() - t0)


def _pool_sweeps(assign, runs):
    """Time the oracle sweeps of per-worker task lists on as many processes
    (one thread each); returns (units, [wall s per run])."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    procs, conns = [], []
    for tasks in assign:
        a, b = ctx.Pipe()
        pr = ctx.Process(target=_oracle_worker, args=(b, tasks), daemon=True)
        pr.start()
        procs.append(pr)
        conns.append(a)
    units = sum(c.recv() for c in conns)
    walls = []
    for _ in range(runs):
        t0 = time.perf_counter()
        for c in conns:
            c.send("go")
        for c in conns:
            c.recv()
        walls.append(time.perf_counter() - t0)
    for c in conns:
        c.send("stop")
    for pr in procs:
        pr.join(timeout=30)
    return units, walls


def cpu_baseline(n_problems: int = 8, n_dirs: int = 2, runs: int = 3):
    """The oracle (FP64, numpy) on the GPU machine's host cores, minimum of
    `runs` runs each:
      * the batch (C4): sweeps of n_dirs directions (the first of two
        quadrants) of its first n_problems problems, on one thread and on one
        process per core with the (problem, direction) sweeps spread over the
        processes by their size;
      * the plain problem (C1: 8x8, p = 1, S4): a whole solve to a 1e-8 outer
        residual, one thread;
      * the channel problem (C3: 128x128, p = 2, S12): a sweep of one
        direction, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import smm as osmm, transport
    from workloads import batched_params, config_channel, config_plain

    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    tasks = []
    for s in range(n_problems):
        prm = batched_params(s)
        nd = prm["sn"] * (prm["sn"] + 2) // 2
        tasks += [(s, (j * nd) // (2 * n_dirs)) for j in range(n_dirs)]
    size = lambda t: batched_params(t[0])["n"] ** 2 * (batched_params(t[0])["p"] + 1) ** 2
    units, walls1 = _pool_sweeps([tasks], runs)
    nw = min(ncpu, len(tasks))
    assign = [[] for _ in range(nw)]
    load = [0.0] * nw
    for t in sorted(tasks, key=lambda t: -size(t)):
        k = int(np.argmin(load))
        assign[k].append(t)
        load[k] += size(t)
    _, wallsN = _pool_sweeps(assign, runs)
    res = {"value": units / min(wallsN), "unit": "elem*angle*DOF/s", "cores": nw, "kind": "oracle",
           "sample": f"oracle FP64 sweeps of {n_dirs} directions of each of batch problems 0..{n_problems - 1} "
                     f"({units} units), {nw} processes of one thread, min of {runs} runs",
           "single_thread": {"value": units / min(walls1), "cores": 1, "runs_s": walls1},
           "all_cores_runs_s": wallsN, "cpu": cpu_model(), "host_cpus": ncpu}
    with threadpool_limits(1):
        pr = osmm.make_problem(config_plain(8, 1, 4))
        ts, its = [], 0
        for _ in range(runs):
            pr.cache.clear()
            t0 = time.perf_counter()
            _, info = osmm.solve(pr, tol=1e-8, max_it=200)
            ts.append(time.perf_counter() - t0)
            its = info["iterations"]
        u1 = pr.ne * pr.n * len(pr.w)
        res["plain_8x8_p1_s4"] = {"time_to_1e-8_s": min(ts), "outer": its, "cores": 1,
                                  "units_per_s": u1 * its / min(ts)}
        pr = osmm.make_problem(config_channel())
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            transport.sweep(pr.mesh, pr.omega[:1], pr.sigma_t, np.ones((pr.ne, pr.n)), None)
            ts.append(time.perf_counter() - t0)
        res["channel_128_p2_s12"] = {"units_per_s": pr.ne * pr.n / min(ts), "cores": 1,
                                     "sample": "sweep of 1 of the 84 directions"}
    return res


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
        # the time before the first outer iteration: building the start
        res[name + "_start_s"] = max(i["t_setup_ms"] for i in infos) * 1e-3
        log(f"{name}: {t:.2f} s, outer its mean {res[name + '_outer_mean']:.2f}, start {res[name + '_start_s']:.4f} s")
    res["learned_start_kept"] = int(L.smm_batch_warmstart_used(batch).sum())
    res["speedup_batched_warm_vs_plain"] = t_plain / res["batched_warm_s"]
    res["speedup_batched_zero_vs_plain"] = t_plain / res["batched_zero_s"]
    # what the learned start costs: inside the solve, the time before the
    # first outer iteration beyond the zero start's (the diffusion start's
    # moment solve, the features, the network); the features and the network
    # also timed on their own (the same calls the solve makes)
    nf, nt, hh, ww = L.smm_batch_warmstart_dims(batch)
    X = torch.zeros((n, hh, ww, nf), dtype=torch.float32, device="cuda")
    Y = torch.zeros((n, hh, ww, nt), dtype=torch.float32, device="cuda")
    split = {"learned_start_in_solve_s": res["batched_warm_start_s"] - res["batched_zero_start_s"],
             "diffusion_start_in_solve_s": res["batched_diffusion_start_s"] - res["batched_zero_start_s"]}
    for name, fn in (("features_s", lambda: L.smm_batch_warmstart_features(batch, 0, n, X)),
                     ("network_forward_s", lambda: [L.smm_cnn_forward(net, X[k:k + 32], min(32, n - k), Y[k:k + 32])
                                                    for k in range(0, n, 32)])):
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        split[name] = best
    per_it = res["batched_zero_s"] / max(res["batched_zero_outer_mean"], 1e-9)
    split["outer_iteration_s"] = per_it
    split["outer_iterations_saved"] = res["batched_zero_outer_mean"] - res["batched_warm_outer_mean"]
    res["learned_start_cost"] = split
    log("learned start cost: " + ", ".join(f"{k} {v:.4f}" for k, v in split.items()))
    L.smm_batch_set_warmstart(batch, None)
    L.smm_batch_destroy(batch)
    L.smm_cnn_destroy(net)
    return res


def moment_discretisations(L, ctx, log):
    """IP versus CG moment system (Sec. 5.1) on the multi-material channel
    problem (128 x 128, p = 2, S12, FP32 sweep), each with its preconditioners:
    wall time to a 1e-8 outer residual from the zero start, and the roofline
    of the CG product kernel
    (FP64 CSR, HBM-bound: 12 B per stored entry, the row pointers, x read
    once and y written once)."""
    import torch
    from workloads import config_channel

    wl = config_channel(n=128, p=2, sn=12)
    common = dict(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-8, inner_tol=1e-10, inner_adapt=1e-2,
                  max_inner=20000, max_outer=60, use_graph=1)
    variants = (("ip_two_level", dict(precond=1), "IP, typed path, two-level PCG"),
                ("ip_block_jacobi", dict(moment_path=1), "IP, per-element path, block-Jacobi PCG"),
                ("cg_jacobi", dict(discretization=L.SMM_DISC_CG), "CG, per-element path, Jacobi PCG"),
                ("cg_two_level", dict(discretization=L.SMM_DISC_CG, precond=1),
                 "CG, per-element path, two-level PCG (Jacobi + bilinear vertex space, one V-cycle)"))
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
    128, p = 2, S12): time of one FP32 sweep of the per-element sweep with
    stored element operators (one workgroup per direction and tile) for
    several tile sizes, with its parts (the parallel pass, the levels),
    outer iterations and wall time to a 1e-8 outer residual (CG moment
    system, FP32 delta sweeps), beside the tabulated Cartesian sweep, which
    has no tiled form, and the assembling per-element sweep (sweep path 5)
    on 32 x 32 tiles."""
    import torch
    from workloads import config_channel

    wl = config_channel(n=128, p=2, sn=12)
    common = dict(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-8, inner_tol=1e-10, inner_adapt=1e-2,
                  max_inner=20000, max_outer=400, use_graph=1, discretization=L.SMM_DISC_CG)
    units = float(wl.n_elem * (wl.p + 1) ** 2 * 84)
    res = {"workload": "channel 128x128 p=2 S12, FP32 delta sweeps, CG moment system, outer 1e-8",
           "units_per_sweep": units, "runs": []}
    for tiles, path in (((0, 0), 0), ((128, 128), 0), ((32, 32), 0), ((16, 16), 0), ((8, 8), 0), ((32, 32), 5)):
        p = L.problem_from_workload(ctx, wl)
        if tiles != (0, 0):
            L.smm_set_sweep_tiles(p, *tiles)
        L.smm_set_sweep_path(p, path)
        ms = L.smm_time_sweep(p, L.SMM_FP32_SWEEP, 5)
        L.smm_solve(p, L.smm_default_opts(**{**common, "max_outer": 1}), raise_on_noconv=False)  # set-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = L.smm_solve(p, L.smm_default_opts(**common), raise_on_noconv=False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        if tiles == (0, 0):
            kind = "tabulated Cartesian sweep (full)"
        elif path == 5:
            kind = f"assembling per-element sweep, tiles {tiles[0]}x{tiles[1]}"
        else:
            kind = f"stored-operator sweep, tiles {tiles[0]}x{tiles[1]}"
        run = {"kernel": kind, "tiles": list(tiles), "sweep_ms": ms, "units_per_s": units / (ms * 1e-3),
               "solve_s": t, "converged": rc == L.SMM_OK, "outer": info["iterations"]}
        if tiles != (0, 0) and path == 0:
            _, part, lev = L.smm_time_sweep_parts(p, L.SMM_FP32_SWEEP, 5)
            run["parts_ms"] = {"particular": part, "levels": lev}
        res["runs"].append(run)
        log(f"{kind}: sweep {ms:.3f} ms, solve {t * 1e3:.1f} ms, {info['iterations']} outer")
        L.smm_problem_destroy(p)
    return res


def curved_sweeps(L, ctx, log):
    """The sweep on curved meshes (the manufactured problem: 32 x 32 elements
    with an order-p map, S8) with stored element operators: per p the FP32
    and FP64 time per sweep and units/s; its parts (the one-off build of the
    operators, the parallel pass psi = A^-1 (M S + inflow), the levels); the
    levels and the time per level; the parallel pass against HBM at its
    algorithmic bytes ((n^2 + 2n) values per element and direction: H = A^-1 M
    and c read, psi written); and, for comparison, the sweep that assembles and
    eliminates every element's system in each sweep (sweep path 5)."""
    from workloads import config_curved_mms

    res = {"workload": "curved manufactured problem, 32x32 elements, order-p map, S8 (40 directions)", "runs": []}
    for p in (2, 3, 4):
        wl = config_curved_mms(32, p, 8)
        prob = L.problem_from_workload(ctx, wl)
        n = (p + 1) ** 2
        pairs = wl.n_elem * 40
        units = float(pairs * n)
        run = {"p": p, "units_per_sweep": units}
        for name, prec in (("fp32", L.SMM_FP32_SWEEP), ("fp64", L.SMM_FP64)):
            ms = L.smm_time_sweep(prob, prec, 10)
            run[name + "_ms"] = ms
            run[name + "_units_per_s"] = units / (ms * 1e-3)
        setup, part, lev_ms = L.smm_time_sweep_parts(prob, L.SMM_FP32_SWEEP, 10)
        nlev = int(L.smm_debug_sweep_graph(prob)[0].max()) + 1
        run["fp32_parts_ms"] = {"operator_build": setup, "particular": part, "levels": lev_ms}
        run["levels"] = nlev
        run["us_per_level"] = 1e3 * lev_ms / nlev
        gbs = 4.0 * pairs * (n * n + 2 * n) / (part * 1e-3) / 1e9
        run["roofline_fp32"] = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                                "traffic": None, "kernel": "gen_inv_particular_kernel"}
        L.smm_set_sweep_path(prob, 5)
        run["assembled_fp32_ms"] = L.smm_time_sweep(prob, L.SMM_FP32_SWEEP, 5)
        log(f"curved 32^2 p={p} S8: FP32 sweep {run['fp32_ms']:.3f} ms (particular {part:.3f}, levels {lev_ms:.3f} = "
            f"{nlev} x {run['us_per_level']:.2f} us; build {setup:.3f}), FP64 {run['fp64_ms']:.3f} ms; assembling "
            f"{run['assembled_fp32_ms']:.3f} ms")
        res["runs"].append(run)
        L.smm_problem_destroy(prob)
    return res


def fp32_error(L, ctx, batch, probs, wls, log):
    """FP32-sweep flux of the batch (outer 1e-8) against its all-FP64 solve
    (outer 1e-10) for every problem, and against the oracle's converged flux
    for three members the oracle solves in seconds."""
    import numpy as np
    from oracle import smm as osmm

    def outputs():
        out = []
        for k, p in enumerate(probs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            out.append(v)
        return out

    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    v32 = outputs()
    o64 = L.smm_default_opts(precision=L.SMM_FP64, delta_sweeps=0, outer_tol=1e-10, inner_tol=1e-12,
                             inner_adapt=3e-3, max_inner=20000, max_outer=150, precond=L.SMM_PRECOND_TWOLEVEL,
                             use_graph=1, anderson=2)
    rc, _ = L.smm_batch_solve(batch, o64, raise_on_noconv=False)
    v64 = outputs()
    errs = np.array([rel(a, b) for a, b in zip(v32, v64)])
    res = {"vs_gpu_fp64_max": float(errs.max()), "vs_gpu_fp64_median": float(np.median(errs)),
           "fp64_converged": rc == L.SMM_OK, "bar": 1e-5, "members_vs_oracle": {}}
    for s in (133, 196, 10):
        if s < len(wls):
            ref, info = osmm.solve(osmm.make_problem(wls[s]), tol=1e-11, max_it=200)
            res["members_vs_oracle"][str(s)] = {"fp32": rel(v32[s], ref), "fp64": rel(v64[s], ref),
                                                "mesh": f"{wls[s].nx}^2 p={wls[s].p} S{wls[s].sn}"}
    log(f"FP32 vs FP64 (all {len(probs)} problems): max {errs.max():.2e}, median {np.median(errs):.2e}; "
        f"vs oracle {res['members_vs_oracle']}")
    return res


def critical_path(L, ctx, log):
    """Wavefront critical path of single sweeps: levels x per-level time
    (sweep time / levels), for the channel problem (C3) and the curved 32^2
    problem at p = 4 (C2) with their own kernels, and for the largest members
    of the batch (C4) with the batch's kernel: each member alone in a batch,
    all its directions at once (one workgroup each, so each level's latency
    is measured without contention)."""
    from workloads import config_batched_problem, config_channel, config_curved_mms

    out = []
    p = L.problem_from_workload(ctx, config_channel())
    lev = 128 + 128 - 1
    ms = L.smm_time_sweep(p, L.SMM_FP32_SWEEP, 10)
    out.append({"case": "channel 128^2 p=2 S12", "kernel": "single-problem Cartesian sweep", "levels": lev,
                "sweep_ms": ms, "us_per_level": 1e3 * ms / lev})
    log(f"critical path channel 128^2 p=2 S12: {lev} levels, {ms:.3f} ms, {1e3 * ms / lev:.2f} us/level")
    L.smm_problem_destroy(p)
    # curved: the level pass alone (the parallel pass before it has no levels)
    p = L.problem_from_workload(ctx, config_curved_mms(32, 4, 8))
    lev = int(L.smm_debug_sweep_graph(p)[0].max()) + 1
    ms = L.smm_time_sweep(p, L.SMM_FP32_SWEEP, 10)
    lev_ms = L.smm_time_sweep_parts(p, L.SMM_FP32_SWEEP, 10)[2]
    out.append({"case": "curved 32^2 p=4 S8", "kernel": "gen_inv_sweep_kernel (levels of the stored-operator sweep)",
                "levels": lev, "sweep_ms": ms, "levels_ms": lev_ms, "us_per_level": 1e3 * lev_ms / lev})
    log(f"critical path curved 32^2 p=4 S8: {lev} levels, {lev_ms:.3f} ms of {ms:.3f} ms, "
        f"{1e3 * lev_ms / lev:.2f} us/level")
    L.smm_problem_destroy(p)
    for s in (23, 9, 0, 19):
        wl = config_batched_problem(s)
        name = f"batch member {s}: {wl.nx}^2 p={wl.p} S{wl.sn}"
        p = L.problem_from_workload(ctx, wl)
        b = L.smm_batch_create(ctx, [p])
        lev = wl.nx + wl.ny - 1
        ms = L.smm_batch_time_sweep(b, L.SMM_FP32_SWEEP, 10)
        out.append({"case": name, "kernel": "b_sweep_mfma_kernel (batch of one)", "levels": lev, "sweep_ms": ms,
                    "us_per_level": 1e3 * ms / lev})
        log(f"critical path {name} (batched kernel): {lev} levels, {ms:.3f} ms, {1e3 * ms / lev:.2f} us/level")
        L.smm_batch_destroy(b)
        L.smm_problem_destroy(p)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed whole solves of the batch")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--problems", type=int, default=256)
    ap.add_argument("--tts-problems", type=int, default=200, help="held-out problems for the time-to-solution run")
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
    ap.add_argument("--solve-only", action="store_true",
                    help="run only the warm-up and timed batch solves and print their time and phases")
    ap.add_argument("--sweep-only", action="store_true",
                    help="run only the batched FP32 sweep of the 256-problem batch (tuned, then 10 timed "
                         "sweeps) and print its roofline JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the problems of a batch are "
              "independent and would be split across GPUs by the caller)", file=sys.stderr)
        sys.exit(2)
    only = args.disc_only or args.tiles_only or args.curved_only or args.sweep_only or args.solve_only

    # the CPU baseline runs first: its worker processes start before this
    # process touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not only:
        cpu = cpu_baseline()
        log(f"cpu baseline {cpu['value']:.3e} units/s on {cpu['cores']} cores "
            f"(one thread {cpu['single_thread']['value']:.3e})")

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
    if args.sweep_only:
        # the source of the sweeps is whatever the batch holds (their time does not depend on it)
        L.smm_batch_time_kernel(batch, L.SMM_KERNEL_SWEEP_FP32, 2)        # tunes grids and streams
        ms = L.smm_batch_time_kernel(batch, L.SMM_KERNEL_SWEEP_FP32, 10)
        rl = roofline("b_sweep_mfma_kernel", "one batched FP32 sweep at 8 B per elem*angle*DOF", 8.0 * units, ms)
        rl["units_per_s"] = units / (ms * 1e-3)
        print(json.dumps({"sweep_ms": ms, "units_per_sweep": units, "roofline": rl}))
        return
    unit_k = np.array([p.n_elem * p.n_node * p.n_dir for p in probs], dtype=float)
    dofs = float(sum(p.n_elem * p.n_node for p in probs))
    log(f"batch of {args.problems} problems: {units:.4g} units per sweep, {dofs:.4g} DOF, "
        f"set-up {time.time() - t0:.1f} s")

    # inner tolerance 3e-3 x the last outer residual: looser inner solves stall
    # the outer iteration of the most scattering members (1e-2: 17 outer
    # iterations at most, 1e-1: no convergence in 150), tighter ones cost more
    # PCG iterations than the outer iterations they save
    opts = L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-8,
                              inner_tol=1e-10, inner_adapt=3e-3, max_inner=20000, max_outer=150,
                              precond=args.precond, use_graph=1, anderson=args.anderson)
    for _ in range(max(args.warmup, 1)):                         # also autotunes the sweep grids
        L.smm_batch_solve(batch, opts, raise_on_noconv=False)
    torch.cuda.synchronize()
    walls = []
    swept = 0.0
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, infos = L.smm_batch_solve(batch, opts, raise_on_noconv=False)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        its = np.array([i["iterations"] for i in infos], dtype=float)
        swept += float(np.dot(unit_k, its))
        assert rc == L.SMM_OK, rc
    wall = sum(walls)
    ms_per_step = 1e3 * wall / args.steps
    value = swept / wall
    phases, cg_its = L.smm_batch_phase_times(batch)
    names = ["source+sweep", "moments+closures+rhs", "pcg", "residual"]
    phase = {n: ms for n, ms in zip(names, phases)}
    its_last = np.array([i["iterations"] for i in infos])
    log(f"{args.steps} solves to 1e-8: {ms_per_step:.1f} ms each (min {1e3 * min(walls):.1f}); outer iterations "
        f"mean {its_last.mean():.2f} max {its_last.max()}; per solve " +
        ", ".join(f"{n} {v:.2f} ms" for n, v in phase.items()) + f"; batched PCG iterations {cg_its}")
    if args.solve_only:
        print(json.dumps({"ms_per_step": ms_per_step, "value": value, "phase_ms_per_step": phase,
                          "batched_pcg_iterations_per_step": cg_its}))
        L.smm_batch_destroy(batch)
        return

    sweep_ms = L.smm_batch_time_kernel(batch, L.SMM_KERNEL_SWEEP_FP32, 5)
    # the sweep against the method's unit roofline: 8 B per elem*angle*DOF in
    # FP32 (psi written by the sweep and read back by the moment contraction)
    rl_sweep = roofline("b_sweep_mfma_kernel", "one batched FP32 sweep (the per-order launches "
                        "b_sweep_mfma_kernel<NB, TPW, MULTI>, each level a product on the matrix cores) "
                        "at 8 B per elem*angle*DOF", 8.0 * units, sweep_ms)
    # the kernel's own bytes: psi written once in FP32 (4 B/unit) + the FP32
    # source read once per element and problem (4/N_dir B/unit)
    own = float(sum(p.n_elem * p.n_node * (4.0 * p.n_dir + 4.0) for p in probs))
    rl_sweep["units_per_s"] = units / (sweep_ms * 1e-3)
    rl_sweep["units_roofline"] = HBM_PEAK_GBS * 1e9 / 8.0
    rl_sweep["kernel_own_bytes_per_launch"] = own
    rl_sweep["kernel_own_gbs"] = own / (sweep_ms * 1e-3) / 1e9
    rl_sweep["kernel_own_frac"] = rl_sweep["kernel_own_gbs"] / HBM_PEAK_GBS
    spmv_ms = L.smm_batch_time_kernel(batch, L.SMM_KERNEL_CG_SPMV, 50)
    # q = A p: p read once and q written once, FP64 (16 B/DOF); 2 N^2 flops per
    # nonzero block (the element's own block and one per interior face)
    spmv_flops = float(sum(2.0 * (wl.p + 1) ** 4 * (wl.nx * wl.ny + 2 * (2 * wl.nx * wl.ny - wl.nx - wl.ny))
                           for wl in wls))
    rl_spmv = roofline_flops("b_cg_k1", "one q = A p over the batch (the per-order launches b_cg_k1<NB>)",
                             spmv_flops, 16.0 * dofs, spmv_ms)
    # the angular moments of the last FP32 sweep (MFMA contraction over the
    # directions): psi read once (4 B/unit), 8 FP64 moment rows written (64 B/DOF)
    mom_ms = L.smm_batch_time_kernel(batch, L.SMM_KERNEL_MOMENTS_FP32, 20)
    rl_mom = roofline("b_moments_kernel", "the angular moments of one FP32 sweep over the batch (8 rows, FP64 out)",
                      4.0 * units + 64.0 * dofs, mom_ms)
    log(f"moments {mom_ms:.3f} ms, {rl_mom['achieved']:.0f} GB/s ({rl_mom['frac']:.3f} of HBM)")
    log(f"sweep {sweep_ms:.3f} ms -> {units / sweep_ms / 1e-3:.3e} units/s, frac {rl_sweep['frac']:.3f} of the "
        f"8 B/unit roofline (own bytes {rl_sweep['kernel_own_gbs']:.0f} GB/s); PCG q=Ap {spmv_ms * 1e3:.1f} us, "
        f"{rl_spmv['achieved']:.2f} TFLOP/s")
    err = fp32_error(L, ctx, batch, probs, wls, log)
    L.smm_batch_destroy(batch)

    tts = disc = tiles = curved = crit = None
    if not args.no_solve:
        crit = critical_path(L, ctx, log)
        tts = time_to_solution(L, ctx, args.tts_problems, log)
        disc = moment_discretisations(L, ctx, log)
        tiles = block_jacobi_sweeps(L, ctx, log)
        curved = curved_sweeps(L, ctx, log)

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
                               "[0,1]^2 16^2..128^2, p 1..4, S4..S12, sigma_t 10^U(-1,2), c U(0.5,0.999); "
                               "a step is one whole batched solve from the zero start to a 1e-8 outer residual",
                   "units_per_sweep": units, "dof": dofs, "parallelism": "single GPU",
                   "outer_iterations_mean": float(its_last.mean()), "outer_iterations_max": int(its_last.max()),
                   "units_swept_per_step": swept / args.steps},
        "step_ms_min": 1e3 * min(walls),
        "phase_ms_per_step": phase,
        "batched_pcg_iterations_per_step": cg_its,
        "sweep_only": {"ms": sweep_ms, "units_per_s": units / (sweep_ms * 1e-3)},
        "roofline": rl_sweep,
        "roofline_pcg_spmv": rl_spmv,
        "roofline_moments": rl_mom,
        "fp32_error": err,
        "critical_path": crit,
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
