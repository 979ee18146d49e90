"""HBM traffic of the dominant kernels from rocprofv3 counters.

Two steps.  On the GPU, under rocprofv3 (one counter per run):

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_fetch> -o pmc -- \\
        python -m paper_2304_07386_amd.counters run
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir_write> -o pmc -- \\
        python -m paper_2304_07386_amd.counters run

`run` builds the 256-problem batch of bench.py, runs one short solve (so the
PCG vectors hold a real state), then launches the batched sweep and the PCG
kernel q = A p a few times each and copies a buffer of known size with
hipMemcpy (calibration).  Then, anywhere:

    python -m paper_2304_07386_amd.counters parse <dir_fetch> <dir_write> --out <json>

reads the per-dispatch counters (KiB), scales each counter by what it reads
for the copy of known size, and writes the HBM bytes per launch of each
kernel (q = A p, the sweep, the angular moments of one sweep), with the
SHA-256 of the kernel source they were taken on.  An
optional third pass (`--pmc` with FLOP_COUNTERS, parsed with `--flops`) adds
the floating-point work the hardware issued for q = A p and the sweep.  Besides
q = A p and the sweep it records the other kernels of one PCG iteration (the
update, the direction update and the continuous-space term), per iteration.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 512 << 20
SWEEP_REPS = 2
SPMV_REPS = 5
MOM_REPS = 3


def run():
    import torch
    from . import smm as L
    from .workload_io import problem_from_workload
    sys.path.insert(0, os.path.dirname(HERE))
    from workloads import config_batched_problem

    ctx = L.smm_ctx_create(0, torch.cuda.current_stream())
    probs = [problem_from_workload(ctx, config_batched_problem(s)) for s in range(256)]
    batch = L.smm_batch_create(ctx, probs)
    o = L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=0.0, inner_tol=1e-10,
                           max_inner=2, max_outer=1, precond=L.SMM_PRECOND_TWOLEVEL)
    L.smm_batch_solve(batch, o, raise_on_noconv=False)
    L.smm_batch_time_kernel(batch, L.SMM_KERNEL_SWEEP_FP32, SWEEP_REPS)
    L.smm_batch_time_kernel(batch, L.SMM_KERNEL_CG_SPMV, SPMV_REPS)
    L.smm_batch_time_kernel(batch, L.SMM_KERNEL_MOMENTS_FP32, MOM_REPS)
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    print("[counters] done", flush=True)


def sweep_launches(nprob=256):
    """Persistent launches per batched sweep: one per order present (as the
    library groups the tasks)."""
    sys.path.insert(0, os.path.dirname(HERE))
    from workloads import config_batched_problem
    return len({config_batched_problem(s).p for s in range(nprob)})


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows):
    """[(kernel name, value)] in dispatch order (values summed over dimensions)."""
    acc = {}
    order = []
    for r in rows:
        key = int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)))
        if key not in acc:
            acc[key] = [r["Kernel_Name"], 0.0]
            order.append(key)
        acc[key][1] += float(r["Counter_Value"])
    return [tuple(acc[k]) for k in sorted(order)]


FLOP_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_FMA_F32",
                 "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32")
SWEEP = "b_sweep_mfma_kernel"   # table key of the batched FP32 sweep (any of its launches)


def _is_sweep(name):
    return "b_sweep_" in name


def _per_dispatch_counters(rows):
    """[(kernel name, {counter: value})] in dispatch order."""
    acc = {}
    for r in rows:
        key = int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)))
        ent = acc.setdefault(key, [r["Kernel_Name"], {}])
        ent[1][r["Counter_Name"]] = ent[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [tuple(acc[k]) for k in sorted(acc)]


def issued_flops(dir_flops):
    """Issued floating-point work per operation from a third counter pass
    (FLOP_COUNTERS): FP64 matrix-core work is SQ_INSTS_VALU_MFMA_MOPS_F64 x
    512 (the counter's unit); FP32 vector work counts every lane of the
    issued FMA (2 flops), ADD and MUL instructions (64 lanes each: an upper
    bound where waves are partly masked)."""
    disp = _per_dispatch_counters(_rows(dir_flops))
    k1 = [(n, c) for n, c in disp if "b_cg_k1" in n]
    nvar = len({n for n, c in k1})
    spmv = [c for n, c in k1[-SPMV_REPS * nvar:]]
    sw = [c for n, c in disp if _is_sweep(n)][-SWEEP_REPS * sweep_launches():]
    mfma = sum(c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) for c in spmv) * 512.0 / SPMV_REPS
    f32m = sum(c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) for c in sw) * 512.0 / SWEEP_REPS
    f32v = sum(64.0 * (2.0 * c.get("SQ_INSTS_VALU_FMA_F32", 0.0) + c.get("SQ_INSTS_VALU_ADD_F32", 0.0)
                       + c.get("SQ_INSTS_VALU_MUL_F32", 0.0)) for c in sw) / SWEEP_REPS
    return {"b_cg_k1": {"issued_flops_per_launch": mfma, "kind": "FP64 MFMA (SQ_INSTS_VALU_MFMA_MOPS_F64 x 512)"},
            SWEEP: {"issued_flops_per_launch": f32m + f32v, "issued_mfma_flops_per_launch": f32m,
                    "issued_valu_flops_per_launch": f32v,
                    "kind": "FP32 MFMA (SQ_INSTS_VALU_MFMA_MOPS_F32 x 512) + FP32 VALU lane slots "
                            "(64 x (2 FMA + ADD + MUL) instructions)"}}


def parse(dir_fetch, dir_write, out, dir_flops=None):
    res = {}
    for which, d in (("fetch", dir_fetch), ("write", dir_write)):
        disp = _per_dispatch(_rows(d))
        copies = [v for n, v in disp if "copyBuffer" in n or "copy" in n.lower() and "smm" not in n]
        big = max(copies) if copies else None
        if not big:
            raise RuntimeError("no calibration copy found")
        scale = (COPY_BYTES / 1024.0) / big           # KiB of the copy / KiB the counter read
        # one q = A p is one launch per order present (b_cg_k1<NB>), or the
        # per-node kernel b_cg_k1n: the last SPMV_REPS rounds of them
        k1 = [(n, v) for n, v in disp if "b_cg_k1" in n]
        nvar = len({n for n, v in k1})
        spmv = [v for n, v in k1[-SPMV_REPS * nvar:]]
        sweeps = [v for n, v in disp if _is_sweep(n)]
        # the timed sweeps: the last SWEEP_REPS * (launches per sweep) dispatches
        sw = sweeps[-SWEEP_REPS * sweep_launches():]
        # the moments of one whole sweep: the last MOM_REPS launches
        mom = [v for n, v in disp if "b_moments_kernel" in n][-MOM_REPS:]
        res[which] = {"scale": scale, "copy_kib": big,
                      "b_cg_k1": 1024.0 * scale * sum(spmv) / SPMV_REPS,
                      SWEEP: 1024.0 * scale * sum(sw) / SWEEP_REPS,
                      "b_moments_kernel": 1024.0 * scale * sum(mom) / max(len(mom), 1)}
        # the other kernels of one PCG iteration, from the short solve (every
        # problem still iterating): the mean dispatch of each kernel, summed
        # over the per-order launches
        for k in ("b_cg_k2", "b_cg_k3g", "cgl_kernel"):
            per = {}
            for n, v in disp:
                if k + "<" in n or (k == "cgl_kernel" and k in n):
                    per.setdefault(n, []).append(v)
            res[which][k] = 1024.0 * scale * sum(sum(v) / len(v) for v in per.values())
    src = os.path.join(HERE, "csrc", "kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    table = {}
    for k in ("b_cg_k1", SWEEP, "b_cg_k2", "b_cg_k3g", "cgl_kernel", "b_moments_kernel"):
        table[k] = {"bytes_per_launch": res["fetch"][k] + res["write"][k],
                    "fetch_bytes": res["fetch"][k], "write_bytes": res["write"][k],
                    "source": "kernels.hip", "sha256": sha}
    if dir_flops:
        for k, v in issued_flops(dir_flops).items():
            table[k].update(v)
    table["_calibration"] = {"copy_bytes": COPY_BYTES, "fetch_scale": res["fetch"]["scale"],
                             "write_scale": res["write"]["scale"]}
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("run")
    p = sub.add_parser("parse")
    p.add_argument("dir_fetch")
    p.add_argument("dir_write")
    p.add_argument("--flops", default=None, help="directory of a third pass with the FLOP_COUNTERS")
    p.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run()
    else:
        parse(a.dir_fetch, a.dir_write, a.out, a.flops)
    return 0


if __name__ == "__main__":
    sys.exit(main())
