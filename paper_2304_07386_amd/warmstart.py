"""Learned warm start: training data from batched solves, training with the
library's own network kernels, and weight files.

Data: for each layout, the diffusion start varphi_D and the converged SMM
solution give the network's features and targets (see include/smm_cnn.h).
Training: Adam on the weighted mean squared error, channel weights 1/variance
of each target channel over the training set, the correction-source channels
(an auxiliary target: the start uses the flux channels) scaled down by
AUX_WEIGHT.  Weights are stored as .npz
(float32 parameters plus JSON metadata), loaded without pickle.

Usage (GPU):
    python -m paper_2304_07386_amd.warmstart --train-seeds 10000:12000 \
        --out paper_2304_07386_amd/weights/warmstart_blobs64_p2_s8.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import smm as L
from .workload_io import problem_from_workload

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_blobs64_p2_s8.npz")
HIDDEN = (32, 32, 32)
AUX_WEIGHT = 0.25


def he_init(channels, seed: int) -> np.ndarray:
    """He-normal 3x3 weights, zero biases, in the smm_cnn parameter layout."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        out.append(rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), cout * cin * 9))
        out.append(np.zeros(cout))
    return np.concatenate(out).astype(np.float32)


def solve_opts(tol=1e-8, precision=L.SMM_FP32_SWEEP, start=L.SMM_START_DIFFUSION, inner_adapt=1e-2,
               precond=L.SMM_PRECOND_TWOLEVEL, anderson=2, start_tol=0.1):
    """Solve options used for data generation and the start comparisons:
    inexact moment solves tied to the outer residual, two-level PCG, Anderson
    mixing of the outer iterates, PCG chunks from graphs; the moment solve
    that builds a diffusion or learned start stops at relative residual
    start_tol (the start only seeds the fixed point)."""
    o = L.smm_default_opts(precision=precision, outer_tol=tol, max_outer=200,
                           inner_tol=1e-10 if precision != L.SMM_FP64 else 1e-13, max_inner=20000,
                           delta_sweeps=1 if precision != L.SMM_FP64 else 0, use_graph=1,
                           inner_adapt=inner_adapt, precond=precond, anderson=anderson, start_tol=start_tol)
    o.start = start
    return o


def generate(ctx, workloads, chunk: int = 250, log=print):
    """Features and targets (device float32 tensors [N][ny][nx][c]) of the
    given workloads, solved in batches of `chunk` problems to a 1e-8 outer
    residual (FP32 sweeps, FP64 moment solves)."""
    import torch
    X = T = None
    n = len(workloads)
    for first in range(0, n, chunk):
        wls = workloads[first:first + chunk]
        t0 = time.time()
        probs = [problem_from_workload(ctx, wl) for wl in wls]
        batch = L.smm_batch_create(ctx, probs)
        nf, nt, ny, nx = L.smm_batch_warmstart_dims(batch)
        if X is None:
            X = torch.empty((n, ny, nx, nf), dtype=torch.float32, device="cuda")
            T = torch.empty((n, ny, nx, nt), dtype=torch.float32, device="cuda")
        o = solve_opts()
        # the diffusion start as the learned start builds it (same tolerance)
        L.smm_batch_diffusion(batch, max(o.inner_tol, o.inner_adapt), o.max_inner)
        rc, infos = L.smm_batch_solve(batch, o, raise_on_noconv=False)
        L.smm_batch_warmstart_features(batch, 0, len(wls), X[first:first + len(wls)])
        L.smm_batch_warmstart_targets(batch, 0, len(wls), T[first:first + len(wls)])
        its = [i["iterations"] for i in infos]
        log(f"[warmstart] data {first + len(wls)}/{n}: {time.time() - t0:.1f} s, outer its mean {np.mean(its):.2f}, "
            f"status {rc}")
        L.smm_batch_destroy(batch)
        del probs
    torch.cuda.synchronize()
    return X, T


def channel_weights(T) -> np.ndarray:
    """1 / variance of each target channel (over all images and pixels); the
    second half (correction source) scaled by AUX_WEIGHT."""
    v = T.reshape(-1, T.shape[-1]).double().var(dim=0).cpu().numpy()
    w = 1.0 / np.maximum(v, 1e-12)
    w[T.shape[-1] // 2:] *= AUX_WEIGHT
    return w.astype(np.float32)


def train(ctx, X, T, epochs=60, batch=32, lr=2e-3, seed=0, log=print, Xval=None, Tval=None):
    """Train a network [nf, 32, 32, 32, nt] on (X, T); returns (net, history)."""
    import torch
    n, ny, nx, nf = X.shape
    nt = T.shape[-1]
    channels = [nf, *HIDDEN, nt]
    net = L.smm_cnn_create(ctx, channels, ny, nx, batch)
    L.smm_cnn_set_params(net, he_init(channels, seed))
    w = channel_weights(T)
    rng = np.random.default_rng(seed + 1)
    steps = n // batch
    total = epochs * steps
    hist = []
    idx_dev = torch.empty(batch, dtype=torch.int32, device="cuda")
    k = 0
    for ep in range(epochs):
        perm = rng.permutation(n).astype(np.int32)
        tl = 0.0
        for s in range(steps):
            idx_dev.copy_(torch.from_numpy(perm[s * batch:(s + 1) * batch]))
            lr_k = lr * 0.5 * (1 + np.cos(np.pi * k / total))   # cosine decay
            loss, _ = L.smm_cnn_loss_grad(net, X, T, idx_dev, batch, w)
            L.smm_cnn_adam_step(net, lr_k)
            tl += loss
            k += 1
        rec = {"epoch": ep, "train_loss": tl / steps}
        if Xval is not None:
            rec["val_loss"] = evaluate(net, Xval, Tval, w)
        hist.append(rec)
        log(f"[warmstart] epoch {ep}: " + ", ".join(f"{a} {b:.4g}" for a, b in rec.items() if a != "epoch"))
    return net, hist, w


def evaluate(net, X, T, w) -> float:
    """Weighted MSE of the network over (X, T), in batches."""
    import torch
    n = X.shape[0]
    tot = 0.0
    b = net.max_batch
    for first in range(0, n - n % b if n >= b else 0, b):
        idx = torch.arange(first, first + b, dtype=torch.int32, device="cuda")
        loss, _ = L.smm_cnn_loss_grad(net, X, T, idx, b, w)
        tot += loss * b
    done = (n // b) * b
    return tot / max(done, 1)


def save(net, path, meta: dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    params = L.smm_cnn_get_params(net)
    meta = dict(meta, channels=net.channels, height=net.height, width=net.width)
    np.savez(path, params=params, meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_meta(path) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return json.loads(bytes(z["meta"]).decode())


def load(ctx, path=DEFAULT_WEIGHTS, max_batch: int = 64):
    """Network with the weights of `path` (an .npz written by save)."""
    with np.load(path, allow_pickle=False) as z:
        params = np.array(z["params"], dtype=np.float32)
        meta = json.loads(bytes(z["meta"]).decode())
    net = L.smm_cnn_create(ctx, meta["channels"], meta["height"], meta["width"], max_batch)
    L.smm_cnn_set_params(net, params)
    return net, meta


def compare_starts(ctx, net, workloads, tol=1e-8, log=print):
    """Solve the workloads as one batch from the zero, diffusion and learned
    starts; returns {start: {"outer": [...], "cg": [...], "ms": t, "used": n}}."""
    import torch
    probs = [problem_from_workload(ctx, wl) for wl in workloads]
    batch = L.smm_batch_create(ctx, probs)
    L.smm_batch_set_warmstart(batch, net)
    out = {}
    for name, start in (("zero", L.SMM_START_ZERO), ("diffusion", L.SMM_START_DIFFUSION),
                        ("learned", L.SMM_START_LEARNED)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, infos = L.smm_batch_solve(batch, solve_opts(tol, start=start), raise_on_noconv=False)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        rec = {"status": rc, "ms": ms, "outer": [i["iterations"] for i in infos],
               "cg": [i["cg_iterations_total"] for i in infos]}
        if start == L.SMM_START_LEARNED:
            rec["used"] = int(L.smm_batch_warmstart_used(batch).sum())
        out[name] = rec
        log(f"[warmstart] {name:9s} start: {ms:9.1f} ms, outer its mean {np.mean(rec['outer']):.2f} "
            f"max {max(rec['outer'])}, CG its mean {np.mean(rec['cg']):.0f}"
            + (f", learned start kept for {rec['used']}/{len(workloads)}" if "used" in rec else ""))
    L.smm_batch_set_warmstart(batch, None)
    L.smm_batch_destroy(batch)
    return out


def _seeds(spec: str):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


def main(argv=None):
    import torch
    from workloads import config_blobs

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train-seeds", default="10000:12000")
    ap.add_argument("--val-seeds", default="20000:20200")
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    ctx = L.smm_ctx_create(0, torch.cuda.current_stream())
    tr = _seeds(a.train_seeds)
    va = _seeds(a.val_seeds)
    t0 = time.time()
    X, T = generate(ctx, [config_blobs(s) for s in tr], log=log)
    Xv, Tv = generate(ctx, [config_blobs(s) for s in va], log=log)
    tgen = time.time() - t0
    t0 = time.time()
    net, hist, w = train(ctx, X, T, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log, Xval=Xv, Tval=Tv)
    ttrain = time.time() - t0
    del X, T, Xv, Tv
    torch.cuda.empty_cache()
    held = compare_starts(ctx, net, [config_blobs(s) for s in va], log=log)
    save(net, a.out, {"train_seeds": a.train_seeds, "val_seeds": a.val_seeds, "epochs": a.epochs,
                      "batch": a.batch, "lr": a.lr, "history": hist, "chan_weight": w.tolist(),
                      "workload": "blobs 64x64 p=2 S8", "t_generate_s": tgen, "t_train_s": ttrain,
                      "held_out": held})
    log(f"[warmstart] saved {a.out} (generate {tgen:.1f} s, train {ttrain:.1f} s)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
