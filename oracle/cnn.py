"""Plain convolutional network for the learned SMM warm start (oracle).

A stack of 3x3 convolutions (zero padding, stride 1) with ReLU between
layers maps per-element features of a layout to per-element outputs
(nodal scalar flux and correction source).  Tensors are NHWC: [batch,
height, width, channels]; weights are [cout, cin, 3, 3].

The network stores weights and activations in bfloat16 and accumulates in
FP32 on the GPU.  This oracle computes in FP64 and rounds to bfloat16 at the
same points (weights, layer inputs, gradients fed back between layers), so
the two differ only by accumulation order and precision.

Parity unpinned by the paper (the network is not in it): the gradients are
pinned by central differences in FP64 on the unrounded network, the Adam
step by its published update rule (Kingma and Ba, 2015).
"""
from __future__ import annotations

import numpy as np


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out.reshape(np.shape(x))


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n,i,j,o] = b[o] + sum_{c,di,dj} w[o,c,di,dj] x[n, i+di-1, j+dj-1, c]."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.zeros((n, h, wd, w.shape[0])) + b
    for di in range(3):
        for dj in range(3):
            y += np.einsum("nijc,oc->nijo", xp[:, di:di + h, dj:dj + wd, :], w[:, :, di, dj])
    return y


def conv3x3_backward(x: np.ndarray, w: np.ndarray, gy: np.ndarray):
    """Gradients of sum(gy * conv3x3(x, w, b)) with respect to x, w and b."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1, :] = x
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for di in range(3):
        for dj in range(3):
            gw[:, :, di, dj] = np.einsum("nijo,nijc->oc", gy, xp[:, di:di + h, dj:dj + wd, :])
            gxp[:, di:di + h, dj:dj + wd, :] += np.einsum("nijo,oc->nijc", gy, w[:, :, di, dj])
    gb = gy.sum(axis=(0, 1, 2))
    return gxp[:, 1:-1, 1:-1, :], gw, gb


def init_params(sizes, seed: int = 0):
    """He-normal weights drawn from SplitMix64-seeded numpy, zero biases.
    sizes: channel counts [c0, c1, ..., cL]."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(sizes[:-1], sizes[1:]):
        std = np.sqrt(2.0 / (9 * cin))
        params.append((rng.normal(0.0, std, (cout, cin, 3, 3)), np.zeros(cout)))
    return params


def forward(params, x: np.ndarray, emulate_bf16: bool = True):
    """Returns (output, cache).  Hidden layers use ReLU; the last is linear."""
    r = bf16 if emulate_bf16 else (lambda a: a)
    a = r(x)
    cache = []
    for k, (w, b) in enumerate(params):
        z = conv3x3(a, r(w), b)
        cache.append((a, z))
        if k < len(params) - 1:
            a = r(np.maximum(z, 0.0))
        else:
            a = z
    return a, cache


def loss_mse(y: np.ndarray, t: np.ndarray, chan_weight: np.ndarray | None = None):
    """Weighted mean squared error: mean over all entries of w_o (y - t)^2,
    w_o a per-output-channel weight (1 if None).  Returns (loss, d loss/dy)."""
    d = y - t
    w = np.ones(y.shape[-1]) if chan_weight is None else np.asarray(chan_weight, float)
    return float(np.mean(w * d * d)), 2.0 * w * d / d.size


def backward(params, cache, gy: np.ndarray, emulate_bf16: bool = True):
    """Parameter gradients [(gw, gb)] given d loss / d output.  The output
    gradient is rounded to bfloat16 like every gradient fed between layers;
    the ReLU derivative is 1 where the stored (rounded) activation is
    positive."""
    r = bf16 if emulate_bf16 else (lambda a: a)
    grads = [None] * len(params)
    g = r(gy)
    for k in range(len(params) - 1, -1, -1):
        w, b = params[k]
        a, z = cache[k]
        if k < len(params) - 1:
            g = g * (cache[k + 1][0] > 0.0)
        gx, gw, gb = conv3x3_backward(a, r(w), g)
        grads[k] = (gw, gb)
        g = r(gx)
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""
    t = state.get("t", 0) + 1
    state["t"] = t
    if "m" not in state:
        state["m"] = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
        state["v"] = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    out = []
    for k, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((w, gw), (b, gb))):
            m = b1 * state["m"][k][j] + (1 - b1) * g
            v = b2 * state["v"][k][j] + (1 - b2) * g * g
            state["m"][k] = tuple(m if i == j else state["m"][k][i] for i in range(2))
            state["v"][k] = tuple(v if i == j else state["v"][k][i] for i in range(2))
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out
