"""Pins of the oracle network (no GPU).

* bfloat16 rounding: exact on representable values, ties to even, 8-bit
  mantissa error bound.
* 3x3 convolution: equals a direct loop over the stencil on a tiny case and a
  scipy correlation per channel pair.
* Backward pass: gradients of the unrounded network equal central
  differences in FP64.
* Adam: reproduces the update rule step by step on a scalar.
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.0e38])
    r = cnn.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 + 2 ** -7
    assert r[2] == 1.0                      # tie -> even
    assert r[3] == 1.0 + 2 ** -6            # tie -> even (up)
    assert r[4] == -2.5 and r[5] == 0.0
    y = np.random.default_rng(0).normal(size=1000)
    assert np.max(np.abs(cnn.bf16(y) - y) / np.abs(y)) <= 2 ** -8


def test_conv_matches_correlation():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 5, 6, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = cnn.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, :, :, c], w[o, c], mode="same") for c in range(3))
            assert np.abs(y[n, :, :, o] - ref).max() < 1e-12
    # one point by direct loops
    n, i, j, o = 1, 0, 5, 2
    s = b[o]
    for c in range(3):
        for di in range(3):
            for dj in range(3):
                ii, jj = i + di - 1, j + dj - 1
                if 0 <= ii < 5 and 0 <= jj < 6:
                    s += w[o, c, di, dj] * x[n, ii, jj, c]
    assert abs(y[n, i, j, o] - s) < 1e-12


def test_gradients_central_differences():
    rng = np.random.default_rng(2)
    params = cnn.init_params([3, 5, 4, 2], seed=3)
    params = [(w, rng.normal(size=b.shape) * 0.1) for w, b in params]
    x = rng.normal(size=(2, 6, 5, 3))
    t = rng.normal(size=(2, 6, 5, 2))

    def loss(ps):
        y, _ = cnn.forward(ps, x, emulate_bf16=False)
        return cnn.loss_mse(y, t)[0]

    y, cache = cnn.forward(params, x, emulate_bf16=False)
    _, gy = cnn.loss_mse(y, t)
    grads = cnn.backward(params, cache, gy, emulate_bf16=False)
    h = 1e-6
    for k in range(len(params)):
        for which in (0, 1):
            arr = params[k][which]
            for idx in list(np.ndindex(arr.shape))[:: max(1, arr.size // 7)]:
                def with_delta(dlt):
                    ps = [(w.copy(), b.copy()) for w, b in params]
                    ps[k][which][idx] += dlt
                    return loss(ps)
                fd = (with_delta(h) - with_delta(-h)) / (2 * h)
                an = grads[k][which][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, which, idx, fd, an)


def test_adam_scalar_sequence():
    p = [(np.array([[[[1.0]]]]), np.array([0.5]))]
    state = {}
    gs = [0.3, -0.1, 0.2]
    m = v = 0.0
    w = 1.0
    for t, g in enumerate(gs, 1):
        p = cnn.adam_step(p, [(np.array([[[[g]]]]), np.array([0.0]))], state, lr=0.01)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        w = w - 0.01 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
        assert abs(p[0][0].item() - w) < 1e-15
