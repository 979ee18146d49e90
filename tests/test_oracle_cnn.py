"""Pins of the oracle network (no GPU).

* bfloat16 rounding: exact on representable values, ties to even, 8-bit
  mantissa error bound.
* 3x3 convolution: equals a direct loop over the stencil on a tiny case and a
  scipy correlation per channel pair.
* Backward pass: gradients of the unrounded network equal central
  differences in FP64.
* Rounded network: the bf16 forward pass and gradients stay within the
  bf16 error bound of the exact (central-difference-pinned) ones.
* Adam, by properties of the method (Kingma and Ba, 2015, Sec. 2-3) rather
  than by its formula: with a constant gradient the bias-corrected moments
  are exact, so every step is lr * g / (|g| + eps); steps do not change when
  all gradients are scaled (eps = 0); with gradients of alternating sign the
  step tends to lr (1 - beta1) / (1 + beta1), the limit of the first moment's
  geometric series; and it minimises a quadratic.
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


def test_rounded_network_within_bf16_bound():
    rng = np.random.default_rng(5)
    params = cnn.init_params([4, 8, 8, 3], seed=6)
    params = [(w, rng.normal(size=b.shape) * 0.1) for w, b in params]
    x = rng.normal(size=(2, 7, 6, 4))
    t = rng.normal(size=(2, 7, 6, 3))
    ye, ce = cnn.forward(params, x, emulate_bf16=False)
    yr, cr = cnn.forward(params, x, emulate_bf16=True)
    # one rounding of each input, weight and hidden activation: a few units of
    # 2^-8 relative to the magnitude of the sums, per layer
    scale = np.abs(ye).max()
    assert 0 < np.abs(yr - ye).max() < 3 * len(params) * 2.0 ** -8 * scale
    _, ge_y = cnn.loss_mse(ye, t)
    _, gr_y = cnn.loss_mse(yr, t)
    ge = cnn.backward(params, ce, ge_y, emulate_bf16=False)
    gr = cnn.backward(params, cr, gr_y, emulate_bf16=True)
    for (gw_e, gb_e), (gw_r, gb_r) in zip(ge, gr):
        # ReLU masks may flip at activations within rounding of zero: compare in norm
        assert np.linalg.norm(gw_r - gw_e) < 0.05 * np.linalg.norm(gw_e)
        assert np.linalg.norm(gb_r - gb_e) < 0.05 * np.linalg.norm(gb_e)


def _adam_run(gs, lr=0.01, eps=1e-8, w0=1.0):
    p = [(np.array([[[[w0]]]]), np.array([0.0]))]
    state, out = {}, [w0]
    for g in gs:
        p = cnn.adam_step(p, [(np.array([[[[g]]]]), np.array([g]))], state, lr=lr, eps=eps)
        out.append(p[0][0].item())
    return np.array(out)


def test_adam_constant_gradient_steps():
    for g in (0.3, -2.0, 1e-3):
        w = _adam_run([g] * 6, lr=0.01)
        assert np.allclose(np.diff(w), -0.01 * g / (abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_scale_invariance():
    gs = list(np.random.default_rng(7).normal(size=12))
    a = _adam_run(gs, eps=0.0)
    b = _adam_run([37.0 * g for g in gs], eps=0.0)
    assert np.abs(a - b).max() < 1e-14


def test_adam_alternating_gradient_limit():
    gs = [0.5 * (-1) ** k for k in range(400)]
    w = _adam_run(gs, lr=0.01)
    step = np.abs(np.diff(w))[-1]
    assert abs(step - 0.01 * 0.1 / 1.9) < 1e-9


def test_adam_minimises_quadratic():
    p = [(np.array([[[[0.0]]]]), np.array([0.0]))]
    state = {}
    for _ in range(3000):
        w = p[0][0].item()
        p = cnn.adam_step(p, [(np.array([[[[w - 3.0]]]]), np.array([0.0]))], state, lr=0.05)
    assert abs(p[0][0].item() - 3.0) < 1e-3


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
