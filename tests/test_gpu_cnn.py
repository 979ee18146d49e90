"""Warm-start network kernels on the GPU against the CPU oracle (oracle.cnn).

Both sides use the same bfloat16-rounded weights and inputs; the GPU
accumulates in FP32 on the matrix cores, the oracle in FP64.  They can then
differ where an FP32 sum lands next to a bf16 rounding boundary: that element
flips by one bf16 ulp (2^-8 relative), which happens to a fraction of order
2^-16 of the entries.  Bars: relative L2 1e-3 for the output and 2e-3 for the
gradients (these also carry the flips of the gradients fed between layers).

* forward output on ragged images (W not a multiple of 16, pixel count not a
  multiple of the 64-pixel wave tile);
* loss and parameter gradients with a gathered mini-batch (index array);
* one Adam step against the update rule applied to the GPU gradient;
* a few hundred steps reduce the loss of a learnable synthetic task.
"""
import numpy as np
import pytest

from oracle import cnn as ocnn

from .gpu_common import announce, rel_l2

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu

CH = [14, 32, 32, 32, 18]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


def _flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def _unflat(v, ch):
    out, k = [], 0
    for cin, cout in zip(ch[:-1], ch[1:]):
        w = v[k:k + cout * cin * 9].reshape(cout, cin, 3, 3)
        k += cout * cin * 9
        b = v[k:k + cout]
        k += cout
        out.append((w.astype(np.float64), b.astype(np.float64)))
    return out


def _params(seed, ch=CH):
    rng = np.random.default_rng(seed)
    ps = ocnn.init_params(ch, seed=seed)
    ps = [(w, rng.normal(0, 0.1, b.shape)) for w, b in ps]
    return _unflat(_flat(ps), ch)     # float32-representable


@pytest.mark.parametrize("shape", [(3, 10, 13), (2, 64, 64), (1, 1, 1)])
def test_forward_matches_oracle(ctx, shape):
    B, H, W = shape
    announce(f"cnn forward {B}x{H}x{W}")
    ps = _params(1)
    net = L.smm_cnn_create(ctx, CH, H, W, B)
    L.smm_cnn_set_params(net, _flat(ps))
    assert np.array_equal(L.smm_cnn_get_params(net), _flat(ps))
    x = np.random.default_rng(2).normal(size=(B, H, W, CH[0])).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros((B, H, W, CH[-1]), dtype=torch.float32, device="cuda")
    L.smm_cnn_forward(net, xd, B, yd)
    torch.cuda.synchronize()
    ref, _ = ocnn.forward(ps, x.astype(np.float64))
    assert rel_l2(yd.cpu().numpy(), ref) < 1e-3
    L.smm_cnn_destroy(net)


def test_gradients_and_adam_match_oracle(ctx):
    announce("cnn loss/gradients with gather + one Adam step")
    H, W, B = 12, 19, 3
    ps = _params(3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(5, H, W, CH[0])).astype(np.float32)
    T = rng.normal(size=(5, H, W, CH[-1])).astype(np.float32)
    idx = np.array([4, 0, 2], dtype=np.int32)
    wch = rng.uniform(0.5, 2.0, CH[-1]).astype(np.float32)
    net = L.smm_cnn_create(ctx, CH, H, W, 4)
    L.smm_cnn_set_params(net, _flat(ps))
    loss, g = L.smm_cnn_loss_grad(net, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(),
                                  torch.from_numpy(idx).cuda(), B, wch, want_grad=True)
    y, cache = ocnn.forward(ps, X[idx].astype(np.float64))
    lref, gy = ocnn.loss_mse(y, T[idx].astype(np.float64), wch.astype(np.float64))
    gref = ocnn.backward(ps, cache, gy)
    assert abs(loss - lref) <= 1e-3 * lref
    gr = _flat(gref)
    assert rel_l2(g, gr) < 2e-3
    for k, ((gw, gb), (rw, rb)) in enumerate(zip(_unflat(g, CH), gref)):
        assert rel_l2(gw, rw) < 2e-3, k
        assert rel_l2(gb, rb) < 2e-3, k
    # Adam from the same gradient
    p0 = _flat(ps)
    L.smm_cnn_adam_step(net, 1e-3)
    p1 = L.smm_cnn_get_params(net)
    state = {}
    pexp = ocnn.adam_step(ps, _unflat(g, CH), state, lr=1e-3)
    assert np.max(np.abs(p1 - _flat(pexp))) < 1e-6
    assert np.max(np.abs(p1 - p0)) > 5e-4
    L.smm_cnn_destroy(net)


def test_training_reduces_loss(ctx):
    """Fit the output of a fixed random teacher network: the loss falls."""
    announce("cnn training on a teacher task")
    ch = [6, 16, 16, 4]
    H = W = 16
    n, B = 64, 16
    teacher = _params(5, ch)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(n, H, W, ch[0])).astype(np.float32)
    T, _ = ocnn.forward(teacher, X.astype(np.float64))
    net = L.smm_cnn_create(ctx, ch, H, W, B)
    L.smm_cnn_set_params(net, _flat(_params(7, ch)))
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T.astype(np.float32)).cuda()
    idx = torch.empty(B, dtype=torch.int32, device="cuda")
    losses = []
    for step in range(300):
        idx.copy_(torch.from_numpy(rng.permutation(n)[:B].astype(np.int32)))
        loss, _ = L.smm_cnn_loss_grad(net, Xd, Td, idx, B)
        L.smm_cnn_adam_step(net, 3e-3)
        losses.append(loss)
    assert np.mean(losses[-20:]) < 0.3 * np.mean(losses[:5]), (losses[:5], losses[-5:])
    L.smm_cnn_destroy(net)
