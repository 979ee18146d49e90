"""Learned warm start of batched solves on the GPU.

* Features (from the diffusion start) and targets (from the converged solve)
  of small blob layouts equal the same quantities computed from the oracle's
  diffusion start, converged solution and last right-hand side (FP64).
* With any network, the learned start converges to the answer of the zero
  start (the start does not change the fixed point); a network whose output
  overflows falls back to the diffusion start for every problem.
* With the trained weights, held-out layouts need fewer outer iterations
  than the zero start (the plain method) and the diffusion start, at an
  unchanged converged answer.
"""
import os

import numpy as np
import pytest

from oracle import smm as osmm
from workloads import config_blobs

from .gpu_common import announce, make_pair, rel_l2

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")
from paper_2304_07386_amd import warmstart as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


def _opts(tol, start, prec=0):
    o = L.smm_default_opts(precision=prec, outer_tol=tol, max_outer=200, inner_tol=1e-14 if prec == 0 else 1e-10,
                           max_inner=20000, delta_sweeps=0 if prec == 0 else 1)
    o.start = start
    return o


def _oracle_features(pr, wl, vD):
    ne, n = pr.ne, pr.n
    nx = wl.nx
    h = 1.0 / nx
    v = vD.reshape(ne, n)
    s = np.maximum(np.abs(v).mean(axis=1), 1e-300)
    ls = np.log10(s)
    F = np.zeros((ne, 5 + n))
    for K in range(ne):
        ex, ey = K % nx, K // nx
        F[K, 0] = np.log10(wl.sigma_t[K])
        F[K, 1] = wl.sigma_s[K] / wl.sigma_t[K]
        F[K, 2] = pr.q[K].mean()
        F[K, 3] = min((ex + 0.5) * h, (nx - ex - 0.5) * h, (ey + 0.5) * h, (wl.ny - ey - 0.5) * h)
    F[:, 4] = ls - ls.mean()
    F[:, 5:] = v / s[:, None] - 1.0
    return F, s


def test_features_and_targets_match_oracle(ctx):
    announce("warm-start features/targets, 2 blob layouts 6x6 p=2 S4, fp64")
    wls = [config_blobs(20000 + k, n=6, p=2, sn=4) for k in range(2)]
    pairs = [make_pair(L, ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, [p for _, p in pairs])
    nf, nt, ny, nx = L.smm_batch_warmstart_dims(batch)
    assert (nf, nt, ny, nx) == (14, 18, 6, 6)
    L.smm_batch_diffusion(batch, 1e-14, 5000)
    X = torch.zeros((2, ny, nx, nf), dtype=torch.float32, device="cuda")
    Tt = torch.zeros((2, ny, nx, nt), dtype=torch.float32, device="cuda")
    L.smm_batch_warmstart_features(batch, 0, 2, X)
    rc, _ = L.smm_batch_solve(batch, _opts(1e-13, L.SMM_START_ZERO))
    assert rc == L.SMM_OK
    L.smm_batch_warmstart_targets(batch, 0, 2, Tt)
    for k, ((pr, _), wl) in enumerate(zip(pairs, wls)):
        vD = osmm.diffusion_start(pr)
        F, s = _oracle_features(pr, wl, vD)
        got = X[k].reshape(-1, nf).cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - F)) < 1e-5 * max(1.0, np.abs(F).max()), k
        ref, info = osmm.solve(pr, tol=1e-13, max_it=200)
        bfix = osmm.rhs_fixed(pr)
        n = pr.n
        t1 = (ref.reshape(-1, n) - vD.reshape(-1, n)) / s[:, None]
        t2 = (info["b"].reshape(-1, n) - bfix.reshape(-1, n)) / ((1.0 / wl.nx) ** 2 * s[:, None])
        gt = Tt[k].reshape(-1, nt).cpu().numpy().astype(np.float64)
        assert rel_l2(gt[:, :n], t1) < 1e-6, k
        assert rel_l2(gt[:, n:], t2) < 1e-6, k
    L.smm_batch_destroy(batch)


def _small_batch(ctx, seeds, n=8):
    wls = [config_blobs(s, n=n, p=2, sn=4) for s in seeds]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    return probs, L.smm_batch_create(ctx, probs)


def test_learned_start_reaches_the_same_fixed_point(ctx):
    announce("learned start with an untrained network and an overflowing one, fp64")
    probs, batch = _small_batch(ctx, [20010, 20011, 20012])
    nf, nt, ny, nx = L.smm_batch_warmstart_dims(batch)
    rc, _ = L.smm_batch_solve(batch, _opts(1e-12, L.SMM_START_ZERO))
    ref = []
    for k, p in enumerate(probs):
        v = np.zeros(p.n_elem * p.n_node)
        L.smm_batch_get_outputs(batch, k, varphi=v)
        ref.append(v)
    ch = [nf, 32, 32, 32, nt]
    for scale, expect in ((0.05, 3), (1e30, 0)):
        net = L.smm_cnn_create(ctx, ch, ny, nx, 2)
        L.smm_cnn_set_params(net, W.he_init(ch, 3) * np.float32(scale))
        L.smm_batch_set_warmstart(batch, net)
        rc, infos = L.smm_batch_solve(batch, _opts(1e-12, L.SMM_START_LEARNED))
        assert rc == L.SMM_OK
        used = L.smm_batch_warmstart_used(batch)
        assert set(used.tolist()) <= {0, 1}
        if expect is not None:
            assert used.sum() == expect
        for k, p in enumerate(probs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            assert rel_l2(v, ref[k]) < 1e-10, (scale, k)
        L.smm_batch_set_warmstart(batch, None)
        L.smm_cnn_destroy(net)
    L.smm_batch_destroy(batch)


@pytest.mark.skipif(not os.path.exists(W.DEFAULT_WEIGHTS), reason="trained weights not present")
def test_trained_network_saves_outer_iterations(ctx):
    """Held-out layouts (64x64, p=2, S8): the learned start needs fewer outer
    iterations than the diffusion start, which needs fewer than zero."""
    announce("trained warm start on 24 held-out blob layouts, fp32 sweeps")
    seeds = list(range(20000, 20024))
    wls = [config_blobs(s) for s in seeds]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    net, meta = W.load(ctx, max_batch=24)
    L.smm_batch_set_warmstart(batch, net)
    its, sols = {}, {}
    for name, start in (("zero", L.SMM_START_ZERO), ("diffusion", L.SMM_START_DIFFUSION),
                        ("learned", L.SMM_START_LEARNED)):
        rc, infos = L.smm_batch_solve(batch, _opts(1e-8, start, prec=1))
        assert rc == L.SMM_OK, name
        its[name] = np.array([i["iterations"] for i in infos])
        sols[name] = []
        for k, p in enumerate(probs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            sols[name].append(v)
    print("outer iterations", {k: float(v.mean()) for k, v in its.items()})
    assert its["learned"].mean() < its["diffusion"].mean() < its["zero"].mean()
    assert L.smm_batch_warmstart_used(batch).sum() == len(seeds)
    for k in range(len(probs)):
        assert rel_l2(sols["learned"][k], sols["zero"][k]) < 1e-6
    L.smm_batch_destroy(batch)
    L.smm_cnn_destroy(net)
