"""Typed Cartesian path and batched solves on the GPU, against the oracle.

* A single Cartesian problem solved through the typed (batched) kernels
  matches the oracle iterate by iterate (K fixed outer iterations) and at
  convergence in FP64 (1e-12), and the per-element path (1e-12).
* A batch of problems with different sizes, orders, S_N sets and materials
  gives, for every problem, bitwise the result of solving that problem alone
  with the same kernels, and matches the oracle (FP64 1e-12, FP32 1e-5).
* Problems converge independently: each stops at its own iteration count.
"""
import numpy as np
import pytest

from oracle import smm as osmm
from workloads import Workload, config_blobs, config_channel, config_plain, structured_ctrl

from .gpu_common import announce, make_pair, rel_l2

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


def _rect(nx, ny, p, sn, nmat, inflow=None, seed=0, c=0.6):
    xv = np.linspace(0.0, 1.3, nx + 1)
    yv = np.linspace(0.0, 0.7, ny + 1)
    rng = np.random.default_rng(seed)
    st = rng.choice([0.4, 3.0, 25.0][:nmat], size=nx * ny)
    wl = Workload("rect", nx, ny, 1, p, sn, structured_ctrl(xv, yv, 1), st, c * st,
                  q_elem=rng.uniform(0.1, 1.0, nx * ny))
    if inflow is not None:
        wl.inflow = ("iso", inflow)
    return wl


def _opts(prec, tol, K=200, path=0, delta=0):
    return L.smm_default_opts(precision=prec, outer_tol=tol, max_outer=K, inner_tol=1e-15 if prec == 0 else 1e-13,
                              max_inner=4000, moment_path=path, delta_sweeps=delta)


def test_typed_fixed_iterations_and_converged(ctx):
    announce("typed path: plain 8x8 p1 S4, 4 fixed iterations and converged, fp64")
    wl = config_plain()
    pr, p = make_pair(L, ctx, wl)
    ref4, _ = osmm.solve(pr, tol=0.0, max_it=4)
    rc, info = L.smm_solve(p, _opts(0, 0.0, K=4), raise_on_noconv=False)
    assert rc == L.SMM_ENOCONV and info["iterations"] == 4
    assert rel_l2(L.smm_get_outputs_host(p)["varphi"], ref4) < 1e-12
    ref, oinfo = osmm.solve(pr, tol=1e-13, max_it=100)
    rc, info = L.smm_solve(p, _opts(0, 1e-13))
    out = L.smm_get_outputs_host(p)
    assert rc == L.SMM_OK and abs(info["iterations"] - oinfo["iterations"]) <= 1
    assert rel_l2(out["varphi"], ref) < 1e-12
    assert rel_l2(out["phi"], oinfo["phi"].ravel()) < 1e-11
    assert rel_l2(out["T"], oinfo["T"].reshape(3, -1)) < 1e-10
    assert rel_l2(out["beta"], oinfo["beta"]) < 1e-10
    # the per-element path gives the same answer
    rc, _ = L.smm_solve(p, _opts(0, 1e-13, path=1))
    assert rel_l2(L.smm_get_outputs_host(p)["varphi"], ref) < 1e-12


def _batch_members():
    return [
        _rect(6, 5, 1, 4, 1, seed=1),
        _rect(5, 7, 2, 6, 2, inflow=0.5, seed=2),
        _rect(4, 4, 3, 8, 3, seed=3, c=0.9),
        _rect(3, 5, 4, 4, 2, seed=4, c=0.3),
        config_plain(8, 2, 12),
    ]


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_matches_single_and_oracle(ctx, prec):
    announce(f"batch of 5 mixed problems, precision {prec}")
    wls = _batch_members()
    pairs = [make_pair(L, ctx, wl) for wl in wls]
    probs = [p for _, p in pairs]
    tol = 1e-13 if prec == 0 else 1e-8
    batch = L.smm_batch_create(ctx, probs)
    rc, infos = L.smm_batch_solve(batch, _opts(prec, tol, delta=prec))
    assert rc == L.SMM_OK
    its = [i["iterations"] for i in infos]
    for k, (pr, p) in enumerate(pairs):
        got = np.zeros(p.n_elem * p.n_node)
        L.smm_batch_get_outputs(batch, k, varphi=got)
        ref, _ = osmm.solve(pr, tol=1e-13, max_it=200)
        bar = 1e-12 if prec == 0 else 1e-5
        assert rel_l2(got, ref) < bar, (k, rel_l2(got, ref))
        # the same problem alone (batch of one) is bitwise identical
        rc1, info1 = L.smm_solve(p, _opts(prec, tol, delta=prec))
        alone = L.smm_get_outputs_host(p)["varphi"]
        assert info1["iterations"] == its[k]
        assert np.array_equal(alone, got), k
    assert len(set(its)) > 1, "problems should converge at different iterations"
    L.smm_batch_destroy(batch)


def test_batch_given_start_is_resume(ctx):
    """Starting from a converged varphi (the warm-start / resume interface)
    converges in one or two iterations to the same answer."""
    announce("batch resume from converged start")
    wls = [config_channel(n=16, side=1.25), config_blobs(20003, n=16)]
    pairs = [make_pair(L, ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, [p for _, p in pairs])
    rc, infos = L.smm_batch_solve(batch, _opts(0, 1e-12))
    sols = []
    for k, (_, p) in enumerate(pairs):
        v = np.zeros(p.n_elem * p.n_node)
        L.smm_batch_get_outputs(batch, k, varphi=v)
        sols.append(v)
    o = _opts(0, 1e-12)
    o.start = L.SMM_START_GIVEN
    rc, infos2 = L.smm_batch_solve(batch, o, varphi0=sols)
    assert rc == L.SMM_OK
    for k, (_, p) in enumerate(pairs):
        assert infos2[k]["iterations"] <= 2 < infos[k]["iterations"]
        v = np.zeros(p.n_elem * p.n_node)
        L.smm_batch_get_outputs(batch, k, varphi=v)
        assert rel_l2(v, sols[k]) < 1e-11
    L.smm_batch_destroy(batch)


def test_graph_replay_is_bitwise_eager(ctx):
    """PCG chunks replayed from captured hipGraphs (use_graph = 1), and whole
    outer iterations replayed from captured graphs (use_graph = 2: source,
    forked sweep launches, moments, closures, right-hand side, PCG start and a
    chunk of PCG iterations, residual), give bitwise the eager results, on
    repeated solves (several replays of each graph, with eager work and
    synchronisations between them)."""
    announce("batch: PCG graph replay vs eager, fp64 and fp32")
    wls = _batch_members()
    probs = [make_pair(L, ctx, wl)[1] for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    for prec, tol in ((0, 1e-12), (1, 1e-8)):
        ref = None
        for use_graph in (0, 1, 2, 2, 0, 1, 2):
            o = _opts(prec, tol, delta=prec)
            o.use_graph = use_graph
            rc, infos = L.smm_batch_solve(batch, o)
            assert rc == L.SMM_OK
            outs = []
            for k, p in enumerate(probs):
                v = np.zeros(p.n_elem * p.n_node)
                L.smm_batch_get_outputs(batch, k, varphi=v)
                outs.append(v)
            its = [(i["iterations"], i["cg_iterations_total"]) for i in infos]
            if ref is None:
                ref = (outs, its)
            else:
                assert its == ref[1]
                for a, b in zip(outs, ref[0]):
                    assert np.array_equal(a, b)
    L.smm_batch_destroy(batch)


def test_adaptive_inner_tolerance(ctx):
    """Inexact moment solves (tolerance tied to the last outer residual) reach
    the same converged answer with fewer PCG iterations."""
    announce("batch: adaptive inner tolerance, fp64")
    wls = _batch_members()
    pairs = [make_pair(L, ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, [p for _, p in pairs])
    rc, tight = L.smm_batch_solve(batch, _opts(0, 1e-12))
    ref = []
    for k, (_, p) in enumerate(pairs):
        v = np.zeros(p.n_elem * p.n_node)
        L.smm_batch_get_outputs(batch, k, varphi=v)
        ref.append(v)
    o = _opts(0, 1e-12)
    o.inner_adapt = 1e-2
    rc, loose = L.smm_batch_solve(batch, o)
    assert rc == L.SMM_OK
    for k, (pr, p) in enumerate(pairs):
        v = np.zeros(p.n_elem * p.n_node)
        L.smm_batch_get_outputs(batch, k, varphi=v)
        assert rel_l2(v, ref[k]) < 1e-10, k
    assert sum(i["cg_iterations_total"] for i in loose) < sum(i["cg_iterations_total"] for i in tight)
    L.smm_batch_destroy(batch)


@pytest.mark.parametrize("prec", [0, 1])
def test_two_level_preconditioner(ctx, prec):
    """The two-level preconditioner (block-Jacobi + Q1 vertex multigrid) gives
    the same converged answers as block-Jacobi and the oracle, with fewer PCG
    iterations; graph replay of its chunks is bitwise the eager result."""
    announce(f"batch: two-level preconditioner, precision {prec}")
    wls = _batch_members() + [config_blobs(20004, n=24), config_channel(n=24, side=1.9)]
    pairs = [make_pair(L, ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, [p for _, p in pairs])
    tol = 1e-13 if prec == 0 else 1e-8
    outs, cgs = {}, {}
    for name, pc, graph in (("bj", 0, 0), ("mg", 1, 0), ("mg_graph", 1, 1), ("mg_itgraph", 1, 2)):
        o = _opts(prec, tol, delta=prec)
        o.precond = pc
        o.use_graph = graph
        rc, infos = L.smm_batch_solve(batch, o)
        assert rc == L.SMM_OK, name
        cgs[name] = sum(i["cg_iterations_total"] for i in infos)
        outs[name] = []
        for k, (_, p) in enumerate(pairs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            outs[name].append(v)
    print("PCG iterations", cgs)
    assert cgs["mg"] < cgs["bj"]
    for k, (pr, p) in enumerate(pairs):
        assert np.array_equal(outs["mg"][k], outs["mg_graph"][k]), k
        assert np.array_equal(outs["mg"][k], outs["mg_itgraph"][k]), k
        if prec == 0:
            assert rel_l2(outs["mg"][k], outs["bj"][k]) < 1e-11, k
        ref, _ = osmm.solve(pr, tol=1e-13, max_it=200)
        assert rel_l2(outs["mg"][k], ref) < (1e-11 if prec == 0 else 1e-5), k
    L.smm_batch_destroy(batch)


@pytest.mark.parametrize("prec", [0, 1])
def test_anderson_mixing(ctx, prec):
    """Anderson mixing of the outer fixed point reaches the same converged
    answers (oracle parity) in fewer outer iterations."""
    announce(f"batch: Anderson mixing, precision {prec}")
    wls = _batch_members() + [config_blobs(20005, n=20), config_channel(n=20, side=1.6)]
    pairs = [make_pair(L, ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, [p for _, p in pairs])
    tol = 1e-12 if prec == 0 else 1e-8
    its, outs = {}, {}
    for depth in (0, 1, 2):
        o = _opts(prec, tol, delta=prec)
        o.precond = L.SMM_PRECOND_TWOLEVEL
        o.anderson = depth
        rc, infos = L.smm_batch_solve(batch, o)
        assert rc == L.SMM_OK, depth
        its[depth] = sum(i["iterations"] for i in infos)
        outs[depth] = []
        for k, (_, p) in enumerate(pairs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            outs[depth].append(v)
    print("outer iterations by Anderson depth", its)
    assert its[2] < its[0] and its[1] < its[0]
    for k, (pr, _) in enumerate(pairs):
        ref, _ = osmm.solve(pr, tol=1e-13, max_it=200)
        for depth in (1, 2):
            assert rel_l2(outs[depth][k], ref) < (1e-10 if prec == 0 else 1e-5), (depth, k)
    L.smm_batch_destroy(batch)


def test_outer_iteration_graph_bench_options(ctx):
    """The options of the benchmark (FP32 delta sweeps, two-level PCG with
    per-problem adaptive tolerances, Anderson mixing of depth 2) on a mixed
    batch: the outer iteration replayed from graphs equals the eager solve bit
    for bit, in iteration counts and fluxes, on two solves in a row."""
    announce("batch: whole-iteration graphs vs eager, bench options")
    wls = _batch_members()
    probs = [make_pair(L, ctx, wl)[1] for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    ref = None
    for use_graph in (0, 2, 2, 1):
        o = L.smm_default_opts(precision=1, delta_sweeps=1, outer_tol=1e-8, inner_tol=1e-10, inner_adapt=1e-2,
                               max_inner=20000, max_outer=100, precond=L.SMM_PRECOND_TWOLEVEL, anderson=2,
                               use_graph=use_graph)
        rc, infos = L.smm_batch_solve(batch, o)
        assert rc == L.SMM_OK
        outs = []
        for k, p in enumerate(probs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            outs.append(v)
        its = [(i["iterations"], i["cg_iterations_total"]) for i in infos]
        if ref is None:
            ref = (outs, its)
        else:
            assert its == ref[1], (use_graph, its, ref[1])
            for a, b in zip(outs, ref[0]):
                assert np.array_equal(a, b)
    L.smm_batch_destroy(batch)
