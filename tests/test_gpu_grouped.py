"""Type-group PCG kernels, forced on, against the dense matrix and the oracle.

A batch uses the type-group kernels (one wave per group of up to 64 elements
sharing their typed blocks; q = A p, the PCG start r = b - A x, the update
with z = D^-1 r and the IP right-hand side on the FP64 matrix cores) when its
groups are densely filled, as in large homogeneous meshes.  The small batches
of the other tests fall below that fill and run the per-node kernels, so here
both choices are forced on the same batches:
* y = A x against the dense typed matrix of every problem, orders 1-4, one
  and several materials, boundary and interior groups (relative 1e-12);
* whole solves with block-Jacobi and two-level PCG: grouped and per-node
  kernels reach the same converged flux (FP64 1e-11) and the oracle's.
"""
import numpy as np
import pytest

from oracle import smm as osmm
from workloads import config_blobs, config_channel, config_plain

from .gpu_common import announce, make_pair, rel_l2
from .test_gpu_batch import _batch_members, _opts

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


def _spmv_members():
    return _batch_members() + [config_plain(12, p, 4) for p in (1, 2, 3, 4)] + [
        config_blobs(20005, n=10, p=3, sn=4), config_channel(n=9, side=1.3)]


@pytest.mark.parametrize("grouped", [1, 0], ids=["grouped", "per_node"])
def test_spmv_matches_dense(ctx, grouped):
    announce(f"batched q = A p, grouped={grouped}, vs the dense typed matrix")
    wls = _spmv_members()
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    L.smm_debug_batch_grouped(batch, grouped)
    rng = np.random.default_rng(11)
    xs = [rng.normal(size=p.n_elem * p.n_node) for p in probs]
    ys = L.smm_debug_batch_spmv(batch, xs)
    hctx = L.smm_ctx_create(-1)
    for k, (wl, x, y) in enumerate(zip(wls, xs, ys)):
        A, _, _ = L.smm_debug_typed_dense(L.problem_from_workload(hctx, wl))
        assert rel_l2(y, A @ x) < 1e-12, (k, wl.name, rel_l2(y, A @ x))
    L.smm_batch_destroy(batch)


@pytest.mark.parametrize("precond", [0, 1], ids=["block_jacobi", "two_level"])
def test_grouped_solve_matches_per_node_and_oracle(ctx, precond):
    announce(f"batched FP64 solves, grouped vs per-node kernels, precond={precond}")
    wls = _batch_members() + [config_plain(16, 4, 4), config_blobs(20006, n=14, p=2, sn=4)]
    pairs = [make_pair(L, ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, [p for _, p in pairs])
    outs = {}
    for grouped in (1, 0):
        L.smm_debug_batch_grouped(batch, grouped)
        o = _opts(0, 1e-13)
        o.precond = precond
        rc, _ = L.smm_batch_solve(batch, o)
        assert rc == L.SMM_OK, grouped
        outs[grouped] = []
        for k, (_, p) in enumerate(pairs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            outs[grouped].append(v)
    for k, (pr, _) in enumerate(pairs):
        assert rel_l2(outs[1][k], outs[0][k]) < 1e-11, k
        ref, _ = osmm.solve(pr, tol=1e-13, max_it=200)
        assert rel_l2(outs[1][k], ref) < 1e-11, k
    L.smm_batch_destroy(batch)


@pytest.mark.parametrize("use_graph", [1, 0], ids=["graph", "eager"])
def test_forked_pcg_launches_bitwise(ctx, use_graph):
    """The per-order launches of each PCG phase run concurrently on forked
    streams (the default) or one after the other; they touch disjoint
    problems, so the solves agree bit for bit, replayed from graphs or not."""
    announce(f"batched solves, forked vs serial per-order PCG launches, use_graph={use_graph}")
    wls = [config_plain(12, p, 4) for p in (1, 2, 3, 4)] + [config_blobs(20007, n=10, p=3, sn=4),
                                                            config_channel(n=9, side=1.3)]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    L.smm_debug_batch_grouped(batch, 1)
    outs, its = {}, {}
    for fork in (1, 0, 1):
        L.smm_debug_batch_cg_fork(batch, fork)
        o = _opts(L.SMM_FP32_SWEEP, 1e-9)
        o.precond = L.SMM_PRECOND_TWOLEVEL
        o.delta_sweeps = 1
        o.use_graph = use_graph
        o.anderson = 2
        rc, infos = L.smm_batch_solve(batch, o)
        assert rc == L.SMM_OK, fork
        vs = []
        for k, p in enumerate(probs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            vs.append(v)
        key = len(outs)
        outs[key], its[key] = vs, [i["iterations"] for i in infos]
    for k in range(len(probs)):
        assert np.array_equal(outs[0][k], outs[1][k]), k
        assert np.array_equal(outs[0][k], outs[2][k]), k
    assert its[0] == its[1] == its[2]
    L.smm_batch_destroy(batch)


@pytest.mark.parametrize("inner", [(1e-15, 1), (1e-15, 2), (1e-3, 4000)], ids=["one_step", "two_steps", "loose"])
def test_grouped_matches_per_node_with_truncated_inner_solves(ctx, inner):
    """The type-group kernels apply x += alpha p in the direction update (the
    update kernel reads neither x nor p), the per-node kernels in the update:
    after PCG solves stopped by max_inner (one or two iterations) or by a loose
    tolerance (mid-chunk, where the direction update of the converging
    iteration still owes x its last step) both give the same iterate up to
    summation order.  A missing or repeated alpha p would differ at the size
    of the step itself."""
    inner_tol, max_inner = inner
    announce(f"grouped vs per-node kernels, 3 outer iterations, inner_tol {inner_tol}, max_inner {max_inner}")
    wls = _batch_members() + [config_plain(16, 4, 4), config_blobs(20006, n=14, p=2, sn=4)]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    outs = {}
    for grouped in (1, 0):
        L.smm_debug_batch_grouped(batch, grouped)
        o = L.smm_default_opts(precision=L.SMM_FP64, outer_tol=0.0, max_outer=3, inner_tol=inner_tol,
                               max_inner=max_inner, precond=L.SMM_PRECOND_TWOLEVEL)
        rc, infos = L.smm_batch_solve(batch, o, raise_on_noconv=False)
        assert rc in (L.SMM_OK, L.SMM_ENOCONV), grouped
        assert all(i["iterations"] == 3 for i in infos), grouped
        outs[grouped] = []
        for k, p in enumerate(probs):
            v = np.zeros(p.n_elem * p.n_node)
            L.smm_batch_get_outputs(batch, k, varphi=v)
            outs[grouped].append(v)
    for k in range(len(probs)):
        assert np.all(np.isfinite(outs[1][k]))
        assert rel_l2(outs[1][k], outs[0][k]) < 1e-10, (k, rel_l2(outs[1][k], outs[0][k]))
    L.smm_batch_destroy(batch)
