"""The full 256-problem batch in the configuration bench.py times, and a
degenerate case, against the oracle.

* The batch of seeds 0..255 (16^2..128^2, p = 1..4, S4..S12) solved to a
  1e-8 outer residual with FP32 delta sweeps, two-level PCG, Anderson mixing
  and graph-replayed PCG chunks: every problem converges to finite values,
  and three members the oracle can solve in seconds (seeds 133, 196, 10:
  17^2 p = 1 S4, 16^2 p = 2 S6, 19^2 p = 3 S4), solved inside that batch,
  match the oracle's converged flux to the FP32 bar (1e-5 relative L2).
* The batched sweep kernel, in the launch configuration of that batch (the
  per-order persistent launches whose anti-diagonals span several 64-slot
  chunks), on seeded sources: sampled directions of members 9 (93^2 p = 4
  S6), 12 (81^2 p = 4), 0 (115^2 p = 2), 19 (99^2 p = 1) and 23 (118^2 p = 3)
  against the oracle's sweep, FP64 to 1e-12 and FP32 to 1e-5 relative L2;
  and the two-material 128^2 channel problem (the several-materials path of
  that kernel) likewise.
* The full-size channel problem: FP32 sweeps within 1e-5 of the all-FP64
  solve.
* No scattering (sigma_s = 0): G does not depend on X, so the second outer
  iterate equals the first (up to the rounding of the second moment solve),
  and the transport scalar flux is one sweep of q.
"""
import numpy as np
import pytest

from oracle import smm as osmm
from oracle import transport
from workloads import config_batched_problem, config_channel

from .gpu_common import announce, rel_l2

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


def test_full_batch_sampled_members(ctx):
    announce("full 256-problem batch, FP32 delta sweeps, two-level PCG, Anderson, graphs; sampled members")
    wls = [config_batched_problem(s) for s in range(256)]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    opts = L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-8, inner_tol=1e-10,
                              inner_adapt=1e-2, max_inner=20000, max_outer=80, precond=L.SMM_PRECOND_TWOLEVEL,
                              use_graph=1, anderson=2)
    rc, infos = L.smm_batch_solve(batch, opts)
    assert rc == L.SMM_OK and all(i["residual"] < 1e-8 for i in infos)
    for k in range(256):
        v = np.zeros(probs[k].n_elem * probs[k].n_node)
        L.smm_batch_get_outputs(batch, k, varphi=v)
        assert np.all(np.isfinite(v)) and v.max() > 0, k
    for s in (133, 196, 10):
        ref, info = osmm.solve(osmm.make_problem(wls[s]), tol=1e-11, max_it=100)
        assert info["converged"]
        v = np.zeros(probs[s].n_elem * probs[s].n_node)
        L.smm_batch_get_outputs(batch, s, varphi=v)
        assert rel_l2(v, ref) < 1e-5, (s, rel_l2(v, ref))
    L.smm_batch_destroy(batch)


def _batched_sweep_vs_oracle(ctx, wls, members, dirs_per_member, seed):
    """Every kernel shape of the batched sweep (and the autotuned choice) in
    the batch's launch configuration, against the oracle's sweep.  The two
    VALU shapes apply each element's operator rows in the same order and
    agree bit for bit; so do the two matrix-core shapes (FP32 only: forcing
    them leaves FP64 sweeps on the tuned VALU shape), whose sums run in
    another order; the autotuned result equals one of them."""
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    rng = np.random.default_rng(seed)
    srcs = [None] * len(wls)
    for k in members:
        srcs[k] = rng.uniform(0.5, 1.5, size=probs[k].n_elem * probs[k].n_node)
    worst = {}
    for k in members:
        pr = osmm.make_problem(wls[k])
        nd = len(pr.w)
        dirs = sorted({(nd * j) // dirs_per_member for j in range(dirs_per_member)} | {nd - 1})
        ref = transport.sweep(pr.mesh, pr.omega[dirs], pr.sigma_t, srcs[k].reshape(pr.ne, pr.n), pr.psibar)
        for prec, bar in ((L.SMM_FP64, 1e-12), (L.SMM_FP32_SWEEP, 1e-5)):
            got = {}
            for shape in (0, 1, 2, 3, -1):
                announce(f"batched sweep member {k} ({wls[k].nx}^2 p={wls[k].p} S{wls[k].sn}) precision {prec} "
                         f"shape {shape}")
                L.smm_debug_batch_sweep_shape(batch, shape)
                psi = L.smm_batch_apply_sweep(batch, prec, srcs, k)
                assert np.all(np.isfinite(psi))
                got[shape] = psi
                for j, d in enumerate(dirs):
                    e = rel_l2(psi[d], ref[j])
                    worst[(k, prec, shape)] = max(worst.get((k, prec, shape), 0.0), e)
                    assert e < bar, (k, prec, shape, d, e)
            assert np.array_equal(got[0], got[1]) and np.array_equal(got[2], got[3])
            if prec == L.SMM_FP64:
                assert np.array_equal(got[0], got[2])
            assert np.array_equal(got[-1], got[0]) or np.array_equal(got[-1], got[2])
    L.smm_batch_destroy(batch)
    return worst


def test_bench_batch_sweep_full_width_vs_oracle(ctx):
    announce("full 256-problem batch: batched sweep kernel vs oracle on sampled members and directions")
    wls = [config_batched_problem(s) for s in range(256)]
    worst = _batched_sweep_vs_oracle(ctx, wls, (9, 12, 0, 19, 23), 4, 2024)
    print("worst rel L2 per (member, precision):", worst, flush=True)


def test_channel_batched_sweep_vs_oracle(ctx):
    announce("channel 128^2 p=2 S12 (two materials) as a batch: batched sweep vs oracle")
    worst = _batched_sweep_vs_oracle(ctx, [config_channel()], (0,), 4, 77)
    print("worst rel L2 per (member, precision):", worst, flush=True)


def test_no_scattering_two_iterations(ctx):
    announce("sigma_s = 0: two outer iterations, phi = one sweep of q")
    wl = config_channel(n=8, p=2, sn=4, side=1.3)
    wl.sigma_s = np.zeros(wl.n_elem)
    pr = osmm.make_problem(wl)
    p = L.problem_from_workload(ctx, wl, q=pr.q)
    rc, info = L.smm_solve(p, L.smm_default_opts(precision=L.SMM_FP64, outer_tol=1e-12, inner_tol=1e-15,
                                                  max_inner=5000))
    # the second moment solve starts from the first's answer: the change is
    # rounding only (well below the 1e-12 outer tolerance)
    assert rc == L.SMM_OK and info["iterations"] == 2 and info["residual"] < 1e-13
    out = L.smm_get_outputs_host(p)
    psi = transport.sweep(pr.mesh, pr.omega, pr.sigma_t, pr.q, pr.psibar)
    phi = np.einsum("d,dkn->kn", pr.w, psi).ravel()
    assert rel_l2(out["phi"], phi) < 1e-12
    ref, _ = osmm.solve(pr, tol=1e-14, max_it=5)
    assert rel_l2(out["varphi"], ref) < 1e-12


@pytest.mark.parametrize("path,outer_tol", [("typed", 1e-3), ("per_element", 1e-3), ("cg", 1e-3),
                                            ("typed", 0.5), ("per_element", 0.5)])
def test_capped_inner_solve_never_converges(ctx, path, outer_tol):
    """Moment solves stopped by max_inner (one PCG iteration each) do not
    count as converged outer iterations: the solve ends with SMM_ENOCONV and
    valid outputs, whatever the outer change -- also when the last outer
    change is below a loose outer tolerance (the status comes from the
    per-problem convergence flag, not from the last residual)."""
    announce(f"capped inner solves ({path}, outer_tol {outer_tol}) -> SMM_ENOCONV")
    wl = config_channel(n=6, p=2, sn=4, side=1.3)
    pr = osmm.make_problem(wl)
    p = L.problem_from_workload(ctx, wl, q=pr.q)
    kw = {"typed": {}, "per_element": dict(moment_path=1), "cg": dict(discretization=L.SMM_DISC_CG)}[path]
    opts = L.smm_default_opts(precision=L.SMM_FP64, outer_tol=outer_tol, inner_tol=1e-12, max_inner=1,
                              max_outer=12, **kw)
    rc, info = L.smm_solve(p, opts, raise_on_noconv=False)
    assert rc == L.SMM_ENOCONV and info["iterations"] == 12
    assert np.all(np.isfinite(L.smm_get_outputs_host(p)["varphi"]))


def test_full_size_fp32_sweep_within_the_fp32_bar(ctx):
    """Full-size channel problem (128 x 128, p = 2, S12), converged: FP32
    delta sweeps with FP64 moments, PCG and residual against the all-FP64
    solve (whose kernels match the oracle at the sizes it can check), within
    1e-5 relative L2."""
    announce("channel 128x128 p2 S12: FP32 sweeps vs FP64, converged")
    wl = config_channel()
    out = []
    for prec, delta in ((L.SMM_FP64, 0), (L.SMM_FP32_SWEEP, 1)):
        p = L.problem_from_workload(ctx, wl)
        rc, _ = L.smm_solve(p, L.smm_default_opts(precision=prec, delta_sweeps=delta, outer_tol=1e-10,
                                                  inner_tol=1e-13, max_inner=20000, max_outer=200,
                                                  precond=L.SMM_PRECOND_TWOLEVEL))
        assert rc == L.SMM_OK
        out.append(L.smm_get_outputs_host(p)["varphi"])
        L.smm_problem_destroy(p)
    assert rel_l2(out[1], out[0]) < 1e-5, rel_l2(out[1], out[0])
