"""Parallel block Jacobi sweep (Sec. 6.5) on the GPU against the oracle.

* One sweep with a lagged input on tiles: FP64 to 1e-12 against the oracle's
  block sweep, straight two-material and curved meshes, ragged tiles.
* Fixed outer iterations with tiles (FP64): the iterates match the oracle's
  block Jacobi SMM iterates to 1e-12.
* Converged (FP64 and FP32 delta sweeps): the fixed point is the one of the
  full sweep (1e-12 / 1e-5 against the oracle's untiled solution), and more
  tiles need more outer iterations.
* Tiles off again gives the full sweep; batches refuse tiled problems.
* Full size (channel 128², p = 2, S12): 32² tiles reach the full sweep's
  fixed point within the FP32 bar.
"""
import numpy as np
import pytest

from oracle import smm as osmm
from oracle import transport as otr
from workloads import config_channel, config_curved_mms, config_plain

from .gpu_common import announce, rel_l2

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


def _pair(ctx, wl, tiles, path=0):
    pr = osmm.make_problem(wl, tiles=tiles)
    iso = isinstance(wl.inflow, tuple) and wl.inflow[0] == "iso"
    p = L.problem_from_workload(ctx, wl, q=pr.q, psibar=None if iso else pr.psibar)
    if tiles is not None:
        L.smm_set_sweep_tiles(p, *tiles)
    L.smm_set_sweep_path(p, path)
    return pr, p


def _two_mat(n=7, p=2, sn=4):
    wl = config_channel(n=n, p=p, sn=sn, side=1.3)
    wl.inflow = ("iso", 0.5)
    return wl


# (workload factory, tiles, sweep path: 0 automatic, i.e. one lane per element
# at p <= 2; 3 one wave per element at every order)
SWEEPS = {
    "twomat7_p2_t3x2": (lambda: _two_mat(), (3, 2), 0),
    "twomat7_p2_t3x2_wavesolve": (lambda: _two_mat(), (3, 2), 3),
    "twomat7_p1_t1x1": (lambda: _two_mat(p=1), (1, 1), 0),
    "plain6_p4_t4x4": (lambda: config_plain(6, 4, 6), (4, 4), 0),
    "curved4_p2_t2x3": (lambda: config_curved_mms(4, 2, 8), (2, 3), 0),
    "curved4_p2_t2x3_wavesolve": (lambda: config_curved_mms(4, 2, 8), (2, 3), 3),
}


@pytest.mark.parametrize("case", list(SWEEPS))
def test_block_sweep_with_lag_fp64(ctx, case):
    factory, tiles, path = SWEEPS[case]
    announce(f"block Jacobi sweep {case}")
    wl = factory()
    pr, p = _pair(ctx, wl, tiles, path)
    rng = np.random.default_rng(4)
    S = rng.uniform(0.5, 1.5, size=(pr.ne, pr.n))
    lag = rng.uniform(0.0, 1.0, size=(len(pr.w), pr.ne, pr.n))
    ref = otr.sweep(pr.mesh, pr.omega, pr.sigma_t, S, pr.psibar, lag, pr.block)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    out = torch.zeros((len(pr.w), pr.ne, pr.n), dtype=torch.float64, device="cuda")
    L.smm_apply_sweep(p, L.SMM_FP64, dev(S), L.SMM_SRC_ISO, dev(lag), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)


@pytest.mark.parametrize("case", ["twomat", "curved"])
def test_block_jacobi_fixed_iterations_fp64(ctx, case):
    K = 5
    announce(f"block Jacobi {K} outer iterations fp64 {case}")
    wl = _two_mat(n=6) if case == "twomat" else config_curved_mms(4, 2, 8)
    pr, p = _pair(ctx, wl, (2, 3))
    ref, _ = osmm.solve(pr, tol=0.0, max_it=K)
    opts = L.smm_default_opts(precision=L.SMM_FP64, outer_tol=0.0, max_outer=K, inner_tol=1e-15,
                              max_inner=5000)
    rc, info = L.smm_solve(p, opts, raise_on_noconv=False)
    assert rc == L.SMM_ENOCONV and info["iterations"] == K
    got = L.smm_get_outputs_host(p)["varphi"]
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)


def test_block_jacobi_converged_same_fixed_point(ctx):
    announce("block Jacobi converged vs full sweep")
    wl = _two_mat(n=8, p=2)
    ref, info_ref = osmm.solve(osmm.make_problem(wl), tol=1e-13, max_it=300)
    its = []
    for tiles in ((8, 8), (4, 4), (2, 2)):
        _, p = _pair(ctx, wl, tiles)
        rc, info = L.smm_solve(p, L.smm_default_opts(precision=L.SMM_FP64, outer_tol=1e-13, inner_tol=1e-15,
                                                     max_inner=5000, max_outer=400))
        assert rc == L.SMM_OK
        assert rel_l2(L.smm_get_outputs_host(p)["varphi"], ref) < 1e-12
        its.append(info["iterations"])
        rc, _ = L.smm_solve(p, L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-9,
                                                  inner_tol=1e-13, max_inner=5000, max_outer=400))
        assert rc == L.SMM_OK
        assert rel_l2(L.smm_get_outputs_host(p)["varphi"], ref) < 1e-5
    assert its == sorted(its) and its[-1] > its[0], its


def test_tiles_off_and_batch_refusal(ctx):
    announce("block Jacobi tiles off / batch refusal")
    wl = _two_mat(n=5, p=1)
    pr, p = _pair(ctx, wl, (2, 2))
    L.smm_set_sweep_tiles(p, 0, 0)
    rng = np.random.default_rng(5)
    S = rng.uniform(0.5, 1.5, size=(pr.ne, pr.n))
    ref = otr.sweep(pr.mesh, pr.omega, pr.sigma_t, S, pr.psibar)
    dev = torch.tensor(S, dtype=torch.float64, device="cuda")
    out = torch.zeros((len(pr.w), pr.ne, pr.n), dtype=torch.float64, device="cuda")
    L.smm_apply_sweep(p, L.SMM_FP64, dev, L.SMM_SRC_ISO, None, out)
    torch.cuda.synchronize()
    assert rel_l2(out.cpu().numpy(), ref) < 1e-12
    L.smm_set_sweep_tiles(p, 2, 2)
    with pytest.raises(L.SmmError) as e:
        L.smm_batch_create(ctx, [p])
    assert e.value.code == L.SMM_EUNSUPPORTED
    with pytest.raises(L.SmmError) as e:
        L.smm_set_sweep_tiles(p, 2, 0)
    assert e.value.code == L.SMM_EINVAL


def test_full_size_tiles_reach_the_untiled_fixed_point(ctx):
    """Full-size channel problem (128 x 128, p = 2, S12, FP32 delta sweeps,
    CG moment system): the tabulated full sweep and the per-element sweep on
    32 x 32 tiles converge to the same fixed point (a property of the block
    Jacobi iteration at any size), within the FP32 bar."""
    announce("channel 128x128 p2 S12: 32x32 tiles vs full sweep, converged")
    wl = config_channel()
    out = []
    for tiles in ((0, 0), (32, 32)):
        p = L.problem_from_workload(ctx, wl)
        if tiles != (0, 0):
            L.smm_set_sweep_tiles(p, *tiles)
        rc, info = L.smm_solve(p, L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-9,
                                                     inner_tol=1e-12, max_inner=20000, max_outer=200,
                                                     discretization=L.SMM_DISC_CG))
        assert rc == L.SMM_OK
        out.append((L.smm_get_outputs_host(p)["varphi"], info["iterations"]))
        L.smm_problem_destroy(p)
    assert rel_l2(out[1][0], out[0][0]) < 1e-5, rel_l2(out[1][0], out[0][0])
    assert out[1][1] > out[0][1]
