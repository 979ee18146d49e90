"""The curved manufactured problem end to end on the GPU (Sec. 6.1): 32 x 32
elements, order-p map (m = p), the sine displacement of the interior control
points, S8, sigma_t = 1, sigma_s = 0.5, p = 2, 3, 4.

* Three fixed FP64 outer iterations from the zero start (moment solves to
  1e-14) against the oracle's three iterations: iterate by iterate within
  1e-12 relative L2 (lagged curved-face couplings included: both sides read
  the previous sweep).
* Converged (outer 1e-10): the FP32-sweep flux (delta sweeps, FP64 moments,
  PCG and residual) within 1e-5 of the FP64 flux; both report their error
  against the exact scalar flux of the manufactured solution.
* Converged FP64 solves on 8^2, 16^2, 32^2: || varphi - phi_ex ||_L2 falls as
  h^{p+1} (observed order >= p + 1 - 0.15 on the last refinement).
"""
import numpy as np
import pytest

from oracle import fem
from oracle import smm as osmm
from workloads import config_curved_mms, mms_phi

from .gpu_common import announce, make_pair, rel_l2

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


@pytest.mark.parametrize("p", [2, 3, 4])
def test_c2_fixed_iterations_fp64(ctx, p):
    announce(f"C2 curved 32^2 p={p} S8: 3 fixed FP64 outer iterations vs oracle")
    pr, gp = make_pair(L, ctx, config_curved_mms(32, p, 8))
    x = np.zeros(pr.ne * pr.n)
    psi = None
    for k in range(1, 4):
        x, ex = osmm.apply_G(pr, x, psi)
        psi = ex["psi"]
        rc, info = L.smm_solve(gp, L.smm_default_opts(precision=L.SMM_FP64, outer_tol=0.0, max_outer=k,
                                                       inner_tol=1e-14, max_inner=50000), raise_on_noconv=False)
        got = L.smm_get_outputs_host(gp)
        e = rel_l2(got["varphi"], x)
        print(f"p={p} iteration {k}: rel L2 {e:.2e}", flush=True)
        assert rc == L.SMM_ENOCONV and info["iterations"] == k
        assert e < 1e-12, (k, e)
    assert rel_l2(got["phi"], ex["phi"].reshape(-1)) < 1e-12


@pytest.mark.parametrize("p", [2, 3, 4])
def test_c2_converged_fp32_vs_fp64(ctx, p):
    announce(f"C2 curved 32^2 p={p} S8: converged FP32 sweep vs FP64")
    wl = config_curved_mms(32, p, 8)
    pr, _ = make_pair(L, ctx, wl)
    out = {}
    for name, prec, delta in (("fp64", L.SMM_FP64, 0), ("fp32", L.SMM_FP32_SWEEP, 1)):
        _, gp = make_pair(L, ctx, wl)
        rc, info = L.smm_solve(gp, L.smm_default_opts(precision=prec, delta_sweeps=delta, outer_tol=1e-10,
                                                       inner_tol=1e-13, max_inner=50000, max_outer=80))
        assert rc == L.SMM_OK
        out[name] = L.smm_get_outputs_host(gp)["varphi"]
        err = fem.l2_error(pr.mesh, out[name].reshape(pr.ne, pr.n), mms_phi)
        print(f"p={p} {name}: {info['iterations']} outer, L2 error vs exact {err:.3e}", flush=True)
        L.smm_problem_destroy(gp)
    e = rel_l2(out["fp32"], out["fp64"])
    print(f"p={p}: FP32 vs FP64 rel L2 {e:.2e}", flush=True)
    assert e < 1e-5


@pytest.mark.parametrize("p", [2, 3, 4])
def test_c2_convergence_order(ctx, p):
    announce(f"C2 curved p={p} S8: FP64 order on 8/16/32")
    errs = []
    for n in (8, 16, 32):
        pr, gp = make_pair(L, ctx, config_curved_mms(n, p, 8))
        rc, _ = L.smm_solve(gp, L.smm_default_opts(precision=L.SMM_FP64, outer_tol=1e-12, inner_tol=1e-14,
                                                    max_inner=50000, max_outer=80))
        assert rc == L.SMM_OK
        v = L.smm_get_outputs_host(gp)["varphi"]
        errs.append(fem.l2_error(pr.mesh, v.reshape(pr.ne, pr.n), mms_phi))
        L.smm_problem_destroy(gp)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print(f"p={p}: errors {errs}, orders {orders}", flush=True)
    assert orders[-1] > p + 1 - 0.15, orders
