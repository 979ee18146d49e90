"""Parity of the HIP path with the FP64 oracle on meshes given element by
element and on explicit angular sets (through the C ABI).

* One sweep (the per-element kernels: one lane per element at p <= 2, one
  wave per element at p >= 3) on seeded sources with random lagged inputs:
  FP64 within 1e-12, FP32 within 1e-5 relative L2, on the curved mesh with
  turned local frames (all face pairings, reversed face parameterisations),
  the unstructured inner-square mesh, that mesh turned (boundaries not along
  x or y), a slanted structured mesh and a product angular set.
* One evaluation of G (eq. moment:smm_fp) in FP64: within 1e-12, with beta
  from every boundary point's own normal where the boundary is not along x
  or y.
* Three fixed FP64 outer iterations, and the converged FP32-sweep flux
  (delta sweeps, beta accumulated like the moments) against the converged
  oracle: 1e-12 and 1e-5.
* The converged flux on the turned-frame mesh equals the structured mesh's,
  node for node, within 1e-12.
"""
import numpy as np
import pytest

from oracle import smm as osmm
from oracle import transport

from .gpu_common import announce, make_pair, rel_l2
from .test_general_mesh_host import CASES, _inner, _rot_curved
from .test_oracle_general_mesh import _node_perm

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _pair(ctx, wl):
    pr = osmm.make_problem(wl)
    iso = isinstance(wl.inflow, tuple) and wl.inflow[0] in ("iso", "attr")
    p = L.problem_from_workload(ctx, wl, q=pr.q, psibar=None if iso else pr.psibar)
    return pr, p


@pytest.mark.parametrize("name", list(CASES))
def test_general_sweep(ctx, name):
    wl = CASES[name]()
    pr, p = _pair(ctx, wl)
    rng = np.random.default_rng(7)
    S = rng.uniform(0.2, 1.5, size=(pr.ne, pr.n))
    lag = rng.uniform(0.0, 1.0, size=(len(pr.w), pr.ne, pr.n))
    ref = transport.sweep(pr.mesh, pr.omega, pr.sigma_t, S, pr.psibar, lag)
    for prec, dt, bar in ((L.SMM_FP64, torch.float64, 1e-12), (L.SMM_FP32_SWEEP, torch.float32, 1e-5)):
        announce(f"general sweep {name} precision {prec}")
        out = torch.zeros((p.n_dir, p.n_elem, p.n_node), dtype=dt, device="cuda")
        L.smm_apply_sweep(p, prec, _dev(S, dt), L.SMM_SRC_ISO, _dev(lag, dt), out, True)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        e = rel_l2(got, ref)
        assert e < bar, (name, prec, e)


@pytest.mark.parametrize("name", ["rotated_p2", "inner_m2_p2", "inner_turned_m2_p3", "slanted_p2",
                                  "inner_product_quad"])
def test_general_apply_G(ctx, name):
    announce(f"general apply_G fp64 {name}")
    pr, p = _pair(ctx, CASES[name]())
    x = np.random.default_rng(5).uniform(0.0, 10.0, pr.ne * pr.n)
    ref, ex = osmm.apply_G(pr, x)
    xin = _dev(x)
    xout = torch.zeros_like(xin)
    L.smm_apply_G(p, L.SMM_FP64, xin, xout, 1e-15, 20000)
    got = xout.cpu().numpy()
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)
    out = L.smm_get_outputs_host(p)
    assert rel_l2(out["phi"], ex["phi"].ravel()) < 1e-12
    assert rel_l2(out["T"], ex["T"].reshape(3, -1)) < 1e-11
    assert rel_l2(out["beta"], ex["beta"]) < 1e-11


@pytest.mark.parametrize("name", ["inner_turned_m2_p3", "rotated_p3"])
def test_general_iterations_and_converged(ctx, name):
    announce(f"general fixed iterations and converged solve {name}")
    wl = CASES[name]()
    pr, p = _pair(ctx, wl)
    ref3, _ = osmm.solve(pr, tol=0.0, max_it=3)
    rc, info = L.smm_solve(p, L.smm_default_opts(precision=L.SMM_FP64, outer_tol=0.0, max_outer=3, inner_tol=1e-15,
                                                  max_inner=20000), raise_on_noconv=False)
    assert rc == L.SMM_ENOCONV and info["iterations"] == 3
    assert rel_l2(L.smm_get_outputs_host(p)["varphi"], ref3) < 1e-12
    ref, oinfo = osmm.solve(pr, tol=1e-13, max_it=200)
    assert oinfo["converged"]
    rc, _ = L.smm_solve(p, L.smm_default_opts(precision=L.SMM_FP64, outer_tol=1e-13, inner_tol=1e-15,
                                               max_inner=20000, max_outer=200))
    assert rc == L.SMM_OK and rel_l2(L.smm_get_outputs_host(p)["varphi"], ref) < 1e-12
    rc, _ = L.smm_solve(p, L.smm_default_opts(precision=L.SMM_FP32_SWEEP, delta_sweeps=1, outer_tol=1e-10,
                                               inner_tol=1e-13, max_inner=20000, max_outer=200))
    e = rel_l2(L.smm_get_outputs_host(p)["varphi"], ref)
    print(f"{name}: FP32 sweeps vs oracle {e:.2e}", flush=True)
    assert rc == L.SMM_OK and e < 1e-5


def test_turned_frames_equal_structured_on_gpu(ctx):
    announce("turned local frames vs structured mesh, converged on the GPU")
    gw = _rot_curved(2)
    from workloads import config_curved_mms
    wl = config_curved_mms(4, 2, 4, amplitude=0.06)
    pr0, p0 = _pair(ctx, wl)
    pr1, p1 = _pair(ctx, gw)
    opts = L.smm_default_opts(precision=L.SMM_FP64, outer_tol=1e-13, inner_tol=1e-15, max_inner=20000, max_outer=200)
    L.smm_solve(p0, opts)
    L.smm_solve(p1, opts)
    v0 = L.smm_get_outputs_host(p0)["varphi"]
    v1 = L.smm_get_outputs_host(p1)["varphi"]
    idx = _node_perm(pr0.mesh, pr1.mesh)
    assert rel_l2(v1, v0[idx]) < 1e-12
