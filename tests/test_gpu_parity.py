"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (relative L2 over coefficient vectors):
  FP64 sweep 1e-12, moments / closures 1e-13, G and K fixed outer iterations
  1e-12, converged FP64 solve 1e-12; FP32 sweep and FP32 converged scalar flux
  1e-5 (the FP32 target; observed errors are ~1e-7).
"""
import numpy as np
import pytest

from oracle import smm as osmm
from oracle import transport
from workloads import config_channel, config_curved_mms, config_plain, structured_ctrl, Workload

from .gpu_common import announce, make_pair, rel_l2

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    return L.smm_ctx_create(0, stream)


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _sweep_gpu(p, prec, S, lag=None, inflow=True):
    dt = torch.float64 if prec == L.SMM_FP64 else torch.float32
    Sd = _dev(S, dt)
    out = torch.zeros((p.n_dir, p.n_elem, p.n_node), dtype=dt, device="cuda")
    lagd = _dev(lag, dt) if lag is not None else None
    L.smm_apply_sweep(p, prec, Sd, L.SMM_SRC_ANISO if S.ndim == 3 else L.SMM_SRC_ISO, lagd, out, inflow)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


SWEEP_CASES = [
    # (name, workload factory, sweep path: 0 auto, 1 per-element kernel, 2 element-row
    # kernel, 3 per-element kernel with one wave per element also at p <= 2,
    # 4 per-element kernel with one lane per row at every order p >= 2,
    # 5 per-element kernel assembling and eliminating in the form 0 picked
    # before the stored element operators; 0 and 1 on curved or non-uniform
    # meshes use the stored operators)
    ("plain8_p1_s4", lambda: config_plain(8, 1, 4), 0),
    ("plain8_p1_s4_general", lambda: config_plain(8, 1, 4), 1),
    ("plain8_p1_s4_rowkernel", lambda: config_plain(8, 1, 4), 2),
    ("plain5_p3_s8_onemat", lambda: config_plain(5, 3, 8), 0),
    ("twomat9x6_p2_s10", lambda: _rect(9, 6, 2, 10, nmat=2), 0),
    ("twomat6x9_p1_s6", lambda: _rect(6, 9, 1, 6, nmat=2), 0),
    ("ragged7x3_p4_s12", lambda: _rect(7, 3, 4, 12), 0),
    ("ragged7x3_p4_s12_rowkernel", lambda: _rect(7, 3, 4, 12), 2),
    ("ragged7x3_p3_s6_general", lambda: _rect(7, 3, 3, 6), 1),
    ("single_p2_s8", lambda: _rect(1, 1, 2, 8), 0),
    ("curved4_p2_s8", lambda: config_curved_mms(4, 2, 8, amplitude=0.09), 0),
    ("curved4_p2_s8_wavesolve", lambda: config_curved_mms(4, 2, 8, amplitude=0.09), 3),
    ("plain8_p2_s4_general", lambda: config_plain(8, 2, 4), 1),
    ("plain8_p1_s4_wavesolve", lambda: config_plain(8, 1, 4), 3),
    ("curved3_p4_s4", lambda: config_curved_mms(3, 4, 4), 0),
    # per-element kernel with one lane per row (Gauss-Jordan): the default at
    # p >= 3, forced at p = 2; and the wave-per-element form at p = 3, 4
    ("curved4_p2_s8_rowsolve", lambda: config_curved_mms(4, 2, 8, amplitude=0.09), 4),
    ("curved5_p3_s6", lambda: config_curved_mms(5, 3, 6, amplitude=0.09), 0),
    ("curved5_p3_s6_wavesolve", lambda: config_curved_mms(5, 3, 6, amplitude=0.09), 3),
    ("curved3_p4_s4_wavesolve", lambda: config_curved_mms(3, 4, 4), 3),
    ("ragged7x3_p4_s12_rowsolve", lambda: _rect(7, 3, 4, 12), 4),
    ("ragged7x3_p4_s12", lambda: _rect(7, 3, 4, 12), 0),
    ("curved4_p2_s8_assembled", lambda: config_curved_mms(4, 2, 8, amplitude=0.09), 5),
    ("curved5_p3_s6_assembled", lambda: config_curved_mms(5, 3, 6, amplitude=0.09), 5),
    ("curved3_p4_s4_assembled", lambda: config_curved_mms(3, 4, 4), 5),
]


def _rect(nx, ny, p, sn, inflow=("iso", 0.4), nmat=3):
    xv = np.linspace(0.0, 1.4, nx + 1)
    yv = np.linspace(0.0, 0.6, ny + 1)
    ne = nx * ny
    rng = np.random.default_rng(nx * 100 + ny)
    st = rng.choice([0.5, 2.0, 7.0][:nmat], size=ne)
    return Workload("rect", nx, ny, 1, p, sn, structured_ctrl(xv, yv, 1), st, 0.5 * st,
                    q_elem=rng.uniform(0.2, 1.0, ne), inflow=inflow)


@pytest.mark.parametrize("name,factory,path", SWEEP_CASES, ids=[c[0] for c in SWEEP_CASES])
def test_sweep_fp64(ctx, name, factory, path):
    announce(f"sweep fp64 {name}")
    wl = factory()
    if name.startswith("curved"):
        wl.inflow = ("iso", 0.3)
        wl.q_fn = None
        wl.q_elem = np.ones(wl.n_elem)
    pr, p = make_pair(L, ctx, wl)
    L.smm_set_sweep_path(p, path)
    rng = np.random.default_rng(7)
    S = rng.uniform(-1.0, 2.0, (pr.ne, pr.n))
    lag = rng.uniform(0.0, 1.0, (len(pr.w), pr.ne, pr.n)) if name.startswith("curved") else None
    ref = transport.sweep(pr.mesh, pr.omega, pr.sigma_t, S, pr.psibar, lag)
    got = _sweep_gpu(p, L.SMM_FP64, S, lag)
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)
    # anisotropic source layout
    Sa = rng.uniform(0.0, 1.0, (len(pr.w), pr.ne, pr.n))
    ref = transport.sweep(pr.mesh, pr.omega, pr.sigma_t, Sa, pr.psibar, lag)
    got = _sweep_gpu(p, L.SMM_FP64, Sa, lag)
    assert rel_l2(got, ref) < 1e-12
    # FP32 sweep against the FP64 oracle
    got32 = _sweep_gpu(p, L.SMM_FP32_SWEEP, S, lag)
    ref = transport.sweep(pr.mesh, pr.omega, pr.sigma_t, S, pr.psibar, lag)
    assert rel_l2(got32, ref) < 1e-5, rel_l2(got32, ref)


@pytest.mark.parametrize("n,p,sn", [(8, 2, 12), (3, 2, 4), (5, 1, 6)])
def test_moments(ctx, n, p, sn):
    announce(f"moments fp64/fp32 on plain{n} p{p} s{sn}")
    wl = config_plain(n, p, sn)
    pr, p = make_pair(L, ctx, wl)
    rng = np.random.default_rng(11)
    psi = rng.uniform(-1, 1, (len(pr.w), pr.ne, pr.n))
    phi, J, P = transport.moments(pr.omega, pr.w, psi)
    mom = torch.zeros((8, pr.ne * pr.n), dtype=torch.float64, device="cuda")
    L.smm_apply_moments(p, L.SMM_FP64, _dev(psi), mom)
    torch.cuda.synchronize()
    m = mom.cpu().numpy()
    assert rel_l2(m[0], phi) < 1e-12
    assert rel_l2(m[1:3], J) < 1e-12
    assert rel_l2(m[3:6], P) < 1e-12
    ax = np.einsum("d,dkn->kn", pr.w * np.abs(pr.omega[:, 0]), psi)
    ay = np.einsum("d,dkn->kn", pr.w * np.abs(pr.omega[:, 1]), psi)
    assert rel_l2(m[6], ax) < 1e-12 and rel_l2(m[7], ay) < 1e-12
    L.smm_apply_moments(p, L.SMM_FP32_SWEEP, _dev(psi, torch.float32), mom)
    torch.cuda.synchronize()
    m32 = mom.cpu().numpy()
    assert rel_l2(m32[0], phi) < 1e-6 and rel_l2(m32[1:3], J) < 1e-6 and rel_l2(m32[3:6], P) < 1e-6
    assert rel_l2(m32[6], ax) < 1e-6 and rel_l2(m32[7], ay) < 1e-6


def _gpu_G(p, x):
    xin = _dev(x)
    xout = torch.zeros_like(xin)
    L.smm_apply_G(p, L.SMM_FP64, xin, xout, 1e-15, 3000)
    return xout.cpu().numpy()


@pytest.mark.parametrize("case", ["plain", "curved", "patch"])
def test_apply_G_fp64(ctx, case):
    announce(f"apply_G fp64 {case}")
    if case == "plain":
        wl = config_plain(6, 2, 6)
    elif case == "curved":
        wl = config_curved_mms(4, 2, 8)
    else:
        from tests.test_oracle_smm import _patch_workload
        wl, _, _ = _patch_workload(2)
    pr, p = make_pair(L, ctx, wl)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 10.0, pr.ne * pr.n)
    ref, ex = osmm.apply_G(pr, x)
    got = _gpu_G(p, x)
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)
    out = L.smm_get_outputs_host(p)
    assert rel_l2(out["phi"], ex["phi"].ravel()) < 1e-12
    assert rel_l2(out["J"], ex["J"].reshape(2, -1)) < 1e-12
    assert rel_l2(out["T"], ex["T"].reshape(3, -1)) < 1e-11
    assert rel_l2(out["beta"], ex["beta"]) < 1e-11


@pytest.mark.parametrize("case", ["plain", "curved"])
def test_fixed_outer_iterations_fp64(ctx, case):
    K = 4
    announce(f"{K} outer iterations fp64 {case}")
    wl = config_plain(8, 1, 4) if case == "plain" else config_curved_mms(4, 2, 8)
    pr, p = make_pair(L, ctx, wl)
    ref, info = osmm.solve(pr, tol=0.0, max_it=K)
    opts = L.smm_default_opts(precision=L.SMM_FP64, outer_tol=0.0, max_outer=K, inner_tol=1e-15,
                              max_inner=3000)
    rc, ginfo = L.smm_solve(p, opts, raise_on_noconv=False)
    assert rc == L.SMM_ENOCONV and ginfo["iterations"] == K
    got = L.smm_get_outputs_host(p)["varphi"]
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)


def test_converged_plain_fp64(ctx):
    announce("converged plain 8x8 p1 S4 fp64")
    wl = config_plain()
    pr, p = make_pair(L, ctx, wl)
    ref, info = osmm.solve(pr, tol=1e-13, max_it=100)
    opts = L.smm_default_opts(precision=L.SMM_FP64, outer_tol=1e-13, inner_tol=1e-15, max_inner=3000)
    rc, ginfo = L.smm_solve(p, opts)
    out = L.smm_get_outputs_host(p)
    assert rc == L.SMM_OK
    assert abs(ginfo["iterations"] - info["iterations"]) <= 1
    assert rel_l2(out["varphi"], ref) < 1e-12
    assert rel_l2(out["phi"], info["phi"].ravel()) < 1e-11
    assert rel_l2(out["T"], info["T"].reshape(3, -1)) < 1e-10


@pytest.mark.parametrize("delta", [1, 0])
def test_converged_fp32_sweep(ctx, delta):
    announce(f"converged plain 8x8 p1 S4 fp32 sweep delta={delta}")
    wl = config_plain()
    pr, p = make_pair(L, ctx, wl)
    ref, info = osmm.solve(pr, tol=1e-12, max_it=100)
    opts = L.smm_default_opts(precision=L.SMM_FP32_SWEEP, outer_tol=1e-8 if delta else 1e-6,
                              inner_tol=1e-13, delta_sweeps=delta)
    rc, ginfo = L.smm_solve(p, opts)
    out = L.smm_get_outputs_host(p)
    assert rc == L.SMM_OK
    assert rel_l2(out["varphi"], ref) < 1e-5, rel_l2(out["varphi"], ref)


def test_channel_full_size_sampled_sweep(ctx):
    """Full-size multi-material case (128 x 128, p = 2, S12) in the launch
    configuration the benchmark times: the FP32 sweep of every direction runs
    on the GPU; the oracle recomputes two sampled directions in FP64."""
    announce("channel 128x128 p2 S12 fp32 sweep, sampled directions")
    wl = config_channel()
    pr = osmm.make_problem(wl)
    p = L.problem_from_workload(ctx, wl)
    rng = np.random.default_rng(3)
    S = rng.uniform(0.0, 1.0, (pr.ne, pr.n))
    got = _sweep_gpu(p, L.SMM_FP32_SWEEP, S)
    for d in (5, 62):
        om = pr.omega[d:d + 1]
        ref = transport.sweep(pr.mesh, om, pr.sigma_t, S, None)
        assert rel_l2(got[d], ref[0]) < 1e-5, (d, rel_l2(got[d], ref[0]))


@pytest.mark.parametrize("p", [2, 3, 4])
def test_curved_full_size_sampled_sweep(ctx, p):
    """Full-size curved manufactured case (32 x 32, order-p geometry, S8) with
    its anisotropic manufactured source and inflow: the FP64 and FP32 sweeps
    of every direction run on the GPU (per-element kernel); the oracle
    recomputes three sampled directions in FP64."""
    announce(f"curved 32x32 p{p} S8 sweep, sampled directions")
    wl = config_curved_mms(32, p, 8)
    pr = osmm.make_problem(wl)
    p_ = L.problem_from_workload(ctx, wl, q=pr.q, psibar=pr.psibar)
    got64 = _sweep_gpu(p_, L.SMM_FP64, pr.q)
    got32 = _sweep_gpu(p_, L.SMM_FP32_SWEEP, pr.q)
    for d in (0, 17, 39):
        sub = pr.psibar[:, :, d:d + 1] if pr.psibar is not None else None
        ref = transport.sweep(pr.mesh, pr.omega[d:d + 1], pr.sigma_t, pr.q[d:d + 1], sub)[0]
        assert rel_l2(got64[d], ref) < 1e-12, (d, rel_l2(got64[d], ref))
        assert rel_l2(got32[d], ref) < 1e-5, (d, rel_l2(got32[d], ref))
