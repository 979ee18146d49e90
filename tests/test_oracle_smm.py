"""Pins of the oracle's SMM moment system and fixed point (no GPU).

* Infinite medium (uniform data, isotropic inflow q/sigma_a): psi = q/sigma_a,
  T = beta = 0 and varphi = 4 pi q/sigma_a is a fixed point of G on any mesh,
  curved included.
* Patch test: psi_d = a + Omega_d.b with a, b in Q_1 and the matching source
  and inflow is reproduced to rounding by the sweep, and varphi = 4 pi a by
  the SMM fixed point (upwind DG and symmetric IP are consistent).
* sigma_s = 0: G is constant, so the second iterate equals the first and the
  transport phi equals one source-iteration sweep.
* The iterated fixed point equals the solution of the linear system
  (I - G_lin) X = G(0).
* IP matrix: symmetric and positive definite.
* Manufactured solution on curved meshes: || varphi - phi_ex || = O(h^{p+1})
  (Sec. 6.1) for p = 1..4 on order-p maps (m = p).
* Curved face and volume gradients: the nodal interpolant of an affine field
  is that field exactly when m <= p, so its physical gradient at every volume
  and face point is the constant gradient, at any order.
* SMM versus the DG S_N solution: difference O(h^{p+1}) (eq. snconv).
* Thick diffusion limit (Sec. 6.2): bounded outer iteration counts that
  fall as epsilon falls.  Trend only, with no parity weight: Table
  tab:tdl_orthog prints 10/8/5/4, the oracle takes 8/5/3/2 (its contraction
  per iteration is faster at every epsilon; the table's start, stopping norm
  and transport discretisation are not stated), so the test checks the trend
  and that the oracle needs no more iterations than the table.
"""
import os

import numpy as np
import pytest

from oracle import fem, smm, transport
from workloads import (Workload, config_curved_mms, config_plain, config_tdl,
                       mms_phi, structured_ctrl)


@pytest.mark.parametrize("curved,p", [(False, 2), (True, 2), (True, 4)])
def test_infinite_medium_fixed_point(curved, p):
    wl = config_curved_mms(n=4, p=p, sn=4) if curved else config_plain(n=4, p=p, sn=6)
    ne = wl.n_elem
    st, ss, q = 2.0, 1.5, 1.0
    wl.sigma_t, wl.sigma_s, wl.q_elem, wl.q_fn = np.full(ne, st), np.full(ne, ss), np.full(ne, q), None
    wl.inflow = ("iso", q / (st - ss))
    prob = smm.make_problem(wl)
    X = np.full(ne * prob.n, 4 * np.pi * q / (st - ss))
    lag = np.full((len(prob.w), ne, prob.n), q / (st - ss))
    G, ex = smm.apply_G(prob, X, psi_lag=lag)
    assert np.abs(G - X).max() < 1e-13 * X.max()
    assert np.abs(ex["psi"] - q / (st - ss)).max() < 1e-13
    assert np.abs(ex["T"]).max() < 1e-13 and np.abs(ex["beta"]).max() < 1e-13
    x, info = smm.solve(prob, tol=1e-12)
    assert info["converged"] and np.abs(x - X).max() < 1e-10 * X.max()


def _patch_workload(p):
    a = lambda x, y: 1 + 0.3 * x + 0.2 * y + 0.1 * x * y
    ax, ay = (lambda x, y: 0.3 + 0.1 * y), (lambda x, y: 0.2 + 0.1 * x)
    bx = lambda x, y: 0.2 + 0.1 * x - 0.3 * y + 0.05 * x * y
    by = lambda x, y: -0.1 + 0.2 * x + 0.1 * y - 0.1 * x * y
    bxx, bxy = (lambda x, y: 0.1 + 0.05 * y), (lambda x, y: -0.3 + 0.05 * x)
    byx, byy = (lambda x, y: 0.2 - 0.1 * y), (lambda x, y: 0.1 - 0.1 * x)
    st, ss = 2.0, 1.2
    psi = lambda x, y, ox, oy: a(x, y) + ox * bx(x, y) + oy * by(x, y)
    q = lambda x, y, ox, oy: (ox * ax(x, y) + oy * ay(x, y) + ox * (ox * bxx(x, y) + oy * byx(x, y))
                              + oy * (ox * bxy(x, y) + oy * byy(x, y)) + st * psi(x, y, ox, oy) - ss * a(x, y))
    xv = np.array([0, 0.1, 0.35, 0.5, 0.8, 1.0])
    yv = np.array([0, 0.2, 0.3, 0.7, 1.0])
    wl = Workload("patch", 5, 4, 1, p, 6, structured_ctrl(xv, yv, 1), np.full(20, st), np.full(20, ss),
                  q_fn=q, inflow=("fn", psi))
    return wl, a, psi


@pytest.mark.parametrize("p", [1, 2])
def test_patch_linear_anisotropy(p):
    wl, a, psi_ex = _patch_workload(p)
    prob = smm.make_problem(wl)
    x, info = smm.solve(prob, tol=1e-14, max_it=100)
    xn = prob.mesh.xnode
    ex = 4 * np.pi * a(xn[..., 0], xn[..., 1]).reshape(-1)
    assert info["converged"]
    assert np.abs(x - ex).max() < 1e-13 * ex.max()
    for d in (0, 7, 20):
        o = prob.omega[d]
        assert np.abs(info["psi"][d] - psi_ex(xn[..., 0], xn[..., 1], o[0], o[1])).max() < 1e-13


def test_no_scattering_degenerate():
    wl = config_plain(n=4, p=1, sn=4)
    wl.sigma_s[:] = 0.0
    prob = smm.make_problem(wl)
    x, info = smm.solve(prob, tol=1e-14, max_it=5)
    assert info["iterations"] == 2 and info["history"][1] == 0.0
    phi_si, _, _ = smm.source_iteration(prob, max_it=1)
    assert np.abs(info["phi"].reshape(-1) - phi_si).max() < 1e-14 * phi_si.max()


def test_fixed_point_equals_direct_solve():
    wl = config_plain(n=4, p=1, sn=4)
    prob = smm.make_problem(wl)
    x, info = smm.solve(prob, tol=1e-15, max_it=100)
    xd = smm.fixed_point_direct(prob)
    assert np.abs(x - xd).max() < 1e-12 * np.abs(xd).max()


@pytest.mark.parametrize("curved", [False, True])
def test_ip_matrix_spd(curved):
    wl = config_curved_mms(n=4, p=2, sn=8) if curved else config_plain(n=8, p=1)
    prob = smm.make_problem(wl)
    A = smm.ip_matrix(prob).toarray()
    assert np.abs(A - A.T).max() < 1e-15 * np.abs(A).max() * 10
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


@pytest.mark.parametrize("p,sn", [(1, 8), (2, 8), (3, 4), (4, 4)])
def test_mms_curved_order(p, sn):
    # the manufactured psi is quadratic in Omega_x, which every level-symmetric
    # set integrates exactly, so S4 serves as well as S8 at p = 3, 4
    errs = []
    for n in (4, 8, 16):
        prob = smm.make_problem(config_curved_mms(n=n, p=p, sn=sn))
        x, info = smm.solve(prob, tol=1e-11, max_it=60)
        assert info["converged"]
        errs.append(fem.l2_error(prob.mesh, x.reshape(prob.ne, prob.n), mms_phi))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > p + 1 - 0.15, orders


@pytest.mark.parametrize("p", [2, 3, 4])
def test_affine_field_gradients_curved(p):
    wl = config_curved_mms(n=3, p=p, sn=4, amplitude=0.09)
    mesh = fem.build_mesh(wl.ctrl, wl.nx, wl.ny, wl.m, wl.p)
    g = np.array([0.7, -1.3])
    u = 0.4 + mesh.xnode @ g                                    # [K, n] nodal values
    vol = np.einsum("kqna,kn->kqa", mesh.gradU, u)
    face = np.einsum("kfqna,kn->kfqa", mesh.gradUf, u)
    assert np.abs(vol - g).max() < 1e-12
    assert np.abs(face - g).max() < 1e-12
    # values at the points reproduce the field too
    assert np.abs(u @ mesh.U.T - (0.4 + mesh.xq @ g)).max() < 1e-13
    for f in range(4):
        assert np.abs(u @ mesh.Uf[f].T - (0.4 + mesh.xf[:, f] @ g)).max() < 1e-13


def test_smm_converges_to_sn_solution():
    diffs = []
    for n in (4, 8, 16):
        wl = config_plain(n=n, p=1, sn=4)
        prob = smm.make_problem(wl)
        x, info = smm.solve(prob, tol=1e-13, max_it=100)
        phi_sn = smm.sn_krylov(prob)
        diffs.append(fem.l2_norm(prob.mesh, (x - phi_sn).reshape(prob.ne, prob.n)))
    orders = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert orders[-1] > 1.7, orders


def test_sn_krylov_matches_source_iteration():
    wl = config_plain(n=3, p=1, sn=4)
    wl.sigma_s[:] = 0.5
    prob = smm.make_problem(wl)
    a = smm.sn_krylov(prob)
    b, its, _ = smm.source_iteration(prob, tol=1e-15)
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_thick_diffusion_limit_iterations():
    counts = []
    for eps in (1e-1, 1e-2, 1e-3, 1e-4):
        prob = smm.make_problem(config_tdl(eps))
        x = np.zeros(prob.ne * prob.n)
        for it in range(1, 30):
            xn, _ = smm.apply_G(prob, x)
            r = np.abs(xn - x).max()
            x = xn
            if r < 1e-6:
                break
        counts.append(it)
    assert counts == sorted(counts, reverse=True)
    assert min(counts) >= 2
    # the paper's counts (golden fixture): the same trend, and no count above
    # the table's (a trend pin: the discretisation details behind the table's
    # exact counts are not stated)
    gold = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "tdl_orthog_smm_iterations.txt"))
    assert np.allclose(gold[:, 0], [1e-1, 1e-2, 1e-3, 1e-4])
    assert np.all(np.diff(gold[:, 1]) <= 0)
    assert np.all(np.array(counts) <= gold[:, 1])
