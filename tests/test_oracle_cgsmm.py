"""Pins of the oracle's continuous (CG) SMM moment system (no GPU).

The oracle defines the CG system as the IP system with test and trial
functions restricted to V_p (Sec. 5.1).  These tests tie it to:
* the CG form as printed (Sec. 5.1), assembled here directly from its own
  terms: the Marshak boundary term, diffusion and absorption on the left; on
  the right Q0, Q1, the inflow and beta terms, the interior-face term
  {grad u / sigma_t}.[T n] and the broken divergence of T.  Agreement checks
  that every interior-face term of the IP form that the restriction drops is
  a jump term;
* V_p itself: (n_x p + 1)(n_y p + 1) unknowns on a structured mesh, curved
  or not, and global polynomials of degree p lie in it;
* one element: V_p = Y_p and no interior faces, so CG and IP coincide;
* the infinite-medium fixed point varphi = 4 pi q / sigma_a and the
  linearly anisotropic patch solution, reproduced to rounding;
* optimal O(h^{p+1}) convergence under the manufactured solution on curved
  meshes (Sec. 6.1: all four methods are optimal) and O(h^{p+1}) distance to
  the DG S_N scalar flux (eq. snconv);
* the thick-diffusion-limit iteration counts of Table tab:tdl_orthog, CG
  column (golden fixture): a trend pin with no parity weight, as for IP.
"""
import os

import numpy as np
import pytest

from oracle import fem, smm, transport
from workloads import config_curved_mms, config_plain, config_tdl, mms_phi

from .test_oracle_smm import _patch_workload


def _direct_cg_lhs(prob):
    """sum_K int_{K cap Gamma_b} E_b0 u phi + int_K grad u . D grad phi +
    int_K sigma_a u phi, element by element, mapped to V_p."""
    mesh, ne, n = prob.mesh, prob.ne, prob.n
    blocks = np.zeros((ne, n, n))
    for K in range(ne):
        D = 1.0 / (3.0 * prob.sigma_t[K])
        sa = prob.sigma_t[K] - prob.sigma_s[K]
        g = mesh.gradU[K]
        for Q in range(len(mesh.wJ[K])):
            blocks[K] += mesh.wJ[K][Q] * (D * g[Q] @ g[Q].T + sa * np.outer(mesh.U[Q], mesh.U[Q]))
        for f in range(4):
            if mesh.nbr[K, f] >= 0:
                continue
            for q in range(len(mesh.dsw[K, f])):
                a, b = mesh.nhat[K, f][q]
                e = np.sum(prob.w * np.abs(prob.omega[:, 0] * a + prob.omega[:, 1] * b)) / np.sum(prob.w)
                blocks[K] += mesh.dsw[K, f][q] * e * np.outer(mesh.Uf[f][q], mesh.Uf[f][q])
    Pc = smm.cg_space(mesh).toarray()
    Abd = np.zeros((ne * n, ne * n))
    for K in range(ne):
        Abd[K * n:(K + 1) * n, K * n:(K + 1) * n] = blocks[K]
    return Pc.T @ Abd @ Pc


def _divh(grad, Tk):
    """Broken divergence of the tensor with nodal components (xx, xy, yy)."""
    dx = [grad[:, :, 0] @ Tk[c] for c in range(3)]
    dy = [grad[:, :, 1] @ Tk[c] for c in range(3)]
    return np.stack([dx[0] + dy[1], dx[1] + dy[2]], axis=1)


def _direct_cg_rhs(prob, T, beta):
    """The right-hand side of the CG form, test functions in V_p."""
    mesh, ne, n = prob.mesh, prob.ne, prob.n
    st = prob.sigma_t
    Q0, Q1 = smm.source_moments(prob)
    jin = transport.inflow_current(mesh, prob.omega, prob.w, prob.psibar)
    b = np.zeros((ne, n))
    for K in range(ne):
        U, g, wJ = mesh.U, mesh.gradU[K], mesh.wJ[K]
        q1 = np.stack([U @ Q1[0, K], U @ Q1[1, K]], axis=1)
        dT = _divh(g, T[:, K])
        for Q in range(len(wJ)):
            b[K] += wJ[Q] * (U[Q] * (U[Q] @ Q0[K]) + g[Q] @ q1[Q] / st[K] - g[Q] @ dT[Q] / st[K])
        for f in range(4):
            bf = mesh.bface_id[K, f]
            if bf < 0:
                continue
            for q in range(len(mesh.dsw[K, f])):
                b[K] -= mesh.dsw[K, f][q] * mesh.Uf[f][q] * (2.0 * jin[bf][q] + beta[bf][q])
    # interior faces: {grad u / sigma_t} . [T n], n from K1 to K2
    for K1 in range(ne):
        for f1 in (1, 2):
            K2 = mesh.nbr[K1, f1]
            if K2 < 0:
                continue
            f2 = fem.OPPOSITE[f1]
            for q in range(len(mesh.dsw[K1, f1])):
                nx, ny = mesh.nhat[K1, f1][q]
                t1 = [mesh.Uf[f1][q] @ T[c, K1] for c in range(3)]
                t2 = [mesh.Uf[f2][q] @ T[c, K2] for c in range(3)]
                jump = np.array([t1[0] * nx + t1[1] * ny - t2[0] * nx - t2[1] * ny,
                                 t1[1] * nx + t1[2] * ny - t2[1] * nx - t2[2] * ny])
                w = mesh.dsw[K1, f1][q]
                b[K1] += w * 0.5 * mesh.gradUf[K1, f1][q] @ jump / st[K1]
                b[K2] += w * 0.5 * mesh.gradUf[K2, f2][q] @ jump / st[K2]
    return smm.cg_space(mesh).T @ b.reshape(-1)


def _varied_problem(curved, p):
    wl = config_curved_mms(n=3, p=p, sn=4) if curved else config_plain(n=3, p=p, sn=6)
    rng = np.random.default_rng(5)
    wl.sigma_t = 10 ** rng.uniform(-0.5, 1.0, wl.n_elem)
    wl.sigma_s = wl.sigma_t * rng.uniform(0.3, 0.9, wl.n_elem)
    if not curved:
        wl.inflow = ("iso", 0.7)
    return smm.make_problem(wl, disc="cg")


@pytest.mark.parametrize("curved", [False, True])
@pytest.mark.parametrize("p", [1, 2])
def test_cg_form_matches_printed_terms(curved, p):
    prob = _varied_problem(curved, p)
    A = smm.cg_matrix(prob).toarray()
    Ad = _direct_cg_lhs(prob)
    assert np.abs(A - Ad).max() < 1e-12 * np.abs(Ad).max()
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0
    rng = np.random.default_rng(7)
    T = rng.normal(size=(3, prob.ne, prob.n))
    beta = rng.normal(size=(int((prob.mesh.bface_id >= 0).sum()), prob.mesh.nq))
    Pc = smm.cg_space(prob.mesh)
    b = Pc.T @ (smm.rhs_fixed(prob) + smm.rhs_correction(prob, T, beta))
    bd = _direct_cg_rhs(prob, T, beta)
    assert np.abs(b - bd).max() < 1e-12 * np.abs(bd).max()


@pytest.mark.parametrize("curved", [False, True])
def test_cg_space(curved):
    p = 3
    wl = config_curved_mms(n=4, p=p, sn=4) if curved else config_plain(n=5, p=p)
    mesh = smm.make_problem(wl).mesh
    Pc = smm.cg_space(mesh)
    assert Pc.shape == (wl.n_elem * (p + 1) ** 2, (wl.nx * p + 1) * (wl.ny * p + 1))
    assert np.all(np.asarray(Pc.sum(axis=1)).ravel() == 1)
    # a global polynomial of degree p in x and y is continuous: its nodal
    # values are reproduced by P_c applied to their restriction
    x, y = mesh.xnode[..., 0].ravel(), mesh.xnode[..., 1].ravel()
    f = 1 + x ** 3 - 2 * x * y ** 2 + y ** 3
    c = np.asarray(Pc.T @ f).ravel() / np.asarray(Pc.sum(axis=0)).ravel()
    assert np.abs(Pc @ c - f).max() < 1e-12


def test_cg_one_element_is_ip():
    wl = config_plain(n=1, p=3, sn=6)
    wl.inflow = ("iso", 0.4)
    x_cg, i1 = smm.solve(smm.make_problem(wl, disc="cg"), tol=1e-14, max_it=100)
    x_ip, i2 = smm.solve(smm.make_problem(wl), tol=1e-14, max_it=100)
    assert i1["converged"] and i2["converged"]
    assert np.abs(x_cg - x_ip).max() < 1e-13 * np.abs(x_ip).max()


@pytest.mark.parametrize("curved,p", [(False, 2), (True, 2), (True, 4)])
def test_cg_infinite_medium_fixed_point(curved, p):
    wl = config_curved_mms(n=4, p=p, sn=4) if curved else config_plain(n=4, p=p, sn=6)
    ne = wl.n_elem
    st, ss, q = 2.0, 1.5, 1.0
    wl.sigma_t, wl.sigma_s, wl.q_elem, wl.q_fn = np.full(ne, st), np.full(ne, ss), np.full(ne, q), None
    wl.inflow = ("iso", q / (st - ss))
    prob = smm.make_problem(wl, disc="cg")
    X = np.full(ne * prob.n, 4 * np.pi * q / (st - ss))
    lag = np.full((len(prob.w), ne, prob.n), q / (st - ss))
    G, _ = smm.apply_G(prob, X, psi_lag=lag)
    assert np.abs(G - X).max() < 1e-13 * X.max()
    x, info = smm.solve(prob, tol=1e-12)
    assert info["converged"] and np.abs(x - X).max() < 1e-10 * X.max()


@pytest.mark.parametrize("p", [1, 2])
def test_cg_patch_linear_anisotropy(p):
    wl, a, _ = _patch_workload(p)
    prob = smm.make_problem(wl, disc="cg")
    x, info = smm.solve(prob, tol=1e-14, max_it=100)
    xn = prob.mesh.xnode
    ex = 4 * np.pi * a(xn[..., 0], xn[..., 1]).reshape(-1)
    assert info["converged"]
    assert np.abs(x - ex).max() < 1e-13 * ex.max()


@pytest.mark.parametrize("p,sn", [(1, 8), (2, 8), (3, 4), (4, 4)])
def test_cg_mms_curved_order(p, sn):
    errs = []
    for n in (4, 8, 16):
        prob = smm.make_problem(config_curved_mms(n=n, p=p, sn=sn), disc="cg")
        x, info = smm.solve(prob, tol=1e-11, max_it=60)
        assert info["converged"]
        errs.append(fem.l2_error(prob.mesh, x.reshape(prob.ne, prob.n), mms_phi))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > p + 1 - 0.15, orders


def test_cg_converges_to_sn_solution():
    diffs = []
    for n in (4, 8, 16):
        prob = smm.make_problem(config_plain(n=n, p=1, sn=4), disc="cg")
        x, info = smm.solve(prob, tol=1e-13, max_it=100)
        phi_sn = smm.sn_krylov(prob)
        diffs.append(fem.l2_norm(prob.mesh, (x - phi_sn).reshape(prob.ne, prob.n)))
    orders = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert orders[-1] > 1.7, orders


def test_cg_thick_diffusion_limit_iterations():
    counts = []
    for eps in (1e-1, 1e-2, 1e-3, 1e-4):
        prob = smm.make_problem(config_tdl(eps), disc="cg")
        x = np.zeros(prob.ne * prob.n)
        for it in range(1, 30):
            xn, _ = smm.apply_G(prob, x)
            r = np.abs(xn - x).max()
            x = xn
            if r < 1e-6:
                break
        counts.append(it)
    assert counts == sorted(counts, reverse=True)
    gold = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "tdl_orthog_cg_smm_iterations.txt"))
    assert np.allclose(gold[:, 0], [1e-1, 1e-2, 1e-3, 1e-4])
    assert np.all(np.array(counts) <= gold[:, 1])
