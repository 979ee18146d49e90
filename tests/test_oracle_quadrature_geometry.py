"""Pins of the oracle's quadrature and geometry against closed forms and
identities (no GPU).

* Level-symmetric sets: sum w = 4 pi, sum w mu^2 = 4 pi/3, odd moments vanish,
  sum w mu^4 = 4 pi/5, sum w mu^2 eta^2 = 4 pi/15 (exact sphere integrals);
  N(N+2)/2 directions in 2D (Sec. 4; S12 has 84 directions as used in Sec. 6.6).
* E_b0 tends to 1/2 as N grows (Sec. 4, eq. eb0_disc and the limit stated
  after eq. smm_bc_disc) and is the same for x and y normals.
* Mesh: element areas sum to the domain area (the boundary is not moved by
  the curved perturbation); the outward n ds integrates to zero on every
  element; the gradient matrices satisfy the integration-by-parts identity
  G + G^T = closed-surface integral of (Omega.n) u_i u_j.
* Local transport operator: symmetric part sigma_t M + 1/2 int |Omega.n| u u,
  hence positive definite.
"""
import math

import numpy as np
import pytest

from oracle import fem, quadrature
from workloads import config_curved_mms, config_plain, structured_ctrl, sine_perturbation


@pytest.mark.parametrize("N", [4, 6, 8, 10, 12])
def test_level_symmetric_moments(N):
    om, w = quadrature.level_symmetric_2d(N)
    assert len(w) == N * (N + 2) // 2
    assert np.all(w > 0)
    assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-15)
    assert np.all(om[:, 2] > 0)
    fp = 4 * math.pi
    assert abs(w.sum() - fp) < 1e-13
    for a in range(2):
        assert abs(np.sum(w * om[:, a])) < 1e-13
        assert abs(np.sum(w * om[:, a] ** 3)) < 1e-13
        assert abs(np.sum(w * om[:, a] ** 2) - fp / 3) < 1e-13
        assert abs(np.sum(w * om[:, a] ** 4) - fp / 5) < 1e-13
    assert abs(np.sum(w * om[:, 0] * om[:, 1])) < 1e-13
    assert abs(np.sum(w * om[:, 0] ** 2 * om[:, 1] ** 2) - fp / 15) < 1e-13


def test_eb0_limit():
    vals = []
    for N in (4, 6, 8, 10, 12):
        om, w = quadrature.level_symmetric_2d(N)
        ex = quadrature.eb0(om, w, np.array([1.0, 0.0]))
        ey = quadrature.eb0(om, w, np.array([0.0, 1.0]))
        assert abs(ex - ey) < 1e-14
        vals.append(ex)
    assert all(v > 0.5 for v in vals)
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert vals[-1] - 0.5 < 0.006


def test_gauss_rules():
    for q in range(1, 8):
        x, w = quadrature.gauss_legendre_unit(q)
        for k in range(2 * q):
            assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14
    for p in range(1, 6):
        g = quadrature.gauss_lobatto_unit(p)
        assert g[0] == 0.0 and g[-1] == 1.0
        assert np.allclose(g, 1 - g[::-1], atol=1e-15)


@pytest.mark.parametrize("curved,p", [(False, 1), (False, 3), (True, 2), (True, 4)])
def test_mesh_identities(curved, p):
    wl = config_curved_mms(n=4, p=p, sn=4) if curved else config_plain(n=3, p=p)
    mesh = fem.build_mesh(wl.ctrl, wl.nx, wl.ny, wl.m, wl.p)
    assert abs(mesh.area.sum() - 1.0) < 1e-14
    # closed-surface integral of n ds vanishes on every element
    tot = mesh.nds.sum(axis=(1, 2))
    assert np.abs(tot).max() < 1e-14
    # integration by parts: G^Om + G^Om^T = oint (Omega.n) u_i u_j
    om = np.array([0.37, -0.81])
    for K in range(mesh.nx * mesh.ny):
        G = om[0] * mesh.Gx[K] + om[1] * mesh.Gy[K]
        S = np.zeros_like(G)
        for f in range(4):
            on = mesh.nds[K, f] @ om
            S += np.einsum("q,qi,qj->ij", on, mesh.Uf[f], mesh.Uf[f])
        assert np.abs(G + G.T - S).max() < 1e-13
    # mass matrix rows sum to the element integral of each basis function,
    # and the basis interpolates the coordinates (iso/super-parametric map)
    assert np.allclose(mesh.M.sum(axis=(1, 2)), mesh.area, atol=1e-14)


def test_local_operator_positive_definite():
    wl = config_curved_mms(n=4, p=3, sn=8)
    mesh = fem.build_mesh(wl.ctrl, wl.nx, wl.ny, wl.m, wl.p)
    om, _ = quadrature.level_symmetric_2d(8)
    for K in (0, 5, 10, 15):
        for d in range(0, 40, 7):
            o = om[d]
            A = 2.0 * mesh.M[K] - o[0] * mesh.Gx[K] - o[1] * mesh.Gy[K]
            sym = 2.0 * mesh.M[K]
            for f in range(4):
                on = mesh.nds[K, f] @ o[:2]
                A += np.einsum("q,qi,qj->ij", np.maximum(on, 0), mesh.Uf[f], mesh.Uf[f])
                sym += 0.5 * np.einsum("q,qi,qj->ij", np.abs(on), mesh.Uf[f], mesh.Uf[f])
            assert np.abs(0.5 * (A + A.T) - sym).max() < 1e-13
            assert np.linalg.eigvalsh(sym).min() > 0


def test_perturbation_keeps_boundary():
    v = np.linspace(0, 1, 5)
    c0 = structured_ctrl(v, v, 2)
    c1 = structured_ctrl(v, v, 2, sine_perturbation(0.05))
    edge = np.zeros(c0.shape[:2], dtype=bool)
    edge[0, :] = edge[-1, :] = edge[:, 0] = edge[:, -1] = True
    assert np.abs(c1[edge] - c0[edge]).max() < 1e-15
    assert np.abs(c1[~edge] - c0[~edge]).max() > 0.01
