"""Two-level preconditioner set-up (host only, no GPU).

* Level 0 is the Galerkin operator P0^T A P0 of the continuous bilinear space
  on the element vertices, with A the typed IP matrix and P0 the bilinear
  interpolation at the Gauss-Lobatto nodes, both built here independently;
  the product is a 9-point stencil (entries farther out vanish).
* Level 1 is the Galerkin operator of level 0 under linear interpolation from
  every other vertex (the last vertex always kept), odd and even grids.
* The level operators are symmetric positive definite.
"""
import numpy as np
import pytest

from oracle.quadrature import gauss_lobatto_unit
from workloads import config_blobs, config_plain

L = pytest.importorskip("paper_2304_07386_amd")


@pytest.fixture(scope="module")
def hctx():
    return L.smm_ctx_create(-1)


def _stencil_dense(A9, nx, ny):
    nv = nx * ny
    D = np.zeros((nv, nv))
    for v in range(nv):
        ix, iy = v % nx, v // nx
        for k in range(9):
            jx, jy = ix + k % 3 - 1, iy + k // 3 - 1
            if 0 <= jx < nx and 0 <= jy < ny:
                D[v, jy * nx + jx] += A9[k, v]
    return D


def _p0(nx, ny, p):
    nb = p + 1
    x = gauss_lobatto_unit(p)
    n = nb * nb
    vx = nx + 1
    P = np.zeros((nx * ny * n, vx * (ny + 1)))
    for K in range(nx * ny):
        ex, ey = K % nx, K // nx
        for b in range(nb):
            for a in range(nb):
                row = K * n + a + nb * b
                for cy in (0, 1):
                    for cx in (0, 1):
                        w = (x[a] if cx else 1 - x[a]) * (x[b] if cy else 1 - x[b])
                        P[row, (ey + cy) * vx + ex + cx] += w
    return P


def _p1d(nf):
    if nf <= 3:
        return np.eye(nf)
    coarse = list(range(0, nf, 2))
    if coarse[-1] != nf - 1:
        coarse.append(nf - 1)
    P = np.zeros((nf, len(coarse)))
    for i in range(nf):
        if i in coarse:
            P[i, coarse.index(i)] = 1.0
        else:
            P[i, coarse.index(i - 1)] = 0.5
            P[i, coarse.index(i + 1)] = 0.5
    return P


@pytest.mark.parametrize("wl", [config_plain(5, 2, 4), config_blobs(20000, n=6, p=2, sn=4), config_plain(4, 3, 4)],
                         ids=["plain5p2", "blobs6p2", "plain4p3"])
def test_galerkin_levels(hctx, wl):
    p = L.problem_from_workload(hctx, wl)
    A, Cm, b = L.smm_debug_typed_dense(p)
    P0 = _p0(wl.nx, wl.ny, wl.p)
    Ac = P0.T @ A @ P0
    A9, vx, vy = L.smm_debug_mg_level(p, 0)
    assert (vx, vy) == (wl.nx + 1, wl.ny + 1)
    D0 = _stencil_dense(A9, vx, vy)
    scale = np.abs(Ac).max()
    assert np.abs(D0 - Ac).max() < 1e-12 * scale
    assert np.allclose(D0, D0.T, atol=1e-13 * scale)
    assert np.linalg.eigvalsh(D0).min() > 0
    if max(vx, vy) > 3:
        P1 = np.kron(_p1d(vy), _p1d(vx))
        A1ref = P1.T @ D0 @ P1
        A9b, cx, cy = L.smm_debug_mg_level(p, 1)
        assert cx * cy == P1.shape[1]
        D1 = _stencil_dense(A9b, cx, cy)
        assert np.abs(D1 - A1ref).max() < 1e-12 * scale
        assert np.linalg.eigvalsh(D1).min() > 0


@pytest.mark.parametrize("k", range(4))
def test_cg_galerkin_levels(hctx, k):
    """The CG system's coarse operator is P1^T A_c P1 with A_c the oracle's
    continuous moment matrix (Sec. 5.1) and P1 the bilinear vertex
    interpolation at its continuous nodes, obtained here from the DG-node
    interpolation P0 = P_c P1 (an interpolated bilinear function is
    continuous, so the least-squares solve is exact)."""
    from oracle import smm as osmm
    from workloads import config_channel, config_curved_mms
    wl = [config_plain(5, 2, 4), config_blobs(20003, n=6, p=3, sn=4), config_curved_mms(n=4, p=2, sn=4),
          config_channel(n=7, p=2, sn=4, side=1.3)][k]
    pr = osmm.make_problem(wl, disc="cg")
    Po = osmm.cg_space(pr.mesh)
    Po = Po.toarray() if hasattr(Po, "toarray") else np.asarray(Po)
    Ao = osmm.cg_matrix(pr)
    Ao = Ao.toarray() if hasattr(Ao, "toarray") else np.asarray(Ao)
    P0 = _p0(wl.nx, wl.ny, wl.p)
    P1 = np.linalg.solve(Po.T @ Po, Po.T @ P0)
    assert np.abs(Po @ P1 - P0).max() < 1e-13
    Ac = P1.T @ Ao @ P1
    p = L.problem_from_workload(hctx, wl, q=pr.q, psibar=pr.psibar)
    A9, vx, vy = L.smm_debug_cg_mg_level(p, 0)
    assert (vx, vy) == (wl.nx + 1, wl.ny + 1)
    D0 = _stencil_dense(A9, vx, vy)
    scale = np.abs(Ac).max()
    assert np.abs(D0 - Ac).max() < 1e-12 * scale
    assert np.linalg.eigvalsh(D0).min() > 0
    if max(vx, vy) > 3:
        P1c = np.kron(_p1d(vy), _p1d(vx))
        A9b, cx, cy = L.smm_debug_cg_mg_level(p, 1)
        D1 = _stencil_dense(A9b, cx, cy)
        assert np.abs(D1 - P1c.T @ D0 @ P1c).max() < 1e-12 * scale
    with pytest.raises(L.SmmError):
        L.smm_debug_cg_mg_level(p, 99)
