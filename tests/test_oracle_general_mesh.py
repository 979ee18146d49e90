"""Pins of the oracle on meshes given element by element (no GPU).

* Local numbering does not change the method: the structured curved mesh
  with each element's local frame turned by a random number of quarter turns
  (so that neighbours meet with every face pairing and with reversed face
  parameterisations) gives the same sweep, IP operator, fixed right-hand side
  and converged SMM flux as the structured mesh, node for node, to rounding.
* An unstructured mesh (a rotated inner square joined to the outer square by
  four quadrilaterals, cut k x k; vertices shared by three elements):
  the infinite-medium fixed point varphi = 4 pi q / sigma_a (isotropic inflow
  given per boundary attribute), the linearly anisotropic patch solution
  (affine a and b; the elements are bilinear, so m <= p reproduces them),
  and O(h^{p+1}) manufactured-solution convergence under k -> 2k -> 4k.
* Inflow per boundary attribute reaches the faces of that attribute only.
* An explicit angular set (a product Gauss-Legendre x azimuth set, not
  level-symmetric): the infinite-medium fixed point still holds (T is a
  nonzero constant, so its divergence and jumps vanish, and beta = 0 by the
  definition of E_b0).
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import fem, smm, transport
from workloads import (config_curved_mms, general_workload, inner_square_mesh, mms_phi, mms_psi,
                       product_quadrature_2d, rotate_elements)


def _node_perm(m0, m1):
    """DOF t of mesh m1 sits where DOF idx[t] of m0 sits (same element)."""
    ne, n, _ = m0.xnode.shape
    idx = np.zeros(ne * n, dtype=int)
    for K in range(ne):
        d, j = cKDTree(m0.xnode[K]).query(m1.xnode[K])
        assert d.max() < 1e-13
        idx[K * n:(K + 1) * n] = K * n + j
    return idx


def rotated_curved(n=4, p=2, sn=4, amp=0.06, seed=3):
    wl = config_curved_mms(n, p, sn, amplitude=amp)
    ctrl_e, nbr = fem.structured_elements(wl.ctrl, n, n, p)
    rot = np.random.default_rng(seed).integers(0, 4, n * n)
    ce, nb = rotate_elements(ctrl_e, nbr, rot)
    return wl, general_workload("rotated", ce, nb, p, p, sn, wl.sigma_t, wl.sigma_s, q_fn=wl.q_fn,
                                inflow=wl.inflow)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_local_numbering_does_not_matter(p):
    wl, gw = rotated_curved(p=p)
    pr0, pr1 = smm.make_problem(wl), smm.make_problem(gw)
    assert pr1.mesh.flip.any() and not pr0.mesh.flip.any()
    assert set(np.unique(pr1.mesh.nbr_face[pr1.mesh.nbr >= 0])) == {0, 1, 2, 3}
    idx = _node_perm(pr0.mesh, pr1.mesh)
    xa = pr0.mesh.xnode.reshape(-1, 2)
    S = (1 + xa[:, 0] ** 2 + 0.3 * xa[:, 1]).reshape(pr0.ne, pr0.n)
    psi0 = transport.sweep(pr0.mesh, pr0.omega, pr0.sigma_t, S, pr0.psibar)
    psi1 = transport.sweep(pr1.mesh, pr1.omega, pr1.sigma_t, S.reshape(-1)[idx].reshape(pr0.ne, pr0.n),
                           pr1.psibar)
    nd = len(pr0.w)
    assert np.abs(psi1.reshape(nd, -1) - psi0.reshape(nd, -1)[:, idx]).max() < 1e-13 * np.abs(psi0).max()
    A0, A1 = smm.ip_matrix(pr0).toarray(), smm.ip_matrix(pr1).toarray()
    assert np.abs(A1 - A0[np.ix_(idx, idx)]).max() < 1e-13 * np.abs(A0).max()
    b0, b1 = smm.rhs_fixed(pr0), smm.rhs_fixed(pr1)
    assert np.abs(b1 - b0[idx]).max() < 1e-13 * np.abs(b0).max()
    x0, i0 = smm.solve(pr0, tol=1e-13)
    x1, i1 = smm.solve(pr1, tol=1e-13)
    assert i0["converged"] and i1["converged"]
    assert np.abs(x1 - x0[idx]).max() < 1e-12 * np.abs(x0).max()


def test_unstructured_infinite_medium():
    ce, nb, at = inner_square_mesh(2, 2, displace=lambda x, y: (0.03 * np.sin(np.pi * x) * np.sin(np.pi * y),
                                                                 -0.02 * np.sin(np.pi * x) * np.sin(np.pi * y)))
    ne = len(ce)
    st, ss, q = 2.0, 1.5, 1.0
    gw = general_workload("inner", ce, nb, 2, 2, 6, np.full(ne, st), np.full(ne, ss), bdr_attr=at,
                          q_elem=np.full(ne, q), inflow=("attr", [q / (st - ss)] * 4))
    prob = smm.make_problem(gw)
    assert abs(prob.mesh.area.sum() - 1.0) < 1e-13
    X = np.full(ne * prob.n, 4 * np.pi * q / (st - ss))
    lag = np.full((len(prob.w), ne, prob.n), q / (st - ss))
    G, ex = smm.apply_G(prob, X, psi_lag=lag)
    assert np.abs(G - X).max() < 1e-13 * X.max()
    assert np.abs(ex["T"]).max() < 1e-13 and np.abs(ex["beta"]).max() < 1e-13
    x, info = smm.solve(prob, tol=1e-12)
    assert info["converged"] and np.abs(x - X).max() < 1e-10 * X.max()


def test_unstructured_patch_linear_anisotropy():
    a = lambda x, y: 1 + 0.3 * x + 0.2 * y
    bx = lambda x, y: 0.2 + 0.1 * x - 0.3 * y
    by = lambda x, y: -0.1 + 0.2 * x + 0.1 * y
    st, ss = 2.0, 1.2
    psi = lambda x, y, ox, oy: a(x, y) + ox * bx(x, y) + oy * by(x, y)
    # Omega.grad psi = Omega_x (0.3 + Omega_x 0.1 + Omega_y 0.2) + Omega_y (0.2 - Omega_x 0.3 + Omega_y 0.1)
    q = lambda x, y, ox, oy: (ox * (0.3 + 0.1 * ox + 0.2 * oy) + oy * (0.2 - 0.3 * ox + 0.1 * oy)
                              + st * psi(x, y, ox, oy) - ss * a(x, y))
    ce, nb, at = inner_square_mesh(2, 1)
    ne = len(ce)
    gw = general_workload("inner", ce, nb, 1, 2, 6, np.full(ne, st), np.full(ne, ss), bdr_attr=at, q_fn=q,
                          inflow=("fn", psi))
    prob = smm.make_problem(gw)
    x, info = smm.solve(prob, tol=1e-14, max_it=100)
    xn = prob.mesh.xnode
    ex = 4 * np.pi * a(xn[..., 0], xn[..., 1]).reshape(-1)
    assert info["converged"]
    assert np.abs(x - ex).max() < 1e-12 * ex.max()
    for d in (0, 7, 20):
        o = prob.omega[d]
        assert np.abs(info["psi"][d] - psi(xn[..., 0], xn[..., 1], o[0], o[1])).max() < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_unstructured_mms_order(p):
    bump = lambda x, y: (0.03 * np.sin(np.pi * x) * np.sin(2 * np.pi * y), 0.02 * np.sin(2 * np.pi * x) * np.sin(np.pi * y))
    errs = []
    for k in (1, 2, 4):
        ce, nb, at = inner_square_mesh(k, p, displace=bump)
        ne = len(ce)
        wl = config_curved_mms(2, p, 4)
        gw = general_workload("inner", ce, nb, p, p, 4, np.full(ne, 1.0), np.full(ne, 0.5), bdr_attr=at,
                              q_fn=wl.q_fn, inflow=("fn", lambda x, y, ox, oy: mms_psi(x, y, ox)))
        prob = smm.make_problem(gw)
        x, info = smm.solve(prob, tol=1e-11, max_it=60)
        assert info["converged"]
        errs.append(fem.l2_error(prob.mesh, x.reshape(prob.ne, prob.n), mms_phi))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > p + 1 - 0.2, orders


def test_inflow_per_boundary_attribute():
    ce, nb, at = inner_square_mesh(2, 1)
    ne = len(ce)
    gw = general_workload("inner", ce, nb, 1, 1, 4, np.ones(ne), np.zeros(ne), bdr_attr=at,
                          q_elem=np.zeros(ne), inflow=("attr", [1.0, 2.0, 3.0, 4.0]))
    prob = smm.make_problem(gw)
    for b, (K, f) in enumerate(prob.mesh.bfaces):
        assert np.all(prob.psibar[b] == 1.0 + at[K, f])
        mid = prob.mesh.xf[K, f].mean(axis=0)
        side = [abs(mid[1]), abs(mid[0] - 1), abs(mid[1] - 1), abs(mid[0])]
        assert side[at[K, f]] < 1e-12


def test_explicit_quadrature_infinite_medium():
    om, w = product_quadrature_2d(1, 8)              # one polar point: mu^2 not integrated exactly
    assert abs(w.sum() - 4 * np.pi) < 1e-13 and np.allclose(np.linalg.norm(om, axis=1), 1)
    P = np.einsum("d,da,db->ab", w, om[:, :2], om[:, :2])
    assert abs(P[0, 0] - 4 * np.pi / 3) > 1e-3          # not level-symmetric: T != 0
    wl = config_curved_mms(4, 2, 4)
    ne = wl.n_elem
    st, ss, q = 2.0, 1.5, 1.0
    wl.sigma_t, wl.sigma_s, wl.q_elem, wl.q_fn = np.full(ne, st), np.full(ne, ss), np.full(ne, q), None
    wl.inflow = ("iso", q / (st - ss))
    wl.quad = (om, w)
    prob = smm.make_problem(wl)
    X = np.full(ne * prob.n, 4 * np.pi * q / (st - ss))
    lag = np.full((len(w), ne, prob.n), q / (st - ss))
    G, ex = smm.apply_G(prob, X, psi_lag=lag)
    assert np.abs(ex["T"]).max() > 1e-3
    assert np.abs(G - X).max() < 1e-12 * X.max()
