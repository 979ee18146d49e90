"""Pins of the oracle's sweep and closures (no GPU).

* Element balance: testing the DG equations with u = 1 gives, per element
  and direction, oint (Omega.n) psi_hat + sigma_t int psi = int S.
* Pure absorber with inflow exp(-sigma_t (Omega.x)/|Omega_perp|^2): the exact
  solution is that function everywhere (attenuation along characteristics);
  one sweep converges at order p+1 in L2.
* The ordered sweep equals a simultaneous solve of the globally assembled
  upwind DG system of each direction (built here independently of the
  element ordering); on a curved mesh the lagged sweep, repeated, converges
  to that same global solution.
* Closures: T and beta vanish identically for every linearly anisotropic
  psi (Sec. 2.2 and Sec. 4: the discrete definitions with E_b0 make the
  boundary factor vanish for a linear-in-angle discrete solution).
"""
import numpy as np
import pytest

from oracle import fem, smm, transport
from workloads import absorber_inflow, config_curved_mms, config_plain


def _balance(prob, psi, S):
    mesh = prob.mesh
    worst = 0.0
    for d, om in enumerate(prob.omega):
        for K in range(prob.ne):
            tot = prob.sigma_t[K] * mesh.M[K].sum(axis=0) @ psi[d, K]
            for f in range(4):
                on = mesh.nds[K, f] @ om[:2]
                own = mesh.Uf[f] @ psi[d, K]
                N = mesh.nbr[K, f]
                if N >= 0:
                    up = mesh.Uf[fem.OPPOSITE[f]] @ psi[d, N]
                else:
                    up = prob.psibar[mesh.bface_id[K, f], :, d] if prob.psibar is not None else 0 * own
                tot += np.sum(np.where(on > 0, on * own, on * up))
            src = mesh.M[K].sum(axis=0) @ S[K]
            worst = max(worst, abs(tot - src) / max(abs(src), 1e-300))
    return worst


def test_sweep_balance():
    wl = config_plain(n=4, p=2, sn=6)
    wl.inflow = ("iso", 0.7)
    prob = smm.make_problem(wl)
    rng = np.random.default_rng(1)
    S = rng.uniform(0.5, 1.5, (prob.ne, prob.n))
    psi = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar)
    assert _balance(prob, psi, S) < 1e-13


@pytest.mark.parametrize("p", [1, 2])
def test_pure_absorber_order(p):
    st = 1.5
    f = absorber_inflow(st)
    errs = []
    for n in (4, 8, 16):
        wl = config_plain(n=n, p=p, sn=4)
        wl.sigma_t[:] = st
        wl.sigma_s[:] = 0.0
        wl.q_elem[:] = 0.0
        wl.inflow = ("fn", f)
        prob = smm.make_problem(wl)
        psi = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, np.zeros((prob.ne, prob.n)), prob.psibar)
        e2 = sum(fem.l2_error(prob.mesh, psi[d], lambda x, y, o=o: f(x, y, o[0], o[1])) ** 2
                 for d, o in enumerate(prob.omega))
        errs.append(np.sqrt(e2))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > p + 1 - 0.15, orders


def _global_dg_solve(prob, S, d):
    """Assemble every element's upwind equations for direction d into one
    block system (inflow couplings as off-diagonal blocks) and solve it."""
    mesh, ne, n = prob.mesh, prob.ne, prob.n
    om = prob.omega[d]
    A = np.zeros((ne * n, ne * n))
    b = np.zeros(ne * n)
    for K in range(ne):
        sl = slice(K * n, (K + 1) * n)
        A[sl, sl] += prob.sigma_t[K] * mesh.M[K] - om[0] * mesh.Gx[K] - om[1] * mesh.Gy[K]
        b[sl] += mesh.M[K] @ S[K]
        for f in range(4):
            on = mesh.nds[K, f] @ om[:2]
            A[sl, sl] += np.einsum("q,qi,qj->ij", np.maximum(on, 0), mesh.Uf[f], mesh.Uf[f])
            N = mesh.nbr[K, f]
            neg = np.maximum(-on, 0)
            if N >= 0:
                sn = slice(N * n, (N + 1) * n)
                A[sl, sn] -= np.einsum("q,qi,qj->ij", neg, mesh.Uf[f], mesh.Uf[fem.OPPOSITE[f]])
            elif prob.psibar is not None:
                b[sl] += np.einsum("q,qi,q->i", neg, mesh.Uf[f], prob.psibar[mesh.bface_id[K, f], :, d])
    return np.linalg.solve(A, b).reshape(ne, n)


def test_sweep_equals_global_solve_straight():
    wl = config_plain(n=4, p=2, sn=4)
    wl.inflow = ("iso", 0.3)
    prob = smm.make_problem(wl)
    rng = np.random.default_rng(2)
    S = rng.uniform(-1, 1, (prob.ne, prob.n))
    psi = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar)
    for d in range(len(prob.w)):
        ref = _global_dg_solve(prob, S, d)
        assert np.abs(psi[d] - ref).max() < 1e-12 * np.abs(ref).max()


def test_lagged_sweep_converges_to_global_solve_curved():
    # strong perturbation so that pointwise inflow disagrees with the chord graph
    wl = config_curved_mms(n=4, p=2, sn=8, amplitude=0.09)
    prob = smm.make_problem(wl)
    S = np.ones((prob.ne, prob.n))
    lagged_dirs = []
    for d, om in enumerate(prob.omega):
        up, _ = transport.sweep_graph(prob.mesh, om)
        on = np.einsum("kfqa,a->kfq", prob.mesh.nds, om[:2])
        inter = prob.mesh.nbr >= 0
        if np.any(inter[..., None] & ~up[..., None] & (on < 0)):
            lagged_dirs.append(d)
    assert lagged_dirs, "test mesh must exercise lagged couplings"
    psi = None
    for _ in range(60):
        psi = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar, psi)
    for d in lagged_dirs[:4]:
        ref = _global_dg_solve(prob, S, d)
        assert np.abs(psi[d] - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("curved", [False, True])
def test_closures_vanish_for_linear_anisotropy(curved):
    wl = config_curved_mms(n=3, p=2, sn=8) if curved else config_plain(n=3, p=2, sn=10)
    prob = smm.make_problem(wl)
    rng = np.random.default_rng(3)
    a = rng.normal(size=(prob.ne, prob.n))
    bx = rng.normal(size=(prob.ne, prob.n))
    by = rng.normal(size=(prob.ne, prob.n))
    psi = (a[None] + prob.omega[:, 0, None, None] * bx[None]
           + prob.omega[:, 1, None, None] * by[None])
    phi, J, T, beta = smm.closures(prob, psi)
    assert np.abs(phi - 4 * np.pi * a).max() < 1e-12
    assert np.abs(J[0] - 4 * np.pi / 3 * bx).max() < 1e-12
    assert np.abs(T).max() < 1e-12
    assert np.abs(beta).max() < 1e-12
    # and a quadratic-in-angle psi gives a non-zero correction
    psi2 = psi + prob.omega[:, 0, None, None] ** 2 * a[None]
    _, _, T2, beta2 = smm.closures(prob, psi2)
    assert np.abs(T2).max() > 1e-2 and np.abs(beta2).max() > 1e-2
