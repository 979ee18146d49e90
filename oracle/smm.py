"""Interior-penalty SMM moment system and the SMM fixed point (oracle).

* IP SMM discretisation (eq. ipsmm, Sec. 5.1): a symmetric interior-penalty
  diffusion operator with Marshak boundary term E_b0 and penalty
  kappa = {(p+1)^2 / (sigma_t h)} (Sec. 6), h = |K|^(1/2), on the left; the
  fixed-source terms and the transport-dependent corrections (beta on the
  boundary, the correction tensor T through its broken divergence,
  eq. broken_Tdiv) on the right.
* The reduced fixed point X = G(X), G(X) = D^{-1} b(L^{-1}(sigma_s/(4 pi) X + q))
  (eq. moment:smm_fp), iterated as X^{k+1} = G(X^k) (eq. fixed-point) until
  the relative max-norm of the change falls below a tolerance.
* The continuous finite element (CG) SMM moment system (Sec. 5.1): the same
  forms with test and trial functions restricted to the continuous space V_p.
  Jumps of V_p functions vanish on interior faces, so every interior-face term
  that carries [u] or [varphi] drops out; the term {grad u / sigma_t}.[T n]
  stays because T is discontinuous.  Selected by ``disc="cg"``.
* Extra modes used only to pin the oracle: plain source iteration on the
  transport equation, a Krylov solve of the DG S_N system with scattering, and
  the fixed point found as the solution of the linear system X = G(X).

The moment solve D^{-1} b is a sparse direct solve (its plain definition); the
paper's CG reaches the same vector.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, transport
from .quadrature import level_symmetric_2d


@dataclass
class OracleProblem:
    mesh: fem.Mesh
    omega: np.ndarray
    w: np.ndarray
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    q: np.ndarray                 # nodal source per steradian: [ne, n] or [nd, ne, n]
    psibar: np.ndarray | None     # [n_bf, nq, nd] or None (vacuum)
    kappa_scale: float = 1.0
    disc: str = "ip"              # moment discretisation: "ip" (Y_p) or "cg" (V_p)
    tiles: tuple | None = None    # (tx, ty): parallel block Jacobi sweep over tiles
    cache: dict = field(default_factory=dict)

    @property
    def block(self):
        """Block id per element for the block Jacobi sweep, or None."""
        if self.tiles is None:
            return None
        return transport.block_ids(self.mesh, *self.tiles)

    @property
    def ne(self):
        return self.mesh.nx * self.mesh.ny

    @property
    def n(self):
        return (self.mesh.p + 1) ** 2


def make_problem(wl, kappa_scale: float = 1.0, disc: str = "ip", tiles=None) -> OracleProblem:
    """Build the oracle's view of a workload (mesh data, S_N set, nodal
    source, inflow at boundary face points).  ``disc`` picks the moment
    discretisation: "ip" (interior penalty, Y_p) or "cg" (continuous, V_p);
    ``tiles`` = (tx, ty) replaces the sweep by the parallel block Jacobi
    sweep over tiles of tx x ty elements (Sec. 6.5)."""
    if disc not in ("ip", "cg"):
        raise ValueError(disc)
    if getattr(wl, "elem_ctrl", None) is not None:
        mesh = fem.build_mesh_general(wl.elem_ctrl, wl.nbr, wl.m, wl.p, wl.bdr_attr)
    else:
        mesh = fem.build_mesh(wl.ctrl, wl.nx, wl.ny, wl.m, wl.p)
    if getattr(wl, "quad", None) is not None:
        omega, w = np.asarray(wl.quad[0], float), np.asarray(wl.quad[1], float)
    else:
        omega, w = level_symmetric_2d(wl.sn)
    ne, n = mesh.nx * mesh.ny, (wl.p + 1) ** 2
    if wl.q_fn is not None:
        xn = mesh.xnode
        q = np.stack([wl.q_fn(xn[..., 0], xn[..., 1], om[0], om[1]) for om in omega])
    else:
        q = np.repeat(np.asarray(wl.q_elem, dtype=float)[:, None], n, axis=1)
    psibar = transport.inflow_at_points(mesh, omega, wl.inflow)
    return OracleProblem(mesh, omega, w, np.asarray(wl.sigma_t, float),
                         np.asarray(wl.sigma_s, float), q, psibar, kappa_scale, disc,
                         None if tiles is None else (int(tiles[0]), int(tiles[1])))


# ----------------------------------------------------------------------------
# IP bilinear form (left-hand side of eq. ipsmm)
# ----------------------------------------------------------------------------

def _interior_faces(mesh):
    """(K1, f1, K2, f2) for each interior face once, K1 < K2 (on a structured
    grid: K1 below or left of K2); the normal of K1's face points from K1 to
    K2, and the face points are K1's."""
    out = []
    for K in range(len(mesh.nbr)):
        for f in range(4):
            N = mesh.nbr[K, f]
            if N > K:
                out.append((K, f, N, int(mesh.nbr_face[K, f])))
    return out


def _side2(mesh, K1, f1, K2, f2):
    """Basis values [q, n] and physical gradients [q, n, 2] of K2 on the
    shared face, at K1's face points."""
    U, G = mesh.Uf[f2], mesh.gradUf[K2, f2]
    return (U[::-1], G[::-1]) if mesh.flip[K1, f1] else (U, G)


def penalty(prob: OracleProblem, K1: int, K2: int) -> float:
    """kappa = average over the two sides of (p+1)^2 / (sigma_t h)."""
    p = prob.mesh.p
    h1, h2 = np.sqrt(prob.mesh.area[K1]), np.sqrt(prob.mesh.area[K2])
    k = 0.5 * ((p + 1) ** 2 / (prob.sigma_t[K1] * h1) + (p + 1) ** 2 / (prob.sigma_t[K2] * h2))
    return prob.kappa_scale * k


def ip_matrix(prob: OracleProblem) -> sp.csr_matrix:
    """Assemble the IP diffusion operator (fixed across iterations)."""
    mesh, ne, n = prob.mesh, prob.ne, prob.n
    D = 1.0 / (3.0 * prob.sigma_t)
    sa = prob.sigma_t - prob.sigma_s
    rows, cols, vals = [], [], []

    def add(Ka, Kb, blk):
        r = Ka * n + np.arange(n)
        c = Kb * n + np.arange(n)
        R, C = np.meshgrid(r, c, indexing="ij")
        rows.append(R.ravel()); cols.append(C.ravel()); vals.append(blk.ravel())

    for K in range(ne):
        g = mesh.gradU[K]                                   # [Q, n, 2]
        blk = D[K] * np.einsum("q,qia,qja->ij", mesh.wJ[K], g, g)
        blk += sa[K] * mesh.M[K]
        for f in range(4):
            if mesh.nbr[K, f] < 0:
                nh = mesh.nhat[K, f]
                e = np.array([np.sum(prob.w * np.abs(prob.omega[:, 0] * a + prob.omega[:, 1] * b))
                              / np.sum(prob.w) for a, b in nh])
                blk += np.einsum("q,qi,qj->ij", mesh.dsw[K, f] * e, mesh.Uf[f], mesh.Uf[f])
        add(K, K, blk)

    for K1, f1, K2, f2 in _interior_faces(mesh):
        kap = penalty(prob, K1, K2)
        nh = mesh.nhat[K1, f1]                              # [q, 2]
        dsw = mesh.dsw[K1, f1]
        U2, G2 = _side2(mesh, K1, f1, K2, f2)
        side = {0: (K1, mesh.Uf[f1], mesh.gradUf[K1, f1], 1.0),
                1: (K2, U2, G2, -1.0)}
        for su in (0, 1):
            Ku, Uu, Gu, sgu = side[su]
            dnu = np.einsum("qia,qa->qi", Gu, nh)          # grad u . n
            for sv in (0, 1):
                Kv, Uv, Gv, sgv = side[sv]
                dnv = np.einsum("qja,qa->qj", Gv, nh)
                blk = (kap * sgu * sgv * np.einsum("q,qi,qj->ij", dsw, Uu, Uv)
                       - sgu * 0.5 * D[Kv] * np.einsum("q,qi,qj->ij", dsw, Uu, dnv)
                       - 0.5 * D[Ku] * sgv * np.einsum("q,qi,qj->ij", dsw, dnu, Uv))
                add(Ku, Kv, blk)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ne * n, ne * n))
    A.sum_duplicates()
    return A


# ----------------------------------------------------------------------------
# Right-hand side of eq. ipsmm
# ----------------------------------------------------------------------------

def source_moments(prob: OracleProblem):
    """Q0 = sum w q_d and Q1 = sum w Omega q_d at the nodes."""
    q = prob.q
    if q.ndim == 2:
        Q0 = q * np.sum(prob.w)
        Q1 = np.stack([q * np.sum(prob.w * prob.omega[:, a]) for a in range(2)])
    else:
        Q0 = np.einsum("d,dkn->kn", prob.w, q)
        Q1 = np.stack([np.einsum("d,dkn->kn", prob.w * prob.omega[:, a], q) for a in range(2)])
    return Q0, Q1


def rhs_fixed(prob: OracleProblem) -> np.ndarray:
    """Fixed part: int u Q0 + int grad u . Q1/sigma_t
    - int_{Gamma0} [u] {Q1.n/sigma_t} - int_{Gamma_b} 2 u J_in."""
    mesh, ne, n = prob.mesh, prob.ne, prob.n
    Q0, Q1 = source_moments(prob)
    jin = transport.inflow_current(mesh, prob.omega, prob.w, prob.psibar)
    b = np.zeros((ne, n))
    st = prob.sigma_t
    for K in range(ne):
        q0 = mesh.U @ Q0[K]
        q1 = np.stack([mesh.U @ Q1[0, K], mesh.U @ Q1[1, K]], axis=1)   # [Q, 2]
        b[K] += np.einsum("q,qi,q->i", mesh.wJ[K], mesh.U, q0)
        b[K] += np.einsum("q,qia,qa->i", mesh.wJ[K], mesh.gradU[K], q1) / st[K]
        for f in range(4):
            bf = mesh.bface_id[K, f]
            if bf >= 0:
                b[K] -= 2.0 * np.einsum("q,qi,q->i", mesh.dsw[K, f], mesh.Uf[f], jin[bf])
    for K1, f1, K2, f2 in _interior_faces(mesh):
        nh, dsw = mesh.nhat[K1, f1], mesh.dsw[K1, f1]
        U2, _ = _side2(mesh, K1, f1, K2, f2)
        q1a = np.stack([mesh.Uf[f1] @ Q1[0, K1], mesh.Uf[f1] @ Q1[1, K1]], axis=1)
        q1b = np.stack([U2 @ Q1[0, K2], U2 @ Q1[1, K2]], axis=1)
        avg = 0.5 * (np.sum(q1a * nh, 1) / st[K1] + np.sum(q1b * nh, 1) / st[K2])
        b[K1] -= np.einsum("q,qi,q->i", dsw, mesh.Uf[f1], avg)
        b[K2] += np.einsum("q,qi,q->i", dsw, U2, avg)
    return b.reshape(-1)


def _divT(grad, T):
    """Broken divergence of the nodal tensor field T (xx, xy, yy) of one
    element at points with basis gradients grad [Q, n, 2]:
    (d_x Txx + d_y Txy, d_x Txy + d_y Tyy)."""
    dx = lambda c: grad[:, :, 0] @ c
    dy = lambda c: grad[:, :, 1] @ c
    return np.stack([dx(T[0]) + dy(T[1]), dx(T[1]) + dy(T[2])], axis=1)


def rhs_correction(prob: OracleProblem, T: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Transport-dependent part: - int_{Gamma_b} u beta
    + int_{Gamma0} [u] {(1/sigma_t) div_h T . n} + int_{Gamma0} {grad_h u / sigma_t} . [T n]
    - int grad_h u . (1/sigma_t) div_h T."""
    mesh, ne, n = prob.mesh, prob.ne, prob.n
    st = prob.sigma_t
    b = np.zeros((ne, n))
    for K in range(ne):
        dT = _divT(mesh.gradU[K], T[:, K, :])
        b[K] -= np.einsum("q,qia,qa->i", mesh.wJ[K], mesh.gradU[K], dT) / st[K]
        for f in range(4):
            bf = mesh.bface_id[K, f]
            if bf >= 0:
                b[K] -= np.einsum("q,qi,q->i", mesh.dsw[K, f], mesh.Uf[f], beta[bf])
    for K1, f1, K2, f2 in _interior_faces(mesh):
        nh, dsw = mesh.nhat[K1, f1], mesh.dsw[K1, f1]
        U2, G2 = _side2(mesh, K1, f1, K2, f2)
        d1 = _divT(mesh.gradUf[K1, f1], T[:, K1, :])
        d2 = _divT(G2, T[:, K2, :])
        avg = 0.5 * (np.sum(d1 * nh, 1) / st[K1] + np.sum(d2 * nh, 1) / st[K2])
        t1 = np.stack([mesh.Uf[f1] @ T[c, K1] for c in range(3)], axis=1)   # [q, 3]
        t2 = np.stack([U2 @ T[c, K2] for c in range(3)], axis=1)
        tn = lambda t: np.stack([t[:, 0] * nh[:, 0] + t[:, 1] * nh[:, 1],
                                 t[:, 1] * nh[:, 0] + t[:, 2] * nh[:, 1]], axis=1)
        jump = tn(t1) - tn(t2)                                            # [T n]
        b[K1] += np.einsum("q,qi,q->i", dsw, mesh.Uf[f1], avg)
        b[K2] -= np.einsum("q,qi,q->i", dsw, U2, avg)
        b[K1] += 0.5 * np.einsum("q,qia,qa->i", dsw, mesh.gradUf[K1, f1], jump) / st[K1]
        b[K2] += 0.5 * np.einsum("q,qia,qa->i", dsw, G2, jump) / st[K2]
    return b.reshape(-1)


# ----------------------------------------------------------------------------
# Continuous (CG) moment system: test and trial spaces V_p (Sec. 5.1)
# ----------------------------------------------------------------------------

def cg_space(mesh) -> sp.csr_matrix:
    """P_c [ne*n, nc]: the DG nodal values of the continuous function with
    unknowns c.  V_p is the subspace of Y_p whose members are continuous
    (Sec. 3.3); with a nodal Gauss-Lobatto basis a member of Y_p is
    continuous exactly when the DG nodes of neighbouring elements that sit at
    the same point carry the same value, so V_p has one unknown per distinct
    node position.  The positions are matched geometrically (within 1e-10 of
    the domain size)."""
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    x = mesh.xnode.reshape(-1, 2)
    N = len(x)
    tol = 1e-10 * max(np.ptp(x[:, 0]), np.ptp(x[:, 1]), 1e-300)
    pairs = cKDTree(x).query_pairs(tol, output_type="ndarray")
    G = sp.csr_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(N, N))
    nc, label = connected_components(G, directed=False)
    return sp.csr_matrix((np.ones(N), (np.arange(N), label)), shape=(N, nc))


def cg_matrix(prob: OracleProblem) -> sp.csr_matrix:
    """The CG SMM bilinear form on V_p: the IP form with both arguments
    restricted to V_p, A_c = P_c^T A_IP P_c."""
    Pc = cg_space(prob.mesh)
    return (Pc.T @ ip_matrix(prob) @ Pc).tocsr()


# ----------------------------------------------------------------------------
# Fixed point
# ----------------------------------------------------------------------------

def _lhs_factor(prob: OracleProblem):
    """Factorisation of the moment system of the problem's discretisation and
    its fixed right-hand side (in Y_p).  The moment solve maps a Y_p
    right-hand side b to the DG vector of the solution: A_IP^-1 b for IP,
    P_c (P_c^T A_IP P_c)^-1 P_c^T b for CG."""
    if "lu" not in prob.cache:
        if prob.disc == "cg":
            Pc = cg_space(prob.mesh)
            A = cg_matrix(prob).tocsc()
            lu = spla.splu(A)
            prob.cache["lu"] = _Restricted(lu, Pc)
        else:
            A = ip_matrix(prob).tocsc()
            prob.cache["lu"] = spla.splu(A)
        prob.cache["A"] = A
        prob.cache["bfix"] = rhs_fixed(prob)
    return prob.cache["lu"], prob.cache["bfix"]


class _Restricted:
    """Moment solve on V_p: restrict the Y_p right-hand side by P_c^T, solve,
    and return the DG nodal values P_c c."""

    def __init__(self, lu, Pc):
        self.lu, self.Pc = lu, Pc

    def solve(self, b):
        return self.Pc @ self.lu.solve(self.Pc.T @ b)


def scattering_source(prob: OracleProblem, varphi: np.ndarray) -> np.ndarray:
    """S = sigma_s/(4 pi) varphi + q (the moment system's scalar flux drives
    the transport equation, eq. moment_coupled)."""
    iso = (prob.sigma_s[:, None] / (4.0 * np.pi)) * varphi.reshape(prob.ne, prob.n)
    return iso + prob.q if prob.q.ndim == 2 else iso[None] + prob.q


def closures(prob: OracleProblem, psi: np.ndarray):
    phi, J, P = transport.moments(prob.omega, prob.w, psi)
    T = transport.correction_tensor(phi, P)
    beta = transport.beta_correction(prob.mesh, prob.omega, prob.w, psi)
    return phi, J, T, beta


def apply_G(prob: OracleProblem, varphi: np.ndarray, psi_lag=None):
    """One evaluation of G: sweep on the scattering source, closures, moment
    solve.  Returns (varphi_new, dict of intermediates)."""
    lu, bfix = _lhs_factor(prob)
    S = scattering_source(prob, varphi)
    psi = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar, psi_lag, prob.block)
    phi, J, T, beta = closures(prob, psi)
    b = bfix + rhs_correction(prob, T, beta)
    return lu.solve(b), {"psi": psi, "phi": phi, "J": J, "T": T, "beta": beta, "b": b}


def diffusion_start(prob: OracleProblem) -> np.ndarray:
    """Initial guess from the moment system with zero corrections."""
    lu, bfix = _lhs_factor(prob)
    return lu.solve(bfix)


def solve(prob: OracleProblem, tol: float = 1e-10, max_it: int = 200, start="zero",
          varphi0=None):
    """Fixed-point iteration X^{k+1} = G(X^k) until
    ||X^{k+1} - X^k||_inf / ||X^{k+1}||_inf < tol.  Returns
    (varphi, info) with the residual history and the last intermediates."""
    if varphi0 is not None:
        x = np.asarray(varphi0, float).reshape(-1).copy()
    elif start == "diffusion":
        x = diffusion_start(prob)
    else:
        x = np.zeros(prob.ne * prob.n)
    hist = []
    psi = None
    for it in range(1, max_it + 1):
        xn, extra = apply_G(prob, x, psi)
        psi = extra["psi"]
        r = np.max(np.abs(xn - x)) / max(np.max(np.abs(xn)), 1e-300)
        hist.append(r)
        x = xn
        if r < tol:
            return x, {"iterations": it, "history": hist, "converged": True, **extra}
    return x, {"iterations": max_it, "history": hist, "converged": False, **extra}


def fixed_point_direct(prob: OracleProblem) -> np.ndarray:
    """The fixed point as the solution of (I - G_lin) X = G(0): G is affine
    in X (SMM is linear in both the transport and moment unknowns), so its
    linear part is tabulated column by column.  Small problems only;
    straight-sided meshes only (no lagged couplings)."""
    N = prob.ne * prob.n
    g0, _ = apply_G(prob, np.zeros(N))
    Glin = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        Glin[:, k] = apply_G(prob, e)[0] - g0
    return np.linalg.solve(np.eye(N) - Glin, g0)


def source_iteration(prob: OracleProblem, tol: float = 1e-12, max_it: int = 10000, phi0=None):
    """Plain source iteration on the DG S_N equations:
    psi^{k+1} = L^{-1}(sigma_s/(4 pi) phi^k + q), phi = sum w psi."""
    phi = np.zeros((prob.ne, prob.n)) if phi0 is None else phi0.reshape(prob.ne, prob.n)
    for it in range(1, max_it + 1):
        psi = transport.sweep(prob.mesh, prob.omega, prob.sigma_t,
                              scattering_source(prob, phi), prob.psibar)
        phin = np.einsum("d,dkn->kn", prob.w, psi)
        r = np.max(np.abs(phin - phi)) / max(np.max(np.abs(phin)), 1e-300)
        phi = phin
        if r < tol:
            return phi.reshape(-1), it, psi
    return phi.reshape(-1), max_it, psi


def sn_krylov(prob: OracleProblem, tol: float = 1e-13):
    """DG S_N scalar flux with scattering solved as the linear system
    (I - sum_d w_d L^{-1} sigma_s/(4 pi)) phi = sum_d w_d L^{-1} q by GMRES
    (straight-sided meshes: one sweep applies L^{-1} exactly)."""
    N = prob.ne * prob.n
    zero = np.zeros_like(prob.q)
    rhs = np.einsum("d,dkn->kn", prob.w,
                    transport.sweep(prob.mesh, prob.omega, prob.sigma_t, prob.q, prob.psibar)).reshape(-1)

    def mv(v):
        S = (prob.sigma_s[:, None] / (4.0 * np.pi)) * v.reshape(prob.ne, prob.n)
        psi = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, None)
        return v - np.einsum("d,dkn->kn", prob.w, psi).reshape(-1)

    op = spla.LinearOperator((N, N), matvec=mv)
    x, info = spla.gmres(op, rhs, rtol=tol, atol=0.0, restart=200, maxiter=50)
    if info != 0:
        raise RuntimeError(f"GMRES did not converge ({info})")
    return x
