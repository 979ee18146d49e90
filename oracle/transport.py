"""Upwind DG S_N transport sweep and angular moments (oracle).

Sec. 4 collocates the transport equation at the S_N directions and
approximates each psi_d in the DG space Y_p; the paper defers the DG weak form
to its references.  The oracle uses the textbook upwind form integrated by
parts once: for every element K and test function u in Q_p(K),

    sum_faces int_f (Omega.n) u psi_hat ds - int_K (Omega.grad u) psi dx
        + int_K sigma_t u psi dx = int_K u S dx,

with psi_hat the element's own trace where Omega.n > 0 and the upwind value
(neighbour trace, or the inflow function on the domain boundary) where
Omega.n < 0, decided pointwise at the face quadrature points.

Elements are visited in upwind order.  The per-direction element graph takes
its edges from the chord normal of each face (the exact integral of n ds over
a face), which makes the graph acyclic on convex quadrilaterals.  A face point
whose pointwise inflow comes from a neighbour that the graph places
downstream -- possible only on curved faces -- reads that neighbour's previous
sweep (the lagging of upper-triangular couplings described for the curved
triple-point mesh in Sec. 6.2).

Parallel block Jacobi sweep (Sec. 6.5, weak scaling): the mesh is split into
blocks, each block is swept on its own in upwind order, and inflow across a
face between two blocks is the neighbour's previous sweep.  The graph then
has edges only inside blocks.  Selected by passing a block id per element.
"""
from __future__ import annotations

import numpy as np

from .fem import Mesh, neighbour_trace


def chord_normals(mesh: Mesh) -> np.ndarray:
    """int_F n ds for every (element, face), outward from the element, from
    the face end points: rotate the chord (dx, dy) to (dy, -dx), with faces
    2 and 3 traversed backwards to keep the counter-clockwise orientation."""
    c = mesh.corner  # [K, 4, 2] corners (0,0),(1,0),(1,1),(0,1)
    out = np.zeros(c.shape)
    pairs = {0: (0, 1, 1.0), 1: (1, 2, 1.0), 2: (3, 2, -1.0), 3: (0, 3, -1.0)}
    for f, (a, b, s) in pairs.items():
        d = c[:, b, :] - c[:, a, :]
        out[:, f, 0] = s * d[:, 1]
        out[:, f, 1] = -s * d[:, 0]
    return out


def block_ids(mesh: Mesh, tx: int, ty: int) -> np.ndarray:
    """Block of each element when the nx x ny element grid is cut into tiles
    of tx x ty elements (the last row and column of tiles may be smaller);
    tiles numbered row by row."""
    i = np.arange(mesh.nx * mesh.ny) % mesh.nx
    j = np.arange(mesh.nx * mesh.ny) // mesh.nx
    return (i // tx) + (j // ty) * (-(-mesh.nx // tx))


def sweep_graph(mesh: Mesh, om: np.ndarray, block: np.ndarray | None = None):
    """Upwind element graph for direction om (edges only between elements of
    the same block when ``block`` is given).

    Returns (upstream[K, f] bool: the neighbour across f is a graph
    predecessor; level[K]: longest-path level from Kahn's algorithm)."""
    ne = mesh.nx * mesh.ny
    cn = chord_normals(mesh)
    flux = cn[..., 0] * om[0] + cn[..., 1] * om[1]       # [K, 4]
    interior = mesh.nbr >= 0
    if block is not None:
        same = np.zeros_like(interior)
        for f in range(4):
            N = mesh.nbr[:, f]
            same[:, f] = (N >= 0) & (block[np.maximum(N, 0)] == block)
        interior = same
    upstream = interior & (flux < 0.0)
    indeg = upstream.sum(axis=1)
    level = np.zeros(ne, dtype=np.int64)
    frontier = [K for K in range(ne) if indeg[K] == 0]
    indeg = indeg.copy()
    seen = 0
    while frontier:
        nxt = []
        for K in sorted(frontier):
            seen += 1
            for f in range(4):
                N = mesh.nbr[K, f]
                if interior[K, f] and flux[K, f] > 0.0:     # K -> N
                    level[N] = max(level[N], level[K] + 1)
                    indeg[N] -= 1
                    if indeg[N] == 0:
                        nxt.append(N)
        frontier = nxt
    if seen != ne:
        raise RuntimeError("sweep graph has a cycle")
    return upstream, level


def sweep(mesh: Mesh, omega: np.ndarray, sigma_t: np.ndarray, S: np.ndarray,
          psibar: np.ndarray | None, psi_lag: np.ndarray | None = None,
          block: np.ndarray | None = None) -> np.ndarray:
    """One application of L^{-1} (of its block Jacobi approximation when
    ``block`` is given): psi[d, K, :] for every direction.

    S: nodal source [ne, n] (shared by all directions) or [n_dir, ne, n].
    psibar: inflow at boundary face points [n_bface, nq, n_dir] (None = vacuum).
    psi_lag: previous sweep, read at lagged face points: curved faces against
    the graph, and faces between blocks (None = 0).
    block: block id per element, or None for the full sweep.
    """
    nd = omega.shape[0]
    ne, n = mesh.nx * mesh.ny, (mesh.p + 1) ** 2
    psi = np.zeros((nd, ne, n))
    Uf = mesh.Uf
    for d in range(nd):
        ox, oy = omega[d, 0], omega[d, 1]
        Sd = S if S.ndim == 2 else S[d]
        upstream, level = sweep_graph(mesh, omega[d], block)
        lag = psi_lag[d] if psi_lag is not None else np.zeros((ne, n))
        for L in range(level.max() + 1):
            Ks = np.nonzero(level == L)[0]
            A = (sigma_t[Ks, None, None] * mesh.M[Ks]
                 - ox * mesh.Gx[Ks] - oy * mesh.Gy[Ks])
            rhs = np.einsum("kij,kj->ki", mesh.M[Ks], Sd[Ks])
            for f in range(4):
                on = ox * mesh.nds[Ks, f, :, 0] + oy * mesh.nds[Ks, f, :, 1]  # [k, q]
                pos = np.maximum(on, 0.0)
                neg = np.maximum(-on, 0.0)
                A += np.einsum("kq,qi,qj->kij", pos, Uf[f], Uf[f])
                val = np.zeros(on.shape)
                for t, K in enumerate(Ks):
                    N = mesh.nbr[K, f]
                    if N < 0:
                        if psibar is not None:
                            val[t] = psibar[mesh.bface_id[K, f], :, d]
                    else:
                        src = psi[d, N] if upstream[K, f] else lag[N]
                        val[t] = neighbour_trace(mesh, K, f, src)
                rhs += np.einsum("kq,qi,kq->ki", neg, Uf[f], val)
            psi[d, Ks] = np.linalg.solve(A, rhs[..., None])[..., 0]
    return psi


def moments(omega: np.ndarray, w: np.ndarray, psi: np.ndarray):
    """Nodal angular moments by S_N quadrature (Sec. 4): phi = sum w psi,
    J = sum w Omega psi, P = sum w Omega (x) Omega psi (in-plane 2x2)."""
    phi = np.einsum("d,dkn->kn", w, psi)
    J = np.stack([np.einsum("d,dkn->kn", w * omega[:, a], psi) for a in range(2)])
    P = np.stack([np.einsum("d,dkn->kn", w * omega[:, a] * omega[:, b], psi)
                  for a, b in ((0, 0), (0, 1), (1, 1))])
    return phi, J, P


def correction_tensor(phi: np.ndarray, P: np.ndarray) -> np.ndarray:
    """T = P - (1/3) I phi (eq. correction_tensor_disc), components
    (xx, xy, yy), nodal."""
    return np.stack([P[0] - phi / 3.0, P[1], P[2] - phi / 3.0])


def boundary_traces(mesh: Mesh, psi: np.ndarray) -> np.ndarray:
    """Interior trace of psi_d at every boundary face point: [n_bf, nq, n_dir]."""
    out = np.zeros((len(mesh.bfaces), mesh.nq, psi.shape[0]))
    for b, (K, f) in enumerate(mesh.bfaces):
        out[b] = (psi[:, K, :] @ mesh.Uf[f].T).T
    return out


def beta_correction(mesh: Mesh, omega: np.ndarray, w: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Boundary correction factor at boundary face points (eq.
    bdr_correction_factor_disc): beta = sum w |Omega.n| psi - E_b0 sum w psi,
    E_b0(n) = sum w |Omega.n| / sum w, psi the element's own trace."""
    tr = boundary_traces(mesh, psi)
    beta = np.zeros(tr.shape[:2])
    for b, (K, f) in enumerate(mesh.bfaces):
        for q in range(mesh.nq):
            nh = mesh.nhat[K, f, q]
            on = np.abs(omega[:, 0] * nh[0] + omega[:, 1] * nh[1])
            e = np.sum(w * on) / np.sum(w)
            beta[b, q] = np.sum(w * on * tr[b, q]) - e * np.sum(w * tr[b, q])
    return beta


def inflow_current(mesh: Mesh, omega: np.ndarray, w: np.ndarray, psibar) -> np.ndarray:
    """Incoming partial current at boundary face points:
    J_in = sum_{Omega.n < 0} w (Omega.n) psibar (Sec. 4, with the normal
    component taken as in Sec. 2.1)."""
    nbf = len(mesh.bfaces)
    jin = np.zeros((nbf, mesh.nq))
    if psibar is None:
        return jin
    for b, (K, f) in enumerate(mesh.bfaces):
        for q in range(mesh.nq):
            nh = mesh.nhat[K, f, q]
            on = omega[:, 0] * nh[0] + omega[:, 1] * nh[1]
            inc = on < 0.0
            jin[b, q] = np.sum(w[inc] * on[inc] * psibar[b, q, inc])
    return jin


def inflow_at_points(mesh: Mesh, omega: np.ndarray, inflow) -> np.ndarray | None:
    """Tabulate an inflow description at boundary face points
    [n_bf, nq, n_dir].  ``inflow`` is "vacuum", ("iso", value),
    ("attr", values) -- isotropic, values[a] on the faces of boundary
    attribute a -- or ("fn", f(x, y, ox, oy))."""
    if inflow is None or (isinstance(inflow, str) and inflow == "vacuum"):
        return None
    nbf = len(mesh.bfaces)
    out = np.zeros((nbf, mesh.nq, omega.shape[0]))
    kind, val = inflow
    for b, (K, f) in enumerate(mesh.bfaces):
        x = mesh.xf[K, f]
        if kind == "iso":
            out[b] = val
        elif kind == "attr":
            out[b] = val[mesh.bdr_attr[K, f]]
        else:
            out[b] = val(x[:, 0:1], x[:, 1:2], omega[None, :, 0], omega[None, :, 1])
    return out
