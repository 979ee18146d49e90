"""Finite-element data for a conforming quadrilateral mesh (oracle).

Follows Sec. 3 of the paper:
* the element map x(xi) = sum_i x_{K,i} l_i(xi) with (m+1)^2 Gauss-Lobatto
  control points (Sec. 3.1);
* Jacobian F, J = det F, grad u = F^{-T} grad_ref u, and face integrals taken
  along the reference edge with the transformed length element (Sec. 3.2);
* the DG space Y_p of mapped Q_p polynomials, here with a Gauss-Lobatto nodal
  basis, lexicographic with the x-index fastest (Sec. 3.3.1);
* interior faces carry a normal pointing from K1 to K2, boundary faces the
  outward normal (Sec. 3.1).

Meshes come as a structured nx x ny grid of shared control points, or
element by element with a neighbour table (any conforming quadrilateral
mesh); the neighbour's face and orientation on each interior face are found
by matching the face control points.

Integrals use Gauss-Legendre rules with p+m+1 points per dimension on volumes
and faces; every polynomial integrand of the SMM forms is then integrated
exactly on affine meshes.

Local face numbering: 0 bottom (eta = 0), 1 right (xi = 1), 2 top (eta = 1),
3 left (xi = 0).  Every face is parameterised by increasing xi (faces 0, 2) or
increasing eta (faces 1, 3), so the two sides of an interior face see the same
parameter at the same physical point.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .quadrature import gauss_legendre_unit, gauss_lobatto_unit


def lagrange_1d(nodes: np.ndarray, x: np.ndarray):
    """Values V[a, q] = l_a(x_q) and derivatives D[a, q] = l_a'(x_q) of the
    Lagrange polynomials through ``nodes`` (product formula)."""
    n = len(nodes)
    x = np.atleast_1d(x)
    V = np.ones((n, len(x)))
    D = np.zeros((n, len(x)))
    for a in range(n):
        for b in range(n):
            if b == a:
                continue
            V[a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
        for b in range(n):
            if b == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[b]))
            for c in range(n):
                if c == a or c == b:
                    continue
                term = term * (x - nodes[c]) / (nodes[a] - nodes[c])
            D[a] += term
    return V, D


def face_nodes(p: int, f: int) -> np.ndarray:
    """Local node indices (a + (p+1) b) on face f, ordered by the face
    parameter."""
    r = np.arange(p + 1)
    if f == 0:
        return r
    if f == 1:
        return p + (p + 1) * r
    if f == 2:
        return (p + 1) * p + r
    return (p + 1) * r


def face_ref_points(f: int, s: np.ndarray):
    """Reference coordinates (xi, eta) of face parameter values s."""
    z, o = np.zeros_like(s), np.ones_like(s)
    return {0: (s, z), 1: (o, s), 2: (s, o), 3: (z, s)}[f]


@dataclass
class Mesh:
    """Structured mesh with per-element geometry and FE data.

    Arrays (K = element, Q = volume point, F = face, q = face point,
    n = (p+1)^2 basis functions):
      detJ[K,Q], wJ[K,Q] (weight * detJ), xq[K,Q,2]
      gradU[K,Q,n,2]   physical basis gradients at volume points
      U[Q,n]           basis values at volume points (reference data)
      nds[K,F,q,2]     weight * (normal * length element) at face points
      nhat[K,F,q,2]    unit outward normal at face points
      xf[K,F,q,2]      physical face points
      Uf[F,q,n]        basis values at face points (reference data)
      gradUf[K,F,q,n,2] physical basis gradients at face points
      nbr[K,F]         neighbour element or -1
      nbr_face[K,F]    the neighbour's local face (-1 on the boundary)
      flip[K,F]        the neighbour parameterises the face the other way
      bdr_attr[K,F]    boundary attribute (-1 on interior faces)
      M, Gx, Gy [K,n,n] element mass and gradient matrices
        M_ij = int u_i u_j,  Gx_ij = int (d u_i/dx) u_j
    """
    nx: int
    ny: int
    m: int
    p: int


def _element_ctrl(ctrl: np.ndarray, i: int, j: int, m: int) -> np.ndarray:
    blk = ctrl[j * m:(j + 1) * m + 1, i * m:(i + 1) * m + 1, :]  # [b][a][2]
    return blk.reshape(-1, 2)  # index a + (m+1) b


def structured_elements(ctrl: np.ndarray, nx: int, ny: int, m: int):
    """Per-element control points [ne][(m+1)^2][2] (index a + (m+1) b) and
    neighbours [ne][4] (-1 on the boundary) of a structured grid, element
    K = j nx + i."""
    ne = nx * ny
    ctrl_e = np.zeros((ne, (m + 1) ** 2, 2))
    nbr = -np.ones((ne, 4), dtype=np.int64)
    for j in range(ny):
        for i in range(nx):
            K = j * nx + i
            ctrl_e[K] = _element_ctrl(ctrl, i, j, m)
            if j > 0:
                nbr[K, 0] = K - nx
            if i < nx - 1:
                nbr[K, 1] = K + 1
            if j < ny - 1:
                nbr[K, 2] = K + nx
            if i > 0:
                nbr[K, 3] = K - 1
    return ctrl_e, nbr


def face_ctrl(m: int, f: int) -> np.ndarray:
    """Indices (a + (m+1) b) of the m+1 control points on face f, ordered by
    the face parameter."""
    r = np.arange(m + 1)
    return {0: r, 1: m + (m + 1) * r, 2: (m + 1) * m + r, 3: (m + 1) * r}[f]


def build_mesh(ctrl: np.ndarray, nx: int, ny: int, m: int, p: int) -> Mesh:
    """Evaluate the geometry and basis data of every element of a structured
    nx x ny mesh (Sec. 3.1-3.3)."""
    ctrl_e, nbr = structured_elements(ctrl, nx, ny, m)
    mesh = build_mesh_general(ctrl_e, nbr, m, p)
    mesh.nx, mesh.ny = nx, ny
    mesh.ctrl = ctrl
    return mesh


def build_mesh_general(ctrl_e: np.ndarray, nbr: np.ndarray, m: int, p: int, bdr_attr=None) -> Mesh:
    """Geometry and basis data of a conforming quadrilateral mesh given
    element by element (Sec. 3.1): ctrl_e [ne][(m+1)^2][2] Gauss-Lobatto
    control points of each element's Q_m map, nbr [ne][4] the element across
    each local face (-1 on the boundary), bdr_attr [ne][4] a boundary
    attribute per boundary face (default: the local face index).

    The two elements on an interior face parameterise it separately; the
    neighbour's face index (nbr_face) and whether the two parameterisations
    run in opposite directions (flip: the neighbour's face point q is this
    element's point nq-1-q) are found by matching the face control points.
    General meshes carry nx = n_elem, ny = 1."""
    ctrl_e = np.asarray(ctrl_e, dtype=float)
    nbr = np.asarray(nbr, dtype=np.int64)
    ne = len(ctrl_e)
    mesh = Mesh(ne, 1, m, p)
    nb = p + 1
    n = nb * nb
    nq = p + m + 1
    sg, wg = gauss_legendre_unit(nq)
    gnodes = gauss_lobatto_unit(p)           # solution basis nodes
    cnodes = gauss_lobatto_unit(m)           # geometry control nodes
    mesh.sol_nodes_1d = gnodes
    mesh.nq = nq
    mesh.sg, mesh.wg = sg, wg

    # volume points: xi fastest
    XI, ETA = np.meshgrid(sg, sg)
    xi, eta = XI.reshape(-1), ETA.reshape(-1)
    wv = np.outer(wg, wg).reshape(-1)

    def basis2d(nodes, xi, eta):
        Va, Da = lagrange_1d(nodes, xi)
        Vb, Db = lagrange_1d(nodes, eta)
        k = len(nodes)
        V = np.einsum("aq,bq->baq", Va, Vb).reshape(k * k, -1)
        Dxi = np.einsum("aq,bq->baq", Da, Vb).reshape(k * k, -1)
        Deta = np.einsum("aq,bq->baq", Va, Db).reshape(k * k, -1)
        return V, Dxi, Deta  # [basis, point]

    def geom(Xc, xi, eta):
        V, Dxi, Deta = basis2d(cnodes, xi, eta)
        x = V.T @ Xc
        x_xi = Dxi.T @ Xc
        x_eta = Deta.T @ Xc
        return x, x_xi, x_eta

    Vs, Dxs, Des = basis2d(gnodes, xi, eta)
    mesh.U = Vs.T.copy()                           # [Q, n]
    mesh.wv = wv
    Q = len(wv)
    mesh.detJ = np.zeros((ne, Q))
    mesh.wJ = np.zeros((ne, Q))
    mesh.xq = np.zeros((ne, Q, 2))
    mesh.gradU = np.zeros((ne, Q, n, 2))
    mesh.xnode = np.zeros((ne, n, 2))
    mesh.area = np.zeros(ne)
    mesh.nds = np.zeros((ne, 4, nq, 2))
    mesh.nhat = np.zeros((ne, 4, nq, 2))
    mesh.dsw = np.zeros((ne, 4, nq))
    mesh.xf = np.zeros((ne, 4, nq, 2))
    mesh.gradUf = np.zeros((ne, 4, nq, n, 2))
    mesh.Uf = np.zeros((4, nq, n))
    mesh.nbr = nbr.copy()
    mesh.corner = np.zeros((ne, 4, 2))   # (x0,y0),(x1,y0),(x1,y1),(x0,y1) in ref corners
    mesh.ctrl_e = ctrl_e

    NX, NE = np.meshgrid(gnodes, gnodes)
    nodal_xi, nodal_eta = NX.reshape(-1), NE.reshape(-1)
    face_data = []
    for f in range(4):
        fx, fe = face_ref_points(f, sg)
        Vf, Dxf, Def = basis2d(gnodes, fx, fe)
        mesh.Uf[f] = Vf.T
        face_data.append((fx, fe, Vf, Dxf, Def))

    for K in range(ne):
        Xc = ctrl_e[K]
        x, x_xi, x_eta = geom(Xc, xi, eta)
        det = x_xi[:, 0] * x_eta[:, 1] - x_eta[:, 0] * x_xi[:, 1]
        if np.any(det <= 0):
            raise ValueError(f"element {K} has non-positive Jacobian")
        mesh.detJ[K] = det
        mesh.wJ[K] = wv * det
        mesh.xq[K] = x
        mesh.area[K] = np.sum(wv * det)
        # grad u = F^{-T} grad_ref u ;  F = [[x_xi, x_eta],[y_xi, y_eta]]
        # d/dx = ( y_eta d/dxi - y_xi d/deta)/J ; d/dy = (-x_eta d/dxi + x_xi d/deta)/J
        gx = (x_eta[:, 1][None, :] * Dxs - x_xi[:, 1][None, :] * Des) / det[None, :]
        gy = (-x_eta[:, 0][None, :] * Dxs + x_xi[:, 0][None, :] * Des) / det[None, :]
        mesh.gradU[K, :, :, 0] = gx.T
        mesh.gradU[K, :, :, 1] = gy.T
        xn, _, _ = geom(Xc, nodal_xi, nodal_eta)
        mesh.xnode[K] = xn
        cx, _, _ = geom(Xc, np.array([0.0, 1.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0, 1.0]))
        mesh.corner[K] = cx
        for f in range(4):
            fx, fe, Vf, Dxf, Def = face_data[f]
            xf, fxi, feta = geom(Xc, fx, fe)
            T = fxi if f in (0, 2) else feta      # tangent along the parameter
            nvec = np.stack([T[:, 1], -T[:, 0]], axis=1)
            if f in (2, 3):
                nvec = -nvec                      # counter-clockwise orientation
            ds = np.linalg.norm(nvec, axis=1)
            mesh.nds[K, f] = wg[:, None] * nvec
            mesh.nhat[K, f] = nvec / ds[:, None]
            mesh.dsw[K, f] = wg * ds
            mesh.xf[K, f] = xf
            detf = fxi[:, 0] * feta[:, 1] - feta[:, 0] * fxi[:, 1]
            gfx = (feta[:, 1][None, :] * Dxf - fxi[:, 1][None, :] * Def) / detf[None, :]
            gfy = (-feta[:, 0][None, :] * Dxf + fxi[:, 0][None, :] * Def) / detf[None, :]
            mesh.gradUf[K, f, :, :, 0] = gfx.T
            mesh.gradUf[K, f, :, :, 1] = gfy.T

    # interior faces: the neighbour's face and the relative orientation, from
    # the face control points (both sides must carry the same points)
    mesh.nbr_face = -np.ones((ne, 4), dtype=np.int64)
    mesh.flip = np.zeros((ne, 4), dtype=bool)
    size = np.sqrt(np.max(mesh.area))
    for K in range(ne):
        for f in range(4):
            N = nbr[K, f]
            if N < 0:
                continue
            if N >= ne or N == K:
                raise ValueError(f"element {K} face {f}: bad neighbour {N}")
            a = ctrl_e[K][face_ctrl(m, f)]
            found = None
            for g in range(4):
                if nbr[N, g] != K:
                    continue
                b = ctrl_e[N][face_ctrl(m, g)]
                if np.abs(a - b).max() <= 1e-10 * size:
                    found = (g, False)
                elif np.abs(a - b[::-1]).max() <= 1e-10 * size:
                    found = (g, True)
                if found:
                    break
            if found is None:
                raise ValueError(f"element {K} face {f} does not match a face of element {N}")
            mesh.nbr_face[K, f], mesh.flip[K, f] = found

    # element matrices
    mesh.M = np.einsum("kq,qi,qj->kij", mesh.wJ, mesh.U, mesh.U)
    mesh.Gx = np.einsum("kq,kqi,qj->kij", mesh.wJ, mesh.gradU[..., 0], mesh.U)
    mesh.Gy = np.einsum("kq,kqi,qj->kij", mesh.wJ, mesh.gradU[..., 1], mesh.U)
    mesh.fnodes = np.array([face_nodes(p, f) for f in range(4)])
    # boundary faces: ordered by element, then local face
    bf = [(K, f) for K in range(ne) for f in range(4) if mesh.nbr[K, f] < 0]
    mesh.bfaces = np.array(bf, dtype=np.int64).reshape(-1, 2)
    mesh.bface_id = -np.ones((ne, 4), dtype=np.int64)
    for b, (K, f) in enumerate(bf):
        mesh.bface_id[K, f] = b
    mesh.bdr_attr = -np.ones((ne, 4), dtype=np.int64)
    for K, f in bf:
        mesh.bdr_attr[K, f] = f if bdr_attr is None else int(np.asarray(bdr_attr)[K, f])
    return mesh


def neighbour_trace(mesh: Mesh, K: int, f: int, nodal_N: np.ndarray) -> np.ndarray:
    """Trace at the face points of element K's face f of the neighbour's nodal
    field nodal_N (values of the element across f), in K's point order."""
    v = mesh.Uf[mesh.nbr_face[K, f]] @ nodal_N
    return v[::-1] if mesh.flip[K, f] else v


OPPOSITE = np.array([2, 3, 0, 1])


def interpolate(mesh: Mesh, nodal: np.ndarray) -> np.ndarray:
    """Values of a nodal DG field [K, n] at the volume points [K, Q]."""
    return nodal @ mesh.U.T


def l2_error(mesh: Mesh, nodal: np.ndarray, exact_fn) -> float:
    """|| u_h - u ||_{L2(D)} by volume quadrature (Sec. 6.1 error norm)."""
    uh = interpolate(mesh, nodal)
    ue = exact_fn(mesh.xq[..., 0], mesh.xq[..., 1])
    return float(np.sqrt(np.sum(mesh.wJ * (uh - ue) ** 2)))


def l2_norm(mesh: Mesh, nodal: np.ndarray) -> float:
    uh = interpolate(mesh, nodal)
    return float(np.sqrt(np.sum(mesh.wJ * uh ** 2)))
