"""Seeded problem generators.

Everything here describes an input problem: a structured quadrilateral mesh
given by its control points (paper Sec. 3.1: a continuous Q_m map whose
control points sit at Gauss-Lobatto positions), piecewise-constant materials
(per element, set by the material at the element centroid), sources and
inflow functions.  No quadrature, basis, transport or moment-system arithmetic
lives here.

Random numbers come from SplitMix64 (Steele, Lea and Flood, 2014), written out
below from its published definition so that every consumer draws the same
stream on any machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "SplitMix64", "lobatto_points_unit", "structured_ctrl", "sine_perturbation",
    "Workload", "config_plain", "config_curved_mms", "config_channel",
    "batched_params", "config_batched_problem", "config_blobs", "config_tdl",
    "mms_psi", "mms_source", "mms_phi", "absorber_inflow", "chebyshev_vertices",
    "rotate_elements", "elements_from_corners", "inner_square_mesh", "general_workload",
    "product_quadrature_2d",
]

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (golden-gamma increment, two xor-shift-multiply
    mixing rounds).  ``uniform()`` returns the top 53 bits as a double in
    [0, 1)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_range(self, a: float, b: float) -> float:
        return a + (b - a) * self.uniform()

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1))


def lobatto_points_unit(m: int) -> np.ndarray:
    """The m+1 Gauss-Lobatto points on [0, 1] where a Q_m mesh places its
    control points: the endpoints plus the roots of the derivative of the
    degree-m Legendre polynomial."""
    if m < 1:
        raise ValueError("mesh order must be >= 1")
    inner = np.polynomial.legendre.Legendre.basis(m).deriv().roots()
    x = np.concatenate([[-1.0], np.sort(inner.real), [1.0]])
    return 0.5 * (x + 1.0)


def chebyshev_vertices(npts: int, a: float = 0.0, b: float = 1.0) -> np.ndarray:
    """1D Chebyshev (extrema) points on [a, b], ascending; a tensor product of
    these gives a boundary-clustered orthogonal mesh."""
    k = np.arange(npts)
    t = -np.cos(np.pi * k / (npts - 1))
    return a + (b - a) * 0.5 * (t + 1.0)


def structured_ctrl(xv: np.ndarray, yv: np.ndarray, m: int, perturb=None) -> np.ndarray:
    """Control-point grid of a structured mesh.

    ``xv`` (nx+1) and ``yv`` (ny+1) are the vertex lines of an orthogonal
    mesh.  Inside each element interval the control points are placed at the
    Gauss-Lobatto positions, giving a grid of shape [ny*m+1][nx*m+1][2]
    (x fastest) shared by neighbouring elements.  ``perturb(x, y) -> (dx, dy)``
    displaces every control point (used for curved meshes)."""
    g = lobatto_points_unit(m)
    nx, ny = len(xv) - 1, len(yv) - 1
    xs = np.empty(nx * m + 1)
    ys = np.empty(ny * m + 1)
    for i in range(nx):
        xs[i * m:(i + 1) * m + 1] = xv[i] + (xv[i + 1] - xv[i]) * g
    for j in range(ny):
        ys[j * m:(j + 1) * m + 1] = yv[j] + (yv[j + 1] - yv[j]) * g
    X, Y = np.meshgrid(xs, ys)  # [ny*m+1][nx*m+1]
    ctrl = np.stack([X, Y], axis=-1)
    if perturb is not None:
        dx, dy = perturb(X, Y)
        ctrl = ctrl + np.stack([dx, dy], axis=-1)
    return np.ascontiguousarray(ctrl)


def sine_perturbation(amplitude: float = 0.05):
    """x' = x + A s, y' = y + A s with s = sin(2 pi x) sin(2 pi y): interior
    points move, points on the boundary of the unit square do not."""
    def f(X, Y):
        s = np.sin(2.0 * np.pi * X) * np.sin(2.0 * np.pi * Y)
        return amplitude * s, amplitude * s
    return f


@dataclass
class Workload:
    """One transport problem on a structured quadrilateral mesh.

    sigma_t, sigma_s: per element (length nx*ny, element index j*nx+i).
    q_elem: isotropic source per steradian, constant per element (or None
    when ``q_fn`` supplies an anisotropic analytic source).
    inflow: "vacuum", ("iso", value) or ("fn", f(x, y, ox, oy)).
    """
    name: str
    nx: int
    ny: int
    m: int
    p: int
    sn: int
    ctrl: np.ndarray
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    q_elem: np.ndarray | None = None
    q_fn: object = None
    inflow: object = "vacuum"
    meta: dict = field(default_factory=dict)
    # a mesh given element by element (any conforming quadrilateral mesh):
    # control points [ne][(m+1)^2][2], neighbours [ne][4] (-1: boundary) and
    # boundary attributes [ne][4]; then nx = ne, ny = 1 and ctrl is unused
    elem_ctrl: np.ndarray | None = None
    nbr: np.ndarray | None = None
    bdr_attr: np.ndarray | None = None
    # an explicit angular quadrature (omega [n_dir][3], w [n_dir]) instead of
    # the level-symmetric set of order sn
    quad: tuple | None = None

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny

    @property
    def units_per_sweep(self) -> int:
        return self.n_elem * self.n_dir * (self.p + 1) ** 2

    @property
    def n_dir(self) -> int:
        if self.quad is not None:
            return len(self.quad[1])
        return self.sn * (self.sn + 2) // 2


def _uniform_square(n: int, m: int, side: float = 1.0, perturb=None):
    v = np.linspace(0.0, side, n + 1)
    return structured_ctrl(v, v, m, perturb)


def config_plain(n: int = 8, p: int = 1, sn: int = 4) -> Workload:
    """Plain SMM case: unit square, n x n affine squares, sigma_t = 1,
    sigma_s = 0.9, q = 1 per steradian, vacuum boundaries."""
    ne = n * n
    return Workload("plain", n, n, 1, p, sn, _uniform_square(n, 1),
                    np.full(ne, 1.0), np.full(ne, 0.9), q_elem=np.full(ne, 1.0))


def config_tdl(eps: float, n: int = 8, p: int = 2, sn: int = 4) -> Workload:
    """Thick-diffusion-limit data: sigma_t = 1/eps, sigma_a = eps, q = eps,
    orthogonal n x n mesh of the unit square, vacuum boundaries."""
    ne = n * n
    st = 1.0 / eps
    return Workload(f"tdl{eps:g}", n, n, 1, p, sn, _uniform_square(n, 1),
                    np.full(ne, st), np.full(ne, st - eps), q_elem=np.full(ne, eps))


# ----------------------------------------------------------------------------
# Manufactured solution on the curved mesh:
#   psi = (1 + sin(pi x) sin(pi y)) (1 + Omega_x^2),  sigma_t = 1, sigma_s = 0.5
# ----------------------------------------------------------------------------

def mms_psi(x, y, ox):
    return (1.0 + np.sin(np.pi * x) * np.sin(np.pi * y)) * (1.0 + ox * ox)


def mms_phi(x, y):
    """Angular integral of mms_psi over the unit sphere: a * (4 pi + 4 pi/3)."""
    a = 1.0 + np.sin(np.pi * x) * np.sin(np.pi * y)
    return a * (16.0 * np.pi / 3.0)


def mms_source(x, y, ox, oy, sigma_t=1.0, sigma_s=0.5):
    """q_d such that mms_psi solves Omega.grad psi + sigma_t psi =
    sigma_s/(4 pi) phi + q with phi the exact angular integral."""
    a = 1.0 + np.sin(np.pi * x) * np.sin(np.pi * y)
    ax = np.pi * np.cos(np.pi * x) * np.sin(np.pi * y)
    ay = np.pi * np.sin(np.pi * x) * np.cos(np.pi * y)
    f = 1.0 + ox * ox
    return f * (ox * ax + oy * ay + sigma_t * a) - sigma_s / (4.0 * np.pi) * mms_phi(x, y)


def config_curved_mms(n: int = 32, p: int = 2, sn: int = 8, amplitude: float = 0.05) -> Workload:
    """Curved-mesh manufactured problem: order-p geometry (m = p), interior
    control points perturbed by the sine field, S8, sigma_t = 1, sigma_s = 0.5."""
    ne = n * n
    ctrl = _uniform_square(n, p, perturb=sine_perturbation(amplitude))
    return Workload("curved_mms", n, n, p, p, sn, ctrl, np.full(ne, 1.0), np.full(ne, 0.5),
                    q_fn=lambda x, y, ox, oy: mms_source(x, y, ox, oy, 1.0, 0.5),
                    inflow=("fn", lambda x, y, ox, oy: mms_psi(x, y, ox)))


def absorber_inflow(sigma_t: float):
    """Inflow for the pure absorber whose exact solution is
    psi_d(x) = exp(-sigma_t (Omega_x x + Omega_y y) / (Omega_x^2 + Omega_y^2)):
    it is constant along each characteristic direction up to attenuation."""
    def f(x, y, ox, oy):
        return np.exp(-sigma_t * (ox * x + oy * y) / (ox * ox + oy * oy))
    return f


# ----------------------------------------------------------------------------
# Multi-material channel case: [0,10]^2, 128 x 128, p = 2, S12.
# ----------------------------------------------------------------------------

def channel_mask(n: int, width: int, seed: int) -> np.ndarray:
    """Boolean [n][n] (row j, column i) marking a channel `width` cells wide
    that leaves the source corner block along +x, bends to +y, to +x and to
    +y again (three right-angle bends) and exits through the far side.  Bend
    positions are drawn from SplitMix64(seed)."""
    rng = SplitMix64(seed)
    mask = np.zeros((n, n), dtype=bool)
    x1 = rng.randint(n // 4, n // 2)          # end of first +x leg (column)
    y1 = rng.randint(n // 3, (2 * n) // 3)    # end of +y leg (row)
    x2 = rng.randint((5 * n) // 8, n - width - 1)
    # leg 1: rows [0, width), columns [0, x1 + width)
    mask[0:width, 0:x1 + width] = True
    # leg 2: columns [x1, x1 + width), rows [0, y1 + width)
    mask[0:y1 + width, x1:x1 + width] = True
    # leg 3: rows [y1, y1 + width), columns [x1, x2 + width)
    mask[y1:y1 + width, x1:x2 + width] = True
    # leg 4: columns [x2, x2 + width), rows [y1, n)
    mask[y1:n, x2:x2 + width] = True
    return mask


def config_channel(n: int = 128, p: int = 2, sn: int = 12, seed: int = 0,
                   side: float = 10.0) -> Workload:
    """Two-material channel problem.  Background: sigma_t = 200, c = 0.9995.
    Channel (13 cells wide at n = 128): sigma_t = 0.2, c = 0.5.  Unit isotropic
    source (per steradian) in the elements whose centroid lies in [0,1]^2;
    vacuum elsewhere on the boundary."""
    h = side / n
    width = max(1, int(round(1.0 / h + 0.2)))  # 13 cells at h = 0.078125
    mask = channel_mask(n, width, seed).reshape(-1)
    st = np.where(mask, 0.2, 200.0)
    c = np.where(mask, 0.5, 0.9995)
    ss = st * c
    ic = (np.arange(n) + 0.5) * h
    cx, cy = np.meshgrid(ic, ic)
    q = ((cx < 1.0) & (cy < 1.0)).astype(float).reshape(-1)
    return Workload("channel", n, n, 1, p, sn, _uniform_square(n, 1, side), st, ss,
                    q_elem=q, meta={"seed": seed, "width": width, "h": h})


# ----------------------------------------------------------------------------
# Batched case: 256 independent homogeneous problems drawn per seed.
# ----------------------------------------------------------------------------

SN_CHOICES = (4, 6, 8, 10, 12)


def batched_params(seed: int) -> dict:
    """Problem parameters for one batch member: n_side ~ U{16..128},
    p ~ U{1..4}, S_N ~ U{4,6,8,10,12}, sigma_t = 10^U(-1,2), c ~ U(0.5,0.999)."""
    rng = SplitMix64(seed)
    n = rng.randint(16, 128)
    p = rng.randint(1, 4)
    sn = SN_CHOICES[rng.randint(0, 4)]
    st = 10.0 ** rng.uniform_range(-1.0, 2.0)
    c = rng.uniform_range(0.5, 0.999)
    return {"n": n, "p": p, "sn": sn, "sigma_t": st, "c": c}


def config_batched_problem(seed: int) -> Workload:
    prm = batched_params(seed)
    n = prm["n"]
    ne = n * n
    return Workload(f"batch{seed}", n, n, 1, prm["p"], prm["sn"], _uniform_square(n, 1),
                    np.full(ne, prm["sigma_t"]), np.full(ne, prm["sigma_t"] * prm["c"]),
                    q_elem=np.full(ne, 1.0), meta=prm)


# ----------------------------------------------------------------------------
# Learned-warm-start case: 64 x 64, p = 2, S8, random disc blobs.
# ----------------------------------------------------------------------------

def blob_layout(seed: int, n: int = 64):
    """Per-element (sigma_t, c) from a background plus K ~ U{4..8} discs
    (centre U([0,1]^2), radius U(0.05, 0.25)); later discs overwrite earlier
    ones.  Each region draws sigma_t = 10^U(-1,2) and c ~ U(0.5, 0.9999)."""
    rng = SplitMix64(seed)
    k = rng.randint(4, 8)
    regions = [(10.0 ** rng.uniform_range(-1.0, 2.0), rng.uniform_range(0.5, 0.9999))]
    discs = []
    for _ in range(k):
        cx, cy = rng.uniform(), rng.uniform()
        r = rng.uniform_range(0.05, 0.25)
        discs.append((cx, cy, r))
        regions.append((10.0 ** rng.uniform_range(-1.0, 2.0), rng.uniform_range(0.5, 0.9999)))
    h = 1.0 / n
    c1 = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c1, c1)
    reg = np.zeros((n, n), dtype=np.int64)
    for b, (cx, cy, r) in enumerate(discs):
        reg[(X - cx) ** 2 + (Y - cy) ** 2 < r * r] = b + 1
    st = np.array([regions[r][0] for r in reg.reshape(-1)])
    c = np.array([regions[r][1] for r in reg.reshape(-1)])
    return st, c, reg


def config_blobs(seed: int, n: int = 64, p: int = 2, sn: int = 8) -> Workload:
    st, c, reg = blob_layout(seed, n)
    ne = n * n
    return Workload(f"blobs{seed}", n, n, 1, p, sn, _uniform_square(n, 1), st, st * c,
                    q_elem=np.full(ne, 1.0), meta={"seed": seed, "regions": reg})


# ----------------------------------------------------------------------------
# Meshes given element by element (unstructured, or with rotated local
# numbering), and a non-level-symmetric angular set.
# ----------------------------------------------------------------------------

def rotate_elements(elem_ctrl: np.ndarray, nbr: np.ndarray, rot) -> tuple:
    """Renumber element K's local frame by rot[K] quarter turns (the same
    physical element): the new face f is the old face f + 1 (mod 4), i.e.
    the new reference point (xi', eta') is the old (1 - eta', xi')."""
    elem_ctrl = np.array(elem_ctrl, dtype=float)
    nbr = np.array(nbr, dtype=np.int64)
    m = int(round(np.sqrt(elem_ctrl.shape[1]))) - 1
    for K, r in enumerate(rot):
        for _ in range(int(r) % 4):
            old = elem_ctrl[K].copy()
            for b2 in range(m + 1):
                for a2 in range(m + 1):
                    elem_ctrl[K, a2 + (m + 1) * b2] = old[(m - b2) + (m + 1) * a2]
            nbr[K] = np.roll(nbr[K], -1)
    return elem_ctrl, nbr


def elements_from_corners(corners: np.ndarray, m: int, displace=None):
    """Elements from their four corners [ne][4][2] (counter-clockwise, local
    corner order (0,0), (1,0), (1,1), (0,1)): the Gauss-Lobatto control
    points of each bilinear quadrilateral, moved by displace(x, y) -> (dx, dy)
    when given; neighbours found by matching face end points."""
    corners = np.asarray(corners, dtype=float)
    g = lobatto_points_unit(m)
    ne = len(corners)
    ctrl = np.zeros((ne, (m + 1) ** 2, 2))
    for K in range(ne):
        c = corners[K]
        for b in range(m + 1):
            for a in range(m + 1):
                u, v = g[a], g[b]
                ctrl[K, a + (m + 1) * b] = ((1 - u) * (1 - v) * c[0] + u * (1 - v) * c[1]
                                            + u * v * c[2] + (1 - u) * v * c[3])
    if displace is not None:
        dx, dy = displace(ctrl[..., 0], ctrl[..., 1])
        ctrl = ctrl + np.stack([dx, dy], axis=-1)
    ends = {0: (0, 1), 1: (1, 2), 2: (3, 2), 3: (0, 3)}
    key = lambda P: (round(float(P[0]), 9), round(float(P[1]), 9))
    faces = {}
    for K in range(ne):
        for f, (a, b) in ends.items():
            faces.setdefault(frozenset((key(corners[K, a]), key(corners[K, b]))), []).append((K, f))
    nbr = -np.ones((ne, 4), dtype=np.int64)
    for lst in faces.values():
        if len(lst) == 2:
            (K1, f1), (K2, f2) = lst
            nbr[K1, f1], nbr[K2, f2] = K2, K1
    return ctrl, nbr


def inner_square_mesh(k: int, m: int = 1, r: float = 0.22, theta: float = 0.3, displace=None):
    """The unit square split into a rotated inner square (half-width r,
    angle theta, centre (0.5, 0.5)) and four quadrilaterals joining its edges
    to the outer edges, each cut into k x k elements by bilinear
    subdivision: an unstructured conforming mesh whose inner-square corners
    are shared by three macro quadrilaterals.  Boundary attribute: the
    outer side (0 bottom, 1 right, 2 top, 3 left)."""
    ct, st = np.cos(theta), np.sin(theta)
    inner = [np.array([0.5 + (x * ct - y * st), 0.5 + (x * st + y * ct)])
             for x, y in ((-r, -r), (r, -r), (r, r), (-r, r))]
    outer = [np.array(v, float) for v in ((0, 0), (1, 0), (1, 1), (0, 1))]
    macros = [inner]
    for s in range(4):
        a, b = s, (s + 1) % 4
        macros.append([outer[a], outer[b], inner[b], inner[a]])
    corners = []
    for M in macros:
        for j in range(k):
            for i in range(k):
                def at(u, v):
                    return ((1 - u) * (1 - v) * M[0] + u * (1 - v) * M[1] + u * v * M[2] + (1 - u) * v * M[3])
                u0, u1, v0, v1 = i / k, (i + 1) / k, j / k, (j + 1) / k
                corners.append([at(u0, v0), at(u1, v0), at(u1, v1), at(u0, v1)])
    corners = np.array(corners)
    ctrl, nbr = elements_from_corners(corners, m, displace)
    attr = -np.ones((len(corners), 4), dtype=np.int64)
    for K in range(len(corners)):
        for f, (a, b) in {0: (0, 1), 1: (1, 2), 2: (3, 2), 3: (0, 3)}.items():
            if nbr[K, f] >= 0:
                continue
            mid = 0.5 * (corners[K, a] + corners[K, b])
            if abs(mid[1]) < 1e-12:
                attr[K, f] = 0
            elif abs(mid[0] - 1) < 1e-12:
                attr[K, f] = 1
            elif abs(mid[1] - 1) < 1e-12:
                attr[K, f] = 2
            else:
                attr[K, f] = 3
    return ctrl, nbr, attr


def general_workload(name, elem_ctrl, nbr, m, p, sn, sigma_t, sigma_s, bdr_attr=None, q_elem=None, q_fn=None,
                     inflow="vacuum", quad=None) -> Workload:
    """A problem on a mesh given element by element."""
    ne = len(elem_ctrl)
    return Workload(name, ne, 1, m, p, sn, None, np.asarray(sigma_t, float), np.asarray(sigma_s, float),
                    q_elem=q_elem, q_fn=q_fn, inflow=inflow, elem_ctrl=np.asarray(elem_ctrl, float),
                    nbr=np.asarray(nbr, np.int64), bdr_attr=None if bdr_attr is None else np.asarray(bdr_attr),
                    quad=quad)


def product_quadrature_2d(n_polar: int, n_azim: int):
    """A product angular set on the upper half sphere (Omega_z > 0): Gauss-
    Legendre in mu = Omega_z on (0, 1) with n_polar points, and n_azim equally
    spaced azimuths offset by half a step; weights doubled for the lower half
    so that they sum to 4 pi (the 2D reduction of Sec. 4).  Directions are
    ordered by azimuth."""
    x, w = np.polynomial.legendre.leggauss(n_polar)
    mu, wm = 0.5 * (x + 1.0), 0.5 * w
    phis = (np.arange(n_azim) + 0.5) * 2.0 * np.pi / n_azim
    om, wt = [], []
    for ph in phis:
        for c, wc in zip(mu, wm):
            s = np.sqrt(1.0 - c * c)
            om.append((s * np.cos(ph), s * np.sin(ph), c))
            wt.append(2.0 * wc * 2.0 * np.pi / n_azim)
    return np.array(om), np.array(wt)
