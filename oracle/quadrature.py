"""Quadrature rules (oracle).

* Level-symmetric S_N sets on the unit sphere, reduced to the 2D half sphere
  (Sec. 4: the transport equation is collocated at discrete directions with
  weights w_d; the 2D problem keeps the directions with positive third
  component and doubles their weights so that the weights sum to 4 pi).
* Gauss-Legendre and Gauss-Lobatto rules on [0, 1] (Sec. 3.1 uses
  Gauss-Lobatto control points; all integrals are evaluated by quadrature on
  the reference element, Sec. 3.2).
"""
from __future__ import annotations

import math
import numpy as np

# First cosine of the level-symmetric sets.  S4 uses the closed form that
# makes the set integrate mu^4 exactly; S8 has mu_1^2 = 1/21 exactly; the
# others are the standard published values.
_MU1 = {
    4: math.sqrt((4.0 - math.sqrt(6.4)) / 12.0),
    6: 0.2666355,
    8: math.sqrt(1.0 / 21.0),
    10: 0.1893213,
    12: 0.1672126,
}


def level_symmetric_octant(N: int):
    """Points and weights of one octant of the level-symmetric S_N set.

    mu_i^2 = mu_1^2 + (i-1) * 2 (1 - 3 mu_1^2) / (N - 2), i = 1..N/2; the
    points are (mu_i, mu_j, mu_k) with i + j + k = N/2 + 2.  Points whose index
    triples are permutations of one another share a weight; the weights solve
    sum w = 1 and sum w mu^(2k) = 1/(2k+1) for k = 2, 3, ... (one equation per
    weight class).  Returns (idx [n,3] 1-based, pts [n,3], w [n])."""
    if N not in _MU1:
        raise ValueError(f"unsupported S_N order {N}")
    half = N // 2
    mu1sq = _MU1[N] ** 2
    delta = 2.0 * (1.0 - 3.0 * mu1sq) / (N - 2) if N > 2 else 0.0
    mu = np.sqrt(mu1sq + delta * np.arange(half))
    idx = []
    for i in range(1, half + 1):
        for j in range(1, half + 1):
            k = half + 2 - i - j
            if 1 <= k <= half:
                idx.append((i, j, k))
    idx = np.array(idx, dtype=np.int64)
    pts = mu[idx - 1]
    classes = sorted({tuple(sorted(t)) for t in map(tuple, idx)})
    cls_of = np.array([classes.index(tuple(sorted(t))) for t in map(tuple, idx)])
    nc = len(classes)
    A = np.zeros((nc, nc))
    b = np.zeros(nc)
    A[0, :] = np.bincount(cls_of, minlength=nc)
    b[0] = 1.0
    for r in range(1, nc):
        k = r + 1
        A[r, :] = np.bincount(cls_of, weights=pts[:, 0] ** (2 * k), minlength=nc)
        b[r] = 1.0 / (2 * k + 1)
    wc = np.linalg.solve(A, b)
    return idx, pts, wc[cls_of]


def level_symmetric_2d(N: int):
    """2D level-symmetric set: directions (Omega_x, Omega_y, Omega_z) with
    Omega_z > 0.  Ordered by quadrant (+,+), (-,+), (-,-), (+,-) and, inside a
    quadrant, by the octant point order of ``level_symmetric_octant``.
    Weights sum to 4 pi.  Returns (omega [n_dir,3], w [n_dir])."""
    _, pts, w = level_symmetric_octant(N)
    signs = [(1, 1), (-1, 1), (-1, -1), (1, -1)]
    om, ww = [], []
    for sx, sy in signs:
        for (a, b, c), wi in zip(pts, w):
            om.append((sx * a, sy * b, c))
            # octant weights sum to 1 -> sphere sum 8; scale to 4 pi and
            # double for the discarded lower hemisphere
            ww.append(wi * (4.0 * math.pi / 8.0) * 2.0)
    return np.array(om), np.array(ww)


def gauss_legendre_unit(q: int):
    """q-point Gauss-Legendre rule on [0, 1] (exact to degree 2q-1)."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto_unit(p: int) -> np.ndarray:
    """p+1 Gauss-Lobatto points on [0, 1]: endpoints and the roots of P_p'."""
    if p < 1:
        raise ValueError("p must be >= 1")
    r = np.polynomial.legendre.Legendre.basis(p).deriv().roots().real
    x = np.concatenate([[-1.0], np.sort(r), [1.0]])
    return 0.5 * (x + 1.0)


def eb0(omega: np.ndarray, w: np.ndarray, n: np.ndarray) -> float:
    """Discrete E_b0 for unit normal n: sum_d w_d |Omega_d . n| / sum_d w_d
    (eq. eb0_disc)."""
    return float(np.sum(w * np.abs(omega[:, 0] * n[0] + omega[:, 1] * n[1])) / np.sum(w))
