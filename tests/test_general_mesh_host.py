"""C-ABI set-up on meshes given element by element and on explicit angular
sets (no GPU): the library's host tables equal the oracle's.

* Geometry, IP operator and fixed right-hand side of eq. ipsmm, nodes and
  boundary points, on: the curved structured mesh with every element's local
  frame turned (all face pairings and reversed face parameterisations), the
  unstructured inner-square mesh (straight and curved), the same mesh turned
  as a whole (boundaries not along x or y: E_b0 per boundary point), a
  structured mesh with a slanted boundary, and a product angular set.
* Inflow given per boundary attribute.
* Sweep graph (levels, upstream faces) bit for bit.
* Refusals: faces that do not match, bad neighbour indices, negative
  attributes, bad explicit sets, tiles and the CG system on general meshes.
"""
import numpy as np
import pytest

from oracle import fem, transport
from oracle import smm as osmm
from workloads import (Workload, config_curved_mms, general_workload, inner_square_mesh, product_quadrature_2d,
                       rotate_elements, structured_ctrl)

L = pytest.importorskip("paper_2304_07386_amd")


@pytest.fixture(scope="module")
def hctx():
    return L.smm_ctx_create(-1)


def _rot_curved(p, sn=4):
    wl = config_curved_mms(4, p, sn, amplitude=0.06)
    ctrl_e, nbr = fem.structured_elements(wl.ctrl, 4, 4, p)
    ce, nb = rotate_elements(ctrl_e, nbr, np.random.default_rng(3).integers(0, 4, 16))
    return general_workload("rotated", ce, nb, p, p, sn, wl.sigma_t, wl.sigma_s, q_fn=wl.q_fn, inflow=wl.inflow)


def _inner(k, m, p, turn=0.0, sn=6, quad=None):
    bump = (lambda x, y: (0.03 * np.sin(np.pi * x) * np.sin(np.pi * y), -0.02 * np.sin(np.pi * x) * np.sin(np.pi * y)))
    ce, nb, at = inner_square_mesh(k, m, displace=bump if m > 1 else None)
    if turn:
        c, s = np.cos(turn), np.sin(turn)
        ce = np.stack([c * ce[..., 0] - s * ce[..., 1], s * ce[..., 0] + c * ce[..., 1]], axis=-1)
    ne = len(ce)
    rng = np.random.default_rng(k * 10 + m)
    st = rng.choice([0.5, 3.0], size=ne)
    return general_workload("inner", ce, nb, m, p, sn, st, 0.6 * st, bdr_attr=at, q_elem=rng.uniform(0.1, 1.0, ne),
                            inflow=("attr", [0.2, 0.0, 0.7, 0.4]), quad=quad)


def _slanted(p):
    xv = np.linspace(0, 1, 4)
    ctrl = structured_ctrl(xv, xv, 1)
    ctrl[..., 0] += 0.3 * ctrl[..., 1]            # a parallelogram: slanted left and right sides
    ne = 9
    return Workload("slanted", 3, 3, 1, p, 6, ctrl, np.full(ne, 2.0), np.full(ne, 1.0), q_elem=np.ones(ne),
                    inflow=("iso", 0.3))


CASES = {
    "rotated_p1": lambda: _rot_curved(1),
    "rotated_p2": lambda: _rot_curved(2),
    "rotated_p3": lambda: _rot_curved(3),
    "inner_m1_p2": lambda: _inner(2, 1, 2),
    "inner_m2_p2": lambda: _inner(2, 2, 2),
    "inner_turned_m2_p3": lambda: _inner(1, 2, 3, turn=0.35),
    "slanted_p2": lambda: _slanted(2),
    "inner_product_quad": lambda: _inner(1, 1, 2, quad=product_quadrature_2d(2, 8)),
    "structured_product_quad": lambda: _with_quad(config_curved_mms(3, 2, 4), product_quadrature_2d(3, 12)),
}


def _with_quad(wl, quad):
    wl.quad = quad
    return wl


@pytest.mark.parametrize("name", list(CASES))
def test_general_setup_matches_oracle(hctx, name):
    wl = CASES[name]()
    pr = osmm.make_problem(wl)
    iso = isinstance(wl.inflow, tuple) and wl.inflow[0] in ("iso", "attr")
    p = L.problem_from_workload(hctx, wl, q=pr.q, psibar=None if iso else pr.psibar)
    A1, b1 = L.smm_debug_ip_dense(p)
    A0 = osmm.ip_matrix(pr).toarray()
    b0 = osmm.rhs_fixed(pr)
    assert np.abs(A1 - A0).max() <= 1e-13 * np.abs(A0).max()
    assert np.abs(b1 - b0).max() <= 1e-13 * max(np.abs(b0).max(), 1.0)
    om, w = L.smm_get_quadrature(p)
    assert np.abs(om - pr.omega).max() < 1e-15 and np.abs(w - pr.w).max() < 1e-14
    assert np.abs(L.smm_get_nodes(p) - pr.mesh.xnode).max() < 1e-14
    xb = L.smm_get_bface_points(p)
    for b, (K, f) in enumerate(pr.mesh.bfaces):
        assert np.abs(xb[b] - pr.mesh.xf[K, f]).max() < 1e-14
    d = L.smm_get_dims(p)
    assert d["cartesian"] == 0
    assert d["general"] == (1 if wl.elem_ctrl is not None else 0)
    lev, up = L.smm_debug_sweep_graph(p)
    for k in range(len(pr.w)):
        ups, lv = transport.sweep_graph(pr.mesh, pr.omega[k])
        bits = (ups.astype(np.uint8) << np.arange(4, dtype=np.uint8)).sum(axis=1).astype(np.uint8)
        assert np.array_equal(lev[k], lv) and np.array_equal(up[k], bits), k


def test_general_refusals(hctx):
    wl = _inner(1, 1, 1)
    ce, nb = wl.elem_ctrl, wl.nbr
    bad = nb.copy()
    K = int(np.nonzero((nb >= 0).all(axis=1) | (nb >= 0).any(axis=1))[0][0])
    f = int(np.nonzero(nb[K] >= 0)[0][0])
    bad[K, f] = (nb[K, f] + 1) % len(ce)          # a neighbour that does not share the face
    if bad[K, f] == K:
        bad[K, f] = (bad[K, f] + 1) % len(ce)
    with pytest.raises(L.SmmError) as e:
        L.smm_problem_create_general(hctx, ce, bad, 1, 1, sn=4)
    assert e.value.code == L.SMM_EINVAL
    bad = nb.copy()
    bad[0, 0] = len(ce)
    with pytest.raises(L.SmmError) as e:
        L.smm_problem_create_general(hctx, ce, bad, 1, 1, sn=4)
    assert e.value.code == L.SMM_EINVAL
    at = np.where(nb < 0, -2, -1)
    with pytest.raises(L.SmmError) as e:
        L.smm_problem_create_general(hctx, ce, nb, 1, 1, bdr_attr=at, sn=4)
    assert e.value.code == L.SMM_EINVAL
    om, w = product_quadrature_2d(2, 8)
    for qbad, code in (((om, 1.01 * w), L.SMM_EINVAL), ((om * 1.01, w), L.SMM_EINVAL),
                       ((np.array([[1.0, 0.0, 0.0]]), np.array([4 * np.pi])), L.SMM_EUNSUPPORTED)):
        with pytest.raises(L.SmmError) as e:
            L.smm_problem_create_general(hctx, ce, nb, 1, 1, quad=qbad)
        assert e.value.code == code
    p = L.smm_problem_create_general(hctx, ce, nb, 1, 1, bdr_attr=wl.bdr_attr, sn=4)
    assert p.dims.general == 1 and p.dims.n_bdr_attr == 4
    with pytest.raises(L.SmmError) as e:
        L.smm_set_sweep_tiles(p, 2, 2)
    assert e.value.code == L.SMM_EUNSUPPORTED
    L.smm_set_materials(p, np.ones(len(ce)), np.full(len(ce), 0.5))
    with pytest.raises(L.SmmError) as e:
        L.smm_debug_cg_system(p)
    assert e.value.code == L.SMM_EUNSUPPORTED
