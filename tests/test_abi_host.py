"""C-ABI library checks that need no GPU.

* libsmm.so loads and exports every function declared in include/*.h.
* Host-only contexts run the one-time setup; its tables equal the oracle's
  (IP operator and fixed right-hand side of eq. ipsmm, quadrature, node
  coordinates) on straight, non-uniform and curved meshes.
* The sweep graph (levels and upstream faces per direction, Sec. 4) equals
  the oracle's bit for bit on curved meshes and with tiles; a mesh whose
  upwind graph has a cycle is refused.
* Argument validation and error codes (forced from the host).
"""
import os
import re

import numpy as np
import pytest

from oracle import smm as osmm
from workloads import config_channel, config_curved_mms, config_plain, structured_ctrl

L = pytest.importorskip("paper_2304_07386_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_header_symbols():
    lib = L.load_library()
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            hdr = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:int|void|const char\*)\s+(smm_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 40
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.EXPORTED) == names


@pytest.fixture(scope="module")
def hctx():
    return L.smm_ctx_create(-1)


def _compare(hctx, wl):
    pr = osmm.make_problem(wl)
    p = L.problem_from_workload(hctx, wl, q=pr.q, psibar=pr.psibar)
    A1, b1 = L.smm_debug_ip_dense(p)
    A0 = osmm.ip_matrix(pr).toarray()
    b0 = osmm.rhs_fixed(pr)
    om, w = L.smm_get_quadrature(p)
    assert np.abs(A1 - A0).max() <= 1e-13 * np.abs(A0).max()
    assert np.abs(b1 - b0).max() <= 1e-13 * max(np.abs(b0).max(), 1.0)
    assert np.abs(om - pr.omega).max() < 1e-15 and np.abs(w - pr.w).max() < 1e-14
    assert np.abs(L.smm_get_nodes(p) - pr.mesh.xnode).max() < 1e-14
    xb = L.smm_get_bface_points(p)
    for b, (K, f) in enumerate(pr.mesh.bfaces):
        assert np.abs(xb[b] - pr.mesh.xf[K, f]).max() < 1e-14
    L.smm_get_dims(p)
    return p


def test_setup_matches_oracle_plain(hctx):
    p = _compare(hctx, config_plain())
    assert p.dims.cartesian == 1 and p.dims.n_material == 1


def test_setup_matches_oracle_curved(hctx):
    for pp in (2, 3):
        p = _compare(hctx, config_curved_mms(n=4, p=pp, sn=8))
        assert p.dims.cartesian == 0


def test_setup_matches_oracle_nonuniform_inflow(hctx):
    from tests.test_oracle_smm import _patch_workload
    wl, _, _ = _patch_workload(3)
    p = _compare(hctx, wl)
    assert p.dims.cartesian == 0


def test_channel_layout_materials(hctx):
    wl = config_channel(n=32, side=2.5)
    p = L.problem_from_workload(hctx, wl)
    L.smm_debug_ip_dense(p)
    L.smm_get_dims(p)
    assert p.dims.cartesian == 1 and p.dims.n_material == 2
    assert set(np.unique(wl.sigma_t)) == {0.2, 200.0}


def test_validation_errors(hctx):
    wl = config_plain(n=2)
    with pytest.raises(L.SmmError) as e:
        L.smm_problem_create(hctx, 2, 2, 1, wl.ctrl, 5, 4)
    assert e.value.code == L.SMM_EINVAL
    with pytest.raises(L.SmmError) as e:
        L.smm_problem_create(hctx, 2, 2, 1, wl.ctrl, 1, 5)
    assert e.value.code == L.SMM_EINVAL
    # inverted element -> det J <= 0
    bad = wl.ctrl.copy()
    bad[1, 1] = [1.5, 1.5]
    with pytest.raises(L.SmmError) as e:
        L.smm_problem_create(hctx, 2, 2, 1, bad, 1, 4)
    assert e.value.code == L.SMM_EINVAL
    # a slanted boundary runs on the per-element paths (E_b0 per boundary point)
    sl = wl.ctrl.copy()
    sl[0, 1] = [0.5, -0.1]
    ps = L.smm_problem_create(hctx, 2, 2, 1, sl, 1, 4)
    assert ps.dims.cartesian == 0
    p = L.smm_problem_create(hctx, 2, 2, 1, wl.ctrl, 1, 4)
    with pytest.raises(L.SmmError) as e:
        L.smm_set_materials(p, np.ones(4), np.full(4, 2.0))
    assert e.value.code == L.SMM_EINVAL
    with pytest.raises(L.SmmError) as e:
        L.smm_debug_ip_dense(p)          # materials not set yet
    assert e.value.code == L.SMM_ESTATE
    L.smm_set_materials(p, np.ones(4), np.full(4, 0.5))
    with pytest.raises(L.SmmError) as e:
        L.smm_set_source(p, np.full((4, 4), np.nan))
    assert e.value.code == L.SMM_EINVAL
    # a host-only context refuses to run the solve path
    with pytest.raises(L.SmmError) as e:
        L.smm_solve(p)
    assert e.value.code == L.SMM_ESTATE


def test_warmstart_calls_need_a_device(hctx):
    """The network lives on a device: a host-only context is refused."""
    lib = L.load_library()
    import ctypes as C
    ch = (C.c_int * 3)(14, 32, 18)
    h = C.c_void_p()
    assert lib.smm_cnn_create(hctx.handle, 2, ch, 8, 8, 4, C.byref(h)) == L.SMM_ESTATE
    assert lib.smm_cnn_create(hctx.handle, 0, ch, 8, 8, 4, C.byref(h)) in (L.SMM_ESTATE, L.SMM_EINVAL)
    assert lib.smm_batch_warmstart_used(None, None) == L.SMM_EINVAL


def test_tiles_and_cg_calls_on_the_host(hctx):
    """smm_set_sweep_tiles and smm_set_sweep_path validate their arguments;
    the continuous system and the tiles are set-up work, so a host-only
    context accepts them, while the device calls that use them are refused."""
    wl = config_plain(n=4, p=2)
    p = L.problem_from_workload(hctx, wl)
    for bad in ((-1, 2), (2, 0), (0, 3)):
        with pytest.raises(L.SmmError) as e:
            L.smm_set_sweep_tiles(p, *bad)
        assert e.value.code == L.SMM_EINVAL
    L.smm_set_sweep_tiles(p, 2, 2)
    L.smm_set_sweep_tiles(p, 0, 0)
    # sweep kernel selection: 0..5 (3 = one wave per element, 4 = one lane per
    # row, 5 = the assembling forms chosen as 0 chooses them)
    for bad in (-1, 6):
        with pytest.raises(L.SmmError) as e:
            L.smm_set_sweep_path(p, bad)
        assert e.value.code == L.SMM_EINVAL
    for path in (3, 4, 5, 0):
        L.smm_set_sweep_path(p, path)
    rowptr, col, val, cmap = L.smm_debug_cg_system(p)
    assert len(rowptr) == (4 * 2 + 1) ** 2 + 1 and cmap.max() == (4 * 2 + 1) ** 2 - 1
    with pytest.raises(L.SmmError) as e:
        L.smm_debug_cg_spmv(p, np.ones(len(rowptr) - 1))
    assert e.value.code == L.SMM_ESTATE
    with pytest.raises(L.SmmError) as e:
        L.smm_solve(p, L.smm_default_opts(discretization=L.SMM_DISC_CG))
    assert e.value.code == L.SMM_ESTATE


def _graph_compare(p, pr, block=None):
    from oracle import transport
    lev, up = L.smm_debug_sweep_graph(p)
    for d in range(len(pr.w)):
        ups, lv = transport.sweep_graph(pr.mesh, pr.omega[d], block)
        bits = (ups.astype(np.uint8) << np.arange(4, dtype=np.uint8)).sum(axis=1).astype(np.uint8)
        assert np.array_equal(lev[d], lv), d
        assert np.array_equal(up[d], bits), d


@pytest.mark.parametrize("amp,p", [(0.09, 2), (0.09, 3), (0.0, 1)])
def test_sweep_graph_matches_oracle(hctx, amp, p):
    wl = config_curved_mms(n=7, p=p, sn=8, amplitude=amp)
    pr = osmm.make_problem(wl)
    _graph_compare(L.problem_from_workload(hctx, wl, q=pr.q, psibar=pr.psibar), pr)


def test_sweep_graph_tiles_match_oracle(hctx):
    from oracle import transport
    wl = config_curved_mms(n=9, p=2, sn=6, amplitude=0.09)
    pr = osmm.make_problem(wl, tiles=(4, 3))
    p = L.problem_from_workload(hctx, wl, q=pr.q, psibar=pr.psibar)
    L.smm_set_sweep_tiles(p, 4, 3)
    _graph_compare(p, pr, transport.block_ids(pr.mesh, 4, 3))


def test_cyclic_sweep_graph_refused(hctx):
    # 2 x 2 straight elements whose shared vertex sits inside the triangle of
    # element 0's other three corners: that chord quadrilateral has a reflex
    # angle there (det J stays positive at the Gauss points), the four faces
    # around the vertex span less than 180 degrees, and directions across
    # them circulate 0 -> 1 -> 3 -> 2 -> 0
    from oracle import fem, transport
    from workloads import Workload
    ctrl = structured_ctrl(np.array([0.0, 1.0, 2.0]), np.array([0.0, 1.0, 2.0]), 1)
    ctrl[1, 1] = (0.48, 0.48)
    wl = Workload("dart", 2, 2, 1, 1, 4, ctrl, np.ones(4), np.full(4, 0.5), q_elem=np.ones(4))
    pr = osmm.make_problem(wl)
    with pytest.raises(RuntimeError, match="cycle"):
        for d in range(len(pr.w)):
            transport.sweep_graph(pr.mesh, pr.omega[d])
    with pytest.raises(L.SmmError) as e:
        L.smm_problem_create(hctx, 2, 2, 1, ctrl, 1, 4)
    assert e.value.code == L.SMM_EUNSUPPORTED and "cycle" in str(e.value)
