"""The library's continuous (CG) moment system against the oracle, host only.

The library numbers the continuous unknowns by the structured node grid and
assembles A_c from element and boundary blocks; the oracle identifies nodes
by position and restricts the IP matrix to V_p.  The numberings differ, so
the comparison is made in the DG view P_c A_c P_c^T, which does not depend
on them, and the two partitions of the DG nodes into continuous unknowns
must be the same.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import smm as osmm
from workloads import config_blobs, config_channel, config_curved_mms, config_plain

L = pytest.importorskip("paper_2304_07386_amd")


@pytest.fixture(scope="module")
def hctx():
    return L.smm_ctx_create(-1)


def _cases():
    return [config_plain(n=5, p=1), config_plain(n=4, p=4, sn=6), config_curved_mms(n=4, p=2, sn=4),
            config_curved_mms(n=3, p=3, sn=4), config_channel(n=6, p=2, sn=4, side=1.3),
            config_blobs(20001, n=6, p=3, sn=4)]


@pytest.mark.parametrize("k", range(6))
def test_cg_system_matches_oracle(hctx, k):
    wl = _cases()[k]
    pr = osmm.make_problem(wl, disc="cg")
    p = L.problem_from_workload(hctx, wl, q=pr.q, psibar=pr.psibar)
    rowptr, col, val, cmap = L.smm_debug_cg_system(p)
    nc = len(rowptr) - 1
    assert nc == (wl.nx * wl.p + 1) * (wl.ny * wl.p + 1)
    assert np.all(np.diff(rowptr) > 0)
    for g in range(nc):
        assert np.all(np.diff(col[rowptr[g]:rowptr[g + 1]]) > 0)
    N = wl.n_elem * (wl.p + 1) ** 2
    Al = sp.csr_matrix((val, col, rowptr), shape=(nc, nc))
    Pl = sp.csr_matrix((np.ones(N), (np.arange(N), cmap)), shape=(N, nc))
    Po = osmm.cg_space(pr.mesh)
    Ao = osmm.cg_matrix(pr)
    # same partition of the DG nodes
    same_l = (Pl @ Pl.T).toarray() > 0
    same_o = (Po @ Po.T).toarray() > 0
    assert np.array_equal(same_l, same_o)
    Dl = (Pl @ Al @ Pl.T).toarray()
    Do = (Po @ Ao @ Po.T).toarray()
    assert np.abs(Dl - Do).max() <= 1e-12 * np.abs(Do).max()
