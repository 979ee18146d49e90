"""Pins of the oracle's parallel block Jacobi sweep (Sec. 6.5), no GPU.

Each block of elements is swept on its own; inflow across a face between
blocks is the previous sweep's.  Tied to:
* one block covering the mesh: the full sweep, exactly;
* consistency: with the exact sweep as the lagged input, the block sweep
  returns the exact sweep (it is a splitting L = L_blocks - B of the same
  operator);
* the SMM fixed point does not change (the lag vanishes at convergence):
  converged fluxes with and without blocks agree;
* more blocks, more outer iterations (Table tab:weak_itr: the outer
  iteration count grows with the number of subdomains).
"""
import numpy as np
import pytest

from oracle import smm, transport
from workloads import config_channel, config_plain


def _two_mat(n=6, p=2, sn=4):
    wl = config_channel(n=n, p=p, sn=sn, side=1.3)
    wl.inflow = ("iso", 0.5)
    return wl


def test_one_block_is_full_sweep():
    prob = smm.make_problem(_two_mat())
    rng = np.random.default_rng(0)
    S = rng.uniform(0.5, 1.5, size=(prob.ne, prob.n))
    full = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar)
    one = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar, None,
                          transport.block_ids(prob.mesh, 6, 6))
    assert np.array_equal(full, one)


@pytest.mark.parametrize("tiles", [(2, 2), (3, 2), (1, 1), (4, 5)])
def test_block_sweep_with_exact_lag_is_exact(tiles):
    for wl in (_two_mat(), config_plain(n=5, p=3, sn=6)):
        prob = smm.make_problem(wl)
        rng = np.random.default_rng(1)
        S = rng.uniform(0.5, 1.5, size=(prob.ne, prob.n))
        full = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar)
        blk = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar, full,
                              transport.block_ids(prob.mesh, *tiles))
        assert np.abs(blk - full).max() < 1e-13 * np.abs(full).max()
        # and without the lag (zero inflow between blocks) it differs
        lag0 = transport.sweep(prob.mesh, prob.omega, prob.sigma_t, S, prob.psibar, None,
                               transport.block_ids(prob.mesh, *tiles))
        assert np.abs(lag0 - full).max() > 1e-3 * np.abs(full).max()


@pytest.mark.parametrize("p", [1, 2])
def test_block_jacobi_fixed_point_unchanged(p):
    wl = _two_mat(n=6, p=p)
    x0, i0 = smm.solve(smm.make_problem(wl), tol=1e-13, max_it=300)
    x1, i1 = smm.solve(smm.make_problem(wl, tiles=(2, 3)), tol=1e-13, max_it=300)
    assert i0["converged"] and i1["converged"]
    assert np.abs(x1 - x0).max() < 1e-10 * np.abs(x0).max()
    assert i1["iterations"] > i0["iterations"]


def test_more_blocks_more_outer_iterations():
    wl = config_plain(n=8, p=1, sn=4)
    counts = []
    for t in (8, 4, 2, 1):
        x, info = smm.solve(smm.make_problem(wl, tiles=(t, t)), tol=1e-8, max_it=500)
        assert info["converged"]
        counts.append(info["iterations"])
    assert counts == sorted(counts) and counts[-1] > counts[0], counts
