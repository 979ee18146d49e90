"""Helpers shared by the GPU tests: device context and oracle/HIP problem
pairs built from the same seeded workload."""
from __future__ import annotations

import sys

import numpy as np

from oracle import smm as osmm


def rel_l2(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def make_pair(L, ctx, wl):
    """Oracle problem and HIP problem on identical inputs (the nodal source
    and inflow tables are built once, by the oracle, and handed to both; an
    isotropic face inflow keeps its compact layout, with the same value)."""
    pr = osmm.make_problem(wl)
    iso_inflow = isinstance(wl.inflow, tuple) and wl.inflow[0] == "iso"
    p = L.problem_from_workload(ctx, wl, q=pr.q, psibar=None if iso_inflow else pr.psibar)
    return pr, p
