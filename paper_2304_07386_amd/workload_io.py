"""Marshal a workloads.Workload description into a libsmm problem.

Analytic sources and inflow functions are evaluated at the node and
boundary-point coordinates the library itself reports; explicit arrays
(``q``, ``psibar``) override them.
"""
from __future__ import annotations

import numpy as np

from . import smm as S


def problem_from_workload(ctx, wl, q=None, psibar=None):
    quad = getattr(wl, "quad", None)
    if getattr(wl, "elem_ctrl", None) is not None:
        prob = S.smm_problem_create_general(ctx, wl.elem_ctrl, wl.nbr, wl.m, wl.p, bdr_attr=wl.bdr_attr,
                                            sn=wl.sn, quad=quad)
    elif quad is not None:
        prob = S.smm_problem_create_q(ctx, wl.nx, wl.ny, wl.m, wl.ctrl, wl.p, quad=quad)
    else:
        prob = S.smm_problem_create(ctx, wl.nx, wl.ny, wl.m, wl.ctrl, wl.p, wl.sn)
    S.smm_set_materials(prob, wl.sigma_t, wl.sigma_s)
    n = prob.n_node
    if q is not None:
        q = np.asarray(q, dtype=np.float64)
        S.smm_set_source(prob, q, S.SMM_SRC_ANISO if q.ndim == 3 else S.SMM_SRC_ISO)
    elif wl.q_fn is not None:
        om, _ = S.smm_get_quadrature(prob)
        xy = S.smm_get_nodes(prob)
        qa = np.stack([wl.q_fn(xy[..., 0], xy[..., 1], o[0], o[1]) for o in om])
        S.smm_set_source(prob, qa, S.SMM_SRC_ANISO)
    else:
        S.smm_set_source(prob, np.repeat(np.asarray(wl.q_elem, float)[:, None], n, axis=1), S.SMM_SRC_ISO)
    if psibar is not None:
        S.smm_set_inflow(prob, psibar, S.SMM_INFLOW_FULL)
    elif isinstance(wl.inflow, str) or wl.inflow is None:
        S.smm_set_inflow(prob, None, S.SMM_INFLOW_VACUUM)
    elif wl.inflow[0] == "iso":
        S.smm_set_inflow(prob, np.full(prob.dims.n_bface, float(wl.inflow[1])), S.SMM_INFLOW_ISO_FACE)
    elif wl.inflow[0] == "attr":
        S.smm_set_inflow(prob, np.asarray(wl.inflow[1], dtype=np.float64), S.SMM_INFLOW_ISO_ATTR)
    else:
        om, _ = S.smm_get_quadrature(prob)
        xy = S.smm_get_bface_points(prob)
        f = wl.inflow[1]
        pb = f(xy[..., 0:1], xy[..., 1:2], om[None, None, :, 0], om[None, None, :, 1])
        S.smm_set_inflow(prob, np.ascontiguousarray(pb), S.SMM_INFLOW_FULL)
    return prob
