"""Thin Python binding of libsmm (include/smm.h).

Argument marshalling only: every computation runs inside libsmm.so (host
setup in C++, the solve path in HIP kernels).  Functions keep the C names;
host arrays are numpy float64, device arrays are torch CUDA tensors (only
their data pointers are passed).  A non-zero status raises SmmError.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmm.so")

SMM_OK, SMM_EINVAL, SMM_ENOMEM, SMM_EHIP, SMM_ENOCONV, SMM_ENAN, SMM_EBREAKDOWN, SMM_EUNSUPPORTED, SMM_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
SMM_FP64, SMM_FP32_SWEEP = 0, 1
SMM_SRC_ISO, SMM_SRC_ANISO = 0, 1
SMM_INFLOW_VACUUM, SMM_INFLOW_ISO_FACE, SMM_INFLOW_FULL, SMM_INFLOW_ISO_ATTR = 0, 1, 2, 3
SMM_QUAD_LEVEL_SYMMETRIC, SMM_QUAD_EXPLICIT = 0, 1
SMM_START_ZERO, SMM_START_DIFFUSION, SMM_START_GIVEN = 0, 1, 2
SMM_DISC_IP, SMM_DISC_CG = 0, 1

EXPORTED = [
    "smm_strerror", "smm_ctx_create", "smm_ctx_destroy", "smm_last_error", "smm_problem_create",
    "smm_problem_create_general", "smm_problem_create_q",
    "smm_problem_destroy", "smm_get_dims", "smm_get_quadrature", "smm_get_nodes", "smm_get_bface_points",
    "smm_set_materials", "smm_set_source", "smm_set_inflow", "smm_default_opts", "smm_solve",
    "smm_get_outputs", "smm_apply_sweep", "smm_apply_moments", "smm_apply_G", "smm_debug_ip_dense",
    "smm_debug_cg_system", "smm_debug_cg_spmv", "smm_time_cg_spmv", "smm_set_sweep_tiles",
    "smm_set_sweep_path", "smm_time_sweep", "smm_debug_typed_dense", "smm_debug_corr_dense",
    "smm_batch_create", "smm_batch_destroy", "smm_batch_solve", "smm_batch_get_outputs",
    "smm_batch_time_sweep", "smm_batch_units", "smm_batch_phase_times", "smm_batch_time_kernel",
    "smm_batch_history", "smm_debug_mg_level", "smm_debug_batch_precond", "smm_debug_batch_spmv",
    "smm_debug_batch_grouped", "smm_debug_sweep_graph", "smm_batch_apply_sweep", "smm_apply_G_noalloc", "smm_solve_history",
    "smm_debug_batch_sweep_shape", "smm_debug_cg_mg_level", "smm_time_sweep_parts", "smm_debug_batch_cg_fork",
    # smm_cnn.h
    "smm_cnn_create", "smm_cnn_destroy", "smm_cnn_num_params", "smm_cnn_set_params", "smm_cnn_get_params",
    "smm_cnn_forward", "smm_cnn_loss_grad", "smm_cnn_adam_step", "smm_batch_warmstart_dims",
    "smm_batch_diffusion", "smm_batch_warmstart_features", "smm_batch_warmstart_targets",
    "smm_batch_set_warmstart", "smm_batch_warmstart_used", "smm_set_warmstart",
]


class SmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsmm error {code}: {msg}")
        self.code = code


class smm_mesh_desc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("m", C.c_int), ("ctrl", C.POINTER(C.c_double))]


class smm_mesh_general_desc(C.Structure):
    _fields_ = [("n_elem", C.c_int), ("m", C.c_int), ("ctrl", C.POINTER(C.c_double)), ("nbr", C.POINTER(C.c_int)),
                ("bdr_attr", C.POINTER(C.c_int))]


class smm_quad_desc(C.Structure):
    _fields_ = [("kind", C.c_int), ("sn_order", C.c_int), ("n_dir", C.c_int), ("omega", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double))]


class smm_problem_dims(C.Structure):
    _fields_ = [("n_elem", C.c_int), ("n_node", C.c_int), ("n_dir", C.c_int), ("n_bface", C.c_int),
                ("nq", C.c_int), ("cartesian", C.c_int), ("n_material", C.c_int), ("n_levels", C.c_int),
                ("n_self_types", C.c_int), ("n_nbr_types", C.c_int), ("general", C.c_int), ("n_bdr_attr", C.c_int)]


class smm_solve_opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("outer_tol", C.c_double), ("max_outer", C.c_int),
                ("inner_tol", C.c_double), ("max_inner", C.c_int), ("start", C.c_int),
                ("delta_sweeps", C.c_int), ("use_graph", C.c_int), ("moment_path", C.c_int),
                ("anderson", C.c_int), ("precond", C.c_int), ("inner_adapt", C.c_double),
                ("discretization", C.c_int), ("kappa_scale", C.c_double), ("start_tol", C.c_double)]


class smm_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("residual", C.c_double), ("residual_abs", C.c_double),
                ("cg_iterations_total", C.c_int), ("cg_iterations_max", C.c_int),
                ("t_total_ms", C.c_double), ("t_setup_ms", C.c_double), ("t_sweep_ms", C.c_double),
                ("t_moments_ms", C.c_double), ("t_cg_ms", C.c_double), ("t_residual_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsmm.so (built in-tree by paper_2304_07386_amd.build).  Raises
    if it is missing: there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libsmm.so not built at {path}; run __graft_entry__.build()")
    lib = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
    sig = {
        "smm_strerror": (C.c_char_p, [ip]),
        "smm_ctx_create": (ip, [ip, vp, C.POINTER(vp)]),
        "smm_ctx_destroy": (ip, [vp]),
        "smm_last_error": (C.c_char_p, [vp]),
        "smm_problem_create": (ip, [vp, C.POINTER(smm_mesh_desc), ip, ip, C.POINTER(vp)]),
        "smm_problem_destroy": (ip, [vp]),
        "smm_problem_create_general": (ip, [vp, C.POINTER(smm_mesh_general_desc), ip, C.POINTER(smm_quad_desc),
                                            C.POINTER(vp)]),
        "smm_problem_create_q": (ip, [vp, C.POINTER(smm_mesh_desc), ip, C.POINTER(smm_quad_desc), C.POINTER(vp)]),
        "smm_get_dims": (ip, [vp, C.POINTER(smm_problem_dims)]),
        "smm_get_quadrature": (ip, [vp, vp, vp]),
        "smm_get_nodes": (ip, [vp, vp]),
        "smm_get_bface_points": (ip, [vp, vp]),
        "smm_set_materials": (ip, [vp, vp, vp]),
        "smm_set_source": (ip, [vp, vp, ip]),
        "smm_set_inflow": (ip, [vp, vp, ip]),
        "smm_default_opts": (None, [C.POINTER(smm_solve_opts)]),
        "smm_solve": (ip, [vp, C.POINTER(smm_solve_opts), vp, C.POINTER(smm_solve_info)]),
        "smm_solve_history": (ip, [vp, ip, vp, vp, C.POINTER(ip)]),
        "smm_set_warmstart": (ip, [vp, vp]),
        "smm_get_outputs": (ip, [vp, vp, vp, vp, vp, vp, ip]),
        "smm_apply_sweep": (ip, [vp, ip, vp, ip, vp, vp, ip]),
        "smm_apply_moments": (ip, [vp, ip, vp, vp]),
        "smm_apply_G": (ip, [vp, ip, vp, vp, C.c_double, ip]),
        "smm_apply_G_noalloc": (ip, [vp, ip, vp, vp, C.c_double, ip]),
        "smm_debug_ip_dense": (ip, [vp, vp, vp]),
        "smm_debug_cg_system": (ip, [vp, vp, vp, vp, vp, vp, vp]),
        "smm_debug_cg_spmv": (ip, [vp, vp, vp]),
        "smm_time_cg_spmv": (ip, [vp, ip, dp]),
        "smm_set_sweep_tiles": (ip, [vp, ip, ip]),
        "smm_set_sweep_path": (ip, [vp, ip]),
        "smm_time_sweep": (ip, [vp, ip, ip, dp]),
        "smm_debug_typed_dense": (ip, [vp, vp, vp, vp]),
        "smm_debug_corr_dense": (ip, [vp, vp]),
        "smm_debug_sweep_graph": (ip, [vp, vp, vp]),
        "smm_batch_apply_sweep": (ip, [vp, ip, C.POINTER(vp), ip, vp]),
        "smm_batch_create": (ip, [vp, C.POINTER(vp), ip, C.POINTER(vp)]),
        "smm_batch_destroy": (ip, [vp]),
        "smm_batch_solve": (ip, [vp, C.POINTER(smm_solve_opts), C.POINTER(vp), C.POINTER(smm_solve_info)]),
        "smm_batch_get_outputs": (ip, [vp, ip, vp, vp, vp, vp, vp, ip]),
        "smm_batch_time_sweep": (ip, [vp, ip, ip, dp]),
        "smm_batch_units": (ip, [vp, dp]),
        "smm_batch_phase_times": (ip, [vp, dp, C.POINTER(C.c_long)]),
        "smm_batch_time_kernel": (ip, [vp, ip, ip, dp]),
        "smm_batch_history": (ip, [vp, ip, ip, vp, vp, C.POINTER(ip)]),
        "smm_debug_mg_level": (ip, [vp, ip, vp, C.POINTER(ip), C.POINTER(ip)]),
        "smm_debug_cg_mg_level": (ip, [vp, ip, vp, C.POINTER(ip), C.POINTER(ip)]),
        "smm_time_sweep_parts": (ip, [vp, ip, ip, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
        "smm_debug_batch_precond": (ip, [vp, ip, C.POINTER(vp), C.POINTER(vp)]),
        "smm_debug_batch_spmv": (ip, [vp, C.POINTER(vp), C.POINTER(vp)]),
        "smm_debug_batch_grouped": (ip, [vp, ip]),
        "smm_debug_batch_sweep_shape": (ip, [vp, ip]),
        "smm_debug_batch_cg_fork": (ip, [vp, ip]),
        "smm_cnn_create": (ip, [vp, ip, C.POINTER(ip), ip, ip, ip, C.POINTER(vp)]),
        "smm_cnn_destroy": (ip, [vp]),
        "smm_cnn_num_params": (ip, [vp, C.POINTER(C.c_size_t)]),
        "smm_cnn_set_params": (ip, [vp, vp, C.c_size_t]),
        "smm_cnn_get_params": (ip, [vp, vp, C.c_size_t]),
        "smm_cnn_forward": (ip, [vp, vp, ip, vp]),
        "smm_cnn_loss_grad": (ip, [vp, vp, vp, ip, vp, ip, vp, dp, vp]),
        "smm_cnn_adam_step": (ip, [vp, C.c_float, C.c_float, C.c_float, C.c_float]),
        "smm_batch_warmstart_dims": (ip, [vp, C.POINTER(ip), C.POINTER(ip), C.POINTER(ip), C.POINTER(ip)]),
        "smm_batch_diffusion": (ip, [vp, C.c_double, ip]),
        "smm_batch_warmstart_features": (ip, [vp, ip, ip, vp]),
        "smm_batch_warmstart_targets": (ip, [vp, ip, ip, vp]),
        "smm_batch_set_warmstart": (ip, [vp, vp]),
        "smm_batch_warmstart_used": (ip, [vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    """Data pointer of a numpy array (host) or torch tensor (device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Context:
    def __init__(self, handle):
        self.handle = handle


def _check(rc, ctx=None):
    if rc != SMM_OK:
        lib = load_library()
        msg = lib.smm_strerror(rc).decode()
        if ctx is not None:
            detail = lib.smm_last_error(ctx.handle)
            if detail:
                msg += f" ({detail.decode()})"
        raise SmmError(rc, msg)


def smm_ctx_create(device: int = 0, stream=None) -> Context:
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
    lib = load_library()
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    h = C.c_void_p()
    _check(lib.smm_ctx_create(device, C.c_void_p(stream) if stream else None, C.byref(h)))
    return Context(h)


def smm_ctx_destroy(ctx: Context):
    load_library().smm_ctx_destroy(ctx.handle)


class Problem:
    """Handle of one smm_problem plus the context it belongs to."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        d = smm_problem_dims()
        _check(load_library().smm_get_dims(handle, C.byref(d)), ctx)
        self.dims = d

    @property
    def n_elem(self):
        return self.dims.n_elem

    @property
    def n_node(self):
        return self.dims.n_node

    @property
    def n_dir(self):
        return self.dims.n_dir


def smm_problem_create(ctx: Context, nx: int, ny: int, m: int, ctrl: np.ndarray, p: int, sn: int) -> Problem:
    lib = load_library()
    ctrl = _f64(ctrl)
    assert ctrl.size == (ny * m + 1) * (nx * m + 1) * 2
    desc = smm_mesh_desc(nx, ny, m, ctrl.ctypes.data_as(C.POINTER(C.c_double)))
    h = C.c_void_p()
    _check(lib.smm_problem_create(ctx.handle, C.byref(desc), p, sn, C.byref(h)), ctx)
    return Problem(ctx, h)


def _quad_desc(sn: int = 0, quad=None):
    """Quadrature descriptor and the arrays it points to (kept alive by the caller)."""
    if quad is None:
        return smm_quad_desc(SMM_QUAD_LEVEL_SYMMETRIC, int(sn), 0, None, None), ()
    om, w = _f64(quad[0]).reshape(-1, 3), _f64(quad[1]).reshape(-1)
    return smm_quad_desc(SMM_QUAD_EXPLICIT, 0, len(w), om.ctypes.data_as(C.POINTER(C.c_double)),
                         w.ctypes.data_as(C.POINTER(C.c_double))), (om, w)


def smm_problem_create_q(ctx: Context, nx: int, ny: int, m: int, ctrl: np.ndarray, p: int, sn: int = 0,
                         quad=None) -> Problem:
    """Structured mesh with the level-symmetric set of order sn, or the
    explicit set quad = (omega [n_dir, 3], w [n_dir])."""
    ctrl = _f64(ctrl)
    assert ctrl.size == (ny * m + 1) * (nx * m + 1) * 2
    desc = smm_mesh_desc(nx, ny, m, ctrl.ctypes.data_as(C.POINTER(C.c_double)))
    qd, keep = _quad_desc(sn, quad)
    h = C.c_void_p()
    _check(load_library().smm_problem_create_q(ctx.handle, C.byref(desc), p, C.byref(qd), C.byref(h)), ctx)
    return Problem(ctx, h)


def smm_problem_create_general(ctx: Context, elem_ctrl: np.ndarray, nbr: np.ndarray, m: int, p: int,
                               bdr_attr=None, sn: int = 0, quad=None) -> Problem:
    """Mesh given element by element: elem_ctrl [ne, (m+1)^2, 2], nbr [ne, 4]
    (-1: boundary), bdr_attr [ne, 4] or None; level-symmetric order sn or an
    explicit set quad = (omega, w)."""
    ctrl = _f64(elem_ctrl)
    ne = len(ctrl)
    assert ctrl.size == ne * (m + 1) ** 2 * 2
    nb = np.ascontiguousarray(np.asarray(nbr, dtype=np.int32).reshape(ne, 4))
    at = None if bdr_attr is None else np.ascontiguousarray(np.asarray(bdr_attr, dtype=np.int32).reshape(ne, 4))
    desc = smm_mesh_general_desc(ne, m, ctrl.ctypes.data_as(C.POINTER(C.c_double)),
                                 nb.ctypes.data_as(C.POINTER(C.c_int)),
                                 None if at is None else at.ctypes.data_as(C.POINTER(C.c_int)))
    qd, keep = _quad_desc(sn, quad)
    h = C.c_void_p()
    _check(load_library().smm_problem_create_general(ctx.handle, C.byref(desc), p, C.byref(qd), C.byref(h)), ctx)
    return Problem(ctx, h)


def smm_problem_destroy(prob: Problem):
    load_library().smm_problem_destroy(prob.handle)


def smm_get_dims(prob: Problem) -> dict:
    d = smm_problem_dims()
    _check(load_library().smm_get_dims(prob.handle, C.byref(d)), prob.ctx)
    prob.dims = d
    return {k: getattr(d, k) for k, _ in d._fields_}


def smm_get_quadrature(prob: Problem):
    om = np.zeros((prob.n_dir, 3))
    w = np.zeros(prob.n_dir)
    _check(load_library().smm_get_quadrature(prob.handle, _ptr(om), _ptr(w)), prob.ctx)
    return om, w


def smm_get_nodes(prob: Problem):
    xy = np.zeros((prob.n_elem, prob.n_node, 2))
    _check(load_library().smm_get_nodes(prob.handle, _ptr(xy)), prob.ctx)
    return xy


def smm_get_bface_points(prob: Problem):
    xy = np.zeros((prob.dims.n_bface, prob.dims.nq, 2))
    _check(load_library().smm_get_bface_points(prob.handle, _ptr(xy)), prob.ctx)
    return xy


def smm_set_materials(prob: Problem, sigma_t, sigma_s):
    st, ss = _f64(sigma_t), _f64(sigma_s)
    _check(load_library().smm_set_materials(prob.handle, _ptr(st), _ptr(ss)), prob.ctx)
    smm_get_dims(prob)


def smm_set_source(prob: Problem, q, layout: int = SMM_SRC_ISO):
    q = _f64(q)
    _check(load_library().smm_set_source(prob.handle, _ptr(q), layout), prob.ctx)


def smm_set_inflow(prob: Problem, psibar=None, layout: int = SMM_INFLOW_VACUUM):
    pb = _f64(psibar) if psibar is not None else None
    _check(load_library().smm_set_inflow(prob.handle, _ptr(pb), layout), prob.ctx)


def smm_default_opts(**kw) -> smm_solve_opts:
    o = smm_solve_opts()
    load_library().smm_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def smm_solve(prob: Problem, opts: smm_solve_opts | None = None, varphi0=None, raise_on_noconv=True):
    """Returns (status, info dict).  SMM_ENOCONV raises unless
    raise_on_noconv is False (outputs stay valid either way)."""
    info = smm_solve_info()
    v0 = _f64(varphi0) if varphi0 is not None else None
    rc = load_library().smm_solve(prob.handle, C.byref(opts) if opts is not None else None, _ptr(v0),
                                  C.byref(info))
    if rc == SMM_ENOCONV and not raise_on_noconv:
        return rc, info.as_dict()
    _check(rc, prob.ctx)
    return rc, info.as_dict()


def smm_get_outputs(prob: Problem, varphi=None, phi=None, J=None, T=None, beta=None, on_device=False):
    _check(load_library().smm_get_outputs(prob.handle, _ptr(varphi), _ptr(phi), _ptr(J), _ptr(T), _ptr(beta),
                                          1 if on_device else 0), prob.ctx)


def smm_solve_history(prob: Problem):
    """(outer residuals, CG iterations) of each outer iteration of the last smm_solve."""
    n = C.c_int()
    _check(load_library().smm_solve_history(prob.handle, 0, None, None, C.byref(n)), prob.ctx)
    r = np.zeros(n.value)
    c = np.zeros(n.value, dtype=np.int32)
    _check(load_library().smm_solve_history(prob.handle, n.value, _ptr(r), _ptr(c), C.byref(n)), prob.ctx)
    return r, c


def smm_set_warmstart(prob: Problem, net):
    """Attach (or detach with None) the warm-start network used by SMM_START_LEARNED in smm_solve."""
    _check(load_library().smm_set_warmstart(prob.handle, None if net is None else net.handle), prob.ctx)


def smm_get_outputs_host(prob: Problem) -> dict:
    """Convenience: all outputs as fresh numpy arrays."""
    L = prob.n_elem * prob.n_node
    out = {"varphi": np.zeros(L), "phi": np.zeros(L), "J": np.zeros((2, L)), "T": np.zeros((3, L)),
           "beta": np.zeros((max(prob.dims.n_bface, 1), prob.dims.nq))}
    smm_get_outputs(prob, out["varphi"], out["phi"], out["J"], out["T"], out["beta"], on_device=False)
    return out


def smm_apply_sweep(prob: Problem, precision: int, S, s_layout: int, psi_lag, psi_out, with_inflow: bool = True):
    _check(load_library().smm_apply_sweep(prob.handle, precision, _ptr(S), s_layout, _ptr(psi_lag), _ptr(psi_out),
                                          1 if with_inflow else 0), prob.ctx)


def smm_apply_moments(prob: Problem, precision: int, psi, mom):
    _check(load_library().smm_apply_moments(prob.handle, precision, _ptr(psi), _ptr(mom)), prob.ctx)


def smm_apply_G(prob: Problem, precision: int, varphi_in, varphi_out, inner_tol: float = 1e-14,
                max_inner: int = 100000):
    _check(load_library().smm_apply_G(prob.handle, precision, _ptr(varphi_in), _ptr(varphi_out), inner_tol,
                                      max_inner), prob.ctx)


def smm_apply_G_noalloc(prob: Problem, precision: int, varphi_in, varphi_out, inner_tol: float = 1e-14,
                        max_inner: int = 100000):
    """smm_apply_G without any device allocation (work vectors in the
    library's fixed per-device array); the problem's tables must be on the
    device already (one smm_apply_G call)."""
    _check(load_library().smm_apply_G_noalloc(prob.handle, precision, _ptr(varphi_in), _ptr(varphi_out),
                                              inner_tol, max_inner), prob.ctx)


def smm_debug_ip_dense(prob: Problem):
    N = prob.n_elem * prob.n_node
    A = np.zeros((N, N))
    b = np.zeros(N)
    _check(load_library().smm_debug_ip_dense(prob.handle, _ptr(A), _ptr(b)), prob.ctx)
    return A, b


def smm_debug_cg_system(prob: Problem):
    """The continuous (CG) moment system as assembled by the library:
    (rowptr, col, val, map) of the CSR matrix A_c and the continuous unknown
    of each DG node."""
    nc, nnz = C.c_int(), C.c_int()
    lib = load_library()
    _check(lib.smm_debug_cg_system(prob.handle, C.byref(nc), C.byref(nnz), None, None, None, None), prob.ctx)
    rowptr = np.zeros(nc.value + 1, dtype=np.int32)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value)
    cmap = np.zeros(prob.n_elem * prob.n_node, dtype=np.int32)
    _check(lib.smm_debug_cg_system(prob.handle, C.byref(nc), C.byref(nnz), _ptr(rowptr), _ptr(col), _ptr(val),
                                   _ptr(cmap)), prob.ctx)
    return rowptr, col, val, cmap


def smm_debug_cg_spmv(prob: Problem, x):
    x = _f64(x)
    y = np.zeros_like(x)
    _check(load_library().smm_debug_cg_spmv(prob.handle, _ptr(x), _ptr(y)), prob.ctx)
    return y


def smm_time_cg_spmv(prob: Problem, reps: int) -> float:
    ms = C.c_double()
    _check(load_library().smm_time_cg_spmv(prob.handle, int(reps), C.byref(ms)), prob.ctx)
    return ms.value


def smm_set_sweep_tiles(prob: Problem, tile_nx: int, tile_ny: int):
    _check(load_library().smm_set_sweep_tiles(prob.handle, int(tile_nx), int(tile_ny)), prob.ctx)


def smm_set_sweep_path(prob: Problem, path: int):
    _check(load_library().smm_set_sweep_path(prob.handle, int(path)), prob.ctx)


def smm_debug_sweep_graph(prob: Problem):
    """(level [n_dir, n_elem], upstream bits [n_dir, n_elem]) of the sweep graph."""
    lev = np.zeros((prob.n_dir, prob.n_elem), dtype=np.int32)
    up = np.zeros((prob.n_dir, prob.n_elem), dtype=np.uint8)
    _check(load_library().smm_debug_sweep_graph(prob.handle, _ptr(lev), _ptr(up)), prob.ctx)
    return lev, up


def smm_time_sweep(prob: Problem, precision: int, reps: int) -> float:
    ms = C.c_double()
    _check(load_library().smm_time_sweep(prob.handle, precision, reps, C.byref(ms)), prob.ctx)
    return ms.value


def smm_debug_typed_dense(prob: Problem):
    N = prob.n_elem * prob.n_node
    A = np.zeros((N, N))
    Cm = np.zeros((N, 3 * N))
    b = np.zeros(N)
    _check(load_library().smm_debug_typed_dense(prob.handle, _ptr(A), _ptr(Cm), _ptr(b)), prob.ctx)
    return A, Cm, b


def smm_debug_corr_dense(prob: Problem):
    N = prob.n_elem * prob.n_node
    Cm = np.zeros((N, 3 * N))
    _check(load_library().smm_debug_corr_dense(prob.handle, _ptr(Cm)), prob.ctx)
    return Cm


class Batch:
    def __init__(self, ctx, handle, probs):
        self.ctx = ctx
        self.handle = handle
        self.probs = list(probs)

    @property
    def n(self):
        return len(self.probs)


def smm_batch_create(ctx: Context, probs) -> Batch:
    arr = (C.c_void_p * len(probs))(*[p.handle.value for p in probs])
    h = C.c_void_p()
    _check(load_library().smm_batch_create(ctx.handle, arr, len(probs), C.byref(h)), ctx)
    return Batch(ctx, h, probs)


def smm_batch_destroy(batch: Batch):
    load_library().smm_batch_destroy(batch.handle)


def smm_batch_solve(batch: Batch, opts: smm_solve_opts | None = None, varphi0=None, raise_on_noconv=True):
    """varphi0: None or a list of per-problem host arrays / device tensors (None entries allowed).
    Returns (status, list of info dicts)."""
    infos = (smm_solve_info * batch.n)()
    keep = []
    v0 = None
    if varphi0 is not None:
        ptrs = []
        for a in varphi0:
            if a is None:
                ptrs.append(None)
            elif isinstance(a, np.ndarray):
                a = _f64(a)
                keep.append(a)
                ptrs.append(a.ctypes.data)
            else:
                ptrs.append(a.data_ptr())
        v0 = (C.c_void_p * batch.n)(*ptrs)
    rc = load_library().smm_batch_solve(batch.handle, C.byref(opts) if opts is not None else None, v0, infos)
    if not (rc == SMM_ENOCONV and not raise_on_noconv):
        _check(rc, batch.ctx)
    return rc, [infos[k].as_dict() for k in range(batch.n)]


def smm_batch_get_outputs(batch: Batch, k: int, varphi=None, phi=None, J=None, T=None, beta=None, on_device=False):
    _check(load_library().smm_batch_get_outputs(batch.handle, k, _ptr(varphi), _ptr(phi), _ptr(J), _ptr(T),
                                                _ptr(beta), 1 if on_device else 0), batch.ctx)


def smm_batch_time_sweep(batch: Batch, precision: int, reps: int) -> float:
    ms = C.c_double()
    _check(load_library().smm_batch_time_sweep(batch.handle, precision, reps, C.byref(ms)), batch.ctx)
    return ms.value


SMM_KERNEL_SWEEP_FP32, SMM_KERNEL_SWEEP_FP64, SMM_KERNEL_CG_SPMV, SMM_KERNEL_MOMENTS_FP32 = 0, 1, 2, 3


def smm_batch_phase_times(batch: Batch):
    """(ms[4] of source+sweep, moments+closures+rhs, PCG, residual; batched PCG iterations)."""
    ms = (C.c_double * 4)()
    n = C.c_long()
    _check(load_library().smm_batch_phase_times(batch.handle, ms, C.byref(n)), batch.ctx)
    return list(ms), n.value


def smm_batch_history(batch: Batch, k: int):
    """(outer residuals, PCG iterations) of each outer iteration of problem k."""
    n = C.c_int()
    _check(load_library().smm_batch_history(batch.handle, k, 0, None, None, C.byref(n)), batch.ctx)
    r = np.zeros(n.value)
    c = np.zeros(n.value, dtype=np.int32)
    _check(load_library().smm_batch_history(batch.handle, k, n.value, _ptr(r), _ptr(c), C.byref(n)), batch.ctx)
    return r, c


def smm_batch_time_kernel(batch: Batch, kernel: int, reps: int) -> float:
    ms = C.c_double()
    _check(load_library().smm_batch_time_kernel(batch.handle, kernel, reps, C.byref(ms)), batch.ctx)
    return ms.value


def smm_batch_units(batch: Batch) -> float:
    u = C.c_double()
    _check(load_library().smm_batch_units(batch.handle, C.byref(u)), batch.ctx)
    return u.value


# ---- learned warm start (smm_cnn.h) -------------------------------------------------

SMM_START_LEARNED = 3
SMM_PRECOND_BJ, SMM_PRECOND_TWOLEVEL = 0, 1


def smm_debug_batch_precond(batch, precond: int, rs):
    """z = M^-1 r per problem (host arrays) with the given PCG preconditioner."""
    rs = [_f64(r) for r in rs]
    zs = [np.zeros_like(r) for r in rs]
    rp = (C.c_void_p * len(rs))(*[r.ctypes.data for r in rs])
    zp = (C.c_void_p * len(zs))(*[z.ctypes.data for z in zs])
    _check(load_library().smm_debug_batch_precond(batch.handle, precond, rp, zp), batch.ctx)
    return zs


def smm_debug_batch_spmv(batch, xs):
    """y = A x per problem (host arrays) with the batch's current PCG kernels."""
    xs = [_f64(x) for x in xs]
    ys = [np.zeros_like(x) for x in xs]
    xp = (C.c_void_p * len(xs))(*[x.ctypes.data for x in xs])
    yp = (C.c_void_p * len(ys))(*[y.ctypes.data for y in ys])
    _check(load_library().smm_debug_batch_spmv(batch.handle, xp, yp), batch.ctx)
    return ys


def smm_batch_apply_sweep(batch, precision: int, sources, k: int):
    """One batched sweep of every problem on the isotropic sources `sources`
    (a list of host arrays [n_elem*n_node], None entries = zero); returns
    problem k's angular flux as a host array [n_dir, n_elem, n_node]."""
    srcs = [None if a is None else _f64(a) for a in sources]
    assert len(srcs) == batch.n
    for a, p in zip(srcs, batch.probs):
        assert a is None or a.size == p.n_elem * p.n_node
    arr = (C.c_void_p * batch.n)(*[None if a is None else a.ctypes.data for a in srcs])
    pk = batch.probs[k]
    psi = np.zeros((pk.n_dir, pk.n_elem, pk.n_node))
    _check(load_library().smm_batch_apply_sweep(batch.handle, precision, arr, int(k), _ptr(psi)), batch.ctx)
    return psi


def smm_debug_batch_sweep_shape(batch, shape: int):
    """Force the batched sweep's kernel shape: 0 column-wave, 1 element-lane, -1 autotuned."""
    _check(load_library().smm_debug_batch_sweep_shape(batch.handle, shape), batch.ctx)


def smm_debug_batch_cg_fork(batch, fork: int):
    _check(load_library().smm_debug_batch_cg_fork(batch.handle, int(fork)), batch.ctx)


def smm_debug_batch_grouped(batch, grouped: int):
    """Force the type-group (1) or per-node (0) PCG kernels, or the automatic choice (-1)."""
    _check(load_library().smm_debug_batch_grouped(batch.handle, grouped), batch.ctx)


def smm_debug_mg_level(prob, level: int):
    """9-point stencil [9][nvy*nvx] of a multigrid level of the two-level preconditioner."""
    nx, ny = C.c_int(), C.c_int()
    lib = load_library()
    _check(lib.smm_debug_mg_level(prob.handle, level, None, C.byref(nx), C.byref(ny)), prob.ctx)
    A = np.zeros((9, nx.value * ny.value))
    _check(lib.smm_debug_mg_level(prob.handle, level, _ptr(A), C.byref(nx), C.byref(ny)), prob.ctx)
    return A, nx.value, ny.value


def smm_time_sweep_parts(prob, precision: int, reps: int):
    """(setup, particular, levels) ms of a sweep with stored element operators."""
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(load_library().smm_time_sweep_parts(prob.handle, int(precision), int(reps), C.byref(a), C.byref(b),
                                               C.byref(c)), prob.ctx)
    return a.value, b.value, c.value

def smm_debug_cg_mg_level(prob, level: int):
    """9-point stencil [9][nvy*nvx] of a multigrid level of the CG system's
    two-level preconditioner."""
    nx, ny = C.c_int(), C.c_int()
    lib = load_library()
    _check(lib.smm_debug_cg_mg_level(prob.handle, level, None, C.byref(nx), C.byref(ny)), prob.ctx)
    A = np.zeros((9, nx.value * ny.value))
    _check(lib.smm_debug_cg_mg_level(prob.handle, level, _ptr(A), C.byref(nx), C.byref(ny)), prob.ctx)
    return A, nx.value, ny.value

class Cnn:
    def __init__(self, ctx, handle, channels, height, width, max_batch):
        self.ctx = ctx
        self.handle = handle
        self.channels = list(channels)
        self.height, self.width, self.max_batch = height, width, max_batch

    @property
    def n_params(self) -> int:
        n = C.c_size_t()
        _check(load_library().smm_cnn_num_params(self.handle, C.byref(n)), self.ctx)
        return n.value


def smm_cnn_create(ctx: Context, channels, height: int, width: int, max_batch: int) -> Cnn:
    ch = (C.c_int * len(channels))(*channels)
    h = C.c_void_p()
    _check(load_library().smm_cnn_create(ctx.handle, len(channels) - 1, ch, height, width, max_batch, C.byref(h)), ctx)
    return Cnn(ctx, h, channels, height, width, max_batch)


def smm_cnn_destroy(net: Cnn):
    load_library().smm_cnn_destroy(net.handle)


def smm_cnn_num_params(net: Cnn) -> int:
    return net.n_params


def smm_cnn_set_params(net: Cnn, params):
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
    _check(load_library().smm_cnn_set_params(net.handle, _ptr(a), a.size), net.ctx)


def smm_cnn_get_params(net: Cnn) -> np.ndarray:
    a = np.zeros(net.n_params, dtype=np.float32)
    _check(load_library().smm_cnn_get_params(net.handle, _ptr(a), a.size), net.ctx)
    return a


def smm_cnn_forward(net: Cnn, x, batch: int, y):
    """x, y: device float32 tensors [batch][H][W][c_in] / [batch][H][W][c_out]."""
    _check(load_library().smm_cnn_forward(net.handle, _ptr(x), batch, _ptr(y)), net.ctx)


def smm_cnn_loss_grad(net: Cnn, x_all, t_all, idx, batch: int, chan_weight=None, want_grad=False):
    """Returns (loss, grad or None).  idx: device int32 tensor or None."""
    loss = C.c_double()
    w = None if chan_weight is None else np.ascontiguousarray(np.asarray(chan_weight, dtype=np.float32))
    g = np.zeros(net.n_params, dtype=np.float32) if want_grad else None
    _check(load_library().smm_cnn_loss_grad(net.handle, _ptr(x_all), _ptr(t_all), int(x_all.shape[0]), _ptr(idx),
                                            batch, _ptr(w), C.byref(loss), _ptr(g)), net.ctx)
    return loss.value, g


def smm_cnn_adam_step(net: Cnn, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    _check(load_library().smm_cnn_adam_step(net.handle, lr, beta1, beta2, eps), net.ctx)


def smm_batch_warmstart_dims(batch: Batch):
    v = [C.c_int() for _ in range(4)]
    _check(load_library().smm_batch_warmstart_dims(batch.handle, *[C.byref(x) for x in v]), batch.ctx)
    return tuple(x.value for x in v)   # (n_features, n_targets, height, width)


def smm_batch_diffusion(batch: Batch, inner_tol: float = 1e-10, max_inner: int = 20000):
    _check(load_library().smm_batch_diffusion(batch.handle, inner_tol, max_inner), batch.ctx)


def smm_batch_warmstart_features(batch: Batch, first: int, count: int, out):
    _check(load_library().smm_batch_warmstart_features(batch.handle, first, count, _ptr(out)), batch.ctx)


def smm_batch_warmstart_targets(batch: Batch, first: int, count: int, out):
    _check(load_library().smm_batch_warmstart_targets(batch.handle, first, count, _ptr(out)), batch.ctx)


def smm_batch_set_warmstart(batch: Batch, net: Cnn | None):
    _check(load_library().smm_batch_set_warmstart(batch.handle, net.handle if net is not None else None), batch.ctx)
    batch._ws_net = net   # keep the network alive while attached


def smm_batch_warmstart_used(batch: Batch) -> np.ndarray:
    u = np.zeros(batch.n, dtype=np.int32)
    _check(load_library().smm_batch_warmstart_used(batch.handle, _ptr(u)), batch.ctx)
    return u
