"""PCG preconditioners on the GPU, applied once, against a CPU emulation.

z = M^-1 r for a batch of problems of different sizes and orders:
* block-Jacobi: z = D^-1 r with D the element diagonal blocks of the typed IP
  matrix;
* two-level: z = D^-1 r + P_c D_c^-1 P_c^T r + P0 V(P0^T r).  P_c injects
  the continuous Q_p functions (nodal values at the Gauss-Lobatto points,
  shared across element faces) into the DG space, D_c is the diagonal of
  P_c^T A P_c (built here from the dense A; orders >= 2 only); V is one
  V-cycle (one damped Jacobi sweep before and one after the coarse
  correction, weight 2/3, the first from zero; restriction the transpose of
  linear interpolation; dense solve on the coarsest grid) on the level
  stencils of the host set-up (pinned in test_mg_host.py).
Bar: relative L2 1e-12 (FP64, only the summation order differs).
"""
import numpy as np
import pytest

from workloads import config_blobs, config_channel, config_plain

from .gpu_common import announce, rel_l2
from .test_gpu_batch import _batch_members
from .test_mg_host import _p0, _p1d, _stencil_dense

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2304_07386_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return L.smm_ctx_create(0, torch.cuda.current_stream())


def _emulate(hctx, wl, r, two_level):
    p = L.problem_from_workload(hctx, wl)
    A, _, _ = L.smm_debug_typed_dense(p)
    n = (wl.p + 1) ** 2
    z = np.zeros_like(r)
    for K in range(wl.nx * wl.ny):
        s = slice(K * n, (K + 1) * n)
        z[s] = np.linalg.solve(A[s, s], r[s])
    if not two_level:
        return z
    levels = []
    lv = 0
    while True:
        try:
            A9, nx, ny = L.smm_debug_mg_level(p, lv)
        except L.SmmError:
            break
        levels.append((_stencil_dense(A9, nx, ny), nx, ny))
        lv += 1
    om = 2.0 / 3.0
    nu = 1  # smoothing steps before and after the coarse correction

    def vcycle(k, b):
        Al, nx, ny = levels[k]
        if k == len(levels) - 1:
            return np.linalg.solve(Al, b)
        d = np.diag(Al)
        x = om * b / d
        for _ in range(nu - 1):
            x = x + om * (b - Al @ x) / d
        P = np.kron(_p1d(ny), _p1d(nx))
        x = x + P @ vcycle(k + 1, P.T @ (b - Al @ x))
        for _ in range(nu):
            x = x + om * (b - Al @ x) / d
        return x

    P0 = _p0(wl.nx, wl.ny, wl.p)
    z = z + P0 @ vcycle(0, P0.T @ r)
    if wl.p >= 2:
        Pc = _pc(wl.nx, wl.ny, wl.p)
        dc = np.diag(Pc.T @ A @ Pc)
        z = z + Pc @ ((Pc.T @ r) / dc)
    return z


def _pc(nx, ny, p):
    """Injection of the continuous Q_p space (nodes of a (nx p + 1) x (ny p + 1)
    grid) into the DG space, element-major with nodes x fastest."""
    nb, gx = p + 1, nx * p + 1
    n = nb * nb
    P = np.zeros((nx * ny * n, gx * (ny * p + 1)))
    for K in range(nx * ny):
        ex, ey = K % nx, K // nx
        for b in range(nb):
            for a in range(nb):
                P[K * n + a + nb * b, (ey * p + b) * gx + ex * p + a] = 1.0
    return P


@pytest.mark.parametrize("precond", [0, 1], ids=["block_jacobi", "two_level"])
def test_preconditioner_matches_emulation(ctx, precond):
    announce(f"PCG preconditioner {precond} applied once vs CPU emulation")
    wls = _batch_members() + [config_blobs(20004, n=12), config_channel(n=9, side=1.3)]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    batch = L.smm_batch_create(ctx, probs)
    rng = np.random.default_rng(7)
    rs = [rng.normal(size=p.n_elem * p.n_node) for p in probs]
    zs = L.smm_debug_batch_precond(batch, precond, rs)
    hctx = L.smm_ctx_create(-1)
    for k, (wl, r, z) in enumerate(zip(wls, rs, zs)):
        ref = _emulate(hctx, wl, r, precond == 1)
        assert rel_l2(z, ref) < 1e-12, (k, rel_l2(z, ref))
    L.smm_batch_destroy(batch)


def test_preconditioner_single_level_member(ctx):
    """A 2 x 2 mesh has a single vertex level (its 3 x 3 grid is the coarsest),
    solved by the coarse-level launch, which runs only when some member of
    the batch needs it; the other members take the workgroup V-cycle."""
    announce("two-level preconditioner, batch with a single-level member vs CPU emulation")
    wls = _batch_members()[:2] + [config_plain(2, 2, 4)]
    probs = [L.problem_from_workload(ctx, wl) for wl in wls]
    hctx = L.smm_ctx_create(-1)
    levels = []
    for wl in wls:
        p = L.problem_from_workload(hctx, wl)
        n = 0
        while True:
            try:
                L.smm_debug_mg_level(p, n)
            except L.SmmError:
                break
            n += 1
        levels.append(n)
    assert levels[-1] == 1 and min(levels[:-1]) > 1, levels
    batch = L.smm_batch_create(ctx, probs)
    rng = np.random.default_rng(11)
    rs = [rng.normal(size=p.n_elem * p.n_node) for p in probs]
    zs = L.smm_debug_batch_precond(batch, 1, rs)
    for k, (wl, r, z) in enumerate(zip(wls, rs, zs)):
        ref = _emulate(hctx, wl, r, True)
        assert rel_l2(z, ref) < 1e-12, (k, rel_l2(z, ref))
    L.smm_batch_destroy(batch)
