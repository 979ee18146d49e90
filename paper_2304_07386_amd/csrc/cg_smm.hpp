// Device side of the continuous (CG) SMM moment solve: FP64 Jacobi-PCG on
// the CSR matrix of V_p, and the maps between the DG and continuous nodes.
#pragma once

#include <hip/hip_runtime.h>

namespace smm {

struct CgsArgs {
    int nc;            // continuous nodes (rows)
    long L;            // DG nodes, ne * n
    const int* rowptr; // [nc + 1]
    const int* col;    // [nnz]
    const double* val; // [nnz]
    const double* dinv;// [nc] 1 / diagonal
    const int* tab;    // [nc][4] DG nodes at each continuous node, -1 padded
    const int* map;    // [L] continuous node of each DG node
    double *b, *x, *r, *z, *p, *q;  // [nc]
    double* part;      // [sblocks + 3 vblocks] block partial sums
    double* scal;      // [16] solver scalars (below)
    int vblocks;       // blocks of the node-wise kernels (256 nodes each)
    int sblocks;       // blocks of the product kernels (32 rows each)
    // two-level preconditioner z = D^-1 r + P_1 V(P_1^T r) (mg != 0): P_1 the
    // bilinear interpolation from the (nx + 1) x (ny + 1) element vertices to
    // the continuous nodes, V one vertex multigrid V-cycle
    int mg;
    int nx, ny, order; // element grid and polynomial order
    double gll[8];     // Gauss-Lobatto points on [0, 1] (order + 1 of them)
    double* rv;        // [(nx + 1)(ny + 1)] P_1^T r (the V-cycle's right-hand side)
    const double* xv;  // the V-cycle's result (a vector of the hierarchy)
};

// vertex multigrid of the two-level preconditioner, levels in global memory
constexpr int CGS_MG_MAXLEV = 12;
struct CgsMG {
    int nlev;                      // levels 0 .. nlev - 1, the last solved by cinv
    int nvx[CGS_MG_MAXLEV], nvy[CGS_MG_MAXLEV];
    const double* A[CGS_MG_MAXLEV];  // [9][nv] stencils, entry k = (dy + 1) 3 + dx + 1
    double* x[CGS_MG_MAXLEV];
    double* t[CGS_MG_MAXLEV];
    double* b[CGS_MG_MAXLEV];        // b[0] is CgsArgs::rv
    const double* cinv;              // dense inverse of the coarsest level
    double omega;                    // Jacobi damping
};

// scal: 0 r.z, 1 bb, 2 r.r, 3 tol^2 bb, 4 converged or stopped (1), 5 iterations
// done, 6 breakdown (p.Ap <= 0), 8 (P_1^T r).x_v of the last V-cycle
constexpr int CGS_SPMV_ROWS = 32;  // rows per 256-thread block, 8 lanes per row

hipError_t cgs_gather(const CgsArgs& a, const double* b_dg, hipStream_t s);   // b = P_c^T b_dg
hipError_t cgs_pick(const CgsArgs& a, const double* x_dg, hipStream_t s);     // x = x_dg at the first DG copy
hipError_t cgs_scatter(const CgsArgs& a, double* x_dg, hipStream_t s);        // x_dg = P_c x
hipError_t cgs_start(const CgsArgs& a, const CgsMG& m, double tol, hipStream_t s);
hipError_t cgs_iterations(const CgsArgs& a, const CgsMG& m, int iters, hipStream_t s);
// y = A_c x over the whole system (the product kernel of the iterations)
hipError_t cgs_spmv(const CgsArgs& a, const double* x, double* y, hipStream_t s);

}  // namespace smm
