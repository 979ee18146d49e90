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
};

// scal: 0 r.z, 1 bb, 2 r.r, 3 tol^2 bb, 4 converged or stopped (1), 5 iterations
// done, 6 breakdown (p.Ap <= 0)
constexpr int CGS_SPMV_ROWS = 32;  // rows per 256-thread block, 8 lanes per row

hipError_t cgs_gather(const CgsArgs& a, const double* b_dg, hipStream_t s);   // b = P_c^T b_dg
hipError_t cgs_pick(const CgsArgs& a, const double* x_dg, hipStream_t s);     // x = x_dg at the first DG copy
hipError_t cgs_scatter(const CgsArgs& a, double* x_dg, hipStream_t s);        // x_dg = P_c x
hipError_t cgs_start(const CgsArgs& a, double tol, hipStream_t s);
hipError_t cgs_iterations(const CgsArgs& a, int iters, hipStream_t s);
// y = A_c x over the whole system (the product kernel of the iterations)
hipError_t cgs_spmv(const CgsArgs& a, const double* x, double* y, hipStream_t s);

}  // namespace smm
