// Launch wrappers of the libsmm device kernels.
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace smm {

// Cartesian wavefront sweep (one workgroup per direction).
struct CartSweepArgs {
    int nx, ny, nd, nb, nmat;
    int s_aniso;                 // S is [nd][ne][n] if 1, else [ne][n]
    const void* S;
    const void* Pm;              // [nmat][nd][n][n]
    const void* Px;              // [nmat][nd][n][nb]
    const void* Py;              // [nmat][nd][n][nb]
    const uint8_t* mat;          // [ne]
    const double* omega;         // [nd][3] (signs select the quadrant)
    const void* bx;              // [nd][ny][nb] boundary traces (or null)
    const void* by;              // [nd][nx][nb]
    void* psi;                   // [nd][ne][n]
    int variant;                 // 0 automatic, 1 element-row kernel only
};
hipError_t launch_sweep_cart(bool fp64, const CartSweepArgs& a, hipStream_t s);

// General (curved) sweep: per element and direction, assemble the local
// upwind matrix in LDS and eliminate it.
struct GenSweepArgs {
    int ne, nd, nb, nq, nbf, nlev;
    int s_aniso;
    const void* S;
    const void* Mk;              // [ne][n][n]
    const void* Gx;
    const void* Gy;
    const void* nds;             // [ne][4][nq][2] weighted n ds
    const void* Lf;              // [nb][nq]
    const void* sigma_t;         // [ne]
    const int* nbr;              // [ne][4]
    const int* bface_of;         // [ne][4]
    const uint8_t* upflag;       // [nd][ne]
    const int* lev_ptr;          // [nd][nlev+1]
    const int* lev_elem;         // [nd][ne]
    const double* omega;         // [nd][3]
    const void* psibar;          // [nd][nbf][nq] or null
    const void* psi_lag;         // [nd][ne][n] or null
    void* psi;                   // [nd][ne][n]
};
hipError_t launch_sweep_general(bool fp64, const GenSweepArgs& a, hipStream_t s);

// mom[16 rows used 8][L] = W[16][nd] psi[nd][L] on the matrix cores
hipError_t launch_moments(bool fp64, const void* psi, int nd, long L, const void* W, int ldw,
                          double* mom, hipStream_t s);

// source S = sigma_s/(4 pi) (x - x_prev) + (add_q ? q : 0) converted to the sweep type
hipError_t launch_source(bool fp64, int ne, int n, int nd_q, const double* sigma_s,
                         const double* x, const double* x_prev, const double* q, void* S,
                         hipStream_t s);

hipError_t launch_axpy_mom(long L, const double* a, double* acc, hipStream_t s);  // acc += a

// T and beta from the 8 moment rows
hipError_t launch_closures(int ne, int n, int nb, int nq, int nbf, const double* mom,
                           const int* bface_K, const int* bface_f, const double* Lf,
                           double eb0x, double eb0y, double* T, double* beta, hipStream_t s);

// b = b_fixed + C T - B beta
hipError_t launch_rhs(int ne, int n, int nq, const double* bfix, const int* bsr_col,
                      const double* corr, const double* T, const int* bface_of,
                      const double* beta_op, const double* beta, double* b, hipStream_t s);

// FP64 block-Jacobi PCG
struct CgState {
    int ne, n;
    const int* col;              // [ne][5]
    const double* A;             // [ne][5][n][n]
    const double* Dinv;          // [ne][n][n]
    const double* b;
    double* x;
    double* r;
    double* z;
    double* p;
    double* q;
    double* part;                // [3][nblocks] partial sums
    double* scal;                // device scalars (see kernels.hip)
    int nblocks;
};
hipError_t cg_start(const CgState& c, double tol, hipStream_t s);
hipError_t cg_iterations(const CgState& c, int iters, double tol, hipStream_t s);

// residual: out[0] = max|x_new - x_old|, out[1] = max|x_new|
hipError_t launch_residual(long L, const double* xn, const double* xo, double* part, int nblocks,
                           double* out, hipStream_t s);

}  // namespace smm
