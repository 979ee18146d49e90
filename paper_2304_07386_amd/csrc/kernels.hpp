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
    void* psi;                   // [nd][psi_ld]
    int variant;                 // 0 automatic, 1 element-row kernel only
    long psi_ld;                 // row stride of psi (>= ne * n); 0 means ne * n
    const void* tab;             // batched sweep: [nmat][nd][nb][nb][lane_rw(nb)] rows
                                 // [Pm | Px | Py] of node column ca (third index), row ca + nb b
};
// padded length of one operator row [Pm | Px | Py] in the batched sweep table
constexpr int lane_rw(int nb) { return (nb * nb + 2 * nb + 7) & ~7; }
hipError_t launch_sweep_cart(bool fp64, const CartSweepArgs& a, hipStream_t s);

// General (curved) sweep: per element and direction, assemble the local
// upwind matrix in LDS and eliminate it.
struct GenSweepArgs {
    int ne, nd, nb, nq, nbf, nlev;
    int ntiles;                  // independent element tiles (1: the full sweep)
    int maxw;                    // most elements in one level of one (direction, tile)
    int wave_solve;              // 0 automatic (one lane per element at p <= 2, one lane per row at
                                 //   p >= 3); 1 one wave per element; 2 one lane per row at p >= 2
    int s_aniso;
    const void* S;
    const void* Mk;              // [ne][n][n]
    const void* Gx;
    const void* Gy;
    const void* nds;             // [ne][4][nq][2] weighted n ds
    const void* Lf;              // [nb][nq]
    const void* sigma_t;         // [ne]
    const int* nbr;              // [ne][4]
    const uint8_t* nbr_face;     // [ne][4] neighbour's face | 4 (its face points run the other way);
                                 //   null: the opposite face, same way (structured grids)
    const int* bface_of;         // [ne][4]
    const uint8_t* upflag;       // [nd][ne]
    const int* lev_ptr;          // [nd][ntiles][nlev+1] offsets into the direction's list
    const int* lev_elem;         // [nd][ne], tile-major, then level
    const double* omega;         // [nd][3]
    const void* psibar;          // [nd][nbf][nq] or null
    const void* psi_lag;         // [nd][ne][n] or null
    void* psi;                   // [nd][ne][n]
    // stored element operators (sweep type; null: assemble and eliminate
    // per sweep): A^-1 M [nd][ne][n][n] by column, A^-1 r [nd][ne][n] (r the
    // boundary inflow terms), face operators [nd][ne][4][nb][n] and the
    // inflow-face mask [nd][ne]
    const void* invA;
    const void* invC;
    const void* invG;
    const uint8_t* inmask;
};
hipError_t launch_sweep_general(bool fp64, const GenSweepArgs& a, hipStream_t s);
// Build the stored element operators of the general sweep (FP64 tables and
// inflow in a, output in FP64 or FP32); invA, invC, invG, inmask sized as in
// GenSweepArgs.
hipError_t launch_gen_inv_setup(bool out_fp64, const GenSweepArgs& a, void* invA, void* invC, void* invG,
                                uint8_t* inmask, hipStream_t s);
// One part of a sweep with the stored operators (a.invA set): 1 the
// particular pass, 2 the levels, 3 both.
hipError_t launch_gen_inv_part(bool fp64, const GenSweepArgs& a, int part, hipStream_t s);

// mom[16 rows used 8][L] = W[16][nd] psi[nd][L] on the matrix cores
hipError_t launch_moments(bool fp64, const void* psi, int nd, long L, const void* W, int ldw,
                          double* mom, hipStream_t s);

// source S = sigma_s/(4 pi) (x - x_prev) + (add_q ? q : 0) converted to the sweep type
hipError_t launch_source(bool fp64, int ne, int n, int nd_q, const double* sigma_s,
                         const double* x, const double* x_prev, const double* q, void* S,
                         hipStream_t s);

hipError_t launch_axpy_mom(long L, const double* a, double* acc, hipStream_t s);  // acc += a

// T and beta from the 8 moment rows
hipError_t launch_beta_general(bool fp64, int nd, int ne, int n, int nb, int nq, int nbf, const void* psi,
                               const double* omega, const double* w, const int* bface_K, const int* bface_f,
                               const double* nhat_b, const double* eb0_pt, const double* Lf, bool accumulate,
                               double* beta, hipStream_t s);
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

// ---------------------------------------------------------------------------
// Batched (typed Cartesian) path.  One descriptor per problem; all pointers
// are device pointers.  Element-block kernels use blocks of
// epb = 256 / n whole elements, mapped to problems by blk2p.
// ---------------------------------------------------------------------------
struct BProb {
    int ne, n, nb, nq, nbf, nd, nx, ldw;
    long L;                        // ne * n
    long Lpad;                     // psi row stride (L rounded up to a multiple of 32)
    double eb0x, eb0y;
    int blk0, nblk;                // element-block range
    long bq0;                      // first flat boundary-point index
    long mw0;                      // first moments wavefront
    double *varphi, *varphi_prev, *x, *b, *r, *z, *p, *q;   // [L]
    const double *bfix, *qsrc, *sigma_s;                    // [L], [L], [ne]
    double *mom, *mom_acc, *T, *beta;                       // [8L], [8L], [3L], [nbf*nq]
    const int *sid, *nid, *bface_of, *bK, *bF;              // [ne], [4ne], [4ne], [nbf], [nbf]
    const double *ip_self, *ip_nbr, *dinv, *c_self, *c_nbr, *bop, *Lf;
    double* scal;                                           // [16] CG scalars
    void* S;                                                // [L] (sweep precision)
    void* psi;                                              // [nd][Lpad]
    const double* W64;                                      // [16][ldw] moment weights
    const float* W32;                                       // [16][ldw]
    double* vdiff;                                          // [L] diffusion start (warm start)
    const float* feat0;                                     // [ne][4] per-element warm-start features
    double hxhy;                                            // element area
    int g0, ng;                                             // type-group range (PCG kernels)
    const double* gll;                                      // [nb] Gauss-Lobatto points on [0,1]
    long e_off;                                             // first element in batch-wide element arrays
    double *aG, *aF;                                        // [3][L] Anderson history: G(X) and G(X) - X
    // two-level preconditioner, continuous-space term (orders >= 2; null
    // otherwise): w = D_c^-1 P_c^T r on the continuous Q_p nodes of the mesh,
    // a (nx p + 1) x (ny p + 1) grid, D_c the diagonal of P_c^T A P_c
    double* cgw;                                            // [ncg]
    const double* cgdc;                                     // [ncg]
};

struct BatchLaunch {
    const BProb* P;                // device array [nprob]
    int nprob;
    const int* blk2p;              // [nblocks]
    int nblocks;
    const int* active;             // [nprob] outer iteration still running
    double* part;                  // [3][nblocks]
    long nbq;                      // total boundary points
    long nmw;                      // total moments wavefronts
    const long* bq0;               // [nprob] prefix (device copy)
    const long* mw0;               // [nprob] prefix (device copy)
    const double* ptol;            // [nprob] per-problem PCG tolerance (nullable: the scalar one)
    // type groups: up to 64 elements of one problem that share the typed blocks
    // of their self and four face couplings (one wave per group)
    int ngroups;
    const int* g_prob;             // [ngroups]
    const int* g_count;            // [ngroups]
    const int* g_ty;               // [ngroups][5] self type, neighbour types (-1: boundary face)
    const int* g_elem;             // [ngroups][64]
    double* gpart;                 // [3][ngroups] per-group partial sums
    int g_nb0[7];                  // groups of order nb - 1 are [g_nb0[nb], g_nb0[nb + 1]) (nb = 2..5)
    int order_mask;                // bit nb: the PCG iterations launch the grouped kernels of that order
    int grouped;                   // 1: PCG on the type groups, 0: per-node element blocks
    int mg;                        // 1: two-level preconditioner (r.z from b_mg_apply)
    double* mg_corner;             // two-level: [4][batch elements] corner sums of r, written by the r update
};

// Two-level preconditioner: continuous Q1 coarse space on the element vertices
// and a vertex multigrid V-cycle for it (one launch per level and step covers
// every problem that has that level).
constexpr int MG_MAXLEV = 12;
struct MGLevelDev {
    const int* off;   // [nprob+1] vertex offsets of this level (0 vertices: problem absent)
    const int* dims;  // [nprob][2] vertex grid
    const double* A;  // [9][nv] stencil, entry k = (dy+1)*3 + (dx+1)
    double *x, *t, *b;
    int nv;
};
struct MGLaunch {
    int nlev;                   // levels of the deepest problem
    MGLevelDev lev[MG_MAXLEV];
    const int* lc;              // [nprob] coarsest level of each problem
    const int* coff;            // [nprob] offset of its dense coarsest inverse
    const double* cinv;
    double omega;               // Jacobi damping
    int nu;                     // damped Jacobi steps before and after the coarse correction (>= 1)
    double* corner;             // [4][batch elements] corner sums of the residual
    int ls;                     // levels >= ls run in one workgroup per problem (nlev: none)
    size_t lds;                 // LDS bytes of that workgroup
    int coarse_any;             // 1: some problem's coarsest level index is below ls (its dense solve has a launch of its own)
    // continuous-space term: blocks of 256 nodes of the Q_p grids, per problem
    const int* cg_blk2p;        // [cg_nblocks] problem of each block
    const int* cg_blk0;         // [nprob + 1] first block of each problem
    double* cg_part;            // [cg_nblocks] per-block partial sums of (P_c^T r).w
    int cg_nblocks;
};
// allows the LDS size of the workgroup V-cycle kernel
hipError_t mg_prepare(size_t lds);
// Coarse correction x0 = V(P0^T r) on the vertex grid (level 0).  With init,
// the corner sums of r are formed first and the correction is added to the
// block-Jacobi z = D^-1 r: z += P0 x0, p = z, partial sums of r.z in part[0].
// Without init (inside the PCG loop) the corner sums come from the r update
// and z is left as D^-1 r: the iteration adds P0 x0 where it uses z.
hipError_t b_mg_apply(const BatchLaunch& B, const MGLaunch& M, bool init, hipStream_t s);
// w = D_c^-1 P_c^T r for every problem with the continuous-space term
hipError_t b_cgl_apply(const BatchLaunch& B, const MGLaunch& M, hipStream_t s);

hipError_t b_source(bool fp64, const BatchLaunch& B, bool delta, hipStream_t s);
// Persistent batched sweep over (problem, direction) tasks.  `threads` is
// b_sweep_threads of the largest problem of the task list, `lds` the largest
// b_sweep_lds; `multi` selects the variant for problems with several materials.
// element-lane shape of the batched sweep: threads = 64 per 64-slot chunk of the
// longest anti-diagonal (at most 4 chunks), no dynamic LDS
hipError_t b_sweep_elem(bool fp64, int nb, bool multi, int threads, int grid, const CartSweepArgs* args,
                        const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s);
hipError_t b_sweep(bool fp64, int nb, bool multi, int threads, size_t lds, int grid, const CartSweepArgs* args,
                   const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s);
// matrix-core shape of the batched sweep (FP32): tiles of 16 elements of an
// anti-diagonal, tpw (2 or 4) tiles per wave; threads = b_sweep_mfma_threads of
// the largest problem (at most 256), lds = b_sweep_mfma_lds with the largest
// nx + ny of the task list
hipError_t b_sweep_mfma(int nb, bool multi, int tpw, int threads, size_t lds, int grid, const CartSweepArgs* args,
                        const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s);
int b_sweep_mfma_threads(int tpw, int nx, int ny);
size_t b_sweep_mfma_lds(int nb, int tpw, int threads, int nxy);
int b_sweep_threads(int nb, int nx, int ny);
size_t b_sweep_lds(bool fp64, int nb, bool multi, int nx, int ny);
// with_T (FP32, accumulating): the launch also forms the closure T from the
// accumulated moments, which b_closures_rhs then skips (t_done)
hipError_t b_moments(bool fp64, const BatchLaunch& B, bool accumulate, bool first, hipStream_t s,
                     bool with_T = false);
// start vectors of every problem: bit 1 varphi_prev = 0, 2 varphi = 0,
// 4 b = bfix and x = 0, 8 varphi = x
hipError_t b_start_vectors(const BatchLaunch& B, int what, hipStream_t s);
hipError_t b_closures_rhs(const BatchLaunch& B, hipStream_t s, bool t_done = false);
hipError_t b_copy_x(const BatchLaunch& B, hipStream_t s);               // x = varphi
hipError_t b_shift(const BatchLaunch& B, hipStream_t s);                // varphi_prev = varphi, varphi = x
hipError_t b_cg_start(const BatchLaunch& B, double tol, hipStream_t s, const MGLaunch* M);
// Side streams for the per-order launches of a PCG iteration: with more than
// one order active, each grouped phase forks from the caller's stream, runs
// the orders concurrently and joins again (graph capture turns this into
// parallel branches).
struct CgFork {
    hipStream_t side[3];
    hipEvent_t fork;
    hipEvent_t join[3];
};
hipError_t b_cg_iterations(const BatchLaunch& B, int iters, hipStream_t s, const MGLaunch* M,
                           const CgFork* F = nullptr);
hipError_t b_cg_spmv(const BatchLaunch& B, hipStream_t s);                // one q = A p launch
hipError_t b_precond(const BatchLaunch& B, const MGLaunch* M, hipStream_t s); // z = M^-1 r (and p = z)
hipError_t b_residual(const BatchLaunch& B, double* out, hipStream_t s);   // out[2*nprob]
// Anderson mixing of the outer fixed point: store G(X) = x and f = x - varphi in
// history slot `slot`; the Gram matrix of the three f slots (out[6*nprob]:
// f0.f0, f0.f1, f0.f2, f1.f1, f1.f2, f2.f2); and varphi_prev = varphi,
// varphi = sum_i coef[3*prob + i] G_i
hipError_t b_aa_store(const BatchLaunch& B, int slot, hipStream_t s);
hipError_t b_aa_gram(const BatchLaunch& B, double* part6, double* out, hipStream_t s);
hipError_t b_aa_mix(const BatchLaunch& B, const double* coef, hipStream_t s);
// warm start: features / targets of problems [first, first + count), the start from
// the network output (varphi = varphi_D + s_K y), and varphi_D = x
hipError_t b_ws_features(const BatchLaunch& B, int first, int count, float* X, int nf, hipStream_t s);
hipError_t b_ws_targets(const BatchLaunch& B, int first, int count, float* T, int nt, hipStream_t s);
hipError_t b_ws_apply(const BatchLaunch& B, const float* Y, int nt, hipStream_t s);
hipError_t b_ws_store_diffusion(const BatchLaunch& B, hipStream_t s);
hipError_t zero_ints(int* p, int n, hipStream_t s);

}  // namespace smm
