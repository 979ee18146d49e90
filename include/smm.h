/*
 * smm.h -- C ABI of libsmm: the high-order DG S_N transport sweep inside the
 * Second Moment Method (Olivier & Haut, "High-Order Finite Element Second
 * Moment Methods for Linear Transport"), on AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. 2, eq. transport / eq. inflow): mono-energetic fixed-source
 * transport with isotropic scattering,
 *     Omega.grad psi + sigma_t psi = sigma_s/(4 pi) int psi dOmega + q,
 *     psi = psibar on inflow boundary points,
 * on a 2D domain meshed by nx * ny quadrilaterals mapped by Q_m polynomials
 * (Sec. 3.1).  The angular flux is discretised by upwind DG in Y_p and S_N
 * collocation (Sec. 4); the SMM moment system is the interior-penalty
 * discretisation eq. ipsmm (Sec. 5.1), solved by FP64 preconditioned CG; the
 * two are coupled by the fixed point X = G(X) (eq. moment:smm_fp).
 *
 * Conventions
 *  - Every call returns int: SMM_OK (0) or a negative SMM_E* code.  No C++
 *    exception crosses the ABI.  smm_strerror() names a code; smm_last_error()
 *    gives the message of the last failure on a context.
 *  - DOF layout: element-major, element index K = j*nx + i (i along x);
 *    inside an element the (p+1)^2 Gauss-Lobatto nodal values are
 *    lexicographic with the x index fastest.
 *  - Directions: level-symmetric S_N, 2D half-sphere set of N(N+2)/2
 *    directions (weights sum to 4 pi), ordered by quadrant (+,+), (-,+),
 *    (-,-), (+,-) and inside a quadrant by octant point order;
 *    smm_get_quadrature() returns them.
 *  - Boundary faces are enumerated by element K, then local face
 *    (0 bottom, 1 right, 2 top, 3 left); each carries nq = p+m+1 Gauss points
 *    ordered by increasing x (faces 0, 2) or increasing y (faces 1, 3) -- on
 *    a mesh given element by element, by the element's own reference
 *    coordinate along the face.
 *  - Ownership: the caller owns every array passed in or out.  Inputs given to
 *    smm_set_* are copied before the call returns.  Arguments documented as
 *    "device" must be device pointers on the context's device; they are read
 *    or written on the context's stream, and the call returns once that work
 *    is queued (smm_apply_* and smm_get_outputs with on_device = 1) or done
 *    (everything else synchronises the stream before returning).
 *  - A context is bound to one device and one HIP stream and must not be used
 *    from two threads at once.
 */
#ifndef SMM_H
#define SMM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SMM_OK 0
#define SMM_EINVAL -1        /* bad argument (sizes, ranges, null pointers, det J <= 0) */
#define SMM_ENOMEM -2        /* device or host allocation failed */
#define SMM_EHIP -3          /* a HIP runtime call failed */
#define SMM_ENOCONV -4       /* outer iteration hit max_outer; outputs hold the last iterate */
#define SMM_ENAN -5          /* NaN or Inf in the outer residual or in the moment solve */
#define SMM_EBREAKDOWN -6    /* CG breakdown: p.Ap <= 0 (moment operator not positive definite) */
#define SMM_EUNSUPPORTED -7  /* valid input the library does not handle (e.g. slanted boundary) */
#define SMM_ESTATE -8        /* call order violated (e.g. solve before set_materials) */

/* precision of the sweep and the angular-moment contraction */
#define SMM_FP64 0
#define SMM_FP32_SWEEP 1

/* source layouts for smm_set_source */
#define SMM_SRC_ISO 0        /* q[n_elem][n_node], per steradian, same for all directions */
#define SMM_SRC_ANISO 1      /* q[n_dir][n_elem][n_node] */

/* inflow layouts for smm_set_inflow */
#define SMM_INFLOW_VACUUM 0  /* psibar = 0 (pointer ignored) */
#define SMM_INFLOW_ISO_FACE 1/* psibar[n_bface]: isotropic, constant per boundary face */
#define SMM_INFLOW_FULL 2    /* psibar[n_bface][nq][n_dir] at the boundary face points */
#define SMM_INFLOW_ISO_ATTR 3/* psibar[n_bdr_attr]: isotropic, one value per boundary attribute */

/* angular quadrature kinds (Sec. 4) */
#define SMM_QUAD_LEVEL_SYMMETRIC 0
#define SMM_QUAD_EXPLICIT 1

/* preconditioners of the moment solve */
#define SMM_PRECOND_BJ 0
#define SMM_PRECOND_TWOLEVEL 1

/* moment-system discretisation (Sec. 5.1) */
#define SMM_DISC_IP 0   /* interior penalty on the DG space Y_p (eq. ipsmm) */
#define SMM_DISC_CG 1   /* continuous finite elements: the same forms on V_p */

/* initial guess for smm_solve */
#define SMM_START_ZERO 0
#define SMM_START_DIFFUSION 1 /* moment system with zero transport corrections */
#define SMM_START_GIVEN 2     /* varphi0 argument (host) */

typedef struct smm_ctx smm_ctx;
typedef struct smm_problem smm_problem;
typedef struct smm_batch smm_batch;

/* Mesh: structured nx * ny quadrilaterals with a continuous Q_m map whose
 * control points sit at the Gauss-Lobatto positions of each element
 * (Sec. 3.1).  ctrl is host memory, shape [ny*m+1][nx*m+1][2] (x fastest),
 * shared between neighbouring elements. */
typedef struct {
    int nx, ny;
    int m;
    const double* ctrl;
} smm_mesh_desc;

/* Mesh given element by element (Sec. 3.1): any conforming quadrilateral
 * mesh.  ctrl (host) [n_elem][(m+1)^2][2]: the Gauss-Lobatto control points
 * of each element's Q_m map, index a + (m+1) b with a along the reference
 * xi axis; every element must be counter-clockwise (det J > 0).  nbr (host)
 * [n_elem][4]: the element across local face f (0: eta = 0, 1: xi = 1,
 * 2: eta = 1, 3: xi = 0), or -1 on the domain boundary; neighbours must
 * name each other and carry the same face control points (the library
 * matches the faces and their orientation; SMM_EINVAL if they do not
 * match).  bdr_attr (host, nullable) [n_elem][4]: a boundary attribute
 * >= 0 on each boundary face (read on boundary faces only; NULL: the local
 * face index).  Element order, local numbering and boundary-face order
 * (element, then local face) are the caller's; DOFs follow them. */
typedef struct {
    int n_elem;
    int m;
    const double* ctrl;
    const int* nbr;
    const int* bdr_attr;
} smm_mesh_general_desc;

/* Angular quadrature (Sec. 4).  SMM_QUAD_LEVEL_SYMMETRIC: the 2D
 * half-sphere level-symmetric set of order sn_order in {4, 6, 8, 10, 12}.
 * SMM_QUAD_EXPLICIT: n_dir directions omega (host, [n_dir][3] unit vectors
 * with Omega_z >= 0 and nonzero in-plane components) and weights w (host,
 * [n_dir], positive, summing to 4 pi within 1e-12 relative), in the order
 * the caller gives them. */
typedef struct {
    int kind;
    int sn_order;
    int n_dir;
    const double* omega;
    const double* w;
} smm_quad_desc;

typedef struct {
    int n_elem;      /* nx * ny */
    int n_node;      /* (p+1)^2 DOF per element */
    int n_dir;       /* S_N directions */
    int n_bface;     /* boundary faces */
    int nq;          /* Gauss points per face (p+m+1) */
    int cartesian;   /* 1: uniform axis-aligned rectangles (operator tables per material and direction) */
    int n_material;  /* distinct sigma_t values (cartesian path) */
    int n_levels;    /* max sweep wavefront levels over directions */
    int n_self_types;/* typed Cartesian path: distinct element blocks (0 until built) */
    int n_nbr_types; /* typed Cartesian path: distinct neighbour blocks */
    int general;     /* 1: mesh given element by element (smm_problem_create_general) */
    int n_bdr_attr;  /* boundary attributes 0 .. n_bdr_attr - 1 */
} smm_problem_dims;

typedef struct {
    int precision;       /* SMM_FP64 or SMM_FP32_SWEEP */
    double outer_tol;    /* stop when max|X^{k+1}-X^k| / max|X^{k+1}| < outer_tol */
    int max_outer;
    double inner_tol;    /* CG relative residual ||r||_2/||b||_2 */
    int max_inner;       /* CG iterations per outer iteration */
    int start;           /* SMM_START_* */
    int delta_sweeps;    /* 1: sweep only the change of the scattering source and
                            accumulate the moments in FP64 (default for FP32_SWEEP) */
    int use_graph;       /* 1: replay the PCG iteration chunks of the typed (batched) path
                            and of the CG moment solve from captured hipGraphs; 2 (typed path):
                            also replay each outer iteration -- scattering source, the forked
                            persistent sweep launches, moments, closures, right-hand side, PCG
                            start and a chunk of PCG iterations (what the last iteration's slowest
                            solve needed, rounded down to an even number, 2..64), residual and
                            Anderson's products --
                            from one captured graph per iteration shape; moment solves that need
                            more iterations continue in replayed chunks.  Results are bitwise
                            those of the eager launches. */
    int moment_path;     /* 0: typed blocks on uniform Cartesian meshes with isotropic
                            sources (batched kernels), else per-element operators;
                            1: always per-element operators */
    int anderson;        /* 0: plain fixed point X <- G(X); 1 or 2: Anderson mixing of the
                            last anderson + 1 iterates (typed path only) */
    int precond;         /* SMM_PRECOND_BJ: block-Jacobi PCG (Jacobi on the CG system);
                            SMM_PRECOND_TWOLEVEL: that plus a continuous Q1 coarse correction
                            on the element vertices, solved by one vertex multigrid V-cycle
                            (IP: typed path; CG: the continuous system of any structured
                            mesh, the coarse operator the Galerkin product with it) */
    double inner_adapt;  /* > 0: the moment solve of outer iteration k stops at the
                            relative residual max(inner_tol, inner_adapt * r_{k-1})
                            (r_0 = 1; per problem in a batch), and the solves that
                            build a diffusion or learned start at
                            max(inner_tol, inner_adapt) unless start_tol is set; 0: always
                            inner_tol */
    int discretization;  /* SMM_DISC_IP (default) or SMM_DISC_CG.  SMM_DISC_CG solves the
                            continuous moment system of Sec. 5.1 (one unknown per node of the
                            (nx p + 1) x (ny p + 1) grid of V_p) by FP64 preconditioned CG
                            (Jacobi, or two-level with SMM_PRECOND_TWOLEVEL) on the per-element
                            path of smm_solve; varphi is returned at the
                            DG nodes (continuous).  `precond` does not apply; Anderson mixing
                            and batches return SMM_EUNSUPPORTED */
    double kappa_scale;  /* factor on the IP penalty kappa = {(p+1)^2 / (sigma_t h)} (Sec. 6; the
                            paper scales it on its distorted mesh), >= 0, default 1.  A new value
                            re-assembles the moment system; a batch keeps the value its problems had
                            when it was created (another value: SMM_EUNSUPPORTED).  A value that
                            makes the operator indefinite ends the solve with SMM_EBREAKDOWN. */
    double start_tol;    /* > 0: the relative residual at which the moment solve that builds a
                            diffusion or learned start stops; 0 (default): max(inner_tol,
                            inner_adapt) when inner_adapt > 0, else inner_tol */
} smm_solve_opts;

typedef struct {
    int iterations;          /* outer iterations done */
    double residual;         /* last relative outer residual */
    double residual_abs;     /* last absolute max-norm change */
    int cg_iterations_total;
    int cg_iterations_max;
    double t_total_ms;       /* wall time of the whole solve call, t_setup_ms included (host clock) */
    double t_setup_ms;       /* before the first outer iteration: device tables on the first
                              * solve, and building the start (diffusion solve, network) */
    /* device time of the outer-iteration phases, summed over the outer
     * iterations (HIP events on the context's stream; in a batch, the batch's
     * launches, which cover every problem): */
    double t_sweep_ms;       /* scattering source and sweep */
    double t_moments_ms;     /* angular moments, closures and right-hand side */
    double t_cg_ms;          /* moment solve (CG) */
    double t_residual_ms;    /* residual, mixing and shift of the iterates */
} smm_solve_info;

const char* smm_strerror(int code);

/* Context bound to HIP device `device` and stream `hip_stream` (a hipStream_t,
 * NULL = the null stream).  device < 0 creates a host-only context: problems
 * may be created and their setup tables inspected, but nothing runs. */
int smm_ctx_create(int device, void* hip_stream, smm_ctx** out);
int smm_ctx_destroy(smm_ctx* ctx);
const char* smm_last_error(smm_ctx* ctx);

/* Geometry, quadrature and basis setup (Sec. 3, Sec. 4).  p in 1..4;
 * sn_order in {4, 6, 8, 10, 12}.  SMM_EINVAL if det J <= 0 at a volume
 * quadrature point; SMM_EUNSUPPORTED if the upwind graph of a direction has
 * a cycle (a chord quadrilateral that is not convex).  Boundary attributes
 * of a structured mesh: the local face index (0 bottom, 1 right, 2 top,
 * 3 left). */
int smm_problem_create(smm_ctx* ctx, const smm_mesh_desc* mesh, int p, int sn_order,
                       smm_problem** out);
/* The same for any conforming quadrilateral mesh given element by element
 * and any angular quadrature (mesh and quad as documented at their types).
 * Such a problem runs on the per-element paths: per-element assembly and
 * elimination in the sweep, the block-sparse IP moment system (eq. ipsmm)
 * with block-Jacobi PCG, and beta at every boundary point from its own
 * normal (Sec. 4); batches, tiles, the CG moment system and Anderson mixing
 * return SMM_EUNSUPPORTED on it.  A structured mesh descriptor with an
 * explicit quadrature goes through smm_problem_create_q. */
int smm_problem_create_general(smm_ctx* ctx, const smm_mesh_general_desc* mesh, int p, const smm_quad_desc* quad,
                               smm_problem** out);
/* smm_problem_create with a quadrature descriptor. */
int smm_problem_create_q(smm_ctx* ctx, const smm_mesh_desc* mesh, int p, const smm_quad_desc* quad,
                         smm_problem** out);
int smm_problem_destroy(smm_problem* prob);
int smm_get_dims(const smm_problem* prob, smm_problem_dims* out);

/* host outputs: omega[n_dir][3], w[n_dir] */
int smm_get_quadrature(const smm_problem* prob, double* omega, double* w);
/* host output: physical coordinates of the DOF nodes [n_elem][n_node][2] */
int smm_get_nodes(const smm_problem* prob, double* xy);
/* host output: physical coordinates of the boundary face points [n_bface][nq][2] */
int smm_get_bface_points(const smm_problem* prob, double* xy);

/* Per-element cross sections (host, length n_elem); requires sigma_t > 0 and
 * 0 <= sigma_s <= sigma_t.  Fixes the IP operator (eq. ipsmm, penalty
 * kappa = {(p+1)^2/(sigma_t h)}, h = |K|^(1/2)). */
int smm_set_materials(smm_problem* prob, const double* sigma_t, const double* sigma_s);
/* Fixed source q per steradian (host), layout SMM_SRC_*. */
int smm_set_source(smm_problem* prob, const double* q, int layout);
/* Inflow psibar (host), layout SMM_INFLOW_*. */
int smm_set_inflow(smm_problem* prob, const double* psibar, int layout);

void smm_default_opts(smm_solve_opts* opts);

/* Fixed-point solve X^{k+1} = G(X^k) (eq. fixed-point).  varphi0 (host,
 * [n_elem*n_node]) is read when opts->start == SMM_START_GIVEN.  Returns
 * SMM_ENOCONV with valid outputs when max_outer is reached, SMM_ENAN when a
 * residual or the moment solve turns non-finite (a non-finite varphi0, say),
 * SMM_EBREAKDOWN when the moment solve meets p.Ap <= 0.  opts->start ==
 * SMM_START_LEARNED (smm_cnn.h) uses the network set by smm_set_warmstart
 * (uniform Cartesian meshes with an isotropic source). */
int smm_solve(smm_problem* prob, const smm_solve_opts* opts, const double* varphi0,
              smm_solve_info* info);

/* Outer residual r_k (and CG iterations of that outer iteration's moment
 * solve, nullable) of each outer iteration of the last smm_solve: the first
 * min(max_len, *len) entries are written (host), *len receives the
 * iteration count. */
int smm_solve_history(const smm_problem* prob, int max_len, double* residual, int* cg_iterations, int* len);

/* Results of the last smm_solve or smm_apply_G.  Any pointer may be NULL.
 * varphi, phi [n_elem*n_node]; J [2][n_elem*n_node]; T [3][n_elem*n_node]
 * (xx, xy, yy); beta [n_bface][nq].  on_device selects device or host
 * destination buffers. */
int smm_get_outputs(smm_problem* prob, double* varphi, double* phi, double* J, double* T,
                    double* beta, int on_device);

/* One application of L^{-1} (Sec. 4), for testing and benchmarking.
 * S: device, [n_elem][n_node] (s_layout SMM_SRC_ISO) or [n_dir][n_elem][n_node]
 * (SMM_SRC_ANISO), of type double (precision SMM_FP64) or float
 * (SMM_FP32_SWEEP).  psi_lag: device, previous sweep [n_dir][n_elem][n_node]
 * read at curved-face points whose upwind neighbour is downstream in the
 * sweep graph (NULL = zero).  psi_out: device [n_dir][n_elem][n_node], same
 * type.  Boundary inflow is the one set by smm_set_inflow (if with_inflow). */
int smm_apply_sweep(smm_problem* prob, int precision, const void* S, int s_layout,
                    const void* psi_lag, void* psi_out, int with_inflow);

/* Angular moments (Sec. 4) of psi (device [n_dir][n_elem][n_node], type per
 * precision) on the matrix cores: mom (device, double [8][n_elem*n_node]) rows
 * phi, J_x, J_y, P_xx, P_xy, P_yy, sum w|Omega_x| psi, sum w|Omega_y| psi. */
int smm_apply_moments(smm_problem* prob, int precision, const void* psi, double* mom);

/* One evaluation of G (eq. moment:smm_fp) in FP64 (or with an FP32 sweep):
 * varphi_in, varphi_out device [n_elem*n_node]; lagged curved-face couplings
 * read zero.  CG runs to inner_tol from varphi_in.  smm_get_outputs then
 * returns this evaluation's moments and closures. */
int smm_apply_G(smm_problem* prob, int precision, const double* varphi_in, double* varphi_out,
                double inner_tol, int max_inner);

/* The same evaluation of G as smm_apply_G, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): this call allocates nothing.  Its work vectors
 * (scattering source, angular flux, moments, closures, right-hand side, CG
 * vectors and partial sums) live in one fixed array of 32 MiB per device,
 * held by the library from the first context on that device until the
 * process ends.  varphi_in and varphi_out (device, [n_elem*n_node]) stay the
 * caller's.  The problem's own tables must already be on the device: call
 * smm_apply_G once after the last smm_set_* change, else SMM_ESTATE.
 * SMM_EINVAL when the work vectors exceed the array (8 * n_elem*n_node *
 * (n_dir + 20) bytes, about, with an isotropic source).  Every call on one
 * device shares that device's array, whose contents are whatever the last
 * call left (each buffer is written before it is read): calls that overlap
 * on one device, from any context or stream, race.  smm_get_outputs is not
 * changed by this call.  On curved meshes the sweep uses the stored element
 * operators of that precision when their memory exists (it is then refilled
 * after a change of materials, which allocates nothing), else it assembles
 * each element's system. */
int smm_apply_G_noalloc(smm_problem* prob, int precision, const double* varphi_in, double* varphi_out,
                        double inner_tol, int max_inner);

/* Host-only inspection of the setup tables (for tests): the IP matrix as
 * dense row-major [N][N] with N = n_elem*n_node (small problems only), and
 * the fixed right-hand side [N]. */
int smm_debug_ip_dense(const smm_problem* prob, double* A, double* b_fixed);

/* Host-only inspection of the sweep graph of Sec. 4 (built from the chord
 * normals; with tiles, edges only inside tiles): level [n_dir][n_elem] gets
 * each element's wavefront level (longest upwind path, Kahn's algorithm) and
 * upstream [n_dir][n_elem] a bit mask whose bit f is set when the neighbour
 * across local face f is a graph predecessor (faces without that bit read
 * inflow, or the lagged previous sweep).  Either pointer may be NULL.
 * SMM_EUNSUPPORTED when the graph has a cycle. */
int smm_debug_sweep_graph(smm_problem* prob, int* level, unsigned char* upstream);

/* Host-only inspection of the continuous (CG) moment system of Sec. 5.1.
 * Writes *nc (continuous unknowns) and *nnz; when rowptr is non-NULL also
 * the CSR matrix A_c (rowptr[nc + 1], col[nnz], val[nnz], columns ascending)
 * and map[n_elem * n_node], the continuous unknown of each DG node (so the DG
 * values of a continuous vector c are c[map[t]]).  All arrays are host memory
 * owned by the caller. */
int smm_debug_cg_system(smm_problem* prob, int* nc, int* nnz, int* rowptr, int* col, double* val, int* map);
/* Host-only inspection of the two-level preconditioner of the CG moment
 * system: the 9-point stencil [9][nvx*nvy] of multigrid level `level`, laid
 * out as smm_debug_mg_level's (level 0: the Galerkin operator P1^T A_c P1 of
 * the bilinear space on the element vertices, P1 its interpolation at the
 * continuous nodes).  A9 may be NULL to query the grid size.  SMM_EINVAL for
 * a level beyond the coarsest, SMM_EUNSUPPORTED on an unstructured mesh. */
int smm_debug_cg_mg_level(smm_problem* prob, int level, double* A9, int* nvx, int* nvy);
/* y = A_c x with the device product kernel of the CG moment solve; x and y are
 * host arrays of nc doubles (nc from smm_debug_cg_system). */
int smm_debug_cg_spmv(smm_problem* prob, const double* x, double* y);
/* Average time in ms of `reps` back-to-back launches of that product kernel
 * on the context stream (HIP events), x = 1. */
int smm_time_cg_spmv(smm_problem* prob, int reps, double* ms_avg);

/* Sweep kernel selection: 0 = automatic (tabulated operators on uniform
 * Cartesian meshes; otherwise the per-element sweep with stored element
 * operators: the inverse of each (element, direction) left-hand side and its
 * inflow-face operators, built in parallel on first use after a change of
 * materials or inflow and kept in device memory, n_dir * n_elem *
 * (n_node^2 + n_node + 4 (p+1) n_node) values of the sweep type; where
 * those would take more than a quarter of the free device memory, the form
 * of path 5); 1 = always the
 * per-element sweep (form as in 0); 2 = on Cartesian meshes, the element-row
 * kernel instead of the column-per-thread one; 3 = the per-element kernel
 * assembling and eliminating with one wave per element at every order; 4 =
 * the same with one lane per row at every order p >= 2; 5 = the same with one
 * lane per row for p >= 3, and for p = 2 unless the levels are wide and spread
 * over many workgroups, otherwise one lane per element.  2 to 5 are for
 * cross-checking the kernels against each other.  Returns SMM_EINVAL outside
 * 0..5. */
int smm_set_sweep_path(smm_problem* prob, int path);

/* Parallel block Jacobi sweep (Sec. 6.5, weak scaling): the element grid is
 * cut into tiles of tile_nx x tile_ny elements (the last row and column of
 * tiles may be smaller), each tile is swept on its own in upwind order, and
 * inflow across a face between tiles is the previous sweep's (zero on the
 * first sweep; in delta sweeps, the previous delta).  The SMM fixed point is
 * unchanged; the outer iteration count grows with the number of tiles.  Runs
 * on the per-element sweep path, one workgroup per (direction, tile).
 * (0, 0) restores the full sweep.  Problems with tiles cannot join a batch
 * (SMM_EUNSUPPORTED); tiles set on a problem after it joined a batch apply
 * to its own smm_solve calls, not to the batch, which sweeps whole meshes.
 * SMM_EINVAL for negative sizes or only one size 0. */
int smm_set_sweep_tiles(smm_problem* prob, int tile_nx, int tile_ny);

/* Time one sweep configuration on device (average ms over `reps` launches
 * measured with HIP events on the context stream); used by the benchmark. */
int smm_time_sweep(smm_problem* prob, int precision, int reps, double* ms_avg);
/* The parts of a per-element sweep with stored element operators, each the
 * average over `reps` rounds (HIP events on the context stream, ms): the
 * build of the operators (*ms_setup, run after every change of materials),
 * the pass psi = A^-1 (M S + boundary inflow) over all elements and
 * directions (*ms_particular) and the pass over the levels (*ms_levels); the
 * last two make one sweep.  SMM_EUNSUPPORTED when the problem does not sweep
 * with stored operators (tabulated Cartesian kernel, an assembling sweep
 * path, or operators too large for the free device memory). */
int smm_time_sweep_parts(smm_problem* prob, int precision, int reps, double* ms_setup, double* ms_particular,
                         double* ms_levels);

/* Host-only inspection of the typed Cartesian representation: the IP matrix
 * [N][N], the correction-source operator [N][3N] (columns: T_xx, T_xy, T_yy
 * blocks of N) and the fixed right-hand side [N], rebuilt from the typed
 * blocks (small problems only; SMM_EUNSUPPORTED if the typed path does not
 * apply). */
int smm_debug_typed_dense(smm_problem* prob, double* A, double* C, double* b_fixed);
/* The same correction-source operator [N][3N] from the per-element assembly. */
int smm_debug_corr_dense(smm_problem* prob, double* C);
/* Host-only inspection of the two-level preconditioner: the 9-point stencil
 * [9][nvx*nvy] (entry k = (dy+1)*3 + (dx+1) couples vertex (x, y) to
 * (x+dx, y+dy)) of multigrid level `level` (0: the Galerkin operator of the
 * continuous Q1 space on the element vertices).  A9 may be NULL to query the
 * grid size. */
int smm_debug_mg_level(smm_problem* prob, int level, double* A9, int* nvx, int* nvy);
/* Testing hook: z = M^-1 r for every problem of a batch with the PCG
 * preconditioner `precond` (SMM_PRECOND_*); r and z are n host pointers of
 * n_elem * n_node values each.  Overwrites the batch's PCG work vectors (the
 * outputs of the last solve become unavailable). */
int smm_debug_batch_precond(smm_batch* batch, int precond, const double* const* r, double* const* z);
/* Testing hook: y = A x, A the typed IP moment matrix (eq. ipsmm) of every
 * problem of a batch, with the batch's current PCG kernels; x and y are n
 * host pointers of n_elem * n_node values each.  Overwrites the batch's PCG
 * work vectors. */
int smm_debug_batch_spmv(smm_batch* batch, const double* const* x, double* const* y);
/* Testing hook: one batched sweep (Sec. 4) of every problem of the batch, in
 * the launch configuration smm_batch_solve uses (one persistent launch per
 * order and workgroup shape, tuned grids and streams, the same task queue),
 * on the isotropic scattering sources S: n host pointers of
 * [n_elem][n_node] doubles (NULL entry: zero source), rounded to the sweep
 * precision, with each problem's own boundary inflow.  psi_k (host,
 * [n_dir][n_elem][n_node] doubles) receives problem k's angular flux.
 * Overwrites the batch's sweep buffers (outputs of the last solve stay). */
int smm_batch_apply_sweep(smm_batch* batch, int precision, const double* const* S, int k, double* psi_k);
/* Testing hook: force the kernel shape of the batch's persistent sweep
 * launches: 0 column-wave (the NB waves of a 64-slot chunk split each
 * element's node columns), 1 element-lane (one wave per chunk, each lane a
 * whole element; anti-diagonals of at most 256 slots, else
 * SMM_EUNSUPPORTED), 2 and 3 matrix cores (each level a product of the
 * element operator with the level's inputs, in tiles of 16 elements, 4 or 2
 * tiles per wave; FP32 sweeps only, FP64 sweeps keep the autotuner's
 * choice; anti-diagonals of at most 256 or 128 slots, else
 * SMM_EUNSUPPORTED), -1 the autotuner's choice per launch.  Grids are tuned
 * again at the next solve or sweep.  Shapes 0 and 1 apply each element's
 * operator rows in the same order, and so do shapes 2 and 3 (in another
 * order: results agree to rounding). */
int smm_debug_batch_sweep_shape(smm_batch* batch, int shape);
/* Testing hook: choose the batch's PCG kernels: 1 the type-group kernels
 * (one wave per group of elements sharing their blocks), 0 the per-node
 * kernels, -1 the automatic choice (group fill).  Results agree up to the
 * summation order.  Drops the captured PCG and outer-iteration graphs.
 * SMM_EUNSUPPORTED if the batch has no type groups. */
int smm_debug_batch_grouped(smm_batch* batch, int grouped);
/* Testing hook: 1 (the default) runs the per-order launches of each PCG
 * phase concurrently on forked streams when the batch holds more than one
 * order, 0 one after the other on the context stream.  The launches touch
 * disjoint problems, so results are bitwise the same.  Drops the captured
 * PCG and outer-iteration graphs.  SMM_EINVAL outside 0..1. */
int smm_debug_batch_cg_fork(smm_batch* batch, int fork);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems (uniform Cartesian meshes, isotropic
 * sources, vacuum or face-wise isotropic inflow) solved together.  Each
 * kernel launch of the outer iteration covers every problem that has not yet
 * converged; the sweep runs as one persistent launch per order p, fed by a
 * queue of (problem, direction) tasks.  The problems stay owned by the
 * caller and must outlive the batch; changing their data afterwards requires
 * a new batch.
 * ------------------------------------------------------------------------- */
int smm_batch_create(smm_ctx* ctx, smm_problem* const* probs, int n, smm_batch** out);
int smm_batch_destroy(smm_batch* batch);
/* varphi0: NULL, or n pointers (host or device, NULL entries allowed) read
 * when opts->start == SMM_START_GIVEN.  info: NULL or n entries.  Returns
 * SMM_ENOCONV if any problem reached max_outer (all outputs stay valid). */
int smm_batch_solve(smm_batch* batch, const smm_solve_opts* opts, const double* const* varphi0,
                    smm_solve_info* info);
/* Outputs of problem k of the last smm_batch_solve (layouts as smm_get_outputs). */
int smm_batch_get_outputs(smm_batch* batch, int k, double* varphi, double* phi, double* J, double* T,
                          double* beta, int on_device);
/* Average time of one batched sweep (all problems, all directions). */
int smm_batch_time_sweep(smm_batch* batch, int precision, int reps, double* ms_avg);
/* Elem*angle*DOF units of one batched sweep. */
int smm_batch_units(const smm_batch* batch, double* units);
/* Time of the outer-iteration phases of the last smm_batch_solve, in ms,
 * summed over its outer iterations (HIP events on the context's stream):
 * ms[0] scattering source and sweep, ms[1] moments, closures and right-hand
 * side, ms[2] PCG moment solve, ms[3] residual and shift.  With use_graph = 2
 * the phases are instead: ms[0] the replayed iteration graph (source through
 * the first PCG chunk and the residual), ms[1] further PCG chunks, ms[2] the
 * residual taken again after them, ms[3] read-back, shift or mixing.
 * cg_iterations (nullable) receives the number of batched PCG iterations
 * launched. */
int smm_batch_phase_times(const smm_batch* batch, double* ms, long* cg_iterations);
/* Outer residual r_k (and PCG iterations, nullable) of each outer iteration of
 * problem k in the last smm_batch_solve: the first min(max_len, *len) entries
 * are written, *len receives the iteration count. */
int smm_batch_history(const smm_batch* batch, int k, int max_len, double* residual, int* cg_iterations, int* len);
/* Average duration (HIP events on the stream each kernel runs on) of reps
 * back-to-back launches of one batched kernel: SMM_KERNEL_SWEEP_FP32 /
 * SMM_KERNEL_SWEEP_FP64 (one whole batched sweep), SMM_KERNEL_CG_SPMV (the
 * PCG kernel q = A p with its partial dot products, on the state left by the
 * last smm_batch_solve), SMM_KERNEL_MOMENTS_FP32 (the angular moments of the
 * last FP32 sweep into the work moments, which the solve's outputs do not
 * read); SMM_ESTATE before any solve for the last two. */
#define SMM_KERNEL_SWEEP_FP32 0
#define SMM_KERNEL_SWEEP_FP64 1
#define SMM_KERNEL_CG_SPMV 2
#define SMM_KERNEL_MOMENTS_FP32 3
int smm_batch_time_kernel(smm_batch* batch, int kernel, int reps, double* ms_avg);

#ifdef __cplusplus
}
#endif

#endif /* SMM_H */
