// Internal data structures of libsmm (host side).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "smm.h"

namespace smm {

// ---------------------------------------------------------------------------
// 1D rules and bases (host_setup.cpp)
// ---------------------------------------------------------------------------
void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& w);
void gauss_lobatto01(int p, std::vector<double>& x);
// L[a*npts + k] = l_a(x_k), dL likewise for the derivative
void lagrange_tables(const std::vector<double>& nodes, const std::vector<double>& pts,
                     std::vector<double>& L, std::vector<double>& dL);
// 2D level-symmetric half-sphere set (quadrant-major), weights sum to 4 pi
int level_symmetric(int N, std::vector<double>& omega, std::vector<double>& w);

// ---------------------------------------------------------------------------
// Problem
// ---------------------------------------------------------------------------
struct DeviceBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct smm_ctx_impl;

struct Problem {
    smm_ctx* ctx = nullptr;
    // sizes
    int nx = 0, ny = 0, m = 0, p = 0, nb = 0, n = 0, nq = 0, ne = 0, nd = 0, nbf = 0, sn = 0;
    int nlev_max = 0;
    // quadrature / basis
    std::vector<double> omega, w;          // [nd][3], [nd]
    std::vector<double> gl;                // solution nodes (nb)
    std::vector<double> sq, wq;            // face / 1D volume Gauss rule (nq)
    std::vector<double> Lf, dLf;           // [nb][nq] 1D basis at Gauss points
    double eb0x = 0, eb0y = 0;             // E_b0 for x- and y-normal boundary faces

    // mesh given element by element (smm_problem_create_general): per-element
    // control points [ne][(m+1)^2][2], neighbours [ne][4] and boundary
    // attributes [ne][4] as given; nx = ne, ny = 1
    bool general = false;
    std::vector<double> ctrl_e;
    std::vector<int> nbr_in, bdr_attr_in;
    bool quad_explicit = false;            // directions given by the caller (not level-symmetric)

    // geometry (general path data, FP64)
    std::vector<double> ctrl;              // copy of control points
    std::vector<double> xnode;             // [ne][n][2]
    std::vector<double> area;              // [ne]
    std::vector<double> Mk, Gxk, Gyk;      // [ne][n][n]
    std::vector<double> nds;               // [ne][4][nq][2] weight * n ds
    std::vector<double> dsw;               // [ne][4][nq]   weight * ds
    std::vector<double> nhat;              // [ne][4][nq][2]
    std::vector<double> xf;                // [ne][4][nq][2]
    std::vector<double> vol_wJ;            // [ne][nq*nq]
    std::vector<double> vol_grad;          // [ne][nq*nq][n][2]
    std::vector<double> face_grad;         // [ne][4][nq][n][2]
    std::vector<double> vol_U;             // [nq*nq][n]
    std::vector<int> nbr;                  // [ne][4]
    std::vector<int> nbr_face;             // [ne][4] neighbour's local face | 4 if its parameter runs the
                                           //   other way (its point nq-1-q is this element's q); -1 boundary
    std::vector<int> bface_attr;           // [nbf] boundary attribute
    int n_bdr_attr = 0;
    bool axis_bdr = true;                  // every boundary normal along x or y (E_b0 one constant per axis)
    std::vector<double> eb0_pt;            // [nbf][nq] E_b0 at each boundary point (eq. eb0_disc)
    std::vector<int> bface_of;             // [ne][4] -> boundary face id or -1
    std::vector<int> bface_K, bface_f;     // [nbf]
    std::vector<double> chord;             // [ne][4][2] integral of n ds (from end points)

    // cartesian fast path
    bool cartesian = false;
    double hx = 0, hy = 0;
    int nmat = 0;
    std::vector<double> mat_sigma;         // [nmat]
    std::vector<uint8_t> mat_of;           // [ne]
    std::vector<double> Pm, Px, Py;        // [nmat][nd][n][n], [nmat][nd][n][nb] x2

    // general-path sweep graph; with tiles (parallel block Jacobi sweep) the
    // graph has edges only inside tiles of tile_x x tile_y elements
    int tile_x = 0, tile_y = 0, ntiles = 1;
    int lev_wmax = 0;                      // most elements in one level of one (direction, tile)
    std::vector<int> lev_ptr;              // [nd][ntiles][nlev_max+1]
    std::vector<int> lev_elem;             // [nd][ne], tile-major, then level
    std::vector<uint8_t> upflag;           // [nd][ne] bit f: neighbour across f is upstream

    double kappa_scale = 1.0;              // factor on the IP penalty (solve option)

    // materials, sources, inflow
    bool have_mat = false;
    std::vector<double> sigma_t, sigma_s;  // [ne]
    int src_layout = SMM_SRC_ISO;
    std::vector<double> q;                 // [ne][n] or [nd][ne][n]
    int inflow_layout = SMM_INFLOW_VACUUM;
    std::vector<double> psibar;            // [nbf][nq][nd] (full layout)

    // moment system (FP64)
    std::vector<int> bsr_col;              // [ne][5] (slot 0 = self, 1+f = neighbour f; -1 none)
    std::vector<double> bsr_val;           // [ne][5][n][n]
    std::vector<double> bjac_inv;          // [ne][n][n]
    std::vector<double> corr_val;          // [ne][5][n][3n] correction-tensor operator
    std::vector<double> beta_op;           // [nbf][n][nq]: dsw_q u_i(q)
    std::vector<double> b_fixed;           // [ne*n]
    bool lhs_ready = false;
    bool rhs_fixed_ready = false;

    bool heavy_ready = false;          // per-element quadrature data present
    bool graph_ready = false;          // per-direction sweep graph present

    // typed moment-system blocks (uniform Cartesian meshes, isotropic source)
    bool typed_ready = false;
    int nself = 0, nnbrt = 0;
    std::vector<int> sid;              // [ne] self-block type
    std::vector<int> nid;              // [ne][4] neighbour-block type (-1 boundary)
    std::vector<double> t_ip_self, t_ip_nbr, t_dinv;   // [nself|nnbrt][n][n]
    std::vector<double> t_c_self, t_c_nbr;             // [nself|nnbrt][n][3n]
    std::vector<double> t_bop;                         // [4][n][nq]
    std::vector<double> t_bfix;                        // [ne][n]

    // continuous (CG) moment system on V_p (cg_smm.cpp)
    bool cg_ready = false;
    int cg_nc = 0;                     // (nx p + 1)(ny p + 1) continuous nodes
    std::vector<int> cg_map;           // [ne][n] DG node -> continuous node
    std::vector<int> cg_tab;           // [nc][4] DG nodes at each continuous node, ascending, -1 padded
    std::vector<int> cg_rowptr, cg_col;// CSR of A_c = P_c^T A P_c (element and boundary terms)
    std::vector<double> cg_val, cg_dinv;

    // device state (api.hip)
    void* dev = nullptr;
};

int setup_geometry(Problem& P, std::string& err, bool heavy);
// the neighbour's face and its point that coincide with point q of face f of K
inline void nbr_point(const Problem& P, int K, int f, int q, int& fN, int& qN) {
    const int code = P.nbr_face[(size_t)K * 4 + f];
    fN = code & 3;
    qN = (code & 4) ? P.nq - 1 - q : q;
}
int ensure_heavy(Problem& P, std::string* err = nullptr);   // per-element quadrature data and sweep graph, on demand
void setup_cartesian_operators(Problem& P);
int setup_sweep_graph(Problem& P, std::string& err);  // SMM_EUNSUPPORTED on a cycle
void assemble_ip(Problem& P);
void add_volume_block(const Problem& P, int K, double* blk);
void add_boundary_block(const Problem& P, int K, int f, double* blk);
void assemble_cg(Problem& P);
void assemble_rhs_fixed(Problem& P);
void assemble_correction_operator(Problem& P);
void cartesian_boundary_traces(const Problem& P, std::vector<double>& bx, std::vector<double>& by);
int lu_invert(int n, double* A);  // in-place inverse, partial pivoting; returns 0 on success
bool typed_applicable(const Problem& P);
int build_typed_blocks(Problem& P, std::string& err);

}  // namespace smm
