// Typed moment-system blocks for uniform Cartesian meshes.
//
// On a mesh of identical axis-aligned rectangles, the IP operator block of an
// element (eq. ipsmm, left-hand side), its block-Jacobi inverse and its
// correction-source blocks depend only on the local configuration: the
// element's cross sections, which faces lie on the boundary, and the total
// cross sections of its face neighbours.  Each distinct configuration is
// assembled once by running the general assembly on a small patch of
// elements (at most 3 x 3) that reproduces the neighbourhood, and every
// element stores the type id of its self block and of its four neighbour
// blocks.  The arithmetic is therefore the general assembly's, and the
// operators of a 128 x 128 problem shrink from hundreds of MB to a few KB.
//
// Applies to isotropic sources (nodal q per steradian) with vacuum or
// face-wise isotropic inflow; the first moment of such a source,
// sum_d w_d Omega_d q, vanishes for the symmetric S_N sets and is taken as 0.
#include <array>
#include <cmath>
#include <cstring>
#include <map>

#include "smm_internal.hpp"

namespace smm {

bool typed_applicable(const Problem& P) {
    // (the typed right-hand side also relies on the symmetry of the
    // level-symmetric set: sum w Omega q = 0 for an isotropic q)
    return P.cartesian && !P.general && !P.quad_explicit && P.src_layout == SMM_SRC_ISO &&
           (P.inflow_layout == SMM_INFLOW_VACUUM || P.inflow_layout == SMM_INFLOW_ISO_FACE);
}

int ensure_heavy(Problem& P, std::string* err_out) {
    std::string err;
    if (!P.heavy_ready) {
        int rc = setup_geometry(P, err, true);
        if (rc != SMM_OK) {
            if (err_out) *err_out = err;
            return rc;
        }
        P.heavy_ready = true;
    }
    if (!P.graph_ready) {
        int rc = setup_sweep_graph(P, err);
        if (rc != SMM_OK) {
            if (err_out) *err_out = err;
            return rc;
        }
        P.graph_ready = true;
    }
    return SMM_OK;
}

namespace {

using Key = std::array<double, 7>;  // sigma_t, sigma_s, boundary bits, sigma_t of the 4 neighbours

Key self_key(const Problem& P, int K) {
    Key k{};
    k[0] = P.sigma_t[K];
    k[1] = P.sigma_s[K];
    int bits = 0;
    for (int f = 0; f < 4; ++f) {
        const int N = P.nbr[K * 4 + f];
        if (N < 0) bits |= 1 << f;
        k[3 + f] = N < 0 ? 0.0 : P.sigma_t[N];
    }
    k[2] = bits;
    return k;
}

// Assemble the general operators on the patch around element (i, j) and copy
// out the blocks of the patch element that stands for it.
int patch_blocks(const Problem& P, int i, int j, std::vector<double>& ip_self, std::vector<double>& dinv,
                 std::vector<double>& c_self, std::vector<double> ip_nbr[4], std::vector<double> c_nbr[4],
                 std::string& err) {
    const int px = std::min(P.nx, 3), py = std::min(P.ny, 3);
    const int ip = (i == 0) ? 0 : (i == P.nx - 1 ? px - 1 : 1);
    const int jp = (j == 0) ? 0 : (j == P.ny - 1 ? py - 1 : 1);
    Problem Q;
    Q.ctx = P.ctx;
    Q.nx = px;
    Q.ny = py;
    Q.m = P.m;
    Q.p = P.p;
    Q.nb = P.nb;
    Q.n = P.n;
    Q.nq = P.nq;
    Q.ne = px * py;
    Q.sn = P.sn;
    Q.kappa_scale = P.kappa_scale;
    Q.omega = P.omega;
    Q.w = P.w;
    Q.nd = P.nd;
    std::vector<double> cgl;
    gauss_lobatto01(P.m, cgl);
    const int ncx = px * P.m + 1, ncy = py * P.m + 1;
    Q.ctrl.assign((size_t)ncx * ncy * 2, 0.0);
    for (int b = 0; b < ncy; ++b)
        for (int a = 0; a < ncx; ++a) {
            const int ia = std::min(a / P.m, px - 1), ib = std::min(b / P.m, py - 1);
            const int la = a - ia * P.m, lb = b - ib * P.m;
            Q.ctrl[((size_t)b * ncx + a) * 2 + 0] = (ia + cgl[la]) * P.hx;
            Q.ctrl[((size_t)b * ncx + a) * 2 + 1] = (ib + cgl[lb]) * P.hy;
        }
    Q.sigma_t.assign(Q.ne, 1.0);
    Q.sigma_s.assign(Q.ne, 0.0);
    for (int qj = 0; qj < py; ++qj)
        for (int qi = 0; qi < px; ++qi) {
            const int K = (j + qj - jp) * P.nx + (i + qi - ip);
            Q.sigma_t[qj * px + qi] = P.sigma_t[K];
            Q.sigma_s[qj * px + qi] = P.sigma_s[K];
        }
    Q.have_mat = true;
    int rc = setup_geometry(Q, err, true);
    if (rc != SMM_OK) return rc;
    assemble_ip(Q);
    assemble_correction_operator(Q);
    const int n = P.n, Kc = jp * px + ip;
    ip_self.assign(&Q.bsr_val[(size_t)Kc * 5 * n * n], &Q.bsr_val[(size_t)Kc * 5 * n * n] + n * n);
    dinv.assign(&Q.bjac_inv[(size_t)Kc * n * n], &Q.bjac_inv[(size_t)Kc * n * n] + n * n);
    c_self.assign(&Q.corr_val[(size_t)Kc * 5 * n * 3 * n], &Q.corr_val[(size_t)Kc * 5 * n * 3 * n] + 3 * n * n);
    for (int f = 0; f < 4; ++f) {
        if (Q.nbr[Kc * 4 + f] < 0) continue;
        const double* a = &Q.bsr_val[((size_t)Kc * 5 + 1 + f) * n * n];
        ip_nbr[f].assign(a, a + n * n);
        const double* c = &Q.corr_val[((size_t)Kc * 5 + 1 + f) * n * 3 * n];
        c_nbr[f].assign(c, c + 3 * n * n);
    }
    return SMM_OK;
}

}  // namespace

int build_typed_blocks(Problem& P, std::string& err) {
    const int n = P.n, nq = P.nq, nb = P.nb;
    std::map<Key, int> selfs;
    std::map<std::array<double, 3>, int> nbrs;
    P.sid.assign(P.ne, -1);
    P.nid.assign((size_t)P.ne * 4, -1);
    P.t_ip_self.clear();
    P.t_dinv.clear();
    P.t_c_self.clear();
    P.t_ip_nbr.clear();
    P.t_c_nbr.clear();
    std::vector<double> ips, dv, cs, ipn[4], cn[4];
    for (int j = 0; j < P.ny; ++j)
        for (int i = 0; i < P.nx; ++i) {
            const int K = j * P.nx + i;
            const Key k = self_key(P, K);
            auto it = selfs.find(k);
            if (it != selfs.end()) {
                P.sid[K] = it->second;
            } else {
                int rc = patch_blocks(P, i, j, ips, dv, cs, ipn, cn, err);
                if (rc != SMM_OK) return rc;
                const int id = (int)selfs.size();
                selfs[k] = id;
                P.sid[K] = id;
                P.t_ip_self.insert(P.t_ip_self.end(), ips.begin(), ips.end());
                P.t_dinv.insert(P.t_dinv.end(), dv.begin(), dv.end());
                P.t_c_self.insert(P.t_c_self.end(), cs.begin(), cs.end());
                for (int f = 0; f < 4; ++f) {
                    const int N = P.nbr[K * 4 + f];
                    if (N < 0) continue;
                    const std::array<double, 3> nk{(double)f, P.sigma_t[K], P.sigma_t[N]};
                    if (nbrs.find(nk) == nbrs.end()) {
                        const int nid = (int)nbrs.size();
                        nbrs[nk] = nid;
                        P.t_ip_nbr.insert(P.t_ip_nbr.end(), ipn[f].begin(), ipn[f].end());
                        P.t_c_nbr.insert(P.t_c_nbr.end(), cn[f].begin(), cn[f].end());
                    }
                }
            }
            for (int f = 0; f < 4; ++f) {
                const int N = P.nbr[K * 4 + f];
                if (N < 0) continue;
                P.nid[(size_t)K * 4 + f] = nbrs.at({(double)f, P.sigma_t[K], P.sigma_t[N]});
            }
        }
    P.nself = (int)selfs.size();
    P.nnbrt = (int)nbrs.size();
    // boundary-factor operator per face orientation: dsw_q u_i(q) (faces of one
    // orientation have identical length elements on a uniform mesh)
    P.t_bop.assign((size_t)4 * n * nq, 0.0);
    for (int f = 0; f < 4; ++f) {
        const double hpar = (f == 0 || f == 2) ? P.hx : P.hy;
        for (int c = 0; c < nb; ++c) {
            int k;
            switch (f) {
                case 0: k = c; break;
                case 1: k = (nb - 1) + nb * c; break;
                case 2: k = c + nb * (nb - 1); break;
                default: k = nb * c; break;
            }
            for (int q = 0; q < nq; ++q) P.t_bop[((size_t)f * n + k) * nq + q] = P.wq[q] * hpar * P.Lf[c * nq + q];
        }
    }
    // fixed right-hand side: (sum w) M q - 2 int_{Gamma_b} u J_in
    double sw = 0;
    for (double wd : P.w) sw += wd;
    std::vector<double> M1((size_t)nb * nb, 0.0);
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
            for (int q = 0; q < nq; ++q) M1[a * nb + b] += P.wq[q] * P.Lf[a * nq + q] * P.Lf[b * nq + q];
    P.t_bfix.assign((size_t)P.ne * n, 0.0);
    for (int K = 0; K < P.ne; ++K) {
        const double* qk = &P.q[(size_t)K * n];
        double* bk = &P.t_bfix[(size_t)K * n];
        for (int b = 0; b < nb; ++b)
            for (int a = 0; a < nb; ++a) {
                double s = 0;
                for (int b2 = 0; b2 < nb; ++b2)
                    for (int a2 = 0; a2 < nb; ++a2) s += M1[a * nb + a2] * M1[b * nb + b2] * qk[a2 + nb * b2];
                bk[a + nb * b] = sw * P.hx * P.hy * s;
            }
        if (P.inflow_layout == SMM_INFLOW_ISO_FACE) {
            for (int f = 0; f < 4; ++f) {
                const int bf = P.bface_of[K * 4 + f];
                if (bf < 0) continue;
                const double nx_ = (f == 1) ? 1.0 : (f == 3 ? -1.0 : 0.0);
                const double ny_ = (f == 2) ? 1.0 : (f == 0 ? -1.0 : 0.0);
                for (int q = 0; q < nq; ++q) {
                    double jin = 0;
                    for (int d = 0; d < P.nd; ++d) {
                        const double on = P.omega[d * 3] * nx_ + P.omega[d * 3 + 1] * ny_;
                        if (on < 0.0) jin += P.w[d] * on * P.psibar[((size_t)bf * nq + q) * P.nd + d];
                    }
                    for (int i = 0; i < n; ++i) bk[i] -= 2.0 * P.t_bop[((size_t)f * n + i) * nq + q] * jin;
                }
            }
        }
    }
    P.typed_ready = true;
    return SMM_OK;
}

}  // namespace smm
