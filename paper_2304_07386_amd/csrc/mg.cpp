// Two-level preconditioner for the typed moment system: host set-up.
//
// The coarse space is the continuous bilinear (Q1) space on the element
// vertices of the uniform Cartesian mesh, embedded into the DG space by
// interpolation at the Gauss-Lobatto nodes (P0).  Its operator is the Galerkin
// product P0^T A P0.  For continuous functions every face jump vanishes, so
// this is a 9-point stencil on the vertex grid; the entries the algebra
// produces farther out are zero up to rounding and are checked and dropped.
// Coarser vertex grids take every other vertex (the last one always kept),
// with 1D linear interpolation (weights 1, 1/2) in each direction and Galerkin
// operators again; a grid of at most 3 x 3 vertices is solved by a dense
// inverse.
#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "mg_internal.hpp"
#include "smm_internal.hpp"

namespace smm {

namespace {

// parents of fine vertex i on a 1D grid of nf vertices: (c0, w0, c1, w1), c1 = -1 if one
struct Par {
    int c0;
    double w0;
    int c1;
    double w1;
};

int coarse_count(int nf) { return nf <= 3 ? nf : (nf - 1 + 1) / 2 + 1; }

Par parents(int i, int nf) {
    if (nf <= 3) return {i, 1.0, -1, 0.0};
    const int nc = coarse_count(nf);
    if (i == nf - 1) return {nc - 1, 1.0, -1, 0.0};
    if (i % 2 == 0) return {i / 2, 1.0, -1, 0.0};
    return {(i - 1) / 2, 0.5, (i + 1) / 2, 0.5};
}

bool invert(std::vector<double> a, int n, std::vector<double>& inv) {
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
        if (!(std::fabs(a[(size_t)piv * n + c]) > 0)) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)c * n + k], a[(size_t)piv * n + k]);
                std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
            }
        const double d = a[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            a[(size_t)c * n + k] /= d;
            inv[(size_t)c * n + k] /= d;
        }
        for (int r = 0; r < n; ++r)
            if (r != c) {
                const double f = a[(size_t)r * n + c];
                if (f == 0) continue;
                for (int k = 0; k < n; ++k) {
                    a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
                    inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
                }
            }
    }
    return true;
}

}  // namespace

int mg_coarse_count(int nf) { return coarse_count(nf); }

// Level 0 from the 5 x 5 vertex windows W[v][25] of the Galerkin product, then
// the coarser levels and the dense inverse of the coarsest one.
static int finish_mg(MGHost& M, int vx, int vy, const std::vector<double>& W, std::string& err);

int build_mg(const Problem& P, MGHost& M, std::string& err) {
    const int nb = P.nb, n = P.n, nx = P.nx, ny = P.ny;
    std::vector<double> x1;
    gauss_lobatto01(P.p, x1);
    M.gll = x1;
    // P_loc[node][corner], node = a + nb b, corner = cx + 2 cy
    std::vector<double> Ploc((size_t)n * 4);
    for (int b = 0; b < nb; ++b)
        for (int a = 0; a < nb; ++a)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx)
                    Ploc[(size_t)(a + nb * b) * 4 + cx + 2 * cy] =
                        (cx ? x1[a] : 1.0 - x1[a]) * (cy ? x1[b] : 1.0 - x1[b]);
    // 4x4 reductions of the typed blocks (row-major [type][n][n] on the host)
    auto reduce = [&](const double* A, double* S) {
        for (int v = 0; v < 4; ++v)
            for (int w = 0; w < 4; ++w) {
                double s = 0;
                for (int i = 0; i < n; ++i) {
                    const double pi = Ploc[(size_t)i * 4 + v];
                    if (pi == 0) continue;
                    double t = 0;
                    for (int j = 0; j < n; ++j) t += A[(size_t)i * n + j] * Ploc[(size_t)j * 4 + w];
                    s += pi * t;
                }
                S[v * 4 + w] = s;
            }
    };
    std::vector<double> Ss((size_t)P.nself * 16), Sn((size_t)std::max(P.nnbrt, 1) * 16);
    for (int s = 0; s < P.nself; ++s) reduce(&P.t_ip_self[(size_t)s * n * n], &Ss[(size_t)s * 16]);
    for (int t = 0; t < P.nnbrt; ++t) reduce(&P.t_ip_nbr[(size_t)t * n * n], &Sn[(size_t)t * 16]);
    // level 0: vertex grid (nx+1) x (ny+1), stencils from a 5x5 window
    const int vx = nx + 1, vy = ny + 1;
    std::vector<double> W((size_t)vx * vy * 25, 0.0);
    auto add = [&](int v, int w, double a) {
        const int ix = v % vx, iy = v / vx, jx = w % vx, jy = w / vx;
        const int dx = jx - ix, dy = jy - iy;
        W[(size_t)v * 25 + (dy + 2) * 5 + (dx + 2)] += a;
    };
    auto gvert = [&](int K, int c) { return (K / nx + (c >> 1)) * vx + K % nx + (c & 1); };
    const int dK[4] = {-nx, 1, nx, -1};
    for (int K = 0; K < P.ne; ++K) {
        const double* S = &Ss[(size_t)P.sid[K] * 16];
        for (int v = 0; v < 4; ++v)
            for (int w = 0; w < 4; ++w) add(gvert(K, v), gvert(K, w), S[v * 4 + w]);
        for (int f = 0; f < 4; ++f) {
            const int t = P.nid[4 * K + f];
            if (t < 0) continue;
            const int N = K + dK[f];
            const double* T = &Sn[(size_t)t * 16];
            for (int v = 0; v < 4; ++v)
                for (int w = 0; w < 4; ++w) add(gvert(K, v), gvert(N, w), T[v * 4 + w]);
        }
    }
    return finish_mg(M, vx, vy, W, err);
}

int build_mg_cg(const Problem& P, MGHost& M, std::string& err) {
    // the continuous system has no face terms: each element couples only its
    // own four vertices, through P_loc^T A_K P_loc of its volume and boundary
    // block (the block the continuous assembly sums)
    const int nb = P.nb, n = P.n, nx = P.nx, ny = P.ny;
    std::vector<double> x1;
    gauss_lobatto01(P.p, x1);
    M.gll = x1;
    std::vector<double> Ploc((size_t)n * 4);
    for (int b = 0; b < nb; ++b)
        for (int a = 0; a < nb; ++a)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx)
                    Ploc[(size_t)(a + nb * b) * 4 + cx + 2 * cy] =
                        (cx ? x1[a] : 1.0 - x1[a]) * (cy ? x1[b] : 1.0 - x1[b]);
    const int vx = nx + 1, vy = ny + 1;
    std::vector<double> W((size_t)vx * vy * 25, 0.0);
    std::vector<double> blk((size_t)n * n);
    for (int K = 0; K < P.ne; ++K) {
        std::fill(blk.begin(), blk.end(), 0.0);
        add_volume_block(P, K, blk.data());
        for (int f = 0; f < 4; ++f)
            if (P.nbr[K * 4 + f] < 0) add_boundary_block(P, K, f, blk.data());
        const int ex = K % nx, ey = K / nx;
        for (int v = 0; v < 4; ++v)
            for (int w = 0; w < 4; ++w) {
                double s = 0;
                for (int i = 0; i < n; ++i) {
                    const double pi = Ploc[(size_t)i * 4 + v];
                    if (pi == 0) continue;
                    double t = 0;
                    for (int j = 0; j < n; ++j) t += blk[(size_t)i * n + j] * Ploc[(size_t)j * 4 + w];
                    s += pi * t;
                }
                const int iv = (ey + (v >> 1)) * vx + ex + (v & 1);
                const int dx = (w & 1) - (v & 1), dy = (w >> 1) - (v >> 1);
                W[(size_t)iv * 25 + (dy + 2) * 5 + (dx + 2)] += s;
            }
    }
    return finish_mg(M, vx, vy, W, err);
}

static int finish_mg(MGHost& M, int vx, int vy, const std::vector<double>& W, std::string& err) {
    MGLevelHost L0;
    L0.nvx = vx;
    L0.nvy = vy;
    L0.A.assign((size_t)9 * vx * vy, 0.0);
    double amax = 0, outside = 0;
    for (int v = 0; v < vx * vy; ++v)
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                const double a = W[(size_t)v * 25 + (dy + 2) * 5 + dx + 2];
                if (std::abs(dx) <= 1 && std::abs(dy) <= 1) {
                    L0.A[(size_t)((dy + 1) * 3 + dx + 1) * vx * vy + v] = a;
                    amax = std::max(amax, std::fabs(a));
                } else {
                    outside = std::max(outside, std::fabs(a));
                }
            }
    if (!(outside <= 1e-9 * amax)) {
        err = "coarse operator is not a 9-point stencil (" + std::to_string(outside / amax) + ")";
        return SMM_EHIP;
    }
    M.lev.clear();
    M.lev.push_back(std::move(L0));
    // coarser levels
    while (M.lev.back().nvx > 3 || M.lev.back().nvy > 3) {
        const MGLevelHost& F = M.lev.back();
        MGLevelHost C;
        C.nvx = coarse_count(F.nvx);
        C.nvy = coarse_count(F.nvy);
        const int nvf = F.nvx * F.nvy, nvc = C.nvx * C.nvy;
        C.A.assign((size_t)9 * nvc, 0.0);
        for (int fy = 0; fy < F.nvy; ++fy)
            for (int fx = 0; fx < F.nvx; ++fx) {
                const int f = fy * F.nvx + fx;
                const Par px = parents(fx, F.nvx), py = parents(fy, F.nvy);
                for (int k = 0; k < 9; ++k) {
                    const double a = F.A[(size_t)k * nvf + f];
                    if (a == 0) continue;
                    const int gx = fx + k % 3 - 1, gy = fy + k / 3 - 1;
                    if (gx < 0 || gy < 0 || gx >= F.nvx || gy >= F.nvy) continue;
                    const Par qx = parents(gx, F.nvx), qy = parents(gy, F.nvy);
                    const int pcx[2] = {px.c0, px.c1}, pcy[2] = {py.c0, py.c1};
                    const double pwx[2] = {px.w0, px.w1}, pwy[2] = {py.w0, py.w1};
                    const int qcx[2] = {qx.c0, qx.c1}, qcy[2] = {qy.c0, qy.c1};
                    const double qwx[2] = {qx.w0, qx.w1}, qwy[2] = {qy.w0, qy.w1};
                    for (int a1 = 0; a1 < 2; ++a1)
                        for (int b1 = 0; b1 < 2; ++b1) {
                            if (pcx[a1] < 0 || pcy[b1] < 0) continue;
                            const int c = pcy[b1] * C.nvx + pcx[a1];
                            const double wc = pwx[a1] * pwy[b1];
                            for (int a2 = 0; a2 < 2; ++a2)
                                for (int b2 = 0; b2 < 2; ++b2) {
                                    if (qcx[a2] < 0 || qcy[b2] < 0) continue;
                                    const int dx = qcx[a2] - pcx[a1], dy = qcy[b2] - pcy[b1];
                                    if (std::abs(dx) > 1 || std::abs(dy) > 1) {
                                        err = "coarse Galerkin product leaves the 9-point stencil";
                                        return SMM_EHIP;
                                    }
                                    C.A[(size_t)((dy + 1) * 3 + dx + 1) * nvc + c] += wc * a * qwx[a2] * qwy[b2];
                                }
                        }
                }
            }
        if (C.nvx == F.nvx && C.nvy == F.nvy) break;  // cannot coarsen further
        M.lev.push_back(std::move(C));
    }
    // dense inverse of the coarsest level
    const MGLevelHost& Lc = M.lev.back();
    const int nc = Lc.nvx * Lc.nvy;
    if (nc > MG_MAX_COARSE) {
        err = "coarsest multigrid level too large";
        return SMM_EUNSUPPORTED;
    }
    std::vector<double> dense((size_t)nc * nc, 0.0);
    for (int v = 0; v < nc; ++v)
        for (int k = 0; k < 9; ++k) {
            const int wx = v % Lc.nvx + k % 3 - 1, wy = v / Lc.nvx + k / 3 - 1;
            if (wx < 0 || wy < 0 || wx >= Lc.nvx || wy >= Lc.nvy) continue;
            dense[(size_t)v * nc + wy * Lc.nvx + wx] += Lc.A[(size_t)k * nc + v];
        }
    if (!invert(dense, nc, M.cinv)) {
        err = "singular coarsest multigrid operator";
        return SMM_EHIP;
    }
    return SMM_OK;
}

}  // namespace smm
