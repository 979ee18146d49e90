// One-time host setup of libsmm: quadrature, bases, element geometry, the
// IP SMM operator (fixed across iterations), the fixed right-hand side, the
// correction-source operator, per-(material, direction) local transport
// operators on Cartesian meshes, and the per-direction sweep graph.
//
// Compiled with -ffp-contract=off so that sign decisions (chord fluxes) are
// reproducible.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <set>
#include <map>

#include "smm_internal.hpp"

namespace smm {

static const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [0,1]: Newton iteration on P_q from the Chebyshev-like
// initial guesses cos(pi (k + 3/4)/(q + 1/2)).
// ---------------------------------------------------------------------------
static void legendre_eval(int n, double x, double& P, double& dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    P = p1;
    dP = n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& w) {
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    for (int k = 0; k < q; ++k) {
        double t = std::cos(kPi * (k + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre_eval(q, t, P, dP);
            double dt = P / dP;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double P, dP;
        legendre_eval(q, t, P, dP);
        // node t in (-1,1) descending in k; map to [0,1] ascending
        x[q - 1 - k] = 0.5 * (t + 1.0);
        w[q - 1 - k] = 1.0 / ((1.0 - t * t) * dP * dP);  // 2/((1-t^2)P'^2) * 1/2
    }
}

// Gauss-Lobatto points: 0, 1 and the roots of P_p' (Newton with
// P_p'' = (2 x P_p' - p(p+1) P_p)/(1 - x^2)), started at -cos(pi k/p).
void gauss_lobatto01(int p, std::vector<double>& x) {
    x.assign(p + 1, 0.0);
    x[0] = 0.0;
    x[p] = 1.0;
    for (int k = 1; k < p; ++k) {
        double t = -std::cos(kPi * k / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre_eval(p, t, P, dP);
            double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
            double dt = dP / d2P;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[k] = 0.5 * (t + 1.0);
    }
    std::sort(x.begin(), x.end());
}

void lagrange_tables(const std::vector<double>& nodes, const std::vector<double>& pts,
                     std::vector<double>& L, std::vector<double>& dL) {
    int nn = (int)nodes.size(), np = (int)pts.size();
    L.assign((size_t)nn * np, 0.0);
    dL.assign((size_t)nn * np, 0.0);
    for (int a = 0; a < nn; ++a) {
        double den = 1.0;
        for (int b = 0; b < nn; ++b)
            if (b != a) den *= (nodes[a] - nodes[b]);
        for (int k = 0; k < np; ++k) {
            double xk = pts[k];
            double v = 1.0;
            for (int b = 0; b < nn; ++b)
                if (b != a) v *= (xk - nodes[b]);
            L[a * np + k] = v / den;
            double s = 0.0;
            for (int b = 0; b < nn; ++b) {
                if (b == a) continue;
                double prod = 1.0;
                for (int c = 0; c < nn; ++c)
                    if (c != a && c != b) prod *= (xk - nodes[c]);
                s += prod;
            }
            dL[a * np + k] = s / den;
        }
    }
}

// Dense Gaussian elimination with partial pivoting: solves A X = B in place
// (A n x n row-major, B n x r row-major); returns 0 on success.
static int dense_solve(int n, double* A, int r, double* B) {
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
        if (A[piv * n + k] == 0.0) return -1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
            for (int j = 0; j < r; ++j) std::swap(B[k * r + j], B[piv * r + j]);
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            if (f == 0.0) continue;
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int j = 0; j < r; ++j) B[i * r + j] -= f * B[k * r + j];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        for (int j = 0; j < r; ++j) {
            double s = B[k * r + j];
            for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * B[c * r + j];
            B[k * r + j] = s / A[k * n + k];
        }
    }
    return 0;
}

int lu_invert(int n, double* A) {
    std::vector<double> a(A, A + (size_t)n * n), I((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
    if (dense_solve(n, a.data(), n, I.data()) != 0) return -1;
    std::memcpy(A, I.data(), sizeof(double) * n * n);
    return 0;
}

// ---------------------------------------------------------------------------
// Level-symmetric S_N.  mu_i^2 = mu_1^2 + (i-1) 2(1-3 mu_1^2)/(N-2); octant
// points (mu_i, mu_j, mu_k), i+j+k = N/2+2; one weight per permutation class
// from sum w = 1, sum w mu^{2k} = 1/(2k+1) (k = 2..#classes).
// ---------------------------------------------------------------------------
int level_symmetric(int N, std::vector<double>& omega, std::vector<double>& w) {
    double mu1;
    switch (N) {
        case 4: mu1 = std::sqrt((4.0 - std::sqrt(6.4)) / 12.0); break;
        case 6: mu1 = 0.2666355; break;
        case 8: mu1 = std::sqrt(1.0 / 21.0); break;
        case 10: mu1 = 0.1893213; break;
        case 12: mu1 = 0.1672126; break;
        default: return -1;
    }
    int h = N / 2;
    double m1s = mu1 * mu1;
    double del = 2.0 * (1.0 - 3.0 * m1s) / (N - 2);
    std::vector<double> mu(h);
    for (int i = 0; i < h; ++i) mu[i] = std::sqrt(m1s + del * i);
    std::vector<int> ii, jj, kk;
    for (int i = 1; i <= h; ++i)
        for (int j = 1; j <= h; ++j) {
            int k = h + 2 - i - j;
            if (k >= 1 && k <= h) { ii.push_back(i); jj.push_back(j); kk.push_back(k); }
        }
    int np = (int)ii.size();
    std::vector<std::array<int, 3>> cls;
    std::vector<int> cid(np);
    {
        std::set<std::array<int, 3>> s;
        for (int t = 0; t < np; ++t) {
            std::array<int, 3> a{ii[t], jj[t], kk[t]};
            std::sort(a.begin(), a.end());
            s.insert(a);
        }
        cls.assign(s.begin(), s.end());
        for (int t = 0; t < np; ++t) {
            std::array<int, 3> a{ii[t], jj[t], kk[t]};
            std::sort(a.begin(), a.end());
            cid[t] = (int)(std::find(cls.begin(), cls.end(), a) - cls.begin());
        }
    }
    int nc = (int)cls.size();
    std::vector<double> A((size_t)nc * nc, 0.0), b(nc, 0.0);
    for (int t = 0; t < np; ++t) A[0 * nc + cid[t]] += 1.0;
    b[0] = 1.0;
    for (int r = 1; r < nc; ++r) {
        int k = r + 1;
        for (int t = 0; t < np; ++t) A[r * nc + cid[t]] += std::pow(mu[ii[t] - 1], 2 * k);
        b[r] = 1.0 / (2 * k + 1);
    }
    if (dense_solve(nc, A.data(), 1, b.data()) != 0) return -1;
    const int sgn[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    omega.clear();
    w.clear();
    for (int qd = 0; qd < 4; ++qd)
        for (int t = 0; t < np; ++t) {
            omega.push_back(sgn[qd][0] * mu[ii[t] - 1]);
            omega.push_back(sgn[qd][1] * mu[jj[t] - 1]);
            omega.push_back(mu[kk[t] - 1]);
            w.push_back(b[cid[t]] * kPi);  // octant sum 1 -> 4 pi over 4 doubled quadrants
        }
    return 0;
}

// ---------------------------------------------------------------------------
// Geometry: element maps, Jacobians, element matrices, face data.
// ---------------------------------------------------------------------------
static inline void ref_face_point(int f, double s, double& xi, double& eta) {
    switch (f) {
        case 0: xi = s; eta = 0.0; break;
        case 1: xi = 1.0; eta = s; break;
        case 2: xi = s; eta = 1.0; break;
        default: xi = 0.0; eta = s; break;
    }
}

int setup_geometry(Problem& P, std::string& err, bool heavy) {
    const int nb = P.nb, n = P.n, nq = P.nq, m = P.m;
    const int ne = P.ne;
    const int ncx = P.nx * m + 1;
    gauss_legendre01(nq, P.sq, P.wq);
    gauss_lobatto01(P.p, P.gl);
    std::vector<double> cgl;
    gauss_lobatto01(m, cgl);
    lagrange_tables(P.gl, P.sq, P.Lf, P.dLf);
    // tables: solution basis at Gauss points and at {0,1}; geometry basis likewise
    std::vector<double> Ls, dLs, Lsb, dLsb, Lg, dLg, Lgb, dLgb, Lgn, dLgn;
    std::vector<double> ends = {0.0, 1.0};
    lagrange_tables(P.gl, P.sq, Ls, dLs);
    lagrange_tables(P.gl, ends, Lsb, dLsb);
    lagrange_tables(cgl, P.sq, Lg, dLg);
    lagrange_tables(cgl, ends, Lgb, dLgb);
    lagrange_tables(cgl, P.gl, Lgn, dLgn);

    P.xnode.assign((size_t)ne * n * 2, 0.0);
    P.area.assign(ne, 0.0);
    P.Mk.assign(heavy ? (size_t)ne * n * n : 0, 0.0);
    P.Gxk.assign(heavy ? (size_t)ne * n * n : 0, 0.0);
    P.Gyk.assign(heavy ? (size_t)ne * n * n : 0, 0.0);
    P.nds.assign((size_t)ne * 4 * nq * 2, 0.0);
    P.dsw.assign((size_t)ne * 4 * nq, 0.0);
    P.nhat.assign((size_t)ne * 4 * nq * 2, 0.0);
    P.xf.assign((size_t)ne * 4 * nq * 2, 0.0);
    const int Q = nq * nq;
    P.vol_wJ.assign((size_t)ne * Q, 0.0);
    P.vol_grad.assign(heavy ? (size_t)ne * Q * n * 2 : 0, 0.0);
    P.face_grad.assign(heavy ? (size_t)ne * 4 * nq * n * 2 : 0, 0.0);
    P.vol_U.assign((size_t)Q * n, 0.0);
    P.nbr.assign((size_t)ne * 4, -1);
    P.chord.assign((size_t)ne * 4 * 2, 0.0);

    for (int qb = 0; qb < nq; ++qb)
        for (int qa = 0; qa < nq; ++qa)
            for (int b = 0; b < nb; ++b)
                for (int a = 0; a < nb; ++a)
                    P.vol_U[(qa + nq * qb) * n + a + nb * b] = Ls[a * nq + qa] * Ls[b * nq + qb];

    std::vector<double> X((size_t)(m + 1) * (m + 1) * 2);
    bool cart = true;
    double hx0 = 0, hy0 = 0;

    if (P.general) cart = false;  // the Cartesian kernels index a structured grid
    for (int j = 0; j < P.ny; ++j)
        for (int i = 0; i < P.nx; ++i) {
            const int K = j * P.nx + i;
            if (P.general) {
                std::copy(&P.ctrl_e[(size_t)K * (m + 1) * (m + 1) * 2],
                          &P.ctrl_e[(size_t)(K + 1) * (m + 1) * (m + 1) * 2], X.begin());
            } else {
                for (int b = 0; b <= m; ++b)
                    for (int a = 0; a <= m; ++a) {
                        const double* c = &P.ctrl[((size_t)(j * m + b) * ncx + (i * m + a)) * 2];
                        X[(a + (m + 1) * b) * 2 + 0] = c[0];
                        X[(a + (m + 1) * b) * 2 + 1] = c[1];
                    }
            }
            // generic evaluator: geometry at (xi, eta) from 1D tables
            auto eval = [&](const double* la, const double* dla, const double* lb, const double* dlb,
                            int sa, int sb, double out[6]) {
                // la[a*sa], lb[b*sb] give l_a(xi), l_b(eta) for a, b = 0..m
                double x = 0, y = 0, xxi = 0, yxi = 0, xeta = 0, yeta = 0;
                for (int b = 0; b <= m; ++b)
                    for (int a = 0; a <= m; ++a) {
                        const double cx = X[(a + (m + 1) * b) * 2], cy = X[(a + (m + 1) * b) * 2 + 1];
                        const double va = la[a * sa], vb = lb[b * sb];
                        const double da = dla[a * sa], db = dlb[b * sb];
                        x += cx * va * vb;
                        y += cy * va * vb;
                        xxi += cx * da * vb;
                        yxi += cy * da * vb;
                        xeta += cx * va * db;
                        yeta += cy * va * db;
                    }
                out[0] = x; out[1] = y; out[2] = xxi; out[3] = yxi; out[4] = xeta; out[5] = yeta;
            };
            // nodes
            for (int b = 0; b < nb; ++b)
                for (int a = 0; a < nb; ++a) {
                    double g[6];
                    eval(&Lgn[a], &dLgn[a], &Lgn[b], &dLgn[b], nb, nb, g);
                    P.xnode[((size_t)K * n + a + nb * b) * 2 + 0] = g[0];
                    P.xnode[((size_t)K * n + a + nb * b) * 2 + 1] = g[1];
                }
            // volume points
            double areaK = 0.0;
            for (int qb = 0; qb < nq; ++qb)
                for (int qa = 0; qa < nq; ++qa) {
                    double g[6];
                    eval(&Lg[qa], &dLg[qa], &Lg[qb], &dLg[qb], nq, nq, g);
                    const double det = g[2] * g[5] - g[4] * g[3];
                    if (!(det > 0.0)) {
                        err = "element " + std::to_string(K) + " has non-positive Jacobian";
                        return SMM_EINVAL;
                    }
                    const int Qi = qa + nq * qb;
                    const double wJ = P.wq[qa] * P.wq[qb] * det;
                    P.vol_wJ[(size_t)K * Q + Qi] = wJ;
                    areaK += wJ;
                    if (!heavy) continue;
                    for (int b = 0; b < nb; ++b)
                        for (int a = 0; a < nb; ++a) {
                            const int k = a + nb * b;
                            const double uxi = dLs[a * nq + qa] * Ls[b * nq + qb];
                            const double ueta = Ls[a * nq + qa] * dLs[b * nq + qb];
                            double* gg = &P.vol_grad[(((size_t)K * Q + Qi) * n + k) * 2];
                            gg[0] = (g[5] * uxi - g[3] * ueta) / det;
                            gg[1] = (-g[4] * uxi + g[2] * ueta) / det;
                        }
                }
            P.area[K] = areaK;
            for (int Qi = 0; heavy && Qi < Q; ++Qi) {
                const double wJ = P.vol_wJ[(size_t)K * Q + Qi];
                for (int r = 0; r < n; ++r) {
                    const double ur = P.vol_U[Qi * n + r];
                    const double* gr = &P.vol_grad[(((size_t)K * Q + Qi) * n + r) * 2];
                    for (int c = 0; c < n; ++c) {
                        const double uc = P.vol_U[Qi * n + c];
                        P.Mk[((size_t)K * n + r) * n + c] += wJ * ur * uc;
                        P.Gxk[((size_t)K * n + r) * n + c] += wJ * gr[0] * uc;
                        P.Gyk[((size_t)K * n + r) * n + c] += wJ * gr[1] * uc;
                    }
                }
            }
            // faces
            for (int f = 0; f < 4; ++f)
                for (int q = 0; q < nq; ++q) {
                    double xi, eta;
                    ref_face_point(f, P.sq[q], xi, eta);
                    // geometry tables at this point
                    const double *la, *dla, *lb, *dlb;
                    int sa, sb;
                    if (f == 0 || f == 2) {
                        la = &Lg[q]; dla = &dLg[q]; sa = nq;
                        lb = &Lgb[f == 0 ? 0 : 1]; dlb = &dLgb[f == 0 ? 0 : 1]; sb = 2;
                    } else {
                        la = &Lgb[f == 3 ? 0 : 1]; dla = &dLgb[f == 3 ? 0 : 1]; sa = 2;
                        lb = &Lg[q]; dlb = &dLg[q]; sb = nq;
                    }
                    double g[6];
                    eval(la, dla, lb, dlb, sa, sb, g);
                    double tx, ty;
                    if (f == 0 || f == 2) { tx = g[2]; ty = g[3]; } else { tx = g[4]; ty = g[5]; }
                    double nx_ = ty, ny_ = -tx;
                    if (f >= 2) { nx_ = -nx_; ny_ = -ny_; }
                    const double ds = std::sqrt(nx_ * nx_ + ny_ * ny_);
                    const size_t fo = ((size_t)K * 4 + f) * nq + q;
                    P.nds[fo * 2 + 0] = P.wq[q] * nx_;
                    P.nds[fo * 2 + 1] = P.wq[q] * ny_;
                    P.dsw[fo] = P.wq[q] * ds;
                    P.nhat[fo * 2 + 0] = nx_ / ds;
                    P.nhat[fo * 2 + 1] = ny_ / ds;
                    P.xf[fo * 2 + 0] = g[0];
                    P.xf[fo * 2 + 1] = g[1];
                    const double det = g[2] * g[5] - g[4] * g[3];
                    if (!heavy) continue;
                    // solution-basis gradients at the face point
                    for (int b = 0; b < nb; ++b)
                        for (int a = 0; a < nb; ++a) {
                            double ua, dua, ub, dub;
                            if (f == 0 || f == 2) {
                                ua = Ls[a * nq + q]; dua = dLs[a * nq + q];
                                ub = Lsb[b * 2 + (f == 0 ? 0 : 1)]; dub = dLsb[b * 2 + (f == 0 ? 0 : 1)];
                            } else {
                                ua = Lsb[a * 2 + (f == 3 ? 0 : 1)]; dua = dLsb[a * 2 + (f == 3 ? 0 : 1)];
                                ub = Ls[b * nq + q]; dub = dLs[b * nq + q];
                            }
                            const double uxi = dua * ub, ueta = ua * dub;
                            double* gg = &P.face_grad[(fo * n + a + nb * b) * 2];
                            gg[0] = (g[5] * uxi - g[3] * ueta) / det;
                            gg[1] = (-g[4] * uxi + g[2] * ueta) / det;
                        }
                }
            // corners and chord normals (exact integrals of n ds)
            double c[4][2];
            const int cidx[4][2] = {{0, 0}, {m, 0}, {m, m}, {0, m}};
            for (int t = 0; t < 4; ++t) {
                c[t][0] = X[(cidx[t][0] + (m + 1) * cidx[t][1]) * 2];
                c[t][1] = X[(cidx[t][0] + (m + 1) * cidx[t][1]) * 2 + 1];
            }
            const int ce[4][2] = {{0, 1}, {1, 2}, {3, 2}, {0, 3}};
            for (int f = 0; f < 4; ++f) {
                const double dx = c[ce[f][1]][0] - c[ce[f][0]][0];
                const double dy = c[ce[f][1]][1] - c[ce[f][0]][1];
                const double s = (f >= 2) ? -1.0 : 1.0;
                P.chord[((size_t)K * 4 + f) * 2 + 0] = s * dy;
                P.chord[((size_t)K * 4 + f) * 2 + 1] = -s * dx;
            }
            // cartesian test: axis-aligned rectangle, affine control points, uniform size
            {
                const double hx = c[1][0] - c[0][0], hy = c[3][1] - c[0][1];
                const double tol = 1e-12 * std::max(std::fabs(hx), std::fabs(hy));
                if (std::fabs(c[1][1] - c[0][1]) > tol || std::fabs(c[2][0] - c[1][0]) > tol ||
                    std::fabs(c[3][0] - c[0][0]) > tol || std::fabs(c[2][1] - c[3][1]) > tol)
                    cart = false;
                for (int b = 0; b <= m && cart; ++b)
                    for (int a = 0; a <= m; ++a) {
                        const double ex = c[0][0] + cgl[a] * hx, ey = c[0][1] + cgl[b] * hy;
                        if (std::fabs(X[(a + (m + 1) * b) * 2] - ex) > tol ||
                            std::fabs(X[(a + (m + 1) * b) * 2 + 1] - ey) > tol) { cart = false; break; }
                    }
                if (K == 0) { hx0 = hx; hy0 = hy; }
                else if (std::fabs(hx - hx0) > 1e-12 * hx0 || std::fabs(hy - hy0) > 1e-12 * hy0)
                    cart = false;
            }
            if (P.general) {
                for (int f = 0; f < 4; ++f) P.nbr[K * 4 + f] = P.nbr_in[(size_t)K * 4 + f];
            } else {
                if (j > 0) P.nbr[K * 4 + 0] = K - P.nx;
                if (i < P.nx - 1) P.nbr[K * 4 + 1] = K + 1;
                if (j < P.ny - 1) P.nbr[K * 4 + 2] = K + P.nx;
                if (i > 0) P.nbr[K * 4 + 3] = K - 1;
            }
        }
    // interior faces: the neighbour's face across f and whether the two
    // parameterisations run the same way, from the face control points (a
    // structured grid: always the opposite face, the same way)
    P.nbr_face.assign((size_t)ne * 4, -1);
    {
        double amax = 0;
        for (int K = 0; K < ne; ++K) amax = std::max(amax, P.area[K]);
        const double tol = 1e-10 * std::sqrt(amax);
        const int mm = m + 1;
        auto fctrl = [&](int K, int f, int t) -> const double* {   // control point t along face f
            int a, b;
            switch (f) {
                case 0: a = t; b = 0; break;
                case 1: a = m; b = t; break;
                case 2: a = t; b = m; break;
                default: a = 0; b = t; break;
            }
            const double* base = P.general ? &P.ctrl_e[(size_t)K * mm * mm * 2] : nullptr;
            if (base) return base + (a + mm * b) * 2;
            const int i = K % P.nx, j = K / P.nx;
            return &P.ctrl[((size_t)(j * m + b) * ncx + (i * m + a)) * 2];
        };
        for (int K = 0; K < ne; ++K)
            for (int f = 0; f < 4; ++f) {
                const int N = P.nbr[K * 4 + f];
                if (N < 0) continue;
                if (N >= ne || N == K) {
                    err = "element " + std::to_string(K) + " face " + std::to_string(f) + ": bad neighbour";
                    return SMM_EINVAL;
                }
                int code = -1;
                for (int g = 0; g < 4 && code < 0; ++g) {
                    if (P.nbr[N * 4 + g] != K) continue;
                    bool same = true, rev = true;
                    for (int t = 0; t <= m; ++t) {
                        const double* a = fctrl(K, f, t);
                        const double* b = fctrl(N, g, t);
                        const double* br = fctrl(N, g, m - t);
                        same = same && std::fabs(a[0] - b[0]) <= tol && std::fabs(a[1] - b[1]) <= tol;
                        rev = rev && std::fabs(a[0] - br[0]) <= tol && std::fabs(a[1] - br[1]) <= tol;
                    }
                    if (same) code = g;
                    else if (rev) code = g | 4;
                }
                if (code < 0) {
                    err = "element " + std::to_string(K) + " face " + std::to_string(f) +
                          " does not match a face of its neighbour " + std::to_string(N);
                    return SMM_EINVAL;
                }
                P.nbr_face[K * 4 + f] = code;
            }
    }
    // boundary faces, ordered by element then local face, with their
    // attributes; E_b0 at every boundary point (eq. eb0_disc: it depends on
    // the normal), and whether all boundary normals are axis-aligned
    P.bface_of.assign((size_t)ne * 4, -1);
    P.bface_K.clear();
    P.bface_f.clear();
    P.bface_attr.clear();
    P.axis_bdr = true;
    P.n_bdr_attr = 0;
    for (int K = 0; K < ne; ++K)
        for (int f = 0; f < 4; ++f)
            if (P.nbr[K * 4 + f] < 0) {
                P.bface_of[K * 4 + f] = (int)P.bface_K.size();
                P.bface_K.push_back(K);
                P.bface_f.push_back(f);
                const int attr = P.general && !P.bdr_attr_in.empty() ? P.bdr_attr_in[(size_t)K * 4 + f] : f;
                if (attr < 0) {
                    err = "element " + std::to_string(K) + " face " + std::to_string(f) + ": negative boundary attribute";
                    return SMM_EINVAL;
                }
                P.bface_attr.push_back(attr);
                P.n_bdr_attr = std::max(P.n_bdr_attr, attr + 1);
                for (int q = 0; q < nq; ++q) {
                    const double* nh = &P.nhat[(((size_t)K * 4 + f) * nq + q) * 2];
                    const double off = (f == 0 || f == 2) ? nh[0] : nh[1];
                    if (std::fabs(off) > 1e-10) P.axis_bdr = false;
                }
            }
    P.nbf = (int)P.bface_K.size();
    P.eb0_pt.assign((size_t)P.nbf * nq, 0.0);
    {
        double sw = 0;
        for (int d = 0; d < P.nd; ++d) sw += P.w[d];
        for (int bf = 0; bf < P.nbf; ++bf)
            for (int q = 0; q < nq; ++q) {
                const double* nh = &P.nhat[(((size_t)P.bface_K[bf] * 4 + P.bface_f[bf]) * nq + q) * 2];
                double se = 0;
                for (int d = 0; d < P.nd; ++d)
                    se += P.w[d] * std::fabs(P.omega[d * 3] * nh[0] + P.omega[d * 3 + 1] * nh[1]);
                P.eb0_pt[(size_t)bf * nq + q] = se / sw;
            }
    }
    if (!P.axis_bdr) cart = false;
    P.cartesian = cart;
    P.hx = hx0;
    P.hy = hy0;
    // E_b0 for x- and y-normal faces (eq. eb0_disc)
    double sw = 0, sx = 0, sy = 0;
    for (int d = 0; d < P.nd; ++d) {
        sw += P.w[d];
        sx += P.w[d] * std::fabs(P.omega[d * 3 + 0]);
        sy += P.w[d] * std::fabs(P.omega[d * 3 + 1]);
    }
    P.eb0x = sx / sw;
    P.eb0y = sy / sw;
    return SMM_OK;
}

// ---------------------------------------------------------------------------
// Cartesian operators.  On a uniform axis-aligned mesh the upwind DG matrix
// A = sigma_t M - Omega_x Gx - Omega_y Gy + (outflow face terms) depends only
// on (sigma_t, direction); with E_x, E_y the inflow-face couplings the element
// solve is psi = A^{-1} M S + A^{-1} E_x t_x + A^{-1} E_y t_y, where t_x, t_y
// are the upwind face traces.  The three products are tabulated per
// (material, direction).
// ---------------------------------------------------------------------------
void setup_cartesian_operators(Problem& P) {
    const int nb = P.nb, n = P.n, nq = P.nq, nd = P.nd;
    std::map<double, int> idx;
    P.mat_of.assign(P.ne, 0);
    P.mat_sigma.clear();
    for (int K = 0; K < P.ne; ++K) {
        auto it = idx.find(P.sigma_t[K]);
        if (it == idx.end()) {
            int id = (int)P.mat_sigma.size();
            idx[P.sigma_t[K]] = id;
            P.mat_sigma.push_back(P.sigma_t[K]);
            P.mat_of[K] = (uint8_t)std::min(id, 255);
        } else {
            P.mat_of[K] = (uint8_t)it->second;
        }
    }
    P.nmat = (int)P.mat_sigma.size();
    if (P.nmat > 256) { P.cartesian = false; return; }
    // 1D reference matrices on [0,1]
    std::vector<double> M1(nb * nb, 0.0), D1(nb * nb, 0.0);
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
            for (int q = 0; q < nq; ++q) {
                M1[a * nb + b] += P.wq[q] * P.Lf[a * nq + q] * P.Lf[b * nq + q];
                D1[a * nb + b] += P.wq[q] * P.dLf[a * nq + q] * P.Lf[b * nq + q];
            }
    const double hx = P.hx, hy = P.hy;
    P.Pm.assign((size_t)P.nmat * nd * n * n, 0.0);
    P.Px.assign((size_t)P.nmat * nd * n * nb, 0.0);
    P.Py.assign((size_t)P.nmat * nd * n * nb, 0.0);
    const int r = n + 2 * nb;
    std::vector<double> A(n * n), B(n * r);
    for (int mt = 0; mt < P.nmat; ++mt)
        for (int d = 0; d < nd; ++d) {
            const double ox = P.omega[d * 3], oy = P.omega[d * 3 + 1], st = P.mat_sigma[mt];
            const int aout = ox > 0 ? nb - 1 : 0, ain = ox > 0 ? 0 : nb - 1;
            const int bout = oy > 0 ? nb - 1 : 0, bin = oy > 0 ? 0 : nb - 1;
            std::fill(A.begin(), A.end(), 0.0);
            std::fill(B.begin(), B.end(), 0.0);
            for (int b = 0; b < nb; ++b)
                for (int a = 0; a < nb; ++a)
                    for (int b2 = 0; b2 < nb; ++b2)
                        for (int a2 = 0; a2 < nb; ++a2) {
                            const int k = a + nb * b, l = a2 + nb * b2;
                            const double Mkl = hx * hy * M1[a * nb + a2] * M1[b * nb + b2];
                            const double Gx = hy * D1[a * nb + a2] * M1[b * nb + b2];
                            const double Gy = hx * M1[a * nb + a2] * D1[b * nb + b2];
                            A[k * n + l] = st * Mkl - ox * Gx - oy * Gy;
                            B[k * r + l] = Mkl;
                        }
            for (int b = 0; b < nb; ++b)
                for (int b2 = 0; b2 < nb; ++b2) {
                    A[(aout + nb * b) * n + (aout + nb * b2)] += std::fabs(ox) * hy * M1[b * nb + b2];
                    B[(ain + nb * b) * r + n + b2] = std::fabs(ox) * hy * M1[b * nb + b2];
                }
            for (int a = 0; a < nb; ++a)
                for (int a2 = 0; a2 < nb; ++a2) {
                    A[(a + nb * bout) * n + (a2 + nb * bout)] += std::fabs(oy) * hx * M1[a * nb + a2];
                    B[(a + nb * bin) * r + n + nb + a2] = std::fabs(oy) * hx * M1[a * nb + a2];
                }
            dense_solve(n, A.data(), r, B.data());
            const size_t o = (size_t)mt * nd + d;
            for (int k = 0; k < n; ++k) {
                for (int l = 0; l < n; ++l) P.Pm[(o * n + k) * n + l] = B[k * r + l];
                for (int c = 0; c < nb; ++c) {
                    P.Px[(o * n + k) * nb + c] = B[k * r + n + c];
                    P.Py[(o * n + k) * nb + c] = B[k * r + n + nb + c];
                }
            }
        }
}

// Boundary inflow as upwind traces: t = M1^{-1} int l(s) psibar(s) ds / ds, the
// L2 projection of the inflow onto P_p of the face, so that E t reproduces the
// inflow integral exactly.  bx[d][j][nb] on the x-inflow side, by[d][i][nb].
void cartesian_boundary_traces(const Problem& P, std::vector<double>& bx, std::vector<double>& by) {
    const int nb = P.nb, nq = P.nq, nd = P.nd;
    bx.assign((size_t)nd * P.ny * nb, 0.0);
    by.assign((size_t)nd * P.nx * nb, 0.0);
    if (P.inflow_layout == SMM_INFLOW_VACUUM) return;
    std::vector<double> M1(nb * nb, 0.0);
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
            for (int q = 0; q < nq; ++q) M1[a * nb + b] += P.wq[q] * P.Lf[a * nq + q] * P.Lf[b * nq + q];
    std::vector<double> Mi = M1;
    lu_invert(nb, Mi.data());
    auto project = [&](int bf, int d, double* out) {
        std::vector<double> rhs(nb, 0.0);
        for (int a = 0; a < nb; ++a)
            for (int q = 0; q < nq; ++q)
                rhs[a] += P.wq[q] * P.Lf[a * nq + q] * P.psibar[((size_t)bf * nq + q) * nd + d];
        for (int a = 0; a < nb; ++a) {
            double s = 0;
            for (int b = 0; b < nb; ++b) s += Mi[a * nb + b] * rhs[b];
            out[a] = s;
        }
    };
    for (int d = 0; d < nd; ++d) {
        const double ox = P.omega[d * 3], oy = P.omega[d * 3 + 1];
        for (int j = 0; j < P.ny; ++j) {
            const int i = ox > 0 ? 0 : P.nx - 1, f = ox > 0 ? 3 : 1;
            project(P.bface_of[(j * P.nx + i) * 4 + f], d, &bx[((size_t)d * P.ny + j) * nb]);
        }
        for (int i = 0; i < P.nx; ++i) {
            const int j = oy > 0 ? 0 : P.ny - 1, f = oy > 0 ? 0 : 2;
            project(P.bface_of[(j * P.nx + i) * 4 + f], d, &by[((size_t)d * P.nx + i) * nb]);
        }
    }
}

// ---------------------------------------------------------------------------
// Sweep graph per direction: edge N -> K across face f of K when the chord
// flux Omega . int_f n_K ds < 0; levels = longest path (Kahn's algorithm).
// ---------------------------------------------------------------------------
// Per direction, the upwind element graph from the chord normals and its
// levels by Kahn's algorithm.  With tiles (the parallel block Jacobi sweep of
// Sec. 6.5) only faces inside a tile are edges; inflow across a tile face is
// the previous sweep's.  Level lists per (direction, tile): lev_ptr holds the
// offsets into the direction's element list, which is ordered by tile, then
// level, then element.  Kahn's algorithm must reach every element: a cycle
// (possible only when some chord quadrilateral is not convex) leaves the
// elements on it and downstream of it unvisited, and the sweep could not
// order them, so the problem is refused (SMM_EUNSUPPORTED) rather than swept
// with a same-level read of a neighbour still being written.
int setup_sweep_graph(Problem& P, std::string& err) {
    const int ne = P.ne, nd = P.nd;
    const int tx = P.tile_x > 0 ? P.tile_x : P.nx, ty = P.tile_y > 0 ? P.tile_y : P.ny;
    const int ntx = (P.nx + tx - 1) / tx, nty = (P.ny + ty - 1) / ty;
    P.ntiles = ntx * nty;
    std::vector<int> tile(ne);
    for (int K = 0; K < ne; ++K) tile[K] = (K % P.nx) / tx + ((K / P.nx) / ty) * ntx;
    auto edge = [&](int K, int f) {
        const int N = P.nbr[K * 4 + f];
        return N >= 0 && tile[N] == tile[K];
    };
    P.upflag.assign((size_t)nd * ne, 0);
    P.nlev_max = 0;
    std::vector<int> level(ne), indeg(ne);
    std::vector<std::vector<int>> lev_of(nd);
    for (int d = 0; d < nd; ++d) {
        const double ox = P.omega[d * 3], oy = P.omega[d * 3 + 1];
        for (int K = 0; K < ne; ++K) {
            uint8_t bits = 0;
            for (int f = 0; f < 4; ++f) {
                if (!edge(K, f)) continue;
                const double fl = ox * P.chord[(K * 4 + f) * 2] + oy * P.chord[(K * 4 + f) * 2 + 1];
                if (fl < 0.0) bits |= (uint8_t)(1u << f);
            }
            P.upflag[(size_t)d * ne + K] = bits;
            indeg[K] = __builtin_popcount(bits);
            level[K] = 0;
        }
        std::vector<int> frontier, next;
        for (int K = 0; K < ne; ++K)
            if (indeg[K] == 0) frontier.push_back(K);
        int visited = 0;
        while (!frontier.empty()) {
            next.clear();
            visited += (int)frontier.size();
            for (int K : frontier)
                for (int f = 0; f < 4; ++f) {
                    if (!edge(K, f)) continue;
                    const int N = P.nbr[K * 4 + f];
                    const double fl = ox * P.chord[(K * 4 + f) * 2] + oy * P.chord[(K * 4 + f) * 2 + 1];
                    if (fl > 0.0) {
                        level[N] = std::max(level[N], level[K] + 1);
                        if (--indeg[N] == 0) next.push_back(N);
                    }
                }
            std::sort(next.begin(), next.end());
            frontier.swap(next);
        }
        if (visited != ne) {
            P.upflag.clear();
            err = "the upwind graph of direction " + std::to_string(d) + " has a cycle (" +
                  std::to_string(ne - visited) + " elements unordered): a chord quadrilateral is not convex";
            return SMM_EUNSUPPORTED;
        }
        for (int K = 0; K < ne; ++K) P.nlev_max = std::max(P.nlev_max, level[K] + 1);
        lev_of[d] = level;
    }
    const int nl = P.nlev_max, nt = P.ntiles;
    P.lev_ptr.assign((size_t)nd * nt * (nl + 1), 0);
    P.lev_elem.assign((size_t)nd * ne, 0);
    std::vector<int> cnt((size_t)nt * nl);
    P.lev_wmax = 0;
    for (int d = 0; d < nd; ++d) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int K = 0; K < ne; ++K) ++cnt[(size_t)tile[K] * nl + lev_of[d][K]];
        for (int c : cnt) P.lev_wmax = std::max(P.lev_wmax, c);
        int pos = 0;
        std::vector<int> start((size_t)nt * nl);
        for (int t = 0; t < nt; ++t)
            for (int l = 0; l <= nl; ++l) {
                P.lev_ptr[((size_t)d * nt + t) * (nl + 1) + l] = pos;
                if (l < nl) {
                    start[(size_t)t * nl + l] = pos;
                    pos += cnt[(size_t)t * nl + l];
                }
            }
        for (int K = 0; K < ne; ++K) {
            int& at = start[(size_t)tile[K] * nl + lev_of[d][K]];
            P.lev_elem[(size_t)d * ne + at++] = K;
        }
    }
    return SMM_OK;
}

// ---------------------------------------------------------------------------
// IP SMM left-hand side (eq. ipsmm), block-sparse rows: slot 0 the element,
// slot 1+f its neighbour across face f.  n_K below is the outward normal of K.
//   volume:   D grad u_i . grad u_j + sigma_a u_i u_j
//   boundary: E_b0 u_i u_j
//   interior (self):  kappa u_i u_j - D_K/2 u_i dn u_j - D_K/2 dn u_i u_j
//   interior (nbr):  -kappa u_i v_j - D_N/2 u_i dn v_j + D_K/2 dn u_i v_j
// ---------------------------------------------------------------------------

static void face_values(const Problem& P, int f, int q, std::vector<double>& u) {
    // basis values at face point q of face f (only face nodes are non-zero)
    const int nb = P.nb, nq = P.nq;
    u.assign(P.n, 0.0);
    for (int c = 0; c < nb; ++c) {
        int k;
        switch (f) {
            case 0: k = c; break;
            case 1: k = (nb - 1) + nb * c; break;
            case 2: k = c + nb * (nb - 1); break;
            default: k = nb * c; break;
        }
        u[k] = P.Lf[c * nq + q];
    }
}

// Element terms of the moment system's bilinear form, added into the n x n
// block blk: int grad u . D grad phi + int sigma_a u phi over element K.
void add_volume_block(const Problem& P, int K, double* blk) {
    const int n = P.n, Q = P.nq * P.nq;
    const double DK = 1.0 / (3.0 * P.sigma_t[K]);
    const double saK = P.sigma_t[K] - P.sigma_s[K];
    for (int Qi = 0; Qi < Q; ++Qi) {
        const double wJ = P.vol_wJ[(size_t)K * Q + Qi];
        const double* G = &P.vol_grad[((size_t)K * Q + Qi) * n * 2];
        const double* U = &P.vol_U[Qi * n];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                blk[i * n + j] += wJ * (DK * (G[i * 2] * G[j * 2] + G[i * 2 + 1] * G[j * 2 + 1]) + saK * U[i] * U[j]);
    }
}

// Marshak boundary term int E_b0 u phi on boundary face f of element K.
void add_boundary_block(const Problem& P, int K, int f, double* blk) {
    const int n = P.n, nq = P.nq;
    std::vector<double> uK;
    const double e_axis = (f == 1 || f == 3) ? P.eb0x : P.eb0y;
    const int bf = P.bface_of[K * 4 + f];
    for (int q = 0; q < nq; ++q) {
        face_values(P, f, q, uK);
        const double e = P.axis_bdr ? e_axis : P.eb0_pt[(size_t)bf * nq + q];
        const double s = P.dsw[((size_t)K * 4 + f) * nq + q] * e;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) blk[i * n + j] += s * uK[i] * uK[j];
    }
}

void assemble_ip(Problem& P) {
    const int n = P.n, nq = P.nq, ne = P.ne;
    P.bsr_col.assign((size_t)ne * 5, -1);
    P.bsr_val.assign((size_t)ne * 5 * n * n, 0.0);
    std::vector<double> uK, uN;
    const double pp = (P.p + 1.0) * (P.p + 1.0);
    for (int K = 0; K < ne; ++K) {
        const double DK = 1.0 / (3.0 * P.sigma_t[K]);
        double* blk0 = &P.bsr_val[((size_t)K * 5) * n * n];
        P.bsr_col[K * 5] = K;
        add_volume_block(P, K, blk0);
        for (int f = 0; f < 4; ++f) {
            const int N = P.nbr[K * 4 + f];
            if (N < 0) {
                add_boundary_block(P, K, f, blk0);
                continue;
            }
            P.bsr_col[K * 5 + 1 + f] = N;
            double* blkN = &P.bsr_val[((size_t)K * 5 + 1 + f) * n * n];
            const double DN = 1.0 / (3.0 * P.sigma_t[N]);
            const double kap = P.kappa_scale * 0.5 * (pp / (P.sigma_t[K] * std::sqrt(P.area[K])) +
                                                      pp / (P.sigma_t[N] * std::sqrt(P.area[N])));
            for (int q = 0; q < nq; ++q) {
                int fN, qN;
                nbr_point(P, K, f, q, fN, qN);
                face_values(P, f, q, uK);
                face_values(P, fN, qN, uN);
                const size_t fo = ((size_t)K * 4 + f) * nq + q;
                const size_t foN = ((size_t)N * 4 + fN) * nq + qN;
                const double nxh = P.nhat[fo * 2], nyh = P.nhat[fo * 2 + 1], s = P.dsw[fo];
                std::vector<double> dnK(n), dnN(n);
                for (int i = 0; i < n; ++i) {
                    dnK[i] = P.face_grad[(fo * n + i) * 2] * nxh + P.face_grad[(fo * n + i) * 2 + 1] * nyh;
                    dnN[i] = P.face_grad[(foN * n + i) * 2] * nxh + P.face_grad[(foN * n + i) * 2 + 1] * nyh;
                }
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        blk0[i * n + j] += s * (kap * uK[i] * uK[j] - 0.5 * DK * uK[i] * dnK[j] -
                                                0.5 * DK * dnK[i] * uK[j]);
                        blkN[i * n + j] += s * (-kap * uK[i] * uN[j] - 0.5 * DN * uK[i] * dnN[j] +
                                                0.5 * DK * dnK[i] * uN[j]);
                    }
            }
        }
    }
    P.bjac_inv.assign((size_t)ne * n * n, 0.0);
    for (int K = 0; K < ne; ++K) {
        std::memcpy(&P.bjac_inv[(size_t)K * n * n], &P.bsr_val[(size_t)K * 5 * n * n], sizeof(double) * n * n);
        lu_invert(n, &P.bjac_inv[(size_t)K * n * n]);
    }
    P.lhs_ready = true;
}

// ---------------------------------------------------------------------------
// Fixed right-hand side: int u Q0 + int grad u . Q1/sigma_t
//   - int_{Gamma0} [u]{Q1.n/sigma_t} - 2 int_{Gamma_b} u J_in,
// with Q0 = sum w q_d, Q1 = sum w Omega q_d at the nodes and
// J_in = sum_{Omega.n<0} w (Omega.n) psibar at the boundary face points.
// ---------------------------------------------------------------------------
void assemble_rhs_fixed(Problem& P) {
    const int n = P.n, nq = P.nq, ne = P.ne, nd = P.nd, Q = nq * nq;
    std::vector<double> Q0((size_t)ne * n, 0.0), Q1x((size_t)ne * n, 0.0), Q1y((size_t)ne * n, 0.0);
    for (int d = 0; d < nd; ++d) {
        const double w = P.w[d], ox = P.omega[d * 3], oy = P.omega[d * 3 + 1];
        for (size_t k = 0; k < (size_t)ne * n; ++k) {
            const double qv = (P.src_layout == SMM_SRC_ISO) ? P.q[k] : P.q[(size_t)d * ne * n + k];
            Q0[k] += w * qv;
            Q1x[k] += w * ox * qv;
            Q1y[k] += w * oy * qv;
        }
    }
    P.b_fixed.assign((size_t)ne * n, 0.0);
    std::vector<double> uK, uN;
    for (int K = 0; K < ne; ++K) {
        double* b = &P.b_fixed[(size_t)K * n];
        const double stK = P.sigma_t[K];
        for (int Qi = 0; Qi < Q; ++Qi) {
            const double wJ = P.vol_wJ[(size_t)K * Q + Qi];
            const double* G = &P.vol_grad[((size_t)K * Q + Qi) * n * 2];
            const double* U = &P.vol_U[Qi * n];
            double q0 = 0, q1x = 0, q1y = 0;
            for (int j = 0; j < n; ++j) {
                q0 += U[j] * Q0[(size_t)K * n + j];
                q1x += U[j] * Q1x[(size_t)K * n + j];
                q1y += U[j] * Q1y[(size_t)K * n + j];
            }
            for (int i = 0; i < n; ++i) b[i] += wJ * (U[i] * q0 + (G[i * 2] * q1x + G[i * 2 + 1] * q1y) / stK);
        }
        for (int f = 0; f < 4; ++f) {
            const int N = P.nbr[K * 4 + f];
            for (int q = 0; q < nq; ++q) {
                const size_t fo = ((size_t)K * 4 + f) * nq + q;
                const double nxh = P.nhat[fo * 2], nyh = P.nhat[fo * 2 + 1], s = P.dsw[fo];
                face_values(P, f, q, uK);
                if (N >= 0) {
                    int fN, qN;
                    nbr_point(P, K, f, q, fN, qN);
                    face_values(P, fN, qN, uN);
                    double ak = 0, an = 0;
                    for (int j = 0; j < n; ++j) {
                        ak += uK[j] * (Q1x[(size_t)K * n + j] * nxh + Q1y[(size_t)K * n + j] * nyh);
                        an += uN[j] * (Q1x[(size_t)N * n + j] * nxh + Q1y[(size_t)N * n + j] * nyh);
                    }
                    const double avg = 0.5 * (ak / stK + an / P.sigma_t[N]);
                    for (int i = 0; i < n; ++i) b[i] -= s * uK[i] * avg;
                } else if (P.inflow_layout != SMM_INFLOW_VACUUM) {
                    const int bf = P.bface_of[K * 4 + f];
                    double jin = 0;
                    for (int d = 0; d < nd; ++d) {
                        const double on = P.omega[d * 3] * nxh + P.omega[d * 3 + 1] * nyh;
                        if (on < 0.0) jin += P.w[d] * on * P.psibar[((size_t)bf * nq + q) * nd + d];
                    }
                    for (int i = 0; i < n; ++i) b[i] -= 2.0 * s * uK[i] * jin;
                }
            }
        }
    }
    P.rhs_fixed_ready = true;
}

// ---------------------------------------------------------------------------
// Correction operator: b_corr = C T - B beta, with T = (Txx, Txy, Tyy) nodal.
//   volume (self):  -1/sigma_K grad u_i . div T_K
//   interior face (self): + u_i/2 div T_K.n/sigma_K + 1/(2 sigma_K) grad u_i . T_K n
//   interior face (nbr):  + u_i/2 div T_N.n/sigma_N - 1/(2 sigma_K) grad u_i . T_N n
//   boundary: - u_i beta
// Column layout of a block row: c*n + j, c in (xx, xy, yy).
// ---------------------------------------------------------------------------
void assemble_correction_operator(Problem& P) {
    const int n = P.n, nq = P.nq, ne = P.ne, Q = nq * nq, n3 = 3 * n;
    P.corr_val.assign((size_t)ne * 5 * n * n3, 0.0);
    std::vector<double> uK, uN;
    for (int K = 0; K < ne; ++K) {
        const double iK = 1.0 / P.sigma_t[K];
        double* c0 = &P.corr_val[((size_t)K * 5) * n * n3];
        for (int Qi = 0; Qi < Q; ++Qi) {
            const double wJ = P.vol_wJ[(size_t)K * Q + Qi];
            const double* G = &P.vol_grad[((size_t)K * Q + Qi) * n * 2];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    const double gix = G[i * 2], giy = G[i * 2 + 1], gjx = G[j * 2], gjy = G[j * 2 + 1];
                    c0[i * n3 + 0 * n + j] -= wJ * iK * gix * gjx;
                    c0[i * n3 + 1 * n + j] -= wJ * iK * (gix * gjy + giy * gjx);
                    c0[i * n3 + 2 * n + j] -= wJ * iK * giy * gjy;
                }
        }
        for (int f = 0; f < 4; ++f) {
            const int N = P.nbr[K * 4 + f];
            if (N < 0) continue;
            const double iN = 1.0 / P.sigma_t[N];
            double* cN = &P.corr_val[((size_t)K * 5 + 1 + f) * n * n3];
            for (int q = 0; q < nq; ++q) {
                int fN, qN;
                nbr_point(P, K, f, q, fN, qN);
                const size_t fo = ((size_t)K * 4 + f) * nq + q;
                const size_t foN = ((size_t)N * 4 + fN) * nq + qN;
                const double nx_ = P.nhat[fo * 2], ny_ = P.nhat[fo * 2 + 1], s = P.dsw[fo];
                face_values(P, f, q, uK);
                face_values(P, fN, qN, uN);
                for (int i = 0; i < n; ++i) {
                    const double gix = P.face_grad[(fo * n + i) * 2], giy = P.face_grad[(fo * n + i) * 2 + 1];
                    for (int j = 0; j < n; ++j) {
                        const double gjx = P.face_grad[(fo * n + j) * 2], gjy = P.face_grad[(fo * n + j) * 2 + 1];
                        const double hjx = P.face_grad[(foN * n + j) * 2], hjy = P.face_grad[(foN * n + j) * 2 + 1];
                        // self: u_i/2 divT_K.n / sigma_K
                        c0[i * n3 + 0 * n + j] += s * 0.5 * uK[i] * iK * nx_ * gjx;
                        c0[i * n3 + 1 * n + j] += s * 0.5 * uK[i] * iK * (nx_ * gjy + ny_ * gjx);
                        c0[i * n3 + 2 * n + j] += s * 0.5 * uK[i] * iK * ny_ * gjy;
                        // self: grad u_i . T_K n / (2 sigma_K)
                        c0[i * n3 + 0 * n + j] += s * 0.5 * iK * gix * nx_ * uK[j];
                        c0[i * n3 + 1 * n + j] += s * 0.5 * iK * (gix * ny_ + giy * nx_) * uK[j];
                        c0[i * n3 + 2 * n + j] += s * 0.5 * iK * giy * ny_ * uK[j];
                        // neighbour: u_i/2 divT_N.n / sigma_N
                        cN[i * n3 + 0 * n + j] += s * 0.5 * uK[i] * iN * nx_ * hjx;
                        cN[i * n3 + 1 * n + j] += s * 0.5 * uK[i] * iN * (nx_ * hjy + ny_ * hjx);
                        cN[i * n3 + 2 * n + j] += s * 0.5 * uK[i] * iN * ny_ * hjy;
                        // neighbour: - grad u_i . T_N n / (2 sigma_K)
                        cN[i * n3 + 0 * n + j] -= s * 0.5 * iK * gix * nx_ * uN[j];
                        cN[i * n3 + 1 * n + j] -= s * 0.5 * iK * (gix * ny_ + giy * nx_) * uN[j];
                        cN[i * n3 + 2 * n + j] -= s * 0.5 * iK * giy * ny_ * uN[j];
                    }
                }
            }
        }
    }
    P.beta_op.assign((size_t)P.nbf * n * nq, 0.0);
    for (int bf = 0; bf < P.nbf; ++bf) {
        const int K = P.bface_K[bf], f = P.bface_f[bf];
        for (int q = 0; q < nq; ++q) {
            face_values(P, f, q, uK);
            const double s = P.dsw[((size_t)K * 4 + f) * nq + q];
            for (int i = 0; i < n; ++i) P.beta_op[((size_t)bf * n + i) * nq + q] = s * uK[i];
        }
    }
}

}  // namespace smm
