// Continuous finite element (CG) SMM moment system, host set-up.
//
// Sec. 5.1 derives the CG moment system from the interior-penalty one by
// taking test and trial functions in V_p, the continuous degree-p space.
// Jumps of V_p functions vanish on interior faces, so only the element terms
// (diffusion with D = 1/(3 sigma_t), absorption) and the Marshak boundary
// term E_b0 remain on the left.  With a Gauss-Lobatto nodal basis on a
// structured nx x ny mesh, V_p has one unknown per grid node
// (gi, gj) = (ex p + a, ey p + b) of the (nx p + 1) x (ny p + 1) node grid,
// shared by the DG nodes of all elements that touch it (at most four), and
// the continuous operator is A_c = sum_K P_K^T A_K P_K with A_K the element
// block above.  Its right-hand side is P_c^T b of the DG right-hand side b:
// the [u] terms of the IP right-hand side cancel between the two sides of
// each face, and the remaining terms are those of the CG form.
//
// Layout of the CSR matrix: row g = gj (nx p + 1) + gi couples to the nodes
// (gi + dx, gj + dy), |dx|, |dy| <= p, of the elements around it; columns are
// stored in increasing order, and each entry is summed over elements in
// increasing element order (the same sum on every build).
#include <algorithm>
#include <cstring>

#include "smm_internal.hpp"

namespace smm {

void assemble_cg(Problem& P) {
    const int p = P.p, nb = P.nb, n = P.n, ne = P.ne;
    const int ncx = P.nx * p + 1, ncy = P.ny * p + 1, nc = ncx * ncy;
    const int w = 2 * p + 1, ns = w * w;
    P.cg_nc = nc;
    P.cg_map.assign((size_t)ne * n, -1);
    P.cg_tab.assign((size_t)nc * 4, -1);
    std::vector<int> cnt(nc, 0);
    for (int K = 0; K < ne; ++K) {
        const int ex = K % P.nx, ey = K / P.nx;
        for (int b = 0; b < nb; ++b)
            for (int a = 0; a < nb; ++a) {
                const int g = (ey * p + b) * ncx + ex * p + a;
                const int t = K * n + a + nb * b;
                P.cg_map[t] = g;
                P.cg_tab[(size_t)g * 4 + cnt[g]++] = t;  // K ascending, so t ascending
            }
    }
    // accumulate the element blocks into stencil slots of each row
    std::vector<double> acc((size_t)nc * ns, 0.0);
    std::vector<uint8_t> used((size_t)nc * ns, 0);
    std::vector<double> blk((size_t)n * n);
    for (int K = 0; K < ne; ++K) {
        std::fill(blk.begin(), blk.end(), 0.0);
        add_volume_block(P, K, blk.data());
        for (int f = 0; f < 4; ++f)
            if (P.nbr[K * 4 + f] < 0) add_boundary_block(P, K, f, blk.data());
        const int ex = K % P.nx, ey = K / P.nx;
        for (int i = 0; i < n; ++i) {
            const int ai = i % nb, bi = i / nb;
            const int g = (ey * p + bi) * ncx + ex * p + ai;
            for (int j = 0; j < n; ++j) {
                const int aj = j % nb, bj = j / nb;
                const int s = (bj - bi + p) * w + (aj - ai + p);
                acc[(size_t)g * ns + s] += blk[i * n + j];
                used[(size_t)g * ns + s] = 1;
            }
        }
    }
    P.cg_rowptr.assign(nc + 1, 0);
    P.cg_col.clear();
    P.cg_val.clear();
    P.cg_dinv.assign(nc, 0.0);
    for (int g = 0; g < nc; ++g) {
        const int gi = g % ncx, gj = g / ncx;
        for (int s = 0; s < ns; ++s) {
            if (!used[(size_t)g * ns + s]) continue;
            const int col = (gj + s / w - p) * ncx + gi + s % w - p;
            P.cg_col.push_back(col);
            P.cg_val.push_back(acc[(size_t)g * ns + s]);
            if (col == g) P.cg_dinv[g] = 1.0 / acc[(size_t)g * ns + s];
        }
        P.cg_rowptr[g + 1] = (int)P.cg_col.size();
    }
    P.cg_ready = true;
}

}  // namespace smm
