// Host-side hierarchy of the two-level preconditioner (see mg.cpp).
#pragma once

#include <string>
#include <vector>

namespace smm {

struct Problem;

constexpr int MG_MAX_COARSE = 16;  // unknowns of the dense coarsest solve
constexpr size_t MG_LDS_CAP = 150 * 1024;  // LDS of the one-workgroup V-cycle on the coarse levels
constexpr int MG_NU = 1;                   // damped Jacobi steps before and after each coarse correction
constexpr int CG_BLOCK = 256;              // nodes per block of the continuous-space kernel (its block size)

struct MGLevelHost {
    int nvx = 0, nvy = 0;
    std::vector<double> A;  // [9][nvx*nvy] stencil, entry k = (dy+1)*3 + (dx+1)
};

struct MGHost {
    std::vector<MGLevelHost> lev;  // lev[0]: element vertices
    std::vector<double> cinv;      // dense inverse of the coarsest level
    std::vector<double> gll;       // Gauss-Lobatto points on [0,1] (nb)
};

int build_mg(const Problem& P, MGHost& M, std::string& err);
// the same hierarchy for the continuous (CG) moment system: level 0 is the
// Galerkin product of the bilinear vertex space with A_c
int build_mg_cg(const Problem& P, MGHost& M, std::string& err);
int mg_coarse_count(int nf);

}  // namespace smm
