// Continuous (CG) SMM moment solve on the GPU (Sec. 5.1): FP64 conjugate
// gradients on A_c c = P_c^T b with the Jacobi preconditioner, A_c the CSR
// matrix of the continuous space V_p.
//
// Kernels:
// * gather b = P_c^T b_dg: one thread per continuous node adds the (at most
//   four) DG entries of its node in ascending DG order;
// * product y = A_c x: eight lanes per row stride over its entries (at most
//   (2p+1)^2 = 81), then a fixed butterfly over the eight lanes; 32 rows per
//   256-thread block, the rows of a block contiguous, so the column reads of
//   neighbouring rows overlap in cache;
// * vector updates one thread per node; every reduction goes through block
//   partials and a one-block kernel that adds them in block order, so each
//   sum (and the iteration) is the same on every run.
// One PCG iteration is four launches: q = A p with partials of p.q; alpha
// from those partials, x += alpha p, r -= alpha q, z = r / diag with partials
// of r.z and r.r; beta from those and p = z + beta p; a one-block launch that
// records r.z, the iteration count and the convergence test.
// With the two-level preconditioner (the coarse space of the IP solve carried
// over to V_p: continuous bilinear functions on the element vertices) two
// launches come between the update and the direction update: the vertex
// right-hand side P_1^T r, and one V-cycle of the vertex multigrid in a
// single workgroup (levels in global memory, steps separated by barriers),
// which also forms (P_1^T r).x_v.  z = D^-1 r stays as it is; the coarse part
// enters r.z through that product and p = z + P_1 x_v + beta p through
// interpolation at each node, so no extra vector pass is needed.  The scalar
// reductions are repeated by every block that needs them (a few thousand
// partials, read from cache), which saves two launches per iteration.  A
// stopped solve (converged, breakdown) makes every later launch of the chunk
// return at once.
#include "cg_smm.hpp"

namespace smm {

namespace {

constexpr int CGS_T = 256;

__device__ __forceinline__ double cgs_block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = CGS_T / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// sum of part[0 .. n) in block order, by the one block of the launch
__device__ __forceinline__ double cgs_sum_parts(const double* part, int n, double* red) {
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += CGS_T) v += part[k];
    return cgs_block_sum(v, red);
}

// partials: p.q per product block at part[0, sblocks), then the node-wise
// kernels' sums k = 0, 1, 2 per node block
__device__ __forceinline__ double* vpart(const CgsArgs& a, int k) { return a.part + a.sblocks + k * a.vblocks; }

// (P_1 x_v) at continuous node g: bilinear in the element holding it (the
// last element of a row or column for the nodes on its far edge)
__device__ __forceinline__ double cgs_coarse_at(const CgsArgs& a, int g) {
    const int po = a.order, ncx = a.nx * po + 1;
    const int gi = g % ncx, gj = g / ncx;
    const int ex = min(gi / po, a.nx - 1), ey = min(gj / po, a.ny - 1);
    const double sx = a.gll[gi - ex * po], sy = a.gll[gj - ey * po];
    const int v = ey * (a.nx + 1) + ex;
    const double* xv = a.xv;
    return (1.0 - sy) * ((1.0 - sx) * xv[v] + sx * xv[v + 1]) +
           sy * ((1.0 - sx) * xv[v + a.nx + 1] + sx * xv[v + a.nx + 2]);
}

// row `row` of A_c times x, summed over the 8 lanes `sub` = 0..7 of the row;
// every lane of the group returns the sum
__device__ __forceinline__ double cgs_row(const CgsArgs& a, const double* __restrict__ x, int row, int sub) {
    double v = 0.0;
    if (row < a.nc) {
        const int e = a.rowptr[row + 1];
        for (int k = a.rowptr[row] + sub; k < e; k += 8) v += a.val[k] * x[a.col[k]];
    }
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    return v;
}

__global__ __launch_bounds__(CGS_T) void cgs_gather_kernel(CgsArgs a, const double* __restrict__ b_dg) {
    const int g = blockIdx.x * CGS_T + threadIdx.x;
    if (g >= a.nc) return;
    double v = 0.0;
    for (int k = 0; k < 4; ++k) {
        const int t = a.tab[g * 4 + k];
        if (t >= 0) v += b_dg[t];
    }
    a.b[g] = v;
}

__global__ __launch_bounds__(CGS_T) void cgs_pick_kernel(CgsArgs a, const double* __restrict__ x_dg) {
    const int g = blockIdx.x * CGS_T + threadIdx.x;
    if (g < a.nc) a.x[g] = x_dg[a.tab[g * 4]];
}

__global__ __launch_bounds__(CGS_T) void cgs_scatter_kernel(CgsArgs a, double* __restrict__ x_dg) {
    const long t = (long)blockIdx.x * CGS_T + threadIdx.x;
    if (t < a.L) x_dg[t] = a.x[a.map[t]];
}

__global__ __launch_bounds__(CGS_T) void cgs_spmv_kernel(CgsArgs a, const double* __restrict__ x,
                                                         double* __restrict__ y) {
    const int row = blockIdx.x * CGS_SPMV_ROWS + (threadIdx.x >> 3);
    const double v = cgs_row(a, x, row, threadIdx.x & 7);
    if ((threadIdx.x & 7) == 0 && row < a.nc) y[row] = v;
}

// r = b - A x
__global__ __launch_bounds__(CGS_T) void cgs_init1(CgsArgs a) {
    const int row = blockIdx.x * CGS_SPMV_ROWS + (threadIdx.x >> 3);
    const double v = cgs_row(a, a.x, row, threadIdx.x & 7);
    if ((threadIdx.x & 7) == 0 && row < a.nc) a.r[row] = a.b[row] - v;
}

// z = r / diag, p = z; partials of r.z, r.r, b.b
__global__ __launch_bounds__(CGS_T) void cgs_init2(CgsArgs a) {
    __shared__ double red[CGS_T];
    const int g = blockIdx.x * CGS_T + threadIdx.x;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    if (g < a.nc) {
        const double r = a.r[g], z = r * a.dinv[g];
        a.z[g] = z;
        if (!a.mg) a.p[g] = z;   // two-level: cgs_init_p after the V-cycle
        rz = r * z;
        rr = r * r;
        bb = a.b[g] * a.b[g];
    }
    rz = cgs_block_sum(rz, red);
    rr = cgs_block_sum(rr, red);
    bb = cgs_block_sum(bb, red);
    if (threadIdx.x == 0) {
        vpart(a, 0)[blockIdx.x] = rz;
        vpart(a, 1)[blockIdx.x] = rr;
        vpart(a, 2)[blockIdx.x] = bb;
    }
}

__global__ __launch_bounds__(CGS_T) void cgs_init3(CgsArgs a, double tol) {
    __shared__ double red[CGS_T];
    const double rz = cgs_sum_parts(vpart(a, 0), a.vblocks, red) + (a.mg ? a.scal[8] : 0.0);
    const double rr = cgs_sum_parts(vpart(a, 1), a.vblocks, red);
    const double bb = cgs_sum_parts(vpart(a, 2), a.vblocks, red);
    if (threadIdx.x == 0) {
        a.scal[0] = rz;
        a.scal[1] = bb;
        a.scal[2] = rr;
        a.scal[3] = tol * tol * bb;
        a.scal[4] = rr <= a.scal[3] ? 1.0 : 0.0;
        a.scal[5] = 0.0;
        a.scal[6] = 0.0;
    }
}

// q = A p; partial sums of p.q per block
__global__ __launch_bounds__(CGS_T) void cgs_k1(CgsArgs a) {
    __shared__ double red[CGS_T];
    if (a.scal[4] != 0.0) return;
    const int row = blockIdx.x * CGS_SPMV_ROWS + (threadIdx.x >> 3);
    const double v = cgs_row(a, a.p, row, threadIdx.x & 7);
    double pq = 0.0;
    if ((threadIdx.x & 7) == 0 && row < a.nc) {
        a.q[row] = v;
        pq = a.p[row] * v;
    }
    pq = cgs_block_sum(pq, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = pq;
}

// alpha = r.z / p.q from the product kernel's partials (every block forms
// the same sum in the same order; p.q <= 0 stops the solve); x += alpha p,
// r -= alpha q, z = r / diag; partials of r.z and r.r
__global__ __launch_bounds__(CGS_T) void cgs_k2(CgsArgs a) {
    __shared__ double red[CGS_T];
    if (a.scal[4] != 0.0) return;
    const double pq = cgs_sum_parts(a.part, a.sblocks, red);
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.scal[6] = pq <= 0.0 ? 1.0 : 2.0;  // 2: not a number (a non-finite right-hand side)
            a.scal[4] = 1.0;
        }
        return;
    }
    const double alpha = a.scal[0] / pq;
    const int g = blockIdx.x * CGS_T + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (g < a.nc) {
        a.x[g] += alpha * a.p[g];
        const double r = a.r[g] - alpha * a.q[g], z = r * a.dinv[g];
        a.r[g] = r;
        a.z[g] = z;
        rz = r * z;
        rr = r * r;
    }
    rz = cgs_block_sum(rz, red);
    rr = cgs_block_sum(rr, red);
    if (threadIdx.x == 0) {
        vpart(a, 0)[blockIdx.x] = rz;
        vpart(a, 1)[blockIdx.x] = rr;
    }
}

// beta = r.z_new / r.z_old and the test ||r|| <= tol ||b|| from the update
// kernel's partials (every block alike); p = z + beta p unless converged.
// r.z_old stays in scal[0] until the next launch records the new one.
__global__ __launch_bounds__(CGS_T) void cgs_k3(CgsArgs a) {
    __shared__ double red[CGS_T];
    if (a.scal[4] != 0.0) return;
    const double rzn = cgs_sum_parts(vpart(a, 0), a.vblocks, red) + (a.mg ? a.scal[8] : 0.0);
    const double rr = cgs_sum_parts(vpart(a, 1), a.vblocks, red);
    const double rzo = a.scal[0];
    const bool conv = rr <= a.scal[3];
    const int g = blockIdx.x * CGS_T + threadIdx.x;
    if (!conv && g < a.nc) {
        const double z = a.z[g] + (a.mg ? cgs_coarse_at(a, g) : 0.0);
        a.p[g] = z + (rzn / rzo) * a.p[g];
    }
}

// two-level start: p = D^-1 r + P_1 x_v
__global__ __launch_bounds__(CGS_T) void cgs_init_p(CgsArgs a) {
    const int g = blockIdx.x * CGS_T + threadIdx.x;
    if (g < a.nc) a.p[g] = a.z[g] + cgs_coarse_at(a, g);
}

// rv = P_1^T r: each vertex gathers the continuous nodes of its (at most four)
// elements, weighted by its bilinear function there
__global__ __launch_bounds__(CGS_T) void cgs_restrict_kernel(CgsArgs a, bool start) {
    if (!start && a.scal[4] != 0.0) return;
    const int nvx = a.nx + 1, v = blockIdx.x * CGS_T + threadIdx.x;
    if (v >= nvx * (a.ny + 1)) return;
    const int p = a.order, ncx = a.nx * p + 1, ncy = a.ny * p + 1;
    const int gi0 = (v % nvx) * p, gj0 = (v / nvx) * p;
    auto w = [&](int d) { return d <= 0 ? a.gll[p + d] : 1.0 - a.gll[d]; };
    double s = 0.0;
    for (int dy = -p; dy <= p; ++dy) {
        const int gj = gj0 + dy;
        if (gj < 0 || gj >= ncy) continue;
        double sr = 0.0;
        for (int dx = -p; dx <= p; ++dx) {
            const int gi = gi0 + dx;
            if (gi < 0 || gi >= ncx) continue;
            sr += w(dx) * a.r[(long)gj * ncx + gi];
        }
        s += w(dy) * sr;
    }
    a.rv[v] = s;
}

// one V-cycle x_v = V(rv) on the vertex levels in one workgroup: one damped
// Jacobi step down (from zero) and up, full-weighting restriction, bilinear
// prolongation (the transposes of each other), the coarsest level by its
// dense inverse; then (P_1^T r).x_v into scal[8]
constexpr int CGS_VT = 1024;
__device__ __forceinline__ void cgs_mg_parents(int i, int nf, int& c0, double& w0, int& c1, double& w1) {
    // coarse parents of fine vertex i of a 1D level of nf vertices (every other
    // vertex kept, the last always; a direction of at most 3 vertices is not
    // coarsened further)
    const int nc = nf <= 3 ? nf : nf / 2 + 1;
    c1 = -1;
    w1 = 0.0;
    if (nf <= 3) {
        c0 = i;
        w0 = 1.0;
    } else if (i == nf - 1) {
        c0 = nc - 1;
        w0 = 1.0;
    } else if ((i & 1) == 0) {
        c0 = i >> 1;
        w0 = 1.0;
    } else {
        c0 = (i - 1) >> 1;
        w0 = 0.5;
        c1 = (i + 1) >> 1;
        w1 = 0.5;
    }
}

__global__ __launch_bounds__(CGS_VT) void cgs_vcycle_kernel(CgsArgs a, CgsMG m, bool start) {
    __shared__ double red[CGS_VT];
    if (!start && a.scal[4] != 0.0) return;
    const int tid = threadIdx.x, lc = m.nlev - 1;
    const double om = m.omega;
    auto apply = [&](int l, const double* x, int v) {
        const int nvx = m.nvx[l], nvy = m.nvy[l], nv = nvx * nvy;
        const int ix = v % nvx, iy = v / nvx;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int jx = ix + k % 3 - 1, jy = iy + k / 3 - 1;
            if (jx < 0 || jy < 0 || jx >= nvx || jy >= nvy) continue;
            s += m.A[l][(long)k * nv + v] * x[jy * nvx + jx];
        }
        return s;
    };
    for (int l = 0; l < lc; ++l) {
        const int nvx = m.nvx[l], nvy = m.nvy[l], nv = nvx * nvy;
        const double* A = m.A[l];
        double *x = m.x[l], *t = m.t[l], *b = m.b[l];
        for (int v = tid; v < nv; v += CGS_VT) x[v] = om * b[v] / A[4L * nv + v];
        __syncthreads();
        for (int v = tid; v < nv; v += CGS_VT) t[v] = b[v] - apply(l, x, v);
        __syncthreads();
        const int cnx = m.nvx[l + 1], cny = m.nvy[l + 1];
        double* bc = m.b[l + 1];
        for (int c = tid; c < cnx * cny; c += CGS_VT) {
            const int cx = c % cnx, cy = c / cnx;
            const int bx = nvx <= 3 ? cx : (cx == cnx - 1 ? nvx - 1 : 2 * cx);
            const int by = nvy <= 3 ? cy : (cy == cny - 1 ? nvy - 1 : 2 * cy);
            double s = 0.0;
            for (int fy = by - 2; fy <= by + 2; ++fy) {
                if (fy < 0 || fy >= nvy) continue;
                int y0, y1;
                double wy0, wy1;
                cgs_mg_parents(fy, nvy, y0, wy0, y1, wy1);
                const double wy = y0 == cy ? wy0 : (y1 == cy ? wy1 : 0.0);
                if (wy == 0.0) continue;
                for (int fx = bx - 2; fx <= bx + 2; ++fx) {
                    if (fx < 0 || fx >= nvx) continue;
                    int x0, x1;
                    double wx0, wx1;
                    cgs_mg_parents(fx, nvx, x0, wx0, x1, wx1);
                    const double wx = x0 == cx ? wx0 : (x1 == cx ? wx1 : 0.0);
                    if (wx != 0.0) s += wx * wy * t[fy * nvx + fx];
                }
            }
            bc[c] = s;
        }
        __syncthreads();
    }
    {
        const int nc = m.nvx[lc] * m.nvy[lc];
        if (tid < nc) {
            double s = 0.0;
            for (int j = 0; j < nc; ++j) s += m.cinv[tid * nc + j] * m.b[lc][j];
            m.x[lc][tid] = s;
        }
    }
    __syncthreads();
    for (int l = lc - 1; l >= 0; --l) {
        const int nvx = m.nvx[l], nvy = m.nvy[l], nv = nvx * nvy, cnx = m.nvx[l + 1];
        const double* A = m.A[l];
        double *x = m.x[l], *t = m.t[l], *b = m.b[l];
        const double* xc = l + 1 == lc ? m.x[l + 1] : m.t[l + 1];
        for (int f = tid; f < nv; f += CGS_VT) {
            int x0, x1, y0, y1;
            double wx0, wx1, wy0, wy1;
            cgs_mg_parents(f % nvx, nvx, x0, wx0, x1, wx1);
            cgs_mg_parents(f / nvx, nvy, y0, wy0, y1, wy1);
            double s = wx0 * wy0 * xc[y0 * cnx + x0];
            if (x1 >= 0) s += wx1 * wy0 * xc[y0 * cnx + x1];
            if (y1 >= 0) s += wx0 * wy1 * xc[y1 * cnx + x0];
            if (x1 >= 0 && y1 >= 0) s += wx1 * wy1 * xc[y1 * cnx + x1];
            x[f] += s;
        }
        __syncthreads();
        for (int v = tid; v < nv; v += CGS_VT) t[v] = x[v] + om * (b[v] - apply(l, x, v)) / A[4L * nv + v];
        __syncthreads();
    }
    // (P_1^T r).x_v, summed in a fixed order (the same on every run)
    const int nv0 = m.nvx[0] * m.nvy[0];
    double s = 0.0;
    for (int v = tid; v < nv0; v += CGS_VT) s += a.rv[v] * a.xv[v];
    red[tid] = s;
    __syncthreads();
    for (int k = CGS_VT / 2; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) a.scal[8] = red[0];
}

// one-block bookkeeping after cgs_k3: r.z, r.r, iteration count, stop flag
__global__ __launch_bounds__(CGS_T) void cgs_note(CgsArgs a) {
    __shared__ double red[CGS_T];
    if (a.scal[4] != 0.0) return;
    const double rzn = cgs_sum_parts(vpart(a, 0), a.vblocks, red) + (a.mg ? a.scal[8] : 0.0);
    const double rr = cgs_sum_parts(vpart(a, 1), a.vblocks, red);
    if (threadIdx.x == 0) {
        a.scal[0] = rzn;
        a.scal[2] = rr;
        a.scal[5] += 1.0;
        if (rr <= a.scal[3]) a.scal[4] = 1.0;
    }
}

}  // namespace

hipError_t cgs_gather(const CgsArgs& a, const double* b_dg, hipStream_t s) {
    hipLaunchKernelGGL(cgs_gather_kernel, dim3(a.vblocks), dim3(CGS_T), 0, s, a, b_dg);
    return hipGetLastError();
}

hipError_t cgs_pick(const CgsArgs& a, const double* x_dg, hipStream_t s) {
    hipLaunchKernelGGL(cgs_pick_kernel, dim3(a.vblocks), dim3(CGS_T), 0, s, a, x_dg);
    return hipGetLastError();
}

hipError_t cgs_scatter(const CgsArgs& a, double* x_dg, hipStream_t s) {
    const unsigned nb = (unsigned)((a.L + CGS_T - 1) / CGS_T);
    hipLaunchKernelGGL(cgs_scatter_kernel, dim3(nb), dim3(CGS_T), 0, s, a, x_dg);
    return hipGetLastError();
}

hipError_t cgs_spmv(const CgsArgs& a, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(cgs_spmv_kernel, dim3(a.sblocks), dim3(CGS_T), 0, s, a, x, y);
    return hipGetLastError();
}

static void cgs_coarse(const CgsArgs& a, const CgsMG& m, bool start, hipStream_t s) {
    const unsigned nvb = (unsigned)(((a.nx + 1) * (a.ny + 1) + CGS_T - 1) / CGS_T);
    hipLaunchKernelGGL(cgs_restrict_kernel, dim3(nvb), dim3(CGS_T), 0, s, a, start);
    hipLaunchKernelGGL(cgs_vcycle_kernel, dim3(1), dim3(CGS_VT), 0, s, a, m, start);
}

hipError_t cgs_start(const CgsArgs& a, const CgsMG& m, double tol, hipStream_t s) {
    hipLaunchKernelGGL(cgs_init1, dim3(a.sblocks), dim3(CGS_T), 0, s, a);
    hipLaunchKernelGGL(cgs_init2, dim3(a.vblocks), dim3(CGS_T), 0, s, a);
    if (a.mg) {
        cgs_coarse(a, m, true, s);
        hipLaunchKernelGGL(cgs_init_p, dim3(a.vblocks), dim3(CGS_T), 0, s, a);
    }
    hipLaunchKernelGGL(cgs_init3, dim3(1), dim3(CGS_T), 0, s, a, tol);
    return hipGetLastError();
}

hipError_t cgs_iterations(const CgsArgs& a, const CgsMG& m, int iters, hipStream_t s) {
    for (int t = 0; t < iters; ++t) {
        hipLaunchKernelGGL(cgs_k1, dim3(a.sblocks), dim3(CGS_T), 0, s, a);
        hipLaunchKernelGGL(cgs_k2, dim3(a.vblocks), dim3(CGS_T), 0, s, a);
        if (a.mg) cgs_coarse(a, m, false, s);
        hipLaunchKernelGGL(cgs_k3, dim3(a.vblocks), dim3(CGS_T), 0, s, a);
        hipLaunchKernelGGL(cgs_note, dim3(1), dim3(CGS_T), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace smm
