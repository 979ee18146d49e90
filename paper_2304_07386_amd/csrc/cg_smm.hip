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
// records r.z, the iteration count and the convergence test.  The scalar
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
        a.p[g] = z;
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
    const double rz = cgs_sum_parts(vpart(a, 0), a.vblocks, red);
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
    const double rzn = cgs_sum_parts(vpart(a, 0), a.vblocks, red);
    const double rr = cgs_sum_parts(vpart(a, 1), a.vblocks, red);
    const double rzo = a.scal[0];
    const bool conv = rr <= a.scal[3];
    const int g = blockIdx.x * CGS_T + threadIdx.x;
    if (!conv && g < a.nc) a.p[g] = a.z[g] + (rzn / rzo) * a.p[g];
}

// one-block bookkeeping after cgs_k3: r.z, r.r, iteration count, stop flag
__global__ __launch_bounds__(CGS_T) void cgs_note(CgsArgs a) {
    __shared__ double red[CGS_T];
    if (a.scal[4] != 0.0) return;
    const double rzn = cgs_sum_parts(vpart(a, 0), a.vblocks, red);
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

hipError_t cgs_start(const CgsArgs& a, double tol, hipStream_t s) {
    hipLaunchKernelGGL(cgs_init1, dim3(a.sblocks), dim3(CGS_T), 0, s, a);
    hipLaunchKernelGGL(cgs_init2, dim3(a.vblocks), dim3(CGS_T), 0, s, a);
    hipLaunchKernelGGL(cgs_init3, dim3(1), dim3(CGS_T), 0, s, a, tol);
    return hipGetLastError();
}

hipError_t cgs_iterations(const CgsArgs& a, int iters, hipStream_t s) {
    for (int t = 0; t < iters; ++t) {
        hipLaunchKernelGGL(cgs_k1, dim3(a.sblocks), dim3(CGS_T), 0, s, a);
        hipLaunchKernelGGL(cgs_k2, dim3(a.vblocks), dim3(CGS_T), 0, s, a);
        hipLaunchKernelGGL(cgs_k3, dim3(a.vblocks), dim3(CGS_T), 0, s, a);
        hipLaunchKernelGGL(cgs_note, dim3(1), dim3(CGS_T), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace smm
