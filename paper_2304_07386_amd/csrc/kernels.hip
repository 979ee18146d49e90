// Device kernels of libsmm (gfx950 / CDNA4).
//
//  * sweep_cart_kernel    Cartesian wavefront sweep: one workgroup per
//                         direction walks the anti-diagonals of the element
//                         grid; the upwind face traces live in LDS.
//  * sweep_general_kernel Curved meshes: per (element, direction) the local
//                         upwind DG matrix is assembled in LDS and eliminated
//                         by one wavefront; levels come from the sweep graph.
//  * sweep_lane_general_kernel  The same at p <= 2 with one lane per element:
//                         the augmented system stays in registers.
//  * gen_inv_*            Curved meshes with stored element operators: the
//                         inverses built once in parallel, a sweep being one
//                         parallel pass and a pass over the levels that adds
//                         the upwind faces' contributions.
//  * moments_kernel       Angular moments mom = W psi on the matrix cores.
//  * closure / rhs / cg   SMM correction tensor and boundary factor, the IP
//                         right-hand side, FP64 block-Jacobi PCG.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace smm {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// 16 bytes of T as one vector
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef v4f type;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    typedef v2d type;
    static constexpr int n = 2;
};

// Global-address-space views of buffer pointers that reach a kernel through a
// descriptor in memory.  Through a generic pointer the compiler emits flat
// instructions, which also count as LDS operations: every wait for the LDS
// before a barrier would then wait for the outstanding HBM loads and stores.
template <typename T>
using gptr = T __attribute__((address_space(1)))*;
template <typename T>
using gcptr = const T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
    return (gptr<T>)(unsigned long)p;
}
template <typename T>
__device__ __forceinline__ gcptr<T> as_global(const T* p) {
    return (gcptr<T>)(unsigned long)p;
}

// ---------------------------------------------------------------------------
// Cartesian sweep.
// For direction d in quadrant (sx, sy), element (i, j) receives its x-face
// trace from (i - sx, j) and its y-face trace from (i, j - sy); all elements
// on one anti-diagonal of the quadrant-oriented grid are independent.  With
// the tabulated operators of the element's material,
//     psi_K = Pm S_K + Px t_x + Py t_y.
// Traces are double-buffered by level parity in LDS so one barrier per level
// suffices.
// ---------------------------------------------------------------------------
template <typename T, int NB>
__global__ __launch_bounds__(1024) void sweep_cart_kernel(CartSweepArgs a) {
    constexpr int N = NB * NB;
    const int d = blockIdx.x;
    const int nx = a.nx, ny = a.ny, nd = a.nd;
    const long ne = (long)nx * ny;
    extern __shared__ __align__(16) unsigned char smem[];
    T* xtr = reinterpret_cast<T*>(smem);  // [2][ny][NB]
    T* ytr = xtr + 2 * ny * NB;           // [2][nx][NB]
    const double ox = a.omega[d * 3], oy = a.omega[d * 3 + 1];
    const bool sx = ox > 0.0, sy = oy > 0.0;
    const T* bx = reinterpret_cast<const T*>(a.bx);
    const T* by = reinterpret_cast<const T*>(a.by);
    for (int t = threadIdx.x; t < ny * NB; t += blockDim.x) {
        const T v = bx ? bx[(long)d * ny * NB + t] : T(0);
        xtr[t] = v;
        xtr[ny * NB + t] = v;
    }
    for (int t = threadIdx.x; t < nx * NB; t += blockDim.x) {
        const T v = by ? by[(long)d * nx * NB + t] : T(0);
        ytr[t] = v;
        ytr[nx * NB + t] = v;
    }
    __syncthreads();
    const int aout = sx ? NB - 1 : 0;
    const int bout = sy ? NB - 1 : 0;
    const T* S = reinterpret_cast<const T*>(a.S) + (a.s_aniso ? (long)d * ne * N : 0);
    T* psi = reinterpret_cast<T*>(a.psi) + (long)d * ne * N;
    const T* Pm = reinterpret_cast<const T*>(a.Pm);
    const T* Px = reinterpret_cast<const T*>(a.Px);
    const T* Py = reinterpret_cast<const T*>(a.Py);
    const int nlev = nx + ny - 1;
    for (int l = 0; l < nlev; ++l) {
        const int i0 = l - (ny - 1) > 0 ? l - (ny - 1) : 0;
        const int i1 = l < nx - 1 ? l : nx - 1;
        const int len = i1 - i0 + 1;
        const int cur = l & 1, nxt = cur ^ 1;
        for (int t = threadIdx.x; t < len * N; t += blockDim.x) {
            const int e = t / N, r = t - e * N;
            const int ip = i0 + e, jp = l - ip;
            const int i = sx ? ip : nx - 1 - ip;
            const int j = sy ? jp : ny - 1 - jp;
            const long K = (long)j * nx + i;
            const long o = (long)a.mat[K] * nd + d;
            const T* pm = Pm + (o * N + r) * N;
            const T* px = Px + (o * N + r) * NB;
            const T* py = Py + (o * N + r) * NB;
            const T* sk = S + K * N;
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < N; ++c) acc += pm[c] * sk[c];
            const T* tx = xtr + (cur * ny + j) * NB;
            const T* ty = ytr + (cur * nx + i) * NB;
#pragma unroll
            for (int c = 0; c < NB; ++c) acc += px[c] * tx[c] + py[c] * ty[c];
            psi[K * N + r] = acc;
            const int ra = r % NB, rb = r / NB;
            if (ra == aout) xtr[(nxt * ny + j) * NB + rb] = acc;
            if (rb == bout) ytr[(nxt * nx + i) * NB + ra] = acc;
        }
        __syncthreads();
    }
}

template <typename T, int NB>
static hipError_t launch_cart_t(const CartSweepArgs& a, hipStream_t s) {
    constexpr int N = NB * NB;
    const int maxlen = a.nx < a.ny ? a.nx : a.ny;
    int threads = ((maxlen * N + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    if (threads < 64) threads = 64;
    const size_t lds = sizeof(T) * 2 * (size_t)(a.nx + a.ny) * NB;
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_cart_kernel<T, NB>), dim3(a.nd), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Column-per-thread Cartesian sweep.  Each element of an anti-diagonal is
// handled by NB threads; thread `ca` owns the element's node column
// {ca + NB b}, so its rows of the tabulated operators [Pm | Px | Py] stay in
// registers for the whole sweep (one or two materials) or are read from LDS
// (more materials).  The source of the next anti-diagonal is prefetched into
// registers while the current one is computed and parked in a double-buffered
// LDS array, so each level costs LDS traffic and one barrier, not a global
// memory round trip.
// ---------------------------------------------------------------------------
// Barrier for LDS-only communication: waits for this wave's LDS operations
// and synchronises the workgroup, but does not wait for outstanding global
// stores (the sweep never reads back what it writes to global memory).  The
// "memory" clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <typename T, int NB, int MREG, int B>
__device__ __forceinline__ void sweep_cart_task(const CartSweepArgs& a, const int d, unsigned char* smem) {
    constexpr int N = NB * NB;
    constexpr int ROWW = N + 2 * NB;
    const int nx = a.nx, ny = a.ny, nd = a.nd;
    const long ne = (long)nx * ny;
    const int maxlen = nx < ny ? nx : ny;
    T* xtr = reinterpret_cast<T*>(smem);  // [2][ny][NB]
    T* ytr = xtr + 2 * ny * NB;           // [2][nx][NB]
    T* sch = ytr + 2 * nx * NB;           // [2][B][maxlen][N] source of two blocks of B levels
    T* tab = sch + 2 * B * maxlen * N;    // [nmat][N][ROWW]   (MREG == 0)
    uint8_t* msh = reinterpret_cast<uint8_t*>(tab + (MREG == 0 ? a.nmat * N * ROWW : 0));  // [ne]
    const int slot = threadIdx.x / NB;
    const int ca = threadIdx.x - slot * NB;
    const double ox = a.omega[d * 3], oy = a.omega[d * 3 + 1];
    const bool sx = ox > 0.0, sy = oy > 0.0;
    const T* Pm = reinterpret_cast<const T*>(a.Pm);
    const T* Px = reinterpret_cast<const T*>(a.Px);
    const T* Py = reinterpret_cast<const T*>(a.Py);
    const auto S = as_global(reinterpret_cast<const T*>(a.S) + (a.s_aniso ? (long)d * ne * N : 0));
    const auto psi = as_global(reinterpret_cast<T*>(a.psi) + (long)d * (a.psi_ld > 0 ? a.psi_ld : ne * N));
    if constexpr (MREG != 1) {
        const auto mat = as_global(a.mat);
        for (long t = threadIdx.x; t < ne; t += blockDim.x) msh[t] = mat[t];
    }

    // operator rows of this thread's node column
    T reg[MREG > 0 ? MREG : 1][NB][ROWW];
    if constexpr (MREG > 0) {
#pragma unroll
        for (int m = 0; m < MREG; ++m) {
            const int mm = m < a.nmat ? m : 0;
            const long o = (long)mm * nd + d;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int r = ca + NB * b;
#pragma unroll
                for (int c = 0; c < N; ++c) reg[m][b][c] = Pm[(o * N + r) * N + c];
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    reg[m][b][N + c] = Px[(o * N + r) * NB + c];
                    reg[m][b][N + NB + c] = Py[(o * N + r) * NB + c];
                }
            }
        }
    } else {
        for (int t = threadIdx.x; t < a.nmat * N; t += blockDim.x) {
            const int m = t / N, r = t - m * N;
            const long o = (long)m * nd + d;
            T* row = tab + (long)t * ROWW;
            for (int c = 0; c < N; ++c) row[c] = Pm[(o * N + r) * N + c];
            for (int c = 0; c < NB; ++c) {
                row[N + c] = Px[(o * N + r) * NB + c];
                row[N + NB + c] = Py[(o * N + r) * NB + c];
            }
        }
    }
    const auto bx = as_global(reinterpret_cast<const T*>(a.bx));
    const auto by = as_global(reinterpret_cast<const T*>(a.by));
    for (int t = threadIdx.x; t < ny * NB; t += blockDim.x) {
        const T v = bx ? bx[(long)d * ny * NB + t] : T(0);
        xtr[t] = v;
        xtr[ny * NB + t] = v;
    }
    for (int t = threadIdx.x; t < nx * NB; t += blockDim.x) {
        const T v = by ? by[(long)d * nx * NB + t] : T(0);
        ytr[t] = v;
        ytr[nx * NB + t] = v;
    }
    const int aout = sx ? NB - 1 : 0;
    const int bout = sy ? NB - 1 : 0;
    const int nlev = nx + ny - 1;
    // element of this slot at level l: returns K or -1
    auto elem = [&](int l, int& i, int& j) -> long {
        if (l >= nlev) return -1;
        const int i0 = l - (ny - 1) > 0 ? l - (ny - 1) : 0;
        const int i1 = l < nx - 1 ? l : nx - 1;
        if (slot > i1 - i0) return -1;
        const int ip = i0 + slot, jp = l - ip;
        i = sx ? ip : nx - 1 - ip;
        j = sy ? jp : ny - 1 - jp;
        return (long)j * nx + i;
    };
    // Source of a block of B levels: loaded into registers at the start of
    // the previous block and parked in LDS at its end.  Loads are issued
    // unconditionally (element 0 stands in for an empty slot), so load and
    // wait sit in one straight-line block with a known number of
    // intervening memory operations.
    T pre[B][NB];
    auto fetch_block = [&](int l0) {
#pragma unroll
        for (int u = 0; u < B; ++u) {
            int i, j;
            long K = elem(l0 + u, i, j);
            K = K < 0 ? 0 : K;
#pragma unroll
            for (int b = 0; b < NB; ++b) pre[u][b] = S[K * N + ca + NB * b];
        }
    };
    auto park_block = [&](int buf) {
        if (slot < maxlen) {
#pragma unroll
            for (int u = 0; u < B; ++u)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    sch[((buf * B + u) * maxlen + slot) * N + ca + NB * b] = pre[u][b];
        }
    };
    fetch_block(0);
    park_block(0);
    lds_barrier();
    for (int l0 = 0, blk = 0; l0 < nlev; l0 += B, ++blk) {
        const int buf = blk & 1;
        fetch_block(l0 + B);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int l = l0 + u;
            if (l >= nlev) break;
            const int cur = l & 1, nxt = cur ^ 1;
            int ci, cj;
            const long K = elem(l, ci, cj);
            if (K >= 0) {
                const int cmat = MREG == 1 ? 0 : (int)msh[K];
                T sv[N], tx[NB], ty[NB];
                const T* sp = sch + ((buf * B + u) * maxlen + slot) * N;
#pragma unroll
                for (int c = 0; c < N; ++c) sv[c] = sp[c];
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    tx[c] = xtr[(cur * ny + cj) * NB + c];
                    ty[c] = ytr[(cur * nx + ci) * NB + c];
                }
                T acc[NB];
                auto apply = [&](const T (&rw)[NB][ROWW]) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        T v = T(0);
#pragma unroll
                        for (int c = 0; c < N; ++c) v += rw[b][c] * sv[c];
#pragma unroll
                        for (int c = 0; c < NB; ++c) v += rw[b][N + c] * tx[c] + rw[b][N + NB + c] * ty[c];
                        acc[b] = v;
                    }
                };
                if constexpr (MREG == 1) {
                    apply(reg[0]);
                } else if constexpr (MREG == 2) {
                    // materials are spatially coherent: take a wave-uniform branch
                    // whenever the wave's elements share one material
                    // The empty asm statements that consume the results end each
                    // branch differently, so the branches are not merged into
                    // per-operand selects.
                    const unsigned long long m1 = __ballot(cmat != 0);
                    const unsigned long long act = __ballot(1);
                    if (m1 == 0ull) {
                        apply(reg[0]);
#pragma unroll
                        for (int b = 0; b < NB; ++b) asm volatile("; material 0" : "+v"(acc[b]));
                    } else if (m1 == act) {
                        apply(reg[1]);
#pragma unroll
                        for (int b = 0; b < NB; ++b) asm volatile("; material 1" : "+v"(acc[b]));
                    } else {
                        T acc0[NB];
                        apply(reg[0]);
#pragma unroll
                        for (int b = 0; b < NB; ++b) acc0[b] = acc[b];
                        apply(reg[1]);
#pragma unroll
                        for (int b = 0; b < NB; ++b) acc[b] = cmat == 0 ? acc0[b] : acc[b];
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const T* row = tab + ((long)cmat * N + ca + NB * b) * ROWW;
                        T v = T(0);
#pragma unroll
                        for (int c = 0; c < N; ++c) v += row[c] * sv[c];
#pragma unroll
                        for (int c = 0; c < NB; ++c) v += row[N + c] * tx[c] + row[N + NB + c] * ty[c];
                        acc[b] = v;
                    }
                }
#pragma unroll
                for (int b = 0; b < NB; ++b) psi[K * N + ca + NB * b] = acc[b];
                if (ca == aout) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) xtr[(nxt * ny + cj) * NB + b] = acc[b];
                }
                ytr[(nxt * nx + ci) * NB + ca] = acc[bout];
            }
            lds_barrier();
        }
        park_block(buf ^ 1);
        lds_barrier();
    }
}

template <typename T, int NB, int MREG, int MAXT, int B>
__global__ __launch_bounds__(MAXT) void sweep_cart2_kernel(CartSweepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_cart_task<T, NB, MREG, B>(a, blockIdx.x, smem);
}

// levels whose source is fetched one block ahead (fewer for large elements,
// to keep the two staged blocks within the LDS of one workgroup)
__host__ __device__ constexpr int cart_block(int NB) { return NB <= 3 ? 6 : 3; }

template <typename T, int NB, int MREG, int MAXT>
static hipError_t launch_cart2_t(const CartSweepArgs& a, hipStream_t s, int threads, size_t lds) {
    constexpr int B = cart_block(NB);
    auto kfn = sweep_cart2_kernel<T, NB, MREG, MAXT, B>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kfn, dim3(a.nd), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// Returns hipErrorNotSupported when the column-per-thread kernel does not
// apply (anti-diagonal longer than the workgroup or LDS too small).
template <typename T, int NB>
static hipError_t try_cart2(const CartSweepArgs& a, hipStream_t s) {
    constexpr int N = NB * NB;
    const int maxlen = a.nx < a.ny ? a.nx : a.ny;
    int threads = ((maxlen * NB + 63) / 64) * 64;
    if (threads > 1024) return hipErrorNotSupported;
    // register-resident operator rows only where they fit without spilling
    constexpr bool f64 = sizeof(T) == 8;
    int mreg = 0;
    if (a.nmat == 1 && NB <= (f64 ? 3 : 4)) mreg = 1;
    else if (a.nmat == 2 && NB <= (f64 ? 2 : 3)) mreg = 2;
    size_t lds = sizeof(T) * (2 * (size_t)(a.nx + a.ny) * NB + 2 * (size_t)cart_block(NB) * maxlen * N);
    if (mreg == 0) lds += sizeof(T) * (size_t)a.nmat * N * (N + 2 * NB);
    if (mreg != 1) lds += (size_t)a.nx * a.ny;
    if (lds > 160 * 1024) return hipErrorNotSupported;
    if (threads <= 512) {
        if (mreg == 1) return launch_cart2_t<T, NB, 1, 512>(a, s, threads, lds);
        if constexpr (NB <= 3) {
            if (mreg == 2) return launch_cart2_t<T, NB, 2, 512>(a, s, threads, lds);
        }
        return launch_cart2_t<T, NB, 0, 512>(a, s, threads, lds);
    }
    if (f64 && NB >= 4) return hipErrorNotSupported;
    return launch_cart2_t<T, NB, 0, 1024>(a, s, threads, lds);
}

template <typename T, int NB>
static hipError_t launch_cart_any(const CartSweepArgs& a, hipStream_t s) {
    if (a.variant != 1) {
        hipError_t e = try_cart2<T, NB>(a, s);
        if (e != hipErrorNotSupported) return e;
    }
    return launch_cart_t<T, NB>(a, s);
}

hipError_t launch_sweep_cart(bool fp64, const CartSweepArgs& a, hipStream_t s) {
    switch (a.nb) {
        case 2: return fp64 ? launch_cart_any<double, 2>(a, s) : launch_cart_any<float, 2>(a, s);
        case 3: return fp64 ? launch_cart_any<double, 3>(a, s) : launch_cart_any<float, 3>(a, s);
        case 4: return fp64 ? launch_cart_any<double, 4>(a, s) : launch_cart_any<float, 4>(a, s);
        case 5: return fp64 ? launch_cart_any<double, 5>(a, s) : launch_cart_any<float, 5>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// General sweep.  Per element K and direction Omega (upwind DG, integrated by
// parts once, pointwise upwinding at the face Gauss points):
//   A_ij = sigma_t M_ij - Omega_x Gx_ij - Omega_y Gy_ij
//          + sum_f sum_q max(Omega.n_q, 0) u_i(q) u_j(q)
//   b_i  = sum_j M_ij S_j + sum_f sum_q max(-Omega.n_q, 0) u_i(q) psi_up(q)
// psi_up is the neighbour's trace (this sweep if the neighbour is upstream in
// the chord graph, else the previous sweep) or the inflow on the boundary.
// One wavefront per element: assembly, elimination without pivoting (the
// symmetric part of A is positive definite) and back substitution in LDS.
// One workgroup per (direction, tile): tiles of the parallel block Jacobi
// sweep are independent within a sweep (the graph has no edges between
// them), so each walks its own levels; without tiles the mesh is one tile.
// ---------------------------------------------------------------------------
constexpr int GEN_MAXQ = 12;
// waves per workgroup (one element each): as many as keep the per-wave LDS
// (the augmented n x (n+1) system, the solution, face data) within 64 KB
template <typename T, int NB>
constexpr int gen_waves() {
    constexpr int N = NB * NB;
    constexpr int per = (int)sizeof(T) * (N * (N + 1) + N + 8 * GEN_MAXQ);
    constexpr int w = (64 * 1024) / per;
    return w >= 16 ? 16 : (w >= 8 ? 8 : 4);
}

template <int NB>
__device__ __forceinline__ int face_pos(int f, int i) {
    const int a = i % NB, b = i / NB;
    switch (f) {
        case 0: return b == 0 ? a : -1;
        case 1: return a == NB - 1 ? b : -1;
        case 2: return b == NB - 1 ? a : -1;
        default: return a == 0 ? b : -1;
    }
}

template <int NB>
__device__ __forceinline__ int face_node(int f, int c) {
    switch (f) {
        case 0: return c;
        case 1: return (NB - 1) + NB * c;
        case 2: return c + NB * (NB - 1);
        default: return NB * c;
    }
}

template <typename T, int NB, int GEN_WAVES = gen_waves<T, NB>()>
__global__ __launch_bounds__(64 * GEN_WAVES) void sweep_general_kernel(GenSweepArgs a) {
    constexpr int N = NB * NB;
    const int d = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nq = a.nq, ne = a.ne;
    __shared__ T Aug[GEN_WAVES][N][N + 1];
    __shared__ T xs[GEN_WAVES][N];
    __shared__ T fval[GEN_WAVES][4][GEN_MAXQ];
    __shared__ T fon[GEN_WAVES][4][GEN_MAXQ];
    const T ox = (T)a.omega[d * 3], oy = (T)a.omega[d * 3 + 1];
    const T* S = reinterpret_cast<const T*>(a.S) + (a.s_aniso ? (long)d * ne * N : 0);
    const T* Mk = reinterpret_cast<const T*>(a.Mk);
    const T* Gx = reinterpret_cast<const T*>(a.Gx);
    const T* Gy = reinterpret_cast<const T*>(a.Gy);
    const T* nds = reinterpret_cast<const T*>(a.nds);
    const T* Lf = reinterpret_cast<const T*>(a.Lf);
    const T* st = reinterpret_cast<const T*>(a.sigma_t);
    const T* pbar = reinterpret_cast<const T*>(a.psibar);
    const T* plag = reinterpret_cast<const T*>(a.psi_lag);
    T* psi = reinterpret_cast<T*>(a.psi);
    const int* lp = a.lev_ptr + ((long)d * a.ntiles + blockIdx.y) * (a.nlev + 1);
    const int* le = a.lev_elem + (long)d * ne;
    for (int l = 0; l < a.nlev; ++l) {
        const int beg = lp[l], end = lp[l + 1];
        for (int base = beg; base < end; base += GEN_WAVES) {
            const int e = base + wv;
            const bool active = e < end;
            const int K = active ? le[e] : le[beg];
            // face Omega.n and inflow values at the face points
            if (lane < 4 * nq) {
                const int f = lane / nq, q = lane - f * nq;
                const T* nn = nds + (((long)K * 4 + f) * nq + q) * 2;
                const T on = ox * nn[0] + oy * nn[1];
                T val = T(0);
                if (on < T(0)) {
                    const int Nb = a.nbr[K * 4 + f];
                    if (Nb < 0) {
                        if (pbar) val = pbar[((long)d * a.nbf + a.bface_of[K * 4 + f]) * nq + q];
                    } else {
                        const bool up = (a.upflag[(long)d * ne + K] >> f) & 1;
                        const T* src = up ? psi : plag;
                        if (src) {
                            const int code = a.nbr_face ? (int)a.nbr_face[K * 4 + f] : ((f + 2) & 3);
                            const int fN = code & 3, qN = (code & 4) ? nq - 1 - q : q;
                            const T* sN = src + ((long)d * ne + Nb) * N;
                            for (int c = 0; c < NB; ++c) val += Lf[c * nq + qN] * sN[face_node<NB>(fN, c)];
                        }
                    }
                }
                fval[wv][f][q] = val;
                fon[wv][f][q] = on;
            }
            __builtin_amdgcn_wave_barrier();
            const T sK = st[K];
            const T* M = Mk + (long)K * N * N;
            const T* gx = Gx + (long)K * N * N;
            const T* gy = Gy + (long)K * N * N;
            for (int idx = lane; idx < N * N; idx += 64) {
                const int i = idx / N, j = idx - i * N;
                T v = sK * M[idx] - ox * gx[idx] - oy * gy[idx];
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const int ci = face_pos<NB>(f, i), cj = face_pos<NB>(f, j);
                    if (ci >= 0 && cj >= 0)
                        for (int q = 0; q < nq; ++q) {
                            const T on = fon[wv][f][q];
                            if (on > T(0)) v += on * Lf[ci * nq + q] * Lf[cj * nq + q];
                        }
                }
                Aug[wv][i][j] = v;
            }
            for (int i = lane; i < N; i += 64) {
                T b = T(0);
                const T* sk = S + (long)K * N;
                for (int j = 0; j < N; ++j) b += M[i * N + j] * sk[j];
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const int ci = face_pos<NB>(f, i);
                    if (ci >= 0)
                        for (int q = 0; q < nq; ++q) {
                            const T on = fon[wv][f][q];
                            if (on < T(0)) b -= on * Lf[ci * nq + q] * fval[wv][f][q];
                        }
                }
                Aug[wv][i][N] = b;
            }
            __builtin_amdgcn_wave_barrier();
            for (int k = 0; k < N; ++k) {
                const T rp = T(1) / Aug[wv][k][k];  // one division per lane and pivot
                const int w = N - k;  // columns k+1 .. N
                for (int idx = lane; idx < (N - 1 - k) * w; idx += 64) {
                    const int i = k + 1 + idx / w, j = k + 1 + idx % w;
                    Aug[wv][i][j] -= Aug[wv][i][k] * rp * Aug[wv][k][j];
                }
                __builtin_amdgcn_wave_barrier();
            }
            for (int k = N - 1; k >= 0; --k) {
                if (lane == 0) xs[wv][k] = Aug[wv][k][N] / Aug[wv][k][k];
                __builtin_amdgcn_wave_barrier();
                const T xk = xs[wv][k];
                for (int i = lane; i < k; i += 64) Aug[wv][i][N] -= Aug[wv][i][k] * xk;
                __builtin_amdgcn_wave_barrier();
            }
            if (active)
                for (int i = lane; i < N; i += 64) psi[((long)d * ne + K) * N + i] = xs[wv][i];
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
}

// The same per-element solve with one lane per element (p <= 2: the n x
// (n+1) augmented system stays in registers): a level's elements are spread
// over the workgroup's lanes, so a level of m elements costs one pass of
// ceil(m / 256) waves instead of m wave-solves.  Same assembly (volume, then
// faces in order), elimination without pivoting (one division per pivot) and
// back substitution by rows.
template <typename T, int NB, bool GENERAL>
__global__ __launch_bounds__(256) void sweep_lane_general_kernel(GenSweepArgs a) {
    constexpr int N = NB * NB;
    const int d = blockIdx.x;
    const int nq = a.nq, ne = a.ne;
    const T ox = (T)a.omega[d * 3], oy = (T)a.omega[d * 3 + 1];
    const T* S = reinterpret_cast<const T*>(a.S) + (a.s_aniso ? (long)d * ne * N : 0);
    const T* Mk = reinterpret_cast<const T*>(a.Mk);
    const T* Gx = reinterpret_cast<const T*>(a.Gx);
    const T* Gy = reinterpret_cast<const T*>(a.Gy);
    const T* nds = reinterpret_cast<const T*>(a.nds);
    const T* Lf = reinterpret_cast<const T*>(a.Lf);
    const T* st = reinterpret_cast<const T*>(a.sigma_t);
    const T* pbar = reinterpret_cast<const T*>(a.psibar);
    const T* plag = reinterpret_cast<const T*>(a.psi_lag);
    T* psi = reinterpret_cast<T*>(a.psi);
    const int* lp = a.lev_ptr + ((long)d * a.ntiles + blockIdx.y) * (a.nlev + 1);
    const int* le = a.lev_elem + (long)d * ne;
    for (int l = 0; l < a.nlev; ++l) {
        const int beg = lp[l], end = lp[l + 1];
        for (int e = beg + (int)threadIdx.x; e < end; e += (int)blockDim.x) {
            const int K = le[e];
            const T sK = st[K];
            const T* M = Mk + (long)K * N * N;
            const T* gx = Gx + (long)K * N * N;
            const T* gy = Gy + (long)K * N * N;
            const T* sk = S + (long)K * N;
            T A[N][N + 1];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T b = T(0);
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const T m = M[i * N + j];
                    A[i][j] = sK * m - ox * gx[i * N + j] - oy * gy[i * N + j];
                    b += m * sk[j];
                }
                A[i][N] = b;
            }
            const uint8_t up = a.upflag[(long)d * ne + K];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int Nb = a.nbr[K * 4 + f];
                const T* src = nullptr;
                if (Nb >= 0) src = ((up >> f) & 1) ? psi : plag;
                // the neighbour's face and orientation (a structured grid: the
                // opposite face, same way)
                const int code = GENERAL ? (int)a.nbr_face[K * 4 + f] : ((f + 2) & 3);
                const int fN = code & 3;
                const bool rev = GENERAL && (code & 4) != 0;
                for (int q = 0; q < nq; ++q) {
                    const T* nn = nds + (((long)K * 4 + f) * nq + q) * 2;
                    const T on = ox * nn[0] + oy * nn[1];
                    if (on > T(0)) {
#pragma unroll
                        for (int c = 0; c < NB; ++c)
#pragma unroll
                            for (int c2 = 0; c2 < NB; ++c2)
                                A[face_node<NB>(f, c)][face_node<NB>(f, c2)] += on * Lf[c * nq + q] * Lf[c2 * nq + q];
                    } else if (on < T(0)) {
                        T val = T(0);
                        if (Nb < 0) {
                            if (pbar) val = pbar[((long)d * a.nbf + a.bface_of[K * 4 + f]) * nq + q];
                        } else if (src) {
                            const T* sN = src + ((long)d * ne + Nb) * N;
                            const int qN = rev ? nq - 1 - q : q;
#pragma unroll
                            for (int c = 0; c < NB; ++c) val += Lf[c * nq + qN] * sN[face_node<NB>(fN, c)];
                        }
#pragma unroll
                        for (int c = 0; c < NB; ++c) A[face_node<NB>(f, c)][N] -= on * Lf[c * nq + q] * val;
                    }
                }
            }
            // one division per pivot; its reciprocal scales the multipliers
            // and the back substitution
            T inv[N];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                inv[k] = T(1) / A[k][k];
#pragma unroll
                for (int i = k + 1; i < N; ++i) {
                    const T m = A[i][k] * inv[k];
#pragma unroll
                    for (int j = k + 1; j <= N; ++j) A[i][j] -= m * A[k][j];
                }
            }
            T x[N];
#pragma unroll
            for (int k = N - 1; k >= 0; --k) {
                T v = A[k][N];
#pragma unroll
                for (int j = k + 1; j < N; ++j) v -= A[k][j] * x[j];
                x[k] = v * inv[k];
            }
            T* out = psi + ((long)d * ne + K) * N;
#pragma unroll
            for (int i = 0; i < N; ++i) out[i] = x[i];
        }
        __syncthreads();
    }
}

// value of v in lane src (ds_bpermute), FP32 or FP64
__device__ __forceinline__ float shfl_t(float v, int src) { return __shfl(v, src); }
__device__ __forceinline__ double shfl_t(double v, int src) { return __shfl(v, src); }

// The same per-element solve with one lane per row: a wave holds 64 / N
// elements (N = (p+1)^2 lanes each; 7, 4, 2 elements at p = 2, 3, 4), lane i
// assembles row i of its element's augmented system [A | b] in registers
// (volume terms, then the faces through node i in order), and the system is
// reduced by Gauss-Jordan elimination without pivoting: for each pivot k every
// other lane of the element reads row k from the lane holding it (lane
// shuffles) and subtracts its multiple, so no back substitution is needed;
// x_i = b_i / A_ii.  The pivot loop is unrolled (register indices are
// compile-time).  Face data are staged first: the element's lanes compute
// Omega.n ds and the upwind trace at all 4 nq face points together (one
// round of independent loads) into LDS, where the face terms read them.  A
// level of m elements takes ceil(m / (64 / N)) wave-solves spread over the
// workgroup's waves.
template <typename T, int NB, int WAVES, bool GENERAL>
__global__ __launch_bounds__(64 * WAVES) void sweep_rows_general_kernel(GenSweepArgs a) {
    constexpr int N = NB * NB;
    constexpr int EPW = 64 / N;   // elements per wave
    const int d = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int eslot = lane / N;           // element of this lane within the wave
    const int i = lane - eslot * N;       // row of this lane
    const bool lane_ok = eslot < EPW;
    const int es = lane_ok ? eslot : 0;
    const int nq = a.nq, ne = a.ne;
    __shared__ T fon[WAVES][EPW][4 * GEN_MAXQ];    // Omega.n (weighted ds) at the face points
    __shared__ T fval[WAVES][EPW][4 * GEN_MAXQ];   // upwind trace at the inflow points
    __shared__ T lfs[NB * GEN_MAXQ];               // face basis at the face points
    const T ox = (T)a.omega[d * 3], oy = (T)a.omega[d * 3 + 1];
    const T* S = reinterpret_cast<const T*>(a.S) + (a.s_aniso ? (long)d * ne * N : 0);
    const T* Mk = reinterpret_cast<const T*>(a.Mk);
    const T* Gx = reinterpret_cast<const T*>(a.Gx);
    const T* Gy = reinterpret_cast<const T*>(a.Gy);
    const T* nds = reinterpret_cast<const T*>(a.nds);
    const T* st = reinterpret_cast<const T*>(a.sigma_t);
    const T* pbar = reinterpret_cast<const T*>(a.psibar);
    const T* plag = reinterpret_cast<const T*>(a.psi_lag);
    T* psi = reinterpret_cast<T*>(a.psi);
    for (int t = threadIdx.x; t < NB * nq; t += blockDim.x) lfs[t] = reinterpret_cast<const T*>(a.Lf)[t];
    __syncthreads();
    const int* lp = a.lev_ptr + ((long)d * a.ntiles + blockIdx.y) * (a.nlev + 1);
    const int* le = a.lev_elem + (long)d * ne;
    for (int l = 0; l < a.nlev; ++l) {
        const int beg = lp[l], end = lp[l + 1];
        for (int base = beg; base < end; base += WAVES * EPW) {
            const int e = base + wv * EPW + eslot;
            const bool act = lane_ok && e < end;
            const int K = act ? le[e] : le[beg];
            // face data of the element, all points at once
            if (lane_ok) {
                const uint8_t up = a.upflag[(long)d * ne + K];
                for (int t = i; t < 4 * nq; t += N) {
                    const int f = t / nq, q = t - f * nq;
                    const T* nn = nds + (((long)K * 4 + f) * nq + q) * 2;
                    const T on = ox * nn[0] + oy * nn[1];
                    T val = T(0);
                    if (on < T(0)) {
                        const int Nb = a.nbr[K * 4 + f];
                        if (Nb < 0) {
                            if (pbar) val = pbar[((long)d * a.nbf + a.bface_of[K * 4 + f]) * nq + q];
                        } else {
                            const T* src = ((up >> f) & 1) ? psi : plag;
                            if (src) {
                                const int code = GENERAL ? (int)a.nbr_face[K * 4 + f] : ((f + 2) & 3);
                                const int fN = code & 3;
                                const int qN = (GENERAL && (code & 4)) ? nq - 1 - q : q;
                                const T* sN = src + ((long)d * ne + Nb) * N;
#pragma unroll
                                for (int c = 0; c < NB; ++c) val += lfs[c * nq + qN] * sN[face_node<NB>(fN, c)];
                            }
                        }
                    }
                    fon[wv][es][t] = on;
                    fval[wv][es][t] = val;
                }
            }
            // row i of [A | b]: volume terms
            T A[N + 1];
            {
                const T sK = st[K];
                const T* M = Mk + ((long)K * N + i) * N;
                const T* gx = Gx + ((long)K * N + i) * N;
                const T* gy = Gy + ((long)K * N + i) * N;
                const T* sk = S + (long)K * N;
                T b = T(0);
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const T m = M[j];
                    A[j] = sK * m - ox * gx[j] - oy * gy[j];
                    b += m * sk[j];
                }
                A[N] = b;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // faces through node i: outflow points couple node i to the face's
            // nodes, inflow points bring the upwind trace
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int c = face_pos<NB>(f, i);
                if (c < 0) continue;
                for (int q = 0; q < nq; ++q) {
                    const T on = fon[wv][es][f * nq + q];
                    const T lc = lfs[c * nq + q];
                    if (on > T(0)) {
#pragma unroll
                        for (int c2 = 0; c2 < NB; ++c2) A[face_node<NB>(f, c2)] += on * lc * lfs[c2 * nq + q];
                    } else if (on < T(0)) {
                        A[N] -= on * lc * fval[wv][es][f * nq + q];
                    }
                }
            }
            // Gauss-Jordan elimination, one pivot at a time: the pivot row's
            // entries come from the lane holding it by lane shuffles
            T diag = T(1);
            const int r0 = es * N;   // lane of row 0 of this lane's element
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const T piv = shfl_t(A[k], r0 + k);
                if (i == k) diag = piv;
                const T m = i == k ? T(0) : A[k] / piv;
#pragma unroll
                for (int j = k + 1; j <= N; ++j) A[j] -= m * shfl_t(A[j], r0 + k);
            }
            if (act) psi[((long)d * ne + K) * N + i] = A[N] / diag;
            // the face data of the next element group overwrite fon / fval
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
}

template <typename T, int NB, bool GENERAL>
static hipError_t launch_rows_g(const GenSweepArgs& a, hipStream_t s) {
    constexpr int N = NB * NB;
    constexpr int EPW = 64 / N;
    // as many waves as the widest level needs, at most 16 (8 in FP64, whose
    // rows need more than the 128 VGPRs a 16-wave workgroup leaves a lane)
    const int need = (a.maxw + EPW - 1) / EPW;
    if constexpr (sizeof(T) == 4) {
        if (need > 8) {
            hipLaunchKernelGGL((sweep_rows_general_kernel<T, NB, 16, GENERAL>), dim3(a.nd, a.ntiles), dim3(1024), 0,
                               s, a);
            return hipGetLastError();
        }
    }
    if (need > 4)
        hipLaunchKernelGGL((sweep_rows_general_kernel<T, NB, 8, GENERAL>), dim3(a.nd, a.ntiles), dim3(512), 0, s, a);
    else if (need > 2)
        hipLaunchKernelGGL((sweep_rows_general_kernel<T, NB, 4, GENERAL>), dim3(a.nd, a.ntiles), dim3(256), 0, s, a);
    else if (need > 1)
        hipLaunchKernelGGL((sweep_rows_general_kernel<T, NB, 2, GENERAL>), dim3(a.nd, a.ntiles), dim3(128), 0, s, a);
    else
        hipLaunchKernelGGL((sweep_rows_general_kernel<T, NB, 1, GENERAL>), dim3(a.nd, a.ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename T, int NB>
static hipError_t launch_rows_t(const GenSweepArgs& a, hipStream_t s) {
    return a.nbr_face ? launch_rows_g<T, NB, true>(a, s) : launch_rows_g<T, NB, false>(a, s);
}

template <typename T, int NB>
static hipError_t launch_inv_t(const GenSweepArgs& a, hipStream_t s);

template <typename T, int NB>
static hipError_t launch_gen_t(const GenSweepArgs& a, hipStream_t s) {
    if (a.nq > GEN_MAXQ || 4 * a.nq > 64) return hipErrorInvalidValue;
    if (a.invA) return launch_inv_t<T, NB>(a, s);
    if constexpr (NB >= 3) {
        // one lane per row: the default at p >= 3; at p = 2 where levels are
        // narrow or workgroups few (the lane-per-element form wins only with
        // wide levels spread over many tiles: measured 0.84 against 1.15 ms on
        // 32^2 tiles of the 128^2 channel, 0.79 against 0.61 ms on the whole
        // curved 32^2 mesh, 1.82 against 0.88 ms on 8^2 tiles); path 4 at p = 2
        const bool rows_p2 = a.maxw <= 16 || (long)a.nd * a.ntiles < 1024;
        if (a.wave_solve == 2 || (a.wave_solve == 0 && (NB >= 4 || rows_p2))) return launch_rows_t<T, NB>(a, s);
    }
    // few workgroups (whole-mesh sweeps: one per direction) take the widest
    // workgroup their levels fill; many (tiles) take 4 waves, so that more
    // workgroups share each CU
    constexpr int WV = gen_waves<T, NB>();
    // p <= 2: one lane per element, in a workgroup of as many waves as the
    // widest level needs (at most 4), so that idle waves take no CU slots;
    // with 8 x 8 tiles (levels of at most 8 elements) this still beats the
    // wave-wide solve, since 8 such workgroups share a CU
    if constexpr (NB <= 3) {
        if (a.wave_solve != 1) {
            const int threads = std::min(256, std::max(64, (a.maxw + 63) / 64 * 64));
            if (a.nbr_face)
                hipLaunchKernelGGL((sweep_lane_general_kernel<T, NB, true>), dim3(a.nd, a.ntiles), dim3(threads), 0,
                                   s, a);
            else
                hipLaunchKernelGGL((sweep_lane_general_kernel<T, NB, false>), dim3(a.nd, a.ntiles), dim3(threads), 0,
                                   s, a);
            return hipGetLastError();
        }
    }
    if (a.nd * a.ntiles < 512 && a.maxw > 4)
        hipLaunchKernelGGL((sweep_general_kernel<T, NB, WV>), dim3(a.nd, a.ntiles), dim3(64 * WV), 0, s, a);
    else
        hipLaunchKernelGGL((sweep_general_kernel<T, NB, 4>), dim3(a.nd, a.ntiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sweep_general(bool fp64, const GenSweepArgs& a, hipStream_t s) {
    switch (a.nb) {
        case 2: return fp64 ? launch_gen_t<double, 2>(a, s) : launch_gen_t<float, 2>(a, s);
        case 3: return fp64 ? launch_gen_t<double, 3>(a, s) : launch_gen_t<float, 3>(a, s);
        case 4: return fp64 ? launch_gen_t<double, 4>(a, s) : launch_gen_t<float, 4>(a, s);
        case 5: return fp64 ? launch_gen_t<double, 5>(a, s) : launch_gen_t<float, 5>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// General sweep with stored element operators.  The left-hand side of an
// element's system (the volume terms and the outflow face terms above)
// depends on the element, the direction and sigma_t but not on the upwind
// data, so it is inverted once, in parallel over every (element, direction)
// pair, and what a sweep needs of A^-1 is kept in device memory:
//   invA   [nd][ne][N][N]      H = A^-1 M by column j, then row i (the lanes
//                              of an element read a column together)
//   invC   [nd][ne][N]         c = A^-1 r, r the boundary inflow terms
//   invG   [nd][ne][N][4][NB]  row i of G_f for every face (a lane's values
//                              contiguous), where for a face f with a
//                              neighbour and an inflow point
//                              G_f = A^-1 E_f F_f with
//                              F_f[c][c'] = sum over the inflow points q of
//                              |Omega.n_q| u_c(q) u_c'(q'), q' the same point
//                              in the neighbour's face numbering, so that the
//                              neighbour's face-node values v enter psi_K as
//                              G_f v (E_f places face node c at its element
//                              node); zero for the other faces
//   inmask [nd][ne]            bit f set when face f has a neighbour and an
//                              inflow point
// A sweep is then psi_K = H S_K + c for all elements at once
// (gen_inv_particular_kernel), followed by the levels in order, each adding
// sum_f G_f v_f from the finished upwind neighbours (gen_inv_sweep_kernel).
// Same lane layout as the row kernel: lane i of an element's N lanes holds
// row i.
// ---------------------------------------------------------------------------
template <typename TO, int NB, bool GENERAL>
__global__ __launch_bounds__(256) void gen_inv_setup_kernel(GenSweepArgs a, TO* invA, TO* invC, TO* invG,
                                                            uint8_t* inmask) {
    constexpr int N = NB * NB;
    constexpr int EPW = 64 / N;
    const int d = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int eslot = lane / N;
    const int i = lane - eslot * N;
    const bool lane_ok = eslot < EPW;
    const int es = lane_ok ? eslot : 0;
    const int nq = a.nq, ne = a.ne;
    const int Kr = (blockIdx.x * 4 + wv) * EPW + es;
    const bool act = lane_ok && Kr < ne;
    const int K = act ? Kr : 0;
    __shared__ double fon[4][EPW][4 * GEN_MAXQ];
    __shared__ double lfs[NB * GEN_MAXQ];
    const double* Lf = reinterpret_cast<const double*>(a.Lf);
    const double* nds = reinterpret_cast<const double*>(a.nds);
    const double* Mk = reinterpret_cast<const double*>(a.Mk) + (long)K * N * N;
    const double* pbar = reinterpret_cast<const double*>(a.psibar);
    for (int t = threadIdx.x; t < NB * nq; t += blockDim.x) lfs[t] = Lf[t];
    const double ox = a.omega[d * 3], oy = a.omega[d * 3 + 1];
    if (lane_ok)
        for (int t = i; t < 4 * nq; t += N) {
            const double* nn = nds + (((long)K * 4 + t / nq) * nq + t % nq) * 2;
            fon[wv][es][t] = ox * nn[0] + oy * nn[1];
        }
    __syncthreads();
    // row i of A: volume terms, then the outflow points of the faces through
    // node i; r_i: the inflow points of its boundary faces (all in FP64
    // whatever the stored type)
    double A[N], E[N];
    {
        const double sK = reinterpret_cast<const double*>(a.sigma_t)[K];
        const double* gx = reinterpret_cast<const double*>(a.Gx) + ((long)K * N + i) * N;
        const double* gy = reinterpret_cast<const double*>(a.Gy) + ((long)K * N + i) * N;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            A[j] = sK * Mk[i * N + j] - ox * gx[j] - oy * gy[j];
            E[j] = j == i ? 1.0 : 0.0;
        }
    }
    double r = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int c = face_pos<NB>(f, i);
        if (c < 0) continue;
        const bool bdr = a.nbr[K * 4 + f] < 0 && pbar;
        const double* pb = bdr ? pbar + ((long)d * a.nbf + a.bface_of[K * 4 + f]) * nq : nullptr;
        for (int q = 0; q < nq; ++q) {
            const double on = fon[wv][es][f * nq + q];
            const double lc = lfs[c * nq + q];
            if (on > 0.0) {
#pragma unroll
                for (int c2 = 0; c2 < NB; ++c2) A[face_node<NB>(f, c2)] += on * lc * lfs[c2 * nq + q];
            } else if (on < 0.0 && bdr) {
                r -= on * lc * pb[q];
            }
        }
    }
    // Gauss-Jordan on [A | I] without pivoting (as in the row kernel); before
    // pivot k the identity columns past k are untouched, so only columns
    // 0..k of the right block take the update
    double diag = 1.0;
    const int r0 = es * N;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double piv = shfl_t(A[k], r0 + k);
        if (i == k) diag = piv;
        const double m = i == k ? 0.0 : A[k] / piv;
#pragma unroll
        for (int j = k + 1; j < N; ++j) A[j] -= m * shfl_t(A[j], r0 + k);
#pragma unroll
        for (int j = 0; j <= k; ++j) E[j] -= m * shfl_t(E[j], r0 + k);
    }
    const double rd = 1.0 / diag;
#pragma unroll
    for (int j = 0; j < N; ++j) E[j] *= rd;   // row i of A^-1
    const long dK = (long)d * ne + K;
    // row i of H = A^-1 M and c = A^-1 r
    double cval = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) cval += E[k] * shfl_t(r, r0 + k);
    if (act) invC[dK * N + i] = (TO)cval;
    for (int j = 0; j < N; ++j) {
        double h = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) h += E[k] * Mk[k * N + j];
        if (act) invA[(dK * N + j) * N + i] = (TO)h;
    }
    unsigned mask = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int Nb = a.nbr[K * 4 + f];
        bool inflow = false;
        for (int q = 0; q < nq; ++q) inflow |= fon[wv][es][f * nq + q] < 0.0;
        const bool use = Nb >= 0 && inflow;
        const int code = GENERAL ? (int)a.nbr_face[K * 4 + f] : ((f + 2) & 3);
        const bool flip = GENERAL && (code & 4);
#pragma unroll
        for (int c2 = 0; c2 < NB; ++c2) {
            double g = 0.0;
            if (use) {
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    double F = 0.0;
                    for (int q = 0; q < nq; ++q) {
                        const double on = fon[wv][es][f * nq + q];
                        const int qN = flip ? nq - 1 - q : q;
                        if (on < 0.0) F -= on * lfs[c * nq + q] * lfs[c2 * nq + qN];
                    }
                    g += E[face_node<NB>(f, c)] * F;
                }
            }
            if (act) invG[(dK * N + i) * 4 * NB + f * NB + c2] = (TO)g;
        }
        if (use) mask |= 1u << f;
    }
    if (act && i == 0) inmask[dK] = (uint8_t)mask;
}

// psi_K = H S_K (+ c when the sweep takes the boundary inflow) for every
// element and direction: the part of the element solution that needs no
// upwind element.  Every load is independent of the others.
template <typename T, int NB>
__global__ __launch_bounds__(256) void gen_inv_particular_kernel(GenSweepArgs a) {
    constexpr int N = NB * NB;
    constexpr int EPW = 64 / N;
    const int d = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int eslot = lane / N;
    const int i = lane - eslot * N;
    const bool lane_ok = eslot < EPW;
    const int es = lane_ok ? eslot : 0;
    const int ne = a.ne;
    const int Kr = (blockIdx.x * 4 + wv) * EPW + es;
    const bool act = lane_ok && Kr < ne;
    const int K = act ? Kr : 0;
    const long dK = (long)d * ne + K;
    const gcptr<T> S = as_global(reinterpret_cast<const T*>(a.S)) + (a.s_aniso ? (long)d * ne * N : 0) + (long)K * N;
    const gcptr<T> H = as_global(reinterpret_cast<const T*>(a.invA)) + dK * N * N + i;
    T x = a.psibar ? as_global(reinterpret_cast<const T*>(a.invC))[dK * N + i] : T(0);
#pragma unroll
    for (int j = 0; j < N; ++j) x += H[(long)j * N] * S[j];
    if (act) as_global(reinterpret_cast<T*>(a.psi))[dK * N + i] = x;
}

// What a lane needs of its element for the level pass, loaded one work item
// ahead: the element, its inflow mask and graph bits, its neighbours and
// their face numbering, psi from the parallel pass and its row of G (4 NB
// contiguous values, loaded as 16-byte vectors).
template <typename T, int NB>
struct InvItem {
    static constexpr int NG = 4 * NB;
    static constexpr int NV = NG / Vec16<T>::n;        // 16-byte vectors in a row of G
    static constexpr int VPL = (NG + NB * NB - 1) / (NB * NB);   // face values a lane loads
    int K;
    unsigned m, up;
    int nb[VPL];         // the neighbour across the face of each of the lane's face values
    unsigned code[VPL];  // and its face number (bit 2: its points run the other way)
    T x;
    T g[NG];
};

// The levels: psi_K += sum over the faces of inmask of G_f v_f, v_f the
// neighbour's face nodes from this sweep (upstream in the graph) or the
// lagged one.  One workgroup per (direction, tile) as in the row kernel; the
// work items (a level, or a workgroup-wide share of a wide level) are taken
// in order, the next one's data loaded while the current one waits for its
// neighbours.  Each of the 4 NB face values of an element is loaded once, by
// one of its lanes (zero for faces without inflow from a neighbour), and
// handed to the others through LDS.
template <typename T, int NB, int WAVES, bool GENERAL>
__global__ __launch_bounds__(64 * WAVES) void gen_inv_sweep_kernel(GenSweepArgs a) {
    constexpr int N = NB * NB;
    constexpr int EPW = 64 / N;
    constexpr int PER = WAVES * EPW;
    constexpr int NG = InvItem<T, NB>::NG;
    constexpr int NV = InvItem<T, NB>::NV;
    constexpr int VPL = InvItem<T, NB>::VPL;
    typedef typename Vec16<T>::type VT;
    static_assert(NG % Vec16<T>::n == 0, "rows of G come in 16-byte vectors");
    const int d = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int eslot = lane / N;
    const int i = lane - eslot * N;
    const bool lane_ok = eslot < EPW;
    const int es = lane_ok ? eslot : 0;
    const int slot = wv * EPW + eslot;
    const int ne = a.ne;
    __shared__ __attribute__((aligned(16))) T vs[WAVES][EPW][NG];
    const gcptr<VT> G = as_global(reinterpret_cast<const VT*>(a.invG));
    const gcptr<T> plag = as_global(reinterpret_cast<const T*>(a.psi_lag));
    const gptr<T> psi = as_global(reinterpret_cast<T*>(a.psi));
    const gcptr<uint8_t> inm = as_global(a.inmask) + (long)d * ne;
    const gcptr<uint8_t> upf = as_global(a.upflag) + (long)d * ne;
    const gcptr<int> nbr = as_global(a.nbr);
    const gcptr<uint8_t> nbfc = as_global(a.nbr_face);
    const int* lp = a.lev_ptr + ((long)d * a.ntiles + blockIdx.y) * (a.nlev + 1);
    const gcptr<int> le = as_global(a.lev_elem) + (long)d * ne;
    // work items in order: (level l, first position base, end of the level);
    // past the last level an item is empty
    struct Pos {
        int l, base, end;
    };
    auto advance = [&](const Pos& p) __attribute__((always_inline)) {
        Pos q = p;
        if (q.l >= a.nlev) return q;
        q.base += PER;
        if (q.base >= q.end) {
            ++q.l;
            q.base = q.end;
            q.end = q.l < a.nlev ? lp[q.l + 1] : q.end;
        }
        return q;
    };
    auto loadK = [&](const Pos& p) __attribute__((always_inline)) {
        const int e = p.base + slot;
        return p.l < a.nlev && lane_ok && e < p.end ? le[e] : -1;
    };
    auto loadData = [&](int Kr, InvItem<T, NB>& it) __attribute__((always_inline)) {
        it.K = Kr;
        const int K = Kr < 0 ? 0 : Kr;
        const long dK = (long)d * ne + K;
        it.m = inm[K];
        it.up = upf[K];
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
            const int t = r * N + i;
            const int f = (t < NG ? t : 0) / NB;
            it.nb[r] = nbr[K * 4 + f];
            it.code[r] = GENERAL ? (unsigned)nbfc[K * 4 + f] : (unsigned)((f + 2) & 3);
        }
        it.x = psi[dK * N + i];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const VT w = G[(dK * N + i) * NV + q];
#pragma unroll
            for (int k = 0; k < Vec16<T>::n; ++k) it.g[q * Vec16<T>::n + k] = w[k];
        }
    };
    if (a.nlev < 1) return;
    // P0: the item being solved (its data in X), P1: the next one (its element
    // in kY), P2: the one after (its element loaded into kX while X is in use)
    Pos P0{0, lp[0], lp[1]};
    Pos P1 = advance(P0);
    Pos P2 = advance(P1);
    InvItem<T, NB> A, B;
    int kA = 0, kB = loadK(P1);
    loadData(loadK(P0), A);
    // One item: the face values are loaded first, then the element two items
    // ahead and the next item's data, so that waiting for the face values
    // leaves those in flight (the load counter drains in issue order); the two
    // item buffers swap roles from one call to the next, so no register copy
    // waits for a load.
    auto item = [&](InvItem<T, NB>& X, InvItem<T, NB>& Y, int& kX, int& kY) __attribute__((always_inline)) {
        T fv[VPL];
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
            const int t = r * N + i;
            fv[r] = T(0);
            if (X.K >= 0 && t < NG) {
                const int f = t / NB, c = t - f * NB;
                const bool upstream = (X.up >> f) & 1;
                const bool ok = ((X.m >> f) & 1) && (upstream || plag);
                const gcptr<T> src = upstream ? gcptr<T>(psi) : plag;
                const int fN = (int)(X.code[r] & 3);
                const int node = fN == 0 ? c : (fN == 1 ? NB - 1 + NB * c : (fN == 2 ? c + NB * (NB - 1) : NB * c));
                if (ok) fv[r] = src[((long)d * ne + X.nb[r]) * N + node];
            }
        }
        kX = loadK(P2);
        loadData(kY, Y);
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
            const int t = r * N + i;
            if (lane_ok && t < NG) vs[wv][es][t] = fv[r];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (X.K >= 0) {
            T x = X.x;
#pragma unroll
            for (int t = 0; t < NG; ++t) x += X.g[t] * vs[wv][es][t];
            psi[((long)d * ne + X.K) * N + i] = x;
        }
        // the next item's face values overwrite vs
        __builtin_amdgcn_wave_barrier();
        if (P1.l != P0.l) __syncthreads();
        P0 = P1;
        P1 = P2;
        P2 = advance(P2);
    };
    while (P0.l < a.nlev) {
        item(A, B, kA, kB);
        if (P0.l >= a.nlev) break;
        item(B, A, kB, kA);
    }
}

template <typename TO, int NB>
static hipError_t launch_inv_setup_t(const GenSweepArgs& a, void* invA, void* invC, void* invG, uint8_t* inmask,
                                     hipStream_t s) {
    constexpr int EPW = 64 / (NB * NB);
    const dim3 grid((a.ne + 4 * EPW - 1) / (4 * EPW), a.nd);
    if (a.nbr_face)
        hipLaunchKernelGGL((gen_inv_setup_kernel<TO, NB, true>), grid, dim3(256), 0, s, a, (TO*)invA, (TO*)invC,
                           (TO*)invG, inmask);
    else
        hipLaunchKernelGGL((gen_inv_setup_kernel<TO, NB, false>), grid, dim3(256), 0, s, a, (TO*)invA, (TO*)invC,
                           (TO*)invG, inmask);
    return hipGetLastError();
}

hipError_t launch_gen_inv_setup(bool out_fp64, const GenSweepArgs& a, void* invA, void* invC, void* invG,
                                uint8_t* inmask, hipStream_t s) {
    if (a.nq > GEN_MAXQ || 4 * a.nq > 64) return hipErrorInvalidValue;
    switch (a.nb) {
        case 2: return out_fp64 ? launch_inv_setup_t<double, 2>(a, invA, invC, invG, inmask, s)
                                : launch_inv_setup_t<float, 2>(a, invA, invC, invG, inmask, s);
        case 3: return out_fp64 ? launch_inv_setup_t<double, 3>(a, invA, invC, invG, inmask, s)
                                : launch_inv_setup_t<float, 3>(a, invA, invC, invG, inmask, s);
        case 4: return out_fp64 ? launch_inv_setup_t<double, 4>(a, invA, invC, invG, inmask, s)
                                : launch_inv_setup_t<float, 4>(a, invA, invC, invG, inmask, s);
        case 5: return out_fp64 ? launch_inv_setup_t<double, 5>(a, invA, invC, invG, inmask, s)
                                : launch_inv_setup_t<float, 5>(a, invA, invC, invG, inmask, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int NB, bool GENERAL>
static hipError_t launch_inv_levels(const GenSweepArgs& a, hipStream_t s) {
    constexpr int EPW = 64 / (NB * NB);
    const int need = (a.maxw + EPW - 1) / EPW;
    const dim3 grid(a.nd, a.ntiles);
    // 16 waves leave 128 VGPRs a lane, too few for two FP64 work items at p = 4
    constexpr bool wide_ok = !(sizeof(T) == 8 && NB >= 5);
    if constexpr (wide_ok) {
        if (need > 8) {
            hipLaunchKernelGGL((gen_inv_sweep_kernel<T, NB, 16, GENERAL>), grid, dim3(1024), 0, s, a);
            return hipGetLastError();
        }
    }
    if (need > 4)
        hipLaunchKernelGGL((gen_inv_sweep_kernel<T, NB, 8, GENERAL>), grid, dim3(512), 0, s, a);
    else if (need > 2)
        hipLaunchKernelGGL((gen_inv_sweep_kernel<T, NB, 4, GENERAL>), grid, dim3(256), 0, s, a);
    else if (need > 1)
        hipLaunchKernelGGL((gen_inv_sweep_kernel<T, NB, 2, GENERAL>), grid, dim3(128), 0, s, a);
    else
        hipLaunchKernelGGL((gen_inv_sweep_kernel<T, NB, 1, GENERAL>), grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

// part 1: the particular pass, 2: the levels, 3: both
template <typename T, int NB>
static hipError_t launch_inv_part_t(const GenSweepArgs& a, int part, hipStream_t s) {
    constexpr int EPW = 64 / (NB * NB);
    if (part & 1) {
        hipLaunchKernelGGL((gen_inv_particular_kernel<T, NB>), dim3((a.ne + 4 * EPW - 1) / (4 * EPW), a.nd),
                           dim3(256), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (part & 2) return a.nbr_face ? launch_inv_levels<T, NB, true>(a, s) : launch_inv_levels<T, NB, false>(a, s);
    return hipSuccess;
}

template <typename T, int NB>
static hipError_t launch_inv_t(const GenSweepArgs& a, hipStream_t s) {
    return launch_inv_part_t<T, NB>(a, 3, s);
}

hipError_t launch_gen_inv_part(bool fp64, const GenSweepArgs& a, int part, hipStream_t s) {
    if (!a.invA || a.nq > GEN_MAXQ || 4 * a.nq > 64 || part < 1 || part > 3) return hipErrorInvalidValue;
    switch (a.nb) {
        case 2: return fp64 ? launch_inv_part_t<double, 2>(a, part, s) : launch_inv_part_t<float, 2>(a, part, s);
        case 3: return fp64 ? launch_inv_part_t<double, 3>(a, part, s) : launch_inv_part_t<float, 3>(a, part, s);
        case 4: return fp64 ? launch_inv_part_t<double, 4>(a, part, s) : launch_inv_part_t<float, 4>(a, part, s);
        case 5: return fp64 ? launch_inv_part_t<double, 5>(a, part, s) : launch_inv_part_t<float, 5>(a, part, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Angular moments on the matrix cores: mom[row][c] = sum_d W[row][d] psi[d][c]
// for rows phi, J_x, J_y, P_xx, P_xy, P_yy, sum w|O_x|, sum w|O_y| (rows 8-15
// of the 16x16 tile are zero).  One wavefront per 16 columns; the 16x16x4
// MFMA takes A[i][k] from lane i + 16 k and B[k][j] from lane j + 16 k; the
// FP32 variant returns D[i][j] in lane j + 16 (i / 4), element i % 4.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void moments_f32_kernel(const float* __restrict__ psi, int nd, long L,
                                                          const float* __restrict__ W, int ldw,
                                                          double* __restrict__ mom) {
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long col0 = wave * 16;
    if (col0 >= L) return;
    const int i = lane & 15, kk = lane >> 4;
    const bool colok = col0 + i < L;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < nd; k += 4) {
        const int dk = k + kk;
        const float av = dk < nd ? W[i * ldw + dk] : 0.f;
        const float bv = (dk < nd && colok) ? psi[(long)dk * L + col0 + i] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    if (kk < 2 && colok) {
#pragma unroll
        for (int r = 0; r < 4; ++r) mom[(long)(4 * kk + r) * L + col0 + i] = (double)acc[r];
    }
}

__global__ __launch_bounds__(256) void moments_f64_kernel(const double* __restrict__ psi, int nd, long L,
                                                          const double* __restrict__ W, int ldw,
                                                          double* __restrict__ mom) {
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long col0 = wave * 16;
    if (col0 >= L) return;
    const int i = lane & 15, kk = lane >> 4;
    const bool colok = col0 + i < L;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nd; k += 4) {
        const int dk = k + kk;
        const double av = dk < nd ? W[i * ldw + dk] : 0.0;
        const double bv = (dk < nd && colok) ? psi[(long)dk * L + col0 + i] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    // the FP64 variant returns D[i][j] in lane j + 16 (i % 4), element i / 4
    if (colok) {
#pragma unroll
        for (int r = 0; r < 2; ++r) mom[(long)(kk + 4 * r) * L + col0 + i] = acc[r];
    }
}

// Wide variant (L divisible by 4): one wavefront covers 64 columns; lane
// (j, k) loads psi[d + k][col0 + 4 j .. 4 j + 3] with one 16-byte (FP32) or
// two 16-byte (FP64) loads and feeds component t to MFMA tile t, so tile t
// holds columns col0 + 4 j + t and each lane stores 4 adjacent columns.
__global__ __launch_bounds__(256) void moments_f32_wide_kernel(const float* __restrict__ psi, int nd, long L,
                                                               const float* __restrict__ W, int ldw,
                                                               double* __restrict__ mom) {
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long col0 = wave * 64;
    if (col0 >= L) return;
    const int j = lane & 15, kk = lane >> 4;
    const long c4 = col0 + 4 * j;
    const bool colok = c4 < L;  // L % 4 == 0, so c4 < L implies c4 + 3 < L
    v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
    for (int k = 0; k < nd; k += 4) {
        const int dk = k + kk;
        const float av = dk < nd ? W[j * ldw + dk] : 0.f;
        v4f bv = {0.f, 0.f, 0.f, 0.f};
        if (dk < nd && colok) bv = *reinterpret_cast<const v4f*>(psi + (long)dk * L + c4);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[1], acc1, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[2], acc2, 0, 0, 0);
        acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[3], acc3, 0, 0, 0);
    }
    if (kk < 2 && colok) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            v4d o = {(double)acc0[r], (double)acc1[r], (double)acc2[r], (double)acc3[r]};
            *reinterpret_cast<v4d*>(mom + (long)(4 * kk + r) * L + c4) = o;
        }
    }
}


__global__ __launch_bounds__(256) void moments_f64_wide_kernel(const double* __restrict__ psi, int nd, long L,
                                                               const double* __restrict__ W, int ldw,
                                                               double* __restrict__ mom) {
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long col0 = wave * 64;
    if (col0 >= L) return;
    const int j = lane & 15, kk = lane >> 4;
    const long c4 = col0 + 4 * j;
    const bool colok = c4 < L;
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
    for (int k = 0; k < nd; k += 4) {
        const int dk = k + kk;
        const double av = dk < nd ? W[j * ldw + dk] : 0.0;
        v2d b01 = {0.0, 0.0}, b23 = {0.0, 0.0};
        if (dk < nd && colok) {
            const v2d* src = reinterpret_cast<const v2d*>(psi + (long)dk * L + c4);
            b01 = src[0];
            b23 = src[1];
        }
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b01[0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b01[1], acc1, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b23[0], acc2, 0, 0, 0);
        acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b23[1], acc3, 0, 0, 0);
    }
    if (colok) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            v4d o = {acc0[r], acc1[r], acc2[r], acc3[r]};
            *reinterpret_cast<v4d*>(mom + (long)(kk + 4 * r) * L + c4) = o;
        }
    }
}

hipError_t launch_moments(bool fp64, const void* psi, int nd, long L, const void* W, int ldw,
                          double* mom, hipStream_t s) {
    if (L % 4 == 0) {
        const long blocks = ((L + 63) / 64 + 3) / 4;
        if (fp64)
            hipLaunchKernelGGL(moments_f64_wide_kernel, dim3(blocks), dim3(256), 0, s, (const double*)psi, nd, L,
                               (const double*)W, ldw, mom);
        else
            hipLaunchKernelGGL(moments_f32_wide_kernel, dim3(blocks), dim3(256), 0, s, (const float*)psi, nd, L,
                               (const float*)W, ldw, mom);
        return hipGetLastError();
    }
    const long waves = (L + 15) / 16;
    const long blocks = (waves + 3) / 4;
    if (fp64)
        hipLaunchKernelGGL(moments_f64_kernel, dim3(blocks), dim3(256), 0, s, (const double*)psi, nd, L,
                           (const double*)W, ldw, mom);
    else
        hipLaunchKernelGGL(moments_f32_kernel, dim3(blocks), dim3(256), 0, s, (const float*)psi, nd, L,
                           (const float*)W, ldw, mom);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scattering source S = sigma_s/(4 pi) (x - x_prev) [+ q]  (x_prev may be null).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void source_kernel(int ne, int n, int nd_q, const double* __restrict__ ss,
                              const double* __restrict__ x, const double* __restrict__ xp,
                              const double* __restrict__ q, T* __restrict__ S) {
    const long L = (long)ne * n;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int dq = blockIdx.y;
    if (t >= L) return;
    const long K = t / n;
    double v = x ? ss[K] * (1.0 / (4.0 * 3.14159265358979323846)) * (xp ? x[t] - xp[t] : x[t]) : 0.0;
    if (q) v += q[(long)dq * L + t];
    S[(long)dq * L + t] = (T)v;
}

hipError_t launch_source(bool fp64, int ne, int n, int nd_q, const double* sigma_s, const double* x,
                         const double* x_prev, const double* q, void* S, hipStream_t s) {
    const long L = (long)ne * n;
    dim3 grid((unsigned)((L + 255) / 256), nd_q > 0 ? nd_q : 1);
    if (fp64)
        hipLaunchKernelGGL(source_kernel<double>, grid, dim3(256), 0, s, ne, n, nd_q, sigma_s, x, x_prev, q,
                           (double*)S);
    else
        hipLaunchKernelGGL(source_kernel<float>, grid, dim3(256), 0, s, ne, n, nd_q, sigma_s, x, x_prev, q,
                           (float*)S);
    return hipGetLastError();
}

__global__ void axpy_kernel(long L, const double* __restrict__ a, double* __restrict__ acc) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < L) acc[t] += a[t];
}

hipError_t launch_axpy_mom(long L, const double* a, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, L, a, acc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Closures: T = P - phi/3 I (xx, xy, yy) at the nodes; beta at boundary face
// points from the interior trace: beta = sum w |Omega.n| psi - E_b0 phi, with
// |Omega.n| = |Omega_x| on x-normal faces (1, 3), |Omega_y| on y-normal faces.
// ---------------------------------------------------------------------------
__global__ void closures_T_kernel(long L, const double* __restrict__ mom, double* __restrict__ T) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L) return;
    const double phi = mom[t];
    T[t] = mom[3 * L + t] - phi / 3.0;
    T[L + t] = mom[4 * L + t];
    T[2 * L + t] = mom[5 * L + t] - phi / 3.0;
}

__global__ void closures_beta_kernel(int n, int nb, int nq, int nbf, long L, const double* __restrict__ mom,
                                     const int* __restrict__ bK, const int* __restrict__ bF,
                                     const double* __restrict__ Lf, double eb0x, double eb0y,
                                     double* __restrict__ beta) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nbf * nq) return;
    const int bf = t / nq, q = t - bf * nq;
    const int K = bK[bf], f = bF[bf];
    const bool xnorm = (f == 1 || f == 3);
    const double* row = mom + (xnorm ? 6 : 7) * L;
    const double e = xnorm ? eb0x : eb0y;
    double v = 0.0;
    for (int c = 0; c < nb; ++c) {
        int k;
        switch (f) {
            case 0: k = c; break;
            case 1: k = (nb - 1) + nb * c; break;
            case 2: k = c + nb * (nb - 1); break;
            default: k = nb * c; break;
        }
        const long idx = (long)K * n + k;
        v += Lf[c * nq + q] * (row[idx] - e * mom[idx]);
    }
    beta[t] = v;
}

// beta on boundaries whose normal is not along x or y: at each boundary
// point, sum over directions of w (|Omega.n| - E_b0(n)) times the element's
// trace of psi (eq. bdr_correction_factor_disc), from psi itself (the moment
// rows hold |Omega_x| and |Omega_y| weights only).  accumulate: add to beta
// (delta sweeps: beta is linear in psi).
template <typename T>
__global__ void closures_beta_general_kernel(int nd, int n, int nb, int nq, int nbf, long ld,
                                             const T* __restrict__ psi, const double* __restrict__ omega,
                                             const double* __restrict__ w, const int* __restrict__ bK,
                                             const int* __restrict__ bF, const double* __restrict__ nhat_b,
                                             const double* __restrict__ eb0_pt, const double* __restrict__ Lf,
                                             int accumulate, double* __restrict__ beta) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nbf * nq) return;
    const int bf = t / nq, q = t - bf * nq;
    const int K = bK[bf], f = bF[bf];
    const double nx = nhat_b[2 * t], ny = nhat_b[2 * t + 1], e = eb0_pt[t];
    double v = 0.0;
    for (int d = 0; d < nd; ++d) {
        const T* pd = psi + (long)d * ld + (long)K * n;
        double tr = 0.0;
        for (int c = 0; c < nb; ++c) {
            int k;
            switch (f) {
                case 0: k = c; break;
                case 1: k = (nb - 1) + nb * c; break;
                case 2: k = c + nb * (nb - 1); break;
                default: k = nb * c; break;
            }
            tr += Lf[c * nq + q] * (double)pd[k];
        }
        v += w[d] * (std::fabs(omega[d * 3] * nx + omega[d * 3 + 1] * ny) - e) * tr;
    }
    beta[t] = accumulate ? beta[t] + v : v;
}

hipError_t launch_beta_general(bool fp64, int nd, int ne, int n, int nb, int nq, int nbf, const void* psi,
                               const double* omega, const double* w, const int* bface_K, const int* bface_f,
                               const double* nhat_b, const double* eb0_pt, const double* Lf, bool accumulate,
                               double* beta, hipStream_t s) {
    if (nbf <= 0) return hipSuccess;
    const long ld = (long)ne * n;
    const dim3 g((nbf * nq + 255) / 256), b(256);
    if (fp64)
        hipLaunchKernelGGL(closures_beta_general_kernel<double>, g, b, 0, s, nd, n, nb, nq, nbf, ld,
                           (const double*)psi, omega, w, bface_K, bface_f, nhat_b, eb0_pt, Lf, accumulate ? 1 : 0,
                           beta);
    else
        hipLaunchKernelGGL(closures_beta_general_kernel<float>, g, b, 0, s, nd, n, nb, nq, nbf, ld,
                           (const float*)psi, omega, w, bface_K, bface_f, nhat_b, eb0_pt, Lf, accumulate ? 1 : 0,
                           beta);
    return hipGetLastError();
}

hipError_t launch_closures(int ne, int n, int nb, int nq, int nbf, const double* mom, const int* bface_K,
                           const int* bface_f, const double* Lf, double eb0x, double eb0y, double* T,
                           double* beta, hipStream_t s) {
    const long L = (long)ne * n;
    hipLaunchKernelGGL(closures_T_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, L, mom, T);
    if (nbf > 0)
        hipLaunchKernelGGL(closures_beta_kernel, dim3((nbf * nq + 255) / 256), dim3(256), 0, s, n, nb, nq, nbf,
                           L, mom, bface_K, bface_f, Lf, eb0x, eb0y, beta);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// IP right-hand side: b = b_fixed + C T - B beta (one thread per row).
// ---------------------------------------------------------------------------
__global__ void rhs_kernel(int ne, int n, int nq, const double* __restrict__ bfix, const int* __restrict__ col,
                           const double* __restrict__ corr, const double* __restrict__ T,
                           const int* __restrict__ bface_of, const double* __restrict__ bop,
                           const double* __restrict__ beta, double* __restrict__ b) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long L = (long)ne * n;
    if (t >= L) return;
    const int K = (int)(t / n), i = (int)(t - (long)K * n);
    const int n3 = 3 * n;
    double v = bfix[t];
    for (int s = 0; s < 5; ++s) {
        const int Kc = col[K * 5 + s];
        if (Kc < 0) continue;
        const double* row = corr + (((long)K * 5 + s) * n + i) * n3;
        for (int c = 0; c < 3; ++c) {
            const double* tv = T + c * L + (long)Kc * n;
            for (int j = 0; j < n; ++j) v += row[c * n + j] * tv[j];
        }
    }
    for (int f = 0; f < 4; ++f) {
        const int bf = bface_of[K * 4 + f];
        if (bf < 0) continue;
        const double* bo = bop + ((long)bf * n + i) * nq;
        const double* be = beta + (long)bf * nq;
        for (int q = 0; q < nq; ++q) v -= bo[q] * be[q];
    }
    b[t] = v;
}

hipError_t launch_rhs(int ne, int n, int nq, const double* bfix, const int* bsr_col, const double* corr,
                      const double* T, const int* bface_of, const double* beta_op, const double* beta,
                      double* b, hipStream_t s) {
    const long L = (long)ne * n;
    hipLaunchKernelGGL(rhs_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, ne, n, nq, bfix, bsr_col,
                       corr, T, bface_of, beta_op, beta, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 PCG with element block-Jacobi preconditioner.
// Blocks cover whole elements (epb = 256 / n elements each) so the
// preconditioner can be applied from LDS.  Device scalars:
//   scal[0] rz   scal[1] rz_old   scal[2] bb   scal[3] rr
//   scal[4] done scal[5] iterations   scal[6] breakdown (1: p.Ap <= 0, 2: non-finite)   scal[7] tol^2 bb
// Reductions are per-block partials summed by every block in a fixed order,
// so results are bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int CG_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = CG_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double sum_partials(const double* part, int nblocks, double* red) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += CG_THREADS) v += part[k];
    return block_sum(v, red);
}

__device__ __forceinline__ void bsr_row(const int* col, const double* A, const double* x, int K, int i, int n,
                                        double& out) {
    double v = 0.0;
    for (int s = 0; s < 5; ++s) {
        const int Kc = col[K * 5 + s];
        if (Kc < 0) continue;
        const double* row = A + (((long)K * 5 + s) * n + i) * n;
        const double* xv = x + (long)Kc * n;
        for (int j = 0; j < n; ++j) v += row[j] * xv[j];
    }
    out = v;
}

// r = b - A x
__global__ __launch_bounds__(CG_THREADS) void cg_init1(CgState c) {
    const int epb = CG_THREADS / c.n;
    const int K = blockIdx.x * epb + threadIdx.x / c.n;
    const int i = threadIdx.x % c.n;
    if (threadIdx.x >= epb * c.n || K >= c.ne) return;
    double ax;
    bsr_row(c.col, c.A, c.x, K, i, c.n, ax);
    const long t = (long)K * c.n + i;
    c.r[t] = c.b[t] - ax;
}

// z = Dinv r, p = z; partials of r.z, r.r, b.b
__global__ __launch_bounds__(CG_THREADS) void cg_init2(CgState c) {
    __shared__ double red[CG_THREADS];
    const int n = c.n, epb = CG_THREADS / n;
    const int K = blockIdx.x * epb + threadIdx.x / n;
    const int i = threadIdx.x % n;
    const bool act = threadIdx.x < epb * n && K < c.ne;
    double rz = 0, rr = 0, bb = 0;
    if (act) {
        const long t = (long)K * n + i;
        const double* D = c.Dinv + ((long)K * n + i) * n;
        double z = 0;
        for (int j = 0; j < n; ++j) z += D[j] * c.r[(long)K * n + j];
        c.z[t] = z;
        c.p[t] = z;
        rz = c.r[t] * z;
        rr = c.r[t] * c.r[t];
        bb = c.b[t] * c.b[t];
    }
    rz = block_sum(rz, red);
    rr = block_sum(rr, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        c.part[blockIdx.x] = rz;
        c.part[c.nblocks + blockIdx.x] = rr;
        c.part[2 * c.nblocks + blockIdx.x] = bb;
    }
}

__global__ __launch_bounds__(CG_THREADS) void cg_init3(CgState c, double tol) {
    __shared__ double red[CG_THREADS];
    const double rz = sum_partials(c.part, c.nblocks, red);
    const double rr = sum_partials(c.part + c.nblocks, c.nblocks, red);
    const double bb = sum_partials(c.part + 2 * c.nblocks, c.nblocks, red);
    if (threadIdx.x == 0) {
        c.scal[0] = rz;
        c.scal[1] = rz;
        c.scal[2] = bb;
        c.scal[3] = rr;
        c.scal[7] = tol * tol * bb;
        c.scal[4] = (rr <= c.scal[7]) ? 1.0 : 0.0;
        c.scal[5] = 0.0;
        c.scal[6] = 0.0;
    }
}

// q = A p; partial p.q
__global__ __launch_bounds__(CG_THREADS) void cg_k1(CgState c) {
    __shared__ double red[CG_THREADS];
    if (c.scal[4] != 0.0) return;
    const int n = c.n, epb = CG_THREADS / n;
    const int K = blockIdx.x * epb + threadIdx.x / n;
    const int i = threadIdx.x % n;
    double pq = 0;
    if (threadIdx.x < epb * n && K < c.ne) {
        double v;
        bsr_row(c.col, c.A, c.p, K, i, n, v);
        const long t = (long)K * n + i;
        c.q[t] = v;
        pq = c.p[t] * v;
    }
    pq = block_sum(pq, red);
    if (threadIdx.x == 0) c.part[blockIdx.x] = pq;
}

// alpha = rz / pq; x += alpha p; r -= alpha q; z = Dinv r; partials r.z, r.r
__global__ __launch_bounds__(CG_THREADS) void cg_k2(CgState c) {
    __shared__ double red[CG_THREADS];
    __shared__ double rl[CG_THREADS];
    if (c.scal[4] != 0.0) return;
    const double pq = sum_partials(c.part, c.nblocks, red);
    const double rz = c.scal[0];
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c.scal[6] = pq <= 0.0 ? 1.0 : 2.0;  // 2: not a number (a non-finite right-hand side)
            c.scal[4] = 1.0;
        }
        return;
    }
    const double alpha = rz / pq;
    const int n = c.n, epb = CG_THREADS / n;
    const int K = blockIdx.x * epb + threadIdx.x / n;
    const int i = threadIdx.x % n;
    const bool act = threadIdx.x < epb * n && K < c.ne;
    double rnew = 0;
    if (act) {
        const long t = (long)K * n + i;
        c.x[t] += alpha * c.p[t];
        rnew = c.r[t] - alpha * c.q[t];
        c.r[t] = rnew;
    }
    rl[threadIdx.x] = rnew;
    __syncthreads();
    double rz2 = 0, rr = 0;
    if (act) {
        const int e0 = (threadIdx.x / n) * n;
        const double* D = c.Dinv + ((long)K * n + i) * n;
        double z = 0;
        for (int j = 0; j < n; ++j) z += D[j] * rl[e0 + j];
        c.z[(long)K * n + i] = z;
        rz2 = rnew * z;
        rr = rnew * rnew;
    }
    rz2 = block_sum(rz2, red);
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        c.part[c.nblocks + blockIdx.x] = rz2;
        c.part[2 * c.nblocks + blockIdx.x] = rr;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) c.scal[1] = rz;
}

// beta = rz_new / rz_old; p = z + beta p; convergence test
__global__ __launch_bounds__(CG_THREADS) void cg_k3(CgState c) {
    __shared__ double red[CG_THREADS];
    if (c.scal[4] != 0.0) return;
    const double rzn = sum_partials(c.part + c.nblocks, c.nblocks, red);
    const double rr = sum_partials(c.part + 2 * c.nblocks, c.nblocks, red);
    const bool conv = rr <= c.scal[7];
    const double beta = rzn / c.scal[1];
    const int n = c.n, epb = CG_THREADS / n;
    const int K = blockIdx.x * epb + threadIdx.x / n;
    const int i = threadIdx.x % n;
    if (!conv && threadIdx.x < epb * n && K < c.ne) {
        const long t = (long)K * n + i;
        c.p[t] = c.z[t] + beta * c.p[t];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c.scal[0] = rzn;
        c.scal[3] = rr;
        c.scal[5] += 1.0;
        if (conv) c.scal[4] = 1.0;
    }
}

hipError_t cg_start(const CgState& c, double tol, hipStream_t s) {
    hipLaunchKernelGGL(cg_init1, dim3(c.nblocks), dim3(CG_THREADS), 0, s, c);
    hipLaunchKernelGGL(cg_init2, dim3(c.nblocks), dim3(CG_THREADS), 0, s, c);
    hipLaunchKernelGGL(cg_init3, dim3(1), dim3(CG_THREADS), 0, s, c, tol);
    return hipGetLastError();
}

hipError_t cg_iterations(const CgState& c, int iters, double tol, hipStream_t s) {
    (void)tol;
    for (int t = 0; t < iters; ++t) {
        hipLaunchKernelGGL(cg_k1, dim3(c.nblocks), dim3(CG_THREADS), 0, s, c);
        hipLaunchKernelGGL(cg_k2, dim3(c.nblocks), dim3(CG_THREADS), 0, s, c);
        hipLaunchKernelGGL(cg_k3, dim3(c.nblocks), dim3(CG_THREADS), 0, s, c);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Outer residual: out[0] = max |xn - xo|, out[1] = max |xn|.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void resid_part(long L, const double* __restrict__ xn,
                                                  const double* __restrict__ xo, double* __restrict__ part,
                                                  int nblocks) {
    __shared__ double r0[256], r1[256];
    double a = 0, b = 0;
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < L; t += (long)nblocks * 256) {
        const double v = xn[t];
        const double dv = fabs(v - xo[t]);
        a = dv > a || dv != dv ? dv : a;
        b = fabs(v) > b || v != v ? fabs(v) : b;
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double x0 = r0[threadIdx.x + s], x1 = r1[threadIdx.x + s];
            r0[threadIdx.x] = (x0 > r0[threadIdx.x] || x0 != x0) ? x0 : r0[threadIdx.x];
            r1[threadIdx.x] = (x1 > r1[threadIdx.x] || x1 != x1) ? x1 : r1[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = r0[0];
        part[nblocks + blockIdx.x] = r1[0];
    }
}

__global__ __launch_bounds__(256) void resid_final(const double* __restrict__ part, int nblocks,
                                                   double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double a = 0, b = 0;
    for (int k = 0; k < nblocks; ++k) {
        const double x0 = part[k], x1 = part[nblocks + k];
        a = (x0 > a || x0 != x0) ? x0 : a;
        b = (x1 > b || x1 != x1) ? x1 : b;
    }
    out[0] = a;
    out[1] = b;
}

hipError_t launch_residual(long L, const double* xn, const double* xo, double* part, int nblocks, double* out,
                           hipStream_t s) {
    hipLaunchKernelGGL(resid_part, dim3(nblocks), dim3(256), 0, s, L, xn, xo, part, nblocks);
    hipLaunchKernelGGL(resid_final, dim3(1), dim3(256), 0, s, part, nblocks, out);
    return hipGetLastError();
}

}  // namespace smm

// ===========================================================================
// Batched typed-Cartesian path
// ===========================================================================
namespace smm {

constexpr int BT = 256;  // threads of element-block kernels

__device__ __forceinline__ int bsearch_prob(const long* pre, int nprob, long idx) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// element-block mapping: problem, element K, node i (or K = -1 when idle)
struct EB {
    int prob, K, i, e0;
};
__device__ __forceinline__ EB eb_map(const BatchLaunch& B) {
    EB r;
    r.prob = B.blk2p[blockIdx.x];
    const BProb& P = B.P[r.prob];
    const int epb = BT / P.n;
    const int le = threadIdx.x / P.n;
    r.i = threadIdx.x - le * P.n;
    r.e0 = le * P.n;
    const int K = (blockIdx.x - P.blk0) * epb + le;
    r.K = (le < epb && K < P.ne) ? K : -1;
    return r;
}

// sum over the 64 lanes of a wave (butterfly; every lane gets the sum)
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// grouped FP64 matrix-core block-row products (defined with the PCG kernels):
// MODE 0: r = b - A x (PCG start), MODE 1: IP right-hand side
template <int MODE>
static void b_group_rows_all(const BatchLaunch& B, hipStream_t s);

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This maps them so that each XCD takes one contiguous range of logical
// workgroup indices: consecutive type groups (neighbouring element rows, whose
// vectors the neighbour faces read again) then share one L2.
__device__ __forceinline__ int xcd_block() {
    const int nwg = gridDim.x, b = blockIdx.x;
    const int k = b & 7, q = nwg >> 3, r = nwg & 7;
    return k * q + (k < r ? k : r) + (b >> 3);
}

// ---- scattering source -----------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BT) void b_source_kernel(BatchLaunch B, int delta) {
    const EB m = eb_map(B);
    if (!B.active[m.prob] || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i;
    const double c = P.sigma_s[m.K] * (1.0 / (4.0 * 3.14159265358979323846));
    double v = delta ? c * (P.varphi[t] - P.varphi_prev[t]) : c * P.varphi[t] + P.qsrc[t];
    reinterpret_cast<T*>(P.S)[t] = (T)v;
}

hipError_t b_source(bool fp64, const BatchLaunch& B, bool delta, hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL(b_source_kernel<double>, dim3(B.nblocks), dim3(BT), 0, s, B, delta ? 1 : 0);
    else
        hipLaunchKernelGGL(b_source_kernel<float>, dim3(B.nblocks), dim3(BT), 0, s, B, delta ? 1 : 0);
    return hipGetLastError();
}

__global__ void zero_ints_kernel(int* p, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0;
}

hipError_t zero_ints(int* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ---- persistent sweep over (problem, direction) tasks ------------------------
// Lane-per-element Cartesian sweep.  Wave w of the workgroup owns node column
// ca = w mod NB of the elements in slots 64 (w / NB) + lane of each
// anti-diagonal, i.e. rows ca + NB b (b < NB) of the element's local solution.
// The operator rows of that column, [Pm | Px | Py], are then the same for all
// lanes of the wave (one material): they are read through the constant address
// space, arrive by scalar loads and enter the FMAs as SGPR operands, so neither
// registers nor LDS hold per-lane copies of the operator.  Waves holding
// elements of several materials make one pass per material present.
// Source and angular flux move between HBM and LDS with element-major flat
// indices (consecutive lanes, consecutive words of one element's block): the
// source of level m + D is loaded into registers during level m and parked in
// LDS during level m + D - 1; the flux of level m is staged in LDS and stored
// during level m + 1.  LDS rows have odd strides, so the lanes' rows fall in
// distinct banks.
template <typename T>
using cptr = const T __attribute__((address_space(4)))*;

// Wave-uniform pointer into the constant address space.  The empty asm makes
// the value opaque, so loads through it are not hoisted out of the level loop:
// the operator is re-read from the scalar cache each level instead of being
// pinned in (far too many) SGPRs.
template <typename T>
__device__ __forceinline__ cptr<T> uniform_rows(const T* p) {
    const unsigned long v = (unsigned long)p;
    unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (cptr<T>)(((unsigned long)hi << 32) | lo);
}

// Word w of a global array whose byte size is below 4 GiB: the 32-bit byte
// offset lets loads and stores use a scalar base plus a vector offset.
template <typename T>
__device__ __forceinline__ T ld_at(gcptr<T> p, unsigned w) {
    return *(gcptr<T>)((const char __attribute__((address_space(1)))*)p + w * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_at(gptr<T> p, unsigned w, T v) {
    *(gptr<T>)((char __attribute__((address_space(1)))*)p + w * (unsigned)sizeof(T)) = v;
}

// Wave-uniform pointer into the constant address space, without the barrier:
// loads through it may be hoisted and kept in SGPRs.
template <typename T>
__device__ __forceinline__ cptr<T> uniform_ptr(const T* p) {
    const unsigned long v = (unsigned long)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return (cptr<T>)(((unsigned long)hi << 32) | lo);
}

__host__ __device__ constexpr int lane_ns(int nb) { return (nb * nb) | 1; }  // LDS row stride of a block
__host__ __device__ constexpr int lane_ts(int nb) { return nb | 1; }         // LDS row stride of a trace
constexpr int LANE_PREFETCH = 3;  // levels between a source load and its use

template <typename T, int NB, bool MULTI, int D>
__device__ __forceinline__ void sweep_lane_task(const CartSweepArgs& a, const int d, unsigned char* smem) {
    constexpr int N = NB * NB;
    constexpr int NS = lane_ns(NB);
    constexpr int TS = lane_ts(NB);
    const int nx = a.nx, ny = a.ny, nd = a.nd;
    const long ne = (long)nx * ny;
    const int maxlen = nx < ny ? nx : ny;
    const int nlev = nx + ny - 1;
    const int nthr = blockDim.x;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ca = w % NB;
    const int chunk0 = (w / NB) * 64;  // first slot of this wave
    const int slot = chunk0 + (tid & 63);
    const int rslot = slot < maxlen ? slot : maxlen - 1;
    T* xtr = reinterpret_cast<T*>(smem);  // [2][ny][TS]
    T* ytr = xtr + 2 * ny * TS;           // [2][nx][TS]
    T* sch = ytr + 2 * nx * TS;           // [2][maxlen][NS] source of a level (by parity)
    T* pst = sch + 2 * maxlen * NS;       // [2][maxlen][NS] flux of a level (by parity)
    uint8_t* msh = reinterpret_cast<uint8_t*>(pst + 2 * maxlen * NS);  // [ne] (MULTI)
    const auto om = as_global(a.omega);
    const double ox = om[d * 3], oy = om[d * 3 + 1];
    const bool sx = ox > 0.0, sy = oy > 0.0;
    const auto S = as_global(reinterpret_cast<const T*>(a.S) + (a.s_aniso ? (long)d * ne * N : 0));
    const auto psi = as_global(reinterpret_cast<T*>(a.psi) + (long)d * (a.psi_ld > 0 ? a.psi_ld : ne * N));
    // operator rows: one scalar-loaded block per wave; small tables (one
    // material, few rows) stay in SGPRs for the whole task
    constexpr int RW = lane_rw(NB);
    constexpr bool HOIST = !MULTI && NB * RW * (int)sizeof(T) <= 64 * 4;
    const T* tab = reinterpret_cast<const T*>(a.tab);
    if constexpr (MULTI) {
        const auto mat = as_global(a.mat);
        for (long t = tid; t < ne; t += nthr) msh[t] = mat[t];
    }
    const auto bx = as_global(reinterpret_cast<const T*>(a.bx));
    const auto by = as_global(reinterpret_cast<const T*>(a.by));
    for (int t = tid; t < ny * NB; t += nthr) {
        const int j = t / NB, c = t - j * NB;
        const T v = bx ? bx[(long)d * ny * NB + t] : T(0);
        xtr[j * TS + c] = v;
        xtr[(ny + j) * TS + c] = v;
    }
    for (int t = tid; t < nx * NB; t += nthr) {
        const int i = t / NB, c = t - i * NB;
        const T v = by ? by[(long)d * nx * NB + t] : T(0);
        ytr[i * TS + c] = v;
        ytr[(nx + i) * TS + c] = v;
    }
    // level geometry: first x index on the quadrant-oriented grid and length
    auto lev_i0 = [&](int l) { return l - (ny - 1) > 0 ? l - (ny - 1) : 0; };
    auto lev_len = [&](int l) {
        const int i1 = l < nx - 1 ? l : nx - 1;
        return l < nlev ? i1 - lev_i0(l) + 1 : 0;
    };
    // The element of slot s at level l is K0(s) + acc(l): K0(s) is its index
    // at level 0 (outside the grid for s > 0) and acc(l) the wave-uniform sum
    // of the steps from level to level (+-nx while the first slot of a level
    // moves along y, +-1 once it moves along x).  ne N < 2^31 words per
    // direction, so word offsets are 32-bit.
    const int dyK = sy ? nx : -nx, dxK = sx ? 1 : -1;
    auto acc_of = [&](int l) { return l <= ny - 1 ? l * dyK : (ny - 1) * dyK + (l - (ny - 1)) * dxK; };
    auto K0 = [&](int s) { return (sy ? -s : ny - 1 + s) * nx + (sx ? s : nx - 1 - s); };
    // flat element-major indices of this thread: f = tid + nthr r covers
    // maxlen * N <= nthr * NB words of a level; word f of a level lies at
    // global word wb[r] + acc(l) N and LDS word lb[r]
    int fe[NB], wb[NB], lb[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int f = tid + nthr * r;
        fe[r] = f / N;
        const int c = f - fe[r] * N;
        wb[r] = K0(fe[r]) * N + c;
        lb[r] = fe[r] * NS + c;
    }
    // loads are issued unconditionally (word 0 stands in for an empty slot)
    auto fetch = [&](int l, T(&dst)[NB]) {
        const int len = lev_len(l), a = acc_of(l) * N;
#pragma unroll
        for (int r = 0; r < NB; ++r) dst[r] = ld_at(S, fe[r] < len ? (unsigned)(wb[r] + a) : 0u);
    };
    auto park = [&](int l, const T(&src)[NB]) {
        const int len = lev_len(l);
        T* dst = sch + (l & 1) * maxlen * NS;
#pragma unroll
        for (int r = 0; r < NB; ++r)
            if (fe[r] < len) dst[lb[r]] = src[r];
    };
    auto flush = [&](int l) {
        const int len = lev_len(l), a = acc_of(l) * N;
        const T* src = pst + (l & 1) * maxlen * NS;
#pragma unroll
        for (int r = 0; r < NB; ++r)
            if (fe[r] < len) st_at(psi, (unsigned)(wb[r] + a), src[lb[r]]);
    };
    // grid coordinates of this thread's own slot: i = ib + isg i0(l),
    // j = jb + jsg (l - i0(l))
    const int ib = sx ? slot : nx - 1 - slot, isg = sx ? 1 : -1;
    const int jb = sy ? -slot : ny - 1 + slot, jsg = sy ? 1 : -1;
    const int aout = sx ? NB - 1 : 0;
    const int bout = sy ? NB - 1 : 0;
    T pre[D][NB];
#pragma unroll
    for (int u = 0; u < D; ++u) fetch(u, pre[u]);
    park(0, pre[0]);
    lds_barrier();
    for (int m0 = 0; m0 < nlev; m0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int m = m0 + u;
            if (m >= nlev) break;
            const int cur = m & 1, nxt = cur ^ 1;
            const int len = lev_len(m);
            fetch(m + D, pre[u]);  // this slot's level m was parked during level m - 1
            if (chunk0 < len) {    // wave-uniform: the wave holds elements of this level
                const bool act = slot < len;
                const int i0 = lev_i0(m);
                const int ci = act ? ib + isg * i0 : 0;
                const int cj = act ? jb + jsg * (m - i0) : 0;
                T sv[N], tx[NB], ty[NB];
                const T* sp = sch + (cur * maxlen + rslot) * NS;
#pragma unroll
                for (int c = 0; c < N; ++c) sv[c] = sp[c];
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    tx[c] = xtr[(cur * ny + cj) * TS + c];
                    ty[c] = ytr[(cur * nx + ci) * TS + c];
                }
                T acc[NB];
                auto apply = [&](int mat, T(&out)[NB]) {
                    // this wave's NB rows, contiguous: row b at b RW
                    const T* rows = tab + (((long)mat * nd + d) * NB + ca) * NB * RW;
                    const cptr<T> tr = HOIST ? uniform_ptr(rows) : uniform_rows(rows);
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        T v = T(0);
#pragma unroll
                        for (int c = 0; c < N; ++c) v += tr[b * RW + c] * sv[c];
#pragma unroll
                        for (int c = 0; c < NB; ++c) v += tr[b * RW + N + c] * tx[c];
#pragma unroll
                        for (int c = 0; c < NB; ++c) v += tr[b * RW + N + NB + c] * ty[c];
                        out[b] = v;
                    }
                };
                if constexpr (!MULTI) {
                    apply(0, acc);
                } else {
                    // one pass per material present in the wave (spatially
                    // coherent layouts: usually one, two at interfaces)
                    const int cm = act ? (int)msh[cj * nx + ci] : -1;
                    unsigned long long todo = __ballot(act);
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[b] = T(0);
                    while (todo) {
                        const int lead = __builtin_ctzll(todo);
                        const int mm = __builtin_amdgcn_readfirstlane(__shfl(cm, lead));
                        T tmp[NB];
                        apply(mm, tmp);
                        const bool mine = cm == mm;
#pragma unroll
                        for (int b = 0; b < NB; ++b) acc[b] = mine ? tmp[b] : acc[b];
                        todo &= ~__ballot(mine);
                    }
                }
                if (act) {
                    T* pp = pst + (cur * maxlen + slot) * NS + ca;
#pragma unroll
                    for (int b = 0; b < NB; ++b) pp[NB * b] = acc[b];
                    if (ca == aout) {
#pragma unroll
                        for (int b = 0; b < NB; ++b) xtr[(nxt * ny + cj) * TS + b] = acc[b];
                    }
                    ytr[(nxt * nx + ci) * TS + ca] = acc[bout];
                }
            }
            if (m > 0) flush(m - 1);
            if (m + 1 < nlev) park(m + 1, pre[(u + 1) % D]);
            lds_barrier();
        }
    }
    flush(nlev - 1);
}

// Workgroups take tasks from a global counter (largest tasks first) until the
// list is exhausted; tasks of problems that have converged are skipped.
template <typename T, int NB, bool MULTI, int MAXT>
__global__ __launch_bounds__(MAXT) void b_sweep_kernel(const CartSweepArgs* __restrict__ args,
                                                        const int2* __restrict__ tasks, int ntasks,
                                                        int* __restrict__ counter,
                                                        const int* __restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int tsk;
    while (true) {
        if (threadIdx.x == 0) tsk = atomicAdd(counter, 1);
        __syncthreads();
        const int t = tsk;
        __syncthreads();
        if (t >= ntasks) break;
        const int2 tk = tasks[t];
        if (!active[tk.x]) continue;
        sweep_lane_task<T, NB, MULTI, LANE_PREFETCH>(args[tk.x], tk.y, smem);
        __syncthreads();
    }
}

// ---- persistent sweep, element-lane shape ------------------------------------
// The same per-element operator as above, another mapping: each lane solves a
// whole element of an anti-diagonal (all N nodes; the N x (N + 2 NB) operator
// rows are wave-uniform scalar operands, as above), a workgroup is one wave per
// 64-slot chunk.  The inflow traces of level m come from level m - 1: the x
// trace from the element left of this one, the y trace from the one below it,
// i.e. from this lane or its neighbour (which one depends only on whether the
// first slot of the level moved along x), passed by lane shuffles; only the
// traces that cross a chunk boundary go through LDS, with one barrier per level
// when the workgroup has several waves.  No other LDS: source and flux move
// straight between HBM and registers.
template <typename T, int NB, bool MULTI>
__device__ __forceinline__ void sweep_elem_task(const CartSweepArgs& a, const int d, T* xb, T* yb) {
    constexpr int N = NB * NB;
    constexpr int RW = lane_rw(NB);
    const int nx = a.nx, ny = a.ny, nd = a.nd;
    const long ne = (long)nx * ny;
    const int nlev = nx + ny - 1;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nw = blockDim.x >> 6;
    const int slot = wv * 64 + lane;
    const auto om = as_global(a.omega);
    const double ox = om[d * 3], oy = om[d * 3 + 1];
    const bool sx = ox > 0.0, sy = oy > 0.0;
    const auto S = as_global(reinterpret_cast<const T*>(a.S) + (a.s_aniso ? (long)d * ne * N : 0));
    const auto psi = as_global(reinterpret_cast<T*>(a.psi) + (long)d * (a.psi_ld > 0 ? a.psi_ld : ne * N));
    const auto bx = as_global(reinterpret_cast<const T*>(a.bx));
    const auto by = as_global(reinterpret_cast<const T*>(a.by));
    const T* tab = reinterpret_cast<const T*>(a.tab);
    const int aout = sx ? NB - 1 : 0;   // outflow x face: node column aout
    const int bout = sy ? NB - 1 : 0;   // outflow y face: node row bout
    T xo[NB], yo[NB];                    // this lane's last outflow traces
#pragma unroll
    for (int c = 0; c < NB; ++c) xo[c] = yo[c] = T(0);
    for (int m = 0; m < nlev; ++m) {
        const int i0 = m - (ny - 1) > 0 ? m - (ny - 1) : 0;
        const int i1 = m < nx - 1 ? m : nx - 1;
        const int len = i1 - i0 + 1;
        const bool moved_x = m > 0 && m - 1 - (ny - 1) >= 0;  // i0(m) = i0(m - 1) + 1
        // traces of level m - 1 from the neighbouring lanes (all lanes take part)
        T xl[NB], yr[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            xl[c] = __shfl_up(xo[c], 1);
            yr[c] = __shfl_down(yo[c], 1);
        }
        if (nw > 1 && m > 0) {
            const int pb = (m - 1) & 1;
            if (lane == 0 && wv > 0)
#pragma unroll
                for (int c = 0; c < NB; ++c) xl[c] = xb[(pb * 4 + wv - 1) * NB + c];
            if (lane == 63 && wv + 1 < nw)
#pragma unroll
                for (int c = 0; c < NB; ++c) yr[c] = yb[(pb * 4 + wv + 1) * NB + c];
        }
        if (wv * 64 < len) {             // wave-uniform: the wave holds elements of this level
            const bool act = slot < len;
            const int ip = i0 + slot;            // quadrant-oriented grid coordinates
            const int jp = m - ip;
            const int ci = act ? (sx ? ip : nx - 1 - ip) : 0;
            const int cj = act ? (sy ? jp : ny - 1 - jp) : 0;
            const unsigned K = (unsigned)(cj * nx + ci);
            T tx[NB], ty[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                // x inflow: the left neighbour was this lane (first slot moved) or the one before
                T vx = moved_x ? xo[c] : xl[c];
                T vy = moved_x ? yr[c] : yo[c];
                if (ip == 0) vx = bx ? bx[((long)d * ny + cj) * NB + c] : T(0);
                if (jp == 0) vy = by ? by[((long)d * nx + ci) * NB + c] : T(0);
                tx[c] = vx;
                ty[c] = vy;
            }
            T sv[N];
#pragma unroll
            for (int c = 0; c < N; ++c) sv[c] = ld_at(S, act ? K * N + c : 0u);
            T out[N];
            auto apply = [&](int mat, T(&o)[N]) {
                const T* blk = tab + ((long)mat * nd + d) * N * RW;
                const cptr<T> tr = uniform_rows(blk);
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    const int row = ((r % NB) * NB + r / NB) * RW;   // row r = ca + NB b of the table
                    T v = T(0);
#pragma unroll
                    for (int c = 0; c < N; ++c) v += tr[row + c] * sv[c];
#pragma unroll
                    for (int c = 0; c < NB; ++c) v += tr[row + N + c] * tx[c];
#pragma unroll
                    for (int c = 0; c < NB; ++c) v += tr[row + N + NB + c] * ty[c];
                    o[r] = v;
                }
            };
            if constexpr (!MULTI) {
                apply(0, out);
            } else {
                const auto mat = as_global(a.mat);
                const int cm = act ? (int)mat[K] : -1;
                unsigned long long todo = __ballot(act);
#pragma unroll
                for (int r = 0; r < N; ++r) out[r] = T(0);
                while (todo) {
                    const int lead = __builtin_ctzll(todo);
                    const int mm = __builtin_amdgcn_readfirstlane(__shfl(cm, lead));
                    T tmp[N];
                    apply(mm, tmp);
                    const bool mine = cm == mm;
#pragma unroll
                    for (int r = 0; r < N; ++r) out[r] = mine ? tmp[r] : out[r];
                    todo &= ~__ballot(mine);
                }
            }
            if (act) {
#pragma unroll
                for (int r = 0; r < N; ++r) st_at(psi, K * N + r, out[r]);
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    xo[c] = out[aout + NB * c];
                    yo[c] = out[c + NB * bout];
                }
            }
        }
        if (nw > 1) {
            const int pb = m & 1;
            if (lane == 63)
#pragma unroll
                for (int c = 0; c < NB; ++c) xb[(pb * 4 + wv) * NB + c] = xo[c];
            if (lane == 0)
#pragma unroll
                for (int c = 0; c < NB; ++c) yb[(pb * 4 + wv) * NB + c] = yo[c];
            __syncthreads();
        }
    }
}

template <typename T, int NB, bool MULTI>
__global__ __launch_bounds__(256) void b_sweep_elem_kernel(const CartSweepArgs* __restrict__ args,
                                                            const int2* __restrict__ tasks, int ntasks,
                                                            int* __restrict__ counter,
                                                            const int* __restrict__ active) {
    __shared__ T xb[2 * 4 * NB], yb[2 * 4 * NB];   // chunk-boundary traces, by level parity
    __shared__ int tsk;
    while (true) {
        if (threadIdx.x == 0) tsk = atomicAdd(counter, 1);
        __syncthreads();
        const int t = tsk;
        __syncthreads();
        if (t >= ntasks) break;
        const int2 tk = tasks[t];
        if (!active[tk.x]) continue;
        sweep_elem_task<T, NB, MULTI>(args[tk.x], tk.y, xb, yb);
        __syncthreads();
    }
}

template <typename T, int NB>
static hipError_t b_sweep_elem_nb(bool multi, int threads, int grid, const CartSweepArgs* args, const int2* tasks,
                                  int ntasks, int* counter, const int* active, hipStream_t s) {
    if (multi)
        hipLaunchKernelGGL((b_sweep_elem_kernel<T, NB, true>), dim3(grid), dim3(threads), 0, s, args, tasks, ntasks,
                           counter, active);
    else
        hipLaunchKernelGGL((b_sweep_elem_kernel<T, NB, false>), dim3(grid), dim3(threads), 0, s, args, tasks, ntasks,
                           counter, active);
    return hipGetLastError();
}

hipError_t b_sweep_elem(bool fp64, int nb, bool multi, int threads, int grid, const CartSweepArgs* args,
                        const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s) {
    // one wave per 64-slot chunk of the longest anti-diagonal, at most four
    if (threads < 64 || threads > 256 || threads % 64 != 0) return hipErrorNotSupported;
    switch (nb) {
        case 2: return fp64 ? b_sweep_elem_nb<double, 2>(multi, threads, grid, args, tasks, ntasks, counter, active, s)
                            : b_sweep_elem_nb<float, 2>(multi, threads, grid, args, tasks, ntasks, counter, active, s);
        case 3: return fp64 ? b_sweep_elem_nb<double, 3>(multi, threads, grid, args, tasks, ntasks, counter, active, s)
                            : b_sweep_elem_nb<float, 3>(multi, threads, grid, args, tasks, ntasks, counter, active, s);
        case 4: return fp64 ? b_sweep_elem_nb<double, 4>(multi, threads, grid, args, tasks, ntasks, counter, active, s)
                            : b_sweep_elem_nb<float, 4>(multi, threads, grid, args, tasks, ntasks, counter, active, s);
        case 5: return fp64 ? b_sweep_elem_nb<double, 5>(multi, threads, grid, args, tasks, ntasks, counter, active, s)
                            : b_sweep_elem_nb<float, 5>(multi, threads, grid, args, tasks, ntasks, counter, active, s);
        default: return hipErrorInvalidValue;
    }
}

int b_sweep_threads(int nb, int nx, int ny) {
    const int maxlen = nx < ny ? nx : ny;
    return 64 * nb * ((maxlen + 63) / 64);
}

size_t b_sweep_lds(bool fp64, int nb, bool multi, int nx, int ny) {
    const size_t t = fp64 ? 8 : 4;
    const int maxlen = nx < ny ? nx : ny;
    size_t lds = t * (2 * (size_t)(nx + ny) * lane_ts(nb) + 4 * (size_t)maxlen * lane_ns(nb));
    if (multi) lds += (size_t)nx * ny;
    return lds;
}

template <typename T, int NB, bool MULTI, int MAXT>
static hipError_t b_sweep_t(int threads, size_t lds, int grid, const CartSweepArgs* args, const int2* tasks,
                            int ntasks, int* counter, const int* active, hipStream_t s) {
    auto kfn = b_sweep_kernel<T, NB, MULTI, MAXT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(threads), lds, s, args, tasks, ntasks, counter, active);
    return hipGetLastError();
}

template <typename T, int NB>
static hipError_t b_sweep_nb(bool multi, int threads, size_t lds, int grid, const CartSweepArgs* args,
                             const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s) {
    if (threads <= 512)
        return multi ? b_sweep_t<T, NB, true, 512>(threads, lds, grid, args, tasks, ntasks, counter, active, s)
                     : b_sweep_t<T, NB, false, 512>(threads, lds, grid, args, tasks, ntasks, counter, active, s);
    return multi ? b_sweep_t<T, NB, true, 1024>(threads, lds, grid, args, tasks, ntasks, counter, active, s)
                 : b_sweep_t<T, NB, false, 1024>(threads, lds, grid, args, tasks, ntasks, counter, active, s);
}

hipError_t b_sweep(bool fp64, int nb, bool multi, int threads, size_t lds, int grid, const CartSweepArgs* args,
                   const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s) {
    // the workgroup must be the NB waves of every 64-slot chunk of the longest
    // anti-diagonal of every task (checked by the caller against each problem)
    if (threads > 1024 || threads % (64 * nb) != 0 || lds > 160 * 1024) return hipErrorNotSupported;
    switch (nb) {
        case 2: return fp64 ? b_sweep_nb<double, 2>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s)
                            : b_sweep_nb<float, 2>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s);
        case 3: return fp64 ? b_sweep_nb<double, 3>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s)
                            : b_sweep_nb<float, 3>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s);
        case 4: return fp64 ? b_sweep_nb<double, 4>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s)
                            : b_sweep_nb<float, 4>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s);
        case 5: return fp64 ? b_sweep_nb<double, 5>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s)
                            : b_sweep_nb<float, 5>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- persistent sweep on the matrix cores (FP32) ----------------------------
// At one level of a (problem, direction) task every element applies the same
// operator R = [Pm | Px | Py] (N rows; N + 2 NB inputs: its source values, the
// x-face and the y-face inflow traces), so the level is the dense product
// D = R X with one column of X per element.  Columns go in tiles of 16
// elements through v_mfma_f32_16x16x4f32 (A[i][k] from lane i + 16 k, B[k][j]
// from lane j + 16 k, D[i][j] in lane j + 16 (i / 4), element i % 4): R is the
// A operand, rows 16 mt + i and inputs 4 t + k zero-padded, held in registers
// for the whole task (reloaded only when a tile holds another material); lane
// j + 16 k supplies inputs 4 t + k of element j -- source values loaded two
// levels ahead, traces read from LDS.  A wave holds TPW tiles (16 TPW slots of
// the anti-diagonal) and skips the tiles past the level's length, so short
// anti-diagonals cost 16-column tiles, not 64-lane waves.  Rows 16 mt + 4 k + r
// of element j (lane j + 16 k) are stored to HBM, and the outflow-face rows to
// the trace arrays in LDS for the next level.
// Raw buffer accesses: an offset at or past the descriptor's byte count reads
// 0 and drops the store, with no memory access, so inactive lanes and tiles
// need no branch around their loads and stores.  The level loop then issues
// the same global operations on every path, and the wait counts the compiler
// inserts stay exact: a level waits for the loads it consumes (issued levels
// earlier), not for every store and prefetch in flight.
constexpr unsigned BUF_OOB = 0x80000000u;
constexpr int BUF_WORD3 = 0x00020000;   // gfx9-family raw buffer descriptor word 3
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, BUF_WORD3);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}


// Input k-slots of the matrix-core sweep.  Slot (t, g) -- MFMA step t, lane
// group g -- holds source value g QS + t of the element while that is below
// N (so a lane's source values are QS consecutive words: one or two vector
// loads), and the 2 NB face traces fill the remaining slots in order of t,
// then g; -1 marks padding.
template <int NB>
struct MfmaSlots {
    static constexpr int N = NB * NB, QS = (N + 3) / 4, NI = N + 2 * NB, KT = (NI + 3) / 4;
    int q[KT][4];
};
template <int NB>
constexpr MfmaSlots<NB> mfma_slots() {
    using S = MfmaSlots<NB>;
    MfmaSlots<NB> s{};
    int e = 0;
    for (int t = 0; t < S::KT; ++t)
        for (int g = 0; g < 4; ++g) {
            if (t < S::QS && g * S::QS + t < S::N) {
                s.q[t][g] = g * S::QS + t;
            } else {
                s.q[t][g] = e < 2 * NB ? S::N + e : -1;
                ++e;
            }
        }
    return s;
}

// QS consecutive words at byte offset off (out of range: zeros), as vector
// loads.  The vector results are converted whole (bit casts of single vector
// elements of these loads were lowered to one repeated word by this compiler).
typedef float v3f __attribute__((ext_vector_type(3)));
template <int QS>
__device__ __forceinline__ void buf_ld_run(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned off2, float (&v)[QS]) {
    if constexpr (QS == 1) {
        v[0] = buf_ld(r, off);
    } else if constexpr (QS == 3) {
        const v3f x = __builtin_bit_cast(v3f, __builtin_amdgcn_raw_buffer_load_b96(r, (int)off, 0, 0));
        v[0] = x.x, v[1] = x.y, v[2] = x.z;
    } else if constexpr (QS == 4) {
        const v4f x = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
        v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w;
    } else {
        static_assert(QS == 7, "source runs of 1, 3, 4 or 7 words");
        // words 0-3 at off, 4-6 at off2 (each range wholly valid or wholly out of range)
        const v4f x = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
        const v3f y = __builtin_bit_cast(v3f, __builtin_amdgcn_raw_buffer_load_b96(r, (int)off2, 0, 0));
        v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w;
        v[4] = y.x, v[5] = y.y, v[6] = y.z;
    }
}

// LDS row of one element's staged result: 16 MT words plus 4 (a row stride
// that is not a multiple of 32 words keeps the vector writes of neighbouring
// slots in different banks; rows of only the faces, written word by word,
// measured slower)
__host__ __device__ constexpr int mfma_rs(int nb) { return 16 * ((nb * nb + 15) / 16) + 4; }
// staged rows per level parity: one per slot of the workgroup, plus the x
// boundary row in front and room for the y boundary row after the level
__host__ __device__ constexpr int mfma_rows(int nslot) { return nslot + 3; }

template <int NB, int TPW, bool MULTI>
__device__ __forceinline__ void sweep_mfma_task(const CartSweepArgs& a, const int d, float* smem) {
    constexpr int N = NB * NB;
    constexpr int NI = N + 2 * NB;      // inputs per element
    constexpr int KT = (NI + 3) / 4;    // MFMA steps along the inputs
    constexpr int MT = (N + 15) / 16;   // row tiles
    constexpr int QS = (N + 3) / 4;     // source values per lane
    constexpr int TS = lane_ts(NB);
    constexpr int RW = lane_rw(NB);
    constexpr int RS = mfma_rs(NB);
    // levels between a source load and its use: as many as about 48 registers
    // of prefetched source allow (2 to 8); the loads of a level then arrive
    // while the levels before it are swept
    constexpr int DR = 48 / (TPW * QS);
    constexpr int D = DR < 2 ? 2 : DR > 8 ? 8 : DR;
    constexpr MfmaSlots<NB> SL = mfma_slots<NB>();
    const int nx = a.nx, ny = a.ny, nd = a.nd;
    const long ne = (long)nx * ny;
    const int nlev = nx + ny - 1;
    const int lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int base = wv * 16 * TPW;     // first slot of this wave
    const int nslot = (int)(blockDim.x >> 6) * 16 * TPW;
    const int prow = mfma_rows(nslot) * RS;   // words per parity
    // [2][rows][RS]: level results by parity, slot s in row s + 1; row 0 and
    // the row after the level hold the next level's boundary inflow
    float* stg = smem;
    float* bxl = stg + 2 * prow;        // [ny][TS] boundary inflow of the x faces, by grid row
    float* byl = bxl + ny * TS;         // [nx][TS] boundary inflow of the y faces, by grid column
    const auto om = as_global(a.omega);
    const double ox = om[d * 3], oy = om[d * 3 + 1];
    const bool sx = ox > 0.0, sy = oy > 0.0;
    const unsigned bytes = (unsigned)(ne * N * sizeof(float));   // < 2^31 (checked by the host)
    const auto Sr = buf_rsrc(reinterpret_cast<const float*>(a.S) + (a.s_aniso ? (long)d * ne * N : 0), bytes);
    const auto Pr = buf_rsrc(reinterpret_cast<float*>(a.psi) + (long)d * (a.psi_ld > 0 ? a.psi_ld : ne * N), bytes);
    const auto Mr = buf_rsrc(a.mat, (unsigned)ne);
    const auto tab = as_global(reinterpret_cast<const float*>(a.tab));
    const auto bx = as_global(reinterpret_cast<const float*>(a.bx));
    const auto by = as_global(reinterpret_cast<const float*>(a.by));
    for (int t = threadIdx.x; t < ny * NB; t += blockDim.x) {
        const int jj = t / NB, c = t - jj * NB;
        bxl[jj * TS + c] = bx ? bx[(long)d * ny * NB + t] : 0.f;
    }
    for (int t = threadIdx.x; t < nx * NB; t += blockDim.x) {
        const int ii = t / NB, c = t - ii * NB;
        byl[ii * TS + c] = by ? by[(long)d * nx * NB + t] : 0.f;
    }
    // input held by this lane's slot of step t
    auto slot_q = [&](int t) {
        const int q0 = SL.q[t][0], q1 = SL.q[t][1], q2 = SL.q[t][2], q3 = SL.q[t][3];
        return g == 0 ? q0 : g == 1 ? q1 : g == 2 ? q2 : q3;
    };
    // operator of material mat in A-operand layout; table row (ca, b) holds node ca + NB b
    float af[MT][KT];
    auto load_op = [&](int mat) {
        const long blk = ((long)mat * nd + d) * N;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int row = 16 * mt + j;
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                const int q = slot_q(t);
                af[mt][t] = (row < N && q >= 0) ? tab[(blk + (row % NB) * NB + row / NB) * RW + q] : 0.f;
            }
        }
    };
    int amat = 0;
    load_op(0);
    // the traces in this lane's slots: word of the upstream element's staged
    // row (x face: node column aout of the left neighbour, row s + dl; y face:
    // node row bout of the lower neighbour, row s + dl + 1); tsrc: the slot
    // holds a source value
    const int aout = sx ? NB - 1 : 0;
    const int bout = sy ? NB - 1 : 0;
    int tdel[KT];
    bool tsrc[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        const int e = slot_q(t) - N;   // trace index (negative: source value or padding)
        tsrc[t] = e < 0;
        tdel[t] = e < 0 ? 0 : e < NB ? aout + NB * e : RS + (e - NB) + NB * bout;
    }
    // element of slot s at level l: K = Ku(l) + s dK, Ku(l) that of slot 0
    const int dK = (sx ? 1 : -1) + (sy ? -nx : nx);
    auto lev_i0 = [&](int l) { return l - (ny - 1) > 0 ? l - (ny - 1) : 0; };
    auto lev_len = [&](int l) {
        const int i1 = l < nx - 1 ? l : nx - 1;
        return l < nlev ? i1 - lev_i0(l) + 1 : 0;
    };
    auto lev_K = [&](int l) {
        const int ip = lev_i0(l), jp = l - ip;
        return (sy ? jp : ny - 1 - jp) * nx + (sx ? ip : nx - 1 - ip);
    };
    // per tile of this lane: slot, K offset s dK in bytes of source run / result rows, staged row
    int sl[TPW], lb[TPW], sb[TPW], sr[TPW];
    const int c0 = g * QS;
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        sl[tt] = base + 16 * tt + j;
        lb[tt] = (sl[tt] * dK * N + c0) * 4;
        sb[tt] = (sl[tt] * dK * N + 4 * g) * 4;
        sr[tt] = sl[tt] * RS;
    }
    // this lane's source words c0 .. c0 + QS - 1 of every tile's element at
    // level l (and its material); lanes past the level or past N read zeros
    const bool run1 = c0 + (QS > 4 ? 4 : QS) <= N;   // first vector of the run inside the element
    const bool run2 = c0 + QS <= N;                   // second vector (QS = 7)
    float pre[D][TPW][QS];
    int pmat[D][TPW];
    auto fetch = [&](int l, float(&dst)[TPW][QS], int(&dm)[TPW]) {
        const int len = lev_len(l);
        const int Ku = lev_K(l);
        const unsigned kb = (unsigned)Ku * (unsigned)(N * 4);
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
            // (both arms of every choice computed first, & on bools: selects, not branches)
            const bool act = sl[tt] < len;
            const unsigned w0 = kb + (unsigned)lb[tt], w1 = w0 + 16u;
            const unsigned o0 = (act & run1) ? w0 : BUF_OOB;
            const unsigned o1 = (act & run2) ? w1 : BUF_OOB;
            buf_ld_run<QS>(Sr, o0, o1, dst[tt]);
            if constexpr (MULTI) {
                const unsigned kk = (unsigned)(Ku + sl[tt] * dK);
                const int mv = (int)__builtin_amdgcn_raw_buffer_load_b8(Mr, (int)(act ? kk : BUF_OOB), 0, 0);
                dm[tt] = act ? mv : -1;
            }
        }
    };
    // boundary inflow of level l into the staged buffer level l - 1 leaves it:
    // the x faces of the element at ip = 0 (l < ny) into row 0, the y faces of
    // the element at jp = 0 (l < nx) into the row after level l - 1's last
    // slot; lanes 0 .. 2 NB - 1 of wave 0 read their value early (get) and
    // store it after the level's own work (put)
    const int bt = threadIdx.x;
    auto get_boundary = [&](int l) {
        const int cj = sy ? l : ny - 1 - l, ci = sx ? l : nx - 1 - l;
        const int ox_ = cj * TS + bt, oy_ = ny * TS + ci * TS + bt - NB;
        const bool okx = (bt < NB) & (l < ny), oky = (bt >= NB) & (bt < 2 * NB) & (l < nx);
        return (okx | oky) ? bxl[okx ? ox_ : oy_] : 0.f;
    };
    auto put_boundary = [&](int l, float v) {
        float* q = stg + ((l + 1) & 1) * prow;
        const int row = (l > 0 ? lev_len(l - 1) : 0) + 1;
        if ((bt < NB) & (l < ny)) q[aout + NB * bt] = v;
        else if ((bt >= NB) & (bt < 2 * NB) & (l < nx)) q[row * RS + (bt - NB) + NB * bout] = v;
    };
    const bool one_wave = blockDim.x == 64;   // LDS operations of one wave need no barrier
    auto level_sync = [&]() {
        if (one_wave) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            lds_barrier();
        }
    };
    lds_barrier();   // boundary arrays complete
    put_boundary(0, get_boundary(0));
#pragma unroll
    for (int u = 0; u < D; ++u) fetch(u, pre[u], pmat[u]);
    lds_barrier();
    for (int m0 = 0; m0 < nlev; m0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int m = m0 + u;
            if (m >= nlev) break;
            const int len = lev_len(m);
            const int i0 = lev_i0(m);
            // neighbours at level m - 1: left (x) in slot s - 1 + dl (row s + dl),
            // lower (y) in slot s + dl (row s + dl + 1), dl = i0(m) - i0(m - 1)
            const int dl = m > 0 ? i0 - lev_i0(m - 1) : 0;
            const int pvu = ((m + 1) & 1) * prow + dl * RS;
            float* cur = stg + (m & 1) * prow;
            const unsigned kb = (unsigned)lev_K(m) * (unsigned)(N * 4);
            const float bnext = wv == 0 ? get_boundary(m + 1) : 0.f;
#pragma unroll
            for (int tt = 0; tt < TPW; ++tt) {
                const int s = sl[tt];
                const bool act = s < len;
                v4f acc[MT];
                if (base + 16 * tt < len) {   // wave-uniform: the tile holds elements of this level
                    const int pv = pvu + sr[tt];
                    float bv[KT];
#pragma unroll
                    for (int t = 0; t < KT; ++t) {
                        if (SL.q[t][0] >= 0 && SL.q[t][0] < N && SL.q[t][3] >= 0 && SL.q[t][3] < N) {
                            bv[t] = pre[u][tt][t < QS ? t : 0];
                        } else {
                            const float tv = stg[pv + tdel[t]];
                            const float sv = t < QS ? pre[u][tt][t < QS ? t : 0] : 0.f;
                            bv[t] = tsrc[t] ? sv : tv;
                        }
                    }

                    auto apply = [&](v4f(&o)[MT]) {
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) o[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int t = 0; t < KT; ++t)
#pragma unroll
                            for (int mt = 0; mt < MT; ++mt)
                                o[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mt][t], bv[t], o[mt], 0, 0, 0);
                    };
                    if constexpr (!MULTI) {
                        apply(acc);
                    } else {
                        // one pass per material present in the tile
                        const int cm = act ? pmat[u][tt] : -1;
                        unsigned long long todo = __ballot(act);
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) acc[mt] = v4f{0.f, 0.f, 0.f, 0.f};
                        while (todo) {
                            const int lead = __builtin_ctzll(todo);
                            const int mm = __builtin_amdgcn_readfirstlane(__shfl(cm, lead));
                            if (mm != amat) {
                                load_op(mm);
                                amat = mm;
                            }
                            v4f tmp[MT];
                            apply(tmp);
                            const bool mine = cm == mm;
#pragma unroll
                            for (int mt = 0; mt < MT; ++mt) acc[mt] = mine ? tmp[mt] : acc[mt];
                            todo &= ~__ballot(mine);
                        }
                    }
                    // the level's results for the next level's traces
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        if (act & (16 * mt + 4 * g < N))
                            *reinterpret_cast<v4f*>(cur + sr[tt] + RS + 16 * mt + 4 * g) = acc[mt];
                } else {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) acc[mt] = __builtin_nondeterministic_value(acc[mt]);
                }
                // rows 16 mt + 4 g .. + 3 of element j: one vector store when
                // all four are rows of the element, else word by word
                const unsigned w = kb + (unsigned)sb[tt];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int r0 = 16 * mt + 4 * g;
                    const unsigned wm = w + 64u * mt;
                    const unsigned o4 = (act & (r0 + 4 <= N)) ? wm : BUF_OOB;
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, acc[mt]), Pr, (int)o4, 0, 0);
                    const int part = (N - 16 * mt) > 0 && (N - 16 * mt) < 16 ? (N - 16 * mt) % 4 : 0;
#pragma unroll
                    for (int r = 0; r < part; ++r) {
                        const unsigned wr = wm + 4u * r;
                        const unsigned o1 = (act & (r0 + r < N) & (r0 + 4 > N)) ? wr : BUF_OOB;
                        buf_st(Pr, o1, acc[mt][r]);
                    }
                }
            }
            if (wv == 0) put_boundary(m + 1, bnext);
            fetch(m + D, pre[u], pmat[u]);
            level_sync();
        }
    }
}

template <int NB, int TPW, bool MULTI>
__global__ __launch_bounds__(256) void b_sweep_mfma_kernel(const CartSweepArgs* __restrict__ args,
                                                           const int2* __restrict__ tasks, int ntasks,
                                                           int* __restrict__ counter,
                                                           const int* __restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int tsk;
    while (true) {
        if (threadIdx.x == 0) tsk = atomicAdd(counter, 1);
        __syncthreads();
        const int t = tsk;
        __syncthreads();
        if (t >= ntasks) break;
        const int2 tk = tasks[t];
        if (!active[tk.x]) continue;
        sweep_mfma_task<NB, TPW, MULTI>(args[tk.x], tk.y, reinterpret_cast<float*>(smem));
        __syncthreads();
    }
}

template <int NB, int TPW, bool MULTI>
static hipError_t b_sweep_mfma_tm(int threads, size_t lds, int grid, const CartSweepArgs* args, const int2* tasks,
                                  int ntasks, int* counter, const int* active, hipStream_t s) {
    auto kfn = b_sweep_mfma_kernel<NB, TPW, MULTI>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(threads), lds, s, args, tasks, ntasks, counter, active);
    return hipGetLastError();
}

template <int NB, int TPW>
static hipError_t b_sweep_mfma_t(bool multi, int threads, size_t lds, int grid, const CartSweepArgs* args,
                                 const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s) {
    return multi ? b_sweep_mfma_tm<NB, TPW, true>(threads, lds, grid, args, tasks, ntasks, counter, active, s)
                 : b_sweep_mfma_tm<NB, TPW, false>(threads, lds, grid, args, tasks, ntasks, counter, active, s);
}

template <int NB>
static hipError_t b_sweep_mfma_nb(bool multi, int tpw, int threads, size_t lds, int grid, const CartSweepArgs* args,
                                  const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s) {
    return tpw == 4 ? b_sweep_mfma_t<NB, 4>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s)
                    : b_sweep_mfma_t<NB, 2>(multi, threads, lds, grid, args, tasks, ntasks, counter, active, s);
}

int b_sweep_mfma_threads(int tpw, int nx, int ny) {
    const int maxlen = nx < ny ? nx : ny;
    const int slots = 16 * tpw;
    return 64 * ((maxlen + slots - 1) / slots);
}

size_t b_sweep_mfma_lds(int nb, int tpw, int threads, int nxy) {
    // two levels of staged results (rows of the workgroup's slots and the
    // boundary rows), then the boundary traces of the nx + ny = nxy rows and columns
    const int nslot = threads / 64 * 16 * tpw;
    return sizeof(float) * (2 * (size_t)mfma_rows(nslot) * mfma_rs(nb) + (size_t)nxy * lane_ts(nb));
}

hipError_t b_sweep_mfma(int nb, bool multi, int tpw, int threads, size_t lds, int grid, const CartSweepArgs* args,
                        const int2* tasks, int ntasks, int* counter, const int* active, hipStream_t s) {
    // one wave per 16 tpw slots of the longest anti-diagonal, at most four waves
    if ((tpw != 2 && tpw != 4) || threads < 64 || threads > 256 || threads % 64 != 0 || lds > 160 * 1024)
        return hipErrorNotSupported;
    switch (nb) {
        case 2: return b_sweep_mfma_nb<2>(multi, tpw, threads, lds, grid, args, tasks, ntasks, counter, active, s);
        case 3: return b_sweep_mfma_nb<3>(multi, tpw, threads, lds, grid, args, tasks, ntasks, counter, active, s);
        case 4: return b_sweep_mfma_nb<4>(multi, tpw, threads, lds, grid, args, tasks, ntasks, counter, active, s);
        case 5: return b_sweep_mfma_nb<5>(multi, tpw, threads, lds, grid, args, tasks, ntasks, counter, active, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- moments (matrix cores), optional FP64 accumulation ----------------------
// A block of columns is 64 columns of one problem (Lpad is a multiple of 32,
// so a lane's 4 columns are 16-byte aligned and a direction's 64 columns one
// 256-byte piece of two whole lines; columns >= L read the zero padding).
// FP32: one workgroup of four waves per block; wave q contracts the rounds q,
// q + 4, ... of 8 directions, the partial sums meet in LDS (added in the
// order q = 0..3), and the 8 moment rows leave as whole rows, 64 consecutive
// FP64 values per store (written column by column from the MFMA layout, the
// rows took 0.6 of the kernel's 1.5 ms).  FP64: one wave per block, all
// directions.
template <typename T>
__global__ __launch_bounds__(256) void b_moments_kernel(BatchLaunch B, int accumulate, int first, int with_T) {
    const int lane = threadIdx.x & 63;
    const long w = sizeof(T) == 4 ? (long)blockIdx.x : ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= B.nmw) return;   // FP32: uniform over the workgroup
    const int prob = bsearch_prob(B.mw0, B.nprob, w);
    if (!B.active[prob]) return;
    const BProb& P = B.P[prob];
    const long col0 = (w - P.mw0) * 64;
    const int j = lane & 15, kk = lane >> 4;
    const long c4 = col0 + 4 * j;
    const bool colok = c4 < P.Lpad;
    const T* psi = reinterpret_cast<const T*>(P.psi);
    const T* W;
    if constexpr (sizeof(T) == 4) W = reinterpret_cast<const T*>(P.W32);
    else W = reinterpret_cast<const T*>(P.W64);
    const int nd = P.nd;
    if constexpr (sizeof(T) == 4) {
        __shared__ v4f part[3][4][64];   // the accumulators of waves 1..3
        __shared__ double tile[8][64];   // moment rows 0..7 of the block's columns
        const int q = threadIdx.x >> 6;
        v4f acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
        // U steps of 4 directions per round, all their loads issued first (1
        // or 4 ran slower)
        constexpr int U = 2;
        const auto pg = as_global(reinterpret_cast<const v4f*>(psi));
        for (int k0 = 4 * U * q; k0 < nd; k0 += 16 * U) {
            v4f bv[U];
            float av[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int dk = k0 + 4 * u + kk;
                const bool in = dk < nd && colok;
                bv[u] = pg[in ? ((long)dk * P.Lpad + c4) / 4 : 0];
                if (!in) bv[u] = v4f{0.f, 0.f, 0.f, 0.f};
                av[u] = dk < nd ? W[j * P.ldw + dk] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[u][c], acc[c], 0, 0, 0);
        }
        if (q > 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) part[q - 1][c][lane] = acc[c];
        }
        __syncthreads();
        if (q == 0) {
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += part[p][c][lane];
            // FP32 layout: row 4 kk + r, column 4 j + c
            if (kk < 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c) tile[4 * kk + r][4 * j + c] = (double)acc[c][r];
            }
        }
        __syncthreads();
        const long col = col0 + lane;
        if (col < P.L) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = 2 * q + i;
                const long o = (long)row * P.L + col;
                const double v = tile[row][lane];
                if (accumulate) {
                    const double a = (first ? 0.0 : P.mom_acc[o]) + v;
                    P.mom_acc[o] = a;
                    tile[row][lane] = a;   // (each thread rewrites only what it read)
                } else {
                    P.mom[o] = v;
                }
            }
        }
        // the closure T from the accumulated rows, as b_T_kernel forms it (the
        // rows are in LDS already: that kernel's reads are saved)
        if (with_T && accumulate) {
            __syncthreads();
            if (q == 0 && col < P.L) {
                const double phi = tile[0][lane];
                P.T[col] = tile[3][lane] - phi / 3.0;
                P.T[P.L + col] = tile[4][lane];
                P.T[2 * P.L + col] = tile[5][lane] - phi / 3.0;
            }
        }
    } else {
        v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0, a2 = a0, a3 = a0;
        for (int k = 0; k < nd; k += 4) {
            const int dk = k + kk;
            const double av = dk < nd ? W[j * P.ldw + dk] : 0.0;
            v2d b01 = {0.0, 0.0}, b23 = {0.0, 0.0};
            if (dk < nd && colok) {
                const v2d* src = reinterpret_cast<const v2d*>(psi + (long)dk * P.Lpad + c4);
                b01 = src[0];
                b23 = src[1];
            }
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b01[0], a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b01[1], a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b23[0], a2, 0, 0, 0);
            a3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b23[1], a3, 0, 0, 0);
        }
        // FP64 layout: row kk + 4 r
        if (colok) {
            for (int r = 0; r < 2; ++r) {
                const int row = kk + 4 * r;
                const double vals[4] = {a0[r], a1[r], a2[r], a3[r]};
                for (int c = 0; c < 4; ++c) {
                    const long col = c4 + c;
                    if (col >= P.L) break;
                    const long o = (long)row * P.L + col;
                    if (accumulate) P.mom_acc[o] = (first ? 0.0 : P.mom_acc[o]) + vals[c];
                    else P.mom[o] = vals[c];
                }
            }
        }
    }
}

hipError_t b_moments(bool fp64, const BatchLaunch& B, bool accumulate, bool first, hipStream_t s, bool with_T) {
    const long blocks = fp64 ? (B.nmw + 3) / 4 : B.nmw;
    if (fp64)
        hipLaunchKernelGGL(b_moments_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, B, accumulate ? 1 : 0,
                           first ? 1 : 0, 0);
    else
        hipLaunchKernelGGL(b_moments_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, B, accumulate ? 1 : 0,
                           first ? 1 : 0, with_T && accumulate ? 1 : 0);
    return hipGetLastError();
}

// ---- closures and right-hand side --------------------------------------------
// T from the moments (which array: mom_acc when accumulating, else mom -- the
// host passes that choice through BProb.mom_acc == mom when not accumulating).
__global__ __launch_bounds__(BT) void b_T_kernel(BatchLaunch B) {
    const EB m = eb_map(B);
    if (!B.active[m.prob] || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i, L = P.L;
    const double* mom = P.mom_acc;
    const double phi = mom[t];
    P.T[t] = mom[3 * L + t] - phi / 3.0;
    P.T[L + t] = mom[4 * L + t];
    P.T[2 * L + t] = mom[5 * L + t] - phi / 3.0;
}

__global__ __launch_bounds__(256) void b_beta_kernel(BatchLaunch B) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B.nbq) return;
    const int prob = bsearch_prob(B.bq0, B.nprob, t);
    if (!B.active[prob]) return;
    const BProb& P = B.P[prob];
    const long lt = t - P.bq0;
    const int bf = (int)(lt / P.nq), q = (int)(lt - (long)bf * P.nq);
    const int K = P.bK[bf], f = P.bF[bf], nb = P.nb;
    const bool xnorm = (f == 1 || f == 3);
    const double* mom = P.mom_acc;
    const double* row = mom + (xnorm ? 6 : 7) * P.L;
    const double e = xnorm ? P.eb0x : P.eb0y;
    double v = 0.0;
    for (int c = 0; c < nb; ++c) {
        int k;
        switch (f) {
            case 0: k = c; break;
            case 1: k = (nb - 1) + nb * c; break;
            case 2: k = c + nb * (nb - 1); break;
            default: k = nb * c; break;
        }
        const long idx = (long)K * P.n + k;
        v += P.Lf[c * P.nq + q] * (row[idx] - e * mom[idx]);
    }
    P.beta[lt] = v;
}

__device__ __forceinline__ int nbr_of(const BProb& P, int K, int f) {
    switch (f) {
        case 0: return K - P.nx;
        case 1: return K + 1;
        case 2: return K + P.nx;
        default: return K - 1;
    }
}

// b = b_fixed + C_self T_K + sum_f C_nbr T_N - sum_{boundary f} B_f beta_f
__global__ __launch_bounds__(BT) void b_rhs_kernel(BatchLaunch B) {
    const EB m = eb_map(B);
    if (!B.active[m.prob] || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    if (B.grouped) return;  // on the matrix cores (rhs_group_mfma)
    const int n = P.n, n3 = 3 * n, K = m.K, i = m.i;
    const long L = P.L;
    double v = P.bfix[(long)K * n + i];
    // blocks are stored column-major: entry (i, col) at col * n + i
    {
        const double* col = P.c_self + (long)P.sid[K] * n * n3 + i;
        for (int c = 0; c < 3; ++c) {
            const double* tv = P.T + c * L + (long)K * n;
            for (int j = 0; j < n; ++j) v += col[(c * n + j) * n] * tv[j];
        }
    }
    for (int f = 0; f < 4; ++f) {
        const int t = P.nid[K * 4 + f];
        if (t >= 0) {
            const int N = nbr_of(P, K, f);
            const double* col = P.c_nbr + (long)t * n * n3 + i;
            for (int c = 0; c < 3; ++c) {
                const double* tv = P.T + c * L + (long)N * n;
                for (int j = 0; j < n; ++j) v += col[(c * n + j) * n] * tv[j];
            }
        } else {
            const int bf = P.bface_of[K * 4 + f];
            const double* bo = P.bop + (long)f * P.nq * n + i;
            const double* be = P.beta + (long)bf * P.nq;
            for (int q = 0; q < P.nq; ++q) v -= bo[q * n] * be[q];
        }
    }
    P.b[(long)K * n + i] = v;
}

hipError_t b_closures_rhs(const BatchLaunch& B, hipStream_t s, bool t_done) {
    if (!t_done) hipLaunchKernelGGL(b_T_kernel, dim3(B.nblocks), dim3(BT), 0, s, B);
    if (B.nbq > 0) hipLaunchKernelGGL(b_beta_kernel, dim3((unsigned)((B.nbq + 255) / 256)), dim3(256), 0, s, B);
    if (B.grouped)
        b_group_rows_all<1>(B, s);
    else
        hipLaunchKernelGGL(b_rhs_kernel, dim3(B.nblocks), dim3(BT), 0, s, B);
    return hipGetLastError();
}

__global__ __launch_bounds__(BT) void b_copy_x_kernel(BatchLaunch B) {
    const EB m = eb_map(B);
    if (!B.active[m.prob] || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i;
    P.x[t] = P.varphi[t];
}

__global__ __launch_bounds__(BT) void b_shift_kernel(BatchLaunch B) {
    const EB m = eb_map(B);
    if (!B.active[m.prob] || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i;
    P.varphi_prev[t] = P.varphi[t];
    P.varphi[t] = P.x[t];
}

// Vectors of a solve's start for every problem of the batch in one launch
// (instead of a copy or fill per problem and vector): bit 1 varphi_prev = 0,
// 2 varphi = 0, 4 b = bfix and x = 0, 8 varphi = x.
__global__ __launch_bounds__(BT) void b_start_vectors_kernel(BatchLaunch B, int what) {
    const EB m = eb_map(B);
    if (m.K < 0) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i;
    if (what & 1) P.varphi_prev[t] = 0.0;
    if (what & 2) P.varphi[t] = 0.0;
    if (what & 4) {
        P.b[t] = P.bfix[t];
        P.x[t] = 0.0;
    }
    if (what & 8) P.varphi[t] = P.x[t];
}

hipError_t b_start_vectors(const BatchLaunch& B, int what, hipStream_t s) {
    hipLaunchKernelGGL(b_start_vectors_kernel, dim3(B.nblocks), dim3(BT), 0, s, B, what);
    return hipGetLastError();
}

hipError_t b_copy_x(const BatchLaunch& B, hipStream_t s) {
    hipLaunchKernelGGL(b_copy_x_kernel, dim3(B.nblocks), dim3(BT), 0, s, B);
    return hipGetLastError();
}

hipError_t b_shift(const BatchLaunch& B, hipStream_t s) {
    hipLaunchKernelGGL(b_shift_kernel, dim3(B.nblocks), dim3(BT), 0, s, B);
    return hipGetLastError();
}

// ---- typed block-Jacobi PCG --------------------------------------------------
// Per-problem scalars (P.scal): 0 rz, 1 rz_old, 2 bb, 3 rr, 4 done, 5 iterations,
// 6 breakdown, 7 tol^2 bb, 8 alpha, 9 beta, 12 the iteration that converged
// while its x += alpha p is still owed (else -1).  With the type-group kernels
// x += alpha p is applied by the direction update, which reads p anyway (the
// update kernel then reads neither x nor p): in the iteration that converges
// the direction update still runs for x, and the next iteration's first
// reduction clears the mark.
// fixed-order sum over the workgroup: wave 0 adds the BT / 64 values of its
// lane's stride, then a butterfly over the wave (three barriers; a tree over
// the workgroup took nine)
__device__ __forceinline__ double b_block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    if (t < 64) {
        double s = red[t];
#pragma unroll
        for (int i = 1; i < BT / 64; ++i) s += red[64 * i + t];
        s = wave_sum(s);
        if (t == 0) red[0] = s;
    }
    __syncthreads();
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double typed_row(const BProb& P, const double* x, int K, int i) {
    const int n = P.n;
    // column-major blocks: entry (i, j) at j * n + i, so the n lanes of an
    // element read n consecutive doubles per j
    const double* col = P.ip_self + (long)P.sid[K] * n * n + i;
    const double* xv = x + (long)K * n;
    double v = 0.0;
    for (int j = 0; j < n; ++j) v += col[j * n] * xv[j];
    for (int f = 0; f < 4; ++f) {
        const int t = P.nid[K * 4 + f];
        if (t < 0) continue;
        const double* cn = P.ip_nbr + (long)t * n * n + i;
        const double* xn = x + (long)nbr_of(P, K, f) * n;
        for (int j = 0; j < n; ++j) v += cn[j * n] * xn[j];
    }
    return v;
}

// node of the continuous Q_p grid ((nx p + 1) x (ny p + 1)) that DG node j of
// element K sits on
__device__ __forceinline__ int cg_node(const BProb& P, int K, int j) {
    const int p = P.nb - 1, gx = P.nx * p + 1;
    return ((K / P.nx) * p + j / P.nb) * gx + (K % P.nx) * p + j % P.nb;
}

__device__ __forceinline__ bool cg_skip(const BatchLaunch& B, int prob) {
    return !B.active[prob] || B.P[prob].scal[4] != 0.0;
}

__global__ __launch_bounds__(BT) void b_cg_init1(BatchLaunch B) {
    const EB m = eb_map(B);
    if (!B.active[m.prob] || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    if (B.grouped) return;  // on the matrix cores (init1_group_mfma)
    const long t = (long)m.K * P.n + m.i;
    P.r[t] = P.b[t] - typed_row(P, P.x, m.K, m.i);
}

// z = D^-1 r, p = z, and the block's partial sums of r.z, r.r, b.b.  The
// block's residuals are staged in LDS (one coalesced load each), the three
// sums reduced in one pass: the products in LDS, 32 lanes per sum adding
// BT / 32 values each (strided), then a butterfly over the 32.
__global__ __launch_bounds__(BT) void b_cg_init2(BatchLaunch B) {
    __shared__ double red[3][BT];
    __shared__ double rl[BT];
    const EB m = eb_map(B);
    const bool act = B.active[m.prob] && m.K >= 0;
    const BProb& P = B.P[m.prob];
    const long t = act ? (long)m.K * P.n + m.i : 0;
    const double rv = act ? P.r[t] : 0.0;
    rl[threadIdx.x] = rv;
    __syncthreads();
    double v[3] = {0.0, 0.0, 0.0};
    if (act) {
        const int n = P.n;
        const double* D = P.dinv + (long)P.sid[m.K] * n * n + m.i;
        double z = 0;
        for (int j = 0; j < n; ++j) z += D[j * n] * rl[m.e0 + j];
        P.z[t] = z;
        P.p[t] = z;
        const double bv = P.b[t];
        v[0] = rv * z;
        v[1] = rv * rv;
        v[2] = bv * bv;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    if (threadIdx.x < 3 * 32) {
        const int k = threadIdx.x >> 5, c = threadIdx.x & 31;
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < BT / 32; ++i) sum += red[k][32 * i + c];
        for (int off = 16; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 32);
        if (c == 0) B.part[(long)k * B.nblocks + blockIdx.x] = sum;
    }
}

// one workgroup per problem: fixed-order sums of the problem's partials
__device__ __forceinline__ double prob_sum(const BatchLaunch& B, const BProb& P, int which, double* red) {
    double v = 0.0;
    for (int k = threadIdx.x; k < P.nblk; k += BT) v += B.part[which * B.nblocks + P.blk0 + k];
    return b_block_sum(v, red);
}

__global__ __launch_bounds__(BT) void b_cg_red_init(BatchLaunch B, double tol) {
    __shared__ double red[BT];
    const int prob = blockIdx.x;
    const BProb& P = B.P[prob];
    const double rz = prob_sum(B, P, 0, red), rr = prob_sum(B, P, 1, red), bb = prob_sum(B, P, 2, red);
    if (threadIdx.x == 0) {
        double* s = P.scal;
        s[0] = rz;
        s[1] = rz;
        s[2] = bb;
        s[3] = rr;
        const double t = B.ptol ? B.ptol[prob] : tol;
        s[7] = t * t * bb;
        s[4] = (!B.active[prob] || rr <= s[7]) ? 1.0 : 0.0;
        s[5] = 0.0;
        s[6] = 0.0;
    }
}

// ---- grouped PCG kernels -----------------------------------------------------
// One wave per type group: its (up to 64) elements share the typed blocks of
// their self and four face couplings, so the block entries are wave-uniform and
// come through scalar loads (SGPR operands of the FMAs), while each lane keeps
// one element's vectors in registers.

// y += A x with A column-major [N][N] (entry (i, j) at j N + i) and x read
// from memory one entry per step (rolled loop over j, y in registers).  A is
// wave-uniform and read-only for the whole kernel: it is read through the
// constant address space, so its entries arrive by scalar loads and enter
// the FMAs as SGPR operands.
typedef const double __attribute__((address_space(4)))* cdptr;

__device__ __forceinline__ cdptr as_const(const double* p) {
    const unsigned long v = (unsigned long)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return (cdptr)(((unsigned long)hi << 32) | lo);
}

template <int N>
__device__ __forceinline__ void block_mv(const double* Ag, const double* __restrict__ x, double (&y)[N]) {
    const cdptr A = as_const(Ag);
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
        const double xj = x[j];
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] += A[j * N + i] * xj;
    }
}

// LDS of a grouped kernel: one slice per wave holding one vector per element
// of the group, row stride N | 1 doubles (odd, so the 64 lanes' rows fall in
// distinct banks).  Global vectors move in and out of it with element-major
// flat indices t = e N + j, so those accesses are coalesced.

__device__ __forceinline__ void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <int NB>
__device__ __forceinline__ void k1_group(const BatchLaunch& B, const BProb& P, int g, int cnt, double* xs) {
    constexpr int N = NB * NB, S = N | 1;
    const int lane = threadIdx.x & 63;
    const int* ty = B.g_ty + g * 5;
    const int myK = B.g_elem[g * 64 + lane];  // every slot holds a valid element
    const int tot = cnt * N;
    double y[N];
#pragma unroll
    for (int i = 0; i < N; ++i) y[i] = 0.0;
    // flat index u = e N + j over the group's vectors of face f (0: the
    // elements themselves, 1-4: their neighbours): lane-consecutive, so the
    // global reads are coalesced
    const auto pg = as_global((const double*)P.p);
    auto load_face = [&](int f, double(&v)[N]) {
#pragma unroll
        for (int it = 0; it < N; ++it) {
            const int u = lane + 64 * it;
            const int e = u / N < 64 ? u / N : 63;
            const int K = __shfl(myK, e);
            const int src = f == 0 ? K : nbr_of(P, K, f - 1);
            v[it] = ld_at(pg, u < tot ? (unsigned)(src * N + (u - (u / N) * N)) : 0u);
        }
    };
    // faces with a neighbour type (wave-uniform: a boundary face of one
    // element of the group is a boundary face of all of them)
    auto next_face = [&](int f) {
        ++f;
        while (f < 5 && ty[f] < 0) ++f;
        return f;
    };
    double v[N];
    load_face(0, v);
    for (int f = 0; f < 5;) {
        const int fn = next_face(f);
        // the next face's vectors are loaded while this face is multiplied
        double vn[N];
        if (fn < 5) load_face(fn, vn);
#pragma unroll
        for (int it = 0; it < N; ++it) {
            const int u = lane + 64 * it;
            if (u < tot) xs[(u / N) * S + (u - (u / N) * N)] = v[it];
        }
        lds_wave_sync();
        block_mv<N>((f == 0 ? P.ip_self : P.ip_nbr) + (long)ty[f] * N * N, xs + lane * S, y);
        lds_wave_sync();
        if (fn < 5)
#pragma unroll
            for (int it = 0; it < N; ++it) v[it] = vn[it];
        f = fn;
    }
    if (lane < cnt)
#pragma unroll
        for (int i = 0; i < N; ++i) xs[lane * S + i] = y[i];
    lds_wave_sync();
    double pq = 0.0;
    const auto qg = as_global(P.q);
#pragma unroll
    for (int it = 0; it < N; ++it) {
        const int u = lane + 64 * it;
        const int e = u / N < 64 ? u / N : 63;
        const int K = __shfl(myK, e);
        if (u < tot) {
            const unsigned o = (unsigned)(K * N + (u - (u / N) * N));
            const double qv = xs[(u / N) * S + (u - (u / N) * N)];
            st_at(qg, o, qv);
            pq += ld_at(pg, o) * qv;
        }
    }
    pq = wave_sum(pq);
    if (lane == 0) B.gpart[g] = pq;
}

// q = A p of one group on the FP64 matrix cores.  Per face the group's block
// product Y (N x 64) += A_f (N x N) X_f (N x 64) is a dense contraction, done
// in 16 x 16 x 4 tiles (rows padded to MB 16, the contraction to KS 4 with
// zeros): A fragments come from global memory (the typed blocks are shared by
// all groups, so they are cache hits) and are loaded before the next face's
// vectors, so waiting for them never waits for the prefetch; X fragments come
// from the face's vectors staged in LDS.  Tile layouts (v_mfma_f64_16x16x4):
// lane (i, k) = (lane % 16, lane / 16) holds A[i][k] and B[k][i]; element r
// of the result holds D[4 r + k][i].
template <int NB>
__device__ __forceinline__ void k1_group_mfma(const BatchLaunch& B, const BProb& P, int g, int cnt, double* xs) {
    constexpr int N = NB * NB, S = N | 1;
    constexpr int MB = (N + 15) / 16, KS = (N + 3) / 4;
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    const int* ty = B.g_ty + g * 5;
    const int myK = B.g_elem[g * 64 + lane];  // every slot holds a valid element
    const auto pg = as_global((const double*)P.p);
    // lane = element: its vector of face f (0: the element itself, 1-4: its
    // neighbours) is N consecutive words, loaded at immediate offsets
    auto load_face = [&](int f, double(&v)[N]) {
        const int src = f == 0 ? myK : nbr_of(P, myK, f - 1);
        const auto row = pg + (unsigned)(src * N);
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = row[j];
    };
    auto next_face = [&](int f) {
        ++f;
        while (f < 5 && ty[f] < 0) ++f;
        return f;
    };
    // block entries of face f (column-major: (i, k) at k N + i) as A tiles
    auto load_blocks = [&](int f, double(&a)[KS][MB]) {
        const auto A = as_global((f == 0 ? P.ip_self : P.ip_nbr) + (long)ty[f] * N * N);
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int rb = 0; rb < MB; ++rb) {
                const int k = 4 * s + kq, r = 16 * rb + i16;
                const bool in = k < N && r < N;
                a[s][rb] = ld_at(A, in ? (unsigned)(k * N + r) : 0u);
                if (!in) a[s][rb] = 0.0;
            }
    };
    v4d acc[MB][4];
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = v4d{0.0, 0.0, 0.0, 0.0};
    double v[N];
    double a[KS][MB];
    load_blocks(0, a);
    load_face(0, v);
    for (int f = 0; f < 5;) {
        const int fn = next_face(f);
#pragma unroll
        for (int j = 0; j < N; ++j) xs[lane * S + j] = v[j];
        lds_wave_sync();
        // the next face's blocks and vectors are loaded while this face's
        // tiles run (unconditionally: after the last face, face 0 again,
        // unused), so the values just staged are dead and their registers
        // are reused
        double an[KS][MB];
        load_blocks(fn < 5 ? fn : 0, an);
        load_face(fn < 5 ? fn : 0, v);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + kq;
            double bf[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) bf[cb] = k < N ? xs[(16 * cb + i16) * S + k] : 0.0;
#pragma unroll
            for (int rb = 0; rb < MB; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s][rb], bf[cb], acc[rb][cb], 0, 0, 0);
        }
        lds_wave_sync();
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int rb = 0; rb < MB; ++rb) a[s][rb] = an[s][rb];
        f = fn;
    }
    // result tiles to LDS (element e = 16 cb + i16, row 16 rb + 4 r + kq),
    // then each lane stores its element's q and forms its part of p.q
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + 4 * r + kq;
                if (row < N) xs[(16 * cb + i16) * S + row] = acc[rb][cb][r];
            }
    lds_wave_sync();
    // q stored flat element-major (coalesced: per-lane rows would write each
    // cache line in many partial pieces)
    double pq = 0.0;
    const auto qg = as_global(P.q);
    const int tot = cnt * N;
#pragma unroll
    for (int it = 0; it < N; ++it) {
        const int u = lane + 64 * it;
        const int e = u / N < 64 ? u / N : 63;
        const int j = u - (u / N) * N;
        const int K = __shfl(myK, e);
        if (u < tot) {
            const unsigned o = (unsigned)(K * N + j);
            const double qv = xs[e * S + j];
            st_at(qg, o, qv);
            pq += ld_at(pg, o) * qv;
        }
    }
    pq = wave_sum(pq);
    if (lane == 0) B.gpart[g] = pq;
}

// Block-row product of one group on the FP64 matrix cores, general form:
// Y (N x 64) = sum over items t < NT of A_t (N x N, column-major) X_t (N x 64),
// item t being (face f(t), vector v(t)): X_t holds, for element e of the
// group, the N words at v(t) + N K_f(e), K_f(e) the element itself (f = 0) or
// its neighbour across face f - 1.  Items whose face is a boundary face of
// the group are skipped.  Same tiles and staging as k1_group_mfma; the result
// is left in LDS, row e = lane of element e (stride S = N | 1).
template <int NB, int NT, class Item>
__device__ __forceinline__ void group_rows_mfma(const BatchLaunch& B, const BProb& P, int g, double* xs,
                                                Item item) {
    constexpr int N = NB * NB, S = N | 1;
    constexpr int MB = (N + 15) / 16, KS = (N + 3) / 4;
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    const int* ty = B.g_ty + g * 5;
    const int myK = B.g_elem[g * 64 + lane];
    // item t: face f, block pointer blk, vector base vec
    auto valid = [&](int t) {
        int f;
        const double* blk;
        const double* vec;
        item(t, f, blk, vec);
        return f == 0 || ty[f] >= 0;
    };
    auto next_item = [&](int t) {
        ++t;
        while (t < NT && !valid(t)) ++t;
        return t;
    };
    auto load_item = [&](int t, double(&a)[KS][MB], double(&v)[N]) {
        int f;
        const double* blk;
        const double* vec;
        item(t, f, blk, vec);
        const auto A = as_global(blk);
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int rb = 0; rb < MB; ++rb) {
                const int k = 4 * s + kq, r = 16 * rb + i16;
                const bool in = k < N && r < N;
                a[s][rb] = ld_at(A, in ? (unsigned)(k * N + r) : 0u);
                if (!in) a[s][rb] = 0.0;
            }
        const int src = f == 0 ? myK : nbr_of(P, myK, f - 1);
        const auto row = as_global(vec) + (unsigned)(src * N);
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = row[j];
    };
    v4d acc[MB][4];
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = v4d{0.0, 0.0, 0.0, 0.0};
    double v[N];
    double a[KS][MB];
    int t = valid(0) ? 0 : next_item(0);
    if (t < NT) load_item(t, a, v);
    while (t < NT) {
        const int tn = next_item(t);
#pragma unroll
        for (int j = 0; j < N; ++j) xs[lane * S + j] = v[j];
        lds_wave_sync();
        double an[KS][MB];
        load_item(tn < NT ? tn : t, an, v);  // unconditional: the staged values are dead
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + kq;
            double bf[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) bf[cb] = k < N ? xs[(16 * cb + i16) * S + k] : 0.0;
#pragma unroll
            for (int rb = 0; rb < MB; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s][rb], bf[cb], acc[rb][cb], 0, 0, 0);
        }
        lds_wave_sync();
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int rb = 0; rb < MB; ++rb) a[s][rb] = an[s][rb];
        t = tn;
    }
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + 4 * r + kq;
                if (row < N) xs[(16 * cb + i16) * S + row] = acc[rb][cb][r];
            }
    lds_wave_sync();
}

// Flat element-major store of a group's rows held in LDS (row e at e S):
// out[K_e N + j] = op(j-th word of row e, in[K_e N + j]), consecutive lanes on
// consecutive words, so the stores are coalesced.
template <int NB, class Op>
__device__ __forceinline__ void group_store_flat(const BatchLaunch& B, int g, int cnt, const double* xs,
                                                 const double* in, double* out, Op op) {
    constexpr int N = NB * NB, S = N | 1;
    const int lane = threadIdx.x & 63;
    const int myK = B.g_elem[g * 64 + lane];
    const int tot = cnt * N;
    const auto ig = as_global(in);
    const auto og = as_global(out);
#pragma unroll
    for (int it = 0; it < N; ++it) {
        const int u = lane + 64 * it;
        const int e = u / N < 64 ? u / N : 63;
        const int j = u - (u / N) * N;
        const int K = __shfl(myK, e);
        if (u < tot) {
            const unsigned o = (unsigned)(K * N + j);
            st_at(og, o, op(xs[e * S + j], ld_at(ig, o)));
        }
    }
}

// r = b - A x for one group (the PCG start), with group_rows_mfma
template <int NB>
__device__ __forceinline__ void init1_group_mfma(const BatchLaunch& B, const BProb& P, int g, int cnt, double* xs) {
    constexpr int N = NB * NB;
    const int* ty = B.g_ty + g * 5;
    group_rows_mfma<NB, 5>(B, P, g, xs, [&](int t, int& f, const double*& blk, const double*& vec) {
        f = t;
        blk = (t == 0 ? P.ip_self : P.ip_nbr) + (long)ty[t] * N * N;
        vec = P.x;
    });
    group_store_flat<NB>(B, g, cnt, xs, P.b, P.r, [](double ax, double b) { return b - ax; });
}

// IP right-hand side of one group: b = bfix + sum over faces and closure
// components c of C_f[:, c] T_c (C_f column-major n x 3n, so component c is
// the n x n block at offset c n^2), minus the boundary terms of the group's
// boundary faces (all its elements share them)
template <int NB>
__device__ __forceinline__ void rhs_group_mfma(const BatchLaunch& B, const BProb& P, int g, int cnt, double* xs) {
    constexpr int N = NB * NB, S = N | 1;
    const int* ty = B.g_ty + g * 5;
    const long L = P.L;
    group_rows_mfma<NB, 15>(B, P, g, xs, [&](int t, int& f, const double*& blk, const double*& vec) {
        f = t / 3;
        const int c = t - 3 * f;
        blk = (f == 0 ? P.c_self : P.c_nbr) + ((long)ty[f] * 3 + c) * N * N;
        vec = P.T + c * L;
    });
    const int lane = threadIdx.x & 63;
    bool bnd = false;
    for (int f = 0; f < 4; ++f) bnd = bnd || ty[f + 1] < 0;
    if (bnd) {  // wave-uniform: boundary terms on the element's row in LDS
        if (lane < cnt) {
            const int K = B.g_elem[g * 64 + lane];
            for (int f = 0; f < 4; ++f) {
                if (ty[f + 1] >= 0) continue;
                const int bf = P.bface_of[K * 4 + f];
                const double* bo = P.bop + (long)f * P.nq * N;
                const double* be = P.beta + (long)bf * P.nq;
                for (int q = 0; q < P.nq; ++q) {
                    const double w = be[q];
#pragma unroll
                    for (int j = 0; j < N; ++j) xs[lane * S + j] -= bo[q * N + j] * w;
                }
            }
        }
        lds_wave_sync();
    }
    group_store_flat<NB>(B, g, cnt, xs, P.bfix, P.b, [](double y, double bfix) { return bfix + y; });
}

template <int NB, int MODE>
__global__ __launch_bounds__(256, 2) void b_group_rows(BatchLaunch B) {
    constexpr int SL = 64 * (NB * NB | 1);
    __shared__ double lds[4 * SL];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = B.g_nb0[NB] + xcd_block() * 4 + w;
    if (g >= B.g_nb0[NB + 1]) return;
    const int prob = B.g_prob[g];
    if (!B.active[prob]) return;
    const BProb& P = B.P[prob];
    if constexpr (MODE == 0)
        init1_group_mfma<NB>(B, P, g, B.g_count[g], lds + w * SL);
    else
        rhs_group_mfma<NB>(B, P, g, B.g_count[g], lds + w * SL);
}

// grouped launches of b_group_rows, one per order present
template <int MODE>
static void b_group_rows_all(const BatchLaunch& B, hipStream_t s) {
    auto go = [&](auto kfn, int nb) {
        const int ng = B.g_nb0[nb + 1] - B.g_nb0[nb];
        if (ng > 0) hipLaunchKernelGGL(kfn, dim3((ng + 3) / 4), dim3(256), 0, s, B);
    };
    go(b_group_rows<2, MODE>, 2);
    go(b_group_rows<3, MODE>, 3);
    go(b_group_rows<4, MODE>, 4);
    go(b_group_rows<5, MODE>, 5);
}

// One launch per order: the groups of order NB are [g_nb0[NB], g_nb0[NB + 1]),
// so each order gets its own register and LDS footprint.
template <int NB>
__global__ __launch_bounds__(256, 2) void b_cg_k1(BatchLaunch B) {
    constexpr int SL = 64 * (NB * NB | 1);
    __shared__ double lds[4 * SL];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = B.g_nb0[NB] + xcd_block() * 4 + w;
    if (g >= B.g_nb0[NB + 1]) return;  // wave-uniform; no workgroup barriers below
    const int prob = B.g_prob[g];
    if (cg_skip(B, prob)) return;
    const BProb& P = B.P[prob];
    if constexpr (NB >= 3)
        k1_group_mfma<NB>(B, P, g, B.g_count[g], lds + w * SL);
    else
        k1_group<NB>(B, P, g, B.g_count[g], lds + w * SL);
}

// ---- per-node PCG kernels (element blocks of BT threads; used when the type
// groups of a batch are sparsely filled) ----------------------------------------
// q = A p and the block's partial sum of p.q.  The p values of the block's
// elements and of their four neighbours are staged in LDS once; thread
// (pair, i) then computes node i of two neighbouring elements, so one load of
// a column entry of a typed block serves both when they share the type.
// (The per-element blocks per workgroup, BT / n, are even for n = 4, 9, 16, 25.)
__device__ __forceinline__ void typed_dot2(const double* __restrict__ ca, const double* __restrict__ cb, bool same,
                                           const double* __restrict__ xa, const double* __restrict__ xb, int n,
                                           double& ya, double& yb) {
    if (same) {
        for (int j = 0; j < n; ++j) {
            const double m = ca[j * n];
            ya += m * xa[j];
            yb += m * xb[j];
        }
    } else {
        for (int j = 0; j < n; ++j) {
            ya += ca[j * n] * xa[j];
            yb += cb[j * n] * xb[j];
        }
    }
}

__global__ __launch_bounds__(BT) void b_cg_k1n(BatchLaunch B) {
    __shared__ double red[BT];
    __shared__ double xs[5 * BT];  // [element][self, 4 neighbours][n]
    const int prob = B.blk2p[blockIdx.x];
    if (cg_skip(B, prob)) return;  // block-uniform
    const BProb& P = B.P[prob];
    const int n = P.n, epb = BT / n, t = threadIdx.x;
    const int K0 = (blockIdx.x - P.blk0) * epb;
    {
        const int le = t / n, i = t - le * n, K = K0 + le;
        if (le < epb && K < P.ne) {
            double* xk = xs + le * 5 * n;
            xk[i] = P.p[(long)K * n + i];
            for (int f = 0; f < 4; ++f)
                xk[(f + 1) * n + i] = P.nid[K * 4 + f] >= 0 ? P.p[(long)nbr_of(P, K, f) * n + i] : 0.0;
        }
    }
    __syncthreads();
    double pq = 0;
    const int pr = t / n, i = t - pr * n;
    const int la = 2 * pr, lb = la + 1, Ka = K0 + la, Kb = K0 + lb;
    if (la < epb && Ka < P.ne) {
        const bool vb = lb < epb && Kb < P.ne;
        const double* xa = xs + la * 5 * n;
        const double* xb = vb ? xs + lb * 5 * n : xa;
        const int Kc = vb ? Kb : Ka;
        double ya = 0, yb = 0;
        const int sa = P.sid[Ka], sb = P.sid[Kc];
        typed_dot2(P.ip_self + (long)sa * n * n + i, P.ip_self + (long)sb * n * n + i, sa == sb, xa, xb, n, ya, yb);
        for (int f = 0; f < 4; ++f) {
            const int ta = P.nid[Ka * 4 + f], tb = P.nid[Kc * 4 + f];
            if (ta >= 0 && tb >= 0) {
                typed_dot2(P.ip_nbr + (long)ta * n * n + i, P.ip_nbr + (long)tb * n * n + i, ta == tb,
                           xa + (f + 1) * n, xb + (f + 1) * n, n, ya, yb);
            } else {
                double dummy = 0;
                if (ta >= 0) typed_dot2(P.ip_nbr + (long)ta * n * n + i, nullptr, true, xa + (f + 1) * n, xa + (f + 1) * n, n, ya, dummy);
                if (tb >= 0) typed_dot2(P.ip_nbr + (long)tb * n * n + i, nullptr, true, xb + (f + 1) * n, xb + (f + 1) * n, n, yb, dummy);
            }
        }
        P.q[(long)Ka * n + i] = ya;
        pq = xa[i] * ya;
        if (vb) {
            P.q[(long)Kb * n + i] = yb;
            pq += xb[i] * yb;
        }
    }
    pq = b_block_sum(pq, red);
    if (t == 0) B.part[blockIdx.x] = pq;
}

// x += alpha p, r -= alpha q, z = D^-1 r (block-Jacobi; two elements per
// thread as in b_cg_k1) and the partial sums of r.z and r.r.
__global__ __launch_bounds__(BT) void b_cg_k2n(BatchLaunch B) {
    __shared__ double red[BT];
    __shared__ double rl[BT];
    const int prob = B.blk2p[blockIdx.x];
    if (cg_skip(B, prob)) return;  // block-uniform
    const BProb& P = B.P[prob];
    const double alpha = P.scal[8];
    const int n = P.n, epb = BT / n, t = threadIdx.x;
    const int K0 = (blockIdx.x - P.blk0) * epb;
    double rr = 0;
    {
        const int le = t / n, i = t - le * n, K = K0 + le;
        double rnew = 0;
        if (le < epb && K < P.ne) {
            const long g = (long)K * n + i;
            P.x[g] += alpha * P.p[g];
            rnew = P.r[g] - alpha * P.q[g];
            P.r[g] = rnew;
        }
        rl[t] = rnew;
        rr = rnew * rnew;
    }
    __syncthreads();
    if (B.mg_corner) {
        // corner sums of r for the coarse correction (thread i < 4 of an element)
        const int le = t / n, i = t - le * n, K = K0 + le;
        if (i < 4 && le < epb && K < P.ne) {
            double c = 0.0;
            for (int j = 0; j < n; ++j) {
                const double xa = P.gll[j % P.nb], yb = P.gll[j / P.nb];
                c += ((i & 1) ? xa : 1.0 - xa) * ((i & 2) ? yb : 1.0 - yb) * rl[le * n + j];
            }
            B.mg_corner[4L * (P.e_off + K) + i] = c;
        }
    }
    double rz = 0;
    const int pr = t / n, i = t - pr * n;
    const int la = 2 * pr, lb = la + 1, Ka = K0 + la, Kb = K0 + lb;
    if (la < epb && Ka < P.ne) {
        const bool vb = lb < epb && Kb < P.ne;
        const double* ra = rl + la * n;
        const double* rb = vb ? rl + lb * n : ra;
        const int sa = P.sid[Ka], sb = P.sid[vb ? Kb : Ka];
        double za = 0, zb = 0;
        typed_dot2(P.dinv + (long)sa * n * n + i, P.dinv + (long)sb * n * n + i, sa == sb, ra, rb, n, za, zb);
        P.z[(long)Ka * n + i] = za;
        rz = ra[i] * za;
        if (vb) {
            P.z[(long)Kb * n + i] = zb;
            rz += rb[i] * zb;
        }
    }
    rz = b_block_sum(rz, red);
    rr = b_block_sum(rr, red);
    if (t == 0) {
        B.part[B.nblocks + blockIdx.x] = rz;
        B.part[2 * B.nblocks + blockIdx.x] = rr;
    }
}

// fixed-order sum of a problem's group partials (one workgroup per problem)
__device__ __forceinline__ double group_sum(const BatchLaunch& B, const BProb& P, int which, double* red) {
    if (!B.grouped) return prob_sum(B, P, which, red);
    double v = 0.0;
    for (int k = threadIdx.x; k < P.ng; k += BT) v += B.gpart[which * B.ngroups + P.g0 + k];
    return b_block_sum(v, red);
}

__global__ __launch_bounds__(BT) void b_cg_red1(BatchLaunch B) {
    __shared__ double red[BT];
    const int prob = blockIdx.x;
    if (cg_skip(B, prob)) {
        if (B.active[prob] && threadIdx.x == 0) B.P[prob].scal[12] = -1.0;
        return;
    }
    const BProb& P = B.P[prob];
    const double pq = group_sum(B, P, 0, red);
    if (threadIdx.x == 0) {
        double* s = P.scal;
        if (!(pq > 0.0)) {
            s[6] = pq <= 0.0 ? 1.0 : 2.0;  // 2: not a number (a non-finite right-hand side)
            s[4] = 1.0;
        } else {
            s[8] = s[0] / pq;
        }
    }
}

template <int NB>
__device__ __forceinline__ void k2_group(const BatchLaunch& B, const BProb& P, int g, int cnt, double* xs) {
    constexpr int N = NB * NB, S = N | 1;
    const int lane = threadIdx.x & 63;
    const int myK = B.g_elem[g * 64 + lane];
    const int tot = cnt * N;
    const double alpha = P.scal[8];
    double rr = 0.0, rz = 0.0;
    const auto rg = as_global(P.r);
    const auto qg = as_global((const double*)P.q);
#pragma unroll
    for (int it = 0; it < N; ++it) {
        const int u = lane + 64 * it;
        const int e = u / N < 64 ? u / N : 63;
        const int K = __shfl(myK, e);
        if (u < tot) {
            const unsigned o = (unsigned)(K * N + (u - (u / N) * N));
            const double r = ld_at(rg, o) - alpha * ld_at(qg, o);
            st_at(rg, o, r);
            rr += r * r;
            xs[(u / N) * S + (u - (u / N) * N)] = r;
        }
    }
    lds_wave_sync();
    double z[N];
#pragma unroll
    for (int i = 0; i < N; ++i) z[i] = 0.0;
    block_mv<N>(P.dinv + (long)B.g_ty[g * 5] * N * N, xs + lane * S, z);
    if (lane < cnt)
#pragma unroll
        for (int i = 0; i < N; ++i) rz += xs[lane * S + i] * z[i];
    if (B.mg_corner && lane < cnt) {
        // corner sums of r for the coarse correction: sum over the nodes of
        // hat_corner(node) r(node), corner = cx + 2 cy
        double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const double yb = P.gll[b];
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                const double xa = P.gll[a], r = xs[lane * S + a + NB * b];
                c[0] += (1.0 - xa) * (1.0 - yb) * r;
                c[1] += xa * (1.0 - yb) * r;
                c[2] += (1.0 - xa) * yb * r;
                c[3] += xa * yb * r;
            }
        }
        const auto co = as_global(B.mg_corner) + (unsigned)(4 * (P.e_off + myK));
#pragma unroll
        for (int k = 0; k < 4; ++k) co[k] = c[k];
    }
    lds_wave_sync();
    if (lane < cnt)
#pragma unroll
        for (int i = 0; i < N; ++i) xs[lane * S + i] = z[i];
    lds_wave_sync();
#pragma unroll
    for (int it = 0; it < N; ++it) {
        const int u = lane + 64 * it;
        const int e = u / N < 64 ? u / N : 63;
        const int K = __shfl(myK, e);
        if (u < tot) st_at(as_global(P.z), (unsigned)(K * N + (u - (u / N) * N)), xs[(u / N) * S + (u - (u / N) * N)]);
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (lane == 0) {
        B.gpart[B.ngroups + g] = rz;
        B.gpart[2 * B.ngroups + g] = rr;
    }
}

// The update with z = D^-1 r on the FP64 matrix cores (vectors still moved
// flat and coalesced)
template <int NB>
__device__ __forceinline__ void k2_group_mfma(const BatchLaunch& B, const BProb& P, int g, int cnt, double* xs) {
    constexpr int N = NB * NB, S = N | 1;
    const int lane = threadIdx.x & 63;
    const int myK = B.g_elem[g * 64 + lane];
    const int tot = cnt * N;
    const double alpha = P.scal[8];
    double rr = 0.0, rz = 0.0;
    const auto rg = as_global(P.r);
    const auto qg = as_global((const double*)P.q);
#pragma unroll
    for (int it = 0; it < N; ++it) {
        const int u = lane + 64 * it;
        const int e = u / N < 64 ? u / N : 63;
        const int K = __shfl(myK, e);
        if (u < tot) {
            const unsigned o = (unsigned)(K * N + (u - (u / N) * N));
            const double r = ld_at(rg, o) - alpha * ld_at(qg, o);
            st_at(rg, o, r);
            rr += r * r;
            xs[(u / N) * S + (u - (u / N) * N)] = r;
        }
    }
    lds_wave_sync();
    if (B.mg_corner && lane < cnt) {
        // corner sums of r for the coarse correction: sum over the nodes of
        // hat_corner(node) r(node), corner = cx + 2 cy
        double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const double yb = P.gll[b];
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                const double xa = P.gll[a], r = xs[lane * S + a + NB * b];
                c[0] += (1.0 - xa) * (1.0 - yb) * r;
                c[1] += xa * (1.0 - yb) * r;
                c[2] += (1.0 - xa) * yb * r;
                c[3] += xa * yb * r;
            }
        }
        const auto co = as_global(B.mg_corner) + (unsigned)(4 * (P.e_off + myK));
#pragma unroll
        for (int k = 0; k < 4; ++k) co[k] = c[k];
    }
    // z = D^-1 r on the FP64 matrix cores: tiles as in k1_group_mfma, A the
    // group's block-Jacobi inverse (column-major), B the staged r
    {
        constexpr int MB = (N + 15) / 16, KS = (N + 3) / 4;
        const int i16 = lane & 15, kq = lane >> 4;
        const auto A = as_global(P.dinv + (long)B.g_ty[g * 5] * N * N);
        v4d acc[MB][4];
#pragma unroll
        for (int rb = 0; rb < MB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + kq;
            double a[MB], bf[4];
#pragma unroll
            for (int rb = 0; rb < MB; ++rb) {
                const int r = 16 * rb + i16;
                const bool in = k < N && r < N;
                a[rb] = ld_at(A, in ? (unsigned)(k * N + r) : 0u);
                if (!in) a[rb] = 0.0;
            }
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) bf[cb] = k < N ? xs[(16 * cb + i16) * S + k] : 0.0;
#pragma unroll
            for (int rb = 0; rb < MB; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], bf[cb], acc[rb][cb], 0, 0, 0);
        }
        lds_wave_sync();
        // each tile entry (row, e) belongs to one lane: r.z from the staged r,
        // then z in its place
#pragma unroll
        for (int rb = 0; rb < MB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * rb + 4 * r + kq, e = 16 * cb + i16;
                    if (row < N && e < cnt) {
                        double* cell = xs + e * S + row;
                        rz += *cell * acc[rb][cb][r];
                        *cell = acc[rb][cb][r];
                    }
                }
    }
    lds_wave_sync();
#pragma unroll
    for (int it = 0; it < N; ++it) {
        const int u = lane + 64 * it;
        const int e = u / N < 64 ? u / N : 63;
        const int K = __shfl(myK, e);
        if (u < tot) st_at(as_global(P.z), (unsigned)(K * N + (u - (u / N) * N)), xs[(u / N) * S + (u - (u / N) * N)]);
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (lane == 0) {
        B.gpart[B.ngroups + g] = rz;
        B.gpart[2 * B.ngroups + g] = rr;
    }
}

// r -= alpha q, z = D^-1 r (block-Jacobi) and the group's partial sums of r.z
// and r.r (x += alpha p waits for the direction update)
template <int NB>
__global__ __launch_bounds__(256, NB == 5 ? 3 : 2) void b_cg_k2(BatchLaunch B) {
    constexpr int SL = 64 * (NB * NB | 1);
    __shared__ double lds[4 * SL];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = B.g_nb0[NB] + xcd_block() * 4 + w;
    if (g >= B.g_nb0[NB + 1]) return;
    const int prob = B.g_prob[g];
    if (cg_skip(B, prob)) return;
    const BProb& P = B.P[prob];
    if constexpr (NB >= 3)
        k2_group_mfma<NB>(B, P, g, B.g_count[g], lds + w * SL);
    else
        k2_group<NB>(B, P, g, B.g_count[g], lds + w * SL);
}

// grouped launches, one per order present
static void b_cg_k1_all(const BatchLaunch& B, hipStream_t s) {
    auto go = [&](auto kfn, int nb) {
        const int ng = B.g_nb0[nb + 1] - B.g_nb0[nb];
        if (ng > 0 && (B.order_mask >> nb & 1)) hipLaunchKernelGGL(kfn, dim3((ng + 3) / 4), dim3(256), 0, s, B);
    };
    go(b_cg_k1<2>, 2);
    go(b_cg_k1<3>, 3);
    go(b_cg_k1<4>, 4);
    go(b_cg_k1<5>, 5);
}


// coarse iterate of a problem on the vertex grid after b_mg_apply
__device__ __forceinline__ const double* mg_x0(const MGLaunch& M, int prob) {
    const MGLevelDev& L = M.lev[0];
    return (M.lc[prob] == 0 ? L.x : L.t) + L.off[prob];
}

// r.z = r.(D^-1 r) + r.(P0 x0), and r.(P0 x0) = (P0^T r).x0 with P0^T r the
// level-0 right-hand side of the coarse correction
__global__ __launch_bounds__(BT) void b_cg_red2(BatchLaunch B, MGLaunch M) {
    __shared__ double red[BT];
    const int prob = blockIdx.x;
    if (cg_skip(B, prob)) return;
    const BProb& P = B.P[prob];
    double rzn = group_sum(B, P, 1, red);
    if (B.mg && P.cgw) {
        // r.(P_c w) = (P_c^T r).w, from the node kernel's block partials
        double v = 0.0;
        for (int k = M.cg_blk0[prob] + threadIdx.x; k < M.cg_blk0[prob + 1]; k += BT) v += M.cg_part[k];
        rzn += b_block_sum(v, red);
    }
    if (B.mg) {
        const MGLevelDev& L = M.lev[0];
        const int nv = L.dims[2 * prob] * L.dims[2 * prob + 1];
        const double* b0 = L.b + L.off[prob];
        const double* x0 = mg_x0(M, prob);
        // four independent partial sums per thread: the loop is bound by the
        // latency of its loads (one sum: 23 us per launch)
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
        int k = threadIdx.x;
        for (; k + 3 * BT < nv; k += 4 * BT) {
            v0 += b0[k] * x0[k];
            v1 += b0[k + BT] * x0[k + BT];
            v2 += b0[k + 2 * BT] * x0[k + 2 * BT];
            v3 += b0[k + 3 * BT] * x0[k + 3 * BT];
        }
        for (; k < nv; k += BT) v0 += b0[k] * x0[k];
        rzn += b_block_sum((v0 + v1) + (v2 + v3), red);
    }
    const double rr = group_sum(B, P, 2, red);
    if (threadIdx.x == 0) {
        double* s = P.scal;
        s[9] = rzn / s[0];
        s[1] = s[0];
        s[0] = rzn;
        s[3] = rr;
        s[5] += 1.0;
        if (rr <= s[7]) {
            s[4] = 1.0;
            s[12] = s[5];
        }
    }
}

// p = z + beta p, with z = D^-1 r + P0 x0 under the two-level preconditioner
__global__ __launch_bounds__(BT) void b_cg_k3(BatchLaunch B, MGLaunch M) {
    const EB m = eb_map(B);
    if (cg_skip(B, m.prob) || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i;
    double z = P.z[t];
    if (B.mg) {
        const int nvx = M.lev[0].dims[2 * m.prob];
        const int ex = m.K % P.nx, ey = m.K / P.nx;
        const double xa = P.gll[m.i % P.nb], yb = P.gll[m.i / P.nb];
        const double* xv = mg_x0(M, m.prob) + ey * nvx + ex;
        z += (1.0 - xa) * (1.0 - yb) * xv[0] + xa * (1.0 - yb) * xv[1] + (1.0 - xa) * yb * xv[nvx] +
             xa * yb * xv[nvx + 1];
        if (P.cgw) z += P.cgw[cg_node(P, m.K, m.i)];
    }
    P.p[t] = z + P.scal[9] * P.p[t];
}

// x += alpha p, then p = z + beta p (z = D^-1 r + P0 x0 with the two-level
// preconditioner) over one type group, flat element-major (coalesced) like the
// update kernel; in the iteration that converged, x += alpha p only
template <int NB>
__global__ __launch_bounds__(256) void b_cg_k3g(BatchLaunch B, MGLaunch M) {
    constexpr int N = NB * NB;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = B.g_nb0[NB] + xcd_block() * 4 + w;
    if (g >= B.g_nb0[NB + 1]) return;
    const int prob = B.g_prob[g];
    if (!B.active[prob]) return;
    const BProb& P = B.P[prob];
    // converged in this iteration: only x += alpha p is left
    const bool last = P.scal[4] != 0.0;
    if (last && P.scal[12] != P.scal[5]) return;
    const int lane = threadIdx.x & 63;
    const int cnt = B.g_count[g], tot = cnt * N;
    const int myK = B.g_elem[g * 64 + lane];
    const double alpha = P.scal[8], beta = P.scal[9];
    const auto zg = as_global((const double*)P.z);
    const auto pg = as_global(P.p);
    const auto xg = as_global(P.x);
    if (last) {
#pragma unroll
        for (int it = 0; it < N; ++it) {
            const int u = lane + 64 * it;
            const int e = u / N < 64 ? u / N : 63;
            const int K = __shfl(myK, e);
            if (u < tot) {
                const unsigned o = (unsigned)(K * N + (u - (u / N) * N));
                st_at(xg, o, ld_at(xg, o) + alpha * ld_at(pg, o));
            }
        }
        return;
    }
    // per lane (element): the vertex of its lower-left corner on the level-0
    // grid and its lower-left node on the continuous grid; a node (a, b) of
    // the element is then base + b gx + a (NB is a constant, so no division
    // per node)
    int nvx = 0, myV = 0, myC = 0, gx = 0;
    const double* x0 = nullptr;
    double gl[NB];
    if (B.mg) {
        nvx = M.lev[0].dims[2 * prob];
        const int ey = myK / P.nx, ex = myK - ey * P.nx;
        myV = ey * nvx + ex;
        gx = P.nx * (NB - 1) + 1;
        myC = ey * (NB - 1) * gx + ex * (NB - 1);
        x0 = mg_x0(M, prob);
#pragma unroll
        for (int a = 0; a < NB; ++a) gl[a] = P.gll[a];
    }
#pragma unroll
    for (int it = 0; it < N; ++it) {
        const int u = lane + 64 * it;
        const int e = u / N < 64 ? u / N : 63;
        const int j = u - (u / N) * N;
        const int K = __shfl(myK, e);
        const int V = __shfl(myV, e);
        const int Cb = __shfl(myC, e);
        if (u < tot) {
            const unsigned o = (unsigned)(K * N + j);
            double z = ld_at(zg, o);
            if (B.mg) {
                const double xa = gl[j % NB], yb = gl[j / NB];
                const double* xv = x0 + V;
                z += (1.0 - xa) * (1.0 - yb) * xv[0] + xa * (1.0 - yb) * xv[1] + (1.0 - xa) * yb * xv[nvx] +
                     xa * yb * xv[nvx + 1];
                if (P.cgw) z += P.cgw[Cb + (j / NB) * gx + j % NB];
            }
            const double pv = ld_at(pg, o);
            st_at(xg, o, ld_at(xg, o) + alpha * pv);
            st_at(pg, o, z + beta * pv);
        }
    }
}

// a new PCG start: clear the done and breakdown flags left by the previous
// solve (the start kernels run for every active problem)
__global__ void b_cg_clear_kernel(BatchLaunch B) {
    const int prob = blockIdx.x * blockDim.x + threadIdx.x;
    if (prob >= B.nprob) return;
    double* s = B.P[prob].scal;
    s[4] = 0.0;
    s[6] = 0.0;
    s[12] = -1.0;
}

hipError_t b_cg_start(const BatchLaunch& B, double tol, hipStream_t s, const MGLaunch* M) {
    hipLaunchKernelGGL(b_cg_clear_kernel, dim3((B.nprob + 255) / 256), dim3(256), 0, s, B);
    if (B.grouped)
        b_group_rows_all<0>(B, s);
    else
        hipLaunchKernelGGL(b_cg_init1, dim3(B.nblocks), dim3(BT), 0, s, B);
    hipLaunchKernelGGL(b_cg_init2, dim3(B.nblocks), dim3(BT), 0, s, B);
    if (B.mg) {
        hipError_t e = b_cgl_apply(B, *M, s);
        if (e != hipSuccess) return e;
        e = b_mg_apply(B, *M, true, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(b_cg_red_init, dim3(B.nprob), dim3(BT), 0, s, B, tol);
    return hipGetLastError();
}

hipError_t b_precond(const BatchLaunch& B, const MGLaunch* M, hipStream_t s) {
    hipLaunchKernelGGL(b_cg_init2, dim3(B.nblocks), dim3(BT), 0, s, B);
    if (B.mg) {
        const hipError_t e = b_cgl_apply(B, *M, s);
        if (e != hipSuccess) return e;
        return b_mg_apply(B, *M, true, s);
    }
    return hipGetLastError();
}

hipError_t b_cg_spmv(const BatchLaunch& B, hipStream_t s) {
    if (B.grouped)
        b_cg_k1_all(B, s);
    else
        hipLaunchKernelGGL(b_cg_k1n, dim3(B.nblocks), dim3(BT), 0, s, B);
    return hipGetLastError();
}

// The grouped kernels of one phase, one launch per active order: on the
// caller's stream, or (F set, more than one order) forked over side streams.
template <typename Launch>
static hipError_t per_order(const BatchLaunch& B, hipStream_t s, const CgFork* F, Launch go) {
    int orders[4], no = 0;
    for (int nb = 2; nb <= 5; ++nb)
        if (B.g_nb0[nb + 1] > B.g_nb0[nb] && (B.order_mask >> nb & 1)) orders[no++] = nb;
    if (!F || no < 2) {
        for (int k = 0; k < no; ++k) go(orders[k], s);
        return hipSuccess;
    }
    hipError_t e = hipEventRecord(F->fork, s);
    for (int k = 1; k < no && e == hipSuccess; ++k) e = hipStreamWaitEvent(F->side[k - 1], F->fork, 0);
    if (e != hipSuccess) return e;
    go(orders[no - 1], s);   // the highest order on the caller's stream
    for (int k = 1; k < no && e == hipSuccess; ++k) {
        go(orders[k - 1], F->side[k - 1]);
        e = hipEventRecord(F->join[k - 1], F->side[k - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, F->join[k - 1], 0);
    }
    return e;
}

hipError_t b_cg_iterations(const BatchLaunch& B, int iters, hipStream_t s, const MGLaunch* M, const CgFork* F) {
    const dim3 blk(256);
    auto grid = [&](int nb) { return dim3((B.g_nb0[nb + 1] - B.g_nb0[nb] + 3) / 4); };
    for (int k = 0; k < iters; ++k) {
        hipError_t e = hipSuccess;
        if (B.grouped)
            e = per_order(B, s, F, [&](int nb, hipStream_t st) {
                switch (nb) {
                    case 2: hipLaunchKernelGGL(b_cg_k1<2>, grid(2), blk, 0, st, B); break;
                    case 3: hipLaunchKernelGGL(b_cg_k1<3>, grid(3), blk, 0, st, B); break;
                    case 4: hipLaunchKernelGGL(b_cg_k1<4>, grid(4), blk, 0, st, B); break;
                    default: hipLaunchKernelGGL(b_cg_k1<5>, grid(5), blk, 0, st, B); break;
                }
            });
        else
            hipLaunchKernelGGL(b_cg_k1n, dim3(B.nblocks), dim3(BT), 0, s, B);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(b_cg_red1, dim3(B.nprob), dim3(BT), 0, s, B);
        if (B.grouped)
            e = per_order(B, s, F, [&](int nb, hipStream_t st) {
                switch (nb) {
                    case 2: hipLaunchKernelGGL(b_cg_k2<2>, grid(2), blk, 0, st, B); break;
                    case 3: hipLaunchKernelGGL(b_cg_k2<3>, grid(3), blk, 0, st, B); break;
                    case 4: hipLaunchKernelGGL(b_cg_k2<4>, grid(4), blk, 0, st, B); break;
                    default: hipLaunchKernelGGL(b_cg_k2<5>, grid(5), blk, 0, st, B); break;
                }
            });
        else
            hipLaunchKernelGGL(b_cg_k2n, dim3(B.nblocks), dim3(BT), 0, s, B);
        if (e != hipSuccess) return e;
        if (B.mg) {
            hipError_t e = b_cgl_apply(B, *M, s);
            if (e != hipSuccess) return e;
            e = b_mg_apply(B, *M, false, s);
            if (e != hipSuccess) return e;
        }
        const MGLaunch Mv = B.mg ? *M : MGLaunch{};
        hipLaunchKernelGGL(b_cg_red2, dim3(B.nprob), dim3(BT), 0, s, B, Mv);
        if (B.grouped)
            e = per_order(B, s, F, [&](int nb, hipStream_t st) {
                switch (nb) {
                    case 2: hipLaunchKernelGGL(b_cg_k3g<2>, grid(2), blk, 0, st, B, Mv); break;
                    case 3: hipLaunchKernelGGL(b_cg_k3g<3>, grid(3), blk, 0, st, B, Mv); break;
                    case 4: hipLaunchKernelGGL(b_cg_k3g<4>, grid(4), blk, 0, st, B, Mv); break;
                    default: hipLaunchKernelGGL(b_cg_k3g<5>, grid(5), blk, 0, st, B, Mv); break;
                }
            });
        else
            hipLaunchKernelGGL(b_cg_k3, dim3(B.nblocks), dim3(BT), 0, s, B, Mv);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ---- learned warm start -------------------------------------------------------
// Flux scale of element K: mean of |varphi_D| over its nodes.
__device__ __forceinline__ double ws_scale(const BProb& P, int K) {
    double s = 0.0;
    for (int j = 0; j < P.n; ++j) s += fabs(P.vdiff[(long)K * P.n + j]);
    return fmax(s / P.n, 1e-300);
}

// Features of element K (pixel K of an ny x nx image): channels 0-3 from feat0,
// 4: log10 s_K minus its problem mean (scal[10]), 5 + i: varphi_D,i / s_K - 1.
__global__ __launch_bounds__(BT) void b_ws_features_kernel(BatchLaunch B, int first, int count, float* X, int nf) {
    const EB m = eb_map(B);
    if (m.K < 0 || m.prob < first || m.prob >= first + count) return;
    const BProb& P = B.P[m.prob];
    const double sK = ws_scale(P, m.K);
    float* px = X + ((long)(m.prob - first) * P.ne + m.K) * nf;
    px[5 + m.i] = (float)(P.vdiff[(long)m.K * P.n + m.i] / sK - 1.0);
    if (m.i == 0) {
        for (int c = 0; c < 4; ++c) px[c] = P.feat0[(long)m.K * 4 + c];
        px[4] = (float)(log10(sK) - P.scal[10]);
    }
}

// problem mean of log10 s_K into scal[10] (one workgroup per problem)
__global__ __launch_bounds__(BT) void b_ws_logmean_kernel(BatchLaunch B, int first, int count) {
    __shared__ double red[BT];
    const int prob = first + blockIdx.x;
    const BProb& P = B.P[prob];
    double v = 0.0;
    for (int K = threadIdx.x; K < P.ne; K += BT) v += log10(ws_scale(P, K));
    v = b_block_sum(v, red);
    if (threadIdx.x == 0) P.scal[10] = v / P.ne;
}

__global__ __launch_bounds__(BT) void b_ws_targets_kernel(BatchLaunch B, int first, int count, float* T, int nt) {
    const EB m = eb_map(B);
    if (m.K < 0 || m.prob < first || m.prob >= first + count) return;
    const BProb& P = B.P[m.prob];
    const double sK = ws_scale(P, m.K);
    const long t = (long)m.K * P.n + m.i;
    float* pt = T + ((long)(m.prob - first) * P.ne + m.K) * nt;
    pt[m.i] = (float)((P.varphi[t] - P.vdiff[t]) / sK);
    pt[P.n + m.i] = (float)((P.b[t] - P.bfix[t]) / (P.hxhy * sK));
}

// Learned start: varphi = varphi_D + s_K y_i (the predicted flux correction);
// a non-finite prediction keeps varphi_D for the element and sets scal[11] = 1.
__global__ __launch_bounds__(BT) void b_ws_apply_kernel(BatchLaunch B, const float* Y, int nt) {
    const EB m = eb_map(B);
    if (m.K < 0 || !B.active[m.prob]) return;
    const BProb& P = B.P[m.prob];
    const double sK = ws_scale(P, m.K);
    const long t = (long)m.K * P.n + m.i;
    const double y = Y[((long)m.prob * P.ne + m.K) * nt + m.i];
    if (!isfinite(y)) {
        P.scal[11] = 1.0;
        P.varphi[t] = P.vdiff[t];
        return;
    }
    P.varphi[t] = P.vdiff[t] + sK * y;
}

// a problem with any non-finite prediction starts from varphi_D everywhere
__global__ __launch_bounds__(BT) void b_ws_fallback_kernel(BatchLaunch B) {
    const EB m = eb_map(B);
    if (m.K < 0 || !B.active[m.prob]) return;
    const BProb& P = B.P[m.prob];
    if (P.scal[11] == 0.0) return;
    const long t = (long)m.K * P.n + m.i;
    P.varphi[t] = P.vdiff[t];
}

// varphi_D = x (after the diffusion solve)
__global__ __launch_bounds__(BT) void b_ws_store_diffusion_kernel(BatchLaunch B) {
    const EB m = eb_map(B);
    if (m.K < 0 || !B.active[m.prob]) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i;
    P.vdiff[t] = P.x[t];
}

hipError_t b_ws_features(const BatchLaunch& B, int first, int count, float* X, int nf, hipStream_t s) {
    hipLaunchKernelGGL(b_ws_logmean_kernel, dim3(count), dim3(BT), 0, s, B, first, count);
    hipLaunchKernelGGL(b_ws_features_kernel, dim3(B.nblocks), dim3(BT), 0, s, B, first, count, X, nf);
    return hipGetLastError();
}

hipError_t b_ws_targets(const BatchLaunch& B, int first, int count, float* T, int nt, hipStream_t s) {
    hipLaunchKernelGGL(b_ws_targets_kernel, dim3(B.nblocks), dim3(BT), 0, s, B, first, count, T, nt);
    return hipGetLastError();
}

hipError_t b_ws_apply(const BatchLaunch& B, const float* Y, int nt, hipStream_t s) {
    hipLaunchKernelGGL(b_ws_apply_kernel, dim3(B.nblocks), dim3(BT), 0, s, B, Y, nt);
    hipLaunchKernelGGL(b_ws_fallback_kernel, dim3(B.nblocks), dim3(BT), 0, s, B);
    return hipGetLastError();
}

hipError_t b_ws_store_diffusion(const BatchLaunch& B, hipStream_t s) {
    hipLaunchKernelGGL(b_ws_store_diffusion_kernel, dim3(B.nblocks), dim3(BT), 0, s, B);
    return hipGetLastError();
}

// ---- two-level preconditioner: vertex multigrid on the Q1 coarse space --------
__device__ __forceinline__ int mg_prob(const int* off, int nprob, int v) {
    int lo = 0, hi = nprob - 1;  // last p with off[p] <= v
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int mg_ccount(int nf) { return nf <= 3 ? nf : nf / 2 + 1; }

// parents of fine vertex i (grid of nf vertices): c0 (w0), c1 (w1; -1 if none)
__device__ __forceinline__ void mg_parents(int i, int nf, int& c0, double& w0, int& c1, double& w1) {
    c1 = -1;
    w1 = 0.0;
    if (nf <= 3) {
        c0 = i;
        w0 = 1.0;
    } else if (i == nf - 1) {
        c0 = mg_ccount(nf) - 1;
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

__device__ __forceinline__ double mg_weight(int i, int nf, int c) {
    int c0, c1;
    double w0, w1;
    mg_parents(i, nf, c0, w0, c1, w1);
    return c0 == c ? w0 : (c1 == c ? w1 : 0.0);
}

// (A x)[v] on a level: 9-point stencil within the problem's vertex grid
__device__ __forceinline__ double mg_apply(const MGLevelDev& L, int o, int nvx, int nvy, int ix, int iy,
                                           const double* x) {
    double s = 0.0;
    const int v = o + iy * nvx + ix;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int jx = ix + k % 3 - 1, jy = iy + k / 3 - 1;
        if (jx < 0 || jy < 0 || jx >= nvx || jy >= nvy) continue;
        s += L.A[(long)k * L.nv + v] * x[o + jy * nvx + jx];
    }
    return s;
}

// level 0 right-hand side, in two steps: the corner sums of every element,
// c[K][corner] = sum over its nodes of hat_corner(node) r(node) (one thread per
// node, reduced over the element's threads in LDS), then per vertex the sum of
// the (<= 4) corner sums at it.
__global__ __launch_bounds__(BT) void mg_corner_kernel(BatchLaunch B, double* corner) {
    __shared__ double w[4][BT];
    const EB m = eb_map(B);
    const bool on = m.K >= 0 && !cg_skip(B, m.prob);
    if (on) {
        const BProb& P = B.P[m.prob];
        const int a = m.i % P.nb, b = m.i / P.nb;
        const double xa = P.gll[a], yb = P.gll[b];
        const double r = P.r[(long)m.K * P.n + m.i];
        w[0][threadIdx.x] = (1.0 - xa) * (1.0 - yb) * r;
        w[1][threadIdx.x] = xa * (1.0 - yb) * r;
        w[2][threadIdx.x] = (1.0 - xa) * yb * r;
        w[3][threadIdx.x] = xa * yb * r;
    }
    __syncthreads();
    if (on && m.i < 4) {
        const BProb& P = B.P[m.prob];
        double s = 0.0;
        for (int j = 0; j < P.n; ++j) s += w[m.i][m.e0 + j];
        corner[4L * (P.e_off + m.K) + m.i] = s;
    }
}

// smooth: also the first damped Jacobi step of level 0 from zero, x = omega
// b / d (pointwise, so it needs no launch of its own)
__global__ __launch_bounds__(BT) void mg_restrict0_kernel(BatchLaunch B, MGLaunch M, const double* corner,
                                                          int smooth) {
    const MGLevelDev& L = M.lev[0];
    const int v = blockIdx.x * BT + threadIdx.x;
    if (v >= L.nv) return;
    const int prob = mg_prob(L.off, B.nprob, v);
    if (cg_skip(B, prob)) return;
    const BProb& P = B.P[prob];
    const int o = L.off[prob], nvx = L.dims[2 * prob], loc = v - o;
    const int ix = loc % nvx, iy = loc / nvx;
    const int nx = nvx - 1, ny = L.dims[2 * prob + 1] - 1;
    const double* c = corner + 4L * P.e_off;
    double s = 0.0;
    for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
            const int ex = ix - cx, ey = iy - cy;
            if (ex < 0 || ey < 0 || ex >= nx || ey >= ny) continue;
            s += c[4L * (ey * nx + ex) + cx + 2 * cy];
        }
    L.b[v] = s;
    if (smooth && M.lc[prob] > 0) L.x[v] = M.omega * s / L.A[4L * L.nv + v];
}

// damped Jacobi: xout = omega b / d (mode 1, the first step from zero) or
// xin + omega (b - A xin) / d (mode 0); mode 2: the residual xout = b - A xin
__global__ __launch_bounds__(BT) void mg_smooth_kernel(BatchLaunch B, MGLaunch M, int l, int mode, const double* xin,
                                                       double* xout) {
    const MGLevelDev& L = M.lev[l];
    const int v = blockIdx.x * BT + threadIdx.x;
    if (v >= L.nv) return;
    const int prob = mg_prob(L.off, B.nprob, v);
    if (cg_skip(B, prob) || M.lc[prob] <= l) return;
    const int o = L.off[prob], nvx = L.dims[2 * prob], nvy = L.dims[2 * prob + 1], loc = v - o;
    if (mode == 1) {
        xout[v] = M.omega * L.b[v] / L.A[4L * L.nv + v];
        return;
    }
    const double ax = mg_apply(L, o, nvx, nvy, loc % nvx, loc / nvx, xin);
    if (mode == 2)
        xout[v] = L.b[v] - ax;
    else
        xout[v] = xin[v] + M.omega * (L.b[v] - ax) / L.A[4L * L.nv + v];
}

// b_{l+1}[c] = sum over fine f of w(f, c) res[f], res the fine residual
__global__ __launch_bounds__(BT) void mg_restrict_kernel(BatchLaunch B, MGLaunch M, int l, const double* res) {
    const MGLevelDev& F = M.lev[l];
    const MGLevelDev& C = M.lev[l + 1];
    const int c = blockIdx.x * BT + threadIdx.x;
    if (c >= C.nv) return;
    const int prob = mg_prob(C.off, B.nprob, c);
    if (cg_skip(B, prob) || M.lc[prob] <= l) return;
    const int fo = F.off[prob], fnx = F.dims[2 * prob], fny = F.dims[2 * prob + 1];
    const int cnx = C.dims[2 * prob], loc = c - C.off[prob];
    const int cx = loc % cnx, cy = loc / cnx;
    // fine vertices with parent c lie within two of its image 2c (or, for the
    // last coarse vertex of an odd grid, at the fine end)
    const int bx = fnx <= 3 ? cx : (cx == cnx - 1 ? fnx - 1 : 2 * cx);
    const int by = fny <= 3 ? cy : (cy == C.dims[2 * prob + 1] - 1 ? fny - 1 : 2 * cy);
    double s = 0.0;
    for (int fy = by - 2; fy <= by + 2; ++fy) {
        if (fy < 0 || fy >= fny) continue;
        const double wy = mg_weight(fy, fny, cy);
        if (wy == 0.0) continue;
        for (int fx = bx - 2; fx <= bx + 2; ++fx) {
            if (fx < 0 || fx >= fnx) continue;
            const double wx = mg_weight(fx, fnx, cx);
            if (wx == 0.0) continue;
            const int f = fo + fy * fnx + fx;
            s += wx * wy * res[f];
        }
    }
    C.b[c] = s;
}

// dense solve at each problem's coarsest level (one workgroup per problem)
__global__ __launch_bounds__(64) void mg_coarse_kernel(BatchLaunch B, MGLaunch M) {
    const int prob = blockIdx.x;
    if (cg_skip(B, prob)) return;
    const int l = M.lc[prob];
    if (l >= M.ls) return;  // solved inside the workgroup V-cycle
    const MGLevelDev& L = M.lev[l];
    const int o = L.off[prob], nc = L.dims[2 * prob] * L.dims[2 * prob + 1];
    const double* Ci = M.cinv + M.coff[prob];
    const int i = threadIdx.x;
    if (i < nc) {
        double s = 0.0;
        for (int j = 0; j < nc; ++j) s += Ci[i * nc + j] * L.b[o + j];
        L.x[o + i] = s;
    }
}

// Levels ls..lc of one problem's V-cycle in one workgroup, with the level
// vectors in LDS (the stencils stay in global memory and are cached): the same
// steps as the per-level launches, separated by barriers instead of launches.
// Input b_ls (global), output the level-ls iterate in t_ls, or in x_ls when ls
// is the problem's coarsest level.
__global__ __launch_bounds__(1024) void mg_vcycle_lds_kernel(BatchLaunch B, MGLaunch M) {
    extern __shared__ __align__(16) double vec[];
    __shared__ int lo[MG_MAXLEV], lnx[MG_MAXLEV], lny[MG_MAXLEV];
    const int prob = blockIdx.x;
    if (cg_skip(B, prob)) return;
    const int lc = M.lc[prob], ls = M.ls;
    if (lc < ls) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) {
        int o = 0;
        for (int l = ls; l <= lc; ++l) {
            lo[l] = o;
            lnx[l] = M.lev[l].dims[2 * prob];
            lny[l] = M.lev[l].dims[2 * prob + 1];
            o += 3 * lnx[l] * lny[l];
        }
    }
    __syncthreads();
    // level l: x at vec + lo[l], t after it, b after t
    auto X = [&](int l) { return vec + lo[l]; };
    auto Tv = [&](int l) { return vec + lo[l] + lnx[l] * lny[l]; };
    auto Bv = [&](int l) { return vec + lo[l] + 2 * lnx[l] * lny[l]; };
    auto apply = [&](int l, const double* x, int ix, int iy) {
        const MGLevelDev& L = M.lev[l];
        const int nvx = lnx[l], nvy = lny[l];
        const int v = L.off[prob] + iy * nvx + ix;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int jx = ix + k % 3 - 1, jy = iy + k / 3 - 1;
            if (jx < 0 || jy < 0 || jx >= nvx || jy >= nvy) continue;
            s += L.A[(long)k * L.nv + v] * x[jy * nvx + jx];
        }
        return s;
    };
    auto diag = [&](int l, int v) { return M.lev[l].A[4L * M.lev[l].nv + M.lev[l].off[prob] + v]; };
    const double om = M.omega;
    const int nu = M.nu;
    {
        const double* bg = M.lev[ls].b + M.lev[ls].off[prob];
        double* b = Bv(ls);
        for (int v = tid; v < lnx[ls] * lny[ls]; v += nt) b[v] = bg[v];
    }
    __syncthreads();
    for (int l = ls; l < lc; ++l) {
        const int nvx = lnx[l], nv = lnx[l] * lny[l];
        double *x = X(l), *t = Tv(l), *b = Bv(l);
        for (int v = tid; v < nv; v += nt) x[v] = om * b[v] / diag(l, v);
        __syncthreads();
        for (int k = 1; k < nu; ++k) {
            const double* src = (k & 1) ? x : t;
            double* dst = (k & 1) ? t : x;
            for (int v = tid; v < nv; v += nt) dst[v] = src[v] + om * (b[v] - apply(l, src, v % nvx, v / nvx)) / diag(l, v);
            __syncthreads();
        }
        // residual of the pre-smoothed iterate into the other vector (free
        // until the post-smoothing)
        double* it = (nu & 1) ? x : t;
        double* res = (nu & 1) ? t : x;
        for (int v = tid; v < nv; v += nt) res[v] = b[v] - apply(l, it, v % nvx, v / nvx);
        __syncthreads();
        const int fnx = nvx, fny = lny[l], cnx = lnx[l + 1], cny = lny[l + 1];
        double* bc = Bv(l + 1);
        for (int c = tid; c < cnx * cny; c += nt) {
            const int cx = c % cnx, cy = c / cnx;
            const int bx = fnx <= 3 ? cx : (cx == cnx - 1 ? fnx - 1 : 2 * cx);
            const int by = fny <= 3 ? cy : (cy == cny - 1 ? fny - 1 : 2 * cy);
            double s = 0.0;
            for (int fy = by - 2; fy <= by + 2; ++fy) {
                if (fy < 0 || fy >= fny) continue;
                const double wy = mg_weight(fy, fny, cy);
                if (wy == 0.0) continue;
                for (int fx = bx - 2; fx <= bx + 2; ++fx) {
                    if (fx < 0 || fx >= fnx) continue;
                    const double wx = mg_weight(fx, fnx, cx);
                    if (wx == 0.0) continue;
                    s += wx * wy * res[fy * fnx + fx];
                }
            }
            bc[c] = s;
        }
        __syncthreads();
    }
    {
        const int nc = lnx[lc] * lny[lc];
        const double* Ci = M.cinv + M.coff[prob];
        const double* b = Bv(lc);
        if (tid < nc) {
            double s = 0.0;
            for (int j = 0; j < nc; ++j) s += Ci[tid * nc + j] * b[j];
            X(lc)[tid] = s;
        }
    }
    __syncthreads();
    for (int l = lc - 1; l >= ls; --l) {
        const int fnx = lnx[l], fny = lny[l], nv = fnx * fny, cnx = lnx[l + 1];
        double *x = X(l), *t = Tv(l), *b = Bv(l);
        double* it = (nu & 1) ? x : t;
        double* other = (nu & 1) ? t : x;
        const double* xc = l + 1 == lc ? X(l + 1) : Tv(l + 1);
        for (int f = tid; f < nv; f += nt) {
            int x0, x1, y0, y1;
            double wx0, wx1, wy0, wy1;
            mg_parents(f % fnx, fnx, x0, wx0, x1, wx1);
            mg_parents(f / fnx, fny, y0, wy0, y1, wy1);
            double s = wx0 * wy0 * xc[y0 * cnx + x0];
            if (x1 >= 0) s += wx1 * wy0 * xc[y0 * cnx + x1];
            if (y1 >= 0) s += wx0 * wy1 * xc[y1 * cnx + x0];
            if (x1 >= 0 && y1 >= 0) s += wx1 * wy1 * xc[y1 * cnx + x1];
            it[f] += s;
        }
        __syncthreads();
        for (int k = 0; k < nu; ++k) {
            const double* src = (k & 1) ? other : it;
            double* dst = (k & 1) ? it : other;
            for (int v = tid; v < nv; v += nt) dst[v] = src[v] + om * (b[v] - apply(l, src, v % fnx, v / fnx)) / diag(l, v);
            __syncthreads();
        }
    }
    {
        const MGLevelDev& L = M.lev[ls];
        const double* src = ls == lc ? X(ls) : Tv(ls);
        double* dst = (ls == lc ? L.x : L.t) + L.off[prob];
        for (int v = tid; v < lnx[ls] * lny[ls]; v += nt) dst[v] = src[v];
    }
}

// x_l[f] += sum over parents c of w(f, c) x_{l+1}[c]; the coarse iterate is in x
// where level l+1 is the problem's coarsest, else in t
__global__ __launch_bounds__(BT) void mg_prolong_kernel(BatchLaunch B, MGLaunch M, int l, double* xf) {
    const MGLevelDev& F = M.lev[l];
    const MGLevelDev& C = M.lev[l + 1];
    const int f = blockIdx.x * BT + threadIdx.x;
    if (f >= F.nv) return;
    const int prob = mg_prob(F.off, B.nprob, f);
    if (cg_skip(B, prob) || M.lc[prob] <= l) return;
    const int fnx = F.dims[2 * prob], fny = F.dims[2 * prob + 1], loc = f - F.off[prob];
    const int cnx = C.dims[2 * prob], co = C.off[prob];
    const double* xc = M.lc[prob] == l + 1 ? C.x : C.t;
    int x0, x1, y0, y1;
    double wx0, wx1, wy0, wy1;
    mg_parents(loc % fnx, fnx, x0, wx0, x1, wx1);
    mg_parents(loc / fnx, fny, y0, wy0, y1, wy1);
    double s = wx0 * wy0 * xc[co + y0 * cnx + x0];
    if (x1 >= 0) s += wx1 * wy0 * xc[co + y0 * cnx + x1];
    if (y1 >= 0) s += wx0 * wy1 * xc[co + y1 * cnx + x0];
    if (x1 >= 0 && y1 >= 0) s += wx1 * wy1 * xc[co + y1 * cnx + x1];
    xf[f] += s;
}

// z += P0 x_0 (bilinear interpolation at the nodes), partial sums of r.z
__global__ __launch_bounds__(BT) void mg_finish_kernel(BatchLaunch B, MGLaunch M, int init) {
    __shared__ double red[BT];
    const EB m = eb_map(B);
    double rz = 0.0;
    if (m.K >= 0 && !cg_skip(B, m.prob)) {
        const BProb& P = B.P[m.prob];
        const MGLevelDev& L = M.lev[0];
        const double* x0 = M.lc[m.prob] == 0 ? L.x : L.t;
        const int o = L.off[m.prob], nvx = L.dims[2 * m.prob];
        const int ex = m.K % P.nx, ey = m.K / P.nx;
        const int a = m.i % P.nb, b = m.i / P.nb;
        const double xa = P.gll[a], yb = P.gll[b];
        const double* xv = x0 + o + ey * nvx + ex;
        double c = (1.0 - xa) * (1.0 - yb) * xv[0] + xa * (1.0 - yb) * xv[1] + (1.0 - xa) * yb * xv[nvx] +
                   xa * yb * xv[nvx + 1];
        if (P.cgw) c += P.cgw[cg_node(P, m.K, m.i)];
        const long t = (long)m.K * P.n + m.i;
        const double z = P.z[t] + c;
        P.z[t] = z;
        if (init) P.p[t] = z;
        rz = P.r[t] * z;
    }
    rz = b_block_sum(rz, red);
    if (threadIdx.x == 0) B.part[(init ? 0 : 1) * B.nblocks + blockIdx.x] = rz;
}

// Continuous-space term of the two-level preconditioner (orders >= 2).  P_c
// injects a continuous Q_p function (values at the Gauss-Lobatto nodes shared
// across element faces) into the DG space; P_c^T r sums the residual over the
// (up to four) element copies of a node.  w = D_c^-1 P_c^T r, D_c the diagonal
// of P_c^T A P_c (host set-up), so the term adds P_c w to z.
template <int PO>
__device__ __forceinline__ double cgl_node(const BProb& P, int i, int nx, int ny, int gx) {
    // PO = p: the divisions by the order are by a constant
    const int gi = i % gx, gj = i / gx;
    const auto rg = as_global((const double*)P.r);
    double rc = 0.0;
#pragma unroll
    for (int cy = 0; cy < 2; ++cy) {
        const int ey = gj / PO - cy;
        if (ey < 0 || ey >= ny || (cy == 1 && gj % PO != 0)) continue;
        const int by = gj - ey * PO;
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
            const int ex = gi / PO - cx;
            if (ex < 0 || ex >= nx || (cx == 1 && gi % PO != 0)) continue;
            const int ax = gi - ex * PO;
            rc += ld_at(rg, (unsigned)((ey * nx + ex) * (PO + 1) * (PO + 1) + ax + (PO + 1) * by));
        }
    }
    return rc;
}

// w = D_c^-1 P_c^T r per node, and per block of nodes the partial sum of
// (P_c^T r).w, summed per problem (in block order) by the r.z reduction
__global__ __launch_bounds__(BT) void cgl_kernel(BatchLaunch B, MGLaunch M) {
    __shared__ double red[BT];
    const int prob = M.cg_blk2p[blockIdx.x];
    if (cg_skip(B, prob)) return;  // block-uniform
    const BProb& P = B.P[prob];
    const int p = P.nb - 1, nx = P.nx, ny = P.ne / P.nx;
    const int gx = nx * p + 1, gy = ny * p + 1;
    const int i = (blockIdx.x - M.cg_blk0[prob]) * BT + threadIdx.x;
    double part = 0.0;
    if (i < gx * gy) {
        double rc;
        switch (p) {
            case 2: rc = cgl_node<2>(P, i, nx, ny, gx); break;
            case 3: rc = cgl_node<3>(P, i, nx, ny, gx); break;
            default: rc = cgl_node<4>(P, i, nx, ny, gx); break;
        }
        const double w = rc / P.cgdc[i];
        P.cgw[i] = w;
        part = rc * w;
    }
    part = b_block_sum(part, red);
    if (threadIdx.x == 0) M.cg_part[blockIdx.x] = part;
}

hipError_t b_cgl_apply(const BatchLaunch& B, const MGLaunch& M, hipStream_t s) {
    if (M.cg_nblocks > 0) hipLaunchKernelGGL(cgl_kernel, dim3(M.cg_nblocks), dim3(BT), 0, s, B, M);
    return hipGetLastError();
}

hipError_t b_mg_apply(const BatchLaunch& B, const MGLaunch& M, bool init, hipStream_t s) {
    auto grid = [](int n) { return dim3((unsigned)((n + BT - 1) / BT)); };
    // per-level launches above level ls, one workgroup per problem below
    const int top = M.ls < M.nlev - 1 ? M.ls : M.nlev - 1;
    if (init) hipLaunchKernelGGL(mg_corner_kernel, dim3(B.nblocks), dim3(BT), 0, s, B, M.corner);
    hipLaunchKernelGGL(mg_restrict0_kernel, grid(M.lev[0].nv), dim3(BT), 0, s, B, M, (const double*)M.corner,
                       top > 0 ? 1 : 0);
    // nu damped Jacobi steps before and after the coarse correction,
    // alternating between x and t; the pre-smoothed iterate ends in x (nu
    // odd) or t (nu even), the residual goes to the other one, and after the
    // post-smoothing the level's result is in t either way
    const int nu = M.nu;
    for (int l = 0; l < top; ++l) {
        const MGLevelDev& L = M.lev[l];
        // (level 0's first step ran with the restriction)
        if (l > 0) hipLaunchKernelGGL(mg_smooth_kernel, grid(L.nv), dim3(BT), 0, s, B, M, l, 1, (const double*)L.x, L.x);
        for (int k = 1; k < nu; ++k) {
            double* src = (k & 1) ? L.x : L.t;
            hipLaunchKernelGGL(mg_smooth_kernel, grid(L.nv), dim3(BT), 0, s, B, M, l, 0, (const double*)src,
                               (k & 1) ? L.t : L.x);
        }
        double* it = (nu & 1) ? L.x : L.t;
        double* other = (nu & 1) ? L.t : L.x;
        hipLaunchKernelGGL(mg_smooth_kernel, grid(L.nv), dim3(BT), 0, s, B, M, l, 2, (const double*)it, other);
        hipLaunchKernelGGL(mg_restrict_kernel, grid(M.lev[l + 1].nv), dim3(BT), 0, s, B, M, l, (const double*)other);
    }
    if (M.ls < M.nlev)
        hipLaunchKernelGGL(mg_vcycle_lds_kernel, dim3(B.nprob), dim3(1024), M.lds, s, B, M);
    if (M.coarse_any) hipLaunchKernelGGL(mg_coarse_kernel, dim3(B.nprob), dim3(64), 0, s, B, M);
    for (int l = top - 1; l >= 0; --l) {
        const MGLevelDev& L = M.lev[l];
        double* it = (nu & 1) ? L.x : L.t;
        hipLaunchKernelGGL(mg_prolong_kernel, grid(L.nv), dim3(BT), 0, s, B, M, l, it);
        for (int k = 0; k < nu; ++k) {
            const bool from_it = (k & 1) == 0;
            double* src = from_it ? it : (it == L.x ? L.t : L.x);
            double* dst = from_it ? (it == L.x ? L.t : L.x) : it;
            hipLaunchKernelGGL(mg_smooth_kernel, grid(L.nv), dim3(BT), 0, s, B, M, l, 0, (const double*)src, dst);
        }
    }
    if (init) hipLaunchKernelGGL(mg_finish_kernel, dim3(B.nblocks), dim3(BT), 0, s, B, M, 1);
    return hipGetLastError();
}

hipError_t mg_prepare(size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(mg_vcycle_lds_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// ---- Anderson mixing of the outer fixed point ------------------------------------
__global__ __launch_bounds__(BT) void b_aa_store_kernel(BatchLaunch B, int slot) {
    const EB m = eb_map(B);
    if (!B.active[m.prob] || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i, o = (long)slot * P.L + t;
    const double g = P.x[t];
    P.aG[o] = g;
    P.aF[o] = g - P.varphi[t];
}

__global__ __launch_bounds__(BT) void b_aa_gram_part(BatchLaunch B, double* part6) {
    __shared__ double red[6][BT];
    const EB m = eb_map(B);
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (B.active[m.prob] && m.K >= 0) {
        const BProb& P = B.P[m.prob];
        const long t = (long)m.K * P.n + m.i;
        const double f0 = P.aF[t], f1 = P.aF[P.L + t], f2 = P.aF[2 * P.L + t];
        v[0] = f0 * f0;
        v[1] = f0 * f1;
        v[2] = f0 * f2;
        v[3] = f1 * f1;
        v[4] = f1 * f2;
        v[5] = f2 * f2;
    }
    // the six sums in one pass: the products in LDS, then 32 lanes per sum
    // add BT / 32 values each (strided, so the reads do not conflict) and a
    // butterfly over the 32 (six butterflies over 64 lanes, one per sum,
    // took twice as long)
#pragma unroll
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    if (threadIdx.x < 6 * 32) {
        const int k = threadIdx.x >> 5, c = threadIdx.x & 31;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < BT / 32; ++i) s += red[k][32 * i + c];
        for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, 32);
        if (c == 0) part6[(long)k * B.nblocks + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(BT) void b_aa_gram_final(BatchLaunch B, const double* part6, double* out) {
    __shared__ double red[BT];
    const int prob = blockIdx.x;
    const BProb& P = B.P[prob];
    for (int k = 0; k < 6; ++k) {
        double v = 0.0;
        for (int j = threadIdx.x; j < P.nblk; j += BT) v += part6[(long)k * B.nblocks + P.blk0 + j];
        v = b_block_sum(v, red);
        if (threadIdx.x == 0) out[6 * prob + k] = v;
    }
}

__global__ __launch_bounds__(BT) void b_aa_mix_kernel(BatchLaunch B, const double* coef) {
    const EB m = eb_map(B);
    if (!B.active[m.prob] || m.K < 0) return;
    const BProb& P = B.P[m.prob];
    const long t = (long)m.K * P.n + m.i;
    const double* c = coef + 3 * m.prob;
    double v = c[0] * P.aG[t];
    if (c[1] != 0.0) v += c[1] * P.aG[P.L + t];
    if (c[2] != 0.0) v += c[2] * P.aG[2 * P.L + t];
    P.varphi_prev[t] = P.varphi[t];
    P.varphi[t] = v;
}

hipError_t b_aa_store(const BatchLaunch& B, int slot, hipStream_t s) {
    hipLaunchKernelGGL(b_aa_store_kernel, dim3(B.nblocks), dim3(BT), 0, s, B, slot);
    return hipGetLastError();
}

hipError_t b_aa_gram(const BatchLaunch& B, double* part6, double* out, hipStream_t s) {
    hipLaunchKernelGGL(b_aa_gram_part, dim3(B.nblocks), dim3(BT), 0, s, B, part6);
    hipLaunchKernelGGL(b_aa_gram_final, dim3(B.nprob), dim3(BT), 0, s, B, (const double*)part6, out);
    return hipGetLastError();
}

hipError_t b_aa_mix(const BatchLaunch& B, const double* coef, hipStream_t s) {
    hipLaunchKernelGGL(b_aa_mix_kernel, dim3(B.nblocks), dim3(BT), 0, s, B, coef);
    return hipGetLastError();
}

// ---- outer residual per problem: out[2 prob] = max|x - varphi|, out[2 prob + 1] = max|x|
__global__ __launch_bounds__(BT) void b_resid_part(BatchLaunch B) {
    __shared__ double r[2][BT];
    const EB m = eb_map(B);
    double a = 0, b = 0;
    if (B.active[m.prob] && m.K >= 0) {
        const BProb& P = B.P[m.prob];
        const long t = (long)m.K * P.n + m.i;
        const double v = P.x[t];
        const double dv = fabs(v - P.varphi[t]);
        a = (dv != dv) ? dv : dv;
        b = fabs(v);
        if (v != v) b = v;
    }
    // the two maxima (NaN propagates; the order does not matter): 32 lanes
    // per maximum take BT / 32 values each, strided, then a butterfly over
    // the 32 (a tree over the workgroup took eight barriers)
    r[0][threadIdx.x] = a;
    r[1][threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int k = threadIdx.x >> 5, c = threadIdx.x & 31;
        double mx = r[k][c];
#pragma unroll
        for (int i = 1; i < BT / 32; ++i) {
            const double x = r[k][32 * i + c];
            mx = (x > mx || x != x) ? x : mx;
        }
        for (int off = 16; off > 0; off >>= 1) {
            const double x = __shfl_xor(mx, off, 32);
            mx = (x > mx || x != x) ? x : mx;
        }
        if (c == 0) B.part[(long)k * B.nblocks + blockIdx.x] = mx;
    }
}

// one workgroup per problem: max over the problem's block partials (a
// maximum does not depend on the order, NaN propagates)
__global__ __launch_bounds__(BT) void b_resid_final(BatchLaunch B, double* out) {
    __shared__ double r0[BT], r1[BT];
    const int prob = blockIdx.x;
    const BProb& P = B.P[prob];
    double a = 0, b = 0;
    for (int k = threadIdx.x; k < P.nblk; k += BT) {
        const double x0 = B.part[P.blk0 + k], x1 = B.part[B.nblocks + P.blk0 + k];
        a = (x0 > a || x0 != x0) ? x0 : a;
        b = (x1 > b || x1 != x1) ? x1 : b;
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    __syncthreads();
    for (int st = BT / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            const double x0 = r0[threadIdx.x + st], x1 = r1[threadIdx.x + st];
            r0[threadIdx.x] = (x0 > r0[threadIdx.x] || x0 != x0) ? x0 : r0[threadIdx.x];
            r1[threadIdx.x] = (x1 > r1[threadIdx.x] || x1 != x1) ? x1 : r1[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * prob] = r0[0];
        out[2 * prob + 1] = r1[0];
    }
}

hipError_t b_residual(const BatchLaunch& B, double* out, hipStream_t s) {
    hipLaunchKernelGGL(b_resid_part, dim3(B.nblocks), dim3(BT), 0, s, B);
    hipLaunchKernelGGL(b_resid_final, dim3(B.nprob), dim3(BT), 0, s, B, out);
    return hipGetLastError();
}

}  // namespace smm
