// Convolutional network for the learned SMM warm start: 3x3 convolutions
// (zero padding, stride 1) over NHWC activations stored in bfloat16, with
// FP32 accumulation on the bf16 matrix cores (v_mfma_f32_16x16x16_bf16).
//
// A convolution is an implicit GEMM: rows are pixels, columns output
// channels, and the reduction runs over (tap, input channel) with
// k = tap * CIN + c.  Channel counts are padded to 16, 32 or 64 so that a
// 16-wide reduction chunk never straddles a tap.
//
// MFMA 16x16x16 bf16 lane layout (wave of 64, lane = i + 16 g):
//   A[i][k]: lane (i, g) holds k = 4g .. 4g+3 of row i
//   B[k][j]: lane (j, g) holds k = 4g .. 4g+3 of column j
//   D[i][j]: lane (j, g) holds rows i = 4g .. 4g+3 of column j
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cnn_kernels.hpp"

namespace smmcnn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bool bf_positive(uint16_t h) { return h != 0 && !(h & 0x8000u); }

constexpr int CT = 256;  // threads per workgroup (4 waves)
constexpr int MB = 4;    // 16-pixel row blocks per wave

// out = conv(X, Wp) with the epilogue selected by MODE:
//   0: hidden layer   bf16(relu(acc + bias))          -> uint16 [npix][COUT]
//   1: output layer   acc + bias, first cout_real ch. -> float  [npix][cout_real]
//   2: input gradient bf16(acc) where mask > 0, else 0 -> uint16 [npix][COUT]
// Wp is [9*CIN/4][COUT][4] bf16: 4 consecutive k of one column are contiguous.
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(CT) void conv3x3_kernel(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Wp,
                                                     const float* __restrict__ bias, void* __restrict__ out,
                                                     const uint16_t* __restrict__ mask, long npix, int H, int W,
                                                     int cout_real) {
    constexpr int NB = COUT / 16, KC = CIN / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    const long base = ((long)blockIdx.x * (CT / 64) + wave) * (16 * MB);
    if (base >= npix) return;  // wave-uniform
    f32x4 acc[MB][NB];
    int py[MB], px[MB];
    long pn[MB];
    bool pv[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        const long p = base + mb * 16 + i;
        pv[mb] = p < npix;
        const long q = pv[mb] ? p : 0;
        px[mb] = (int)(q % W);
        const long r = q / W;
        py[mb] = (int)(r % H);
        pn[mb] = r / H;
    }
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const uint16_t* src[MB];
        bool ok[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int y = py[mb] + dy, x = px[mb] + dx;
            ok[mb] = pv[mb] && y >= 0 && y < H && x >= 0 && x < W;
            src[mb] = ok[mb] ? X + (((pn[mb] * H + y) * W + x) * CIN + 4 * g) : X;
        }
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            bf16x4 b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                b[nb] = *reinterpret_cast<const bf16x4*>(Wp + ((long)((tap * CIN + kc * 16) / 4 + g) * COUT + nb * 16 + i) * 4);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                bf16x4 a = bf16x4{0, 0, 0, 0};
                if (ok[mb]) a = *reinterpret_cast<const bf16x4*>(src[mb] + kc * 16);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[nb], acc[mb][nb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const long p = base + mb * 16 + 4 * g + e;
            if (p >= npix) continue;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int o = nb * 16 + i;
                const float v = acc[mb][nb][e];
                if constexpr (MODE == 0) {
                    const float z = v + bias[o];  // ReLU that keeps NaN (fmaxf would drop it)
                    reinterpret_cast<uint16_t*>(out)[p * COUT + o] = f2bf(z < 0.f ? 0.f : z);
                } else if constexpr (MODE == 1) {
                    if (o < cout_real) reinterpret_cast<float*>(out)[p * cout_real + o] = v + bias[o];
                } else {
                    reinterpret_cast<uint16_t*>(out)[p * COUT + o] = bf_positive(mask[p * COUT + o]) ? f2bf(v) : 0;
                }
            }
        }
    }
}

// Weight gradient partials of one block of pixels [p0, p0 + ppb):
//   part[blk][o][tap][c] = sum_p G[p][o] A[p shifted by tap][c],  part[blk][COUT*9*CIN + o] = sum_p G[p][o]
// as a GEMM with rows o, columns (tap, c) and the reduction over pixels.
template <int CIN, int COUT>
__global__ __launch_bounds__(CT) void conv3x3_wgrad_kernel(const uint16_t* __restrict__ A, const uint16_t* __restrict__ G,
                                                           float* __restrict__ part, long npix, int H, int W, int ppb) {
    constexpr int NCB = 9 * CIN / 16, OB = COUT / 16, CPW = (NCB + 3) / 4, CPT = CIN / 16;
    constexpr long stride = (long)COUT * 9 * CIN + COUT;
    __shared__ float red[CT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    const long p0 = (long)blockIdx.x * ppb;
    const long p1 = p0 + ppb < npix ? p0 + ppb : npix;
    f32x4 acc[CPW][OB];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) acc[c][ob] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (long pk = p0; pk < p1; pk += 16) {
        long pe[4];
        int ye[4], xe[4];
        long ne_[4];
        bool ve[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            pe[e] = pk + 4 * g + e;
            ve[e] = pe[e] < p1;
            const long q = ve[e] ? pe[e] : p0;
            xe[e] = (int)(q % W);
            const long r = q / W;
            ye[e] = (int)(r % H);
            ne_[e] = r / H;
        }
        bf16x4 ga[OB];
#pragma unroll
        for (int ob = 0; ob < OB; ++ob)
#pragma unroll
            for (int e = 0; e < 4; ++e) ga[ob][e] = ve[e] ? (short)G[pe[e] * COUT + ob * 16 + i] : (short)0;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int cb = wave + 4 * c;
            if (cb >= NCB) break;
            const int tap = cb / CPT, cbase = (cb % CPT) * 16;
            const int dy = tap / 3 - 1, dx = tap % 3 - 1;
            bf16x4 bb;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int y = ye[e] + dy, x = xe[e] + dx;
                const bool ok = ve[e] && y >= 0 && y < H && x >= 0 && x < W;
                bb[e] = ok ? (short)A[((ne_[e] * H + y) * W + x) * CIN + cbase + i] : (short)0;
            }
#pragma unroll
            for (int ob = 0; ob < OB; ++ob)
                acc[c][ob] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ga[ob], bb, acc[c][ob], 0, 0, 0);
        }
    }
    float* dst = part + (long)blockIdx.x * stride;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int cb = wave + 4 * c;
        if (cb >= NCB) break;
#pragma unroll
        for (int ob = 0; ob < OB; ++ob)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = ob * 16 + 4 * g + e;
                dst[(long)o * 9 * CIN + cb * 16 + i] = acc[c][ob][e];
            }
    }
    // bias: thread t sums channel t % COUT over every (CT / COUT)-th pixel
    {
        constexpr int PL = CT / COUT;
        const int o = threadIdx.x % COUT, pl = threadIdx.x / COUT;
        float s = 0.f;
        for (long p = p0 + pl; p < p1; p += PL) s += bf2f(G[p * COUT + o]);
        red[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < COUT) {
            float t = 0.f;
            for (int k = 0; k < PL; ++k) t += red[k * COUT + threadIdx.x];
            dst[(long)COUT * 9 * CIN + threadIdx.x] = t;
        }
    }
}

// grad[woff + idx] = sum over blocks of the partials (fixed order, double)
__global__ void wgrad_reduce_kernel(const float* __restrict__ part, int nblk, long stride, float* __restrict__ gw,
                                    float* __restrict__ gb, long nw) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= stride) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(long)b * stride + idx];
    if (idx < nw) gw[idx] = (float)s;
    else gb[idx - nw] = (float)s;
}

// Xb[b][pix][c] = bf16(X_all[idx[b]][pix][c]) for c < c_real, 0 for padding
__global__ void gather_input_kernel(const float* __restrict__ X, const int* __restrict__ idx, int n_all, int batch,
                                    long hw, int c_real, int c_pad, uint16_t* __restrict__ Xb, int* __restrict__ bad) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)batch * hw * c_pad;
    if (t >= total) return;
    const int c = (int)(t % c_pad);
    const long r = t / c_pad;
    const long pix = r % hw;
    const int b = (int)(r / hw);
    const long src = idx ? idx[b] : b;
    const bool ok = src >= 0 && src < n_all;
    if (!ok && bad) *bad = 1;
    Xb[t] = (c < c_real && ok) ? f2bf(X[(src * hw + pix) * c_real + c]) : (uint16_t)0;
}

// Weighted mean squared error and its gradient (rounded to bf16):
//   loss = sum_{b,pix,o} w_o (y - t)^2 * scale,  G = bf16(2 w_o (y - t) scale), scale = 1 / (batch hw c_real)
__global__ __launch_bounds__(CT) void loss_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                  const int* __restrict__ idx, int n_all, const float* __restrict__ wch,
                                                  int batch, long hw, int c_real, int c_pad, double scale,
                                                  uint16_t* __restrict__ G, double* __restrict__ part,
                                                  int* __restrict__ bad) {
    __shared__ double red[CT];
    const long t = (long)blockIdx.x * CT + threadIdx.x;
    const long total = (long)batch * hw * c_pad;
    double l = 0.0;
    if (t < total) {
        const int c = (int)(t % c_pad);
        const long r = t / c_pad;
        const long pix = r % hw;
        const int b = (int)(r / hw);
        uint16_t gv = 0;
        const long src = idx ? idx[b] : b;
        const bool ok = src >= 0 && src < n_all;
        if (!ok && bad) *bad = 1;
        if (c < c_real && ok) {
            const float d = Y[((long)b * hw + pix) * c_real + c] - T[(src * hw + pix) * c_real + c];
            const float w = wch[c];
            l = (double)w * d * d * scale;
            gv = f2bf((float)(2.0 * w * d * scale));
        }
        G[t] = gv;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = CT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(CT) void sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[CT];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += CT) s += part[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = CT / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam on the FP32 master parameters; c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, long n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
}

// bf16 copies of one layer's master weights W[o][tap][c]: the forward operand
// Wp[(tap*cin + c)/4][o][c%4] and the input-gradient operand (taps flipped,
// roles of o and c swapped) Wt[((8-tap)*cout + o)/4][c][o%4].
__global__ void pack_weights_kernel(const float* __restrict__ Wm, int cin, int cout, uint16_t* __restrict__ Wp,
                                    uint16_t* __restrict__ Wt) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long)cout * 9 * cin) return;
    const int c = (int)(k % cin);
    const int tap = (int)((k / cin) % 9);
    const int o = (int)(k / (9L * cin));
    const uint16_t w = f2bf(Wm[k]);
    Wp[(((long)(tap * cin + c) / 4) * cout + o) * 4 + (c & 3)] = w;
    Wt[(((long)((8 - tap) * cout + o) / 4) * cin + c) * 4 + (o & 3)] = w;
}

// ---- launchers ------------------------------------------------------------------

template <int CIN, int COUT, int MODE>
static hipError_t conv_t(const ConvLaunch& c, hipStream_t s) {
    const long waves = (c.npix + 16 * MB - 1) / (16 * MB);
    const unsigned grid = (unsigned)((waves + 3) / 4);
    hipLaunchKernelGGL((conv3x3_kernel<CIN, COUT, MODE>), dim3(grid), dim3(CT), 0, s, c.X, c.Wp, c.bias, c.out, c.mask,
                       c.npix, c.H, c.W, c.cout_real);
    return hipGetLastError();
}

template <int CIN, int MODE>
static hipError_t conv_c(const ConvLaunch& c, hipStream_t s) {
    switch (c.cout) {
        case 16: return conv_t<CIN, 16, MODE>(c, s);
        case 32: return conv_t<CIN, 32, MODE>(c, s);
        case 64: return conv_t<CIN, 64, MODE>(c, s);
    }
    return hipErrorInvalidValue;
}

template <int MODE>
static hipError_t conv_m(const ConvLaunch& c, hipStream_t s) {
    switch (c.cin) {
        case 16: return conv_c<16, MODE>(c, s);
        case 32: return conv_c<32, MODE>(c, s);
        case 64: return conv_c<64, MODE>(c, s);
    }
    return hipErrorInvalidValue;
}

hipError_t conv3x3(const ConvLaunch& c, hipStream_t s) {
    if (c.npix <= 0) return hipSuccess;
    switch (c.mode) {
        case 0: return conv_m<0>(c, s);
        case 1: return conv_m<1>(c, s);
        case 2: return conv_m<2>(c, s);
    }
    return hipErrorInvalidValue;
}

template <int CIN, int COUT>
static hipError_t wgrad_t(const WgradLaunch& w, hipStream_t s) {
    hipLaunchKernelGGL((conv3x3_wgrad_kernel<CIN, COUT>), dim3(w.nblk), dim3(CT), 0, s, w.A, w.G, w.part, w.npix, w.H,
                       w.W, w.ppb);
    const long stride = (long)COUT * 9 * CIN + COUT;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((stride + 255) / 256)), dim3(256), 0, s, w.part, w.nblk,
                       stride, w.gw, w.gb, (long)COUT * 9 * CIN);
    return hipGetLastError();
}

template <int CIN>
static hipError_t wgrad_c(const WgradLaunch& w, hipStream_t s) {
    switch (w.cout) {
        case 16: return wgrad_t<CIN, 16>(w, s);
        case 32: return wgrad_t<CIN, 32>(w, s);
        case 64: return wgrad_t<CIN, 64>(w, s);
    }
    return hipErrorInvalidValue;
}

hipError_t conv3x3_wgrad(const WgradLaunch& w, hipStream_t s) {
    if (w.npix <= 0 || w.nblk <= 0) return hipErrorInvalidValue;
    switch (w.cin) {
        case 16: return wgrad_c<16>(w, s);
        case 32: return wgrad_c<32>(w, s);
        case 64: return wgrad_c<64>(w, s);
    }
    return hipErrorInvalidValue;
}

hipError_t gather_input(const float* X, const int* idx, int n_all, int batch, long hw, int c_real, int c_pad,
                        uint16_t* Xb, int* bad, hipStream_t s) {
    const long total = (long)batch * hw * c_pad;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_input_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, idx, n_all,
                       batch, hw, c_real, c_pad, Xb, bad);
    return hipGetLastError();
}

hipError_t mse_loss(const float* Y, const float* T, const int* idx, int n_all, const float* wch, int batch, long hw,
                    int c_real, int c_pad, uint16_t* G, double* part, double* loss, int* bad, hipStream_t s) {
    const long total = (long)batch * hw * c_pad;
    const int nblk = (int)((total + CT - 1) / CT);
    const double scale = 1.0 / ((double)batch * hw * c_real);
    hipLaunchKernelGGL(loss_kernel, dim3(nblk), dim3(CT), 0, s, Y, T, idx, n_all, wch, batch, hw, c_real, c_pad, scale,
                       G, part, bad);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(CT), 0, s, part, nblk, loss);
    return hipGetLastError();
}

long mse_loss_blocks(int batch, long hw, int c_pad) { return ((long)batch * hw * c_pad + CT - 1) / CT; }

hipError_t adam(float* p, float* m, float* v, const float* g, long n, float lr, float b1, float b2, float eps, float c1,
                float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t pack_weights(const float* Wm, int cin, int cout, uint16_t* Wp, uint16_t* Wt, hipStream_t s) {
    const long n = (long)cout * 9 * cin;
    hipLaunchKernelGGL(pack_weights_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Wm, cin, cout, Wp, Wt);
    return hipGetLastError();
}

}  // namespace smmcnn
