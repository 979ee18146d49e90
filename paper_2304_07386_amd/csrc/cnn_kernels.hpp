// Launch descriptors of the warm-start network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smmcnn {

struct ConvLaunch {
    int mode;            // 0 hidden (bias + ReLU, bf16 out), 1 output (bias, fp32 out), 2 input gradient (masked)
    int cin, cout;       // padded channel counts (16, 32 or 64)
    int cout_real;       // mode 1: channels written
    const uint16_t* X;   // [npix][cin] bf16
    const uint16_t* Wp;  // [9*cin/4][cout][4] bf16
    const float* bias;   // [cout] (modes 0, 1)
    void* out;
    const uint16_t* mask;  // mode 2: [npix][cout] bf16 activations
    long npix;
    int H, W;
};

struct WgradLaunch {
    int cin, cout;
    const uint16_t* A;  // layer input [npix][cin]
    const uint16_t* G;  // output gradient [npix][cout]
    float* part;        // [nblk][cout*9*cin + cout]
    float* gw;          // [cout][9][cin]
    float* gb;          // [cout]
    long npix;
    int H, W, ppb, nblk;
};

hipError_t conv3x3(const ConvLaunch& c, hipStream_t s);
hipError_t conv3x3_wgrad(const WgradLaunch& w, hipStream_t s);
// idx (nullable) selects images of X / T; an index outside [0, n_all) yields
// zeros and sets *bad = 1
hipError_t gather_input(const float* X, const int* idx, int n_all, int batch, long hw, int c_real, int c_pad,
                        uint16_t* Xb, int* bad, hipStream_t s);
hipError_t mse_loss(const float* Y, const float* T, const int* idx, int n_all, const float* wch, int batch, long hw,
                    int c_real, int c_pad, uint16_t* G, double* part, double* loss, int* bad, hipStream_t s);
long mse_loss_blocks(int batch, long hw, int c_pad);
hipError_t adam(float* p, float* m, float* v, const float* g, long n, float lr, float b1, float b2, float eps, float c1,
                float c2, hipStream_t s);
hipError_t pack_weights(const float* Wm, int cin, int cout, uint16_t* Wp, uint16_t* Wt, hipStream_t s);

}  // namespace smmcnn
