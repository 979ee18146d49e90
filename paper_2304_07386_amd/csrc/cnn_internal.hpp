// Internal state of a warm-start network (smm_cnn.h).
#pragma once

#include <stdint.h>

#include <vector>

struct smm_ctx;

struct smm_cnn {
    smm_ctx* ctx = nullptr;
    int L = 0, H = 0, W = 0, maxB = 0;
    std::vector<int> ch, chp;              // real and padded channel counts, L + 1 each
    std::vector<size_t> woff, boff, poff;  // per layer: master weight / bias offsets, packed weight offsets
    size_t nmaster = 0;
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;  // padded FP32 [nmaster]
    uint16_t *Wp = nullptr, *Wt = nullptr;  // bf16 forward / input-gradient operands
    std::vector<uint16_t*> act;             // layer inputs, bf16 [maxB][H][W][chp[l]]
    float* y = nullptr;                     // output [maxB][H][W][ch[L]]
    uint16_t *g0 = nullptr, *g1 = nullptr;  // gradient ping-pong buffers
    float* part = nullptr;
    size_t part_stride_max = 0;
    int part_blocks_max = 0;
    long loss_blocks_max = 0;
    double *loss_part = nullptr, *loss = nullptr;
    float* chan_w = nullptr;
    int* bad = nullptr;                     // device flag: image index out of range
    int t = 0;
    bool have_grad = false;
    std::vector<void*> allocs;
};

namespace smm {
// forward pass of images idx[0..batch) (idx device, nullable) of the n_all images x_all into y (device)
int cnn_forward_dev(smm_cnn* net, const float* x_all, int n_all, const int* idx, int batch, float* y);
}
