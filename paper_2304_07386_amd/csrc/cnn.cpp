// Host side of the warm-start network: parameter layout, device buffers,
// forward pass, backward pass and Adam (C ABI of smm_cnn.h).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/smm_cnn.h"
#include "api_internal.hpp"
#include "cnn_internal.hpp"
#include "cnn_kernels.hpp"

using smm::fail;

namespace {

int pad_channels(int c) { return c <= 16 ? 16 : c <= 32 ? 32 : 64; }

constexpr int WGRAD_PPB = 1024;  // pixels per weight-gradient partial

}  // namespace

extern "C" {

int smm_cnn_create(smm_ctx* ctx, int n_layers, const int* channels, int height, int width, int max_batch,
                   smm_cnn** out) {
    if (!ctx || !out || !channels) return SMM_EINVAL;
    *out = nullptr;
    if (ctx->device < 0) return fail(ctx, SMM_ESTATE, "smm_cnn_create needs a device context");
    if (n_layers < 1 || n_layers > 16 || height < 1 || width < 1 || max_batch < 1 ||
        (long)height * width * max_batch > (1L << 31))
        return fail(ctx, SMM_EINVAL, "smm_cnn_create: bad sizes");
    for (int l = 0; l <= n_layers; ++l)
        if (channels[l] < 1 || channels[l] > 64) return fail(ctx, SMM_EINVAL, "smm_cnn_create: channels must be 1..64");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SMM_EHIP, "hipSetDevice");
    auto* net = new smm_cnn();
    net->ctx = ctx;
    net->L = n_layers;
    net->H = height;
    net->W = width;
    net->maxB = max_batch;
    net->ch.assign(channels, channels + n_layers + 1);
    for (int c : net->ch) net->chp.push_back(pad_channels(c));
    size_t off = 0, poff = 0;
    for (int l = 0; l < n_layers; ++l) {
        const size_t nw = (size_t)net->chp[l + 1] * 9 * net->chp[l];
        net->woff.push_back(off);
        off += nw;
        net->boff.push_back(off);
        off += net->chp[l + 1];
        net->poff.push_back(poff);
        poff += nw;
    }
    net->nmaster = off;
    const long hw = (long)height * width, npix = hw * max_batch;
    int maxc = 0;
    for (int c : net->chp) maxc = std::max(maxc, c);
    size_t part = 0;
    for (int l = 0; l < n_layers; ++l) part = std::max(part, (size_t)net->chp[l + 1] * 9 * net->chp[l] + net->chp[l + 1]);
    net->part_stride_max = part;
    net->part_blocks_max = (int)((npix + WGRAD_PPB - 1) / WGRAD_PPB);
    net->loss_blocks_max = smmcnn::mse_loss_blocks(max_batch, hw, net->chp[n_layers]);
    auto alloc = [&](void** p, size_t bytes) {
        if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) return false;
        net->allocs.push_back(*p);
        return true;
    };
    bool ok = alloc((void**)&net->master, sizeof(float) * off) && alloc((void**)&net->m, sizeof(float) * off) &&
              alloc((void**)&net->v, sizeof(float) * off) && alloc((void**)&net->grad, sizeof(float) * off) &&
              alloc((void**)&net->Wp, sizeof(uint16_t) * poff) && alloc((void**)&net->Wt, sizeof(uint16_t) * poff) &&
              alloc((void**)&net->y, sizeof(float) * npix * net->ch[n_layers]) &&
              alloc((void**)&net->g0, sizeof(uint16_t) * npix * maxc) &&
              alloc((void**)&net->g1, sizeof(uint16_t) * npix * maxc) &&
              alloc((void**)&net->part, sizeof(float) * part * net->part_blocks_max) &&
              alloc((void**)&net->loss_part, sizeof(double) * net->loss_blocks_max) &&
              alloc((void**)&net->loss, sizeof(double)) && alloc((void**)&net->chan_w, sizeof(float) * 64) &&
              alloc((void**)&net->bad, sizeof(int));
    net->act.assign(n_layers, nullptr);
    for (int l = 0; ok && l < n_layers; ++l) ok = alloc((void**)&net->act[l], sizeof(uint16_t) * npix * net->chp[l]);
    if (!ok) {
        smm_cnn_destroy(net);
        return fail(ctx, SMM_ENOMEM, "smm_cnn_create: device allocation failed");
    }
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, hipMemsetAsync(net->master, 0, sizeof(float) * off, s));
    HIPCHK(ctx, hipMemsetAsync(net->m, 0, sizeof(float) * off, s));
    HIPCHK(ctx, hipMemsetAsync(net->v, 0, sizeof(float) * off, s));
    HIPCHK(ctx, hipMemsetAsync(net->Wp, 0, sizeof(uint16_t) * poff, s));
    HIPCHK(ctx, hipMemsetAsync(net->Wt, 0, sizeof(uint16_t) * poff, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    *out = net;
    return SMM_OK;
}

int smm_cnn_destroy(smm_cnn* net) {
    if (!net) return SMM_OK;
    if (net->ctx && net->ctx->device >= 0) (void)hipSetDevice(net->ctx->device);
    for (void* p : net->allocs) (void)hipFree(p);
    delete net;
    return SMM_OK;
}

int smm_cnn_num_params(const smm_cnn* net, size_t* n) {
    if (!net || !n) return SMM_EINVAL;
    size_t k = 0;
    for (int l = 0; l < net->L; ++l) k += (size_t)net->ch[l + 1] * net->ch[l] * 9 + net->ch[l + 1];
    *n = k;
    return SMM_OK;
}

}  // extern "C"

namespace smm {

// external W[o][c][3][3], b[o] (real channels)  <->  master W[o][tap][c], b[o] (padded)
static void to_master(const smm_cnn* net, const float* ext, std::vector<float>& mst) {
    mst.assign(net->nmaster, 0.f);
    size_t e = 0;
    for (int l = 0; l < net->L; ++l) {
        const int ci = net->ch[l], co = net->ch[l + 1], cip = net->chp[l];
        for (int o = 0; o < co; ++o)
            for (int c = 0; c < ci; ++c)
                for (int t = 0; t < 9; ++t) mst[net->woff[l] + ((size_t)o * 9 + t) * cip + c] = ext[e++];
        for (int o = 0; o < co; ++o) mst[net->boff[l] + o] = ext[e++];
    }
}

static void from_master(const smm_cnn* net, const std::vector<float>& mst, float* ext) {
    size_t e = 0;
    for (int l = 0; l < net->L; ++l) {
        const int ci = net->ch[l], co = net->ch[l + 1], cip = net->chp[l];
        for (int o = 0; o < co; ++o)
            for (int c = 0; c < ci; ++c)
                for (int t = 0; t < 9; ++t) ext[e++] = mst[net->woff[l] + ((size_t)o * 9 + t) * cip + c];
        for (int o = 0; o < co; ++o) ext[e++] = mst[net->boff[l] + o];
    }
}

static int pack_all(smm_cnn* net) {
    for (int l = 0; l < net->L; ++l)
        HIPCHK(net->ctx, smmcnn::pack_weights(net->master + net->woff[l], net->chp[l], net->chp[l + 1],
                                              net->Wp + net->poff[l], net->Wt + net->poff[l], net->ctx->stream));
    return SMM_OK;
}

// forward pass of images idx[0..batch) of x_all; activations kept for the backward pass
int cnn_forward_dev(smm_cnn* net, const float* x_all, int n_all, const int* idx, int batch, float* y) {
    smm_ctx* c = net->ctx;
    hipStream_t s = c->stream;
    const long hw = (long)net->H * net->W, npix = hw * batch;
    HIPCHK(c, smmcnn::gather_input(x_all, idx, n_all, batch, hw, net->ch[0], net->chp[0], net->act[0], net->bad, s));
    for (int l = 0; l < net->L; ++l) {
        smmcnn::ConvLaunch cl{};
        const bool last = l == net->L - 1;
        cl.mode = last ? 1 : 0;
        cl.cin = net->chp[l];
        cl.cout = net->chp[l + 1];
        cl.cout_real = net->ch[l + 1];
        cl.X = net->act[l];
        cl.Wp = net->Wp + net->poff[l];
        cl.bias = net->master + net->boff[l];
        cl.out = last ? (void*)y : (void*)net->act[l + 1];
        cl.npix = npix;
        cl.H = net->H;
        cl.W = net->W;
        HIPCHK(c, smmcnn::conv3x3(cl, s));
    }
    return SMM_OK;
}

}  // namespace smm

extern "C" {

int smm_cnn_set_params(smm_cnn* net, const float* params, size_t n) {
    if (!net || !params) return SMM_EINVAL;
    size_t k;
    smm_cnn_num_params(net, &k);
    if (n != k) return fail(net->ctx, SMM_EINVAL, "smm_cnn_set_params: expected " + std::to_string(k) + " floats");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return fail(net->ctx, SMM_EINVAL, "smm_cnn_set_params: non-finite parameter");
    std::vector<float> mst;
    smm::to_master(net, params, mst);
    smm_ctx* c = net->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(net->master, mst.data(), sizeof(float) * mst.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(net->m, 0, sizeof(float) * net->nmaster, c->stream));
    HIPCHK(c, hipMemsetAsync(net->v, 0, sizeof(float) * net->nmaster, c->stream));
    int rc;
    if ((rc = smm::pack_all(net))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    net->t = 0;
    net->have_grad = false;
    return SMM_OK;
}

int smm_cnn_get_params(smm_cnn* net, float* params, size_t n) {
    if (!net || !params) return SMM_EINVAL;
    size_t k;
    smm_cnn_num_params(net, &k);
    if (n != k) return fail(net->ctx, SMM_EINVAL, "smm_cnn_get_params: expected " + std::to_string(k) + " floats");
    smm_ctx* c = net->ctx;
    std::vector<float> mst(net->nmaster);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(mst.data(), net->master, sizeof(float) * mst.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    smm::from_master(net, mst, params);
    return SMM_OK;
}

int smm_cnn_forward(smm_cnn* net, const float* x, int batch, float* y) {
    if (!net || !x || !y) return SMM_EINVAL;
    if (batch < 0 || batch > net->maxB) return fail(net->ctx, SMM_EINVAL, "smm_cnn_forward: batch exceeds max_batch");
    if (batch == 0) return SMM_OK;
    HIPCHK(net->ctx, hipSetDevice(net->ctx->device));
    return smm::cnn_forward_dev(net, x, batch, nullptr, batch, y);
}

int smm_cnn_loss_grad(smm_cnn* net, const float* x_all, const float* t_all, int n_all, const int* idx, int batch,
                      const float* chan_weight, double* loss, float* grad) {
    if (!net || !x_all || !t_all) return SMM_EINVAL;
    smm_ctx* c = net->ctx;
    if (batch < 1 || batch > net->maxB) return fail(c, SMM_EINVAL, "smm_cnn_loss_grad: batch must be 1..max_batch");
    if (n_all < 1 || (!idx && n_all < batch)) return fail(c, SMM_EINVAL, "smm_cnn_loss_grad: n_all too small");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int L = net->L, cL = net->ch[L];
    std::vector<float> w(cL, 1.f);
    if (chan_weight)
        for (int k = 0; k < cL; ++k) w[k] = chan_weight[k];
    HIPCHK(c, hipMemcpyAsync(net->chan_w, w.data(), sizeof(float) * cL, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemsetAsync(net->bad, 0, sizeof(int), s));
    int rc;
    if ((rc = smm::cnn_forward_dev(net, x_all, n_all, idx, batch, net->y))) return rc;
    const long hw = (long)net->H * net->W, npix = hw * batch;
    uint16_t* g = net->g0;
    uint16_t* gnext = net->g1;
    HIPCHK(c, smmcnn::mse_loss(net->y, t_all, idx, n_all, net->chan_w, batch, hw, cL, net->chp[L], g, net->loss_part,
                               net->loss, net->bad, s));
    const int nblk = (int)((npix + WGRAD_PPB - 1) / WGRAD_PPB);
    for (int l = L - 1; l >= 0; --l) {
        smmcnn::WgradLaunch wl{};
        wl.cin = net->chp[l];
        wl.cout = net->chp[l + 1];
        wl.A = net->act[l];
        wl.G = g;
        wl.part = net->part;
        wl.gw = net->grad + net->woff[l];
        wl.gb = net->grad + net->boff[l];
        wl.npix = npix;
        wl.H = net->H;
        wl.W = net->W;
        wl.ppb = WGRAD_PPB;
        wl.nblk = nblk;
        HIPCHK(c, smmcnn::conv3x3_wgrad(wl, s));
        if (l > 0) {
            smmcnn::ConvLaunch cl{};
            cl.mode = 2;
            cl.cin = net->chp[l + 1];
            cl.cout = net->chp[l];
            cl.X = g;
            cl.Wp = net->Wt + net->poff[l];
            cl.out = gnext;
            cl.mask = net->act[l];
            cl.npix = npix;
            cl.H = net->H;
            cl.W = net->W;
            HIPCHK(c, smmcnn::conv3x3(cl, s));
            std::swap(g, gnext);
        }
    }
    double lv = 0;
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&lv, net->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(&bad, net->bad, sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<float> mst;
    if (grad) {
        mst.resize(net->nmaster);
        HIPCHK(c, hipMemcpyAsync(mst.data(), net->grad, sizeof(float) * mst.size(), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    if (bad) {
        net->have_grad = false;
        return fail(c, SMM_EINVAL, "smm_cnn_loss_grad: image index outside [0, n_all)");
    }
    if (loss) *loss = lv;
    if (grad) smm::from_master(net, mst, grad);
    net->have_grad = true;
    return SMM_OK;
}

int smm_cnn_adam_step(smm_cnn* net, float lr, float beta1, float beta2, float eps) {
    if (!net) return SMM_EINVAL;
    smm_ctx* c = net->ctx;
    if (!net->have_grad) return fail(c, SMM_ESTATE, "smm_cnn_adam_step: no gradient (call smm_cnn_loss_grad)");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(c, SMM_EINVAL, "smm_cnn_adam_step: bad hyper-parameters");
    HIPCHK(c, hipSetDevice(c->device));
    net->t += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, net->t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, net->t)));
    HIPCHK(c, smmcnn::adam(net->master, net->m, net->v, net->grad, (long)net->nmaster, lr, beta1, beta2, eps, c1, c2,
                           c->stream));
    int rc;
    if ((rc = smm::pack_all(net))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SMM_OK;
}

}  // extern "C"
