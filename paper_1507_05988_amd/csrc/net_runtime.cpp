// net_runtime.cpp -- host side of the learned coarse propagator: parameter layout, workspace,
// forward / backward / optimiser sequencing and the C ABI (fcn_net_* in include/fcn.h).
//
// Network: 4 complex 5x5 valid convolutions 1 -> C -> C -> C -> 1 with complex biases and
// CReLU (ReLU on real and imaginary parts) after layers 1-3.  An input window of H x W
// output points is read with an 8-point halo (the receptive field), so layer l maps
// (H + 16 - 4l) x (W + 16 - 4l) to (H + 12 - 4l) x (W + 12 - 4l).
// Parameters (caller-owned FP32 buffer), per layer: W[co][ci][25] as (re, im), b[co] as (re, im).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fcn.h"
#include "net_internal.h"

using namespace fcn;

namespace {
size_t al(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

struct fcn_net_s {
    int C = 32;
    int act_bf16 = 1;
    int mfma = 1;             // BF16 layers 64 -> 64 real channels on the matrix cores
    int cin[4], cout[4];      // complex channels per layer
    size_t poff[5];           // float offsets of the layers' parameters; poff[4] = total
    // bound state
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    int max_b = 0, max_h = 0, max_w = 0, training = 0;
    bool bound = false;
    int64_t adam_t = 0;
    // workspace pieces
    float *wr[4], *br[4], *wt[4], *gwr[4], *gbr[4];
    void *wA[4];              // packed MFMA weight fragments (layers that use the matrix cores)
    void *act[4];             // act[0]: input; act[1..3]: post-activations of layers 1..3
    float *out = nullptr;     // FP32 [b][2][h][w]
    float *g[2];              // FP32 gradient ping-pong
    float *gout = nullptr;    // FP32 loss gradient [b][2][h][w]
    float *wpart = nullptr;   // per-image partial weight gradients of the hidden layers (matrix-core form)
    double *nd = nullptr;     // loss partials [b][2]
    int *row0 = nullptr;      // loss row offsets [b]
    std::string err;

    size_t act_bytes() const { return act_bf16 ? 2 : 4; }
    bool use_mfma(int l) const { return act_bf16 && mfma && l < 3 && conv5_mfma_supported(2 * cin[l], 2 * cout[l]); }
};

namespace {

fcn_status net_fail(fcn_net_t n, fcn_status st, const std::string &msg) {
    if (n) n->err = msg;
    return st;
}
fcn_status net_hip(fcn_net_t n, hipError_t e, const char *what) {
    return net_fail(n, FCN_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Workspace layout for (B, H, W); when p is null only the size is computed.
size_t layout(fcn_net_t n, int B, int H, int W, int training, unsigned char *p) {
    size_t o = 0;
    auto take = [&](size_t bytes) -> unsigned char * {
        unsigned char *r = p ? p + o : nullptr;
        o = al(o + bytes);
        return r;
    };
    for (int l = 0; l < 4; l++) {
        const size_t nw = (size_t)(2 * n->cout[l]) * (2 * n->cin[l]) * 25;
        n->wr[l] = (float *)take(nw * 4);
        n->br[l] = (float *)take((size_t)2 * n->cout[l] * 4);
        n->wt[l] = (float *)take(nw * 4);
        n->gwr[l] = (float *)take(training ? nw * 4 : 0);
        n->gbr[l] = (float *)take(training ? (size_t)2 * n->cout[l] * 4 : 0);
        n->wA[l] = n->use_mfma(l) ? take(conv5_mfma_weight_bytes(2 * n->cin[l])) : nullptr;
    }
    const size_t ab = n->act_bytes();
    const size_t C2 = 2 * (size_t)n->C;
    n->act[0] = take((size_t)B * 2 * (H + 16) * (W + 16) * ab);
    if (training) {
        n->act[1] = take((size_t)B * C2 * (H + 12) * (W + 12) * ab);
        n->act[2] = take((size_t)B * C2 * (H + 8) * (W + 8) * ab);
        n->act[3] = take((size_t)B * C2 * (H + 4) * (W + 4) * ab);
    } else {  // inference: layers ping-pong between two buffers of the largest size
        n->act[1] = take((size_t)B * C2 * (H + 12) * (W + 12) * ab);
        n->act[2] = take((size_t)B * C2 * (H + 8) * (W + 8) * ab);
        n->act[3] = n->act[1];
    }
    n->out = (float *)take((size_t)B * 2 * H * W * 4);
    const size_t gsz = training ? (size_t)B * C2 * (H + 12) * (W + 12) * 4 : 0;
    n->g[0] = (float *)take(gsz);
    n->g[1] = (float *)take(gsz);
    n->gout = (float *)take(training ? (size_t)B * 2 * H * W * 4 : 0);
    n->wpart = (float *)take(training ? conv5_wgrad_part_floats(B, (int)C2, (int)C2) * 4 : 0);
    n->nd = (double *)take((size_t)B * 2 * 8);
    n->row0 = (int *)take((size_t)B * 4);
    return o;
}

// (H_in, W_in) of layer l for output window (H, W)
inline int lin_h(int l, int H) { return H + 16 - 4 * l; }

hipError_t expand_all(fcn_net_t n) {
    hipError_t e = hipSuccess;
    for (int l = 0; l < 4 && e == hipSuccess; l++) {
        e = launch_expand_weights(n->params + n->poff[l], n->wr[l], n->br[l], n->cout[l], n->cin[l], n->stream);
        if (e == hipSuccess && n->use_mfma(l)) e = launch_pack_mfma_weights(n->wr[l], n->wA[l], 2 * n->cin[l], n->stream);
        if (e == hipSuccess && n->training)
            e = launch_flip_transpose(n->wr[l], n->wt[l], 2 * n->cout[l], 2 * n->cin[l], n->stream);
    }
    return e;
}

fcn_status check_dims(fcn_net_t n, int B, int H, int W) {
    if (!n->bound) return net_fail(n, FCN_E_STATE, "network is not bound");
    if (B < 1 || H < 1 || W < 1 || B > n->max_b || H > n->max_h || W > n->max_w)
        return net_fail(n, FCN_E_SIZE, "batch or window larger than the bound workspace");
    return FCN_OK;
}

}  // namespace

namespace fcn {
hipStream_t net_stream(fcn_net_t n) { return n->stream; }
}  // namespace fcn

extern "C" {

fcn_status fcn_net_create(int32_t channels, int32_t act_bf16, fcn_net_t *out) {
    if (!out) return FCN_E_ARG;
    *out = nullptr;
    if (channels < 1 || channels > 64 || act_bf16 < 0 || act_bf16 > 2) return FCN_E_ARG;
    fcn_net_t n = new fcn_net_s();
    n->C = channels;
    n->act_bf16 = act_bf16 ? 1 : 0;
    n->mfma = act_bf16 == 1 ? 1 : 0;
    const int ci[4] = {1, channels, channels, channels}, co[4] = {channels, channels, channels, 1};
    size_t o = 0;
    for (int l = 0; l < 4; l++) {
        n->cin[l] = ci[l];
        n->cout[l] = co[l];
        n->poff[l] = o;
        o += (size_t)2 * co[l] * ci[l] * 25 + (size_t)2 * co[l];
    }
    n->poff[4] = o;
    *out = n;
    return FCN_OK;
}

fcn_status fcn_net_param_count(fcn_net_t n, size_t *nfloats) {
    if (!n || !nfloats) return FCN_E_ARG;
    *nfloats = n->poff[4];
    return FCN_OK;
}

fcn_status fcn_net_workspace_size(fcn_net_t n, int32_t max_batch, int32_t max_h, int32_t max_w, int32_t training,
                                  size_t *bytes) {
    if (!n || !bytes || max_batch < 1 || max_h < 1 || max_w < 1) return FCN_E_ARG;
    *bytes = layout(n, max_batch, max_h, max_w, training, nullptr);
    return FCN_OK;
}

fcn_status fcn_net_bind(fcn_net_t n, float *params, float *grads, float *adam_m, float *adam_v, void *ws,
                        size_t ws_bytes, int32_t max_batch, int32_t max_h, int32_t max_w, int32_t training,
                        void *stream) {
    if (!n) return FCN_E_ARG;
    n->err.clear();
    if (!params || !ws) return net_fail(n, FCN_E_ARG, "NULL parameter or workspace buffer");
    if (training && (!grads || !adam_m || !adam_v)) return net_fail(n, FCN_E_ARG, "training needs grads and Adam state");
    if (((uintptr_t)ws & 255) != 0) return net_fail(n, FCN_E_ARG, "workspace must be 256-byte aligned");
    if (max_batch < 1 || max_h < 1 || max_w < 1) return net_fail(n, FCN_E_ARG, "bad maximum sizes");
    const size_t need = layout(n, max_batch, max_h, max_w, training, nullptr);
    if (ws_bytes < need) return net_fail(n, FCN_E_SIZE, "workspace too small");
    n->params = params;
    n->grads = grads;
    n->m = adam_m;
    n->v = adam_v;
    n->ws = (unsigned char *)ws;
    n->ws_bytes = ws_bytes;
    n->max_b = max_batch;
    n->max_h = max_h;
    n->max_w = max_w;
    n->training = training ? 1 : 0;
    n->stream = (hipStream_t)stream;
    layout(n, max_batch, max_h, max_w, training, n->ws);
    n->bound = true;
    n->adam_t = 0;
    hipError_t e = expand_all(n);
    return e == hipSuccess ? FCN_OK : net_hip(n, e, "expand weights");
}

fcn_status fcn_net_refresh(fcn_net_t n) {
    if (!n) return FCN_E_ARG;
    if (!n->bound) return net_fail(n, FCN_E_STATE, "network is not bound");
    hipError_t e = expand_all(n);
    return e == hipSuccess ? FCN_OK : net_hip(n, e, "expand weights");
}

fcn_status fcn_net_input(fcn_net_t n, const void *fields, const fcn_net_sample *samples, int32_t batch, int32_t nr,
                         int32_t nt, int32_t h, int32_t w) {
    if (!n) return FCN_E_ARG;
    n->err.clear();
    fcn_status st = check_dims(n, batch, h, w);
    if (st != FCN_OK) return st;
    if (!fields || !samples || nr < 3 || nt < 1) return net_fail(n, FCN_E_ARG, "bad field arguments");
    hipError_t e = launch_net_input(n->act_bf16, (const float2 *)fields, (const NetSample *)samples, batch, nr, nt, h,
                                    w, n->act[0], n->stream);
    return e == hipSuccess ? FCN_OK : net_hip(n, e, "net input");
}

fcn_status fcn_net_forward(fcn_net_t n, int32_t batch, int32_t h, int32_t w, float *out) {
    if (!n) return FCN_E_ARG;
    n->err.clear();
    fcn_status st = check_dims(n, batch, h, w);
    if (st != FCN_OK) return st;
    hipError_t e = hipSuccess;
    // activation buffers: input act[0] -> act[1] -> act[2] -> act[3] -> out (FP32)
    for (int l = 0; l < 4 && e == hipSuccess; l++) {
        const int Hi = lin_h(l, h), Wi = lin_h(l, w), Ho = Hi - 4, Wo = Wi - 4;
        const void *src = n->act[l];
        void *dst = (l < 3) ? n->act[l + 1] : (void *)n->out;
        if (n->use_mfma(l))
            e = launch_conv5_mfma(src, n->wA[l], n->br[l], dst, batch, 2 * n->cin[l], Hi, Wi, Ho, Wo, 1, n->stream);
        else
            e = launch_conv5(n->act_bf16, 1, l < 3 ? 1 : 0, src, n->wr[l], n->br[l], dst, batch, 2 * n->cin[l], Hi, Wi,
                             2 * n->cout[l], Ho, Wo, 0, l < 3 ? 1 : 0, n->stream);
    }
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(out, n->out, (size_t)batch * 2 * h * w * 4, hipMemcpyDeviceToDevice, n->stream);
    return e == hipSuccess ? FCN_OK : net_hip(n, e, "forward");
}

fcn_status fcn_net_loss(fcn_net_t n, const float *target, const int32_t *row0_host, int32_t batch, int32_t h,
                        int32_t w, int32_t with_grad, double *loss) {
    if (!n) return FCN_E_ARG;
    n->err.clear();
    fcn_status st = check_dims(n, batch, h, w);
    if (st != FCN_OK) return st;
    if (!target || !row0_host || !loss) return net_fail(n, FCN_E_ARG, "NULL argument");
    if (with_grad && !n->training) return net_fail(n, FCN_E_STATE, "gradients need a training workspace");
    hipError_t e = hipMemcpyAsync(n->row0, row0_host, (size_t)batch * 4, hipMemcpyHostToDevice, n->stream);
    if (e == hipSuccess) e = launch_loss(n->out, target, n->row0, batch, h, w, n->nd, with_grad ? n->gout : nullptr, n->stream);
    std::vector<double> nd((size_t)2 * batch);
    if (e == hipSuccess) e = hipMemcpyAsync(nd.data(), n->nd, nd.size() * 8, hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) return net_hip(n, e, "loss");
    double s = 0.0;
    for (int b = 0; b < batch; b++) s += nd[2 * b] / (nd[2 * b + 1] > 0.0 ? nd[2 * b + 1] : 1.0);
    *loss = s / batch;
    return FCN_OK;
}

fcn_status fcn_net_backward(fcn_net_t n, int32_t batch, int32_t h, int32_t w) {
    if (!n) return FCN_E_ARG;
    n->err.clear();
    fcn_status st = check_dims(n, batch, h, w);
    if (st != FCN_OK) return st;
    if (!n->training) return net_fail(n, FCN_E_STATE, "backward needs a training workspace");
    hipError_t e = hipSuccess;
    const float *gcur = n->gout;  // gradient of layer l's output
    int pp = 0;
    for (int l = 3; l >= 0 && e == hipSuccess; l--) {
        const int Hi = lin_h(l, h), Wi = lin_h(l, w), Ho = Hi - 4, Wo = Wi - 4;
        const int Ci = 2 * n->cin[l], Co = 2 * n->cout[l];
        // parameter gradients of layer l
        e = launch_conv5_wgrad(n->act_bf16, n->act[l], gcur, n->gwr[l], n->gbr[l],
                               conv5_wgrad_part_floats(batch, Ci, Co) ? n->wpart : nullptr, batch, Ci, Hi, Wi, Co, Ho,
                               Wo, n->stream);
        if (e == hipSuccess)
            e = launch_contract_grads(n->gwr[l], n->gbr[l], n->grads + n->poff[l], n->cout[l], n->cin[l], n->stream);
        if (l == 0) break;
        // gradient of layer l's input = gradient of layer l-1's post-activation, then through its ReLU
        float *gnext = n->g[pp];
        pp ^= 1;
        if (e == hipSuccess)
            e = launch_conv5(0, 0, 0, gcur, n->wt[l], nullptr, gnext, batch, Co, Ho, Wo, Ci, Hi, Wi, 4, 0, n->stream);
        if (e == hipSuccess) e = launch_relu_mask(n->act_bf16, gnext, n->act[l], (size_t)batch * Ci * Hi * Wi, n->stream);
        gcur = gnext;
    }
    return e == hipSuccess ? FCN_OK : net_hip(n, e, "backward");
}

fcn_status fcn_net_adam(fcn_net_t n, float lr, float beta1, float beta2, float eps) {
    if (!n) return FCN_E_ARG;
    n->err.clear();
    if (!n->bound || !n->training) return net_fail(n, FCN_E_STATE, "Adam needs a bound training network");
    n->adam_t++;
    const float c1 = 1.0f - std::pow(beta1, (float)n->adam_t);
    const float c2 = 1.0f - std::pow(beta2, (float)n->adam_t);
    hipError_t e = launch_adam(n->params, n->grads, n->m, n->v, n->poff[4], lr, beta1, beta2, eps, c1, c2, n->stream);
    if (e == hipSuccess) e = expand_all(n);
    return e == hipSuccess ? FCN_OK : net_hip(n, e, "adam");
}

fcn_status fcn_net_target(fcn_net_t n, const void *fine, const void *coarse, const fcn_net_sample *samples,
                          int32_t batch, int32_t nr, int32_t nt, int32_t h, int32_t w, float *target) {
    if (!n) return FCN_E_ARG;
    n->err.clear();
    fcn_status st = check_dims(n, batch, h, w);
    if (st != FCN_OK) return st;
    if (!fine || !coarse || !samples || !target) return net_fail(n, FCN_E_ARG, "NULL argument");
    hipError_t e = launch_net_target((const float2 *)fine, (const float2 *)coarse, (const NetSample *)samples, batch,
                                     nr, nt, h, w, target, n->stream);
    return e == hipSuccess ? FCN_OK : net_hip(n, e, "target");
}

fcn_status fcn_net_apply(fcn_net_t n, const void *base, const fcn_net_sample *samples, int32_t batch, int32_t nr,
                         int32_t nt, void *dst) {
    if (!n) return FCN_E_ARG;
    n->err.clear();
    fcn_status st = check_dims(n, batch, nr, nt);
    if (st != FCN_OK) return st;
    if (!base || !samples || !dst) return net_fail(n, FCN_E_ARG, "NULL argument");
    hipError_t e = launch_net_apply(n->out, (const float2 *)base, (const NetSample *)samples, batch, nr, nt,
                                    (float2 *)dst, n->stream);
    return e == hipSuccess ? FCN_OK : net_hip(n, e, "apply");
}

const char *fcn_net_last_error(fcn_net_t n) { return n ? n->err.c_str() : "NULL network"; }

fcn_status fcn_net_destroy(fcn_net_t n) {
    if (!n) return FCN_E_ARG;
    delete n;
    return FCN_OK;
}

fcn_status fcn_parareal_update(const void *g_new, const void *f_old, const void *g_old, const void *u_prev, void *u_new,
                               int32_t nr, int32_t nt, double *part_dev, int32_t nparts, void *stream) {
    if (!g_new || !f_old || !g_old || !u_prev || !u_new || !part_dev || nr < 1 || nt < 1 || nparts < 1 || nparts > 4096)
        return FCN_E_ARG;
    hipError_t e = launch_parareal_update((const float2 *)g_new, (const float2 *)f_old, (const float2 *)g_old,
                                          (const float2 *)u_prev, (float2 *)u_new, nr, nt, part_dev, nparts,
                                          (hipStream_t)stream);
    return e == hipSuccess ? FCN_OK : FCN_E_HIP;
}

}  // extern "C"
