// net_internal.h -- shared declarations of the learned coarse propagator's kernels and host
// runtime.  Not part of the public ABI (include/fcn.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace fcn {

struct bf16_t {
    uint16_t v;
};

// One network sample: a window of the complex FP32 field of one instance (public layout
// fcn_net_sample in include/fcn.h, same field order).
struct NetSample {
    int64_t field_off;   // complex elements: the field the sample reads (input) or writes (apply)
    int64_t coarse_off;  // complex elements: the coarse field (targets, apply)
    int32_t row0, col0;  // first row (r index) and column (t index) of the window
    float in_scale;      // network input = field * in_scale
    float out_scale;     // network output = (fine - coarse) / out_scale
};

hipError_t launch_conv5(int act_bf16, int in_kind, int out_kind, const void *in, const float *w, const float *bias,
                        void *out, int B, int Cin, int Hin, int Win, int Cout, int Hout, int Wout, int pad, int relu,
                        hipStream_t s);
// BF16 MFMA convolution of the Cin -> 64 real-channel layers (Cin = 32 or 64), valid, BF16 in
// and out; its weights are packed from the real-form FP32 weights by launch_pack_mfma_weights
// into conv5_mfma_weight_bytes(Cin) bytes.
bool conv5_mfma_supported(int Cin, int Cout);
size_t conv5_mfma_weight_bytes(int Cin);
hipError_t launch_pack_mfma_weights(const float *wr, void *wA, int Cin, hipStream_t s);
hipError_t launch_conv5_mfma(const void *in, const void *wA, const float *bias, void *out, int B, int Cin, int Hin,
                             int Win, int Hout, int Wout, int relu, hipStream_t s);
// Weight and bias gradients of a 5x5 layer.  part: NULL, or conv5_wgrad_part_floats(B, Cin, Cout)
// floats of scratch, which selects the matrix-core form for square layers of 16, 32, 48 or 64
// real channels (0 floats: the vector kernel is used).
size_t conv5_wgrad_part_floats(int B, int Cin, int Cout);
hipError_t launch_conv5_wgrad(int act_bf16, const void *in, const float *g, float *gw, float *gb, float *part, int B,
                              int Cin, int Hin, int Win, int Cout, int Hout, int Wout, hipStream_t s);
hipError_t launch_relu_mask(int act_bf16, float *g, const void *act, size_t n, hipStream_t s);
hipError_t launch_expand_weights(const float *pc, float *wr, float *br, int cout, int cin, hipStream_t s);
hipError_t launch_flip_transpose(const float *w, float *wt, int cout, int cin, hipStream_t s);
hipError_t launch_contract_grads(const float *gwr, const float *gbr, float *gc, int cout, int cin, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s);
hipError_t launch_loss(const float *pred, const float *tgt, const int *row0, int B, int H, int W, double *nd,
                       float *grad, hipStream_t s);
hipError_t launch_net_input(int act_bf16, const float2 *fields, const NetSample *smp, int B, int nr, int nt, int H,
                            int W, void *out, hipStream_t s);
hipError_t launch_net_target(const float2 *fine, const float2 *coarse, const NetSample *smp, int B, int nr, int nt,
                             int H, int W, float *out, hipStream_t s);
hipError_t launch_net_apply(const float *net, const float2 *base, const NetSample *smp, int B, int nr, int nt,
                            float2 *dst, hipStream_t s);
hipError_t launch_parareal_update(const float2 *g_new, const float2 *f_old, const float2 *g_old, const float2 *u_prev,
                                  float2 *u_new, int nr, int nt, double *part, int nblocks, hipStream_t s);

}  // namespace fcn
