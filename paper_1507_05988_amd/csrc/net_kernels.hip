// net_kernels.hip -- kernels of the learned coarse z-propagator: a complex-valued
// convolutional operator on the (r, t) grid (4 layers of 5x5 complex convolutions,
// 1 -> C -> C -> C -> 1 complex channels, CReLU between layers), its gradients and its
// optimiser, plus the helpers that cut network inputs and targets out of FCN fields and
// apply the network's correction.  Not part of the paper (an addition of this project).
//
// A complex layer with weights W = Wr + i Wi acts on (re, im) channel pairs as the real
// layer [[Wr, -Wi], [Wi, Wr]]: the kernels below are real 5x5 convolutions on 2C real
// channels, and the complex parameters are expanded to / contracted from that form.
// Activations are stored as FP32 or BF16 (type A), every sum is accumulated in FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "net_internal.h"

namespace fcn {

// ---------------------------------------------------------------- activation storage

__device__ __forceinline__ float ld_act(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float ld_act(const bf16_t *p, size_t i) {
    return __uint_as_float(((uint32_t)p[i].v) << 16);
}
__device__ __forceinline__ void st_act(float *p, size_t i, float x) { p[i] = x; }
// FP32 -> BF16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ void st_act(bf16_t *p, size_t i, float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        p[i].v = (uint16_t)((u >> 16) | 0x40u);
        return;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    p[i].v = (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------- 5x5 convolution

constexpr int CV_TH = 16, CV_TW = 64, CV_CIT = 8, CV_PX = 4;
constexpr int CV_PITCH = CV_TW + 8;  // LDS row pitch in floats (16-byte aligned rows)

// out[b][co][y][x] = bias[co] + sum_{ci,ky,kx} in[b][ci][y+ky-pad][x+kx-pad] w[co][ci][ky][kx]
// (in read as 0 outside [0,Hin) x [0,Win)), ReLU when relu != 0.  Valid convolution with
// pad = 0; with pad = 4, flipped and transposed weights it is the input gradient.
// Workgroup: a 16 x 64 output tile and COT output channels; thread (ty, q) computes the 4
// adjacent outputs x = 4q .. 4q+3 of row ty for all COT channels.  Input channels are
// staged 8 at a time in LDS with the 4-point halo; a thread reads its 8-wide input window
// of each kernel row as two aligned 16-byte loads and slides it over the 5 taps.  Weight
// addresses are uniform across the workgroup, so they are read with scalar loads and
// every FMA takes one operand from an SGPR.  Channels beyond Cout reuse the last
// channel's weights and are not stored.
// Grid: x = ceil(Wout/64), y = ceil(Hout/16), z = B * ceil(Cout/COT); 256 threads.
template <typename AI, typename AO, int COT>
__global__ void __launch_bounds__(256) conv5_kernel(const AI *__restrict__ in, const float *__restrict__ w,
                                                    const float *__restrict__ bias, AO *__restrict__ out, int Cin,
                                                    int Hin, int Win, int Cout, int Hout, int Wout, int pad,
                                                    int relu) {
    __shared__ __align__(16) float s_in[CV_CIT][CV_TH + 4][CV_PITCH];
    const int co_groups = (Cout + COT - 1) / COT;
    const int b = blockIdx.z / co_groups;
    const int co0 = (blockIdx.z % co_groups) * COT;
    const int y0 = blockIdx.y * CV_TH, x0 = blockIdx.x * CV_TW;
    const int tid = threadIdx.x, ty = tid >> 4, q = tid & 15;
    const int clast = Cout - 1 - co0;  // last valid channel of the group, relative to co0
    float acc[CV_PX][COT];
#pragma unroll
    for (int j = 0; j < CV_PX; j++)
#pragma unroll
        for (int c = 0; c < COT; c++) acc[j][c] = 0.0f;

    for (int ci0 = 0; ci0 < Cin; ci0 += CV_CIT) {
        constexpr int TW4 = CV_TW + 4;
        constexpr int TILE = (CV_TH + 4) * TW4;
        for (int idx = tid; idx < CV_CIT * TILE; idx += 256) {
            const int ci = idx / TILE, rem = idx % TILE;
            const int yy = rem / TW4, xx = rem % TW4;
            const int gy = y0 + yy - pad, gx = x0 + xx - pad;
            float v = 0.0f;
            if (ci0 + ci < Cin && gy >= 0 && gy < Hin && gx >= 0 && gx < Win)
                v = ld_act(in, (((size_t)b * Cin + ci0 + ci) * Hin + gy) * Win + gx);
            s_in[ci][yy][xx] = v;
        }
        __syncthreads();
        const int nci = min(CV_CIT, Cin - ci0);
        for (int ci = 0; ci < nci; ci++) {
            const float *wc = w + ((size_t)co0 * Cin + ci0 + ci) * 25;
#pragma unroll
            for (int ky = 0; ky < 5; ky++) {
                const float4 lo = *reinterpret_cast<const float4 *>(&s_in[ci][ty + ky][4 * q]);
                const float4 hi = *reinterpret_cast<const float4 *>(&s_in[ci][ty + ky][4 * q + 4]);
                const float r[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
                for (int kx = 0; kx < 5; kx++) {
#pragma unroll
                    for (int c = 0; c < COT; c++) {
                        const float wv = wc[(size_t)min(c, clast) * Cin * 25 + ky * 5 + kx];
#pragma unroll
                        for (int j = 0; j < CV_PX; j++) acc[j][c] = fmaf(r[j + kx], wv, acc[j][c]);
                    }
                }
            }
        }
        __syncthreads();
    }
    const int y = y0 + ty;
    if (y < Hout) {
#pragma unroll
        for (int c = 0; c < COT; c++) {
            const int co = co0 + c;
            if (co < Cout) {
                const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
                for (int j = 0; j < CV_PX; j++) {
                    const int x = x0 + 4 * q + j;
                    if (x < Wout) {
                        float v = acc[j][c] + bv;
                        if (relu && v < 0.0f) v = 0.0f;  // NaN propagates
                        st_act(out, (((size_t)b * Cout + co) * Hout + y) * Wout + x, v);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- BF16 MFMA convolution

// The 64 -> 64 real-channel layers as an implicit GEMM on the matrix cores:
// out[co][p] = sum_{tap, ci} W[co][ci][tap] in[ci][p + tap], one v_mfma_f32_16x16x32_bf16 per
// (16 output channels) x (16 pixels) x (32 input channels of one tap).  Operand layout of
// that instruction (lane l of the wave): A[m = l % 16][k = 8 (l / 16) + i], B[k = 8 (l / 16) + i]
// [n = l % 16], i < 8; result C[m = 4 (l / 16) + i][n = l % 16], i < 4.  A = weights (m: output
// channel), B = inputs (n: pixel), so a lane's B operand is 8 consecutive input channels of
// one pixel: the input tile is staged in LDS channel-innermost ([y][x][c], 72 BF16 per pixel,
// 8 of them padding that spreads the 16-byte reads over the banks).  A fragments are packed
// once per weight update in exactly the lane order (pack_mfma_weights_kernel) and read with
// one 16-byte load per lane.
// Workgroup: 4 x 64 outputs, 4 waves; wave w computes output row w, 4 pixel tiles x 4 channel
// tiles (16 accumulators of 4 floats).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int MF_TH = 4, MF_TW = 64, MF_COUT = 64;

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// wA[((t * KC + kc) * 4 + ct) * 64 + lane] = W[16 ct + lane % 16][32 kc + 8 (lane / 16) + i][t], i < 8
__global__ void pack_mfma_weights_kernel(const float *__restrict__ wr, uint4 *__restrict__ wA, int cin, int kc_n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 25 * kc_n * 4 * 64) return;
    const int lane = idx & 63, ct = (idx >> 6) & 3, tk = idx >> 8;
    const int kc = tk % kc_n, t = tk / kc_n;
    const int co = 16 * ct + (lane & 15), ci0 = 32 * kc + 8 * (lane >> 4);
    uint16_t h[8];
#pragma unroll
    for (int i = 0; i < 8; i++) h[i] = bf16_rne(wr[((size_t)co * cin + ci0 + i) * 25 + t]);
    uint4 v;
    v.x = h[0] | ((uint32_t)h[1] << 16);
    v.y = h[2] | ((uint32_t)h[3] << 16);
    v.z = h[4] | ((uint32_t)h[5] << 16);
    v.w = h[6] | ((uint32_t)h[7] << 16);
    wA[idx] = v;
}

// Valid 5x5 convolution, BF16 in and out, Cin = 32 KC, Cout = 64; grid (ceil(Wout/64),
// ceil(Hout/4), B), 256 threads.
template <int KC>
__global__ void __launch_bounds__(256) conv5_mfma_kernel(const bf16_t *__restrict__ in, const uint4 *__restrict__ wA,
                                                         const float *__restrict__ bias, bf16_t *__restrict__ out,
                                                         int Hin, int Win, int Hout, int Wout, int relu) {
    constexpr int CIN = 32 * KC;
    constexpr int PIXS = CIN + 8;           // BF16 per staged pixel
    constexpr int SW = MF_TW + 4, SH = MF_TH + 4;
    __shared__ __align__(16) uint16_t s_in[SH * SW * PIXS];
    const int b = blockIdx.z;
    const int y0 = blockIdx.y * MF_TH, x0 = blockIdx.x * MF_TW;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

    // a thread stages 8 channels of one pixel: 8 coalesced 2-byte loads (lanes on consecutive
    // pixels), one 16-byte LDS store
    for (int idx = tid; idx < (CIN / 8) * SH * SW; idx += 256) {
        const int g = idx / (SH * SW), rem = idx % (SH * SW);
        const int yy = rem / SW, xx = rem % SW;
        const int gy = y0 + yy, gx = x0 + xx;
        const bool ok = gy < Hin && gx < Win;
        uint32_t h[8];
#pragma unroll
        for (int i = 0; i < 8; i++) h[i] = ok ? in[(((size_t)b * CIN + 8 * g + i) * Hin + gy) * Win + gx].v : 0u;
        uint4 v;
        v.x = h[0] | (h[1] << 16);
        v.y = h[2] | (h[3] << 16);
        v.z = h[4] | (h[5] << 16);
        v.w = h[6] | (h[7] << 16);
        *reinterpret_cast<uint4 *>(&s_in[(yy * SW + xx) * PIXS + 8 * g]) = v;
    }
    __syncthreads();

    f32x4_t acc[4][4];
#pragma unroll
    for (int pt = 0; pt < 4; pt++)
#pragma unroll
        for (int ct = 0; ct < 4; ct++) acc[pt][ct] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    const int n = lane & 15, kg = lane >> 4;
    // step it = t KC + kc: tap t, input channels 32 kc .. 32 kc + 31.  The weight fragments of
    // step it + 1 are loaded while step it's products run (they come from L2, the latency two
    // wavefronts per SIMD would otherwise leave exposed).
    constexpr int NIT = 25 * KC;
    uint4 wc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ct++) wc[ct] = wA[ct * 64 + lane];
    for (int it = 0; it < NIT; it++) {
        const int t = it / KC, kc = it % KC;
        const int ky = t / 5, kx = t % 5;
        uint4 wn[4];
        if (it + 1 < NIT) {
#pragma unroll
            for (int ct = 0; ct < 4; ct++) wn[ct] = wA[((it + 1) * 4 + ct) * 64 + lane];
        }
        bf16x8_t a[4];
#pragma unroll
        for (int ct = 0; ct < 4; ct++) a[ct] = __builtin_bit_cast(bf16x8_t, wc[ct]);
#pragma unroll
        for (int pt = 0; pt < 4; pt++) {
            const uint4 xv = *reinterpret_cast<const uint4 *>(
                &s_in[((wave + ky) * SW + 16 * pt + n + kx) * PIXS + 32 * kc + 8 * kg]);
            const bf16x8_t bx = __builtin_bit_cast(bf16x8_t, xv);
#pragma unroll
            for (int ct = 0; ct < 4; ct++) acc[pt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ct], bx, acc[pt][ct], 0, 0, 0);
        }
        if (it + 1 < NIT) {
#pragma unroll
            for (int ct = 0; ct < 4; ct++) wc[ct] = wn[ct];
        }
    }

    const int y = y0 + wave;
    if (y < Hout) {
#pragma unroll
        for (int pt = 0; pt < 4; pt++) {
            const int x = x0 + 16 * pt + n;
            if (x < Wout) {
#pragma unroll
                for (int ct = 0; ct < 4; ct++)
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const int co = 16 * ct + 4 * kg + i;
                        float v = acc[pt][ct][i] + bias[co];
                        if (relu && v < 0.0f) v = 0.0f;  // NaN propagates
                        out[(((size_t)b * MF_COUT + co) * Hout + y) * Wout + x].v = bf16_rne(v);
                    }
            }
        }
    }
}

// gw[co][ci][ky][kx] = sum_{b,y<Hout,x<Wout} in[b][ci][y+ky][x+kx] g[b][co][y][x]
// gb[co] = sum g[b][co][y][x] (written by the ci = 0 block).  One workgroup per (co, ci)
// and a fixed reduction tree: deterministic.
template <typename AI>
__global__ void __launch_bounds__(256) conv5_wgrad_kernel(const AI *__restrict__ in, const float *__restrict__ g,
                                                          float *__restrict__ gw, float *__restrict__ gb, int B,
                                                          int Cin, int Hin, int Win, int Cout, int Hout, int Wout) {
    const int co = blockIdx.x / Cin, ci = blockIdx.x % Cin;
    float acc[26];
#pragma unroll
    for (int k = 0; k < 26; k++) acc[k] = 0.0f;
    const size_t npx = (size_t)B * Hout * Wout;
    for (size_t p = threadIdx.x; p < npx; p += 256) {
        const int x = (int)(p % Wout);
        const int y = (int)((p / Wout) % Hout);
        const int b = (int)(p / ((size_t)Wout * Hout));
        const float gv = g[(((size_t)b * Cout + co) * Hout + y) * Wout + x];
        const size_t base = (((size_t)b * Cin + ci) * Hin + y) * Win + x;
#pragma unroll
        for (int ky = 0; ky < 5; ky++)
#pragma unroll
            for (int kx = 0; kx < 5; kx++) acc[ky * 5 + kx] = fmaf(ld_act(in, base + (size_t)ky * Win + kx), gv, acc[ky * 5 + kx]);
        acc[25] += gv;
    }
    __shared__ float red[256][27];
#pragma unroll
    for (int k = 0; k < 26; k++) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int k = 0; k < 26; k++) red[threadIdx.x][k] += red[threadIdx.x + h][k];
        }
        __syncthreads();
    }
    if (threadIdx.x < 25) gw[((size_t)co * Cin + ci) * 25 + threadIdx.x] = red[0][threadIdx.x];
    if (threadIdx.x == 25 && ci == 0 && gb) gb[co] = red[0][25];
}

// Weight gradient of a layer with Ci = Co = 16 NT real channels on the matrix cores:
// gw[co][ci][5 ky + kx] = sum_{b, y, x} g[b][co][y][x] in[b][ci][y + ky][x + kx] as 25 GEMMs
// (m = co, n = ci, k = output pixel), one v_mfma_f32_16x16x4_f32 per 16 co x 16 ci x 4 pixels:
// FP32 operands and accumulation, so the products and sums are those of the vector kernel
// above up to the order of the additions.  Operand layout of that instruction (lane l):
// A[m = l % 16][k = l / 16], B[k = l / 16][n = l % 16], D[m = 4 (l / 16) + i][n = l % 16], i < 4.
// Workgroup (b, ky): image b and kernel row ky; NT waves, wave w the output channels
// 16 w .. 16 w + 15 against all NT input-channel tiles and the 5 taps kx (5 NT accumulator tiles).
// Per segment of 64 pixels of an output row y the workgroup stages g[b][.][y][.] and
// in[b][.][y + ky][.] (with the 4-pixel halo) in LDS as FP32 [channel][x] (odd pitches; zero
// gradient beyond Wout), then runs its MFMAs over the segment's pixels.  The workgroups with ky = 0 also sum g per channel (bias).
// Partial sums go to part[b][ky][co][ci][kx] and part_b[b][co]; conv5_wgrad_reduce_kernel adds
// the images in a fixed order, so the result is deterministic.
typedef float f32x4v __attribute__((ext_vector_type(4)));

template <typename AI, int NT>
__global__ void __launch_bounds__(256) conv5_wgrad_mfma_kernel(const AI *__restrict__ in, const float *__restrict__ g,
                                                               float *__restrict__ part, float *__restrict__ part_b,
                                                               int Hin, int Win, int Hout, int Wout) {
    constexpr int C = 16 * NT;
    constexpr int XS = 64;               // pixels of a row segment
    constexpr int GP = XS + 1, IP = XS + 5;  // odd pitches
    __shared__ float gs[C * GP];         // g[b][c][y][x0 + x], x < XS
    __shared__ float is[C * IP];         // in[b][c][y + ky][x0 + x], x < XS + 4
    const int b = blockIdx.x / 5, ky = blockIdx.x % 5;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    f32x4v acc[NT][5];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int kx = 0; kx < 5; kx++) acc[t][kx] = f32x4v{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    const int m = lane & 15, kq = lane >> 4;
    for (int y = 0; y < Hout; y++) {
        for (int x0 = 0; x0 < Wout; x0 += XS) {
            const int seg = min(XS, (Wout - x0 + 3) & ~3);  // a multiple of 4; zero gradient beyond Wout
            __syncthreads();
            for (int idx = tid; idx < C * XS; idx += 64 * NT) {
                const int c = idx / XS, x = idx % XS, gx = x0 + x;
                gs[c * GP + x] = gx < Wout ? g[(((size_t)b * C + c) * Hout + y) * Wout + gx] : 0.0f;
            }
            for (int idx = tid; idx < C * (XS + 4); idx += 64 * NT) {
                const int c = idx / (XS + 4), x = idx % (XS + 4), gx = x0 + x;
                is[c * IP + x] = gx < Win ? ld_act(in, (((size_t)b * C + c) * Hin + y + ky) * Win + gx) : 0.0f;
            }
            __syncthreads();
            if (ky == 0 && tid < C)
                for (int x = 0; x < XS; x++) bsum += gs[tid * GP + x];
            for (int ks = 0; ks < seg / 4; ks++) {
                const float a = gs[(16 * wave + m) * GP + 4 * ks + kq];
#pragma unroll
                for (int t = 0; t < NT; t++)
#pragma unroll
                    for (int kx = 0; kx < 5; kx++) {
                        const float bv = is[(16 * t + m) * IP + 4 * ks + kq + kx];
                        acc[t][kx] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[t][kx], 0, 0, 0);
                    }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int kx = 0; kx < 5; kx++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int co = 16 * wave + 4 * kq + i, ci = 16 * t + m;
                part[((((size_t)b * 5 + ky) * C + co) * C + ci) * 5 + kx] = acc[t][kx][i];
            }
    if (ky == 0 && tid < C) part_b[(size_t)b * C + tid] = bsum;
}

// gw[co][ci][5 ky + kx] = sum_b part[b][ky][co][ci][kx], gb[co] = sum_b part_b[b][co], images in order.
__global__ void conv5_wgrad_reduce_kernel(const float *__restrict__ part, const float *__restrict__ part_b,
                                          float *__restrict__ gw, float *__restrict__ gb, int B, int C) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = C * C * 25;
    if (idx < n) {
        const int kx = idx % 5, ci = (idx / 5) % C, co = (idx / (5 * C)) % C, ky = idx / (5 * C * C);
        float s = 0.0f;
        for (int b = 0; b < B; b++) s += part[((((size_t)b * 5 + ky) * C + co) * C + ci) * 5 + kx];
        gw[((size_t)co * C + ci) * 25 + 5 * ky + kx] = s;
    } else if (idx < n + C && gb) {
        const int co = idx - n;
        float s = 0.0f;
        for (int b = 0; b < B; b++) s += part_b[(size_t)b * C + co];
        gb[co] = s;
    }
}

// g[i] *= (act[i] > 0): gradient through ReLU, from the stored post-activation.
template <typename A>
__global__ void relu_mask_kernel(float *g, const A *act, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(ld_act(act, i) > 0.0f)) g[i] = 0.0f;
}

// ---------------------------------------------------------------- complex <-> real weights

// Complex layer parameters: W[co][ci][25] as (re, im) pairs, then b[co] as (re, im).
// Real form: Wr[2co+a][2ci+c][25] with blocks [[re, -im], [im, re]], br[2co+a].
__global__ void expand_weights_kernel(const float *pc, float *wr, float *br, int cout, int cin) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * cin * 25;
    if (i < nw) {
        const int k = i % 25, ci = (i / 25) % cin, co = i / (25 * cin);
        const float re = pc[2 * i], im = pc[2 * i + 1];
        const int C2 = 2 * cin;
        wr[((size_t)(2 * co) * C2 + 2 * ci) * 25 + k] = re;
        wr[((size_t)(2 * co) * C2 + 2 * ci + 1) * 25 + k] = -im;
        wr[((size_t)(2 * co + 1) * C2 + 2 * ci) * 25 + k] = im;
        wr[((size_t)(2 * co + 1) * C2 + 2 * ci + 1) * 25 + k] = re;
    } else if (i < nw + cout) {
        const int co = i - nw;
        br[2 * co] = pc[2 * nw + 2 * co];
        br[2 * co + 1] = pc[2 * nw + 2 * co + 1];
    }
}

// wT[ci][co][24-k] = w[co][ci][k]: weights of the input-gradient convolution.
__global__ void flip_transpose_kernel(const float *w, float *wt, int cout, int cin) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cout * cin * 25) return;
    const int k = i % 25, ci = (i / 25) % cin, co = i / (25 * cin);
    wt[((size_t)ci * cout + co) * 25 + (24 - k)] = w[i];
}

// Wirtinger-pair gradient of the complex parameters from the real-form gradients:
// dL/dRe W = G[2co][2ci] + G[2co+1][2ci+1],  dL/dIm W = -G[2co][2ci+1] + G[2co+1][2ci].
__global__ void contract_grads_kernel(const float *gwr, const float *gbr, float *gc, int cout, int cin) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * cin * 25;
    const int C2 = 2 * cin;
    if (i < nw) {
        const int k = i % 25, ci = (i / 25) % cin, co = i / (25 * cin);
        const float g00 = gwr[((size_t)(2 * co) * C2 + 2 * ci) * 25 + k];
        const float g01 = gwr[((size_t)(2 * co) * C2 + 2 * ci + 1) * 25 + k];
        const float g10 = gwr[((size_t)(2 * co + 1) * C2 + 2 * ci) * 25 + k];
        const float g11 = gwr[((size_t)(2 * co + 1) * C2 + 2 * ci + 1) * 25 + k];
        gc[2 * i] = g00 + g11;
        gc[2 * i + 1] = g10 - g01;
    } else if (i < nw + cout) {
        const int co = i - nw;
        gc[2 * nw + 2 * co] = gbr[2 * co];
        gc[2 * nw + 2 * co + 1] = gbr[2 * co + 1];
    }
}

// ---------------------------------------------------------------- optimiser and loss

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// r weight of crop row y: the global radial index row0 + y (1/8 on the axis row).
__device__ __forceinline__ double rweight(int m) { return m == 0 ? 0.125 : (double)m; }

// Per sample b: num = sum w (pred - tgt)^2, den = sum w tgt^2 over 2 x H x W (FP64), one
// workgroup per sample, fixed tree.  out[2b] = num, out[2b+1] = den.
__global__ void __launch_bounds__(256) loss_reduce_kernel(const float *pred, const float *tgt, const int *row0, int H,
                                                          int W, double *out) {
    const int b = blockIdx.x;
    const size_t n = (size_t)2 * H * W;
    double num = 0.0, den = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 256) {
        const int y = (int)((i / W) % H);
        const double w = rweight(row0[b] + y);
        const double p = pred[b * n + i], t = tgt[b * n + i];
        num += w * (p - t) * (p - t);
        den += w * t * t;
    }
    __shared__ double sn[256], sd[256];
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sn[threadIdx.x] += sn[threadIdx.x + h];
            sd[threadIdx.x] += sd[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * b] = sn[0];
        out[2 * b + 1] = sd[0];
    }
}

// loss = (1/B) sum_b num_b / den_b; grad = dloss/dpred = 2 w (pred - tgt) / (B den_b)
__global__ void loss_grad_kernel(const float *pred, const float *tgt, const int *row0, int B, int H, int W,
                                 const double *nd, float *grad) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)2 * H * W;
    if (i >= n * B) return;
    const int b = (int)(i / n);
    const int y = (int)((i % n) / W) % H;
    const double den = nd[2 * b + 1] > 0.0 ? nd[2 * b + 1] : 1.0;
    grad[i] = (float)(2.0 * rweight(row0[b] + y) * ((double)pred[i] - (double)tgt[i]) / ((double)B * den));
}

// ---------------------------------------------------------------- fields <-> network tensors

// Network input for sample b: rows row0-8 .. row0+H+7 and columns col0-8 .. col0+W+7 of the
// complex field of its instance, scaled by in_scale: row -m reads row m (the field is even in
// r, dA/dr = 0 at the axis), rows >= nr read 0 (A = 0 at r_max), columns wrap (periodic t).
// out[b][0|1][H+16][W+16] (re, im planes).
template <typename A>
__global__ void net_input_kernel(const float2 *fields, const NetSample *smp, int nr, int nt, int H, int W, A *out) {
    const int Hp = H + 16, Wp = W + 16;
    const size_t per = (size_t)Hp * Wp;
    const int b = blockIdx.y;
    const NetSample s = smp[b];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (size_t)gridDim.x * blockDim.x) {
        const int yy = (int)(i / Wp), xx = (int)(i % Wp);
        int r = s.row0 - 8 + yy;
        if (r < 0) r = -r;
        int t = (s.col0 - 8 + xx) % nt;
        if (t < 0) t += nt;
        float2 v = make_float2(0.0f, 0.0f);
        if (r < nr) v = fields[s.field_off + (size_t)r * nt + t];
        st_act(out, ((size_t)b * 2 + 0) * per + i, v.x * s.in_scale);
        st_act(out, ((size_t)b * 2 + 1) * per + i, v.y * s.in_scale);
    }
}

// Training target for sample b: (fine - coarse) / out_scale on rows row0.., columns col0..,
// out[b][0|1][H][W].
__global__ void net_target_kernel(const float2 *fine, const float2 *coarse, const NetSample *smp, int nr, int nt,
                                  int H, int W, float *out) {
    const size_t per = (size_t)H * W;
    const int b = blockIdx.y;
    const NetSample s = smp[b];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i % W);
        const int r = s.row0 + y;
        int t = (s.col0 + x) % nt;
        if (t < 0) t += nt;
        float2 d = make_float2(0.0f, 0.0f);
        if (r >= 0 && r < nr) {
            const float2 f = fine[s.field_off + (size_t)r * nt + t];
            const float2 c = coarse[s.coarse_off + (size_t)r * nt + t];
            d = make_float2(f.x - c.x, f.y - c.y);
        }
        const float rs = 1.0f / s.out_scale;
        out[((size_t)b * 2 + 0) * per + i] = d.x * rs;
        out[((size_t)b * 2 + 1) * per + i] = d.y * rs;
    }
}

// Full-grid correction: dst[r][t] = base[r][t] + out_scale * (net re + i net im); the r_max row
// stays 0.  net[b][0|1][nr][nt] with sample b the whole grid of its instance.
__global__ void net_apply_kernel(const float *net, const float2 *base, const NetSample *smp, int nr, int nt,
                                 float2 *dst) {
    const size_t per = (size_t)nr * nt;
    const int b = blockIdx.y;
    const NetSample s = smp[b];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / nt);
        const float2 c = base[s.coarse_off + i];
        const float sc = s.out_scale;
        float2 o = make_float2(c.x + sc * net[((size_t)b * 2 + 0) * per + i], c.y + sc * net[((size_t)b * 2 + 1) * per + i]);
        if (r == nr - 1) o = make_float2(0.0f, 0.0f);
        dst[s.field_off + i] = o;
    }
}

// Parareal correction U_new = G_new + F_old - G_old on one window field (complex FP32), with
// per-workgroup FP64 partial sums of |U_new - U_prev|^2 and |U_new|^2 (r-weighted):
// part[2 * blockIdx.x] and part[2 * blockIdx.x + 1].
__global__ void __launch_bounds__(256) parareal_update_kernel(const float2 *g_new, const float2 *f_old,
                                                              const float2 *g_old, const float2 *u_prev,
                                                              float2 *u_new, int nr, int nt, double *part) {
    const size_t n = (size_t)nr * nt;
    double dn = 0.0, un = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float2 a = g_new[i], f = f_old[i], g = g_old[i];
        const float2 u = make_float2(a.x + (f.x - g.x), a.y + (f.y - g.y));
        const float2 q = u_prev[i];
        const double w = rweight((int)(i / nt));
        dn += w * ((double)(u.x - q.x) * (u.x - q.x) + (double)(u.y - q.y) * (u.y - q.y));
        un += w * ((double)u.x * u.x + (double)u.y * u.y);
        u_new[i] = u;
    }
    __shared__ double s1[256], s2[256];
    s1[threadIdx.x] = dn;
    s2[threadIdx.x] = un;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

// ---------------------------------------------------------------- launchers

template <typename AI, typename AO>
static hipError_t conv5_t(const AI *in, const float *w, const float *bias, AO *out, int B, int Cin, int Hin, int Win,
                          int Cout, int Hout, int Wout, int pad, int relu, hipStream_t s) {
    const dim3 block(256);
    if (Cout <= 2) {
        dim3 grid((Wout + CV_TW - 1) / CV_TW, (Hout + CV_TH - 1) / CV_TH, B * ((Cout + 1) / 2));
        hipLaunchKernelGGL((conv5_kernel<AI, AO, 2>), grid, block, 0, s, in, w, bias, out, Cin, Hin, Win, Cout, Hout,
                           Wout, pad, relu);
    } else {
        dim3 grid((Wout + CV_TW - 1) / CV_TW, (Hout + CV_TH - 1) / CV_TH, B * ((Cout + 15) / 16));
        hipLaunchKernelGGL((conv5_kernel<AI, AO, 16>), grid, block, 0, s, in, w, bias, out, Cin, Hin, Win, Cout, Hout,
                           Wout, pad, relu);
    }
    return hipGetLastError();
}

hipError_t launch_conv5(int act_bf16, int in_kind, int out_kind, const void *in, const float *w, const float *bias,
                        void *out, int B, int Cin, int Hin, int Win, int Cout, int Hout, int Wout, int pad, int relu,
                        hipStream_t s) {
    // kinds: 0 = FP32 tensor, 1 = tensor in the network's activation type
    if (act_bf16) {
        if (in_kind && out_kind)
            return conv5_t((const bf16_t *)in, w, bias, (bf16_t *)out, B, Cin, Hin, Win, Cout, Hout, Wout, pad, relu, s);
        if (in_kind && !out_kind)
            return conv5_t((const bf16_t *)in, w, bias, (float *)out, B, Cin, Hin, Win, Cout, Hout, Wout, pad, relu, s);
        if (!in_kind && out_kind)
            return conv5_t((const float *)in, w, bias, (bf16_t *)out, B, Cin, Hin, Win, Cout, Hout, Wout, pad, relu, s);
    }
    return conv5_t((const float *)in, w, bias, (float *)out, B, Cin, Hin, Win, Cout, Hout, Wout, pad, relu, s);
}

bool conv5_mfma_supported(int Cin, int Cout) { return Cout == MF_COUT && (Cin == 32 || Cin == 64); }

size_t conv5_mfma_weight_bytes(int Cin) { return (size_t)25 * (Cin / 32) * 4 * 64 * sizeof(uint4); }

hipError_t launch_pack_mfma_weights(const float *wr, void *wA, int Cin, hipStream_t s) {
    const int n = 25 * (Cin / 32) * 4 * 64;
    hipLaunchKernelGGL(pack_mfma_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, s, wr, (uint4 *)wA, Cin, Cin / 32);
    return hipGetLastError();
}

hipError_t launch_conv5_mfma(const void *in, const void *wA, const float *bias, void *out, int B, int Cin, int Hin,
                             int Win, int Hout, int Wout, int relu, hipStream_t s) {
    if (Hout != Hin - 4 || Wout != Win - 4) return hipErrorInvalidValue;
    const dim3 grid((Wout + MF_TW - 1) / MF_TW, (Hout + MF_TH - 1) / MF_TH, B);
    if (Cin == 64)
        hipLaunchKernelGGL(conv5_mfma_kernel<2>, grid, dim3(256), 0, s, (const bf16_t *)in, (const uint4 *)wA, bias,
                           (bf16_t *)out, Hin, Win, Hout, Wout, relu);
    else if (Cin == 32)
        hipLaunchKernelGGL(conv5_mfma_kernel<1>, grid, dim3(256), 0, s, (const bf16_t *)in, (const uint4 *)wA, bias,
                           (bf16_t *)out, Hin, Win, Hout, Wout, relu);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

size_t conv5_wgrad_part_floats(int B, int Cin, int Cout) {
    return Cin == Cout && Cin % 16 == 0 && Cin <= 64 ? (size_t)B * 25 * Cin * Cin + (size_t)B * Cin : 0;
}

template <typename AI, int NT>
static hipError_t launch_wgrad_mfma(const AI *in, const float *g, float *gw, float *gb, float *part, int B, int Hin,
                                    int Win, int Hout, int Wout, hipStream_t s) {
    constexpr int C = 16 * NT;
    float *part_b = part + (size_t)B * 25 * C * C;
    hipLaunchKernelGGL((conv5_wgrad_mfma_kernel<AI, NT>), dim3(B * 5), dim3(64 * NT), 0, s, in, g, part, part_b, Hin,
                       Win, Hout, Wout);
    const int n = C * C * 25 + C;
    hipLaunchKernelGGL(conv5_wgrad_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, s, part, part_b, gw, gb, B, C);
    return hipGetLastError();
}

hipError_t launch_conv5_wgrad(int act_bf16, const void *in, const float *g, float *gw, float *gb, float *part, int B,
                              int Cin, int Hin, int Win, int Cout, int Hout, int Wout, hipStream_t s) {
    // the matrix-core form when the partials buffer is there and the layer is square with a
    // multiple of 16 channels (the hidden layers)
    if (part && conv5_wgrad_part_floats(B, Cin, Cout)) {
        const int nt = Cin / 16;
        if (act_bf16) {
            const bf16_t *x = (const bf16_t *)in;
            if (nt == 1) return launch_wgrad_mfma<bf16_t, 1>(x, g, gw, gb, part, B, Hin, Win, Hout, Wout, s);
            if (nt == 2) return launch_wgrad_mfma<bf16_t, 2>(x, g, gw, gb, part, B, Hin, Win, Hout, Wout, s);
            if (nt == 3) return launch_wgrad_mfma<bf16_t, 3>(x, g, gw, gb, part, B, Hin, Win, Hout, Wout, s);
            return launch_wgrad_mfma<bf16_t, 4>(x, g, gw, gb, part, B, Hin, Win, Hout, Wout, s);
        }
        const float *x = (const float *)in;
        if (nt == 1) return launch_wgrad_mfma<float, 1>(x, g, gw, gb, part, B, Hin, Win, Hout, Wout, s);
        if (nt == 2) return launch_wgrad_mfma<float, 2>(x, g, gw, gb, part, B, Hin, Win, Hout, Wout, s);
        if (nt == 3) return launch_wgrad_mfma<float, 3>(x, g, gw, gb, part, B, Hin, Win, Hout, Wout, s);
        return launch_wgrad_mfma<float, 4>(x, g, gw, gb, part, B, Hin, Win, Hout, Wout, s);
    }
    if (act_bf16)
        hipLaunchKernelGGL(conv5_wgrad_kernel<bf16_t>, dim3(Cout * Cin), dim3(256), 0, s, (const bf16_t *)in, g, gw,
                           gb, B, Cin, Hin, Win, Cout, Hout, Wout);
    else
        hipLaunchKernelGGL(conv5_wgrad_kernel<float>, dim3(Cout * Cin), dim3(256), 0, s, (const float *)in, g, gw, gb,
                           B, Cin, Hin, Win, Cout, Hout, Wout);
    return hipGetLastError();
}

hipError_t launch_relu_mask(int act_bf16, float *g, const void *act, size_t n, hipStream_t s) {
    const int grid = (int)((n + 255) / 256);
    if (act_bf16)
        hipLaunchKernelGGL(relu_mask_kernel<bf16_t>, dim3(grid), dim3(256), 0, s, g, (const bf16_t *)act, n);
    else
        hipLaunchKernelGGL(relu_mask_kernel<float>, dim3(grid), dim3(256), 0, s, g, (const float *)act, n);
    return hipGetLastError();
}

hipError_t launch_expand_weights(const float *pc, float *wr, float *br, int cout, int cin, hipStream_t s) {
    const int n = cout * cin * 25 + cout;
    hipLaunchKernelGGL(expand_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, s, pc, wr, br, cout, cin);
    return hipGetLastError();
}

hipError_t launch_flip_transpose(const float *w, float *wt, int cout, int cin, hipStream_t s) {
    const int n = cout * cin * 25;
    hipLaunchKernelGGL(flip_transpose_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, wt, cout, cin);
    return hipGetLastError();
}

hipError_t launch_contract_grads(const float *gwr, const float *gbr, float *gc, int cout, int cin, hipStream_t s) {
    const int n = cout * cin * 25 + cout;
    hipLaunchKernelGGL(contract_grads_kernel, dim3((n + 255) / 256), dim3(256), 0, s, gwr, gbr, gc, cout, cin);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_loss(const float *pred, const float *tgt, const int *row0, int B, int H, int W, double *nd,
                       float *grad, hipStream_t s) {
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(B), dim3(256), 0, s, pred, tgt, row0, H, W, nd);
    const size_t n = (size_t)B * 2 * H * W;
    if (grad)
        hipLaunchKernelGGL(loss_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pred, tgt, row0, B, H,
                           W, (const double *)nd, grad);
    return hipGetLastError();
}

hipError_t launch_net_input(int act_bf16, const float2 *fields, const NetSample *smp, int B, int nr, int nt, int H,
                            int W, void *out, hipStream_t s) {
    const size_t per = (size_t)(H + 16) * (W + 16);
    dim3 grid((unsigned)std::min<size_t>((per + 255) / 256, 4096), B);
    if (act_bf16)
        hipLaunchKernelGGL(net_input_kernel<bf16_t>, grid, dim3(256), 0, s, fields, smp, nr, nt, H, W, (bf16_t *)out);
    else
        hipLaunchKernelGGL(net_input_kernel<float>, grid, dim3(256), 0, s, fields, smp, nr, nt, H, W, (float *)out);
    return hipGetLastError();
}

hipError_t launch_net_target(const float2 *fine, const float2 *coarse, const NetSample *smp, int B, int nr, int nt,
                             int H, int W, float *out, hipStream_t s) {
    const size_t per = (size_t)H * W;
    dim3 grid((unsigned)std::min<size_t>((per + 255) / 256, 4096), B);
    hipLaunchKernelGGL(net_target_kernel, grid, dim3(256), 0, s, fine, coarse, smp, nr, nt, H, W, out);
    return hipGetLastError();
}

hipError_t launch_net_apply(const float *net, const float2 *base, const NetSample *smp, int B, int nr, int nt,
                            float2 *dst, hipStream_t s) {
    const size_t per = (size_t)nr * nt;
    dim3 grid((unsigned)std::min<size_t>((per + 255) / 256, 4096), B);
    hipLaunchKernelGGL(net_apply_kernel, grid, dim3(256), 0, s, net, base, smp, nr, nt, dst);
    return hipGetLastError();
}

hipError_t launch_parareal_update(const float2 *g_new, const float2 *f_old, const float2 *g_old, const float2 *u_prev,
                                  float2 *u_new, int nr, int nt, double *part, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(parareal_update_kernel, dim3(nblocks), dim3(256), 0, s, g_new, f_old, g_old, u_prev, u_new, nr,
                       nt, part);
    return hipGetLastError();
}

}  // namespace fcn
