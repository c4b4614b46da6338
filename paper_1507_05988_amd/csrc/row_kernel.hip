// row_kernel.hip -- the row pass of the FCN z-step on gfx950.
//
// One workgroup holds one r-row (or several rows when nt is small) of nt complex values
// in LDS and runs, per row and in this order (the re-organised three-part step of Sec. 4,
// whose third part of step n and first part of step n+1 are the same rows):
//   inverse FFT of the spectrum (Eq. antifourier), scaled by 1/nt
//   -> nonlinear half step with dz_{n-1} (Eq. Anhalf1)           = A^n
//   -> diagnostics of A^n (energy, fluence, peak I, peak rho, peak phase rate)
//   -> nonlinear half step with dz_n (Eq. Anhalf)
//   -> forward FFT (first loop of Sec. 3.1), spectrum written back in place.
// Each row is read once and written once from HBM.
//
// Nonlinear half step (Sec. 3.2): intensities I_p = |A_p|^2 are taken before the update;
// the electron density follows d rho/dt = sigma_K I^K (rho_at - rho) (Eq. ionization with
// sigma_K rho_at = beta^(K)/(K hbar w0)) from rho = 0 at t_min, one classical RK4 step per
// grid interval with the mid-interval intensity (I_p + I_{p+1})/2.  One RK4 step of this
// linear equation is the affine map rho -> (1 - S_p) rho + S_p rho_at with S_p written out
// below, so the density along the row is an exclusive scan of affine maps: each thread
// composes the maps of its E contiguous points, the workgroup scans the compositions in
// FP64 with wavefront shuffles, then each thread replays its points.  The update is
// A <- A exp(h Re N) (cos(h Im N) + i sin(h Im N)) with N of Eq. nonlinearpart.
// Intensity, density, N and the diagnostics are FP64 in both precisions; the FP32 path
// rounds h Re N and h Im N to FP32 before expf/sincosf.
#include "fcn_internal.h"
#include "fft.hpp"

namespace fcn {

__device__ __forceinline__ double ipow(double x, int k) {
    double r = 1.0;
    while (k > 0) {
        if (k & 1) r *= x;
        x *= x;
        k >>= 1;
    }
    return r;
}

template <typename R>
__device__ __forceinline__ c2<R> nl_rotate(c2<R> a, double decay, double phase);
template <>
__device__ __forceinline__ c2<float> nl_rotate<float>(c2<float> a, double decay, double phase) {
    const float e = expf((float)decay);
    float s, c;
    sincosf((float)phase, &s, &c);
    return cmul<float>(a, mk<float>(e * c, e * s));
}
template <>
__device__ __forceinline__ c2<double> nl_rotate<double>(c2<double> a, double decay, double phase) {
    const double e = exp(decay);
    double s, c;
    sincos(phase, &s, &c);
    return cmul<double>(a, mk<double>(e * c, e * s));
}

struct DiagAcc {
    double sum, imax, rmax, phimax;
};

// Shuffle helpers within a segment of W lanes (W a power of two <= 64).
template <int W>
__device__ __forceinline__ double seg_up(double v, int d) {
    return __shfl_up(v, d, W);
}
template <int W>
__device__ __forceinline__ double seg_xor(double v, int d) {
    return __shfl_xor(v, d, W);
}

// Workgroup-shared scratch of the row kernel beyond the row buffers.
struct RowScratch {
    double scan_a[16], scan_b[16];  // per-wave inclusive composition (cross-wave scan)
    double diag[16][4];             // per-wave diagnostics partials
};

// Exclusive scan over the T threads of a row of the affine maps (a, b): x -> a x + b,
// earlier threads applied first.  Returns b of the exclusive prefix (the density at the
// thread's first point, the row starting from rho = 0).  All threads must call it.
template <int T>
__device__ __forceinline__ double row_exclusive_scan(double a, double b, int tr, RowScratch &sh) {
    constexpr int W = T < 64 ? T : 64;
    const int lane = tr & (W - 1);
    // inclusive within the segment
#pragma unroll
    for (int d = 1; d < W; d <<= 1) {
        const double pa = seg_up<W>(a, d);
        const double pb = seg_up<W>(b, d);
        if (lane >= d) {
            b = a * pb + b;
            a = a * pa;
        }
    }
    double pre_a = 1.0, pre_b = 0.0;  // composition of the earlier waves of this row
    if constexpr (T > 64) {
        const int wave = threadIdx.x >> 6;
        const int first_wave = wave - (tr >> 6);
        if (lane == 63) {
            sh.scan_a[wave] = a;
            sh.scan_b[wave] = b;
        }
        __syncthreads();
        for (int w = first_wave; w < wave; w++) {
            pre_b = sh.scan_a[w] * pre_b + sh.scan_b[w];
            pre_a = sh.scan_a[w] * pre_a;
        }
        __syncthreads();
        b = a * pre_b + b;
        a = a * pre_a;
    }
    // exclusive: inclusive of the previous thread
    double eb = seg_up<W>(b, 1);
    if (lane == 0) eb = pre_b;  // first lane of a wave: prefix of earlier waves (0 for tr = 0)
    return eb;
}

// Sum / max reductions over the T threads of a row; result valid in every thread.
template <int T>
__device__ __forceinline__ DiagAcc row_reduce(DiagAcc v, int tr, RowScratch &sh) {
    constexpr int W = T < 64 ? T : 64;
#pragma unroll
    for (int d = W / 2; d >= 1; d >>= 1) {
        v.sum += seg_xor<W>(v.sum, d);
        v.imax = fmax(v.imax, seg_xor<W>(v.imax, d));
        v.rmax = fmax(v.rmax, seg_xor<W>(v.rmax, d));
        v.phimax = fmax(v.phimax, seg_xor<W>(v.phimax, d));
    }
    if constexpr (T > 64) {
        const int wave = threadIdx.x >> 6;
        const int first_wave = wave - (tr >> 6);
        if ((tr & 63) == 0) {
            sh.diag[wave][0] = v.sum;
            sh.diag[wave][1] = v.imax;
            sh.diag[wave][2] = v.rmax;
            sh.diag[wave][3] = v.phimax;
        }
        __syncthreads();
        DiagAcc t{0.0, 0.0, 0.0, 0.0};
        for (int w = first_wave; w < first_wave + T / 64; w++) {
            t.sum += sh.diag[w][0];
            t.imax = fmax(t.imax, sh.diag[w][1]);
            t.rmax = fmax(t.rmax, sh.diag[w][2]);
            t.phimax = fmax(t.phimax, sh.diag[w][3]);
        }
        __syncthreads();
        v = t;
    }
    return v;
}

// One nonlinear sub-step on the E contiguous points c[] (positions tr*E + k) of a row.
// i_next: intensity of the point after the chunk (pre-update; unused by the last thread).
// h: exponent length (dz/2).  APPLY: update c; DIAG: accumulate diagnostics into acc.
// scan: workgroup-uniform switch for the density scan (it holds barriers when T > 64);
// rows whose instance has no density term run it with S = 0, which keeps rho = 0.
template <typename R, int T, int E>
__device__ __forceinline__ void nl_sub_step(c2<R> (&c)[E], const DevInst &in, double i_next, double h, bool apply,
                                            bool diag, bool scan, DiagAcc &acc, int tr, RowScratch &sh) {
    double inten[E];
#pragma unroll
    for (int k = 0; k < E; k++) inten[k] = (double)c[k].x * (double)c[k].x + (double)c[k].y * (double)c[k].y;

    double rho[E];
    const bool need_rho = in.need_rho != 0.0;
    if (scan) {
        const double dt = in.dtau, sk = in.sigma_K, ra = in.rho_at;
        const int K = in.K;
        double S[E];
        double ca = 1.0, cb = 0.0;
        double g0 = sk * ipow(inten[0], K);
#pragma unroll
        for (int k = 0; k < E; k++) {
            const double i1 = (k + 1 < E) ? inten[k + 1] : i_next;
            const double g1 = sk * ipow(i1, K);
            const double gh = sk * ipow(0.5 * (inten[k] + i1), K);
            // classical RK4 step of d rho/dt = g(t)(rho_at - rho) over dt:
            // rho' = rho + S (rho_at - rho)
            const double a0 = dt * g0, ah = dt * gh, a1 = dt * g1;
            const double u2 = 1.0 - 0.5 * a0;
            const double u3 = 1.0 - 0.5 * ah * u2;
            const double u4 = 1.0 - ah * u3;
            const double s = (a0 + 2.0 * ah * u2 + 2.0 * ah * u3 + a1 * u4) * (1.0 / 6.0);
            S[k] = need_rho ? s : 0.0;
            // compose this step after the chunk's earlier steps
            cb = (1.0 - S[k]) * cb + S[k] * ra;
            ca = (1.0 - S[k]) * ca;
            g0 = g1;
        }
        double r = row_exclusive_scan<T>(ca, cb, tr, sh);
#pragma unroll
        for (int k = 0; k < E; k++) {
            rho[k] = r;
            r = (1.0 - S[k]) * r + S[k] * ra;
        }
    } else {
#pragma unroll
        for (int k = 0; k < E; k++) rho[k] = 0.0;
    }

#pragma unroll
    for (int k = 0; k < E; k++) {
        const double I = inten[k];
        const double kerr = I * (in.ck1 + I * (in.ck2 + I * (in.ck3 + I * in.ck4)));
        const double im_n = kerr + in.c_plasma * rho[k];
        if (diag) {
            acc.sum += I;
            acc.imax = fmax(acc.imax, I);
            acc.rmax = fmax(acc.rmax, rho[k]);
            acc.phimax = fmax(acc.phimax, in.phi_kerr * fabs(kerr) + in.phi_plasma * rho[k]);
        }
        if (apply) {
            const double re_n = in.c_mpa * ipow(I, in.K - 1) + in.c_coll * rho[k];
            c[k] = nl_rotate<R>(c[k], h * re_n, h * im_n);
        }
    }
}

__device__ __forceinline__ double dz_rule(double phi, double max_phase, double dz_min, double dz_max) {
    double dz = phi > 0.0 ? max_phase / phi : dz_max;
    return fmin(fmax(dz, dz_min), dz_max);
}

__host__ __device__ constexpr int row_threads(int nt, int e) {
    return (nt / e) >= 256 ? nt / e : 256;
}

template <typename R, int NT, int E, int FLAGS>
struct RowCfg {
    static constexpr int T = NT / E;
    static constexpr int RPW = T >= 256 ? 1 : 256 / T;
    static constexpr int THREADS = T * RPW;
    static constexpr int LROW = NT + NT / 32;
};

template <typename R, int NT, int E, int FLAGS>
__global__ void __launch_bounds__(row_threads(NT, E)) row_kernel(RowArgs a) {
    using Cfg = RowCfg<R, NT, E, FLAGS>;
    constexpr int T = Cfg::T;
    constexpr int RPW = Cfg::RPW;
    constexpr bool BOOK = (FLAGS & RK_STAGE_LEN) == 0 && (FLAGS & (RK_NL_A | RK_NL_B | RK_DIAG)) != 0;
    constexpr bool NEED_CHUNK = (FLAGS & (RK_NL_A | RK_NL_B | RK_DIAG)) != 0;
    __shared__ c2<R> lds[RPW * Cfg::LROW];
    __shared__ RowScratch sh;

    const int tid = threadIdx.x;
    const int tr = tid % T;
    const int rw = tid / T;
    const int item_idx = blockIdx.x * RPW + rw;
    const bool active = item_idx < a.nitems;
    const RowItem it = a.items[active ? item_idx : 0];
    const DevInst in = a.inst[it.inst];
    c2<R> *row_lds = lds + rw * Cfg::LROW;
    c2<R> *g = reinterpret_cast<c2<R> *>(a.field) + in.field_off + (int64_t)it.m * NT;
    const c2<R> *tw = reinterpret_cast<const c2<R> *>(a.twiddle) + in.tw_off;

    int64_t n = 0;
    double dz_a = 0.0, dz_b = 0.0;
    if constexpr (BOOK) {
        n = a.state->cnt_row;
        if constexpr ((FLAGS & RK_NL_A) != 0) dz_a = a.dz_ring[((n - 1) & 1) * a.batch + it.inst];
        if constexpr ((FLAGS & RK_NL_B) != 0) {
            if (a.dz_mode == DZ_ADAPTIVE) {
                const double phi = __longlong_as_double((long long)a.phi_slot[((n - 1) & 1) * a.batch + it.inst]);
                dz_b = dz_rule(phi, a.max_phase, a.dz_min, a.dz_max);
            } else if (a.dz_mode == DZ_REPLAY) {
                dz_b = a.dz_log[(n - a.log_base) * a.batch + it.inst];
            } else {
                dz_b = in.dz_fixed;
            }
        }
    }
    if constexpr ((FLAGS & RK_STAGE_LEN) != 0) dz_b = 2.0 * a.stage_len;

    c2<R> v[E];
#pragma unroll
    for (int k = 0; k < E; k++) v[k] = active ? g[tr + k * T] : czero<R>();

    if constexpr ((FLAGS & RK_IFFT_IN) != 0) {
        row_fft<R, NT, E, +1>(v, row_lds, tr, tw);
        const R sc = R(1.0 / NT);
#pragma unroll
        for (int k = 0; k < E; k++) v[k] = cscale<R>(v[k], sc);
    }

    if constexpr (NEED_CHUNK) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < E; k++) row_lds[lpad(tr + k * T)] = v[k];
        __syncthreads();
        c2<R> c[E];
#pragma unroll
        for (int k = 0; k < E; k++) c[k] = row_lds[lpad(tr * E + k)];
        DiagAcc acc{0.0, 0.0, 0.0, 0.0};
        const bool scan = __syncthreads_or(active && in.need_rho != 0.0) != 0;

        if constexpr ((FLAGS & RK_NL_A) != 0) {
            c2<R> nx = row_lds[lpad(tr < T - 1 ? tr * E + E : 0)];
            const double i_next = (double)nx.x * (double)nx.x + (double)nx.y * (double)nx.y;
            nl_sub_step<R, T, E>(c, in, i_next, 0.5 * dz_a, true, false, scan, acc, tr, sh);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < E; k++) row_lds[lpad(tr * E + k)] = c[k];
            __syncthreads();
        }
        if constexpr ((FLAGS & (RK_NL_B | RK_DIAG)) != 0) {
            c2<R> nx = row_lds[lpad(tr < T - 1 ? tr * E + E : 0)];
            const double i_next = (double)nx.x * (double)nx.x + (double)nx.y * (double)nx.y;
            nl_sub_step<R, T, E>(c, in, i_next, 0.5 * dz_b, (FLAGS & RK_NL_B) != 0, (FLAGS & RK_DIAG) != 0, scan, acc,
                                 tr, sh);
        }
        if constexpr ((FLAGS & RK_DIAG) != 0) {
            acc = row_reduce<T>(acc, tr, sh);
            if (active && tr == 0) {
                double *rd = a.row_diag + 4 * (int64_t)(in.row_base + it.m);
                rd[0] = acc.sum;
                rd[1] = acc.imax;
                rd[2] = acc.rmax;
                rd[3] = acc.phimax;
                if (!(acc.sum <= 1.0e300)) atomicOr(&a.state->nonfinite, 1);  // NaN or overflow
                if constexpr (BOOK) {
                    atomicMax(&a.phi_slot[(n & 1) * a.batch + it.inst],
                              (unsigned long long)__double_as_longlong(acc.phimax));
                    if (a.seed_slots)
                        atomicMax(&a.phi_slot[((n - 1) & 1) * a.batch + it.inst],
                                  (unsigned long long)__double_as_longlong(acc.phimax));
                }
            }
        }
        if constexpr ((FLAGS & RK_STORE) != 0) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < E; k++) row_lds[lpad(tr * E + k)] = c[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < E; k++) v[k] = row_lds[lpad(tr + k * T)];
        }
    }

    if constexpr ((FLAGS & RK_FFT_OUT) != 0) row_fft<R, NT, E, -1>(v, row_lds, tr, tw);

    if constexpr ((FLAGS & RK_STORE) != 0) {
        if (active) {
#pragma unroll
            for (int k = 0; k < E; k++) g[tr + k * T] = v[k];
        }
    }

    if constexpr (BOOK) {
        // step bookkeeping, once per instance (by the workgroup holding row 0)
        if (active && it.m == 0 && tr == 0) {
            if constexpr ((FLAGS & RK_NL_B) != 0) {
                a.dz_ring[(n & 1) * a.batch + it.inst] = dz_b;
                if (a.dz_mode == DZ_ADAPTIVE && a.dz_log != nullptr)
                    a.dz_log[(n - a.log_base) * a.batch + it.inst] = dz_b;
            }
        }
        if (blockIdx.x == 0 && tid == 0) a.state->cnt_col = n;
    }
}

// ------------------------------------------------------------------ launch table

template <typename R, int NT, int FLAGS>
static hipError_t launch_row_t(const RowArgs &a, int grid, hipStream_t s) {
    constexpr int E = 8;
    using Cfg = RowCfg<R, NT, E, FLAGS>;
    hipLaunchKernelGGL((row_kernel<R, NT, E, FLAGS>), dim3(grid), dim3(Cfg::THREADS), 0, s, a);
    return hipGetLastError();
}

template <typename R, int FLAGS>
static hipError_t launch_row_nt(int nt, const RowArgs &a, int grid, hipStream_t s) {
    switch (nt) {
        case 64: return launch_row_t<R, 64, FLAGS>(a, grid, s);
        case 128: return launch_row_t<R, 128, FLAGS>(a, grid, s);
        case 256: return launch_row_t<R, 256, FLAGS>(a, grid, s);
        case 512: return launch_row_t<R, 512, FLAGS>(a, grid, s);
        case 1024: return launch_row_t<R, 1024, FLAGS>(a, grid, s);
        case 2048: return launch_row_t<R, 2048, FLAGS>(a, grid, s);
        case 4096: return launch_row_t<R, 4096, FLAGS>(a, grid, s);
        case 8192: return launch_row_t<R, 8192, FLAGS>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

// Flag combinations used by the runtime.
constexpr int RK_FIRST = RK_NL_B | RK_DIAG | RK_FFT_OUT | RK_STORE;
constexpr int RK_MIDDLE = RK_IFFT_IN | RK_NL_A | RK_DIAG | RK_NL_B | RK_FFT_OUT | RK_STORE;
constexpr int RK_LAST = RK_IFFT_IN | RK_NL_A | RK_DIAG | RK_STORE;
constexpr int RK_DIAG_ONLY = RK_DIAG;
constexpr int RK_T_FFT = RK_FFT_OUT | RK_STORE;
constexpr int RK_T_IFFT = RK_IFFT_IN | RK_STORE;
constexpr int RK_T_NL = RK_NL_B | RK_STORE | RK_STAGE_LEN;

template <typename R>
static hipError_t launch_row_p(int nt, int flags, const RowArgs &a, int grid, hipStream_t s) {
    switch (flags) {
        case RK_FIRST: return launch_row_nt<R, RK_FIRST>(nt, a, grid, s);
        case RK_MIDDLE: return launch_row_nt<R, RK_MIDDLE>(nt, a, grid, s);
        case RK_LAST: return launch_row_nt<R, RK_LAST>(nt, a, grid, s);
        case RK_DIAG_ONLY: return launch_row_nt<R, RK_DIAG_ONLY>(nt, a, grid, s);
        case RK_T_FFT: return launch_row_nt<R, RK_T_FFT>(nt, a, grid, s);
        case RK_T_IFFT: return launch_row_nt<R, RK_T_IFFT>(nt, a, grid, s);
        case RK_T_NL: return launch_row_nt<R, RK_T_NL>(nt, a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

int row_rows_per_group(int nt, int elems) {
    const int t = nt / elems;
    return t >= 256 ? 1 : 256 / t;
}

hipError_t launch_row(int precision, int nt, int elems, int flags, const RowArgs &a, int grid, hipStream_t s) {
    if (elems != 8) return hipErrorInvalidValue;
    return precision == 0 ? launch_row_p<double>(nt, flags, a, grid, s) : launch_row_p<float>(nt, flags, a, grid, s);
}

// ------------------------------------------------------------------ small kernels

// One workgroup per instance: reduces the per-row partials of the last row pass into a
// diagnostics record (layout in include/fcn.h).
__global__ void __launch_bounds__(256) finalize_kernel(const DevInst *insts, int batch, const double *row_diag,
                                                       const double *zpos, const double *dz_ring,
                                                       const DevState *state, double *out) {
    const int i = blockIdx.x;
    const DevInst in = insts[i];
    __shared__ double se[256], si[256], sr[256], sp[256];
    double e = 0.0, im = 0.0, rm = 0.0, pm = 0.0;
    double *rec = out + in.diag_off;
    for (int m = threadIdx.x; m < in.nr; m += blockDim.x) {
        const double *rd = row_diag + 4 * (int64_t)(in.row_base + m);
        const double w = m == 0 ? 0.125 : (double)m;
        e += w * rd[0];
        im = fmax(im, rd[1]);
        rm = fmax(rm, rd[2]);
        pm = fmax(pm, rd[3]);
        rec[DIAG_SCALARS + m] = in.dtau * rd[0];
    }
    se[threadIdx.x] = e;
    si[threadIdx.x] = im;
    sr[threadIdx.x] = rm;
    sp[threadIdx.x] = pm;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            se[threadIdx.x] += se[threadIdx.x + h];
            si[threadIdx.x] = fmax(si[threadIdx.x], si[threadIdx.x + h]);
            sr[threadIdx.x] = fmax(sr[threadIdx.x], sr[threadIdx.x + h]);
            sp[threadIdx.x] = fmax(sp[threadIdx.x], sp[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t n = state->cnt_row;
        rec[0] = 2.0 * 3.14159265358979323846 * in.dr * in.dr * in.dtau * se[0];
        rec[1] = si[0];
        rec[2] = row_diag[4 * (int64_t)in.row_base + 1];
        rec[3] = sr[0];
        rec[4] = sp[0];
        rec[5] = zpos[i];
        rec[6] = (double)n;
        rec[7] = n > 0 ? dz_ring[((n - 1) & 1) * batch + i] : 0.0;
    }
}

hipError_t launch_finalize(const DevInst *inst, int batch, const double *row_diag, const double *zpos,
                           const double *dz_ring, const DevState *state, double *out, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(batch), dim3(256), 0, s, inst, batch, row_diag, zpos, dz_ring, state,
                       out);
    return hipGetLastError();
}

// Resets the step state: counters to n0, phase slots, dz ring and z positions to zero.
__global__ void init_state_kernel(DevState *state, unsigned long long *phi_slot, double *dz_ring, double *zpos,
                                  int batch, int64_t n0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        state->cnt_col = n0;
        state->cnt_row = n0;
        state->nonfinite = 0;
    }
    if (i < 2 * batch) {
        phi_slot[i] = 0ull;
        dz_ring[i] = 0.0;
    }
    if (i < batch) zpos[i] = 0.0;
}

hipError_t launch_init_state(DevState *state, unsigned long long *phi_slot, double *dz_ring, double *zpos, int batch,
                             int64_t n0, hipStream_t s) {
    const int threads = 256;
    const int grid = (2 * batch + threads - 1) / threads;
    hipLaunchKernelGGL(init_state_kernel, dim3(grid), dim3(threads), 0, s, state, phi_slot, dz_ring, zpos, batch, n0);
    return hipGetLastError();
}

__global__ void clear_flag_kernel(DevState *state) { state->nonfinite = 0; }

hipError_t launch_clear_flag(DevState *state, hipStream_t s) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, state);
    return hipGetLastError();
}

}  // namespace fcn
