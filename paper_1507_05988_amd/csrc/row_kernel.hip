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
// FP64 (DPP lane moves inside a wavefront, LDS across wavefronts), then each thread replays
// its points.  The update is A <- A exp(h Re N) (cos(h Im N) + i sin(h Im N)) with N of
// Eq. nonlinearpart.  FP64 kernels compute everything in FP64.  FP32 kernels compute the
// intensity, the Kerr rate, the multiphoton term and the RK4 factors in FP32 on the scaled
// intensity u = I / I_ref (NlPoint<float>), compose, scan and replay the density in FP64,
// form h N in FP64 when a density term is on, and accumulate the diagnostics in FP64.
#include <hip/hip_ext.h>

#include <type_traits>

#include "fcn_internal.h"
#include "fft.hpp"

namespace fcn {

// x^k for 0 <= k < 32 by square-and-multiply over a fixed five bits (no data-dependent
// branches; k is uniform across the workgroup).
__device__ __forceinline__ double ipow(double x, int k) {
    double r = 1.0;
#pragma unroll
    for (int b = 0; b < 5; b++) {
        r = (k & (1 << b)) ? r * x : r;
        x *= x;
    }
    return r;
}

__device__ __forceinline__ float ipowf_(float x, int k) {
    float r = 1.0f;
#pragma unroll
    for (int b = 0; b < 5; b++) {
        r = (k & (1 << b)) ? r * x : r;
        x *= x;
    }
    return r;
}

// A exp(decay + i phase) written as A + A delta with
//   delta = expm1(decay) (cos phase + i sin phase) + (cos phase - 1) + i sin phase,
// with cos phase - 1 and expm1(decay) evaluated directly, so every small quantity keeps full
// relative precision.  Rounding exp(decay) and cos(phase) themselves next to 1 would bias |A|
// by up to half an ulp per update, the same way at every step (a systematic energy drift in
// FP32).
// sin(th) and cos(th) - 1 in FP32: Taylor series through th^9 and th^10 for |th| <= 0.4
// (truncation below 1.1e-12 of the value), the library functions beyond.  cos(th) - 1 comes
// from its own series, never from a rounded cos(th) next to 1.
__device__ __forceinline__ void sin_cosm1(float th, float *sn, float *cm1) {
    if (fabsf(th) <= 0.4f) {
        const float t2 = th * th;
        *sn = th * (1.0f + t2 * (-1.0f / 6.0f + t2 * (1.0f / 120.0f + t2 * (-1.0f / 5040.0f + t2 * (1.0f / 362880.0f)))));
        *cm1 = t2 * (-0.5f + t2 * (1.0f / 24.0f + t2 * (-1.0f / 720.0f + t2 * (1.0f / 40320.0f +
                                                                            t2 * (-1.0f / 3628800.0f)))));
    } else {
        float c;
        sincosf(th, sn, &c);
        *cm1 = c - 1.0f;
    }
}
// expm1 of |x| <= 0.1 through x^7 (truncation below 3e-12), the library function beyond.
__device__ __forceinline__ float expm1_small(float x) {
    if (fabsf(x) <= 0.1f)
        return x * (1.0f + x * (0.5f + x * (1.0f / 6.0f + x * (1.0f / 24.0f + x * (1.0f / 120.0f +
                                                                                   x * (1.0f / 720.0f +
                                                                                        x * (1.0f / 5040.0f)))))));
    return expm1f(x);
}

// A exp(decay + i phase) = A + A delta, delta = e (cos + i sin) + (cos - 1) + i sin, e = expm1(decay)
__device__ __forceinline__ c2<float> nl_rotate_f(c2<float> a, float decay, float phase) {
    const float em1 = expm1_small(decay);
    float sn, c1;
    sin_cosm1(phase, &sn, &c1);
    const float dr = em1 * (1.0f + c1) + c1;
    const float di = sn * (1.0f + em1);
    return mk<float>(a.x + (a.x * dr - a.y * di), a.y + (a.x * di + a.y * dr));
}
// A exp(i phase) = A + A ((cos - 1) + i sin): the pure phase rotation (no absorption term)
__device__ __forceinline__ c2<float> nl_phase_f(c2<float> a, float phase) {
    float sn, c1;
    sin_cosm1(phase, &sn, &c1);
    return mk<float>(a.x + (a.x * c1 - a.y * sn), a.y + (a.x * sn + a.y * c1));
}
// FP64: cos phase - 1 = -2 sin^2(phase/2), sin phase = 2 sin(phase/2) cos(phase/2)
__device__ __forceinline__ c2<double> nl_phase_d(c2<double> a, double phase) {
    double sh, ch;
    sincos(0.5 * phase, &sh, &ch);
    const double sn = 2.0 * sh * ch;
    const double c1 = -2.0 * sh * sh;
    return mk<double>(a.x + (a.x * c1 - a.y * sn), a.y + (a.x * sn + a.y * c1));
}
__device__ __forceinline__ c2<double> nl_rotate_d(c2<double> a, double decay, double phase) {
    const double em1 = expm1(decay);
    double sh, ch;
    sincos(0.5 * phase, &sh, &ch);
    const double sn = 2.0 * sh * ch;
    const double c1 = -2.0 * sh * sh;
    const double dr = em1 * (1.0 + c1) + c1;
    const double di = sn * (1.0 + em1);
    return mk<double>(a.x + (a.x * dr - a.y * di), a.y + (a.x * di + a.y * dr));
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

// Data-parallel-primitive (DPP) move of a double across the lanes of a wavefront: CTRL is a
// GFX9 DPP control (row_shr:n = 0x110 + n, row_bcast:15 = 0x142, row_bcast:31 = 0x143,
// wave_shr:1 = 0x138); lanes without a source, or outside ROW_MASK, get `old`.  A register
// move between lanes, where a shuffle is a round trip through the LDS crossbar.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double old, double v) {
    const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)x, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// One step of the inclusive scan: compose the map received from an earlier lane (pa, pb)
// before this lane's (a, b) when `take`.
__device__ __forceinline__ void scan_take(double &a, double &b, double pa, double pb, bool take) {
    if (take) {
        b = a * pb + b;
        a = a * pa;
    }
}

// Workgroup-shared scratch of the row kernel beyond the row buffers.
struct RowScratch {
    double scan_a[16], scan_b[16];  // per-wave inclusive composition (cross-wave scan)
    double diag[16][4];             // per-wave diagnostics partials
};

// Exclusive scan over the T threads of a row of the affine maps (a, b): x -> a x + b,
// earlier threads applied first.  Returns b of the exclusive prefix (the density at the
// thread's first point, the row starting from rho = 0); `incl` receives b of the inclusive
// prefix, which is bit for bit the value the next thread receives as its exclusive prefix.
// All threads must call it.
template <int T>
__device__ __forceinline__ double row_exclusive_scan(double a, double b, int tr, RowScratch &sh, double &incl) {
    constexpr int W = T < 64 ? T : 64;
    const int lane = tr & (W - 1);
    // inclusive within the segment
    if constexpr (W == 64) {
        // whole wavefronts: shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the last
        // lane of row 0 (2) into row 1 (3), then lane 31 into rows 2 and 3
        scan_take(a, b, dpp_move<0x111>(1.0, a), dpp_move<0x111>(0.0, b), (lane & 15) >= 1);
        scan_take(a, b, dpp_move<0x112>(1.0, a), dpp_move<0x112>(0.0, b), (lane & 15) >= 2);
        scan_take(a, b, dpp_move<0x114>(1.0, a), dpp_move<0x114>(0.0, b), (lane & 15) >= 4);
        scan_take(a, b, dpp_move<0x118>(1.0, a), dpp_move<0x118>(0.0, b), (lane & 15) >= 8);
        scan_take(a, b, dpp_move<0x142, 0xa>(1.0, a), dpp_move<0x142, 0xa>(0.0, b), (lane & 16) != 0);
        scan_take(a, b, dpp_move<0x143, 0xc>(1.0, a), dpp_move<0x143, 0xc>(0.0, b), lane >= 32);
    } else {
#pragma unroll
        for (int d = 1; d < W; d <<= 1) {
            const double pa = seg_up<W>(a, d);
            const double pb = seg_up<W>(b, d);
            scan_take(a, b, pa, pb, lane >= d);
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
    incl = b;
    // exclusive: inclusive of the previous thread; the first lane of a wave takes the prefix
    // of the earlier waves (0 for tr = 0)
    if constexpr (W == 64) {
        return dpp_move<0x138>(pre_b, b);
    } else {
        double eb = seg_up<W>(b, 1);
        if (lane == 0) eb = pre_b;
        return eb;
    }
}

// Sum / max reductions over the T threads of a row; result valid in every thread.
template <int T>
__device__ __forceinline__ DiagAcc row_reduce(DiagAcc v, int tr, RowScratch &sh) {
    constexpr int W = T < 64 ? T : 64;
    if constexpr (W == 64) {
        // whole wavefronts: the same DPP pattern as the scan accumulates the wavefront's
        // total in lane 63
        const int lane = tr & 63;
        auto take = [&](DiagAcc o, bool t) {
            if (t) {
                v.sum += o.sum;
                v.imax = fmax(v.imax, o.imax);
                v.rmax = fmax(v.rmax, o.rmax);
                v.phimax = fmax(v.phimax, o.phimax);
            }
        };
#define FCN_DIAG_MOVE(CTRL, RM) \
    DiagAcc{dpp_move<CTRL, RM>(0.0, v.sum), dpp_move<CTRL, RM>(0.0, v.imax), dpp_move<CTRL, RM>(0.0, v.rmax), \
            dpp_move<CTRL, RM>(0.0, v.phimax)}
        take(FCN_DIAG_MOVE(0x111, 0xf), (lane & 15) >= 1);
        take(FCN_DIAG_MOVE(0x112, 0xf), (lane & 15) >= 2);
        take(FCN_DIAG_MOVE(0x114, 0xf), (lane & 15) >= 4);
        take(FCN_DIAG_MOVE(0x118, 0xf), (lane & 15) >= 8);
        take(FCN_DIAG_MOVE(0x142, 0xa), (lane & 16) != 0);
        take(FCN_DIAG_MOVE(0x143, 0xc), lane >= 32);
#undef FCN_DIAG_MOVE
        if constexpr (T == 64) {  // one wavefront per row: every lane takes lane 63's total
            auto bcast = [](double x) {
                const long long b = __double_as_longlong(x);
                const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
                return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
            };
            v = DiagAcc{bcast(v.sum), bcast(v.imax), bcast(v.rmax), bcast(v.phimax)};
        }
    } else {
#pragma unroll
        for (int d = W / 2; d >= 1; d >>= 1) {
            v.sum += seg_xor<W>(v.sum, d);
            v.imax = fmax(v.imax, seg_xor<W>(v.imax, d));
            v.rmax = fmax(v.rmax, seg_xor<W>(v.rmax, d));
            v.phimax = fmax(v.phimax, seg_xor<W>(v.phimax, d));
        }
    }
    if constexpr (T > 64) {
        const int wave = threadIdx.x >> 6;
        const int first_wave = wave - (tr >> 6);
        if ((tr & 63) == 63) {  // the lane holding the wavefront's total
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

// Per-point pieces of the nonlinear operator N (Eq. nonlinearpart) in the kernel's
// arithmetic.  FP64 kernels evaluate everything in FP64.  FP32 kernels work on the scaled
// intensity u = I / I_ref (see DevInst): the Kerr rate, the multiphoton term and the RK4
// quantities dtau sigma_K I^K = u^K (exactly, with I_ref = (sigma_K dtau)^(-1/K)) are FP32 and
// cannot overflow; the density itself is always accumulated in FP64.
template <typename R>
struct NlPoint;

template <>
struct NlPoint<double> {
    double I, ik1;  // I and I^(K-1)
    __device__ __forceinline__ void load(c2<double> a, const DevInst &in, bool k1) {
        I = a.x * a.x + a.y * a.y;
        ik1 = k1 ? ipow(I, in.K - 1) : 0.0;
    }
    __device__ __forceinline__ double intensity() const { return I; }
    __device__ __forceinline__ double dt_g(const DevInst &in) const { return in.dtau * in.sigma_K * ik1 * I; }
    static __device__ __forceinline__ double dt_g_of(double Imid, const DevInst &in) {
        return in.dtau * in.sigma_K * ipow(Imid, in.K);
    }
    // avalanche rate times dtau, dtau (sigma_c / U_i) I
    __device__ __forceinline__ double dt_a(const DevInst &in) const { return in.dtau * in.c_aval * I; }
    static __device__ __forceinline__ double dt_a_of(double Imid, const DevInst &in) {
        return in.dtau * in.c_aval * Imid;
    }
    __device__ __forceinline__ double mid_arg(const NlPoint &o) const { return 0.5 * (I + o.I); }
    __device__ __forceinline__ double kerr(const DevInst &in) const {
        return I * (in.ck1 + I * (in.ck2 + I * (in.ck3 + I * in.ck4)));
    }
    __device__ __forceinline__ c2<double> apply(c2<double> a, const DevInst &in, double h, double rho) const {
        const double im_n = kerr(in) + in.c_plasma * rho;
        const double re_n = in.c_mpa * ik1 + in.c_coll * rho;
        return nl_rotate_d(a, h * re_n, h * im_n);
    }
    // N = i Kerr rate only (no absorption or density term in the launch)
    __device__ __forceinline__ c2<double> apply_phase(c2<double> a, const DevInst &in, double h) const {
        return nl_phase_d(a, h * kerr(in));
    }
};

template <>
struct NlPoint<float> {
    float ii, u, uk1;  // I, I/I_ref, (I/I_ref)^(K-1)
    __device__ __forceinline__ void load(c2<float> a, const DevInst &in, bool k1) {
        ii = a.x * a.x + a.y * a.y;
        u = ii * in.f_inv_iref;
        uk1 = k1 ? ipowf_(u, in.K - 1) : 0.0f;
    }
    __device__ __forceinline__ double intensity() const { return (double)ii; }
    __device__ __forceinline__ float dt_g(const DevInst &) const { return uk1 * u; }
    static __device__ __forceinline__ float dt_g_of(float umid, const DevInst &in) { return ipowf_(umid, in.K); }
    __device__ __forceinline__ float dt_a(const DevInst &in) const { return in.f_aval * u; }
    static __device__ __forceinline__ float dt_a_of(float umid, const DevInst &in) { return in.f_aval * umid; }
    __device__ __forceinline__ float mid_arg(const NlPoint &o) const { return 0.5f * (u + o.u); }
    __device__ __forceinline__ float kerr_f(const DevInst &in) const {
        return u * (in.fk1 + u * (in.fk2 + u * (in.fk3 + u * in.fk4)));
    }
    __device__ __forceinline__ double kerr(const DevInst &in) const { return (double)kerr_f(in); }
    __device__ __forceinline__ c2<float> apply(c2<float> a, const DevInst &in, float h, double rho,
                                               bool with_rho) const {
        const float kr = kerr_f(in);
        if (!with_rho) return nl_rotate_f(a, h * (in.f_mpa * uk1), h * kr);
        const double im_n = (double)kr + in.c_plasma * rho;
        const double re_n = (double)(in.f_mpa * uk1) + in.c_coll * rho;
        return nl_rotate_f(a, (float)((double)h * re_n), (float)((double)h * im_n));
    }
    __device__ __forceinline__ c2<float> apply(c2<float> a, const DevInst &in, float h, double rho) const {
        return apply(a, in, h, rho, true);
    }
    __device__ __forceinline__ c2<float> apply_phase(c2<float> a, const DevInst &in, float h) const {
        return nl_phase_f(a, h * kerr_f(in));
    }
};

// One nonlinear sub-step A <- A exp(h N) on the E points c[] of a thread.
//  scan = true: c[] holds the contiguous points tr*E + k of the row and nx the point after
//    the chunk (pre-update; for the last thread any value, it only feeds the unused last
//    interval).  The density follows from the RK4 affine maps scanned over the row.  With
//    upd_next, nx is also advanced, with the density its own thread uses, so the next
//    sub-step has its neighbour intensity without another LDS exchange.
//  scan = false (no density term in the workgroup): pointwise, any layout, nx unused.
// The exact density step has S = 1 - exp(-int g dt) in [0, 1); an RK4 factor S outside [0, 1]
// (a non-negative rate with sigma_K I^K dtau beyond the method's stability limit, 2.785 at
// constant rate) sets *unstable: the density then leaves [0, rho_at] and runs away.
// NOABS (launches whose instances have neither a density nor an absorption term, scan false):
// N = i Kerr rate, a pure phase rotation.
// AVAL (scan true, some instance with the avalanche rate): the density equation
// d rho/dt = g (rho_at - rho) + a rho, g = sigma_K I^K, a = (sigma_c/U_i) I, is linear with
// coefficients d = a - g and source g rho_at; one RK4 step is rho -> (1 - P) rho + Q rho_at with
// P = -(D0 + 2 Dh v2 + 2 Dh v3 + D1 v4)/6, v2 = 1 + D0/2, v3 = 1 + Dh v2/2, v4 = 1 + Dh v3, and
// Q = (G0 + 2 w2 + 2 w3 + w4)/6, w2 = Gh + Dh G0/2, w3 = Gh + Dh w2/2, w4 = G1 + D1 w3, in units of
// dtau (D = (a - g) dtau, G = g dtau at the interval's start, middle and end); without the
// avalanche P = Q = S.  An RK4 factor 1 - P < 0 or Q < 0 (the exact ones are positive) sets
// *unstable.
// Must be called by every thread of the workgroup (the scan holds barriers when T > 64).
template <typename R, int T, int E, bool NOABS, bool AVAL>
__device__ __forceinline__ void nl_sub_step(c2<R> (&c)[E], c2<R> &nx, const DevInst &in, R h, bool apply,
                                            bool diag, bool scan, bool upd_next, DiagAcc &acc, int tr,
                                            RowScratch &sh, int32_t *unstable) {
    using S_t = decltype(NlPoint<R>{}.dt_g(in));
    constexpr bool F32 = std::is_same<R, float>::value;
    const bool k1 = !NOABS && in.need_ik1 != 0.0;
    NlPoint<R> pt[E];
#pragma unroll
    for (int k = 0; k < E; k++) pt[k].load(c[k], in, k1);

    double rho[E];
    double rho_end = 0.0;
    NlPoint<R> pn;
    if (scan) {
        pn.load(nx, in, k1);
        const bool need_rho = in.need_rho != 0.0;
        const double ra = in.rho_at;
        S_t S[E];             // P (= Q without the avalanche)
        S_t Qv[AVAL ? E : 1];  // Q with the avalanche
        double ca = 1.0, cb = 0.0;
        S_t a0 = pt[0].dt_g(in);
        bool bad = false;
#pragma unroll
        for (int k = 0; k < E; k++) {
            const NlPoint<R> &p1 = (k + 1 < E) ? pt[k + 1] : pn;
            const S_t a1 = p1.dt_g(in);
            const S_t ah = NlPoint<R>::dt_g_of(pt[k].mid_arg(p1), in);
            const S_t one = S_t(1), half = S_t(0.5);
            // the row's last interval (last thread, last point) wraps to t_min and is never used
            const bool used = k + 1 < E || tr + 1 < T;
            if constexpr (AVAL) {
                const S_t d0 = pt[k].dt_a(in) - a0;
                const S_t dh = NlPoint<R>::dt_a_of(pt[k].mid_arg(p1), in) - ah;
                const S_t d1 = p1.dt_a(in) - a1;
                const S_t v2 = one + half * d0;
                const S_t v3 = one + half * dh * v2;
                const S_t v4 = one + dh * v3;
                const S_t pv = -(d0 + S_t(2) * dh * v2 + S_t(2) * dh * v3 + d1 * v4) * S_t(1.0 / 6.0);
                const S_t w2 = ah + half * dh * a0;
                const S_t w3 = ah + half * dh * w2;
                const S_t w4 = a1 + d1 * w3;
                const S_t qv = (a0 + S_t(2) * w2 + S_t(2) * w3 + w4) * S_t(1.0 / 6.0);
                S[k] = need_rho ? pv : S_t(0);
                Qv[k] = need_rho ? qv : S_t(0);
                if (!(S[k] <= S_t(1) && Qv[k] >= S_t(0)) && used) bad = true;
                const double pd = (double)S[k], qd = (double)Qv[k];
                cb = (1.0 - pd) * cb + qd * ra;
                ca = (1.0 - pd) * ca;
            } else {
                // one classical RK4 step of d rho/dt = g(t) (rho_at - rho), in units of dt g:
                // rho' = rho + S (rho_at - rho)
                const S_t u2 = one - half * a0;
                const S_t u3 = one - half * ah * u2;
                const S_t u4 = one - ah * u3;
                const S_t sv = (a0 + S_t(2) * ah * u2 + S_t(2) * ah * u3 + a1 * u4) * S_t(1.0 / 6.0);
                S[k] = need_rho ? sv : S_t(0);
                if (!(S[k] >= S_t(0) && S[k] <= S_t(1)) && used) bad = true;
                const double sd = (double)S[k];
                cb = (1.0 - sd) * cb + sd * ra;  // compose after the chunk's earlier steps
                ca = (1.0 - sd) * ca;
            }
            a0 = a1;
        }
        if (bad) atomicOr(unstable, 1);
        double r = row_exclusive_scan<T>(ca, cb, tr, sh, rho_end);
#pragma unroll
        for (int k = 0; k < E; k++) {
            rho[k] = r;
            const double sd = (double)S[k];
            r = (1.0 - sd) * r + (AVAL ? (double)Qv[AVAL ? k : 0] : sd) * ra;
        }
    } else {
#pragma unroll
        for (int k = 0; k < E; k++) rho[k] = 0.0;
    }

    // FP32 kernels without the density keep the two maxima in FP32 (a maximum is exact in any
    // precision) and convert once; the sum of intensities is always accumulated in FP64
    float imax32 = 0.0f, phi32 = 0.0f;
#pragma unroll
    for (int k = 0; k < E; k++) {
        if (diag) {
            const double I = pt[k].intensity();
            acc.sum += I;
            if (F32 && !scan) {
                if constexpr (F32) {
                    imax32 = fmaxf(imax32, pt[k].ii);
                    phi32 = fmaxf(phi32, fabsf(pt[k].kerr_f(in)));
                }
            } else {
                acc.imax = fmax(acc.imax, I);
                acc.rmax = fmax(acc.rmax, rho[k]);
                acc.phimax = fmax(acc.phimax, in.phi_kerr * fabs(pt[k].kerr(in)) + in.phi_plasma * rho[k]);
            }
        }
        if (apply) {
            if constexpr (NOABS)
                c[k] = pt[k].apply_phase(c[k], in, h);
            else if constexpr (F32)
                c[k] = pt[k].apply(c[k], in, h, rho[k], scan);
            else
                c[k] = pt[k].apply(c[k], in, h, rho[k]);
        }
    }
    if (diag && F32 && !scan) {
        acc.imax = fmax(acc.imax, (double)imax32);
        acc.phimax = fmax(acc.phimax, in.phi_kerr * (double)phi32);
    }
    // the neighbour's first point with the density its own thread uses (the scan's prefix, not
    // this thread's replayed value, which may differ in the last bit): a fused pass then
    // advances every point exactly as two separate passes would
    if (apply && scan && upd_next) nx = pn.apply(nx, in, h, rho_end);
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
    // FP32: the first half of the twiddle table (and of its low parts with RK_TW_PAIR) is
    // staged in LDS (FP64 kernels keep the global table: the extra LDS and addressing push
    // them into register spills)
    static constexpr bool PAIR = (FLAGS & RK_TW_PAIR) != 0;
    static constexpr int TWH = PAIR ? NT : NT / 2;
    static constexpr int TWP = TWH + TWH / 32;  // padded like the rows (lpad)
    static constexpr bool TW_LDS = sizeof(c2<R>) == 8 && sizeof(c2<R>) * (size_t)(RPW * LROW + TWP) <= 150 * 1024;
    static constexpr int TWN = TW_LDS ? TWP : 1;
    static_assert(!PAIR || sizeof(R) == 4, "twiddle pairs are for FP32 arithmetic");
};

// Position of frequency p in a pair-order row (see RK_FFT_OUT): column s at 2s, column nt - s at
// 2s + 1, columns 0 and nt/2 at 0 and 1.
template <int NT>
__device__ __forceinline__ int pair_pos(int p) {
    return p < NT / 2 ? 2 * p : (p == NT / 2 ? 1 : 2 * (NT - p) + 1);
}

// R: arithmetic precision; ST: storage precision of the field (ST = float with R = double is
// the FP32-storage mode: FP64 arithmetic, FP32 loads and stores).
template <typename R, typename ST, int NT, int E, int FLAGS>
__global__ void __launch_bounds__(row_threads(NT, E)) row_kernel(RowArgs a) {
    using Cfg = RowCfg<R, NT, E, FLAGS>;
    constexpr int T = Cfg::T;
    constexpr int RPW = Cfg::RPW;
    constexpr bool BOOK = (FLAGS & RK_STAGE_LEN) == 0 && (FLAGS & (RK_NL_A | RK_NL_B | RK_DIAG)) != 0;
    constexpr bool NEED_CHUNK = (FLAGS & (RK_NL_A | RK_NL_B | RK_DIAG)) != 0;
    __shared__ c2<R> lds[RPW * Cfg::LROW];
    __shared__ c2<R> twl[Cfg::TWN];
    __shared__ RowScratch sh;
    constexpr bool FFTS = (FLAGS & (RK_IFFT_IN | RK_FFT_OUT)) != 0;
    // a z-step's FP32 spectrum is in pair order; an FP64 one, and the stand-alone transform
    // stages', in natural order
    constexpr bool PAIR_ORDER = (FLAGS & (RK_NL_A | RK_NL_B)) != 0 && sizeof(ST) == 4;
    constexpr bool PAIRS_IN = PAIR_ORDER && (FLAGS & RK_IFFT_IN) != 0;
    constexpr bool PAIRS_OUT = PAIR_ORDER && (FLAGS & RK_FFT_OUT) != 0;

    const int tid = threadIdx.x;
    const int tr = tid % T;
    const int rw = tid / T;
    c2<R> *row_lds = lds + rw * Cfg::LROW;
    // every row of a launch has the same nt, so one twiddle table serves them all: it is staged
    // in LDS once per workgroup, and the workgroup then steps through its rows (groups of RPW
    // rows blockIdx.x, blockIdx.x + gridDim.x, ...)
    const c2<R> *tw = reinterpret_cast<const c2<R> *>(a.twiddle) + a.inst[a.items[0].inst].tw_off;
    const c2<R> *twp = tw;
    if constexpr (FFTS && Cfg::TW_LDS) {
        for (int i = tid; i < NT / 2; i += Cfg::THREADS) {
            twl[lpad(i)] = tw[i];
            if constexpr (Cfg::PAIR) twl[lpad(NT / 2 + i)] = tw[NT + i];  // low parts: table of NT after the NT highs
        }
        __syncthreads();
        twp = twl;
    }
    int64_t n = 0;
    if constexpr (BOOK) n = a.state->cnt_row;
    // adaptive mode: the largest phase rate of this thread's rows (first thread of a row slot),
    // kept while consecutive rows belong to one instance and max-reduced into the instance's
    // slot when the instance changes and at the end (an atomic per run of rows, not per row)
    int phi_inst = -1;
    double phi_run = 0.0;
    auto flush_phi = [&]() {
        if (phi_inst < 0) return;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(phi_run);
        atomicMax(&a.phi_slot[(n & 1) * a.batch + phi_inst], bits);
        if (a.seed_slots) atomicMax(&a.phi_slot[((n - 1) & 1) * a.batch + phi_inst], bits);
    };

    for (int grp = blockIdx.x; grp * RPW < a.nitems; grp += gridDim.x) {
    const int item_idx = grp * RPW + rw;
    const bool active = item_idx < a.nitems;
    const RowItem it = a.items[active ? item_idx : 0];
    const DevInst in = a.inst[it.inst];
    c2<ST> *g = reinterpret_cast<c2<ST> *>(a.field) + in.field_off + (int64_t)it.m * NT;

    double dz_a = 0.0, dz_b = 0.0;
    if constexpr (BOOK) {
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
    for (int k = 0; k < E; k++) {
        const int p = tr + k * T;
        v[k] = active ? ccast<R, ST>(g[PAIRS_IN ? pair_pos<NT>(p) : p]) : czero<R>();
    }

    if constexpr ((FLAGS & RK_IFFT_IN) != 0) {
        row_fft<R, NT, E, +1, Cfg::TW_LDS, Cfg::PAIR>(v, row_lds, tr, twp);
        const R sc = R(1.0 / NT);
#pragma unroll
        for (int k = 0; k < E; k++) v[k] = cscale<R>(v[k], sc);
    }

    if constexpr (NEED_CHUNK) {
        DiagAcc acc{0.0, 0.0, 0.0, 0.0};
        // the density scan needs contiguous points per thread; a launch without any density
        // term applies the nonlinear step pointwise on the strided registers instead
        constexpr bool scan = (FLAGS & RK_SCAN) != 0;
        constexpr bool NOABS = (FLAGS & RK_NOABS) != 0;
        constexpr bool AVAL = (FLAGS & RK_AVAL) != 0;
        static_assert(!AVAL || scan, "the avalanche rate is part of the density scan");
        static_assert(!(scan && NOABS), "a launch without absorption or density has no scan");
        const R ha = R(0.5 * dz_a), hb = R(0.5 * dz_b);
        constexpr bool DO_A = (FLAGS & RK_NL_A) != 0;
        constexpr bool DO_B = (FLAGS & RK_NL_B) != 0;
        constexpr bool DO_D = (FLAGS & RK_DIAG) != 0;
        if constexpr (scan) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < E; k++) row_lds[lpad(tr + k * T)] = v[k];
            __syncthreads();
            c2<R> c[E];
#pragma unroll
            for (int k = 0; k < E; k++) c[k] = row_lds[lpad(tr * E + k)];
            c2<R> nx = row_lds[lpad(tr < T - 1 ? tr * E + E : 0)];
            int32_t *unst = &a.state->unstable;
            if constexpr (DO_A) nl_sub_step<R, T, E, false, AVAL>(c, nx, in, ha, true, false, true, true, acc, tr, sh, unst);
            if constexpr (DO_B || DO_D)
                nl_sub_step<R, T, E, false, AVAL>(c, nx, in, hb, DO_B, DO_D, true, false, acc, tr, sh, unst);
            if constexpr ((FLAGS & RK_STORE) != 0) {
                __syncthreads();
#pragma unroll
                for (int k = 0; k < E; k++) row_lds[lpad(tr * E + k)] = c[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < E; k++) v[k] = row_lds[lpad(tr + k * T)];
            }
        } else if constexpr (NOABS && DO_A) {
            // Kerr phase only: the rotations leave |A| unchanged, so NL(dz_n/2) o NL(dz_{n-1}/2)
            // is one rotation by (dz_{n-1} + dz_n)/2 times the Kerr rate of the same intensity,
            // and the diagnostics of A^n are those of that intensity
            c2<R> unused = czero<R>();
            const R hab = DO_B ? R(0.5 * dz_a + 0.5 * dz_b) : ha;
            nl_sub_step<R, T, E, NOABS, false>(v, unused, in, hab, true, DO_D, false, false, acc, tr, sh,
                                               &a.state->unstable);
        } else {
            c2<R> unused = czero<R>();
            int32_t *unst = &a.state->unstable;
            if constexpr (DO_A) nl_sub_step<R, T, E, NOABS, false>(v, unused, in, ha, true, false, false, false, acc, tr, sh, unst);
            if constexpr (DO_B || DO_D)
                nl_sub_step<R, T, E, NOABS, false>(v, unused, in, hb, DO_B, DO_D, false, false, acc, tr, sh, unst);
        }
        if constexpr (DO_D) {
            acc = row_reduce<T>(acc, tr, sh);
            if (active && tr == 0) {
                double *rd = a.row_diag + 4 * (int64_t)(in.row_base + it.m);
                rd[0] = acc.sum;
                rd[1] = acc.imax;
                rd[2] = acc.rmax;
                rd[3] = acc.phimax;
                if (!(acc.sum <= 1.0e300)) atomicOr(&a.state->nonfinite, 1);  // NaN or overflow
                // the phase-rate slots feed the adaptive rule only (all rows of an instance
                // share one slot, so the rows' maxima are combined before the atomic)
                if (BOOK && a.dz_mode == DZ_ADAPTIVE) {
                    if (it.inst != phi_inst) {
                        flush_phi();
                        phi_inst = it.inst;
                        phi_run = acc.phimax;
                    } else {
                        phi_run = fmax(phi_run, acc.phimax);
                    }
                }
            }
        }
    }

    if constexpr ((FLAGS & RK_FFT_OUT) != 0) row_fft<R, NT, E, -1, Cfg::TW_LDS, Cfg::PAIR>(v, row_lds, tr, twp);

    if constexpr ((FLAGS & RK_STORE) != 0) {
        if (active) {
#pragma unroll
            for (int k = 0; k < E; k++) {
                const int p = tr + k * T;
                g[PAIRS_OUT ? pair_pos<NT>(p) : p] = ccast<ST, R>(v[k]);
            }
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
    }
    }  // rows of this workgroup
    if constexpr (BOOK) {
        flush_phi();
        if (blockIdx.x == 0 && tid == 0) a.state->cnt_col = n;
    }
}

// ------------------------------------------------------------------ launch table

// Launches go through hipExtLaunchKernelGGL: with non-null events it records them at the
// kernel's own start and end (timing without the gaps between launches).
template <typename R, typename ST, int NT, int FLAGS>
static hipError_t launch_row_t(const RowArgs &a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    constexpr int E = row_elems_for(NT, sizeof(R) == 8);
    using Cfg = RowCfg<R, NT, E, FLAGS>;
    hipExtLaunchKernelGGL((row_kernel<R, ST, NT, E, FLAGS>), dim3(grid), dim3(Cfg::THREADS), 0, s, e0, e1, 0, a);
    return hipGetLastError();
}

template <typename R, typename ST, int FLAGS>
static hipError_t launch_row_nt(int nt, const RowArgs &a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (nt) {
        case 64: return launch_row_t<R, ST, 64, FLAGS>(a, grid, s, e0, e1);
        case 128: return launch_row_t<R, ST, 128, FLAGS>(a, grid, s, e0, e1);
        case 256: return launch_row_t<R, ST, 256, FLAGS>(a, grid, s, e0, e1);
        case 512: return launch_row_t<R, ST, 512, FLAGS>(a, grid, s, e0, e1);
        case 1024: return launch_row_t<R, ST, 1024, FLAGS>(a, grid, s, e0, e1);
        case 2048: return launch_row_t<R, ST, 2048, FLAGS>(a, grid, s, e0, e1);
        case 4096: return launch_row_t<R, ST, 4096, FLAGS>(a, grid, s, e0, e1);
        case 8192: return launch_row_t<R, ST, 8192, FLAGS>(a, grid, s, e0, e1);
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

// X: flags added to every combination at compile time (RK_TW_PAIR for FP32 with twiddle pairs)
template <typename R, typename ST, int X = 0>
static hipError_t launch_row_p(int nt, int flags, const RowArgs &a, int grid, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
    switch (flags) {
        case RK_FIRST: return launch_row_nt<R, ST, (RK_FIRST) | X>(nt, a, grid, s, e0, e1);
        case RK_MIDDLE: return launch_row_nt<R, ST, (RK_MIDDLE) | X>(nt, a, grid, s, e0, e1);
        case RK_LAST: return launch_row_nt<R, ST, (RK_LAST) | X>(nt, a, grid, s, e0, e1);
        case RK_DIAG_ONLY: return launch_row_nt<R, ST, (RK_DIAG_ONLY) | X>(nt, a, grid, s, e0, e1);
        case RK_T_NL: return launch_row_nt<R, ST, (RK_T_NL) | X>(nt, a, grid, s, e0, e1);
        case RK_FIRST | RK_SCAN: return launch_row_nt<R, ST, (RK_FIRST | RK_SCAN) | X>(nt, a, grid, s, e0, e1);
        case RK_MIDDLE | RK_SCAN: return launch_row_nt<R, ST, (RK_MIDDLE | RK_SCAN) | X>(nt, a, grid, s, e0, e1);
        case RK_LAST | RK_SCAN: return launch_row_nt<R, ST, (RK_LAST | RK_SCAN) | X>(nt, a, grid, s, e0, e1);
        case RK_DIAG_ONLY | RK_SCAN: return launch_row_nt<R, ST, (RK_DIAG_ONLY | RK_SCAN) | X>(nt, a, grid, s, e0, e1);
        case RK_T_NL | RK_SCAN: return launch_row_nt<R, ST, (RK_T_NL | RK_SCAN) | X>(nt, a, grid, s, e0, e1);
        case RK_FIRST | RK_SCAN | RK_AVAL:
            return launch_row_nt<R, ST, (RK_FIRST | RK_SCAN | RK_AVAL) | X>(nt, a, grid, s, e0, e1);
        case RK_MIDDLE | RK_SCAN | RK_AVAL:
            return launch_row_nt<R, ST, (RK_MIDDLE | RK_SCAN | RK_AVAL) | X>(nt, a, grid, s, e0, e1);
        case RK_LAST | RK_SCAN | RK_AVAL:
            return launch_row_nt<R, ST, (RK_LAST | RK_SCAN | RK_AVAL) | X>(nt, a, grid, s, e0, e1);
        case RK_DIAG_ONLY | RK_SCAN | RK_AVAL:
            return launch_row_nt<R, ST, (RK_DIAG_ONLY | RK_SCAN | RK_AVAL) | X>(nt, a, grid, s, e0, e1);
        case RK_T_NL | RK_SCAN | RK_AVAL:
            return launch_row_nt<R, ST, (RK_T_NL | RK_SCAN | RK_AVAL) | X>(nt, a, grid, s, e0, e1);
        case RK_FIRST | RK_NOABS: return launch_row_nt<R, ST, (RK_FIRST | RK_NOABS) | X>(nt, a, grid, s, e0, e1);
        case RK_MIDDLE | RK_NOABS: return launch_row_nt<R, ST, (RK_MIDDLE | RK_NOABS) | X>(nt, a, grid, s, e0, e1);
        case RK_LAST | RK_NOABS: return launch_row_nt<R, ST, (RK_LAST | RK_NOABS) | X>(nt, a, grid, s, e0, e1);
        case RK_DIAG_ONLY | RK_NOABS:
            return launch_row_nt<R, ST, (RK_DIAG_ONLY | RK_NOABS) | X>(nt, a, grid, s, e0, e1);
        case RK_T_NL | RK_NOABS: return launch_row_nt<R, ST, (RK_T_NL | RK_NOABS) | X>(nt, a, grid, s, e0, e1);
        case RK_T_FFT: return launch_row_nt<R, ST, (RK_T_FFT) | X>(nt, a, grid, s, e0, e1);
        case RK_T_IFFT: return launch_row_nt<R, ST, (RK_T_IFFT) | X>(nt, a, grid, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

int row_rows_per_group(int nt, int elems) {
    const int t = nt / elems;
    return t >= 256 ? 1 : 256 / t;
}

hipError_t launch_row(int precision, int nt, int elems, int flags, const RowArgs &a, int grid, hipStream_t s,
                      hipEvent_t e0, hipEvent_t e1) {
    if (elems != row_elems_for(nt, row_fp64_arith(precision))) return hipErrorInvalidValue;
    switch (precision) {
        case 0: return launch_row_p<double, double>(nt, flags, a, grid, s, e0, e1);
        case 1: return launch_row_p<float, float>(nt, flags, a, grid, s, e0, e1);
        case 2: return launch_row_p<double, float>(nt, flags, a, grid, s, e0, e1);
        case 3: return launch_row_p<float, float, RK_TW_PAIR>(nt, flags, a, grid, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ small kernels

// One workgroup per instance: reduces the per-row partials of the last row pass into a
// diagnostics record (layout in include/fcn.h): radial rows weighted by w_m (energy
// 2 pi dr^2 dtau sum_m w_m sum_p |A|^2), Cartesian points by 1 (energy dx dy dtau sum |A|^2).
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
        const double w = in.geom ? 1.0 : (m == 0 ? 0.125 : (double)m);  // radial: w_0 = 1/8, w_m = m
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
        rec[0] = in.e_unit * se[0];
        rec[1] = si[0];
        rec[2] = row_diag[4 * (int64_t)(in.row_base + in.axis_row) + 1];
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

// Resets the step state of every lane: counters to n0, flags, phase slots, dz ring and z
// positions to zero.
__global__ void init_state_kernel(DevState *state, int nstates, unsigned long long *phi_slot, double *dz_ring,
                                  double *zpos, int batch, int64_t n0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nstates) {
        state[i].cnt_col = n0;
        state[i].cnt_row = n0;
        state[i].nonfinite = 0;
        state[i].unstable = 0;
    }
    if (i < 2 * batch) {
        phi_slot[i] = 0ull;
        dz_ring[i] = 0.0;
    }
    if (i < batch) zpos[i] = 0.0;
}

hipError_t launch_init_state(DevState *state, int nstates, unsigned long long *phi_slot, double *dz_ring,
                             double *zpos, int batch, int64_t n0, hipStream_t s) {
    const int threads = 256;
    const int n = 2 * batch > nstates ? 2 * batch : nstates;
    const int grid = (n + threads - 1) / threads;
    hipLaunchKernelGGL(init_state_kernel, dim3(grid), dim3(threads), 0, s, state, nstates, phi_slot, dz_ring, zpos,
                       batch, n0);
    return hipGetLastError();
}

__global__ void clear_flag_kernel(DevState *state, int nstates) {
    const int i = threadIdx.x;
    if (i < nstates) {
        state[i].nonfinite = 0;
        state[i].unstable = 0;
    }
}

hipError_t launch_clear_flag(DevState *state, int nstates, hipStream_t s) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(64), 0, s, state, nstates);
    return hipGetLastError();
}

}  // namespace fcn
