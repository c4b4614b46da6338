// fft.hpp -- LDS-staged Stockham FFT of one row of NT points held by T = NT/E threads.
//
// Data convention between stages ("strided layout"): thread tr holds v[k] = x[tr + k*T],
// k < E.  A forward transform maps the strided layout of x to the strided layout of
// X_k = sum_j x_j exp(-2 pi i jk/NT); the inverse uses exp(+2 pi i jk/NT), unscaled.
//
// Each pass of radix RADIX takes butterfly j (inputs x[j + r NT/RADIX]) to outputs at
// (j/Ns) Ns RADIX + (j mod Ns) + r Ns after the twiddle W_{Ns RADIX}^{(j mod Ns) r}
// (the self-sorting Stockham formulation), starting from Ns = 1.  The first pass reads
// the strided registers directly and the last pass returns its results in strided
// registers, so a transform of P passes makes P-1 round trips through LDS.
// Twiddles W_NT^k come from a table rounded once from FP64 values.
#pragma once

#include "cplx.hpp"

namespace fcn {

// LDS index with one pad element every 32 (breaks the power-of-two strides of the
// chunk and Stockham accesses across banks).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

// cos(2 pi j / 16) for j in [0, 16).
__device__ __forceinline__ constexpr double cos16(int j) {
    constexpr double c1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double c2 = 0.70710678118654752440;  // cos(pi/4)
    constexpr double s1 = 0.38268343236508977173;  // sin(pi/8)
    j &= 15;
    switch (j) {
        case 0: return 1.0;
        case 1: return c1;
        case 2: return c2;
        case 3: return s1;
        case 4: return 0.0;
        case 5: return -s1;
        case 6: return -c2;
        case 7: return -c1;
        case 8: return -1.0;
        case 9: return -c1;
        case 10: return -c2;
        case 11: return -s1;
        case 12: return 0.0;
        case 13: return s1;
        case 14: return c2;
        default: return c1;
    }
}
__device__ __forceinline__ constexpr double sin16(int j) { return cos16(j - 4); }

// Product of x and a constant C held as C_hi + C_lo (C_hi = C rounded to R, C_lo the
// rounded remainder): one rounding of the full product.  Rounding C alone to FP32 would
// shrink or stretch every product by the same relative amount (|W_8|^2 = 1 - 4e-8 with
// cos(pi/4) rounded), a bias the FFT would apply identically at every z-step.
template <typename R>
__device__ __forceinline__ R mul_const(R x, double c) {
    const R hi = R(c);
    const R lo = R(c - (double)hi);
    return fma(x, hi, x * lo);
}
template <typename R>
__device__ __forceinline__ R mul_const2(R x, double cx, R y, double cy) {  // x cx + y cy
    const R xh = R(cx), xl = R(cx - (double)xh);
    const R yh = R(cy), yl = R(cy - (double)yh);
    return fma(x, xh, fma(y, yh, x * xl + y * yl));
}

// x * W_N^k with W_N = exp(DIR 2 pi i / N), N <= 16, k compile-time after unrolling.
template <typename R, int N, int DIR>
__device__ __forceinline__ c2<R> mul_wn(c2<R> x, int k) {
    if (k == 0) return x;
    if (4 * k == N) return mk<R>(-R(DIR) * x.y, R(DIR) * x.x);  // times DIR*i
    const int j = (16 / N) * k;
    const double c = cos16(j);
    const double s = double(DIR) * sin16(j);
    if (j == 2 || j == 6 || j == 10 || j == 14) {
        // |c| = |s| = 1/sqrt(2): s = c gives (c (x - y), c (x + y)); s = -c gives
        // (c (x + y), c (y - x)); one sum, one difference and two products by c
        const R u = (c == s) ? x.x - x.y : x.x + x.y;
        const R v = (c == s) ? x.x + x.y : x.y - x.x;
        return mk<R>(mul_const<R>(u, c), mul_const<R>(v, c));
    }
    return mk<R>(mul_const2<R>(x.x, c, x.y, -s), mul_const2<R>(x.x, s, x.y, c));
}

// In-register DFT of N = 1, 2, 4, 8 or 16 points, radix-2 decimation in time.
template <typename R, int N, int DIR>
struct SmallDFT {
    static __device__ __forceinline__ void run(c2<R> *x) {
        c2<R> e[N / 2], o[N / 2];
#pragma unroll
        for (int k = 0; k < N / 2; k++) {
            e[k] = x[2 * k];
            o[k] = x[2 * k + 1];
        }
        SmallDFT<R, N / 2, DIR>::run(e);
        SmallDFT<R, N / 2, DIR>::run(o);
#pragma unroll
        for (int k = 0; k < N / 2; k++) {
            c2<R> t = mul_wn<R, N, DIR>(o[k], k);
            x[k] = cadd<R>(e[k], t);
            x[k + N / 2] = csub<R>(e[k], t);
        }
    }
};
template <typename R, int DIR>
struct SmallDFT<R, 1, DIR> {
    static __device__ __forceinline__ void run(c2<R> *) {}
};
template <typename R, int DIR>
struct SmallDFT<R, 2, DIR> {
    static __device__ __forceinline__ void run(c2<R> *x) {
        c2<R> a = x[0], b = x[1];
        x[0] = cadd<R>(a, b);
        x[1] = csub<R>(a, b);
    }
};

template <typename R, int NT, int E, int DIR, int NS>
struct StockhamPass {
    static constexpr int T = NT / E;
    static constexpr int RADIX = (NT / NS >= E) ? E : NT / NS;
    static constexpr int BF = E / RADIX;  // butterflies per thread
    static constexpr bool LAST = (NS * RADIX == NT);

    // v holds this pass's inputs: v[q*RADIX + r] = x[j + r*NT/RADIX], j = tr + q*T.
    // tw: HALF = false: W_NT^k for k < NT; HALF = true: k < NT/2 (W^(k+NT/2) = -W^k), an LDS
    // copy with entry i at lpad(i).
    // PAIR: each twiddle is hi + lo (hi the table above, lo the same-size table after it),
    // so the transform's constants carry about twice the working precision.
    template <bool HALF, bool PAIR>
    static __device__ __forceinline__ void run(c2<R> (&v)[E], c2<R> *lds, int tr, const c2<R> *__restrict__ tw) {
#pragma unroll
        for (int q = 0; q < BF; q++) {
            const int j = tr + q * T;
            if constexpr (NS > 1) {
                const int jm = j & (NS - 1);
#pragma unroll
                for (int r = 1; r < RADIX; r++) {
                    const int idx = jm * r * (NT / (NS * RADIX));
                    constexpr int TN = HALF ? NT / 2 : NT;  // entries of one table
                    const int ti = HALF ? (idx & (NT / 2 - 1)) : idx;
                    const bool neg = HALF && idx >= NT / 2;
                    // the LDS copy (HALF) is padded like the data rows: the twiddle indices of a
                    // pass are multiples of NT/(NS*RADIX), which would put every lane of a
                    // wavefront on the same bank
                    c2<R> w = tw[HALF ? lpad(ti) : ti];
                    if (neg) w = mk<R>(-w.x, -w.y);
                    if constexpr (PAIR) {
                        c2<R> wl = tw[HALF ? lpad(TN + ti) : TN + ti];
                        if (neg) wl = mk<R>(-wl.x, -wl.y);
                        v[q * RADIX + r] = (DIR < 0) ? cmul_pair<R>(v[q * RADIX + r], w, wl)
                                                     : cmulc_pair<R>(v[q * RADIX + r], w, wl);
                    } else {
                        v[q * RADIX + r] = (DIR < 0) ? cmul<R>(v[q * RADIX + r], w) : cmulc<R>(v[q * RADIX + r], w);
                    }
                }
            }
            SmallDFT<R, RADIX, DIR>::run(&v[q * RADIX]);
        }
        if constexpr (LAST) {
            // outputs x[j + r*NS] = x[tr + T*(q + r*BF)] -> strided register k = q + r*BF
            c2<R> o[E];
#pragma unroll
            for (int q = 0; q < BF; q++)
#pragma unroll
                for (int r = 0; r < RADIX; r++) o[q + r * BF] = v[q * RADIX + r];
#pragma unroll
            for (int k = 0; k < E; k++) v[k] = o[k];
        } else {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < BF; q++) {
                const int j = tr + q * T;
                const int base = (j / NS) * NS * RADIX + (j & (NS - 1));
#pragma unroll
                for (int r = 0; r < RADIX; r++) lds[lpad(base + r * NS)] = v[q * RADIX + r];
            }
            __syncthreads();
            using Next = StockhamPass<R, NT, E, DIR, NS * RADIX>;
#pragma unroll
            for (int q = 0; q < Next::BF; q++)
#pragma unroll
                for (int r = 0; r < Next::RADIX; r++)
                    v[q * Next::RADIX + r] = lds[lpad(tr + q * T + r * (NT / Next::RADIX))];
            Next::template run<HALF, PAIR>(v, lds, tr, tw);
        }
    }
};

// Full transform, strided layout in and out.  DIR = -1 forward, +1 inverse (unscaled).
// HALF: tw is an LDS copy of the first NT/2 table entries, entry i at lpad(i).  PAIR: tw is
// followed by a table of the same size holding the low parts of the twiddles (with HALF:
// low part of entry i at lpad(NT/2 + i)).  Every thread of the workgroup must call
// it (it contains barriers).
template <typename R, int NT, int E, int DIR, bool HALF = false, bool PAIR = false>
__device__ __forceinline__ void row_fft(c2<R> (&v)[E], c2<R> *lds, int tr, const c2<R> *__restrict__ tw) {
    static_assert(NT >= E && (NT & (NT - 1)) == 0, "NT must be a power of two >= E");
    StockhamPass<R, NT, E, DIR, 1>::template run<HALF, PAIR>(v, lds, tr, tw);
}

}  // namespace fcn
