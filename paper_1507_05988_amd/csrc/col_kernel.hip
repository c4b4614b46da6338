// col_kernel.hip -- the column pass of the FCN z-step on gfx950: for every frequency
// column p, A~^{n+1}_{.,p} = (M_abc^p)^{-1} M_def^p A~^n_{.,p} (Eq. matrix; second loop of
// Sec. 3.1), in place on the spectrum.
//
// Matrices (Eq. matrix1 and the coefficient list after it), with s = dz/(4 k0 dr^2) and
// g_p = k'' omega_p^2 dz/4:
//   row 0      (dA/dr = 0 at the axis):  b = 1 + i(4s - g), c = -4is;  e = conj(b), f = 4is
//   row m      (1 <= m <= nr-2):         a = -is(1 - 1/2m), b = 1 + i(2s - g), c = -is(1 + 1/2m);
//                                        d = -a, e = conj(b), f = -c
//   row nr-1   (A = 0 at r_max):         b = 1, right-hand side 0
// c_m and f_m use (1 + 1/2m): the centred 1/r dA/dr term adds +1/(2m dr^2) to the A_{m+1}
// coefficient (Eqs. diff2-diff3); the printed (1 - 1/2m) would cancel it.
//
// Layout: the spectrum is [nr][nt] with p contiguous, so a workgroup takes W adjacent
// frequencies (lanes read W consecutive complex values of a row: coalesced) and all nr rows.
// The tridiagonal solve is a partitioned ("divide and conquer") elimination without
// pivoting, so each element is read once and written once:
//   1. thread (p, k) owns rows [kL, kL+L) of column p: it forms the right-hand side
//      M_def x from its rows and one halo row on each side, then eliminates its interior
//      rows 1..L-2 so every interior unknown is x_i = D_i - A_i x_first - C_i x_last;
//   2. substituting that into its first and last rows gives two equations that couple only
//      chunk boundary unknowns: a tridiagonal system of 2S unknowns per column (S chunks),
//      solved in LDS by parallel cyclic reduction;
//   3. each thread back-substitutes its interior rows and writes its L outputs.
// No pivoting is needed: with W = diag(1/8, 1, 2, ...) the operator dz/2 L is
// W-skew-Hermitian, so after the diagonal similarity W^(1/2) the matrix I - dz/2 L has
// Hermitian part I, which keeps every elimination (any symmetric ordering) well posed.
#include <hip/hip_ext.h>

#include "fcn_internal.h"
#include "cplx.hpp"

namespace fcn {

template <typename R>
struct Eq {  // lower, upper, rhs of one normalised (unit diagonal) reduced equation
    c2<R> l, u, r;
};

// 1 / z for the pivots of the elimination.  They depend on the operator only, never on the
// field, and |z|^2 stays of order one (the matrix has Hermitian part I after the diagonal
// similarity above), so the hardware reciprocal refined by Newton-Raphson steps
// r <- r + r (1 - d r) replaces the IEEE division sequence: two steps from the
// reciprocal's estimate reach the FP64 rounding level, one step the FP32 level.
template <typename R>
__device__ __forceinline__ c2<R> pivot_rcp(c2<R> z) {
    const R d = z.x * z.x + z.y * z.y;
    R r;
    if constexpr (sizeof(R) == 8) {
        r = __builtin_amdgcn_rcp(d);
        r = fma(r, fma(-d, r, 1.0), r);
        r = fma(r, fma(-d, r, 1.0), r);
    } else {
        r = __builtin_amdgcn_rcpf(d);
        r = fmaf(r, fmaf(-d, r, 1.0f), r);
    }
    return mk<R>(z.x * r, -z.y * r);
}

// R: arithmetic precision; ST: storage precision of the spectrum (see the row kernel).
template <typename R, typename ST, int W, int L>
__global__ void __launch_bounds__(512) col_kernel(ColArgs a) {
    static_assert(L >= 4, "at least two interior rows per chunk");
    extern __shared__ unsigned char smem_raw[];
    Eq<R> *red = reinterpret_cast<Eq<R> *>(smem_raw);  // [W][2S + 1]

    // Workgroups are dispatched round-robin over the 8 XCDs (b -> XCD b mod 8).  Give each
    // XCD a contiguous range of column tiles so tiles sharing 128-byte lines (W*sizeof < 128)
    // meet in the same L2.
    const int nb = gridDim.x, b = blockIdx.x;
    const int xcd = b & 7, per = nb >> 3, rem = nb & 7;
    const int tile = xcd * per + min(xcd, rem) + (b >> 3);
    const ColItem it = a.items[tile];
    const DevInst in = a.inst[it.inst];
    const int nr = in.nr, nt = in.nt;
    const int t = threadIdx.x;
    const int pl = t % W;
    const int k = t / W;
    const int S = blockDim.x / W;
    const int nred = 2 * S;
    const int p = it.p0 + pl;
    // one spare entry per column: a stride of 2S entries would put the W columns of a
    // wavefront on the same LDS banks (2S * sizeof(Eq) is a multiple of 256 bytes)
    Eq<R> *myred = red + pl * (nred + 1);

    int64_t n = 0;
    double dz;
    if (a.use_stage_len) {
        dz = a.stage_len;
    } else {
        n = a.state->cnt_col;
        dz = a.dz_ring[(n & 1) * a.batch + it.inst];
    }
    const int q = p < nt / 2 ? p : p - nt;
    const R s = R(dz * in.diff_unit);
    const R g = R((double)q * (double)q * in.gvd_unit * dz);
    const R bi_in = R(2) * s - g;      // Im b, interior rows
    const R bi_ax = R(4) * s - g;      // Im b, axis row
    const double *rc = a.rowcoef + 2 * (int64_t)in.rowcoef_off;

    c2<ST> *col = reinterpret_cast<c2<ST> *>(a.field) + in.field_off + p;
    const int m0 = k * L;

    // ---- load rows m0-1 .. m0+L (halo included); rows outside [0, nr) read as 0
    c2<R> x[L + 2];
#pragma unroll
    for (int i = 0; i < L + 2; i++) {
        const int m = m0 - 1 + i;
        x[i] = (m >= 0 && m < nr) ? ccast<R, ST>(col[(int64_t)m * nt]) : czero<R>();
    }

    // Row m of M_abc as (l, b, u) = (i lr, 1 + i bi, i ur) and of M_def x, computed on the fly.
    // x[i + 1] holds row m0 + i.
    auto row_coef = [&](int i, R &lr, R &bi, R &ur) {
        const int m = m0 + i;
        if (m == 0) {
            lr = R(0);
            bi = bi_ax;
            ur = R(-4) * s;
        } else if (m < nr - 1) {
            lr = -s * R(rc[2 * m]);
            bi = bi_in;
            ur = -s * R(rc[2 * m + 1]);
        } else {  // r_max row (x = 0) and padding rows beyond nr: identity
            lr = R(0);
            bi = R(0);
            ur = R(0);
        }
    };
    // d x_{m-1} + e x_m + f x_{m+1} with d = -l, e = conj(b), f = -u (zero on the r_max row)
    auto rhs_of = [&](int i, R lr, R bi, R ur) -> c2<R> {
        const int m = m0 + i;
        if (m >= nr - 1) return czero<R>();
        const c2<R> xm = x[i + 1];
        c2<R> v = mk<R>(xm.x + bi * xm.y, xm.y - bi * xm.x);
        v = cadd<R>(v, cmul_i<R>(x[i], -lr));
        return cadd<R>(v, cmul_i<R>(x[i + 2], -ur));
    };

    R lr0, bi0, ur0, lrL, biL, urL;
    row_coef(0, lr0, bi0, ur0);
    row_coef(L - 1, lrL, biL, urL);
    const c2<R> rhs0 = rhs_of(0, lr0, bi0, ur0);
    const c2<R> rhsL = rhs_of(L - 1, lrL, biL, urL);

    // ---- local elimination of interior rows 1..L-2:  x_i = rp_i - sp_i x_first - mu_i x_{i+1}
    c2<R> mu[L], rp[L], sp[L];
    {
        R lr, bi, ur;
        row_coef(1, lr, bi, ur);
        c2<R> ip = pivot_rcp<R>(mk<R>(R(1), bi));
        mu[1] = cmul<R>(mk<R>(R(0), ur), ip);
        rp[1] = cmul<R>(rhs_of(1, lr, bi, ur), ip);
        sp[1] = cmul<R>(mk<R>(R(0), lr), ip);
#pragma unroll
        for (int i = 2; i <= L - 2; i++) {
            row_coef(i, lr, bi, ur);
            // pivot b_i - l_i mu_{i-1}
            const c2<R> lmu = cmul_i<R>(mu[i - 1], lr);
            ip = pivot_rcp<R>(mk<R>(R(1) - lmu.x, bi - lmu.y));
            mu[i] = cmul<R>(mk<R>(R(0), ur), ip);
            rp[i] = cmul<R>(csub<R>(rhs_of(i, lr, bi, ur), cmul_i<R>(rp[i - 1], lr)), ip);
            sp[i] = cmul<R>(cmul_i<R>(sp[i - 1], -lr), ip);
        }
    }
    // backward sweep for the representation of x_1 and x_{L-2} in (x_first, x_last)
    c2<R> D = rp[L - 2], A = sp[L - 2], C = mu[L - 2];
    const c2<R> Dl = D, Al = A, Cl = C;
#pragma unroll
    for (int i = L - 3; i >= 1; i--) {
        D = csub<R>(rp[i], cmul<R>(mu[i], D));
        A = csub<R>(sp[i], cmul<R>(mu[i], A));
        C = mk<R>(-(mu[i].x * C.x - mu[i].y * C.y), -(mu[i].x * C.y + mu[i].y * C.x));
    }
    // D, A, C now describe x_1; Dl, Al, Cl describe x_{L-2}.

    // ---- reduced equations of the chunk's first and last rows
    // first: l_0 X_prev + (b_0 - u_0 A_1) x_first - u_0 C_1 x_last = r_0 - u_0 D_1
    // last:  -l_{L-1} A_{L-2} x_first + (b_{L-1} - l_{L-1} C_{L-2}) x_last + u_{L-1} X_next
    //        = r_{L-1} - l_{L-1} D_{L-2}
    Eq<R> e0, e1;
    {
        const c2<R> u0 = mk<R>(R(0), ur0);
        const c2<R> uA = cmul<R>(u0, A);
        const c2<R> idg = pivot_rcp<R>(mk<R>(R(1) - uA.x, bi0 - uA.y));
        e0.l = cmul<R>(mk<R>(R(0), lr0), idg);
        const c2<R> uC = cmul<R>(u0, C);
        e0.u = cmul<R>(mk<R>(-uC.x, -uC.y), idg);
        e0.r = cmul<R>(csub<R>(rhs0, cmul<R>(u0, D)), idg);

        const c2<R> lL = mk<R>(R(0), lrL);
        const c2<R> lC = cmul<R>(lL, Cl);
        const c2<R> idg1 = pivot_rcp<R>(mk<R>(R(1) - lC.x, biL - lC.y));
        const c2<R> lA = cmul<R>(lL, Al);
        e1.l = cmul<R>(mk<R>(-lA.x, -lA.y), idg1);
        e1.u = cmul<R>(mk<R>(R(0), urL), idg1);
        e1.r = cmul<R>(csub<R>(rhsL, cmul<R>(lL, Dl)), idg1);
    }

    // ---- parallel cyclic reduction on the 2S reduced unknowns of each column
    const int i0 = 2 * k, i1 = 2 * k + 1;
    myred[i0] = e0;
    myred[i1] = e1;
    __syncthreads();
    for (int h = 1; h < nred; h <<= 1) {
        Eq<R> ne[2];
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int i = i0 + j;
            const Eq<R> me = j == 0 ? e0 : e1;
            Eq<R> lo, hi;
            if (i - h >= 0) lo = myred[i - h]; else lo = Eq<R>{czero<R>(), czero<R>(), czero<R>()};
            if (i + h < nred) hi = myred[i + h]; else hi = Eq<R>{czero<R>(), czero<R>(), czero<R>()};
            // eq_i - l_i eq_{i-h} - u_i eq_{i+h}, then renormalise
            const c2<R> dg = csub<R>(csub<R>(mk<R>(R(1), R(0)), cmul<R>(me.l, lo.u)), cmul<R>(me.u, hi.l));
            const c2<R> idg = pivot_rcp<R>(dg);
            const c2<R> nl = cmul<R>(cmul<R>(me.l, lo.l), idg);
            const c2<R> nu = cmul<R>(cmul<R>(me.u, hi.u), idg);
            const c2<R> nrh = cmul<R>(csub<R>(csub<R>(me.r, cmul<R>(me.l, lo.r)), cmul<R>(me.u, hi.r)), idg);
            ne[j] = Eq<R>{mk<R>(-nl.x, -nl.y), mk<R>(-nu.x, -nu.y), nrh};
        }
        __syncthreads();
        e0 = ne[0];
        e1 = ne[1];
        myred[i0] = e0;
        myred[i1] = e1;
        __syncthreads();
    }
    const c2<R> xf = e0.r;  // x_first
    const c2<R> xl = e1.r;  // x_last

    // ---- back-substitution and store
    c2<R> out[L];
    out[0] = xf;
    out[L - 1] = xl;
    c2<R> nxt = xl;
#pragma unroll
    for (int i = L - 2; i >= 1; i--) {
        nxt = csub<R>(csub<R>(rp[i], cmul<R>(sp[i], xf)), cmul<R>(mu[i], nxt));
        out[i] = nxt;
    }
#pragma unroll
    for (int i = 0; i < L; i++) {
        const int m = m0 + i;
        if (m < nr) col[(int64_t)m * nt] = ccast<ST, R>(out[i]);
    }

    if (!a.use_stage_len && t == 0) {
        if (blockIdx.x == 0) a.state->cnt_row = n + 1;
        if (it.p0 == 0) {
            a.zpos[it.inst] += dz;
            a.phi_slot[((n + 1) & 1) * a.batch + it.inst] = 0ull;  // slot of A^{n-1}, consumed
        }
    }
}

template <typename R, typename ST, int W, int L>
static hipError_t launch_col_t(int nr, const ColArgs &a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int S = (nr + L - 1) / L;
    const int threads = W * S;
    if (threads > 512) return hipErrorInvalidValue;
    const size_t shm = sizeof(Eq<R>) * (size_t)W * (2 * S + 1);
    hipExtLaunchKernelGGL((col_kernel<R, ST, W, L>), dim3(grid), dim3(threads), (uint32_t)shm, s, e0, e1, 0, a);
    return hipGetLastError();
}

template <typename R, typename ST>
static hipError_t launch_col_p(int w, int l, int nr, const ColArgs &a, int grid, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
    if (w == 1 && l == 8) return launch_col_t<R, ST, 1, 8>(nr, a, grid, s, e0, e1);
    if (w == 1 && l == 16) return launch_col_t<R, ST, 1, 16>(nr, a, grid, s, e0, e1);
    if (w == 2 && l == 8) return launch_col_t<R, ST, 2, 8>(nr, a, grid, s, e0, e1);
    if (w == 2 && l == 16) return launch_col_t<R, ST, 2, 16>(nr, a, grid, s, e0, e1);
    if (w == 4 && l == 8) return launch_col_t<R, ST, 4, 8>(nr, a, grid, s, e0, e1);
    if (w == 4 && l == 16) return launch_col_t<R, ST, 4, 16>(nr, a, grid, s, e0, e1);
    if (w == 8 && l == 8) return launch_col_t<R, ST, 8, 8>(nr, a, grid, s, e0, e1);
    if (w == 8 && l == 16) return launch_col_t<R, ST, 8, 16>(nr, a, grid, s, e0, e1);
    if (w == 16 && l == 8) return launch_col_t<R, ST, 16, 8>(nr, a, grid, s, e0, e1);
    if (w == 16 && l == 16) return launch_col_t<R, ST, 16, 16>(nr, a, grid, s, e0, e1);
    if (w == 32 && l == 8) return launch_col_t<R, ST, 32, 8>(nr, a, grid, s, e0, e1);
    return hipErrorInvalidValue;
}

hipError_t launch_col(int precision, int w, int l, int nr, const ColArgs &a, int grid, hipStream_t s, hipEvent_t e0,
                      hipEvent_t e1) {
    switch (precision) {
        case 0: return launch_col_p<double, double>(w, l, nr, a, grid, s, e0, e1);
        case 1: return launch_col_p<float, float>(w, l, nr, a, grid, s, e0, e1);
        case 2:  // FP32 storage, FP64 arithmetic
        case 3: return launch_col_p<double, float>(w, l, nr, a, grid, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fcn
