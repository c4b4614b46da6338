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
// Layout: the spectrum is [nr][nt], each row's nt values contiguous.  Frequencies p and nt - p
// have the same matrices (only omega_p^2 enters), so a thread solves the pair together: the
// elimination factors, pivots and reduced-system coefficients depend on the operator only and
// are computed once for both right-hand sides.  A workgroup takes W adjacent pair slots
// s = p0 .. p0+W-1 (columns s and nt - s; s = 0 and s = nt/2 are their own partners) and all nr
// rows.  Within a z-step the row pass leaves each FP32 row in pair order (PAIRS): entries 2s and
// 2s + 1 hold columns s and nt - s (0 < s < nt/2), entries 0 and 1 columns 0 and nt/2.  A lane
// then moves both columns of its pair with one load and one store per row and the W lanes of a
// tile cover 2W contiguous values (64 bytes of FP32 spectrum at W = 4, where the natural order
// gives two 32-byte pieces at p0 and nt - p0 - W + 1; a copy with this tile geometry runs at
// 6.4 against 4.2 TB/s).  An FP64 spectrum (16-byte values: the natural order already gives
// 64-byte pieces) and the stand-alone CN stage stay in natural order.
// The tridiagonal solve is a partitioned ("divide and conquer") elimination without
// pivoting, so each element is read once and written once:
//   1. thread (s, k) owns rows [kL, kL+L) of its two columns: it forms the right-hand sides
//      M_def x from its rows and one halo row on each side, then eliminates its interior
//      rows 1..L-2 so every interior unknown is x_i = D_i - A_i x_first - C_i x_last;
//   2. substituting that into its first and last rows gives two equations per chunk coupling
//      only chunk-boundary unknowns (2S unknowns per column, S chunks); one cyclic-reduction
//      step eliminates every chunk's last unknown using the neighbouring chunk's equation,
//      leaving an S-unknown tridiagonal system in the chunks' first unknowns, solved in LDS by
//      parallel cyclic reduction (log2 S levels, one equation per thread);
//   3. each thread recovers its last unknown from its own equation and the next chunk's first
//      unknown, back-substitutes its interior rows and writes its L outputs of both columns.
// No pivoting is needed: with W = diag(1/8, 1, 2, ...) the operator dz/2 L is
// W-skew-Hermitian, so after the diagonal similarity W^(1/2) the matrix I - dz/2 L has
// Hermitian part I, which keeps every elimination (any symmetric ordering) well posed.
//
// Cartesian instances (Delta_perp = d2/dx2 + d2/dy2, field [ny][nx][nt]): the same solver runs
// once along x for every (y line, pair slot) and then along y for every (x line, pair slot), two
// launches of the CART variant.  A system is one line of n = nx (or ny) points at the stride nt
// (or nx nt) with
//   rows 1 .. n-2:   a = c = -is, b = 1 + i(2s - g),  d = f = is, e = conj(b)
//   rows 0 and n-1 (the walls, A = 0):  identity, right-hand side 0
// s = dz/(4 k0 dx^2) (dy for y) and g = k'' omega_p^2 dz / 8, half the GVD term in each axis.
// The axis operators are skew-Hermitian, so the unweighted matrix already has Hermitian part I.
#include <hip/hip_ext.h>

#include "fcn_internal.h"
#include "cplx.hpp"

namespace fcn {

// 1 / z for the pivots of the elimination.  They depend on the operator only, never on the
// field, and |z|^2 stays of order one (the matrix has Hermitian part I after the diagonal
// similarity above), so the hardware reciprocal refined by Newton-Raphson steps
// r <- r + r (1 - d r) replaces the IEEE division sequence: each step squares the relative
// error of the estimate (at most 2^-24.4 for the FP64 one, measured on 4M values over 40
// binades), so two steps reach the FP64 rounding level and one step 2^-48.7, far below the
// rounding of an FP32 spectrum (FP64_FULL = false: FP64 arithmetic on FP32 storage); one step
// from the FP32 estimate reaches the FP32 level.
template <typename R, bool FP64_FULL = true>
__device__ __forceinline__ c2<R> pivot_rcp(c2<R> z) {
    const R d = z.x * z.x + z.y * z.y;
    R r;
    if constexpr (sizeof(R) == 8) {
        r = __builtin_amdgcn_rcp(d);
        r = fma(r, fma(-d, r, 1.0), r);
        if constexpr (FP64_FULL) r = fma(r, fma(-d, r, 1.0), r);
    } else {
        r = __builtin_amdgcn_rcpf(d);
        r = fmaf(r, fmaf(-d, r, 1.0f), r);
    }
    return mk<R>(z.x * r, -z.y * r);
}

// a - b c for complex values
template <typename R>
__device__ __forceinline__ c2<R> cmsub(c2<R> a, c2<R> b, c2<R> c) {
    return mk<R>(fma(-b.x, c.x, fma(b.y, c.y, a.x)), fma(-b.x, c.y, fma(-b.y, c.x, a.y)));
}

// The two columns of a pair slot in pair order, moved as one 16-byte access.
template <typename T>
struct __attribute__((aligned(2 * sizeof(c2<T>)))) cpair {
    c2<T> a, b;
};

// R: arithmetic precision; ST: storage precision of the spectrum (see the row kernel);
// PAIRS: the spectrum is in pair order.
template <typename R, typename ST, int W, int L, bool CART, bool PAIRS>
__global__ void __launch_bounds__(512) col_kernel(ColArgs a) {
    static_assert(L >= 4, "at least two interior rows per chunk");
    extern __shared__ unsigned char smem_raw[];
    constexpr bool FULL = sizeof(ST) == sizeof(R);  // pivots to the arithmetic's full precision

    // Workgroups are dispatched round-robin over the 8 XCDs (b -> XCD b mod 8).  Give each
    // XCD a contiguous range of column tiles so tiles sharing 128-byte lines (W*sizeof < 128)
    // meet in the same L2.
    const int nb = gridDim.x, b = blockIdx.x;
    const int xcd = b & 7, per = nb >> 3, rem = nb & 7;
    const int tile = xcd * per + min(xcd, rem) + (b >> 3);
    const ColItem it = a.items[tile];
    const DevInst in = a.inst[it.inst];
    const int nt = in.nt;
    // the system: nr unknowns at the element stride rs from the line's first element
    const bool xdir = CART && a.dir == COL_X;
    const int nr = CART ? (xdir ? in.nx : in.ny) : in.nr;
    const int64_t rs = CART && !xdir ? (int64_t)in.nx * nt : (int64_t)nt;
    const int64_t line_off = CART ? (xdir ? (int64_t)it.line * in.nx * nt : (int64_t)it.line * nt) : 0;
    const int t = threadIdx.x;
    const int pl = t % W;
    const int k = t / W;
    const int S = blockDim.x / W;
    // reduced equations in LDS, one array per coefficient, entry (pair slot, chunk) at
    // chunk * W + slot = the thread index: the lanes of a wavefront touch consecutive 8- or
    // 16-byte words at every access (also at the +-h neighbours of the reduction), so no two
    // lanes of a group share a bank.  Two sets of the four arrays: each reduction level reads
    // one set and writes the other, so a level needs one barrier instead of two.
    const int ws = W * S;
    c2<R> *set_a = reinterpret_cast<c2<R> *>(smem_raw);
    c2<R> *set_b = set_a + 4 * ws;
    const int me = t;

    const int slot = it.p0 + pl;          // columns slot and nt - slot
    const bool live = slot <= nt / 2;     // the last tile of an instance can be partly empty
    const int p1 = live ? slot : 0;
    const int p2 = (nt - p1) & (nt - 1);  // p1 itself for slots 0 and nt/2
    const bool store2 = live && p2 != p1;

    int64_t n = 0;
    double dz;
    if (a.use_stage_len) {
        dz = a.stage_len;
    } else {
        n = a.state->cnt_col;
        dz = a.dz_ring[(n & 1) * a.batch + it.inst];
    }
    // q^2 = slot^2 for both columns (q = slot for p1 < nt/2, q = -nt/2 for p1 = nt/2)
    const R s = R(dz * (CART && !xdir ? in.diff_unit_y : in.diff_unit));
    const R g = R((double)p1 * (double)p1 * in.gvd_unit * dz);
    const R bi_in = R(2) * s - g;      // Im b, interior rows
    const R bi_ax = R(4) * s - g;      // Im b, axis row
    const double *rc = a.rowcoef + 2 * (int64_t)in.rowcoef_off;

    c2<ST> *line0 = reinterpret_cast<c2<ST> *>(a.field) + in.field_off + line_off;
    c2<ST> *col1 = line0 + p1;
    c2<ST> *col2 = line0 + p2;
    // pair order: the slot's pair entry (columns 0 and nt/2 share entry 0; the lone column nt/2
    // is its second half) and the row stride in pairs (rs is even: nt is)
    const bool second = p1 == nt / 2;
    cpair<ST> *pcol = reinterpret_cast<cpair<ST> *>(line0) + (second ? 0 : p1);
    const int64_t prs = rs / 2;
    const int m0 = k * L;

    // ---- load rows m0-1 .. m0+L (halo included) of both columns (the lone columns 0 and nt/2
    // solve their own column twice in natural order; in pair order the second right-hand side
    // of slot 0 is column nt/2, solved alongside and not stored).  A row outside [0, nr) is read
    // from the nearest row inside: such a value only ever meets an exact zero coefficient (the
    // axis row's lower neighbour, the identity rows from nr - 1 on), so any finite value serves.
    c2<ST> x1[L + 2], x2[L + 2];
#pragma unroll
    for (int i = 0; i < L + 2; i++) {
        const int m = min(max(m0 - 1 + i, 0), nr - 1);
        if constexpr (PAIRS) {
            const cpair<ST> v = pcol[(int64_t)m * prs];
            x1[i] = second ? v.b : v.a;
            x2[i] = v.b;
        } else {
            x1[i] = col1[(int64_t)m * rs];
            x2[i] = col2[(int64_t)m * rs];
        }
    }

    // Row m of M_abc as (l, b, u) = (i lr, 1 + i bi, i ur) and of M_def x, computed on the fly.
    // x[i + 1] holds row m0 + i.
    auto row_coef = [&](int i, R &lr, R &bi, R &ur) {
        const int m = m0 + i;
        if (CART) {
            const bool inner = m > 0 && m < nr - 1;
            lr = inner ? -s : R(0);
            bi = inner ? bi_in : R(0);
            ur = inner ? -s : R(0);
        } else if (m == 0) {
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
    auto rhs_of = [&](const c2<ST> (&x)[L + 2], int i, R lr, R bi, R ur) -> c2<R> {
        const int m = m0 + i;
        if (m >= nr - 1 || (CART && m <= 0)) return czero<R>();
        const c2<R> xm = ccast<R, ST>(x[i + 1]);
        c2<R> v = mk<R>(xm.x + bi * xm.y, xm.y - bi * xm.x);
        v = cadd<R>(v, cmul_i<R>(ccast<R, ST>(x[i]), -lr));
        return cadd<R>(v, cmul_i<R>(ccast<R, ST>(x[i + 2]), -ur));
    };

    R lr0, bi0, ur0, lrL, biL, urL;
    row_coef(0, lr0, bi0, ur0);
    row_coef(L - 1, lrL, biL, urL);
    const c2<R> rhs0_1 = rhs_of(x1, 0, lr0, bi0, ur0), rhs0_2 = rhs_of(x2, 0, lr0, bi0, ur0);
    const c2<R> rhsL_1 = rhs_of(x1, L - 1, lrL, biL, urL), rhsL_2 = rhs_of(x2, L - 1, lrL, biL, urL);

    // ---- local elimination of interior rows 1..L-2:  x_i = rp_i - sp_i x_first - mu_i x_{i+1}
    // (mu, sp: the operator's, shared by both columns; rp1, rp2: one per column)
    c2<R> mu[L], sp[L], rp1[L], rp2[L];
    {
        R lr, bi, ur;
        row_coef(1, lr, bi, ur);
        c2<R> ip = pivot_rcp<R, FULL>(mk<R>(R(1), bi));
        mu[1] = cmul_i<R>(ip, ur);
        sp[1] = cmul_i<R>(ip, lr);
        rp1[1] = cmul<R>(rhs_of(x1, 1, lr, bi, ur), ip);
        rp2[1] = cmul<R>(rhs_of(x2, 1, lr, bi, ur), ip);
#pragma unroll
        for (int i = 2; i <= L - 2; i++) {
            row_coef(i, lr, bi, ur);
            // pivot b_i - l_i mu_{i-1}
            const c2<R> lmu = cmul_i<R>(mu[i - 1], lr);
            ip = pivot_rcp<R, FULL>(mk<R>(R(1) - lmu.x, bi - lmu.y));
            mu[i] = cmul_i<R>(ip, ur);
            sp[i] = cmul<R>(cmul_i<R>(sp[i - 1], -lr), ip);
            rp1[i] = cmul<R>(csub<R>(rhs_of(x1, i, lr, bi, ur), cmul_i<R>(rp1[i - 1], lr)), ip);
            rp2[i] = cmul<R>(csub<R>(rhs_of(x2, i, lr, bi, ur), cmul_i<R>(rp2[i - 1], lr)), ip);
        }
    }
    // backward sweep for the representation of x_1 and x_{L-2} in (x_first, x_last)
    c2<R> D1 = rp1[L - 2], D2 = rp2[L - 2], A = sp[L - 2], C = mu[L - 2];
    const c2<R> Dl1 = D1, Dl2 = D2, Al = A, Cl = C;
#pragma unroll
    for (int i = L - 3; i >= 1; i--) {
        D1 = cmsub<R>(rp1[i], mu[i], D1);
        D2 = cmsub<R>(rp2[i], mu[i], D2);
        A = cmsub<R>(sp[i], mu[i], A);
        C = cmul<R>(mu[i], mk<R>(-C.x, -C.y));
    }
    // D, A, C now describe x_1; Dl, Al, Cl describe x_{L-2}.

    // ---- reduced equations of the chunk's first and last rows (unit diagonal)
    // first (X_2k):   l0 X_{2k-1} + X_2k + u0 X_{2k+1} = r0
    //   from l_0 X_prev + (b_0 - u_0 A_1) x_first - u_0 C_1 x_last = r_0 - u_0 D_1
    // last (X_2k+1):  l1 X_2k + X_{2k+1} + u1 X_{2k+2} = r1
    //   from -l_{L-1} A_{L-2} x_first + (b_{L-1} - l_{L-1} C_{L-2}) x_last + u_{L-1} X_next
    //        = r_{L-1} - l_{L-1} D_{L-2}
    c2<R> l0, u0, r0_1, r0_2, l1, u1, r1_1, r1_2;
    {
        const c2<R> uA = cmul_i<R>(A, ur0);
        const c2<R> idg = pivot_rcp<R, FULL>(mk<R>(R(1) - uA.x, bi0 - uA.y));
        l0 = cmul_i<R>(idg, lr0);
        u0 = cmul<R>(cmul_i<R>(C, -ur0), idg);
        r0_1 = cmul<R>(csub<R>(rhs0_1, cmul_i<R>(D1, ur0)), idg);
        r0_2 = cmul<R>(csub<R>(rhs0_2, cmul_i<R>(D2, ur0)), idg);

        const c2<R> lC = cmul_i<R>(Cl, lrL);
        const c2<R> idg1 = pivot_rcp<R, FULL>(mk<R>(R(1) - lC.x, biL - lC.y));
        l1 = cmul<R>(cmul_i<R>(Al, -lrL), idg1);
        u1 = cmul_i<R>(idg1, urL);
        r1_1 = cmul<R>(csub<R>(rhsL_1, cmul_i<R>(Dl1, lrL)), idg1);
        r1_2 = cmul<R>(csub<R>(rhsL_2, cmul_i<R>(Dl2, lrL)), idg1);
    }

    // ---- one cyclic-reduction step: eliminate X_{2k-1} (the previous chunk's last equation)
    // and X_{2k+1} (this chunk's) from this chunk's first equation.  Chunk 0 has l0 = 0
    // exactly (the axis or wall row has no lower coupling), so it reads its own entry in place
    // of a missing neighbour: 0 times a finite value.  The reduction below does the same at both
    // ends: an equation whose neighbour at distance h is outside [0, S) has an exactly zero
    // coupling to it (true for h = 1, the first chunk's l0 and the last chunk's u1 being 0, and
    // kept by every level, whose new couplings are products with the old ones).
    set_a[me] = l1;
    set_a[ws + me] = u1;
    set_a[2 * ws + me] = r1_1;
    set_a[3 * ws + me] = r1_2;
    __syncthreads();
    const int prev = k > 0 ? me - W : me;
    const c2<R> pl1 = set_a[prev], pu1 = set_a[ws + prev];
    const c2<R> pr1 = set_a[2 * ws + prev], pr2 = set_a[3 * ws + prev];
    c2<R> yl, yu, yr1, yr2;  // Y_{k-1}, Y_{k+1} coefficients and right-hand sides, unit diagonal
    {
        const c2<R> dg = cmsub<R>(cmsub<R>(mk<R>(R(1), R(0)), l0, pu1), u0, l1);
        const c2<R> idg = pivot_rcp<R, FULL>(dg);
        const c2<R> nl = cmul<R>(cmul<R>(l0, pl1), idg);
        const c2<R> nu = cmul<R>(cmul<R>(u0, u1), idg);
        yl = mk<R>(-nl.x, -nl.y);
        yu = mk<R>(-nu.x, -nu.y);
        yr1 = cmul<R>(cmsub<R>(cmsub<R>(r0_1, l0, pr1), u0, r1_1), idg);
        yr2 = cmul<R>(cmsub<R>(cmsub<R>(r0_2, l0, pr2), u0, r1_2), idg);
    }

    // ---- parallel cyclic reduction on the S equations Y_k of each column pair (set b holds
    // the current level; set a was last read before the barrier below)
    c2<R> *cur = set_b, *nxt = set_a;
    cur[me] = yl;
    cur[ws + me] = yu;
    cur[2 * ws + me] = yr1;
    cur[3 * ws + me] = yr2;
    __syncthreads();
    for (int h = 1; h < S; h <<= 1) {
        const int lo = k - h >= 0 ? me - h * W : me;
        const int hi = k + h < S ? me + h * W : me;
        const c2<R> ll = cur[lo], lu = cur[ws + lo], lr1 = cur[2 * ws + lo], lr2 = cur[3 * ws + lo];
        const c2<R> hl = cur[hi], hu = cur[ws + hi], hr1 = cur[2 * ws + hi], hr2 = cur[3 * ws + hi];
        // eq_k - l_k eq_{k-h} - u_k eq_{k+h}, then renormalise (operator part shared)
        const c2<R> dg = cmsub<R>(cmsub<R>(mk<R>(R(1), R(0)), yl, lu), yu, hl);
        const c2<R> idg = pivot_rcp<R, FULL>(dg);
        const c2<R> nl = cmul<R>(cmul<R>(yl, ll), idg);
        const c2<R> nu = cmul<R>(cmul<R>(yu, hu), idg);
        yr1 = cmul<R>(cmsub<R>(cmsub<R>(yr1, yl, lr1), yu, hr1), idg);
        yr2 = cmul<R>(cmsub<R>(cmsub<R>(yr2, yl, lr2), yu, hr2), idg);
        yl = mk<R>(-nl.x, -nl.y);
        yu = mk<R>(-nu.x, -nu.y);
        // the other set was last read one level ago, before the previous barrier
        nxt[me] = yl;
        nxt[ws + me] = yu;
        nxt[2 * ws + me] = yr1;
        nxt[3 * ws + me] = yr2;
        __syncthreads();
        c2<R> *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    // x_first of both columns; x_last from this chunk's last equation and the next chunk's first
    const c2<R> xf1 = yr1, xf2 = yr2;
    const int next = k + 1 < S ? me + W : me;  // the last chunk has u1 = 0
    const c2<R> nf1 = cur[2 * ws + next], nf2 = cur[3 * ws + next];
    const c2<R> xl1 = cmsub<R>(cmsub<R>(r1_1, l1, xf1), u1, nf1);
    const c2<R> xl2 = cmsub<R>(cmsub<R>(r1_2, l1, xf2), u1, nf2);

    // ---- back-substitution and store
    c2<R> o1[L], o2[L];
    o1[0] = xf1;
    o2[0] = xf2;
    o1[L - 1] = xl1;
    o2[L - 1] = xl2;
    c2<R> n1 = xl1, n2 = xl2;
#pragma unroll
    for (int i = L - 2; i >= 1; i--) {
        n1 = cmsub<R>(cmsub<R>(rp1[i], sp[i], xf1), mu[i], n1);
        n2 = cmsub<R>(cmsub<R>(rp2[i], sp[i], xf2), mu[i], n2);
        o1[i] = n1;
        o2[i] = n2;
    }
#pragma unroll
    for (int i = 0; i < L; i++) {
        const int m = m0 + i;
        if (live && m < nr) {
            if constexpr (PAIRS) {
                if (store2) {
                    cpair<ST> v;
                    v.a = ccast<ST, R>(o1[i]);
                    v.b = ccast<ST, R>(o2[i]);
                    pcol[(int64_t)m * prs] = v;
                } else {
                    reinterpret_cast<c2<ST> *>(pcol + (int64_t)m * prs)[second ? 1 : 0] = ccast<ST, R>(o1[i]);
                }
            } else {
                col1[(int64_t)m * rs] = ccast<ST, R>(o1[i]);
                if (store2) col2[(int64_t)m * rs] = ccast<ST, R>(o2[i]);
            }
        }
    }

    // step bookkeeping by the last solve of the step (a Cartesian instance's y launch)
    if (!a.use_stage_len && t == 0 && (!CART || a.dir == COL_Y)) {
        if (blockIdx.x == 0) a.state->cnt_row = n + 1;
        if (it.p0 == 0 && it.line == 0) {
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
    const size_t shm = 8 * sizeof(c2<R>) * (size_t)W * S;
    const bool cart = a.dir != COL_RADIAL;
    if constexpr (sizeof(ST) == 4) {  // pair order is an FP32 spectrum's only
        if (a.pair_order) {
            if (!cart)
                hipExtLaunchKernelGGL((col_kernel<R, ST, W, L, false, true>), dim3(grid), dim3(threads),
                                      (uint32_t)shm, s, e0, e1, 0, a);
            else
                hipExtLaunchKernelGGL((col_kernel<R, ST, W, L, true, true>), dim3(grid), dim3(threads),
                                      (uint32_t)shm, s, e0, e1, 0, a);
            return hipGetLastError();
        }
    } else {
        if (a.pair_order) return hipErrorInvalidValue;
    }
    if (!cart)
        hipExtLaunchKernelGGL((col_kernel<R, ST, W, L, false, false>), dim3(grid), dim3(threads), (uint32_t)shm, s,
                              e0, e1, 0, a);
    else
        hipExtLaunchKernelGGL((col_kernel<R, ST, W, L, true, false>), dim3(grid), dim3(threads), (uint32_t)shm, s,
                              e0, e1, 0, a);
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
    // 6 rows per thread: the FP64-arithmetic solve of a pair stays within 168 registers
    // (three wavefronts per SIMD instead of two at 8 rows)
    if (w == 1 && l == 6) return launch_col_t<R, ST, 1, 6>(nr, a, grid, s, e0, e1);
    if (w == 2 && l == 6) return launch_col_t<R, ST, 2, 6>(nr, a, grid, s, e0, e1);
    if (w == 4 && l == 6) return launch_col_t<R, ST, 4, 6>(nr, a, grid, s, e0, e1);
    if (w == 8 && l == 6) return launch_col_t<R, ST, 8, 6>(nr, a, grid, s, e0, e1);
    if (w == 1 && l == 4) return launch_col_t<R, ST, 1, 4>(nr, a, grid, s, e0, e1);
    if (w == 2 && l == 4) return launch_col_t<R, ST, 2, 4>(nr, a, grid, s, e0, e1);
    if (w == 4 && l == 4) return launch_col_t<R, ST, 4, 4>(nr, a, grid, s, e0, e1);
    if (w == 8 && l == 4) return launch_col_t<R, ST, 8, 4>(nr, a, grid, s, e0, e1);
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
