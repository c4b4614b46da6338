/*
 * fcn_cartesian.c -- plain, slow, FP64 CPU oracle of the linear part of the FCN z-step on a
 * Cartesian transverse grid, Delta_perp = d2/dx2 + d2/dy2 (the alternative transverse
 * operator named beside Eq. nlse of Ma & Lin, arXiv:1507.05988, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or constant with the HIP
 * path.  The transforms along t and the nonlinear half steps of a Cartesian step are the
 * radial oracle's own routines applied to the nx * ny rows of the field (neither depends on
 * the transverse geometry); this file adds only what the geometry changes.
 *
 * Reading (the paper discretises only the radial Laplacian, Sec. 3.1): in the frequency
 * domain every column p obeys dA~/dz = (Lx + Ly) A~ with
 *   Lx = (i/2k0) d2/dx2 + i k'' omega_p^2 / 4,   Ly = (i/2k0) d2/dy2 + i k'' omega_p^2 / 4
 * (the GVD term of Eq. freqdomainlinear split evenly between the two axes).  The linear part
 * applies the paper's Crank-Nicholson scheme (Eqs. diff1-diff2) to one axis at a time,
 *   A* = (1 - dz/2 Lx)^-1 (1 + dz/2 Lx) A~^n,   A~^{n+1} = (1 - dz/2 Ly)^-1 (1 + dz/2 Ly) A*,
 * each a tridiagonal system per (line, p) solved by the chasing (Thomas) method.  On the
 * tensor-product grid Lx and Ly commute, so this product equals the Peaceman-Rachford
 * alternating-direction form of the two-dimensional Crank-Nicholson step, second order in dz.
 * Grid: x_i = -x_max + i dx, dx = 2 x_max / (nx - 1), i < nx (y likewise); A = 0 on the four
 * walls (the Cartesian counterpart of A = 0 at r_max, Eq. bound), so rows 0 and n-1 of every
 * system are identity rows with a zero right-hand side.
 * Field layout: complex [ny][nx][nt], t contiguous, interleaved.
 * All arithmetic is IEEE double; OpenMP splits lines statically and the loop bodies do not
 * depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_DIFFRACTION 1u
#define ORC_GVD 2u

typedef struct {
    int32_t nx, ny, nt;
    double x_max, y_max, t_min, t_max;
    double lambda0, n0, k2;
    uint32_t terms;
} orc_cart;

static int bad_cart(const orc_cart *c)
{
    if (c->nx < 3 || c->ny < 3 || c->nt < 2) return 1;
    if (!(c->x_max > 0.0) || !(c->y_max > 0.0) || !(c->t_max > c->t_min)) return 1;
    if (!(c->lambda0 > 0.0) || !(c->n0 > 0.0)) return 1;
    return 0;
}

/* omega_p = 2 pi q / (Nt dtau), q = p for p < Nt/2 and p - Nt otherwise (unshifted DFT). */
static double omega_of(int p, int nt, double dtau)
{
    int q = (p < nt / 2) ? p : p - nt;
    return 2.0 * M_PI * (double)q / ((double)nt * dtau);
}

/* Chasing method for a tridiagonal system a_j x_{j-1} + b_j x_j + c_j x_{j+1} = r_j. */
static void chase(int n, const cplx *a, const cplx *b, const cplx *c, const cplx *r, cplx *x, cplx *cp,
                  cplx *dp)
{
    cp[0] = c[0] / b[0];
    dp[0] = r[0] / b[0];
    for (int j = 1; j < n; j++) {
        cplx den = b[j] - a[j] * cp[j - 1];
        cp[j] = (j < n - 1) ? c[j] / den : 0.0;
        dp[j] = (r[j] - a[j] * dp[j - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int j = n - 2; j >= 0; j--) x[j] = dp[j] - cp[j] * x[j + 1];
}

/* Crank-Nicholson matrices of one axis (n points, spacing h) for frequency column p:
 * (1 - dz/2 L) has sub/super-diagonal -i dz/(4 k0 h^2) and diagonal
 * 1 + i dz/(2 k0 h^2) - i k'' omega_p^2 dz / 8; (1 + dz/2 L) the conjugate signs of the
 * i-terms.  Rows 0 and n-1 are the walls: identity on the left, zero on the right. */
static void axis_matrices(const orc_cart *c, int n, double h, double dz, int p, cplx *a, cplx *b, cplx *cc,
                          cplx *d, cplx *e, cplx *f)
{
    const double k0 = 2.0 * M_PI * c->n0 / c->lambda0;
    const double dtau = (c->t_max - c->t_min) / (double)c->nt;
    const double diff = (c->terms & ORC_DIFFRACTION) ? dz / (4.0 * k0 * h * h) : 0.0;
    const double w = omega_of(p, c->nt, dtau);
    const double gvd = (c->terms & ORC_GVD) ? c->k2 * w * w * dz / 8.0 : 0.0;
    for (int j = 0; j < n; j++) {
        if (j == 0 || j == n - 1) {
            a[j] = 0.0;
            b[j] = 1.0;
            cc[j] = 0.0;
            d[j] = 0.0;
            e[j] = 0.0;
            f[j] = 0.0;
            continue;
        }
        a[j] = -I * diff;
        b[j] = 1.0 + I * 2.0 * diff - I * gvd;
        cc[j] = -I * diff;
        d[j] = I * diff;
        e[j] = 1.0 - I * 2.0 * diff + I * gvd;
        f[j] = I * diff;
    }
}

/* Exposed for the tests: the six diagonals (each n complex) of axis 0 (x) or 1 (y). */
int orc_cart_matrices(const orc_cart *c, int axis, double dz, int p, double *abcdef)
{
    if (bad_cart(c) || axis < 0 || axis > 1 || p < 0 || p >= c->nt) return 1;
    const int n = axis == 0 ? c->nx : c->ny;
    const double h = axis == 0 ? 2.0 * c->x_max / (double)(c->nx - 1) : 2.0 * c->y_max / (double)(c->ny - 1);
    cplx *m = (cplx *)abcdef;
    axis_matrices(c, n, h, dz, p, m, m + n, m + 2 * n, m + 3 * n, m + 4 * n, m + 5 * n);
    return 0;
}

/* One axis of the linear part on a spectrum [ny][nx][nt]: for every frequency column p and
 * every line of the other axis, A~ <- (M_abc)^-1 M_def A~ along the axis. */
int orc_cart_cn_axis(const orc_cart *c, double *field, double dz, int axis, int nthreads)
{
    if (bad_cart(c) || axis < 0 || axis > 1) return 1;
    const int nx = c->nx, ny = c->ny, nt = c->nt;
    const int n = axis == 0 ? nx : ny;         /* unknowns per system */
    const int lines = axis == 0 ? ny : nx;     /* systems per frequency */
    const double h = axis == 0 ? 2.0 * c->x_max / (double)(nx - 1) : 2.0 * c->y_max / (double)(ny - 1);
    const size_t stride = axis == 0 ? (size_t)nt : (size_t)nx * nt;  /* between consecutive unknowns */
    cplx *A = (cplx *)field;
#pragma omp parallel num_threads(nthreads)
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n * 11);
        cplx *a = buf, *b = a + n, *cc = b + n, *d = cc + n, *e = d + n, *f = e + n;
        cplx *col = f + n, *rhs = col + n, *x = rhs + n, *cp = x + n, *dp = cp + n;
#pragma omp for schedule(static)
        for (int p = 0; p < nt; p++) {
            axis_matrices(c, n, h, dz, p, a, b, cc, d, e, f);
            for (int line = 0; line < lines; line++) {
                const size_t base = (axis == 0 ? (size_t)line * nx * nt : (size_t)line * nt) + (size_t)p;
                for (int j = 0; j < n; j++) col[j] = A[base + (size_t)j * stride];
                for (int j = 0; j < n; j++) {
                    cplx s = e[j] * col[j];
                    if (j > 0) s += d[j] * col[j - 1];
                    if (j < n - 1) s += f[j] * col[j + 1];
                    rhs[j] = s;
                }
                chase(n, a, b, cc, rhs, x, cp, dp);
                for (int j = 0; j < n; j++) A[base + (size_t)j * stride] = x[j];
            }
        }
        free(buf);
    }
    return 0;
}
