/*
 * fcn_oracle.c -- plain, slow, FP64 CPU oracle of the 2D+1 split-step Fourier /
 * Crank-Nicholson (FCN) z-step of Ma & Lin, "Parallel simulation for the ultra-short
 * laser pulses' propagation in air" (arXiv:1507.05988).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP implementation.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or constant with the HIP path.
 *
 * Every routine follows the paper's own order of operations:
 *   - one z-step is NL(dz/2), then the linear part over dz, then NL(dz/2)
 *     (Sec. 3, Eq. nlseq and the serial summary at the end of Sec. 3);
 *   - the linear part is a forward DFT of every r-row, one Crank-Nicholson solve
 *     per frequency column by the chasing (Thomas) method, and an inverse DFT of
 *     every row (Sec. 3.1, Eqs. freqdomainlinear-antifourier and its three loops);
 *   - the nonlinear half step integrates the electron density along t with
 *     classical RK4 and multiplies A by exp(dz/2 N) (Sec. 3.2, Eqs. Anhalf,
 *     Anhalf1, ionization, nonlinearpart).
 * Readings where the paper is silent or misprinted:
 *   - c_j and f_j use (1 + 1/2j): the 1/r term adds +1/(2j dr^2) on A_{j+1}
 *     (derived from Eqs. diff2-diff3; the printed (1 - 1/2j) cancels the 1/r term);
 *   - the plasma term uses omega_pe^2/omega0^2 = rho/rho_c;
 *   - RK4 mid-stage intensity is the mean of the two neighbouring grid intensities,
 *     rho = 0 at the first grid time, intensities taken before the update;
 *   - collisional absorption -(sigma_c/2) rho is an extra switchable term, and so is
 *     avalanche ionisation, a rate (sigma_c / U_i) I rho added to the density equation
 *     (neither is in the paper);
 *   - DFT: forward exp(-i w t) unnormalised, inverse scaled by 1/Nt.
 * All arithmetic is IEEE double.  OpenMP splits rows or columns statically; the loop
 * bodies do not depend on the thread count, so results are bitwise identical for
 * any number of threads (the paper's Sec. 5.1 accuracy statement).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Term switches (the same bit values as the terms mask of the public C interface). */
#define ORC_DIFFRACTION 1u
#define ORC_GVD 2u
#define ORC_KERR 4u
#define ORC_PLASMA 8u
#define ORC_MPA 16u
#define ORC_COLL 32u
#define ORC_AVAL 64u

/* One pulse on its grid.  Field layout: complex [nr][nt], t contiguous, interleaved. */
typedef struct {
    int32_t nr, nt;
    double r_max, t_min, t_max;
    double lambda0, n0, k2;
    double n2, n4, n6, n8;
    int32_t K;
    double sigma_K, rho_at, sigma_c;
    double U_i; /* ionisation potential [J] of the avalanche rate */
    uint32_t terms;
} orc_params;

/* CODATA 2018 values. */
static const double ORC_C = 299792458.0;
static const double ORC_HBAR = 1.054571817e-34;
static const double ORC_ME = 9.1093837015e-31;
static const double ORC_QE = 1.602176634e-19;
static const double ORC_EPS0 = 8.8541878128e-12;

typedef struct {
    double k0;     /* carrier wave number 2 pi n0 / lambda0 */
    double w0;     /* carrier angular frequency 2 pi c / lambda0 */
    double rho_c;  /* critical density eps0 m_e w0^2 / q_e^2, so omega_pe^2/omega0^2 = rho/rho_c */
    double betaK;  /* multiphoton absorption coefficient beta^(K) = K hbar w0 sigma_K rho_at */
    double dr, dtau;
} orc_derived;

static orc_derived derive(const orc_params *p)
{
    orc_derived d;
    d.k0 = 2.0 * M_PI * p->n0 / p->lambda0;
    d.w0 = 2.0 * M_PI * ORC_C / p->lambda0;
    d.rho_c = ORC_EPS0 * ORC_ME * d.w0 * d.w0 / (ORC_QE * ORC_QE);
    d.betaK = (double)p->K * ORC_HBAR * d.w0 * p->sigma_K * p->rho_at;
    d.dr = p->r_max / (double)(p->nr - 1);
    d.dtau = (p->t_max - p->t_min) / (double)p->nt;
    return d;
}

static int bad_params(const orc_params *p)
{
    if (p->nr < 3 || p->nt < 2) return 1;
    if (p->nt & (p->nt - 1)) return 1; /* radix-2 transform */
    if (!(p->r_max > 0.0) || !(p->t_max > p->t_min) || !(p->lambda0 > 0.0) || !(p->n0 > 0.0)) return 1;
    if (p->K < 1) return 1;
    if ((p->terms & ORC_AVAL) && !(p->U_i > 0.0)) return 1;
    return 0;
}

/* ---------------------------------------------------------------- DFT (Sec. 3.1) */

/* tw[k] = exp(-2 pi i k / n) for 0 <= k < n/2, each entry from its own cos/sin call. */
static cplx *make_twiddles(int n)
{
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)(n / 2 > 0 ? n / 2 : 1));
    for (int k = 0; k < n / 2; k++) {
        double ang = -2.0 * M_PI * (double)k / (double)n;
        tw[k] = cos(ang) + I * sin(ang);
    }
    return tw;
}

/* Iterative radix-2 decimation-in-time FFT of one row; forward X_k = sum_j x_j e^{-2 pi i jk/n},
 * inverse uses the conjugate kernel and divides by n. */
static void fft_row(cplx *x, int n, int inverse, const cplx *tw)
{
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            cplx t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, stride = n / len;
        for (int i = 0; i < n; i += len) {
            for (int k = 0; k < half; k++) {
                cplx w = tw[k * stride];
                if (inverse) w = conj(w);
                cplx u = x[i + k];
                cplx v = x[i + k + half] * w;
                x[i + k] = u + v;
                x[i + k + half] = u - v;
            }
        }
    }
    if (inverse) {
        double s = 1.0 / (double)n;
        for (int i = 0; i < n; i++) x[i] *= s;
    }
}

/* First / third loop of the linear part: transform every r-row along t. */
int orc_fft_rows(double *field, int nr, int nt, int inverse, int nthreads)
{
    if (nr < 1 || nt < 2 || (nt & (nt - 1))) return 1;
    cplx *a = (cplx *)field;
    cplx *tw = make_twiddles(nt);
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int m = 0; m < nr; m++) fft_row(a + (size_t)m * nt, nt, inverse, tw);
    free(tw);
    return 0;
}

/* ------------------------------------------------ Crank-Nicholson (Sec. 3.1) */

/* Angular frequency of column p of the unshifted DFT: omega_p = 2 pi q / (Nt dtau),
 * q = p for p < Nt/2 and p - Nt otherwise. */
static double omega_of(int p, int nt, double dtau)
{
    int q = (p < nt / 2) ? p : p - nt;
    return 2.0 * M_PI * (double)q / ((double)nt * dtau);
}

/* Entries of M_abc^p (a: sub-diagonal, b: diagonal, c: super-diagonal) and M_def^p for
 * frequency column p (Eqs. matrix, matrix1 and the coefficient list after them).
 * a[0], c[nr-1], d[0], f[nr-1] are outside the matrices and set to 0. */
static void cn_matrices(const orc_params *pp, const orc_derived *dv, double dz, int p,
                        cplx *a, cplx *b, cplx *c, cplx *d, cplx *e, cplx *f)
{
    const int nr = pp->nr;
    const double kdr2 = dv->k0 * dv->dr * dv->dr;
    const double diff = (pp->terms & ORC_DIFFRACTION) ? 1.0 : 0.0;
    double w = omega_of(p, pp->nt, dv->dtau);
    const double gvd = (pp->terms & ORC_GVD) ? pp->k2 * w * w * dz / 4.0 : 0.0;

    /* j = 0: the axis row from the Neumann condition dA/dr = 0 (Eq. bound). */
    a[0] = 0.0;
    b[0] = 1.0 + I * diff * dz / kdr2 - I * gvd;
    c[0] = -I * diff * dz / kdr2;
    d[0] = 0.0;
    e[0] = 1.0 - I * diff * dz / kdr2 + I * gvd;
    f[0] = I * diff * dz / kdr2;
    for (int j = 1; j <= nr - 2; j++) {
        double lo = 1.0 - 1.0 / (2.0 * j);
        double hi = 1.0 + 1.0 / (2.0 * j); /* corrected sign of the c_j, f_j factor */
        a[j] = -I * diff * dz / (4.0 * kdr2) * lo;
        b[j] = 1.0 + I * diff * dz / (2.0 * kdr2) - I * gvd;
        c[j] = -I * diff * dz / (4.0 * kdr2) * hi;
        d[j] = I * diff * dz / (4.0 * kdr2) * lo;
        e[j] = 1.0 - I * diff * dz / (2.0 * kdr2) + I * gvd;
        f[j] = I * diff * dz / (4.0 * kdr2) * hi;
    }
    /* j = Nr-1: A = 0 at r_max (Eq. bound): a = 0, b = 1, d = e = 0. */
    a[nr - 1] = 0.0;
    b[nr - 1] = 1.0;
    c[nr - 1] = 0.0;
    d[nr - 1] = 0.0;
    e[nr - 1] = 0.0;
    f[nr - 1] = 0.0;
}

/* Exposed for the tests: writes a,b,c,d,e,f (each nr complex) into abcdef (6*nr complex). */
int orc_cn_matrices(const orc_params *pp, double dz, int p, double *abcdef)
{
    if (bad_params(pp) || p < 0 || p >= pp->nt) return 1;
    orc_derived dv = derive(pp);
    cplx *m = (cplx *)abcdef;
    int nr = pp->nr;
    cn_matrices(pp, &dv, dz, p, m, m + nr, m + 2 * nr, m + 3 * nr, m + 4 * nr, m + 5 * nr);
    return 0;
}

/* Chasing method (Thomas algorithm) for a b c x = rhs, no pivoting. */
static void thomas(int n, const cplx *a, const cplx *b, const cplx *c, const cplx *rhs, cplx *x,
                   cplx *cp, cplx *dp)
{
    cp[0] = c[0] / b[0];
    dp[0] = rhs[0] / b[0];
    for (int j = 1; j < n; j++) {
        cplx den = b[j] - a[j] * cp[j - 1];
        cp[j] = (j < n - 1) ? c[j] / den : 0.0;
        dp[j] = (rhs[j] - a[j] * dp[j - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int j = n - 2; j >= 0; j--) x[j] = dp[j] - cp[j] * x[j + 1];
}

/* Second loop of the linear part: for each frequency column p,
 * A~^{n+1}_{.,p} = (M_abc^p)^{-1} M_def^p A~^n_{.,p}.  Field is in the frequency domain. */
int orc_cn_columns(const orc_params *pp, double *field, double dz, int nthreads)
{
    if (bad_params(pp)) return 1;
    orc_derived dv = derive(pp);
    const int nr = pp->nr, nt = pp->nt;
    cplx *A = (cplx *)field;
#pragma omp parallel num_threads(nthreads)
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)nr * 11);
        cplx *a = buf, *b = a + nr, *c = b + nr, *d = c + nr, *e = d + nr, *f = e + nr;
        cplx *col = f + nr, *rhs = col + nr, *x = rhs + nr, *cp = x + nr, *dp = cp + nr;
#pragma omp for schedule(static)
        for (int p = 0; p < nt; p++) {
            cn_matrices(pp, &dv, dz, p, a, b, c, d, e, f);
            for (int j = 0; j < nr; j++) col[j] = A[(size_t)j * nt + p];
            for (int j = 0; j < nr; j++) {
                cplx s = e[j] * col[j];
                if (j > 0) s += d[j] * col[j - 1];
                if (j < nr - 1) s += f[j] * col[j + 1];
                rhs[j] = s;
            }
            thomas(nr, a, b, c, rhs, x, cp, dp);
            for (int j = 0; j < nr; j++) A[(size_t)j * nt + p] = x[j];
        }
        free(buf);
    }
    return 0;
}

/* --------------------------------------------- nonlinear half step (Sec. 3.2) */

/* Right-hand side of the rate equation (Eq. ionization):
 * d rho/dt = beta^(K) / (K hbar w0) |A|^{2K} (1 - rho/rho_at), plus the avalanche rate
 * (sigma_c / U_i) |A|^2 rho when that term is switched on. */
static double rate(const orc_params *pp, const orc_derived *dv, double intensity, double rho)
{
    double coef = dv->betaK / ((double)pp->K * ORC_HBAR * dv->w0);
    double r = coef * pow(intensity, (double)pp->K) * (1.0 - rho / pp->rho_at);
    if (pp->terms & ORC_AVAL) r += pp->sigma_c / pp->U_i * intensity * rho;
    return r;
}

/* Electron density along one row by classical RK4 in t, starting from rho = 0 at the
 * first grid time.  The intensity between grid points is the mean of its neighbours. */
static void rho_row(const orc_params *pp, const orc_derived *dv, const double *inten, double *rho)
{
    const int nt = pp->nt;
    const double h = dv->dtau;
    rho[0] = 0.0;
    if (pp->rho_at <= 0.0) {
        for (int q = 1; q < nt; q++) rho[q] = 0.0;
        return;
    }
    for (int q = 0; q + 1 < nt; q++) {
        double i0 = inten[q], i1 = inten[q + 1], ih = 0.5 * (i0 + i1);
        double r = rho[q];
        double k1 = rate(pp, dv, i0, r);
        double k2 = rate(pp, dv, ih, r + 0.5 * h * k1);
        double k3 = rate(pp, dv, ih, r + 0.5 * h * k2);
        double k4 = rate(pp, dv, i1, r + h * k3);
        rho[q + 1] = r + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
    }
}

int orc_rho_row(const orc_params *pp, const double *inten, double *rho)
{
    if (bad_params(pp)) return 1;
    orc_derived dv = derive(pp);
    rho_row(pp, &dv, inten, rho);
    return 0;
}

/* N for one point (Eq. nonlinearpart, with the readings above). */
static cplx nl_operator(const orc_params *pp, const orc_derived *dv, double inten, double rho)
{
    cplx nhat = 0.0;
    if (pp->terms & ORC_KERR) {
        double kerr = pp->n2 * inten + pp->n4 * inten * inten + pp->n6 * pow(inten, 3.0) +
                      pp->n8 * pow(inten, 4.0);
        nhat += I * (dv->k0 / pp->n0) * kerr;
    }
    if (pp->terms & ORC_PLASMA) nhat += -I * (dv->k0 / 2.0) * (rho / dv->rho_c);
    if (pp->terms & ORC_MPA) nhat += -(dv->betaK / 2.0) * pow(inten, (double)(pp->K - 1));
    if (pp->terms & ORC_COLL) nhat += -(pp->sigma_c / 2.0) * rho;
    return nhat;
}

static int needs_rho(const orc_params *pp) { return (pp->terms & (ORC_PLASMA | ORC_COLL)) != 0; }

/* A <- A exp(hz N) for every point (Eqs. Anhalf / Anhalf1): per row, the intensities
 * are read first, then the density, then the operator, then the update. */
int orc_nl_half(const orc_params *pp, double *field, double hz, int nthreads)
{
    if (bad_params(pp)) return 1;
    orc_derived dv = derive(pp);
    const int nr = pp->nr, nt = pp->nt;
    cplx *A = (cplx *)field;
#pragma omp parallel num_threads(nthreads)
    {
        double *inten = (double *)malloc(sizeof(double) * (size_t)nt * 2);
        double *rho = inten + nt;
#pragma omp for schedule(static)
        for (int m = 0; m < nr; m++) {
            cplx *row = A + (size_t)m * nt;
            for (int q = 0; q < nt; q++) inten[q] = creal(row[q]) * creal(row[q]) + cimag(row[q]) * cimag(row[q]);
            if (needs_rho(pp))
                rho_row(pp, &dv, inten, rho);
            else
                memset(rho, 0, sizeof(double) * (size_t)nt);
            for (int q = 0; q < nt; q++) row[q] *= cexp(hz * nl_operator(pp, &dv, inten[q], rho[q]));
        }
        free(inten);
    }
    return 0;
}

/* ----------------------------------------------------------- one step (Sec. 3) */

static int linear_part(const orc_params *pp, double *field, double dz, int nthreads)
{
    if (orc_fft_rows(field, pp->nr, pp->nt, 0, nthreads)) return 1;
    if (orc_cn_columns(pp, field, dz, nthreads)) return 1;
    return orc_fft_rows(field, pp->nr, pp->nt, 1, nthreads);
}

/* A^{n+1} from A^n: nonlinear half step, linear part over dz, nonlinear half step. */
int orc_step(const orc_params *pp, double *field, double dz, int nthreads)
{
    if (bad_params(pp)) return 1;
    if (orc_nl_half(pp, field, 0.5 * dz, nthreads)) return 1;
    if (linear_part(pp, field, dz, nthreads)) return 1;
    return orc_nl_half(pp, field, 0.5 * dz, nthreads);
}

/* nsteps steps with step lengths dz[0..nsteps-1]. */
int orc_propagate(const orc_params *pp, double *field, int nsteps, const double *dz, int nthreads)
{
    for (int n = 0; n < nsteps; n++)
        if (orc_step(pp, field, dz[n], nthreads)) return 1;
    return 0;
}

/* ------------------------------------------------------------ diagnostics */

/* out[0] energy E = 2 pi dr^2 dtau [ 1/8 sum_p |A_0p|^2 + sum_{m>=1} m sum_p |A_mp|^2 ]
 * out[1] peak intensity, out[2] on-axis peak intensity, out[3] peak electron density,
 * out[4] peak nonlinear phase rate (k0/n0)|sum_j n_2j I^j| + (k0/2) rho/rho_c  [rad/m];
 * fluence[m] = dtau sum_p |A_mp|^2 (may be NULL). */
int orc_diagnostics(const orc_params *pp, const double *field, double *out, double *fluence, int nthreads)
{
    if (bad_params(pp)) return 1;
    orc_derived dv = derive(pp);
    const int nr = pp->nr, nt = pp->nt;
    const cplx *A = (const cplx *)field;
    double *rowsum = (double *)calloc((size_t)nr, sizeof(double));
    double *rowimax = (double *)calloc((size_t)nr, sizeof(double));
    double *rowrho = (double *)calloc((size_t)nr, sizeof(double));
    double *rowphi = (double *)calloc((size_t)nr, sizeof(double));
#pragma omp parallel num_threads(nthreads)
    {
        double *inten = (double *)malloc(sizeof(double) * (size_t)nt * 2);
        double *rho = inten + nt;
#pragma omp for schedule(static)
        for (int m = 0; m < nr; m++) {
            const cplx *row = A + (size_t)m * nt;
            double s = 0.0, imax = 0.0, rmax = 0.0, phimax = 0.0;
            for (int q = 0; q < nt; q++) {
                inten[q] = creal(row[q]) * creal(row[q]) + cimag(row[q]) * cimag(row[q]);
                s += inten[q];
                if (inten[q] > imax) imax = inten[q];
            }
            if (needs_rho(pp))
                rho_row(pp, &dv, inten, rho);
            else
                memset(rho, 0, sizeof(double) * (size_t)nt);
            for (int q = 0; q < nt; q++) {
                double phi = 0.0, x = inten[q];
                if (pp->terms & ORC_KERR)
                    phi += (dv.k0 / pp->n0) *
                           fabs(pp->n2 * x + pp->n4 * x * x + pp->n6 * x * x * x + pp->n8 * x * x * x * x);
                if (pp->terms & ORC_PLASMA) phi += (dv.k0 / 2.0) * rho[q] / dv.rho_c;
                if (phi > phimax) phimax = phi;
                if (rho[q] > rmax) rmax = rho[q];
            }
            rowsum[m] = s;
            rowimax[m] = imax;
            rowrho[m] = rmax;
            rowphi[m] = phimax;
        }
        free(inten);
    }
    double e = 0.125 * rowsum[0];
    double imax = 0.0, rmax = 0.0, phimax = 0.0;
    for (int m = 1; m < nr; m++) e += (double)m * rowsum[m];
    for (int m = 0; m < nr; m++) {
        if (rowimax[m] > imax) imax = rowimax[m];
        if (rowrho[m] > rmax) rmax = rowrho[m];
        if (rowphi[m] > phimax) phimax = rowphi[m];
        if (fluence) fluence[m] = dv.dtau * rowsum[m];
    }
    out[0] = 2.0 * M_PI * dv.dr * dv.dr * dv.dtau * e;
    out[1] = imax;
    out[2] = rowimax[0];
    out[3] = rmax;
    out[4] = phimax;
    free(rowsum);
    free(rowimax);
    free(rowrho);
    free(rowphi);
    return 0;
}

/* Adaptive step length: dz = clamp(max_phase / Phi, dz_min, dz_max). Phi = 0 gives dz_max. */
static double dz_rule(double phi, double max_phase, double dz_min, double dz_max)
{
    double dz = (phi > 0.0) ? max_phase / phi : dz_max;
    if (dz > dz_max) dz = dz_max;
    if (dz < dz_min) dz = dz_min;
    return dz;
}

/* nsteps adaptive steps.  The step from A^n to A^{n+1} uses Phi measured on A^{n-1}
 * (one step of lag); the first step uses Phi of A^0.  dz_log[n] receives each dz. */
int orc_propagate_adaptive(const orc_params *pp, double *field, int nsteps, double max_phase,
                           double dz_min, double dz_max, double *dz_log, int nthreads)
{
    if (bad_params(pp)) return 1;
    double phi_prev = 0.0;
    for (int n = 0; n < nsteps; n++) {
        double diag[5];
        if (orc_diagnostics(pp, field, diag, NULL, nthreads)) return 1;
        double phi_lag = (n == 0) ? diag[4] : phi_prev;
        double dz = dz_rule(phi_lag, max_phase, dz_min, dz_max);
        dz_log[n] = dz;
        if (orc_step(pp, field, dz, nthreads)) return 1;
        phi_prev = diag[4];
    }
    return 0;
}
