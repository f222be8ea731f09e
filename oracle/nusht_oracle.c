/*
 * Direct-sum oracle for the spin-0 nonuniform spherical harmonic transform.
 *
 * TEST INFRASTRUCTURE, NOT THE PRODUCT.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What it computes (arXiv:2406.14542, Sec. II.A):
 *   - type 2 / synthesis, Eq. (3), written for a real field:
 *       f_i = sum_l [ a_l0 lam_l0(x_i) + 2 sum_{m=1}^{min(l,M)} Re(a_lm e^{i m phi_i}) lam_lm(x_i) ]
 *     with x_i = cos(theta_i) and lam_lm the orthonormal associated Legendre
 *     function with the Condon-Shortley phase, so that Y_lm = lam_lm(cos theta) e^{i m phi}
 *     (Eq. (1) and its footnote: P_l^m = d^l_{m0} sqrt((2l+1)/4pi)).
 *     The coefficients of negative m follow from a_{l,-m} = (-1)^m conj(a_lm); only
 *     m >= 0 is stored and the imaginary part of a_l0 is ignored.
 *   - type 1 / adjoint, Eq. (2): c_lm = sum_i f_i lam_lm(x_i) e^{-i m phi_i}, 0 <= m <= min(l, M).
 *   - the gradient of the synthesis with respect to theta_i and phi_i.
 *
 * Nothing here is fast on purpose: every point runs the three-term recurrence in l for
 * every m from scratch (O(N L^2)), in IEEE double, with no blocking or symmetry tricks.
 *
 *   lam_mm(x) = (-1)^m sqrt((2m+1)/(4 pi) * prod_{k=1}^m (2k-1)/(2k)) * (1-x^2)^{m/2}
 *   lam_{m+1,m}(x) = x sqrt(2m+3) lam_mm(x)
 *   lam_lm(x) = a_lm (x lam_{l-1,m}(x) - b_lm lam_{l-2,m}(x)),
 *     a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
 *
 * Exponent range: for l of a few thousand, lam_mm drops far below the smallest double
 * near the poles while lam_lm for larger l is of order one again.  The recurrence is
 * therefore run on a mantissa with a separate integer power-of-two exponent shared by
 * the two most recent terms; each value is turned into a plain double (rounding to 0
 * or a subnormal when it is that small) only when it is used.
 *
 * Near the poles cos(theta) cannot carry 1 - cos(theta) to full relative precision, and
 * lam_lm for large l is sensitive to exactly that (d lam / d x ~ l^2).  So every product
 * x * v in the recurrence is formed as v - y v with y = 1 - cos(theta) = 2 sin^2(theta/2)
 * in the northern hemisphere, and as -v + y v with y = 1 + cos(theta) = 2 cos^2(theta/2)
 * in the southern one; it is the same recurrence with x written exactly.
 *
 * Coefficient layout: complex128 interleaved, m-major triangle,
 *   index(l, m) = m (2 lmax + 1 - m) / 2 + l,  m <= l <= lmax.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_D 3.14159265358979323846

/* cos(theta) written as sgn * (1 - y) with y known to full relative precision */
typedef struct {
    double x;   /* cos(theta), for places where plain accuracy is enough */
    double s;   /* sin(theta) */
    double y;   /* 1 - |cos(theta)| */
    int north;  /* theta <= pi/2 */
} angle_t;

static angle_t make_angle(double theta)
{
    angle_t a;
    a.x = cos(theta);
    a.s = sin(theta);
    a.north = theta <= 0.5 * PI_D;
    if (a.north) {
        double h = sin(0.5 * theta);
        a.y = 2.0 * h * h;
    } else {
        double h = cos(0.5 * theta);
        a.y = 2.0 * h * h;
    }
    return a;
}

/* x * v */
static double xmul(const angle_t* a, double v)
{
    return a->north ? v - a->y * v : a->y * v - v;
}

int64_t oracle_nalm(int lmax, int mmax)
{
    return (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
}

static int64_t alm_index(int lmax, int l, int m)
{
    return (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
}

/* Keep |v0|,|v1| away from overflow and underflow by moving a power of two into *e. */
static void renorm2(double* v0, double* v1, int* e)
{
    double big = fabs(*v1) > fabs(*v0) ? fabs(*v1) : fabs(*v0);
    if (big == 0.0) return;
    if (big > 0x1p200 || big < 0x1p-200) {
        int k;
        frexp(big, &k);
        *v0 = ldexp(*v0, -k);
        *v1 = ldexp(*v1, -k);
        *e += k;
    }
}

static void renorm4(double* v0, double* v1, double* d0, double* d1, int* e)
{
    double big = fabs(*v0);
    if (fabs(*v1) > big) big = fabs(*v1);
    if (fabs(*d0) > big) big = fabs(*d0);
    if (fabs(*d1) > big) big = fabs(*d1);
    if (big == 0.0) return;
    if (big > 0x1p200 || big < 0x1p-200) {
        int k;
        frexp(big, &k);
        *v0 = ldexp(*v0, -k);
        *v1 = ldexp(*v1, -k);
        *d0 = ldexp(*d0, -k);
        *d1 = ldexp(*d1, -k);
        *e += k;
    }
}

static double coef_a(int l, int m)
{
    double L = l, M = m;
    return sqrt((4.0 * L * L - 1.0) / (L * L - M * M));
}

static double coef_b(int l, int m)
{
    double L1 = l - 1, M = m;
    return sqrt((L1 * L1 - M * M) / (4.0 * L1 * L1 - 1.0));
}

/* lam_mm as mantissa * 2^exp, advanced from lam_{m-1,m-1} by the factor
   -sqrt((2m+1)/(2m)) * sin(theta). */
static void lam_mm_step(int m, double s, double* mant, int* ex)
{
    int k;
    *mant *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
    if (*mant == 0.0) return;
    *mant = frexp(*mant, &k);
    *ex += k;
}

/* The scaled column: lam_lm(cos theta) = mant[l - m] * 2^ex[l - m] for l = m..lmax, given
   lam_mm = pm * 2^pe.  Every function of this file that needs lam_lm goes through here, and
   so do the pins (oracle_lambda_column). */
static void column_scaled(int lmax, int m, const angle_t* ang, double pm, int pe, double* mant,
                          int* ex)
{
    double v0 = pm, v1;
    int e = pe;
    mant[0] = v0;
    ex[0] = e;
    if (m + 1 > lmax) return;
    v1 = sqrt(2.0 * m + 3.0) * xmul(ang, v0);
    mant[1] = v1;
    ex[1] = e;
    for (int l = m + 2; l <= lmax; ++l) {
        double v2 = coef_a(l, m) * (xmul(ang, v1) - coef_b(l, m) * v0);
        v0 = v1;
        v1 = v2;
        renorm2(&v0, &v1, &e);
        mant[l - m] = v1;
        ex[l - m] = e;
    }
}

/* lam[l - m] = lam_lm(cos theta) as plain doubles (rounded to 0 or a subnormal when that
   small); mant and ex are caller scratch of lmax + 1 entries. */
static void lambda_column(int lmax, int m, const angle_t* ang, double pm, int pe, double* lam,
                          double* mant, int* ex)
{
    column_scaled(lmax, m, ang, pm, pe, mant, ex);
    for (int l = m; l <= lmax; ++l) lam[l - m] = ldexp(mant[l - m], ex[l - m]);
}

/* lam_00 = 1/sqrt(4 pi) as mantissa * 2^exponent */
static void lam_00(double* pm, int* pe)
{
    int k;
    *pm = frexp(1.0 / sqrt(4.0 * PI_D), &k);
    *pe = k;
}

/* Same column and its theta-derivative.  With x = cos(theta), s = sin(theta):
     d lam_mm / d theta = m cos(theta) * [c_m sin^{m-1}(theta)]   (no division by s)
     d lam_l / d theta = a_lm (-s lam_{l-1} + x dlam_{l-1} - b_lm dlam_{l-2}).
   pm1 * 2^pe1 is c_m sin^{m-1} theta (used only for m >= 1). */
static void lambda_column_d(int lmax, int m, const angle_t* ang, double pm, int pe, double pm1,
                            int pe1, double* lam, double* dlam)
{
    double x = ang->x, s = ang->s;
    /* bring both start values onto the same exponent */
    int e = pe;
    double v0 = pm;
    double d0 = 0.0;
    if (m >= 1) d0 = ldexp(m * x * pm1, pe1 - e);
    if (pm == 0.0) { /* lam_mm is exactly zero (pole, m >= 1): use the derivative's exponent */
        e = pe1;
        v0 = 0.0;
        d0 = m * x * pm1;
    }
    lam[0] = ldexp(v0, e);
    dlam[0] = ldexp(d0, e);
    if (m + 1 > lmax) return;
    double a1 = sqrt(2.0 * m + 3.0);
    double v1 = a1 * xmul(ang, v0);
    double d1 = a1 * (-s * v0 + xmul(ang, d0));
    lam[1] = ldexp(v1, e);
    dlam[1] = ldexp(d1, e);
    for (int l = m + 2; l <= lmax; ++l) {
        double a = coef_a(l, m), b = coef_b(l, m);
        double v2 = a * (xmul(ang, v1) - b * v0);
        double d2 = a * (-s * v1 + xmul(ang, d1) - b * d0);
        v0 = v1;
        v1 = v2;
        d0 = d1;
        d1 = d2;
        renorm4(&v0, &v1, &d0, &d1, &e);
        lam[l - m] = ldexp(v1, e);
        dlam[l - m] = ldexp(d1, e);
    }
}

static int pick_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Column of lam_lm(cos theta), l = m..lmax, for the pins: value = mant[l-m] * 2^ex[l-m]
   exactly as the recurrence carries it (no rounding to double range). */
void oracle_lambda_column(int lmax, int m, double theta, double* mant, int* ex)
{
    angle_t ang = make_angle(theta);
    double pm;
    int pe;
    lam_00(&pm, &pe);
    for (int j = 1; j <= m; ++j) lam_mm_step(j, ang.s, &pm, &pe);
    column_scaled(lmax, m, &ang, pm, pe, mant, ex);
}

/* The same column in x87 80-bit long double (range about 1e+-4932), with no exponent
   tracking at all: an independent check of the scaled recurrence above. */
void oracle_lambda_column_ld(int lmax, int m, double theta, double* mant, int* ex)
{
    long double th = theta;
    long double x = cosl(th), s = sinl(th);
    long double v = 1.0L / sqrtl(4.0L * 3.14159265358979323846264338327950288L);
    for (int j = 1; j <= m; ++j) v *= -sqrtl((2.0L * j + 1.0L) / (2.0L * j)) * s;
    long double v0 = v, v1;
    int k;
    mant[0] = (double)frexpl(v0, &k);
    ex[0] = k;
    if (m + 1 > lmax) return;
    v1 = x * sqrtl(2.0L * m + 3.0L) * v0;
    mant[1] = (double)frexpl(v1, &k);
    ex[1] = k;
    for (int l = m + 2; l <= lmax; ++l) {
        long double L = l, M = m, L1 = l - 1;
        long double a = sqrtl((4.0L * L * L - 1.0L) / (L * L - M * M));
        long double b = sqrtl((L1 * L1 - M * M) / (4.0L * L1 * L1 - 1.0L));
        long double v2 = a * (x * v1 - b * v0);
        v0 = v1;
        v1 = v2;
        mant[l - m] = (double)frexpl(v1, &k);
        ex[l - m] = k;
    }
}

/* Type 2, Eq. (3): out[b*npts + i] = f_i for map b. alm: [nmaps][nalm] complex interleaved. */
void oracle_synthesis(int lmax, int mmax, int64_t npts, const double* theta, const double* phi,
                      const double* alm, int nmaps, double* out, int nthreads)
{
    int64_t nalm = oracle_nalm(lmax, mmax);
    int nt = pick_threads(nthreads);
#pragma omp parallel num_threads(nt)
    {
        double* lam = (double*)malloc(sizeof(double) * (lmax + 1));
        double* mant = (double*)malloc(sizeof(double) * (lmax + 1));
        int* ex = (int*)malloc(sizeof(int) * (lmax + 1));
        double* acc = (double*)malloc(sizeof(double) * 2 * nmaps);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < npts; ++i) {
            angle_t ang = make_angle(theta[i]);
            double pm;
            int pe;
            lam_00(&pm, &pe);
            for (int b = 0; b < nmaps; ++b) out[(int64_t)b * npts + i] = 0.0;
            for (int m = 0; m <= mmax; ++m) {
                if (m > 0) lam_mm_step(m, ang.s, &pm, &pe);
                lambda_column(lmax, m, &ang, pm, pe, lam, mant, ex);
                for (int b = 0; b < 2 * nmaps; ++b) acc[b] = 0.0;
                for (int l = m; l <= lmax; ++l) {
                    const double* a = alm + 2 * alm_index(lmax, l, m);
                    for (int b = 0; b < nmaps; ++b) {
                        acc[2 * b] += a[2 * b * nalm] * lam[l - m];
                        acc[2 * b + 1] += a[2 * b * nalm + 1] * lam[l - m];
                    }
                }
                double c = cos(m * phi[i]), sn = sin(m * phi[i]);
                for (int b = 0; b < nmaps; ++b) {
                    double v;
                    if (m == 0)
                        v = acc[2 * b];
                    else
                        v = 2.0 * (acc[2 * b] * c - acc[2 * b + 1] * sn);
                    out[(int64_t)b * npts + i] += v;
                }
            }
        }
        free(lam);
        free(mant);
        free(ex);
        free(acc);
    }
}

/* Type 1, Eq. (2), restricted to the m-columns listed in mlist (each 0 <= m <= lmax).
   out: [nmaps][ncols][lmax+1] complex interleaved; entry l < m is left zero.
   Per-thread partial sums are reduced in thread order, so the result does not depend
   on scheduling for a fixed thread count. */
void oracle_adjoint_columns(int lmax, int64_t npts, const double* theta, const double* phi,
                            const double* f, int nmaps, int ncols, const int* mlist, double* out,
                            int nthreads)
{
    int nt = pick_threads(nthreads);
    int maxm = 0;
    for (int c = 0; c < ncols; ++c)
        if (mlist[c] > maxm) maxm = mlist[c];
    /* column slot of each m (the listed m must be distinct) */
    int* slot = (int*)malloc(sizeof(int) * (maxm + 1));
    for (int m = 0; m <= maxm; ++m) slot[m] = -1;
    for (int c = 0; c < ncols; ++c) slot[mlist[c]] = c;
    size_t per = (size_t)nmaps * ncols * (lmax + 1) * 2;
    double* part = (double*)calloc(per * nt, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* mine = part + per * tid;
        double* lam = (double*)malloc(sizeof(double) * (lmax + 1));
        double* mant = (double*)malloc(sizeof(double) * (lmax + 1));
        int* ex = (int*)malloc(sizeof(int) * (lmax + 1));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < npts; ++i) {
            angle_t ang = make_angle(theta[i]);
            double pm;
            int pe;
            lam_00(&pm, &pe);
            int mcur = 0;
            /* visit the columns in increasing m so lam_mm can be advanced incrementally */
            for (int m = 0; m <= maxm; ++m) {
                if (m > mcur) {
                    lam_mm_step(m, ang.s, &pm, &pe);
                    mcur = m;
                }
                int c = slot[m];
                if (c < 0) continue;
                lambda_column(lmax, m, &ang, pm, pe, lam, mant, ex);
                double cr = cos(m * phi[i]), ci = -sin(m * phi[i]);
                for (int b = 0; b < nmaps; ++b) {
                    double fv = f[(int64_t)b * npts + i];
                    double* dst = mine + (((size_t)b * ncols + c) * (lmax + 1)) * 2;
                    for (int l = m; l <= lmax; ++l) {
                        dst[2 * l] += fv * lam[l - m] * cr;
                        dst[2 * l + 1] += fv * lam[l - m] * ci;
                    }
                }
            }
        }
        free(lam);
        free(mant);
        free(ex);
    }
    memset(out, 0, sizeof(double) * per);
    for (int t = 0; t < nt; ++t)
        for (size_t j = 0; j < per; ++j) out[j] += part[per * t + j];
    free(part);
    free(slot);
}

/* Full type 1 into the m-major triangle: out [nmaps][nalm] complex interleaved. */
void oracle_adjoint(int lmax, int mmax, int64_t npts, const double* theta, const double* phi,
                    const double* f, int nmaps, double* out, int nthreads)
{
    int64_t nalm = oracle_nalm(lmax, mmax);
    int ncols = mmax + 1;
    int* ml = (int*)malloc(sizeof(int) * ncols);
    for (int m = 0; m <= mmax; ++m) ml[m] = m;
    double* cols = (double*)malloc(sizeof(double) * 2 * (size_t)nmaps * ncols * (lmax + 1));
    oracle_adjoint_columns(lmax, npts, theta, phi, f, nmaps, ncols, ml, cols, nthreads);
    for (int b = 0; b < nmaps; ++b)
        for (int m = 0; m <= mmax; ++m)
            for (int l = m; l <= lmax; ++l) {
                const double* src = cols + (((size_t)b * ncols + m) * (lmax + 1) + l) * 2;
                double* dst = out + 2 * ((int64_t)b * nalm + alm_index(lmax, l, m));
                dst[0] = src[0];
                dst[1] = src[1];
            }
    free(cols);
    free(ml);
}

/* Synthesis plus its derivatives with respect to the point coordinates:
     f_i, df/dtheta_i, df/dphi_i = sum 2 Re(i m a_lm e^{i m phi}) lam_lm. */
void oracle_synthesis_grad(int lmax, int mmax, int64_t npts, const double* theta,
                           const double* phi, const double* alm, int nmaps, double* f,
                           double* dth, double* dph, int nthreads)
{
    int64_t nalm = oracle_nalm(lmax, mmax);
    int nt = pick_threads(nthreads);
#pragma omp parallel num_threads(nt)
    {
        double* lam = (double*)malloc(sizeof(double) * (lmax + 1));
        double* lam_d = (double*)malloc(sizeof(double) * (lmax + 1));
        double* dlam = (double*)malloc(sizeof(double) * (lmax + 1));
        double* mant = (double*)malloc(sizeof(double) * (lmax + 1));
        int* ex = (int*)malloc(sizeof(int) * (lmax + 1));
        double* acc = (double*)malloc(sizeof(double) * 4 * nmaps);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < npts; ++i) {
            angle_t ang = make_angle(theta[i]);
            /* pm*2^pe = c_m s^m ; pm1*2^pe1 = c_m s^(m-1) */
            double pm, pm1 = 0.0;
            int pe, pe1 = 0, k;
            lam_00(&pm, &pe);
            for (int b = 0; b < nmaps; ++b) {
                f[(int64_t)b * npts + i] = 0.0;
                dth[(int64_t)b * npts + i] = 0.0;
                dph[(int64_t)b * npts + i] = 0.0;
            }
            for (int m = 0; m <= mmax; ++m) {
                if (m > 0) {
                    /* c_m s^(m-1) = -sqrt((2m+1)/(2m)) * c_{m-1} s^(m-1) */
                    pm1 = -sqrt((2.0 * m + 1.0) / (2.0 * m)) * pm;
                    pe1 = pe;
                    if (pm1 != 0.0) {
                        pm1 = frexp(pm1, &k);
                        pe1 += k;
                    }
                    lam_mm_step(m, ang.s, &pm, &pe);
                }
                /* lam from the shared scaled column; the forward-mode recurrence is used
                   for the derivative only */
                lambda_column(lmax, m, &ang, pm, pe, lam, mant, ex);
                lambda_column_d(lmax, m, &ang, pm, pe, pm1, pe1, lam_d, dlam);
                for (int b = 0; b < 4 * nmaps; ++b) acc[b] = 0.0;
                for (int l = m; l <= lmax; ++l) {
                    const double* a = alm + 2 * alm_index(lmax, l, m);
                    for (int b = 0; b < nmaps; ++b) {
                        double ar = a[2 * b * nalm], ai = a[2 * b * nalm + 1];
                        acc[4 * b + 0] += ar * lam[l - m];
                        acc[4 * b + 1] += ai * lam[l - m];
                        acc[4 * b + 2] += ar * dlam[l - m];
                        acc[4 * b + 3] += ai * dlam[l - m];
                    }
                }
                double c = cos(m * phi[i]), sn = sin(m * phi[i]);
                for (int b = 0; b < nmaps; ++b) {
                    double gr = acc[4 * b], gi = acc[4 * b + 1];
                    double dr = acc[4 * b + 2], di = acc[4 * b + 3];
                    int64_t o = (int64_t)b * npts + i;
                    if (m == 0) {
                        f[o] += gr;
                        dth[o] += dr;
                    } else {
                        f[o] += 2.0 * (gr * c - gi * sn);
                        dth[o] += 2.0 * (dr * c - di * sn);
                        /* d/dphi Re(G e^{i m phi}) = Re(i m G e^{i m phi}) = -m Im(G e^{i m phi}) */
                        dph[o] += -2.0 * m * (gr * sn + gi * c);
                    }
                }
            }
        }
        free(lam);
        free(lam_d);
        free(dlam);
        free(mant);
        free(ex);
        free(acc);
    }
}
