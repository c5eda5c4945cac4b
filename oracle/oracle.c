/*
 * FP64 CPU oracle for the correlation of two unions of balls.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark load it.  It shares no code, header or table with the
 * HIP path.
 *
 * What it computes (Behandish & Ilies, "Analytic Methods for Geometric Modeling
 * via Spherical Decomposition"):
 *
 *  - A shape is a union of balls whose defining function is the weighted sum of
 *    ball indicators (union as a sum, Sec. 2.1 eq. eq_un; weighted knots,
 *    Sec. 2.2 eq. eq_Psum; closed L2 balls, eq. eq_L2ball; the indicator is the
 *    alpha -> infinity limit of the bump kernel, eq. eq_psi).
 *  - The score of B moved by (R, t) against A is the inner product
 *    g(R, t) = <f_A, f_{(R,t)B}> (Sec. 3.1 eq. eq_relg_0), with the motion
 *    acting as x -> R x + t (App. B).
 *
 * o1_*: the plain method.  The inner product of two ball indicators is the
 * volume of their intersection (the null-volume lemma, Sec. 2.1 eq. eq_null),
 * a closed-form lens volume V(d; a, b).  Summing over all pairs gives g.
 *
 * o2_*: the band-limited Fourier route.  Each ball's indicator has the radial
 * Fourier transform Bhat(k; r) = 4 pi (sin kr - kr cos kr) / k^3; the shape
 * transform is the knot NDFT weighted by it (Sec. 2.5 eq. eq_rhoPhat, with the
 * CFT convention of App. C eq. eq_CFT_int); the correlation spectrum is
 * F_A * conj(F_RB) (Sec. 3.2 eq. eq_ccghat).  The modes kept are
 * k = 2 pi m / L for |m_d| < N/2 on an L-periodic box; the Nyquist planes are
 * left at zero.  The inverse transform to the translation grid is done in
 * Python with an FP64 FFT.
 *
 * lift_*: the 4D lifted correlation (Sec. 2.2 eq. eq_rhoA, eq_L2cone,
 * eq_coneconv; Sec. 3.1 Lemma 2, eq. eq_ORA, eq_convgA).  Knot (x, r) of the
 * fixed shape carries the half-cone {(y, s) : |y - x| <= r - s, s <= r}
 * (trimmed far below every height used here), knot (y0, rho) of the moved
 * shape its r-mirror, the upward cone {(y, s) : |y - y0| <= rho + s,
 * s >= -rho}; the moved shape's cones are translated by the 4D lifted
 * translation (t, h).  A pair's 4D intersection is the set of (y, s) with
 * |y - x| + |y - (R y0 + t)| <= r + rho - h, whose 4D volume
 * W(d; P) = integral over y of (P - |y - p| - |y - q|)_+ is, with
 * P = r + rho - h and d = |p - q|,
 *     W(d; P) = pi (P^2 - d^2)^2 / 24   for d < P, else 0
 * (at each height s it is the lens volume of two balls whose radii sum to P,
 * integrated over s).  The slice at height h of the lifted correlation is the
 * sum of c_i d_j W over pairs; its 3D Fourier transform in t is
 *     What(k; P) = 4 pi^2 (x^3 cos x - 6 x^2 sin x - 15 x cos x + 15 sin x) / (3 k^7),
 * x = k P, which equals integral_0^P Bhat(k; u) Bhat(k; P - u) du.
 *
 * raster_*: the uniform-grid baseline of Sec. 5.2 / Sec. 6.2 (rasterize each
 * union, correlate the two grids).  The fixed shape is sampled at
 * origin + h u, the moved shape (turned by R) at h v, u, v in [0, n)^3 (v
 * read periodically as -n/2 .. n/2-1), a sample being 1 when it lies in some
 * ball (|p - c|^2 <= r^2 in FP64).  The count at translation index t is
 * sum_u a(u) b(u - t) with periodic indices: the number of grid samples
 * where the fixed shape meets the moved one translated by origin + h t; its
 * volume estimate is h^3 times the count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Lens volume: volume of B(0, a) intersected with B(d e, b).
 * Zero when the balls are apart (d >= a + b); the smaller ball's volume when
 * one contains the other (d <= |a - b|); otherwise the sum of two spherical
 * caps, which reduces to pi (a+b-d)^2 (d^2 + 2d(a+b) - 3(a-b)^2) / (12 d). */
double orc_lens_volume(double d, double a, double b)
{
    if (d >= a + b) return 0.0;
    if (d <= fabs(a - b)) {
        double m = a < b ? a : b;
        return 4.0 * M_PI * m * m * m / 3.0;
    }
    double s = a + b - d;
    return M_PI * s * s * (d * d + 2.0 * d * (a + b) - 3.0 * (a - b) * (a - b)) / (12.0 * d);
}

/* Fourier transform of the indicator of B(0, r) at |k| (angular wavenumber,
 * transform kernel exp(-i k.x)).  For kr < 0.5 the Taylor series of
 * sin x - x cos x = sum_{n>=1} (-1)^{n+1} 2n x^{2n+1} / (2n+1)! is summed
 * instead, since the closed form cancels there. */
double orc_ball_ft(double k, double r)
{
    double x = k * r;
    if (x < 0.5) {
        /* (sin x - x cos x) / x^3 = sum_{n>=1} (-1)^{n+1} 2n x^{2n-2} / (2n+1)! */
        double sum = 0.0, xp = 1.0, fact = 6.0;
        for (int n = 1; n <= 12; ++n) {
            double t = 2.0 * n * xp / fact;
            sum += (n % 2 == 1) ? t : -t;
            xp *= x * x;
            fact *= (2.0 * n + 2.0) * (2.0 * n + 3.0);
        }
        return 4.0 * M_PI * r * r * r * sum;
    }
    return 4.0 * M_PI * (sin(x) - x * cos(x)) / (k * k * k);
}

/* Rotation matrix (row-major) of the unit quaternion q = (w, x, y, z),
 * Hamilton convention, normalised here. */
void orc_quat_to_rot(const double *q, double *R)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void rotate(const double *R, const double *p, double *out)
{
    out[0] = R[0] * p[0] + R[1] * p[1] + R[2] * p[2];
    out[1] = R[3] * p[0] + R[4] * p[1] + R[5] * p[2];
    out[2] = R[6] * p[0] + R[7] * p[1] + R[8] * p[2];
}

/* Plain score at arbitrary translations: for each t,
 * sum_i sum_j c_i d_j V(|x_i - (R y_j + t)|; r_i, rho_j).
 * Balls are rows (x, y, z, r, w). */
void orc_o1_points(const double *A, int64_t nA, const double *B, int64_t nB,
                   const double *R, const double *t, int64_t nt, double *out)
{
    double *rb = (double *)malloc(sizeof(double) * 3 * (size_t)(nB > 0 ? nB : 1));
    for (int64_t j = 0; j < nB; ++j) rotate(R, B + 5 * j, rb + 3 * j);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < nt; ++p) {
        double acc = 0.0;
        for (int64_t i = 0; i < nA; ++i) {
            const double *a = A + 5 * i;
            for (int64_t j = 0; j < nB; ++j) {
                double dx = a[0] - (rb[3 * j + 0] + t[3 * p + 0]);
                double dy = a[1] - (rb[3 * j + 1] + t[3 * p + 1]);
                double dz = a[2] - (rb[3 * j + 2] + t[3 * p + 2]);
                double d = sqrt(dx * dx + dy * dy + dz * dz);
                acc += a[4] * B[5 * j + 4] * orc_lens_volume(d, a[3], B[5 * j + 3]);
            }
        }
        out[p] = acc;
    }
    free(rb);
}

/* Plain score on the grid t = origin + h * (ix, iy, iz), 0 <= i < n, stored
 * [iz][iy][ix].  Walks the pairs instead of the translations: pair (i, j)
 * contributes only where |x_i - R y_j - t| < r_i + rho_j, so only grid points
 * in that ball's bounding box are visited; every skipped term is zero.
 * Not periodic.  Work is split over z-slabs so that no two threads write the
 * same output. */
void orc_o1_grid(const double *A, int64_t nA, const double *B, int64_t nB,
                 const double *R, const double *origin, double h, int n, double *out)
{
    size_t total = (size_t)n * n * n;
    memset(out, 0, sizeof(double) * total);
    double *rb = (double *)malloc(sizeof(double) * 3 * (size_t)(nB > 0 ? nB : 1));
    for (int64_t j = 0; j < nB; ++j) rotate(R, B + 5 * j, rb + 3 * j);
#pragma omp parallel for schedule(dynamic, 1)
    for (int iz = 0; iz < n; ++iz) {
        double tz = origin[2] + h * iz;
        for (int64_t i = 0; i < nA; ++i) {
            const double *a = A + 5 * i;
            for (int64_t j = 0; j < nB; ++j) {
                double reach = a[3] + B[5 * j + 3];
                /* centre of the support ball in translation space */
                double cx = a[0] - rb[3 * j + 0], cy = a[1] - rb[3 * j + 1], cz = a[2] - rb[3 * j + 2];
                if (fabs(tz - cz) >= reach) continue;
                int x0 = (int)ceil((cx - reach - origin[0]) / h), x1 = (int)floor((cx + reach - origin[0]) / h);
                int y0 = (int)ceil((cy - reach - origin[1]) / h), y1 = (int)floor((cy + reach - origin[1]) / h);
                if (x0 < 0) x0 = 0;
                if (y0 < 0) y0 = 0;
                if (x1 > n - 1) x1 = n - 1;
                if (y1 > n - 1) y1 = n - 1;
                double w = a[4] * B[5 * j + 4];
                for (int iy = y0; iy <= y1; ++iy) {
                    double ty = origin[1] + h * iy;
                    for (int ix = x0; ix <= x1; ++ix) {
                        double tx = origin[0] + h * ix;
                        double dx = cx - tx, dy = cy - ty, dz = cz - tz;
                        double d = sqrt(dx * dx + dy * dy + dz * dz);
                        out[((size_t)iz * n + iy) * n + ix] += w * orc_lens_volume(d, a[3], B[5 * j + 3]);
                    }
                }
            }
        }
    }
    free(rb);
}

/* Signed mode number stored at index i of an n-point axis (FFT order). */
static int mode_of(int i, int n) { return i < n / 2 ? i : i - n; }

/* Band-limited shape spectrum F(k_m) = sum_i c_i Bhat(|k_m|; r_i) exp(-i k_m . R x_i)
 * with k_m = 2 pi m / L, for every m with |m_d| < n/2, stored in FFT order as
 * re/im[mz][my][mx] (n^3 each); entries with some m_d = -n/2 stay zero.
 * exp(-i k.x) is the product of its three axis factors, each from cos/sin;
 * Bhat is evaluated once per knot for each distinct |m|^2.  Knots are taken in
 * chunks only so that these per-knot tables stay small: every mode still adds
 * the knots' terms in knot order. */
#define ORC_CHUNK 64
void orc_o2_spectrum(const double *balls, int64_t nb, const double *R, int n, double L,
                     double *re, double *im)
{
    size_t total = (size_t)n * n * n;
    memset(re, 0, sizeof(double) * total);
    memset(im, 0, sizeof(double) * total);
    int half = n / 2;
    int m2max = 3 * (half - 1) * (half - 1);
    double dk = 2.0 * M_PI / L;
    double *bt = (double *)malloc(sizeof(double) * ORC_CHUNK * (size_t)(m2max + 1));
    double *ef = (double *)malloc(sizeof(double) * ORC_CHUNK * 6 * (size_t)n); /* [knot][axis][i][re,im] */
    double *cw = (double *)malloc(sizeof(double) * ORC_CHUNK);
    for (int64_t b0 = 0; b0 < nb; b0 += ORC_CHUNK) {
        int cnt = (int)((nb - b0) < ORC_CHUNK ? (nb - b0) : ORC_CHUNK);
#pragma omp parallel for schedule(static)
        for (int c = 0; c < cnt; ++c) {
            const double *ball = balls + 5 * (b0 + c);
            double p[3];
            rotate(R, ball, p);
            cw[c] = ball[4];
            for (int m2 = 0; m2 <= m2max; ++m2)
                bt[(size_t)c * (m2max + 1) + m2] = orc_ball_ft(dk * sqrt((double)m2), ball[3]);
            for (int ax = 0; ax < 3; ++ax)
                for (int i = 0; i < n; ++i) {
                    double ph = dk * mode_of(i, n) * p[ax];
                    double *e = ef + (((size_t)c * 3 + ax) * n + i) * 2;
                    e[0] = cos(ph);
                    e[1] = -sin(ph);
                }
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int iz = 0; iz < n; ++iz) {
            int mz = mode_of(iz, n);
            if (mz == -half) continue;
            for (int c = 0; c < cnt; ++c) {
                const double *ex = ef + ((size_t)c * 3 + 0) * n * 2;
                const double *ey = ef + ((size_t)c * 3 + 1) * n * 2;
                const double *ez = ef + ((size_t)c * 3 + 2) * n * 2 + 2 * iz;
                const double *b = bt + (size_t)c * (m2max + 1);
                for (int iy = 0; iy < n; ++iy) {
                    int my = mode_of(iy, n);
                    if (my == -half) continue;
                    double yr = ez[0] * ey[2 * iy] - ez[1] * ey[2 * iy + 1];
                    double yi = ez[0] * ey[2 * iy + 1] + ez[1] * ey[2 * iy];
                    size_t row = ((size_t)iz * n + iy) * n;
                    for (int ix = 0; ix < n; ++ix) {
                        int mx = mode_of(ix, n);
                        if (mx == -half) continue;
                        double s = cw[c] * b[mx * mx + my * my + mz * mz];
                        re[row + ix] += s * (yr * ex[2 * ix] - yi * ex[2 * ix + 1]);
                        im[row + ix] += s * (yr * ex[2 * ix + 1] + yi * ex[2 * ix]);
                    }
                }
            }
        }
    }
    free(bt); free(ef); free(cw);
}

/* ---- 4D lifted correlation ------------------------------------------------ */

/* 4D volume of the intersection of a downward and an upward cone whose apex
 * heights differ by P (radii summing to P at every common height) and whose
 * axes are d apart. */
double orc_lift_w(double d, double P)
{
    if (!(P > 0.0) || d >= P) return 0.0;
    double u = P * P - d * d;
    return M_PI * u * u / 24.0;
}

/* 3D Fourier transform of t -> W(|t|; P) at |k| (kernel exp(-i k.t)).  For
 * x = k P < 2 the closed form cancels to x^7 and the Taylor series
 * P^7 (4 pi^2 / 3) sum_n (-1)^n (2n+2)(2n+4)(2n+6) x^(2n) / (2n+7)! is summed
 * until a term falls below 1e-18 of the sum; zero for P <= 0. */
double orc_lift_what(double k, double P)
{
    if (!(P > 0.0)) return 0.0;
    double x = k * P;
    if (x < 2.0) {
        double x2 = x * x, term = 1.0, sum = 0.0;
        double fact = 5040.0; /* (2n+7)! at n = 0 */
        for (int n = 0; n < 40; ++n) {
            double c = (2.0 * n + 2) * (2.0 * n + 4) * (2.0 * n + 6) / fact;
            double t = ((n & 1) ? -1.0 : 1.0) * c * term;
            sum += t;
            if (fabs(t) < 1e-18 * fabs(sum)) break;
            term *= x2;
            fact *= (2.0 * n + 8) * (2.0 * n + 9);
        }
        double p2 = P * P;
        return 4.0 * M_PI * M_PI / 3.0 * p2 * p2 * p2 * P * sum;
    }
    double k2 = k * k, k7 = k2 * k2 * k2 * k;
    return 4.0 * M_PI * M_PI *
           (x * x * x * cos(x) - 6.0 * x * x * sin(x) - 15.0 * x * cos(x) + 15.0 * sin(x)) / (3.0 * k7);
}

/* Plain slice at height h of the lifted correlation on the grid
 * t = origin + hs * (ix, iy, iz), [iz][iy][ix], not periodic:
 * sum_ij c_i d_j W(|x_i - R y_j - t|; r_i + rho_j - h), pair by pair over
 * the grid points of each pair's support (every skipped term is zero). */
void orc_o1_lift_grid(const double *A, int64_t nA, const double *B, int64_t nB, const double *R,
                      const double *origin, double hs, int n, double h, double *out)
{
    size_t total = (size_t)n * n * n;
    memset(out, 0, sizeof(double) * total);
    double *rb = (double *)malloc(sizeof(double) * 3 * (size_t)(nB > 0 ? nB : 1));
    for (int64_t j = 0; j < nB; ++j) rotate(R, B + 5 * j, rb + 3 * j);
#pragma omp parallel for schedule(dynamic, 1)
    for (int iz = 0; iz < n; ++iz) {
        double tz = origin[2] + hs * iz;
        for (int64_t i = 0; i < nA; ++i) {
            const double *a = A + 5 * i;
            for (int64_t j = 0; j < nB; ++j) {
                double P = a[3] + B[5 * j + 3] - h;
                if (!(P > 0.0)) continue;
                double cx = a[0] - rb[3 * j + 0], cy = a[1] - rb[3 * j + 1], cz = a[2] - rb[3 * j + 2];
                if (fabs(tz - cz) >= P) continue;
                int x0 = (int)ceil((cx - P - origin[0]) / hs), x1 = (int)floor((cx + P - origin[0]) / hs);
                int y0 = (int)ceil((cy - P - origin[1]) / hs), y1 = (int)floor((cy + P - origin[1]) / hs);
                if (x0 < 0) x0 = 0;
                if (y0 < 0) y0 = 0;
                if (x1 > n - 1) x1 = n - 1;
                if (y1 > n - 1) y1 = n - 1;
                double w = a[4] * B[5 * j + 4];
                for (int iy = y0; iy <= y1; ++iy) {
                    double ty = origin[1] + hs * iy;
                    for (int ix = x0; ix <= x1; ++ix) {
                        double tx = origin[0] + hs * ix;
                        double dx = cx - tx, dy = cy - ty, dz = cz - tz;
                        out[((size_t)iz * n + iy) * n + ix] += w * orc_lift_w(sqrt(dx * dx + dy * dy + dz * dz), P);
                    }
                }
            }
        }
    }
    free(rb);
}

/* Band-limited spectrum of the slice at height h:
 * G(k_m) = sum_ij c_i d_j What(|k_m|; r_i + rho_j - h) exp(-i k_m . (x_i - R y_j)),
 * k_m = 2 pi m / L, |m_d| < n/2, in FFT order re/im[mz][my][mx] (Nyquist
 * planes zero).  This is the 4D product rho_A conj(rho_RB) fhat_D^2
 * (eq. eq_convgA) brought back to height h, summed pair by pair: a pair's
 * phase is the product of its three axis factors; What is tabulated per pair
 * over the distinct |m|^2.  Threads split the z-planes of the output. */
void orc_o2_lift_spectrum(const double *A, int64_t nA, const double *B, int64_t nB, const double *R, int n,
                          double L, double h, double *re, double *im)
{
    size_t total = (size_t)n * n * n;
    memset(re, 0, sizeof(double) * total);
    memset(im, 0, sizeof(double) * total);
    int half = n / 2;
    int m2max = 3 * (half - 1) * (half - 1);
    double dk = 2.0 * M_PI / L;
    double *rb = (double *)malloc(sizeof(double) * 3 * (size_t)(nB > 0 ? nB : 1));
    for (int64_t j = 0; j < nB; ++j) rotate(R, B + 5 * j, rb + 3 * j);
#pragma omp parallel
    {
        double *tab = (double *)malloc(sizeof(double) * (size_t)(m2max + 1));
        double *ef = (double *)malloc(sizeof(double) * 4 * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int iz = 0; iz < n; ++iz) {
            int mz = iz < half ? iz : iz - n;
            if (mz == -half) continue;
            for (int64_t i = 0; i < nA; ++i) {
                const double *a = A + 5 * i;
                for (int64_t j = 0; j < nB; ++j) {
                    double P = a[3] + B[5 * j + 3] - h;
                    if (!(P > 0.0)) continue;
                    double w = a[4] * B[5 * j + 4];
                    double p[3] = {a[0] - rb[3 * j], a[1] - rb[3 * j + 1], a[2] - rb[3 * j + 2]};
                    for (int m2 = 0; m2 <= m2max; ++m2) tab[m2] = w * orc_lift_what(dk * sqrt((double)m2), P);
                    for (int ax = 0; ax < 2; ++ax)
                        for (int q = 0; q < n; ++q) {
                            double ph = dk * (q < half ? q : q - n) * p[ax];
                            ef[(ax * n + q) * 2] = cos(ph);
                            ef[(ax * n + q) * 2 + 1] = -sin(ph);
                        }
                    double phz = dk * mz * p[2];
                    double zr = cos(phz), zi = -sin(phz);
                    for (int iy = 0; iy < n; ++iy) {
                        int my = iy < half ? iy : iy - n;
                        if (my == -half) continue;
                        const double *ey = ef + (n + iy) * 2;
                        double yr = zr * ey[0] - zi * ey[1], yi = zr * ey[1] + zi * ey[0];
                        size_t row = ((size_t)iz * n + iy) * n;
                        for (int ix = 0; ix < n; ++ix) {
                            int mx = ix < half ? ix : ix - n;
                            if (mx == -half) continue;
                            const double *ex = ef + ix * 2;
                            double s = tab[mx * mx + my * my + mz * mz];
                            re[row + ix] += s * (yr * ex[0] - yi * ex[1]);
                            im[row + ix] += s * (yr * ex[1] + yi * ex[0]);
                        }
                    }
                }
            }
        }
        free(tab);
        free(ef);
    }
    free(rb);
}

/* ---- rasterization baseline ------------------------------------------------ */

static int inside_any(const double *p, const double *c, const double *r2, int64_t nb)
{
    for (int64_t i = 0; i < nb; ++i) {
        double dx = p[0] - c[3 * i], dy = p[1] - c[3 * i + 1], dz = p[2] - c[3 * i + 2];
        if (dx * dx + dy * dy + dz * dz <= r2[i]) return 1;
    }
    return 0;
}

/* The two sample grids, [z][y][x] bytes: a(u) of A at origin + h u, b(v) of
 * R B at h v with v the signed index of FFT order (v - n for v >= n/2). */
void orc_raster_bitmaps(const double *A, int64_t nA, const double *B, int64_t nB, const double *R,
                        const double *origin, double h, int n, unsigned char *a, unsigned char *b)
{
    double *ca = (double *)malloc(sizeof(double) * 3 * (size_t)(nA > 0 ? nA : 1));
    double *ra = (double *)malloc(sizeof(double) * (size_t)(nA > 0 ? nA : 1));
    double *cb = (double *)malloc(sizeof(double) * 3 * (size_t)(nB > 0 ? nB : 1));
    double *rb = (double *)malloc(sizeof(double) * (size_t)(nB > 0 ? nB : 1));
    for (int64_t i = 0; i < nA; ++i) {
        ca[3 * i] = A[5 * i];
        ca[3 * i + 1] = A[5 * i + 1];
        ca[3 * i + 2] = A[5 * i + 2];
        ra[i] = A[5 * i + 3] * A[5 * i + 3];
    }
    for (int64_t j = 0; j < nB; ++j) {
        rotate(R, B + 5 * j, cb + 3 * j);
        rb[j] = B[5 * j + 3] * B[5 * j + 3];
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                size_t i = ((size_t)z * n + y) * n + x;
                double pa[3] = {origin[0] + h * x, origin[1] + h * y, origin[2] + h * z};
                double pb[3] = {h * (x < n / 2 ? x : x - n), h * (y < n / 2 ? y : y - n), h * (z < n / 2 ? z : z - n)};
                a[i] = (unsigned char)inside_any(pa, ca, ra, nA);
                b[i] = (unsigned char)inside_any(pb, cb, rb, nB);
            }
    free(ca); free(ra); free(cb); free(rb);
}

/* counts[k] = sum_u a(u) b(u - t_k) (periodic indices) at the translation
 * indices t_k = (tx, ty, tz) of idx[3k..3k+2]. */
void orc_raster_counts(const unsigned char *a, const unsigned char *b, int n, const int *idx, int64_t nt,
                       int64_t *counts)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nt; ++k) {
        int tx = idx[3 * k], ty = idx[3 * k + 1], tz = idx[3 * k + 2];
        int64_t c = 0;
        for (int z = 0; z < n; ++z) {
            int bz = ((z - tz) % n + n) % n;
            for (int y = 0; y < n; ++y) {
                int by = ((y - ty) % n + n) % n;
                const unsigned char *ar = a + ((size_t)z * n + y) * n;
                const unsigned char *br = b + ((size_t)bz * n + by) * n;
                for (int x = 0; x < n; ++x) c += ar[x] & br[((x - tx) % n + n) % n];
            }
        }
        counts[k] = c;
    }
}

/* Threads of the OpenMP loops above (timing only: results do not depend on
 * it, every output element is summed by one thread in a fixed order). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int orc_get_threads(void) { return omp_get_max_threads(); }
