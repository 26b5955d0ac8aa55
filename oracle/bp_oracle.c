/*
 * FP64 reference backprojection and forward projection (test infrastructure).
 *
 * This file is part of the CPU oracle.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product library never
 * does.  It shares no code, header or table with the HIP library.
 *
 * Operation (paper, Section 2.2 and the "LineRec" item of Section 3: direct
 * discretisation of the backprojection line integral with linear
 * interpolation):
 *
 *   f[z][iy][ix] = scale * sum_a ( (1-w) Q(j0) + w Q(j0+1) )
 *     x = ix - floor(N/2),  y = iy - floor(N/2)
 *     s = x cos(theta_a) + y sin(theta_a) + center      (detector coordinate)
 *     j0 = floor(s),  w = s - j0
 *     Q(j) = q[z][a][j] for 0 <= j < n_det, else 0
 *
 * In the 16-bit mode (paper, Section 2.1: 16-bit arithmetic, higher
 * precision where accuracy needs it) the two weights are held as IEEE
 * binary16 numbers: (1-w) and w are each rounded to the nearest binary16
 * value (ties to even), products and sums stay exact/FP64 here.  Flag w16.
 *
 * The forward projector is the transpose of that map with scale 1: every
 * voxel deposits (1-w) f into bin j0 and w f into bin j0+1 of each angle.
 * Both are written in double precision with libm sin/cos, in the plainest
 * loop order.  OpenMP only splits independent outputs over threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}


/* Nearest IEEE binary16 value of a finite x with |x| < 65504, ties to even:
 * binary16 keeps 11 significant bits, and below 2^-14 (subnormals) a fixed
 * spacing of 2^-24.  x / ulp is exact (ulp is a power of two) and nearbyint
 * rounds ties to even in the default rounding mode. */
static double round_binary16(double x)
{
    if (x == 0.0) return x;
    int e;
    (void)frexp(fabs(x), &e);          /* |x| = m 2^e, m in [0.5, 1): leading bit 2^(e-1) */
    int lead = e - 1;
    if (lead < -14) lead = -14;
    const double ulp = ldexp(1.0, lead - 10);
    return nearbyint(x / ulp) * ulp;
}

double oracle_round_binary16(double x) { return round_binary16(x); }

/* The two interpolation weights of one tap pair. */
static void tap_weights(double w, int w16, double *wa, double *wb)
{
    if (w16) {
        *wa = round_binary16(1.0 - w);
        *wb = round_binary16(w);
    } else {
        *wa = 1.0 - w;
        *wb = w;
    }
}

/* q: [nz][na][n] filtered rows; f: [nz][N][N] output (overwritten). */
void oracle_backproject(const double *q, int64_t nz, int64_t na, int64_t n,
                        const double *angles, double center, int64_t N,
                        double scale, int w16, double *f)
{
    const int64_t half = N / 2;
    double *ct = (double *)malloc((size_t)na * sizeof(double));
    double *st = (double *)malloc((size_t)na * sizeof(double));
    for (int64_t a = 0; a < na; ++a) { ct[a] = cos(angles[a]); st[a] = sin(angles[a]); }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t iy = 0; iy < N; ++iy) {
            const double y = (double)(iy - half);
            for (int64_t ix = 0; ix < N; ++ix) {
                const double x = (double)(ix - half);
                double acc = 0.0;
                for (int64_t a = 0; a < na; ++a) {
                    const double s = x * ct[a] + y * st[a] + center;
                    const double fl = floor(s);
                    const int64_t j0 = (int64_t)fl;
                    const double w = s - fl;
                    const double *row = q + (z * na + a) * n;
                    const double q0 = (j0 >= 0 && j0 < n) ? row[j0] : 0.0;
                    const double q1 = (j0 + 1 >= 0 && j0 + 1 < n) ? row[j0 + 1] : 0.0;
                    double wa, wb;
                    tap_weights(w, w16, &wa, &wb);
                    acc += wa * q0 + wb * q1;
                }
                f[(z * N + iy) * N + ix] = scale * acc;
            }
        }
    }
    free(ct);
    free(st);
}

/* Backprojection of one slice evaluated only at listed voxels (for sampled
 * checks of large volumes).  q: [na][n]; out[k] is the value at (ix[k], iy[k]). */
void oracle_backproject_points(const double *q, int64_t na, int64_t n,
                               const double *angles, double center, int64_t N,
                               double scale, int w16, const int64_t *ix, const int64_t *iy,
                               int64_t npts, double *out)
{
    const int64_t half = N / 2;
    double *ct = (double *)malloc((size_t)na * sizeof(double));
    double *st = (double *)malloc((size_t)na * sizeof(double));
    for (int64_t a = 0; a < na; ++a) { ct[a] = cos(angles[a]); st[a] = sin(angles[a]); }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < npts; ++k) {
        const double x = (double)(ix[k] - half);
        const double y = (double)(iy[k] - half);
        double acc = 0.0;
        for (int64_t a = 0; a < na; ++a) {
            const double s = x * ct[a] + y * st[a] + center;
            const double fl = floor(s);
            const int64_t j0 = (int64_t)fl;
            const double w = s - fl;
            const double *row = q + a * n;
            const double q0 = (j0 >= 0 && j0 < n) ? row[j0] : 0.0;
            const double q1 = (j0 + 1 >= 0 && j0 + 1 < n) ? row[j0 + 1] : 0.0;
            double wa, wb;
            tap_weights(w, w16, &wa, &wb);
            acc += wa * q0 + wb * q1;
        }
        out[k] = scale * acc;
    }
    free(ct);
    free(st);
}

/* f: [nz][N][N]; sino: [nz][na][n] output (overwritten).  Scatter form of the
 * transpose: each (slice, angle) row is owned by one thread, so the order of
 * additions into a bin is the fixed voxel order. */
void oracle_radon(const double *f, int64_t nz, int64_t N, const double *angles,
                  double center, int64_t na, int64_t n, double *sino)
{
    const int64_t half = N / 2;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t a = 0; a < na; ++a) {
            double *row = sino + (z * na + a) * n;
            memset(row, 0, (size_t)n * sizeof(double));
            const double c = cos(angles[a]), sn = sin(angles[a]);
            for (int64_t iy = 0; iy < N; ++iy) {
                const double y = (double)(iy - half);
                for (int64_t ix = 0; ix < N; ++ix) {
                    const double x = (double)(ix - half);
                    const double v = f[(z * N + iy) * N + ix];
                    const double s = x * c + y * sn + center;
                    const double fl = floor(s);
                    const int64_t j0 = (int64_t)fl;
                    const double w = s - fl;
                    if (j0 >= 0 && j0 < n) row[j0] += (1.0 - w) * v;
                    if (j0 + 1 >= 0 && j0 + 1 < n) row[j0 + 1] += w * v;
                }
            }
        }
    }
}

/*
 * Fourier-domain backprojection ("FourierRec", paper Sections 2.2 and 3: the
 * backprojection evaluated with exponentials in the frequency domain instead
 * of linear interpolation in space).  What that method evaluates, written out
 * without any gridding or fast transform:
 *
 *   f(x, y) = scale * sum_a y_a(m_a),   m_a = x cos(theta_a) + y sin(theta_a) + pos0
 *   y_a(m)  = (1/L) Re sum_{k=-L/2}^{L/2} w_k Y_a[k mod L] exp(2 pi i k m / L)
 *   w_k = 1/2 for k = -L/2 and k = L/2, else 1
 *
 * y_a is the real trigonometric interpolant of the padded filtered row whose
 * DFT is Y_a (length L); pos0 is the padded-row position of the rotation axis.
 * Y: one slice, [na][L] complex as separate real and imaginary arrays.
 * Output at the listed voxels (ix[p], iy[p]); x = ix - floor(N/2), likewise y.
 */
void oracle_fourier_backproject_points(const double *Yre, const double *Yim, int64_t na, int64_t L,
                                       const double *angles, double pos0, int64_t N, double scale,
                                       const int64_t *ix, const int64_t *iy, int64_t npts, double *out)
{
    const int64_t half = N / 2;
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npts; ++p) {
        const double x = (double)(ix[p] - half);
        const double y = (double)(iy[p] - half);
        double acc = 0.0;
        for (int64_t a = 0; a < na; ++a) {
            const double m = x * cos(angles[a]) + y * sin(angles[a]) + pos0;
            const double *yr = Yre + a * L;
            const double *yi = Yim + a * L;
            double row = 0.0;
            for (int64_t k = -L / 2; k <= L / 2; ++k) {
                const double wk = (k == -L / 2 || k == L / 2) ? 0.5 : 1.0;
                const int64_t kk = ((k % L) + L) % L;
                const double ph = two_pi * (double)k * m / (double)L;
                /* Re(Y exp(i ph)) */
                row += wk * (yr[kk] * cos(ph) - yi[kk] * sin(ph));
            }
            acc += row / (double)L;
        }
        out[p] = scale * acc;
    }
}

/*
 * Laminographic backprojection (paper, Section 2.2: the direct line-integral
 * backprojector is kept because it also serves laminographic geometry, where
 * the rotation axis is tilted with respect to the beam).  Reading of the
 * geometry: rotation axis tilted by phi from the beam (phi = pi/2 is
 * ordinary tomography); at rotation angle theta the voxel (x, y, z) is seen
 * at detector column u and row v
 *
 *   u = x cos(theta) + y sin(theta) + center_u
 *   v = (-x sin(theta) + y cos(theta)) cos(phi) + z sin(phi) + center_v
 *
 * with x = ix - floor(N/2), y = iy - floor(N/2), z = iz - floor(Nz/2), and
 *
 *   f(ix, iy, iz) = scale * sum_a  bilinear(Q_a, v, u)
 *
 * where Q_a is the filtered projection [rows][n] of angle a and taps outside
 * the detector read zero.  q: [na][rows][n].  Output at the listed voxels.
 */
static double lam_tap(const double *img, int64_t rows, int64_t n, int64_t r, int64_t c)
{
    return (r >= 0 && r < rows && c >= 0 && c < n) ? img[r * n + c] : 0.0;
}

void oracle_lamino_backproject_points(const double *q, int64_t na, int64_t rows, int64_t n,
                                      const double *angles, double center_u, double center_v,
                                      double phi, int64_t N, int64_t Nz, double scale,
                                      const int64_t *ix, const int64_t *iy, const int64_t *iz,
                                      int64_t npts, double *out)
{
    const double cphi = cos(phi), sphi = sin(phi);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        const double x = (double)(ix[p] - N / 2);
        const double y = (double)(iy[p] - N / 2);
        const double z = (double)(iz[p] - Nz / 2);
        double acc = 0.0;
        for (int64_t a = 0; a < na; ++a) {
            const double c = cos(angles[a]), s = sin(angles[a]);
            const double u = x * c + y * s + center_u;
            const double v = (-x * s + y * c) * cphi + z * sphi + center_v;
            const double fu = floor(u), fv = floor(v);
            const int64_t c0 = (int64_t)fu, r0 = (int64_t)fv;
            const double wu = u - fu, wv = v - fv;
            const double *img = q + a * rows * n;
            const double top = (1.0 - wu) * lam_tap(img, rows, n, r0, c0) + wu * lam_tap(img, rows, n, r0, c0 + 1);
            const double bot = (1.0 - wu) * lam_tap(img, rows, n, r0 + 1, c0) + wu * lam_tap(img, rows, n, r0 + 1, c0 + 1);
            acc += (1.0 - wv) * top + wv * bot;
        }
        out[p] = scale * acc;
    }
}
