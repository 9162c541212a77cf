/*
 * FP64 CPU oracle for the batched complex DFT.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library itself never does.  It shares no code, header, table or constant
 * with the GPU path.
 *
 * Data layout: complex values are stored as interleaved (re, im) doubles,
 * batch-major, row b element n at index 2*(b*n_len + n).
 *
 * What is computed (the paper, Section II-A, the DFT definition):
 *     X[k] = sum_{n=0}^{N-1} x[n] * exp(sign * 2*pi*i * n*k / N)
 * with sign = -1 for the forward transform (W_N = e^{-2 pi i / N}) and
 * sign = +1 for the backward transform.  Neither direction is scaled.
 *
 * Two independent routes to the same result:
 *   oracle_dft_direct   the O(N^2) sum itself, any N >= 1;
 *   oracle_fft          recursive radix-2 decimation in time (the N = 2*(N/2)
 *                       case of the Cooley-Tukey factorization, Section II-A
 *                       eq. (1)), bottoming out in the direct sum at N <= 64.
 * Every root of unity is evaluated directly with cos/sin of an exactly
 * reduced argument (m mod N); nothing is obtained by a recurrence.
 *
 * oracle_spectral_energy is the reference for the differentiable transform:
 *     L = sum_b sum_k w_k^2 |Y_b[k]|^2,   Y_b = F x_b,
 *     dL/dRe x + i dL/dIm x = F^H (2 w^2 .* Y_b)
 * (F is symmetric, so F^H is the backward, sign = +1, unscaled transform).
 *
 * oracle_matched_filter is the reference for the fused range-compression
 * chain named in the paper's future work (Section IX-A): out = F^{-1}(conj(H) .* F x).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_DIRECT_MAX 64

static const double ORACLE_TWO_PI = 6.28318530717958647692528676655900577;

/* exp(sign * 2 pi i m / n) for 0 <= m < n, evaluated directly in FP64. */
static void unit_root(int64_t m, int64_t n, int sign, double *re, double *im)
{
    double ang = ORACLE_TWO_PI * (double)m / (double)n;
    *re = cos(ang);
    *im = (double)sign * sin(ang);
}

/* Direct DFT of n elements read with element stride xs (in complex units). */
static void dft_direct_strided(const double *x, int64_t xs, double *out,
                               int64_t n, int sign, double *roots)
{
    for (int64_t m = 0; m < n; ++m)
        unit_root(m, n, sign, &roots[2 * m], &roots[2 * m + 1]);
    for (int64_t k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t m = (j * k) % n;           /* exponent reduced exactly */
            double wr = roots[2 * m], wi = roots[2 * m + 1];
            double xr = x[2 * j * xs], xi = x[2 * j * xs + 1];
            sr += xr * wr - xi * wi;
            si += xr * wi + xi * wr;
        }
        out[2 * k] = sr;
        out[2 * k + 1] = si;
    }
}

/* Radix-2 DIT: transform of the even-indexed half into out[0, n/2), of the
 * odd-indexed half into out[n/2, n), then X[k] = E[k] + w^k O[k] and
 * X[k + n/2] = E[k] - w^k O[k], w = exp(sign 2 pi i / n). */
static void fft_recursive(const double *x, int64_t xs, double *out, int64_t n,
                          int sign, double *roots)
{
    if (n <= ORACLE_DIRECT_MAX) {
        dft_direct_strided(x, xs, out, n, sign, roots);
        return;
    }
    int64_t h = n / 2;
    fft_recursive(x, 2 * xs, out, h, sign, roots);
    fft_recursive(x + 2 * xs, 2 * xs, out + 2 * h, h, sign, roots);
    for (int64_t k = 0; k < h; ++k) {
        double wr, wi;
        unit_root(k, n, sign, &wr, &wi);
        double er = out[2 * k], ei = out[2 * k + 1];
        double orr = out[2 * (h + k)], oi = out[2 * (h + k) + 1];
        double tr = wr * orr - wi * oi;
        double ti = wr * oi + wi * orr;
        out[2 * k] = er + tr;
        out[2 * k + 1] = ei + ti;
        out[2 * (h + k)] = er - tr;
        out[2 * (h + k) + 1] = ei - ti;
    }
}

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

static int check_args(const void *x, const void *y, int64_t n, int64_t batch, int sign)
{
    if (!x || !y) return -1;
    if (n < 1 || batch < 0) return -2;
    if (sign != -1 && sign != 1) return -3;
    return 0;
}

int oracle_version(void) { return 1; }

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Direct O(N^2) DFT of every row; any n >= 1. */
int oracle_dft_direct(const double *x, double *y, int64_t n, int64_t batch, int sign)
{
    int rc = check_args(x, y, n, batch, sign);
    if (rc) return rc;
    int fail = 0;
#pragma omp parallel
    {
        double *roots = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        if (!roots) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < batch; ++b)
            if (roots) dft_direct_strided(x + 2 * b * n, 1, y + 2 * b * n, n, sign, roots);
        free(roots);
    }
    return fail ? -4 : 0;
}

/* Recursive radix-2 FFT of every row; n a power of two, or any n <= 64. */
int oracle_fft(const double *x, double *y, int64_t n, int64_t batch, int sign)
{
    int rc = check_args(x, y, n, batch, sign);
    if (rc) return rc;
    if (n > ORACLE_DIRECT_MAX && !is_pow2(n)) return -2;
    int fail = 0;
#pragma omp parallel
    {
        double *roots = (double *)malloc(sizeof(double) * 2 * ORACLE_DIRECT_MAX);
        if (!roots) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < batch; ++b)
            if (roots) fft_recursive(x + 2 * b * n, 1, y + 2 * b * n, n, sign, roots);
        free(roots);
    }
    return fail ? -4 : 0;
}

/* Loss and gradient of L = sum_b sum_k w_k^2 |(F x_b)[k]|^2.
 * row_loss[b] receives the per-row sum, grad receives F^H(2 w^2 .* F x_b). */
int oracle_spectral_energy(const double *x, const double *w, int64_t n, int64_t batch,
                           double *row_loss, double *grad)
{
    if (!x || !w || !row_loss || !grad) return -1;
    if (n < 1 || batch < 0) return -2;
    if (n > ORACLE_DIRECT_MAX && !is_pow2(n)) return -2;
    int fail = 0;
#pragma omp parallel
    {
        double *roots = (double *)malloc(sizeof(double) * 2 * ORACLE_DIRECT_MAX);
        double *yb = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        if (!roots || !yb) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < batch; ++b) {
            if (!roots || !yb) continue;
            fft_recursive(x + 2 * b * n, 1, yb, n, -1, roots);
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                double w2 = w[k] * w[k];
                double yr = yb[2 * k], yi = yb[2 * k + 1];
                acc += w2 * (yr * yr + yi * yi);
                yb[2 * k] = 2.0 * w2 * yr;
                yb[2 * k + 1] = 2.0 * w2 * yi;
            }
            row_loss[b] = acc;
            fft_recursive(yb, 1, grad + 2 * b * n, n, +1, roots);
        }
        free(roots);
        free(yb);
    }
    return fail ? -4 : 0;
}

/* out_b = F^{-1}(conj(H) .* F x_b) with F^{-1} = (1/N) * backward transform;
 * h is one complex filter spectrum of length n shared by every row. */
int oracle_matched_filter(const double *x, const double *h, int64_t n, int64_t batch,
                          double *out)
{
    if (!x || !h || !out) return -1;
    if (n < 1 || batch < 0) return -2;
    if (n > ORACLE_DIRECT_MAX && !is_pow2(n)) return -2;
    int fail = 0;
#pragma omp parallel
    {
        double *roots = (double *)malloc(sizeof(double) * 2 * ORACLE_DIRECT_MAX);
        double *yb = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        if (!roots || !yb) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < batch; ++b) {
            if (!roots || !yb) continue;
            fft_recursive(x + 2 * b * n, 1, yb, n, -1, roots);
            for (int64_t k = 0; k < n; ++k) {
                double hr = h[2 * k], hi = -h[2 * k + 1];   /* conj(H_k) */
                double yr = yb[2 * k], yi = yb[2 * k + 1];
                yb[2 * k] = hr * yr - hi * yi;
                yb[2 * k + 1] = hr * yi + hi * yr;
            }
            double *ob = out + 2 * b * n;
            fft_recursive(yb, 1, ob, n, +1, roots);
            for (int64_t k = 0; k < 2 * n; ++k) ob[k] /= (double)n;
        }
        free(roots);
        free(yb);
    }
    return fail ? -4 : 0;
}
