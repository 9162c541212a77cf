/*
 * Host driver that runs the FP64 oracle over a set of its pins, built with
 * the address and undefined-behaviour sanitizers (test infrastructure).
 * Checks: delta -> constant, shifted delta -> W^{n0 k}, tone -> one bin,
 * recursion = direct sum, backward(forward(x)) = N x, unit weight gives
 * grad = 2 N x, H = 1 leaves the matched filter the identity, and every
 * entry point's argument checks.  Exit status 0 when all hold.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_dft_direct(const double *x, double *y, int64_t n, int64_t batch, int sign);
int oracle_fft(const double *x, double *y, int64_t n, int64_t batch, int sign);
int oracle_spectral_energy(const double *x, const double *w, int64_t n, int64_t batch,
                           double *row_loss, double *grad);
int oracle_matched_filter(const double *x, const double *h, int64_t n, int64_t batch,
                          double *out);

static int failures = 0;

static void expect(int cond, const char *what, int64_t n)
{
    if (!cond) {
        printf("FAIL %s n=%lld\n", what, (long long)n);
        ++failures;
    }
}

static double lcg(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

static double max_diff(const double *a, const double *b, int64_t len)
{
    double m = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double d = fabs(a[i] - b[i]);
        if (d > m) m = d;
    }
    return m;
}

static void pins(int64_t n, int64_t batch)
{
    const int64_t len = 2 * n * batch;
    double *x = calloc((size_t)len, sizeof(double));
    double *y = calloc((size_t)len, sizeof(double));
    double *z = calloc((size_t)len, sizeof(double));
    double *w = calloc((size_t)n, sizeof(double));
    double *rows = calloc((size_t)batch, sizeof(double));
    double *h = calloc((size_t)(2 * n), sizeof(double));
    uint64_t s = 12345u + (uint64_t)n;
    const double PI2 = 6.283185307179586476925286766559;

    /* row b: delta at n0 = (7 b) mod n */
    for (int64_t b = 0; b < batch; ++b) x[2 * (b * n + (7 * b) % n)] = 1.0;
    expect(oracle_fft(x, y, n, batch, -1) == 0, "fft rc", n);
    double err = 0.0;
    for (int64_t b = 0; b < batch; ++b) {
        int64_t n0 = (7 * b) % n;
        for (int64_t k = 0; k < n; ++k) {
            double a = -PI2 * (double)((n0 * k) % n) / (double)n;
            err = fmax(err, fabs(y[2 * (b * n + k)] - cos(a)));
            err = fmax(err, fabs(y[2 * (b * n + k) + 1] - sin(a)));
        }
    }
    expect(err <= 1e-12, "shifted delta", n);

    /* tone e^{+2 pi i k0 m / n} -> n at bin k0 */
    const int64_t k0 = (3 * n) / 7;
    for (int64_t m = 0; m < n; ++m) {
        double a = PI2 * (double)((k0 * m) % n) / (double)n;
        x[2 * m] = cos(a);
        x[2 * m + 1] = sin(a);
    }
    expect(oracle_fft(x, y, n, 1, -1) == 0, "tone rc", n);
    err = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double want = k == k0 ? (double)n : 0.0;
        err = fmax(err, fabs(y[2 * k] - want) + fabs(y[2 * k + 1]));
    }
    expect(err <= 1e-9 * (double)n, "tone", n);

    /* random rows: recursion = direct sum; backward(forward(x)) = n x */
    for (int64_t i = 0; i < len; ++i) x[i] = lcg(&s);
    expect(oracle_fft(x, y, n, batch, -1) == 0, "fft rc", n);
    if (n <= 1024) {
        expect(oracle_dft_direct(x, z, n, batch, -1) == 0, "direct rc", n);
        expect(max_diff(y, z, len) <= 1e-12 * (double)n, "recursion vs direct", n);
    }
    expect(oracle_fft(y, z, n, batch, +1) == 0, "backward rc", n);
    for (int64_t i = 0; i < len; ++i) z[i] /= (double)n;
    expect(max_diff(z, x, len) <= 1e-13 * log2((double)n + 1.0), "roundtrip", n);

    /* unit weight: grad = 2 n x and row loss = n ||x_b||^2 */
    for (int64_t k = 0; k < n; ++k) w[k] = 1.0;
    expect(oracle_spectral_energy(x, w, n, batch, rows, z) == 0, "energy rc", n);
    err = 0.0;
    for (int64_t i = 0; i < len; ++i) err = fmax(err, fabs(z[i] - 2.0 * (double)n * x[i]));
    expect(err <= 1e-10 * (double)n, "unit weight gradient", n);
    for (int64_t b = 0; b < batch; ++b) {
        double e2 = 0.0;
        for (int64_t k = 0; k < 2 * n; ++k) e2 += x[2 * b * n + k] * x[2 * b * n + k];
        expect(fabs(rows[b] - (double)n * e2) <= 1e-10 * (double)n * e2, "unit weight loss", n);
    }

    /* H = 1: the matched filter is the identity */
    for (int64_t k = 0; k < n; ++k) h[2 * k] = 1.0, h[2 * k + 1] = 0.0;
    expect(oracle_matched_filter(x, h, n, batch, z) == 0, "filter rc", n);
    expect(max_diff(z, x, len) <= 1e-13 * log2((double)n + 1.0), "identity filter", n);

    free(x), free(y), free(z), free(w), free(rows), free(h);
}

int main(void)
{
    for (int64_t n = 1; n <= 4096; n *= 2) pins(n, 3);
    pins(3, 2);   /* a non-power of two: direct sum */
    pins(48, 2);
    /* argument checks */
    double a[4] = {0}, b[4] = {0};
    expect(oracle_fft(NULL, b, 2, 1, -1) != 0, "null input", 2);
    expect(oracle_fft(a, b, 0, 1, -1) != 0, "zero length", 0);
    expect(oracle_fft(a, b, 2, 1, 0) != 0, "bad sign", 2);
    expect(oracle_fft(a, b, 96, 1, -1) != 0, "non-power of two above 64", 96);
    expect(oracle_spectral_energy(a, NULL, 2, 1, b, b) != 0, "null weight", 2);
    expect(oracle_matched_filter(a, NULL, 2, 1, b) != 0, "null filter", 2);
    expect(oracle_fft(a, b, 2, 0, -1) == 0, "empty batch", 2);
    if (failures) return 1;
    printf("oracle pins clean\n");
    return 0;
}
