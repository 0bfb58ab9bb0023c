/*
 * Runs the oracle's plain C loops (oracle/ref.c) on small inputs under the
 * address and undefined-behaviour sanitizers (built by
 * tests/test_sanitized_host.py).  Besides the sanitizers' own checks it tests
 * two facts of the definitions: H = diag(d) + g sum_j X_j is symmetric
 * (<x, H y> = <H x, y>), and a Clenshaw step written over b_{k+2} equals the
 * same step written to a separate buffer.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_energies(int n, const double *h, const double *J, double *E);
void orc_hmatvec(int n, const double *d, double g, const double complex *x, double complex *y);
void orc_clenshaw_step(int n, const double *d, double g, double ckr, double cki, const double complex *v,
                       const double complex *b1, const double complex *b2, double complex *out);
void orc_clenshaw_final(int n, const double *d, double g, double c0r, double c0i, const double complex *v,
                        const double complex *b1, const double complex *b2, double complex *out);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double uni(void)   /* xorshift64*, uniform in (-1, 1) */
{
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 2685821657736338717ull) >> 11) / 4503599627370496.0 - 1.0;
}

int main(void)
{
    for (int n = 1; n <= 12; ++n) {
        const int64_t N = (int64_t)1 << n;
        const int np = n * (n - 1) / 2;
        double *h = malloc(sizeof(double) * n), *J = malloc(sizeof(double) * (np ? np : 1));
        double *E = malloc(sizeof(double) * N);
        double complex *x = malloc(sizeof(double complex) * N), *y = malloc(sizeof(double complex) * N);
        double complex *hx = malloc(sizeof(double complex) * N), *hy = malloc(sizeof(double complex) * N);
        double complex *b2 = malloc(sizeof(double complex) * N), *o = malloc(sizeof(double complex) * N);
        for (int j = 0; j < n; ++j) h[j] = uni();
        for (int p = 0; p < np; ++p) J[p] = uni();
        for (int64_t i = 0; i < N; ++i) {
            x[i] = uni() + I * uni();
            y[i] = uni() + I * uni();
            b2[i] = uni() + I * uni();
        }
        orc_energies(n, h, J, E);
        orc_hmatvec(n, E, 0.37, x, hx);
        orc_hmatvec(n, E, 0.37, y, hy);
        double complex a = 0.0, b = 0.0;
        double scale = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            a += conj(x[i]) * hy[i];
            b += conj(hx[i]) * y[i];
            scale += cabs(x[i]) * cabs(hy[i]);
        }
        if (cabs(a - b) > 1e-12 * (scale + 1.0)) {
            fprintf(stderr, "n=%d: <x, Hy> != <Hx, y>\n", n);
            return 1;
        }
        orc_clenshaw_step(n, E, 0.37, 0.25, -0.5, y, x, b2, o);
        orc_clenshaw_step(n, E, 0.37, 0.25, -0.5, y, x, b2, b2);
        for (int64_t i = 0; i < N; ++i)
            if (o[i] != b2[i]) {
                fprintf(stderr, "n=%d: in-place step differs at %lld\n", n, (long long)i);
                return 1;
            }
        orc_clenshaw_final(n, E, 0.37, 1.0, 0.0, y, x, b2, o);
        free(h); free(J); free(E); free(x); free(y); free(hx); free(hy); free(b2); free(o);
    }
    printf("ORACLE LOOPS OK\n");
    return 0;
}
