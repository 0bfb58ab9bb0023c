/*
 * Plain CPU reference loops for the oracle (test infrastructure only).
 *
 * These are the O(N)-per-call vector operations of the method, written as the
 * plain definitions with no blocking or reordering beyond an OpenMP split of the
 * element loop.  The algorithm around them (coefficients, degree choice, the
 * order of the recurrence) lives in oracle/__init__.py.  Complex values are C99
 * double complex (interleaved re, im), qubit j is bit j of the index.
 *
 * Only tests/, the smoke check and the benchmark's CPU baseline may load this.
 */
#include <complex.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Ising energy of every basis state (section I, H_P diagonal; SK form of the
 * paper's test sets): E(z) = sum_{j<k} J_jk s_j s_k + sum_j h_j s_j with
 * s_j = 1 - 2*bit_j(z); J is the packed row-major upper triangle. */
void orc_energies(int n, const double *h, const double *J, double *E)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) {
        double e = 0.0;
        int64_t p = 0;
        for (int j = 0; j < n; ++j) {
            const double sj = ((z >> j) & 1) ? -1.0 : 1.0;
            e += h[j] * sj;
            for (int k = j + 1; k < n; ++k, ++p) {
                const double sk = ((z >> k) & 1) ? -1.0 : 1.0;
                e += J[p] * sj * sk;
            }
        }
        E[z] = e;
    }
}

/* y = d .* x + g * (sum_j X_j) x, i.e. (H x) for H = diag(d) + g * H_G with
 * H_G = sum_j X_j applied by its definition: (H_G x)[i] = sum_j x[i XOR 2^j]
 * (section I; section II.D states the same operator recursively). */
void orc_hmatvec(int n, const double *d, double g,
                 const double complex *x, double complex *y)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double complex s = 0.0;
        for (int j = 0; j < n; ++j)
            s += x[i ^ ((int64_t)1 << j)];
        y[i] = d[i] * x[i] + g * s;
    }
}

/* One step of the matrix Clenshaw recurrence (section II.B.3, Eq. recursion):
 * out = 2 H b1 - b2 + ck v, with H = diag(d) + g * H_G.  out may alias b2
 * (each element of b2 is read only by the element it overwrites, which is the
 * in-place update of section II.D). */
void orc_clenshaw_step(int n, const double *d, double g, double ckr, double cki,
                       const double complex *v, const double complex *b1,
                       const double complex *b2, double complex *out)
{
    const int64_t N = (int64_t)1 << n;
    const double complex ck = ckr + cki * I;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double complex s = 0.0;
        for (int j = 0; j < n; ++j)
            s += b1[i ^ ((int64_t)1 << j)];
        const double complex hb = d[i] * b1[i] + g * s;
        out[i] = (2.0 * hb - b2[i]) + ck * v[i];
    }
}

/* Final Clenshaw step: out = H b1 - b2 + c0 v (Eq. recursion, last line). */
void orc_clenshaw_final(int n, const double *d, double g, double c0r, double c0i,
                        const double complex *v, const double complex *b1,
                        const double complex *b2, double complex *out)
{
    const int64_t N = (int64_t)1 << n;
    const double complex c0 = c0r + c0i * I;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double complex s = 0.0;
        for (int j = 0; j < n; ++j)
            s += b1[i ^ ((int64_t)1 << j)];
        const double complex hb = d[i] * b1[i] + g * s;
        out[i] = (hb - b2[i]) + c0 * v[i];
    }
}

/* Thread count the OpenMP runtime will use for the loops above. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
