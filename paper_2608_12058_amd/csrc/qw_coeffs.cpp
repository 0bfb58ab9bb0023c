// Host-side coefficient setup for the Chebyshev expansion of exp(-i a x).
//
//  * Bessel values J_m(a) by Miller's backward recurrence (section II.B.1 names
//    Miller's algorithm for the Bessel functions of Eq. cheb), in double
//    precision with overflow rescaling, normalised by J_0 + 2 sum J_2m = 1.
//  * Degree selection from the truncation tail (Eq. TruncError).
//  * Caratheodory-Fejer correction (section II.C, Eq. iter) of the cos and sin
//    parts, with the Laurent recurrence stopped once it has decayed.
//
// Everything here is scalar host work, negligible next to one hypercube matvec.
#include "qw_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace qw {

// Order beyond which J_m(x) is below ~1e-18 of its peak: past the turning
// point m = x the decay is governed by the Airy transition of width x^(1/3).
int bessel_cutoff(double x)
{
    x = std::fabs(x);
    return (int)std::ceil(x + 14.0 * std::cbrt(std::max(x, 1.0)) + 50.0);
}

int bessel_miller(double a, int mmax, double *J)
{
    if (!std::isfinite(a) || mmax < 0) return -1;
    const double x = std::fabs(a);
    if (x == 0.0) {
        for (int m = 0; m <= mmax; ++m) J[m] = (m == 0) ? 1.0 : 0.0;
        return 0;
    }
    // Start well above both the requested order and the transition region so
    // that the dominant (Y-like) solution has died out by order mmax.
    int start = std::max(mmax, bessel_cutoff(x)) + 40 + (int)(6.0 * std::cbrt(x));
    start += (start & 1);
    std::vector<double> f(start + 2, 0.0);
    f[start + 1] = 0.0;
    f[start] = 1e-280;
    const double big = 1e250, shrink = 1e-250;
    for (int m = start; m >= 1; --m) {
        f[m - 1] = (2.0 * m / x) * f[m] - f[m + 1];
        if (std::fabs(f[m - 1]) > big) {
            for (int q = m - 1; q <= start; ++q) f[q] *= shrink;
        }
    }
    // J_0 + 2 (J_2 + J_4 + ...) = 1
    double s = 0.0;
    for (int m = start; m >= 2; m -= 2) s += f[m];
    s = f[0] + 2.0 * s;
    const double inv = 1.0 / s;
    for (int m = 0; m <= mmax; ++m) {
        double v = f[m] * inv;
        if (a < 0 && (m & 1)) v = -v;  // J_m(-x) = (-1)^m J_m(x)
        J[m] = v;
    }
    return 0;
}

// alpha_0 = J_0(a), alpha_m = 2 J_m(a): exp(-i a x) = sum (-i)^m alpha_m T_m(x).
static void cheb_alpha(double a, std::vector<double> &alpha)
{
    const int M = bessel_cutoff(a);
    alpha.assign(M + 1, 0.0);
    bessel_miller(a, M, alpha.data());
    for (int m = 1; m <= M; ++m) alpha[m] *= 2.0;
}

// Smallest K with sum_{m>K} |alpha_m| <= tol; returns -1 if the table is too short.
static int tail_degree(const std::vector<double> &alpha, double tol, double *tail_out)
{
    const int M = (int)alpha.size() - 1;
    double tail = 0.0;  // sum_{m > K} |alpha_m|, grown from the top
    int K = M;
    for (int k = M; k >= 0; --k) {
        const double next = tail + std::fabs(alpha[k]);  // sum over m >= k
        if (next > tol) { K = k; break; }
        tail = next;
        K = k - 1;
    }
    if (K < 0) K = 0;  // even the constant term is below tol
    if (tail_out) {
        double t = 0.0;
        for (int m = M; m > K; --m) t += std::fabs(alpha[m]);
        *tail_out = t;
    }
    return K;
}

// Cyclic Jacobi eigensolver for a small dense symmetric matrix (row-major).
// On return w holds the eigenvalues and column j of V the j-th eigenvector.
static void jacobi_eig(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &V)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    double fro = 0.0;
    for (double v : A) fro += v * v;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (off <= 1e-34 * fro || off == 0.0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

// Real CF correction of the degree-m truncation of f = sum_{j=0}^{M} c_j T_j
// (c_0 not halved).  The tail c_{m+1..M} forms a Hankel matrix; its eigenpair
// (lam, u) of largest |lam| defines the Laurent series b of lam times a
// Blaschke product: b_j = c_j for j > m and, for j = m, m-1, ..., -m,
//     b_j = -(b_{j+1} u_1 + ... + b_{j+K-1} u_{K-1}) / u_0     (Eq. iter)
// with u 0-indexed here.  The corrected polynomial is p_0 = c_0 - b_0,
// p_j = c_j - b_j - b_{-j}.  Returns 0, or -1 if u_0 vanishes.
int cf_real(const double *c, int M, int m, double *p, double *lam_out)
{
    const int K = M - m;
    if (K <= 0) {
        for (int j = 0; j <= m; ++j) p[j] = (j <= M) ? c[j] : 0.0;
        *lam_out = 0.0;
        return 0;
    }
    std::vector<double> Hk((size_t)K * K, 0.0);
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) {
            const int idx = m + 1 + i + j;
            Hk[(size_t)i * K + j] = (idx <= M) ? c[idx] : 0.0;
        }
    std::vector<double> w, V;
    jacobi_eig(K, Hk, w, V);
    int sel = 0;
    for (int i = 1; i < K; ++i)
        if (std::fabs(w[i]) > std::fabs(w[sel])) sel = i;
    const double lam = w[sel];
    std::vector<double> u(K);
    for (int i = 0; i < K; ++i) u[i] = V[(size_t)i * K + sel];
    double umax = 0.0;
    for (double v : u) umax = std::max(umax, std::fabs(v));
    if (std::fabs(u[0]) <= 1e-14 * umax) return -1;

    // b_j stored at b[j + m] for j = -m .. M + K
    std::vector<double> b((size_t)(2 * m + M + K + 2), 0.0);
    for (int j = m + 1; j <= M; ++j) b[j + m] = c[j];
    const double thresh = 1e-18 * std::max(std::fabs(lam), 1e-300);
    int small_run = 0;
    for (int j = m; j >= -m; --j) {
        double s = 0.0;
        for (int i = 1; i < K; ++i) s += b[j + i + m] * u[i];
        const double bj = -s / u[0];
        b[j + m] = bj;
        // Early exit (section II.C): once a full window of K-1 consecutive
        // values is negligible the rest of the expansion is negligible too.
        small_run = (std::fabs(bj) < thresh) ? small_run + 1 : 0;
        if (small_run >= std::max(K - 1, 1)) break;  // remaining b_j stay 0
    }
    p[0] = c[0] - b[m];
    for (int j = 1; j <= m; ++j) p[j] = c[j] - b[j + m] - b[-j + m];
    *lam_out = lam;
    return 0;
}

// CF polynomial of exp(-i a x) with combined degree at most K, as alpha_m
// (c_m = (-i)^m alpha_m).  cos(a x) (even) is set up at an odd nominal degree
// and sin(a x) (odd) at an even one, so that each Hankel matrix decouples into
// two blocks instead of carrying +-lambda pairs.  Returns the estimate
// |lam_cos| + |lam_sin| or a negative value on failure.
static double cf_alpha_for_degree(double x, const std::vector<double> &J, int K, std::vector<double> &alpha)
{
    const int M = (int)J.size() - 1;
    std::vector<double> cc(M + 1, 0.0), cs(M + 1, 0.0);
    for (int m = 0; m <= M; ++m) {
        const double sgn = ((m / 2) & 1) ? -1.0 : 1.0;  // (-1)^floor(m/2)
        if ((m & 1) == 0) cc[m] = (m == 0) ? J[0] : 2.0 * sgn * J[m];
        else cs[m] = 2.0 * sgn * J[m];
    }
    (void)x;
    const int Kc = (K % 2 == 0) ? K : K - 1;   // even effective degree of the cos part
    const int Ks = (K % 2 == 1) ? K : K - 1;   // odd effective degree of the sin part
    std::vector<double> pc(Kc + 2, 0.0), ps(std::max(Ks + 2, 1), 0.0);
    double lc = 0.0, ls = 0.0;
    if (cf_real(cc.data(), M, Kc + 1, pc.data(), &lc) != 0) return -1.0;
    if (Ks >= 0) {
        if (cf_real(cs.data(), M, Ks + 1, ps.data(), &ls) != 0) return -1.0;
    } else {
        for (int m = 0; m <= M; ++m) ls += std::fabs(cs[m]);  // zero polynomial
    }
    alpha.assign(K + 1, 0.0);
    for (int m = 0; m <= K; ++m) {
        const double sgn = ((m / 2) & 1) ? -1.0 : 1.0;
        if ((m & 1) == 0) alpha[m] = (m <= Kc + 1) ? sgn * pc[m] : 0.0;
        else alpha[m] = (m <= Ks + 1) ? sgn * ps[m] : 0.0;
    }
    return std::fabs(lc) + std::fabs(ls);
}

int coefficients(double a, double tol, int method, std::vector<double> &alpha, int *K_out, double *err_out)
{
    if (!std::isfinite(a) || !(tol > 0.0) || !std::isfinite(tol)) return -1;
    std::vector<double> al;
    cheb_alpha(std::fabs(a), al);
    double tail = 0.0;
    int K = tail_degree(al, tol, &tail);
    double err = tail;
    if (method == 1) {
        // Lower the degree from the Chebyshev one while the CF estimate holds.
        std::vector<double> J(al.size());
        J[0] = al[0];
        for (size_t m = 1; m < al.size(); ++m) J[m] = 0.5 * al[m];
        // trim the tail to where it is negligible (the padding delta k)
        double peak = 0.0;
        for (double v : J) peak = std::max(peak, std::fabs(v));
        int M = (int)J.size() - 1;
        while (M > 0 && std::fabs(J[M]) < 1e-17 * peak) --M;
        J.resize(M + 1);
        std::vector<double> best, trial;
        double best_err = -1.0;
        int best_K = -1;
        for (int k = K; k >= 0; --k) {
            const double e = cf_alpha_for_degree(std::fabs(a), J, k, trial);
            if (e < 0.0 || e > tol) break;
            best = trial;
            best_err = e;
            best_K = k;
        }
        if (best_K >= 0) {
            al = best;
            K = best_K;
            err = best_err;
        } else {
            al.resize(K + 1);  // CF failed: keep the Chebyshev coefficients
        }
    }
    al.resize(K + 1);
    if (a < 0)
        for (int m = 1; m <= K; m += 2) al[m] = -al[m];
    alpha = al;
    *K_out = K;
    if (err_out) *err_out = err;
    return 0;
}

}  // namespace qw
