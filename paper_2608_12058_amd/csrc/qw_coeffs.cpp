// Host-side coefficient setup for the Chebyshev expansion of exp(-i a x).
//
//  * Bessel values J_m(a) by Miller's backward recurrence (section II.B.1 names
//    Miller's algorithm for the Bessel functions of Eq. cheb), in double
//    precision with overflow rescaling, normalised by J_0 + 2 sum J_2m = 1.
//  * Degree selection from the truncation tail (Eq. TruncError).
//  * Caratheodory-Fejer correction (section II.C, Eq. iter) of the cos and sin
//    parts, with the Laurent recurrence stopped once it has decayed.  The
//    dominant eigenpair of each tail Hankel matrix comes from a Householder
//    reduction to tridiagonal form, bisection and inverse iteration (0.5 ms for
//    a = 450 at 2^-23, three candidate degrees; a cyclic Jacobi solver took 2.7).
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

// Eigenpair of largest |lambda| of a small dense symmetric matrix A (n x n,
// row-major): Householder reduction to a tridiagonal matrix T = Q^T A Q, the
// two extreme eigenvalues of T by bisection on Sturm counts, the eigenvector
// of T by inverse iteration, and u = Q y.  About (4/3) n^3 flops for the
// reduction and O(n^2) for the rest.
namespace {

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x (the
// negative pivots of the LDL^T factorisation of T - x I).
int sturm_below(const std::vector<double> &d, const std::vector<double> &e, double x)
{
    const int n = (int)d.size();
    const double tiny = 1e-300;
    int cnt = 0;
    double q = d[0] - x;
    for (int i = 0;; ++i) {
        if (q == 0.0) q = -tiny;
        if (q < 0.0) ++cnt;
        if (i + 1 == n) break;
        q = (d[i + 1] - x) - e[i] * e[i] / q;
    }
    return cnt;
}

// Solves (T - lam I) x = b in place (b -> x) by Gaussian elimination with
// partial pivoting on the tridiagonal band (a row exchange adds one entry of
// fill two places right of the diagonal); zero pivots become eps * scale.
void tridiag_shifted_solve(const std::vector<double> &d, const std::vector<double> &e, double lam, double scale,
                           std::vector<double> &b)
{
    const int n = (int)d.size();
    std::vector<double> dg(n), up(n, 0.0), up2(n, 0.0), lo(n, 0.0);
    std::vector<char> sw(n, 0);
    for (int i = 0; i < n; ++i) dg[i] = d[i] - lam;
    for (int i = 0; i + 1 < n; ++i) {
        up[i] = e[i];
        lo[i] = e[i];
    }
    const double eps = 1e-16 * std::max(scale, 1e-300);
    // row i holds (lo[i-1] | dg[i], up[i], up2[i]) after elimination of the columns before i
    for (int i = 0; i + 1 < n; ++i) {
        double sub = lo[i];                 // entry (i+1, i)
        if (std::fabs(dg[i]) >= std::fabs(sub)) {
            if (dg[i] == 0.0) dg[i] = eps;
            const double f = sub / dg[i];
            lo[i] = f;
            dg[i + 1] -= f * up[i];
            if (i + 2 < n) { /* up[i+1] unchanged: row i has no entry in column i+2 */ }
            sw[i] = 0;
        } else {
            // exchange rows i and i+1, then eliminate
            const double f = dg[i] / sub;
            const double r0 = up[i], r1 = up2[i];                       // old row i, columns i+1, i+2
            const double s0 = dg[i + 1], s1 = (i + 2 < n) ? up[i + 1] : 0.0;   // old row i+1
            dg[i] = sub;
            up[i] = s0;
            up2[i] = s1;
            lo[i] = f;
            dg[i + 1] = r0 - f * s0;
            if (i + 2 < n) up[i + 1] = r1 - f * s1;
            sw[i] = 1;
        }
    }
    if (dg[n - 1] == 0.0) dg[n - 1] = eps;
    for (int i = 0; i + 1 < n; ++i) {
        if (sw[i]) std::swap(b[i], b[i + 1]);
        b[i + 1] -= lo[i] * b[i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = b[i];
        if (i + 1 < n) v -= up[i] * b[i + 1];
        if (i + 2 < n) v -= up2[i] * b[i + 2];
        b[i] = v / dg[i];
    }
}

}  // namespace

static void dominant_eig(int n, std::vector<double> A, double &lam, std::vector<double> &u)
{
    u.assign(n, 0.0);
    if (n == 1) {
        lam = A[0];
        u[0] = 1.0;
        return;
    }
    // Householder: column k below the diagonal -> (alpha, 0, ..., 0) by
    // H_k = I - 2 v v^T on indices k+1 .. n-1 (v of unit length, or zero).
    std::vector<std::vector<double>> V;
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        std::vector<double> v(m);
        double nx = 0.0;
        for (int i = 0; i < m; ++i) {
            v[i] = A[(size_t)(k + 1 + i) * n + k];
            nx += v[i] * v[i];
        }
        nx = std::sqrt(nx);
        if (nx == 0.0) {
            V.push_back(std::vector<double>(m, 0.0));
            continue;
        }
        const double alpha = (v[0] > 0.0) ? -nx : nx;
        v[0] -= alpha;
        double nv = 0.0;
        for (double x : v) nv += x * x;
        nv = std::sqrt(nv);
        for (double &x : v) x /= nv;
        // trailing block B (rows/cols k+1..): B <- B - 2 v q^T - 2 q v^T,
        // p = B v, q = p - (v^T p) v
        std::vector<double> p(m, 0.0);
        for (int i = 0; i < m; ++i) {
            double acc = 0.0;
            const double *row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
            for (int j = 0; j < m; ++j) acc += row[j] * v[j];
            p[i] = acc;
        }
        double vp = 0.0;
        for (int i = 0; i < m; ++i) vp += v[i] * p[i];
        for (int i = 0; i < m; ++i) p[i] -= vp * v[i];
        for (int i = 0; i < m; ++i) {
            double *row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
            for (int j = 0; j < m; ++j) row[j] -= 2.0 * (v[i] * p[j] + p[i] * v[j]);
        }
        A[(size_t)(k + 1) * n + k] = alpha;
        A[(size_t)k * n + (k + 1)] = alpha;
        for (int i = 1; i < m; ++i) {
            A[(size_t)(k + 1 + i) * n + k] = 0.0;
            A[(size_t)k * n + (k + 1 + i)] = 0.0;
        }
        V.push_back(v);
    }
    std::vector<double> d(n), e(n - 1);
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];

    // Gershgorin interval, then bisection for the largest and the smallest
    // eigenvalue; keep the one of larger magnitude.
    double lo = d[0], hi = d[0], scale = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    scale = std::max(std::fabs(lo), std::fabs(hi));
    auto bisect = [&](bool top) {
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;
            const int c = sturm_below(d, e, mid);
            if (top ? (c == n) : (c >= 1)) b = mid;
            else a = mid;
        }
        return 0.5 * (a + b);
    };
    const double lmax = bisect(true), lmin = bisect(false);
    lam = (std::fabs(lmax) >= std::fabs(lmin)) ? lmax : lmin;

    // inverse iteration on T - lam I
    std::vector<double> y(n);
    for (int i = 0; i < n; ++i) y[i] = 1.0 + 0.01 * i;   // any start with a component along the eigenvector
    for (int it = 0; it < 3; ++it) {
        tridiag_shifted_solve(d, e, lam, scale, y);
        double ny = 0.0;
        for (double x : y) ny += x * x;
        ny = std::sqrt(ny);
        for (double &x : y) x /= ny;
    }
    // u = Q y = H_0 H_1 ... H_{n-3} y
    u = y;
    for (int k = (int)V.size() - 1; k >= 0; --k) {
        const std::vector<double> &v = V[k];
        const int m = (int)v.size();
        double dot = 0.0;
        for (int i = 0; i < m; ++i) dot += v[i] * u[k + 1 + i];
        for (int i = 0; i < m; ++i) u[k + 1 + i] -= 2.0 * dot * v[i];
    }
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
    double lam = 0.0;
    std::vector<double> u;
    dominant_eig(K, Hk, lam, u);
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
