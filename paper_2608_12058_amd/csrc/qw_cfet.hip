// Time-dependent anneal H(t) = A(t) H_P + B(t) sum_j X_j by the fourth-order
// commutator-free Magnus integrator (section III.B; Alvermann and Fehske's
// commutator-free exponential time propagation).  Every exponential
// exp(-i h (alpha H_P + beta sum_j X_j)) is one call of the Chebyshev action on
// tables prepared once per call, so the hot path is the same fused pass
// schedule as for a time-independent H.
//
// One step of length h from t uses the Gauss nodes t_{1,2} = t + (1/2 -+ sqrt3/6) h
// and weights a_{1,2} = 1/4 +- sqrt3/6:
//   psi <- exp(-i h (a2 H(t1) + a1 H(t2))) exp(-i h (a1 H(t1) + a2 H(t2))) psi.
// Expanding both sides in h (noncommutative series in H_P and sum_j X_j, with
// A and B Taylor-expanded at t) gives agreement through h^4 and a local error
//   U_step - U_exact = h^5 E5 + O(h^6),
//   E5 = (i/4320) H'''' - (1/1080) [H, H'''] - (1/720) [H', H'']
//        - (i/720) [H, [H, H'']] - (i/2160) [H', [H, H']] + (1/2880) [H, [H, [H, H']]],
// derivatives in t at the step start.  With H^(a) = A^(a) H_P + B^(a) F,
// [H^(a), H^(b)] = W_ab [H_P, F], W_ab = A^(a) B^(b) - A^(b) B^(a), and
// ||[X, Y]|| <= 2 ||X|| ||Y||, the error norm is bounded by a formula in the
// schedule's derivatives and three numbers of the instance: ||H_P - c||,
// ||F|| = n and ||[H_P, F]|| <= sum_j 2 (|h_j| + sum_k |J_jk|) (the commutator
// with X_j is X_j times the energy change of flipping spin j).  That bound
// costs O(1) per step, so step sizes are chosen without trial runs.
#include "qw_internal.h"
#include "qw_prepared.h"
#include "qwexp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace qw {

namespace {

constexpr int MAX_DEG = 16;
constexpr int MAX_STEPS = 1 << 20;

struct Schedule {
    std::vector<double> a, b;   // monomial coefficients in s = t / T
    double T;

    // d^m/dt^m of a polynomial in s at time t
    static double deriv(const std::vector<double> &p, double T, double t, int m)
    {
        const double s = t / T;
        double acc = 0.0, sp = 1.0;
        for (int k = m; k < (int)p.size(); ++k) {
            double f = 1.0;
            for (int i = 0; i < m; ++i) f *= (double)(k - i);
            acc += p[k] * f * sp;
            sp *= s;
        }
        return acc / std::pow(T, m);
    }
    double A(double t, int m = 0) const { return deriv(a, T, t, m); }
    double B(double t, int m = 0) const { return deriv(b, T, t, m); }
};

struct Instance {
    int n;
    double pshift;   // ||H_P - c||  = (max E - min E) / 2
    double pabs;     // ||H_P||      = max |E|
    double comm;     // bound on ||[H_P, sum_j X_j]||
};

double commutator_bound(int n, const double *h, const double *J)
{
    double total = 0.0;
    for (int j = 0; j < n; ++j) {
        double f = std::fabs(h[j]);
        for (int k = 0; k < n; ++k) {
            if (k == j) continue;
            const int a = std::min(j, k), b = std::max(j, k);
            f += std::fabs(J[a * n - a * (a + 1) / 2 + (b - a - 1)]);
        }
        total += 2.0 * f;
    }
    return total;
}

// Bound on ||E5|| at time t (leading local error per h^5).
double step_bound(const Schedule &S, const Instance &I, double t)
{
    double A[5], B[5];
    for (int m = 0; m < 5; ++m) {
        A[m] = S.A(t, m);
        B[m] = S.B(t, m);
    }
    auto W = [&](int p, int q) { return std::fabs(A[p] * B[q] - A[q] * B[p]); };
    const double F = (double)I.n;
    const double nH = std::fabs(A[0]) * I.pshift + std::fabs(B[0]) * F;    // ||H - shift||
    const double nH1 = std::fabs(A[1]) * I.pshift + std::fabs(B[1]) * F;   // ||H' - shift||
    const double nH4 = std::fabs(A[4]) * I.pabs + std::fabs(B[4]) * F;     // ||H''''||
    const double C = I.comm;
    return nH4 / 4320.0 + W(0, 3) * C / 1080.0 + W(1, 2) * C / 720.0 + W(0, 2) * 2.0 * nH * C / 720.0 +
           W(0, 1) * 2.0 * nH1 * C / 2160.0 + W(0, 1) * 4.0 * nH * nH * C / 2880.0;
}

qw_status read_schedule(const double *A_coef, int A_deg, const double *B_coef, int B_deg, double T, Schedule *S)
{
    if (!A_coef || !B_coef || A_deg < 0 || B_deg < 0 || A_deg > MAX_DEG || B_deg > MAX_DEG) {
        set_error("schedule polynomials need 0 <= degree <= 16");
        return QW_EINVAL;
    }
    if (!(T > 0.0) || !std::isfinite(T)) { set_error("T must be positive and finite"); return QW_EINVAL; }
    S->a.assign(A_coef, A_coef + A_deg + 1);
    S->b.assign(B_coef, B_coef + B_deg + 1);
    for (double x : S->a)
        if (!std::isfinite(x)) { set_error("A has a non-finite coefficient"); return QW_EINVAL; }
    for (double x : S->b)
        if (!std::isfinite(x)) { set_error("B has a non-finite coefficient"); return QW_EINVAL; }
    S->T = T;
    return QW_OK;
}

template <typename R>
qw_status cfet_impl(int n, const double *h, const double *J, const double *A_coef, int A_deg, const double *B_coef,
                    int B_deg, double T, int steps, double tol, const void *psi_in, void *psi_out,
                    double *step_sizes, int step_cap, void *workspace, size_t ws_bytes, void *stream,
                    qw_cfet_info *info)
{
    if (n < 1 || n > 32 || !h || (n > 1 && !J)) { set_error("need 1 <= n <= 32 and (h, J)"); return QW_EINVAL; }
    for (int j = 0; j < n; ++j)
        if (!std::isfinite(h[j])) { set_error("h has a non-finite entry"); return QW_EINVAL; }
    for (int p = 0; p < n * (n - 1) / 2; ++p)
        if (!std::isfinite(J[p])) { set_error("J has a non-finite entry"); return QW_EINVAL; }
    if (!(tol > 0.0) || !std::isfinite(tol)) { set_error("tol must be positive and finite"); return QW_EINVAL; }
    if (steps < 0 || steps > MAX_STEPS) { set_error("steps must be in 0..2^20"); return QW_EINVAL; }
    if (!psi_in || !psi_out) { set_error("psi_in and psi_out are required"); return QW_EINVAL; }
    Schedule S;
    qw_status st = read_schedule(A_coef, A_deg, B_coef, B_deg, T, &S);
    if (st != QW_OK) return st;

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool timing = info && info->timing;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (timing) {
        if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess ||
            hipEventRecord(ev0, s) != hipSuccess) {
            set_error("hipEvent setup failed");
            if (ev0) (void)hipEventDestroy(ev0);
            if (ev1) (void)hipEventDestroy(ev1);
            return QW_EHIP;
        }
    }
    auto cleanup = [&]() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    };

    EnergyTables Tb{};
    double emin = 0.0, emax = 0.0;
    st = prepare_energy<R>(n, h, J, workspace, ws_bytes, stream, &Tb, &emin, &emax);
    if (st != QW_OK) { cleanup(); return st; }
    Instance I{n, 0.5 * (emax - emin), std::max(std::fabs(emin), std::fabs(emax)), commutator_bound(n, h, J)};

    const double r3 = std::sqrt(3.0);
    const double c1 = 0.5 - r3 / 6.0, c2 = 0.5 + r3 / 6.0;
    const double a1 = 0.25 + r3 / 6.0, a2 = 0.25 - r3 / 6.0;
    const bool adaptive = (steps == 0);
    // error budget: adaptive -> half to the Magnus steps, half to the series
    const double rate = 0.5 * tol / T;                            // local error per unit time
    const double trunc_share = adaptive ? 0.25 : 0.5;             // per exponential, times h / T
    const double floor_tol = (sizeof(R) == 4) ? std::ldexp(1.0, -26) : 1e-15;

    int nsteps = 0, nexp = 0;
    long long terms = 0;
    double errb = 0.0, hmin = T, hmax = 0.0, t = 0.0;
    const void *src = psi_in;
    while (t < T) {
        double hs;
        double b = step_bound(S, I, t);
        if (adaptive) {
            hs = (b > 0.0) ? std::pow(rate / b, 0.25) : (T - t);
            // look again at the middle of the proposed step
            const double bm = step_bound(S, I, std::min(T, t + 0.5 * hs));
            b = std::max(b, bm);
            hs = (b > 0.0) ? std::pow(rate / b, 0.25) : (T - t);
            if (hs >= T - t || (T - t - hs) < 1e-9 * T) hs = T - t;
        } else {
            hs = (nsteps == steps - 1) ? (T - t) : T / steps;
        }
        if (nsteps >= MAX_STEPS || !(hs > 0.0)) {
            cleanup();
            set_error("the tolerance needs more than 2^20 steps");
            return QW_ENOCONV;
        }
        const double t1 = t + c1 * hs, t2 = t + c2 * hs;
        const double A1 = S.A(t1), A2 = S.A(t2), B1 = S.B(t1), B2 = S.B(t2);
        const double al[2] = {a1 * A1 + a2 * A2, a2 * A1 + a1 * A2};
        const double be[2] = {a1 * B1 + a2 * B2, a2 * B1 + a1 * B2};
        const double tol_exp = std::max(floor_tol, trunc_share * tol * hs / T);
        for (int e = 0; e < 2; ++e) {
            qw_info ai{};
            st = scaled_action<R>(n, h, J, Tb, al[e], emin, emax, be[e], hs, src, psi_out, tol_exp, workspace,
                                  ws_bytes, stream, &ai);
            if (st != QW_OK) { cleanup(); return st; }
            src = psi_out;
            terms += ai.K;
            ++nexp;
        }
        if (step_sizes && nsteps < step_cap) step_sizes[nsteps] = hs;
        errb += b * std::pow(hs, 5);
        hmin = std::min(hmin, hs);
        hmax = std::max(hmax, hs);
        ++nsteps;
        t += hs;
        if (!adaptive && nsteps == steps) break;
    }
    if (info) {
        info->steps = nsteps;
        info->exponentials = nexp;
        info->terms = terms;
        info->err_bound = errb;
        info->h_min = hmin;
        info->h_max = hmax;
        info->comm_bound = I.comm;
        info->total_ms = 0.f;
        if (timing) {
            if (hipEventRecord(ev1, s) != hipSuccess || hipEventSynchronize(ev1) != hipSuccess ||
                hipEventElapsedTime(&info->total_ms, ev0, ev1) != hipSuccess) {
                cleanup();
                set_error("hipEvent timing failed");
                return QW_EHIP;
            }
        }
    }
    cleanup();
    return QW_OK;
}

}  // namespace

}  // namespace qw

using namespace qw;

extern "C" {

qw_status qw_anneal_cfet4_c64(int n, const double *h, const double *J, const double *A_coef, int A_deg,
                              const double *B_coef, int B_deg, double T, int steps, double tol, const void *psi_in,
                              void *psi_out, double *step_sizes, int step_cap, void *workspace, size_t ws_bytes,
                              void *stream, qw_cfet_info *info)
{
    return cfet_impl<float>(n, h, J, A_coef, A_deg, B_coef, B_deg, T, steps, tol, psi_in, psi_out, step_sizes,
                            step_cap, workspace, ws_bytes, stream, info);
}

qw_status qw_anneal_cfet4_c128(int n, const double *h, const double *J, const double *A_coef, int A_deg,
                               const double *B_coef, int B_deg, double T, int steps, double tol, const void *psi_in,
                               void *psi_out, double *step_sizes, int step_cap, void *workspace, size_t ws_bytes,
                               void *stream, qw_cfet_info *info)
{
    return cfet_impl<double>(n, h, J, A_coef, A_deg, B_coef, B_deg, T, steps, tol, psi_in, psi_out, step_sizes,
                             step_cap, workspace, ws_bytes, stream, info);
}

qw_status qw_cfet4_step_bound(int n, const double *h, const double *J, const double *A_coef, int A_deg,
                              const double *B_coef, int B_deg, double T, double emin, double emax, double t,
                              double *bound)
{
    if (n < 1 || n > 32 || !h || (n > 1 && !J) || !bound || !(emax >= emin)) {
        set_error("bad arguments");
        return QW_EINVAL;
    }
    Schedule S;
    qw_status st = read_schedule(A_coef, A_deg, B_coef, B_deg, T, &S);
    if (st != QW_OK) return st;
    const Instance I{n, 0.5 * (emax - emin), std::max(std::fabs(emin), std::fabs(emax)), commutator_bound(n, h, J)};
    *bound = step_bound(S, I, t);
    return QW_OK;
}

}  // extern "C"
