// exp(-i t H) psi for H = diag(E) + gamma sum_j X_j: kernels and C-ABI.
//
// Method (Hopkins & Kendon): shift and bound the spectrum (section II.A),
// expand exp(-i a x) in Chebyshev polynomials (Eq. cheb, or the CF correction of
// section II.C), and evaluate with the matrix Clenshaw recurrence
// (Alg. 2 / Eq. recursion) written in place into the b_{k+2} buffer
// (section II.D), with the hypercube sum applied matrix-free.
//
// Device layout: psi, b1, b2 are interleaved complex vectors of N = 2^n
// amplitudes (bit j of the index = qubit j); the normalised diagonal
// d = (E - c)/r is a real vector of N, or recomputed per tile in the fused
// passes of both end orientations: complex64 from 26 qubits (from 31 never
// stored, where it would crowd the 288 GB), complex128 from 26 to 30 qubits.
//
// Per Clenshaw term the state is streamed in P passes (P = 1 for n <= 13 in
// complex64): the first pass loads a contiguous tile of 2^13 amplitudes of
// b_{k+1} into LDS, sums the flips of its low 13 bits, and fuses the diagonal,
// the coefficient axpy and the three-term update; each further pass loads a
// tile spanning a group of high bits (plus contiguous "passenger" bits for
// coalescing) and adds that group's flips.  Small instances (n <= 13) run the
// whole recurrence inside one workgroup with the vector resident in LDS.
#include "qw_kernels.h"
#include "qw_prepared.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace qw {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Kernels: energies, spectral bound, normalisation
// ---------------------------------------------------------------------------

template <typename R>
__global__ void __launch_bounds__(256) k_minmax_diag(const R *d, uint64_t N, double *part)
{
    double mn = INFINITY, mx = -INFINITY;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double v = (double)d[i];
        if (v != v) {   // NaN: fmin / fmax would drop it; make the range non-finite instead
            mn = -INFINITY;
            mx = INFINITY;
        }
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    block_minmax(mn, mx, part);
}

template <int D = 0>
__global__ void __launch_bounds__(256) k_fill_zero(double *x, uint64_t count)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

template <typename R>
__global__ void __launch_bounds__(256) k_normalize_diag(const R *E, uint64_t N, double c, double inv_r, R *d)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x)
        d[i] = (R)(((double)E[i] - c) * inv_r);
}


// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------


struct WsLayout {
    size_t b1, b2, d, part, red, hj, q, qt, ft, coef, items, norms, total;
};

static WsLayout ws_layout(int n, int prec, bool otf)
{
    const size_t N = size_t(1) << n;
    const size_t cs = (prec == 64) ? 8 : 16, rs = (prec == 64) ? 4 : 8;
    WsLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    L.b1 = take(N * cs);
    L.b2 = take(N * cs);
    L.d = otf ? size_t(-1) : take(N * rs);
    L.part = take(2 * MAXPART * sizeof(double));
    L.red = take(2 * sizeof(double));
    L.hj = take((32 + 32 * 31 / 2) * sizeof(double));
    L.q = take((size_t(1) << LB_TAB) * sizeof(double));
    L.qt = take(4 * (size_t(1) << TB_WIDE) * sizeof(double));   // split pair tables, per orientation
    // on the fly (every orientation, or the top one of the split shape): per-tile
    // fields, tiles of >= 2^12 amplitudes
    const bool top = (n >= OTF_TOP_NMIN);
    L.ft = (otf || top) ? take(4 * (N >> TB_NARROW) * TILE_FIELDS * sizeof(double)) : size_t(-1);
    L.coef = (n <= Cfg<float>::TB) ? take((size_t)(KMAX_ONCHIP + 1) * cs) : size_t(-1);
    L.items = take(256);
    L.norms = take(KMAX_MON * sizeof(double));
    L.total = off;
    return L;
}


// Host copy of (h, J) for the upload of setup_tables.  The asynchronous copy
// reads it when the stream reaches it, so it must outlive that point: calls
// whose bound read-back follows the upload (which synchronises the stream)
// need nothing more; otherwise the destructor synchronises once.
struct HostTables {
    hipStream_t s = nullptr;
    std::vector<double> hj;
    bool pending = false;
    ~HostTables()
    {
        if (pending) (void)hipStreamSynchronize(s);
    }
};

// Upload h, J (staged in `keep`), build the Q table; returns the tables view.
static qw_status setup_tables(int n, const double *h, const double *J, char *ws, const WsLayout &L,
                              hipStream_t s, EnergyTables *T, HostTables &keep)
{
    const int np = n * (n - 1) / 2;
    keep.s = s;
    keep.hj.assign(n + np, 0.0);
    std::memcpy(keep.hj.data(), h, n * sizeof(double));
    if (np) std::memcpy(keep.hj.data() + n, J, np * sizeof(double));
    double *dhj = reinterpret_cast<double *>(ws + L.hj);
    QW_HIP(hipMemcpyAsync(dhj, keep.hj.data(), keep.hj.size() * sizeof(double), hipMemcpyHostToDevice, s));
    keep.pending = true;
    T->h = dhj;
    T->J = dhj + n;
    T->Q = reinterpret_cast<double *>(ws + L.q);
    T->n = n;
    T->LB = std::min(n, LB_TAB);
    const int nq = 1 << T->LB;
    hipLaunchKernelGGL(k_qtable<0>, dim3((nq + 255) / 256), dim3(256), 0, s, *T, const_cast<double *>(T->Q));
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// Min / max of the energies: the one synchronising read-back of a call.
template <typename R>
static qw_status minmax(int n, const R *diag, const EnergyTables *T, char *ws, const WsLayout &L,
                        hipStream_t s, double *emin, double *emax, HostTables *keep = nullptr)
{
    double *part = reinterpret_cast<double *>(ws + L.part);
    double *red = reinterpret_cast<double *>(ws + L.red);
    int np;
    if (diag) {
        const uint64_t N = uint64_t(1) << n;
        np = grid_for(N, 256 * 16, MAXPART);
        hipLaunchKernelGGL(k_minmax_diag<R>, dim3(np), dim3(256), 0, s, diag, N, part);
    } else {
        const uint64_t ntiles = uint64_t(1) << (n - T->LB);
        np = grid_for(ntiles, 1, MAXPART);
        hipLaunchKernelGGL(k_minmax_energy<0>, dim3(np), dim3(256), 0, s, *T, part);
    }
    QW_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_minmax_final<0>, dim3(1), dim3(256), 0, s, part, np, red);
    QW_HIP(hipGetLastError());
    double h2[2];
    QW_HIP(hipMemcpyAsync(h2, red, sizeof(h2), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    if (keep) keep->pending = false;   // the upload of (h, J) has been read
    *emin = h2[0];
    *emax = h2[1];
    return QW_OK;
}


template <typename R>
static qw_status validate(int n, const R *diag, const double *h, const double *J, double gamma, double t,
                          const void *psi_in, const void *psi_out, double tol, int method, void *ws)
{
    if (n < 1 || n > 32) { set_error("n must be in 1..32"); return QW_EINVAL; }
    if (!finite(gamma) || !finite(t)) { set_error("gamma and t must be finite"); return QW_EINVAL; }
    if (!(tol > 0.0) || !finite(tol)) { set_error("tol must be positive and finite"); return QW_EINVAL; }
    if (method != QW_CHEB && method != QW_CF) { set_error("unknown method"); return QW_EINVAL; }
    if (!psi_in || !psi_out) { set_error("psi_in and psi_out are required"); return QW_EINVAL; }
    if (!ws) { set_error("workspace is required"); return QW_EINVAL; }
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) { set_error("workspace must be 256-byte aligned"); return QW_EINVAL; }
    if ((reinterpret_cast<uintptr_t>(psi_in) & 15) != 0 || (reinterpret_cast<uintptr_t>(psi_out) & 15) != 0) {
        set_error("state vectors must be 16-byte aligned");
        return QW_EINVAL;
    }
    if (!diag) {
        if (!h || (n > 1 && !J)) { set_error("diag == NULL requires h and J"); return QW_EINVAL; }
        for (int j = 0; j < n; ++j)
            if (!finite(h[j])) { set_error("h has a non-finite entry"); return QW_EINVAL; }
        for (int p = 0; p < n * (n - 1) / 2; ++p)
            if (!finite(J[p])) { set_error("J has a non-finite entry"); return QW_EINVAL; }
    }
    return QW_OK;
}

// Spectral shift / bound, optionally uploading tables.  Leaves T valid when
// diag == NULL.
template <typename R>
static qw_status bound_impl(int n, const R *diag, const double *h, const double *J, double gamma,
                            char *ws, const WsLayout &L, hipStream_t s, EnergyTables *T,
                            double *c, double *r)
{
    HostTables keep;
    if (!diag) {
        qw_status st = setup_tables(n, h, J, ws, L, s, T, keep);
        if (st != QW_OK) return st;
    }
    double emin, emax;
    qw_status st = minmax<R>(n, diag, T, ws, L, s, &emin, &emax, &keep);
    if (st != QW_OK) return st;
    if (!finite(emin) || !finite(emax)) { set_error("diagonal has non-finite entries"); return QW_EINVAL; }
    *c = 0.5 * (emax + emin);
    *r = 0.5 * (emax - emin) + n * std::fabs(gamma);
    return QW_OK;
}

template <typename R, int TB, int NT, bool WITH_OTF, bool STREAM>
static void launch_shape(const PassArgs<R> &a, int mode, bool otf, uint64_t ntiles, hipStream_t s,
                         bool keep_pd = false)
{
    const dim3 grid((unsigned)ntiles), block(NT);
    if constexpr (STREAM) {
        if (keep_pd && !otf) {
            if (mode == PM_START) hipLaunchKernelGGL((k_pass<R, TB, NT, PM_START, false, true, true>), grid, block, 0, s, a);
            else if (mode == PM_FUSED) hipLaunchKernelGGL((k_pass<R, TB, NT, PM_FUSED, false, true, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_pass<R, TB, NT, PM_ADD, false, true, true>), grid, block, 0, s, a);
            return;
        }
    }
    if constexpr (WITH_OTF) {
        if (otf && mode == PM_START) { hipLaunchKernelGGL((k_pass<R, TB, NT, PM_START, true, STREAM>), grid, block, 0, s, a); return; }
        if (otf && mode == PM_FUSED) { hipLaunchKernelGGL((k_pass<R, TB, NT, PM_FUSED, true, STREAM>), grid, block, 0, s, a); return; }
    }
    if (mode == PM_START) hipLaunchKernelGGL((k_pass<R, TB, NT, PM_START, false, STREAM>), grid, block, 0, s, a);
    else if (mode == PM_FUSED) hipLaunchKernelGGL((k_pass<R, TB, NT, PM_FUSED, false, STREAM>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_pass<R, TB, NT, PM_ADD, false, STREAM>), grid, block, 0, s, a);
}

// Launches one pass in the tile shape chosen for the call (the on-the-fly
// diagonal exists for the complex64 default and wide shapes: every fused pass
// from 31 qubits, the top orientation's of the split shape; add passes never
// read the diagonal; the streaming hint for the shapes used at large n).
template <typename R>
static void launch_pass(const PassArgs<R> &a, int mode, bool otf, uint64_t ntiles, hipStream_t s, TileCfg cfg)
{
    if constexpr (sizeof(R) == 4) {
        const bool kp = cfg.keep_pd;
        if (cfg.tb == TB_WIDE) {
            if (cfg.stream) return launch_shape<R, TB_WIDE, NT_WIDE, true, true>(a, mode, otf, ntiles, s, kp);
            return launch_shape<R, TB_WIDE, NT_WIDE, true, false>(a, mode, otf, ntiles, s);
        }
        if (cfg.tb == TB_NARROW) {
            if (cfg.stream) return launch_shape<R, TB_NARROW, NT_NARROW, false, true>(a, mode, otf, ntiles, s, kp);
            return launch_shape<R, TB_NARROW, NT_NARROW, false, false>(a, mode, otf, ntiles, s);
        }
        if (cfg.nt == NT_MID) {
            if (cfg.stream) return launch_shape<R, Cfg<R>::TB, NT_MID, false, true>(a, mode, otf, ntiles, s, kp);
            return launch_shape<R, Cfg<R>::TB, NT_MID, false, false>(a, mode, otf, ntiles, s);
        }
        if (cfg.stream) return launch_shape<R, Cfg<R>::TB, Cfg<R>::NT, true, true>(a, mode, otf, ntiles, s, kp);
        return launch_shape<R, Cfg<R>::TB, Cfg<R>::NT, true, false>(a, mode, otf, ntiles, s);
    } else {
        if (cfg.nt == NT_NARROW) return launch_shape<R, TB_NARROW, NT_NARROW, false, false>(a, mode, otf, ntiles, s);
        if (cfg.stream) return launch_shape<R, Cfg<R>::TB, Cfg<R>::NT, true, true>(a, mode, otf, ntiles, s, cfg.keep_pd);
        return launch_shape<R, Cfg<R>::TB, Cfg<R>::NT, true, false>(a, mode, otf, ntiles, s);
    }
}

// Read back ||b_k||^2 (k = 1..K-1), ||y||^2 (slot 0) and ||v||^2 (slot K+1);
// fill the evaluation-error bound of section II.B.3,
//   sum_k u||b_k|| + u||c_k v - b_{k+2}|| + sqrt(d) gamma_d ||b_{k+1}||,
// using ||c_k v - b_{k+2}|| <= |c_k| ||v|| + ||b_{k+2}||, d = n + 1, and report
// QW_EDIVERGE if a vector exceeds what a valid bound allows: with ||H~|| <= 1,
// b_k = sum_{m>=k} c_m U_{m-k}(H~) v and |U_j| <= j + 1 on [-1, 1], so
// ||b_k|| <= sum_{m>=k} |c_m| (m - k + 1) ||v||, and ||y|| <= (1 + tol) ||v||.
static qw_status check_growth(int n, int K, const std::vector<double> &alpha, double tol, double u,
                              const double *dnorms, hipStream_t s, qw_info *info)
{
    std::vector<double> sq(K + 2);
    QW_HIP(hipMemcpyAsync(sq.data(), dnorms, sq.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    const double nv = std::sqrt(sq[K + 1]);
    std::vector<double> nb(K + 3, 0.0);
    for (int k = 1; k < K; ++k) nb[k] = std::sqrt(sq[k]);
    nb[K] = std::fabs(alpha[K]) * nv;
    nb[0] = std::sqrt(sq[0]);
    const double d = n + 1, gd = d * u / (1.0 - d * u);
    double bound = 0.0;
    for (int k = 0; k <= K; ++k)
        bound += u * nb[k] + u * (std::fabs(alpha[k]) * nv + nb[k + 2]) + std::sqrt(d) * gd * nb[k + 1];
    double worst = 0.0;   // max ratio of a norm to its a-priori limit
    double tail = 0.0, tailw = 0.0;   // sum_{m>=k} |c_m| and sum_{m>=k} |c_m| (m - k + 1)
    for (int k = K; k >= 1; --k) {
        tailw += tail + std::fabs(alpha[k]);
        tail += std::fabs(alpha[k]);
        const double lim = tailw * nv * (1.0 + 1e-3) + 64.0 * u * nv;
        if (k < K && lim > 0.0) worst = std::max(worst, nb[k] / lim);
    }
    worst = std::max(worst, nb[0] / ((1.0 + tol + 1e-3) * nv + 1e-300));
    if (info) {
        info->eval_bound = bound;
        info->growth = worst;
        info->out_norm = nb[0];
    }
    if (worst > 1.0) {
        set_error("the Clenshaw vectors grew past the limit of a valid spectral bound (growth " +
                  std::to_string(worst) + "): the given radius is too small");
        return QW_EDIVERGE;
    }
    return QW_OK;
}

// Optional HIP-event timing of an action call: mark(0) before the setup,
// mark(1) before the Clenshaw loop, finish() after the last kernel.
struct EventTimer {
    bool on;
    hipStream_t s;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    EventTimer(bool on_, hipStream_t s_) : on(on_), s(s_)
    {
        if (on)
            for (auto &e : ev)
                if (hipEventCreate(&e) != hipSuccess) on = false;
    }
    ~EventTimer()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int i)
    {
        if (on) (void)hipEventRecord(ev[i], s);
    }
    qw_status finish(qw_info *info)
    {
        if (!on) return QW_OK;
        QW_HIP(hipEventRecord(ev[2], s));
        QW_HIP(hipEventSynchronize(ev[2]));
        float a = 0.f, b = 0.f;
        QW_HIP(hipEventElapsedTime(&a, ev[0], ev[1]));
        QW_HIP(hipEventElapsedTime(&b, ev[1], ev[2]));
        info->setup_ms = a;
        info->loop_ms = b;
        return QW_OK;
    }
};

// timing == 2: an event after every pass; pass_ms[o] sums the durations of
// the passes over orientation o of the plan (the final step included).
struct PassTimer {
    bool on;
    hipStream_t s;
    std::vector<hipEvent_t> ev;
    std::vector<int> slot;
    size_t used = 0;
    PassTimer(bool on_, hipStream_t s_, size_t count) : on(on_), s(s_)
    {
        if (!on) return;
        ev.resize(count, nullptr);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) { on = false; break; }
    }
    ~PassTimer()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int sl)
    {
        if (on && used < ev.size()) {
            (void)hipEventRecord(ev[used++], s);
            slot.push_back(sl);
        }
    }
    qw_status finish(qw_info *info)
    {
        if (!on || used < 2) return QW_OK;
        QW_HIP(hipEventSynchronize(ev[used - 1]));
        for (int p = 0; p < 4; ++p) info->pass_ms[p] = 0.f;
        for (size_t i = 1; i < used; ++i) {
            float ms = 0.f;
            QW_HIP(hipEventElapsedTime(&ms, ev[i - 1], ev[i]));
            const int sl = slot[i];
            if (sl >= 0 && sl < 4) info->pass_ms[sl] += ms;
        }
        return QW_OK;
    }
};

// Caller-supplied polynomial: p(x) = sum_k coef_k T_k(x) (Chebyshev basis,
// Clenshaw) or sum_k coef_k x^k (monomial basis, Horner's rule), complex
// coefficients as (re, im) pairs.
struct PolyIn {
    const double *coef;
    int K;
    int horner;
};

template <typename R>
static qw_status action_impl(int n, const R *diag, const double *h, const double *J, double gamma, double t,
                             const void *psi_in, void *psi_out, double tol, int method, void *workspace,
                             size_t ws_bytes, void *stream, qw_info *info, const double *given_cr = nullptr,
                             const PolyIn *poly = nullptr, const Prepared *prep = nullptr)
{
    using C = typename Cplx<R>::T;
    using V = CVec<R>;
    qw_status st = validate<R>(n, diag, h, J, gamma, t, psi_in, psi_out, tol, method, workspace);
    if (st != QW_OK) return st;
    const bool otf = (diag == nullptr && n >= OTF_NMIN && sizeof(R) == 4);
    const WsLayout L = ws_layout(n, prec_of<R>(), otf);
    if (ws_bytes < L.total) {
        set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
        return QW_ENOMEM;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    const uint64_t N = uint64_t(1) << n;
    EventTimer timer(info && info->timing, s);
    timer.mark(0);

    EnergyTables T{};
    HostTables keep;   // (h, J) staged for an upload with no read-back after it
    double c = 0.0, r = 0.0;
    if (poly && info && info->monitor) { set_error("the norm monitor applies to exp(-itH) only"); return QW_EINVAL; }
    const bool monitor = !poly && ((info && info->monitor) || (given_cr && !prep));
    if (given_cr) {
        c = given_cr[0];
        r = given_cr[1];
        if (!finite(c) || !(r > 0.0) || !finite(r)) { set_error("the given bound needs finite c and r > 0"); return QW_EINVAL; }
        if (!diag) {
            if (prep) {
                T = prep->T;
            } else {
                st = setup_tables(n, h, J, ws, L, s, &T, keep);
                if (st != QW_OK) return st;
            }
        }
    } else {
        st = bound_impl<R>(n, diag, h, J, gamma, ws, L, s, &T, &c, &r);
        if (st != QW_OK) return st;
    }

    // g = gamma / r; in single precision round g towards zero and take
    // r = gamma / g, which is still a bound and makes g exact in float.
    double g = (r > 0.0) ? gamma / r : 0.0;
    if (sizeof(R) == 4 && gamma != 0.0 && r > 0.0 && !poly) {
        float gf = (float)g;
        if (std::fabs((double)gf) > std::fabs(g)) gf = std::nextafter(gf, 0.0f);
        g = (double)gf;
        r = gamma / g;
    }
    const double inv_r = (r > 0.0) ? 1.0 / r : 0.0;
    const double ph_r = poly ? 1.0 : std::cos(t * c), ph_i = poly ? 0.0 : -std::sin(t * c);   // exp(-i t c)
    const uint64_t nvec = N / V::N;
    const int eg = grid_for(nvec, 256 * 4, 1 << 16);

    if (info) {
        const int want = info->timing, mon = info->monitor;
        std::memset(info, 0, sizeof(*info));
        info->timing = want;
        info->monitor = mon;
        info->n = n;
        info->shift_c = c;
        info->radius_r = r;
        info->method = method;
    }
    const C *psi = static_cast<const C *>(psi_in);
    C *out = static_cast<C *>(psi_out);
    if (r == 0.0) {
        // H = c I: exp(-itH) psi = exp(-itc) psi; a caller's polynomial is taken at H~ = 0
        double sr = ph_r, si = ph_i;
        if (poly) {
            sr = si = 0.0;
            for (int k = 0; k <= poly->K; ++k) {
                const double tk = poly->horner ? (k == 0 ? 1.0 : 0.0)
                                               : ((k & 1) ? 0.0 : ((k & 2) ? -1.0 : 1.0));   // T_k(0)
                sr += tk * poly->coef[2 * k];
                si += tk * poly->coef[2 * k + 1];
            }
        }
        timer.mark(1);
        hipLaunchKernelGGL(k_scale<R>, dim3(eg), dim3(256), 0, s, reinterpret_cast<const V *>(psi),
                           reinterpret_cast<V *>(out), (R)sr, (R)si, nvec);
        QW_HIP(hipGetLastError());
        return timer.finish(info);
    }

    // normalised diagonal d~ = (E' - c) / r of the energies E' = escale * E
    const double es = prep ? prep->escale : 1.0;
    const double norm_c = (es != 0.0) ? c / es : 0.0, norm_inv_r = es * inv_r;
    R *dn = otf ? nullptr : reinterpret_cast<R *>(ws + L.d);
    double *qt = reinterpret_cast<double *>(ws + L.qt);
    // orientations and launch shapes; the end orientations rebuild the diagonal
    // where the plan says so, and the stored one is formed only if a pass reads it
    const std::vector<OrientSpec> plan = action_plan<R>(n, diag == nullptr);
    bool any_otf = false;
    for (const OrientSpec &o : plan) any_otf = any_otf || o.otf;
    if (any_otf && !(L.ft != size_t(-1))) { set_error("internal: no per-tile field table for this size"); return QW_EINVAL; }
    double *ft = any_otf ? reinterpret_cast<double *>(ws + L.ft) : nullptr;
    const uint64_t ft_stride = (N >> TB_NARROW) * TILE_FIELDS;   // doubles per orientation
    if (!otf && plan_reads_diag(plan)) {
        if (diag) {
            hipLaunchKernelGGL(k_normalize_diag<R>, dim3(grid_for(N, 256 * 8, 1 << 16)), dim3(256), 0, s,
                               diag, N, c, inv_r, dn);
        } else {
            hipLaunchKernelGGL(k_normalize_energy<R>, dim3(grid_for(N >> T.LB, 1, 1 << 16)), dim3(256), 0, s,
                               T, norm_c, norm_inv_r, dn);
        }
    }
    QW_HIP(hipGetLastError());

    // coefficients (host, double): c_k = (-i)^k alpha_k, or the caller's
    const double a = poly ? 0.0 : t * r;
    std::vector<double> alpha;
    int K = 0;
    double err = 0.0;
    if (poly) {
        K = poly->K;
    } else if (coefficients(a, tol, method, alpha, &K, &err) != 0) {
        set_error("coefficient setup failed");
        return QW_ENOCONV;
    }
    std::vector<double> cre(K + 1), cim(K + 1);
    for (int k = 0; k <= K; ++k) {
        if (poly) {
            cre[k] = poly->coef[2 * k];
            cim[k] = poly->coef[2 * k + 1];
        } else {
            coef_of(alpha, k, cre[k], cim[k]);
        }
    }
    const bool horner = poly && poly->horner;
    if (info) {
        info->K = K;
        info->a = a;
        info->trunc_bound = err;
        info->passes = (int)plan.size();
        for (size_t o = 0; o < plan.size(); ++o)
            if (plan[o].otf) info->otf_mask |= 1 << o;
    }

    if (n <= Cfg<R>::TB && !monitor) {
        // on-chip: whole recurrence in one workgroup
        if (K > KMAX_ONCHIP) { set_error("degree too large for the on-chip path"); return QW_ENOMEM; }
        std::vector<C> ch(K + 1);
        for (int k = 0; k <= K; ++k) {
            ch[k].x = (R)cre[k];
            ch[k].y = (R)cim[k];
        }
        C *dcoef = reinterpret_cast<C *>(ws + L.coef);
        OnchipItem<R> item{psi, out, dn, dcoef, (R)g, (R)ph_r, (R)ph_i, n, K};
        if (horner) {
            item.two = R(1);
            item.sub = R(0);
        }
        OnchipItem<R> *ditem = reinterpret_cast<OnchipItem<R> *>(ws + L.items);
        QW_HIP(hipMemcpyAsync(dcoef, ch.data(), ch.size() * sizeof(C), hipMemcpyHostToDevice, s));
        QW_HIP(hipMemcpyAsync(ditem, &item, sizeof(item), hipMemcpyHostToDevice, s));
        timer.mark(1);
        hipLaunchKernelGGL((k_onchip<R, Cfg<R>::TB, ONCHIP_NT>), dim3(1), dim3(ONCHIP_NT), 0, s,
                           (const OnchipItem<R> *)ditem, (const int *)nullptr, 1);
        QW_HIP(hipGetLastError());
        QW_HIP(hipStreamSynchronize(s));  // host copies of ch/item go out of scope
        keep.pending = false;
        return timer.finish(info);
    }

    if (K == 0) {
        const double cr = cre[0], ci = cim[0];
        const double pr = cr * ph_r - ci * ph_i, pi = cr * ph_i + ci * ph_r;
        timer.mark(1);
        hipLaunchKernelGGL(k_scale<R>, dim3(eg), dim3(256), 0, s, reinterpret_cast<const V *>(psi),
                           reinterpret_cast<V *>(out), (R)pr, (R)pi, nvec);
        QW_HIP(hipGetLastError());
        return timer.finish(info);
    }

    C *X = reinterpret_cast<C *>(ws + L.b1);
    C *Y = reinterpret_cast<C *>(ws + L.b2);
    double *norms = reinterpret_cast<double *>(ws + L.norms);
    if (monitor) {
        if (K + 2 > KMAX_MON) { set_error("degree too large for the norm monitor"); return QW_ENOMEM; }
        // cleared by a kernel, not a memset node, so that the call can be captured
        hipLaunchKernelGGL(k_fill_zero<0>, dim3(grid_for(K + 2, 256, 256)), dim3(256), 0, s, norms,
                           (uint64_t)(K + 2));
        hipLaunchKernelGGL(k_norm2<R>, dim3(grid_for(nvec, 256 * 8, 4096)), dim3(256), 0, s,
                           reinterpret_cast<const V *>(psi), nvec, norms + K + 1);
    }
    const int P = (int)plan.size();
    if (P > 4) { set_error("internal: more than four orientations"); return QW_EINVAL; }
    for (int o = 0; o < P; ++o) {
        if (!plan[o].otf) continue;
        // the on-the-fly shapes (2^13 tiles with 512 threads, 2^14 with 1024)
        // fill every tile: the split pair table needs L + h = TB
        const PassPlan &pl = plan[o].pl;
        const TileCfg &pc = plan[o].fused;
        const int log_nt = (pc.nt == 1024) ? 10 : 9;
        const bool shape_ok = (sizeof(R) == 4 && pc.tb == TB_WIDE && pc.nt == NT_WIDE) ||
                              (pc.tb == Cfg<R>::TB && pc.nt == Cfg<R>::NT);
        if (pl.L + pl.h != pc.tb || !shape_ok || pc.tb - log_nt > QS_MAX_R) {
            set_error("internal: on-the-fly tile shape");
            return QW_EINVAL;
        }
        hipLaunchKernelGGL(k_qsplit_orient<0>, dim3(((1 << log_nt) + 255) / 256), dim3(256), 0, s, T.h, n, pl.L,
                           pl.g0, pl.h, log_nt, sizeof(R) == 4 ? 1 : 0, norm_inv_r, qt + (size_t)o * (1 << TB_WIDE));
        const uint64_t nt = N >> (pl.L + pl.h);
        hipLaunchKernelGGL(k_tile_fields<0>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, T.h, n, pl.L,
                           pl.g0, pl.h, nt, norm_c, norm_inv_r, ft + (size_t)o * ft_stride);
    }
    timer.mark(1);
    // Clenshaw start b_K = c_K psi (b_{K+1} = 0 is never read: the first pass
    // takes acc = NULL).  With several orientations the passes of term K-1 read
    // psi and scale it as they load it, so b_K is never stored; with one
    // orientation it is stored, since term K-2 reads it again as b_{k+2}.
    const bool fuse_start = (P >= 2);
    if (!fuse_start) {
        const double cr = cre[K], ci = cim[K];
        hipLaunchKernelGGL(k_scale<R>, dim3(eg), dim3(256), 0, s, reinterpret_cast<const V *>(psi),
                           reinterpret_cast<V *>(X), (R)cr, (R)ci, nvec);
        QW_HIP(hipGetLastError());
    }
    PassArgs<R> pa{};
    pa.psi = psi;
    pa.d = dn;
    pa.g = (R)g;
    pa.n = n;
    const std::vector<SchedPass> sched = fused_schedule(K, P);
    PassTimer ptimer(info && info->timing == 2, s, sched.size() + 1);
    ptimer.mark(-1);
    auto scale_of = [horner](int k) { return (k == 0 || horner) ? R(1) : R(2); };
    pa.sub = horner ? R(0) : R(1);
    for (const SchedPass &sp : sched) {
        const OrientSpec &os = plan[sp.orient];
        const PassPlan &pl = os.pl;
        double cr = 0.0, ci = 0.0;
        pa.b1 = X;
        pa.b1_scaled = 0;
        if (fuse_start && sp.k == K - 1) {
            // b_{k+1} = b_K = c_K psi; X is free and takes the FUSED pass's dst2
            pa.b1 = psi;
            pa.b1_scaled = 1;
            pa.b1r = (R)cre[K];
            pa.b1i = (R)cim[K];
        }
        pa.L = pl.L;
        pa.g0 = pl.g0;
        pa.h = pl.h;
        pa.Qt = qt + (size_t)sp.orient * (1 << TB_WIDE);
        const bool pass_otf = os.otf && sp.mode != PM_ADD;
        pa.Ft = os.otf ? ft + (size_t)sp.orient * ft_stride : nullptr;
        pa.pr = R(1);
        pa.pi = R(0);
        pa.dst2 = nullptr;
        pa.norm_acc = nullptr;
        if (sp.mode == PM_START) {
            cr = cre[sp.k];
            ci = cim[sp.k];
            pa.acc = (sp.k == K - 1 || horner) ? nullptr : Y;
            pa.dst = sp.fin ? out : Y;
            pa.scale = scale_of(sp.k);
            if (sp.fin) { pa.pr = (R)ph_r; pa.pi = (R)ph_i; }
            if (monitor && P == 1) pa.norm_acc = norms + sp.k;
        } else if (sp.mode == PM_ADD) {
            pa.acc = Y;
            pa.dst = sp.fin ? out : Y;
            pa.scale = scale_of(sp.k);
            if (sp.fin) {
                pa.pr = (R)ph_r;
                pa.pi = (R)ph_i;
                if (monitor) pa.norm_acc = norms;
            }
        } else {
            cr = cre[sp.k - 1];
            ci = cim[sp.k - 1];
            pa.acc = Y;
            pa.dst = Y;
            pa.dst2 = X;
            pa.scale = scale_of(sp.k);
            pa.scale2 = scale_of(sp.k - 1);
            if (monitor) pa.norm_acc = norms + sp.k;
        }
        pa.cr = (R)cr;
        pa.ci = (R)ci;
        const uint64_t ntiles = N >> (pl.L + pl.h);
        pa.xcd_order = os.xcd;
        launch_pass<R>(pa, sp.mode, pass_otf, ntiles, s, sp.mode == PM_ADD ? os.add : os.fused);
        ptimer.mark(sp.orient);
        if (sp.mode == PM_FUSED || (sp.mode == PM_START && P == 1)) std::swap(X, Y);
    }
    QW_HIP(hipGetLastError());
    qw_status tst = timer.finish(info);
    if (tst != QW_OK) return tst;
    tst = ptimer.finish(info);
    if (tst != QW_OK || !monitor) return tst;
    tst = check_growth(n, K, alpha, tol, sizeof(R) == 4 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53), norms, s,
                       info);
    keep.pending = false;   // check_growth synchronised the stream
    return tst;
}

template <typename R>
static qw_status bound_entry(int n, const R *diag, const double *h, const double *J, double gamma,
                             double *c, double *r, void *workspace, size_t ws_bytes, void *stream)
{
    if (n < 1 || n > 32 || !c || !r || !workspace || !finite(gamma)) { set_error("bad arguments"); return QW_EINVAL; }
    if (!diag && (!h || (n > 1 && !J))) { set_error("diag == NULL requires h and J"); return QW_EINVAL; }
    const WsLayout L = ws_layout(n, prec_of<R>(), diag == nullptr && n >= OTF_NMIN && sizeof(R) == 4);
    if (ws_bytes < L.total) { set_error("workspace too small"); return QW_ENOMEM; }
    EnergyTables T{};
    return bound_impl<R>(n, diag, h, J, gamma, static_cast<char *>(workspace), L,
                         reinterpret_cast<hipStream_t>(stream), &T, c, r);
}

// Host-side check of a pass plan's index map (used by the CPU tests): every
// (tile, element) pair must hit each index of [0, 2^n) exactly once and every
// flipped partner must stay inside the tile.
int check_plan(int n, int prec)
{
    const std::vector<OrientSpec> spec = (prec == 64) ? action_plan<float>(n, true) : action_plan<double>(n, true);
    const uint64_t N = uint64_t(1) << n;
    int covered_bits = 0;
    for (const OrientSpec &os : spec) {
        const PassPlan &p = os.pl;
        if (p.L + p.h > os.fused.tb || p.L + p.h > os.add.tb || p.L + p.h > n) return -1;
        if (os.otf && p.L + p.h != os.fused.tb) return -7;
        if (p.L > p.g0 && p.g0 != 0) return -2;
        std::vector<uint8_t> seen(N, 0);
        const uint64_t ntiles = N >> (p.L + p.h);
        const uint32_t TE = 1u << (p.L + p.h);
        for (uint64_t t = 0; t < ntiles; ++t) {
            const uint64_t base = tile_base(t, p.L, p.g0, p.h);
            for (uint32_t e = 0; e < TE; ++e) {
                const uint64_t idx = tile_index(base, e, p.L, p.g0);
                if (idx >= N || seen[idx]) return -3;
                seen[idx] = 1;
                for (int j = 0; j < p.h; ++j) {
                    const uint32_t pe = e ^ (1u << (p.L + j));
                    if (pe >= TE) return -4;
                    if (tile_index(base, pe, p.L, p.g0) != (idx ^ (uint64_t(1) << (p.g0 + j)))) return -5;
                }
            }
        }
        covered_bits += p.h;
    }
    return covered_bits == n ? (int)spec.size() : -6;
}

template <typename R>
static qw_status poly_entry(int n, const R *diag, const double *h, const double *J, double gamma, double c, double r,
                            const double *coef, int K, qw_basis basis, const void *psi_in, void *psi_out,
                            void *workspace, size_t ws_bytes, void *stream, qw_info *info)
{
    if (basis != QW_BASIS_CHEB && basis != QW_BASIS_MONO) { set_error("unknown basis"); return QW_EINVAL; }
    if (K < 0 || K > QW_POLY_KMAX || !coef) { set_error("need coef with K + 1 entries, 0 <= K <= QW_POLY_KMAX"); return QW_EINVAL; }
    for (int k = 0; k < 2 * (K + 1); ++k)
        if (!finite(coef[k])) { set_error("coef has a non-finite entry"); return QW_EINVAL; }
    if (!finite(c) || !finite(r)) { set_error("c and r must be finite"); return QW_EINVAL; }
    const PolyIn poly{coef, K, basis == QW_BASIS_MONO ? 1 : 0};
    const double cr[2] = {c, r};
    return action_impl<R>(n, diag, h, J, gamma, 0.0, psi_in, psi_out, 1.0, QW_CHEB, workspace, ws_bytes, stream,
                          info, r > 0.0 ? cr : nullptr, &poly);
}

template <typename R>
qw_status prepare_energy(int n, const double *h, const double *J, void *workspace, size_t ws_bytes, void *stream,
                         EnergyTables *T, double *emin, double *emax)
{
    if (n < 1 || n > 32 || !h || (n > 1 && !J) || !workspace) { set_error("bad arguments"); return QW_EINVAL; }
    const WsLayout L = ws_layout(n, prec_of<R>(), n >= OTF_NMIN && sizeof(R) == 4);
    if (ws_bytes < L.total) {
        set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
        return QW_ENOMEM;
    }
    char *ws = static_cast<char *>(workspace);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HostTables keep;
    qw_status st = setup_tables(n, h, J, ws, L, s, T, keep);
    if (st != QW_OK) return st;
    return minmax<R>(n, nullptr, T, ws, L, s, emin, emax, &keep);
}

template <typename R>
qw_status scaled_action(int n, const double *h, const double *J, const EnergyTables &T, double alpha, double emin,
                        double emax, double beta, double t, const void *psi_in, void *psi_out, double tol,
                        void *workspace, size_t ws_bytes, void *stream, qw_info *info)
{
    const double c = alpha * 0.5 * (emax + emin);
    const double r = std::fabs(alpha) * 0.5 * (emax - emin) + n * std::fabs(beta);
    const Prepared prep{T, alpha};
    if (!(r > 0.0)) {
        // H' = c I (here c = 0 as well): the identity
        if (psi_out == psi_in) return QW_OK;
        QW_HIP(hipMemcpyAsync(psi_out, psi_in, (size_t(1) << n) * 2 * sizeof(R), hipMemcpyDeviceToDevice,
                              reinterpret_cast<hipStream_t>(stream)));
        return QW_OK;
    }
    const double cr[2] = {c, r};
    return action_impl<R>(n, nullptr, h, J, beta, t, psi_in, psi_out, tol, QW_CHEB, workspace, ws_bytes, stream, info,
                          cr, nullptr, &prep);
}

template qw_status prepare_energy<float>(int, const double *, const double *, void *, size_t, void *, EnergyTables *,
                                         double *, double *);
template qw_status prepare_energy<double>(int, const double *, const double *, void *, size_t, void *, EnergyTables *,
                                          double *, double *);
template qw_status scaled_action<float>(int, const double *, const double *, const EnergyTables &, double, double,
                                        double, double, double, const void *, void *, double, void *, size_t, void *,
                                        qw_info *);
template qw_status scaled_action<double>(int, const double *, const double *, const EnergyTables &, double, double,
                                         double, double, double, const void *, void *, double, void *, size_t, void *,
                                         qw_info *);

// ---------------------------------------------------------------------------
// Entry point without a caller workspace: its scratch is a file-scope device
// array of fixed size (each GPU the library runs on holds one until the
// process ends), sized for the complex64 workspace of NOALLOC_NMAX qubits.
// Host code must not pass the array's name to a kernel (it is a host-side
// stand-in there): its device address is taken once per device with
// hipGetSymbolAddress and used instead.
// ---------------------------------------------------------------------------
static constexpr int NOALLOC_NMAX = 20;
static constexpr size_t NOALLOC_BYTES = size_t(22) << 20;   // >= ws_layout(20, 64, false).total
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

static constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array, looked up on first use with
// the device current.
static qw_status scratch_for_current_device(void **ptr)
{
    int dev = -1;
    QW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) { set_error("device index out of range"); return QW_EINVAL; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        QW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0) { set_error("scratch symbol address"); return QW_EHIP; }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return QW_OK;
}

}  // namespace qw

using namespace qw;

extern "C" {

qw_status qw_expm_action_c64_noalloc(int n, const float *diag, const double *h, const double *J, double gamma,
                                     double t, const void *psi_in, void *psi_out, double tol, qw_method method,
                                     void *stream, qw_info *info)
{
    if (n < 1 || n > NOALLOC_NMAX) {
        set_error("qw_expm_action_c64_noalloc: n must be in 1.." + std::to_string(NOALLOC_NMAX) +
                  " (its fixed device scratch holds the workspace of " + std::to_string(NOALLOC_NMAX) + " qubits)");
        return QW_EINVAL;
    }
    const size_t need = ws_layout(n, 64, false).total;
    if (need > NOALLOC_BYTES) { set_error("internal: scratch array too small"); return QW_ENOMEM; }
    void *ws = nullptr;
    const qw_status st = scratch_for_current_device(&ws);
    if (st != QW_OK) return st;
    return action_impl<float>(n, diag, h, J, gamma, t, psi_in, psi_out, tol, (int)method, ws, NOALLOC_BYTES,
                              stream, info);
}


const char *qw_last_error(void) { return g_err.c_str(); }
const char *qw_version(void) { return "qwexp 0.15 (gfx950, fused passes, per-orientation launch plans from 25 qubits, contiguous middle orientation, diagonal rebuilt in the end orientations in complex64 and complex128, complex64 flips of a thread's own vectors from registers)"; }

size_t qw_workspace_bytes(int n, int precision, int on_the_fly)
{
    if (n < 1 || n > 32 || (precision != 64 && precision != 128)) return 0;
    return ws_layout(n, precision, on_the_fly != 0).total;
}

qw_status qw_bessel_j(double a, int mmax, double *J)
{
    if (!J || mmax < 0 || !std::isfinite(a)) { set_error("bad arguments"); return QW_EINVAL; }
    return bessel_miller(a, mmax, J) == 0 ? QW_OK : QW_EINVAL;
}

qw_status qw_cheb_coeffs(double a, double tol, qw_method method, int kmax, double *alpha, int *K_out, double *err)
{
    if (!alpha || !K_out || kmax < 0) { set_error("bad arguments"); return QW_EINVAL; }
    if (!std::isfinite(a) || !(tol > 0.0) || !std::isfinite(tol)) { set_error("a must be finite and tol > 0"); return QW_EINVAL; }
    if (method != QW_CHEB && method != QW_CF) { set_error("unknown method"); return QW_EINVAL; }
    std::vector<double> al;
    int K = 0;
    double e = 0.0;
    if (coefficients(a, tol, (int)method, al, &K, &e) != 0) { set_error("coefficient setup failed"); return QW_ENOCONV; }
    *K_out = K;
    if (err) *err = e;
    if (K > kmax) { set_error("kmax too small"); return QW_ENOMEM; }
    std::memcpy(alpha, al.data(), (K + 1) * sizeof(double));
    return QW_OK;
}

qw_status qw_spectral_bound_f32(int n, const float *diag, const double *h, const double *J, double gamma,
                                double *c, double *r, void *workspace, size_t ws_bytes, void *stream)
{
    return bound_entry<float>(n, diag, h, J, gamma, c, r, workspace, ws_bytes, stream);
}

qw_status qw_spectral_bound_f64(int n, const double *diag, const double *h, const double *J, double gamma,
                                double *c, double *r, void *workspace, size_t ws_bytes, void *stream)
{
    return bound_entry<double>(n, diag, h, J, gamma, c, r, workspace, ws_bytes, stream);
}

qw_status qw_expm_action_c64(int n, const float *diag, const double *h, const double *J, double gamma, double t,
                             const void *psi_in, void *psi_out, double tol, qw_method method, void *workspace,
                             size_t ws_bytes, void *stream, qw_info *info)
{
    return action_impl<float>(n, diag, h, J, gamma, t, psi_in, psi_out, tol, (int)method, workspace, ws_bytes,
                              stream, info);
}

qw_status qw_expm_action_c128(int n, const double *diag, const double *h, const double *J, double gamma, double t,
                              const void *psi_in, void *psi_out, double tol, qw_method method, void *workspace,
                              size_t ws_bytes, void *stream, qw_info *info)
{
    return action_impl<double>(n, diag, h, J, gamma, t, psi_in, psi_out, tol, (int)method, workspace, ws_bytes,
                               stream, info);
}

qw_status qw_expm_action_c64_bounded(int n, const float *diag, const double *h, const double *J, double gamma,
                                     double t, double c, double r, const void *psi_in, void *psi_out, double tol,
                                     qw_method method, void *workspace, size_t ws_bytes, void *stream, qw_info *info)
{
    const double cr[2] = {c, r};
    return action_impl<float>(n, diag, h, J, gamma, t, psi_in, psi_out, tol, (int)method, workspace, ws_bytes,
                              stream, info, cr);
}

qw_status qw_expm_action_c128_bounded(int n, const double *diag, const double *h, const double *J, double gamma,
                                      double t, double c, double r, const void *psi_in, void *psi_out, double tol,
                                      qw_method method, void *workspace, size_t ws_bytes, void *stream,
                                      qw_info *info)
{
    const double cr[2] = {c, r};
    return action_impl<double>(n, diag, h, J, gamma, t, psi_in, psi_out, tol, (int)method, workspace, ws_bytes,
                               stream, info, cr);
}

qw_status qw_poly_action_c64(int n, const float *diag, const double *h, const double *J, double gamma, double c,
                             double r, const double *coef, int K, qw_basis basis, const void *psi_in, void *psi_out,
                             void *workspace, size_t ws_bytes, void *stream, qw_info *info)
{
    return poly_entry<float>(n, diag, h, J, gamma, c, r, coef, K, basis, psi_in, psi_out, workspace, ws_bytes, stream,
                             info);
}

qw_status qw_poly_action_c128(int n, const double *diag, const double *h, const double *J, double gamma, double c,
                              double r, const double *coef, int K, qw_basis basis, const void *psi_in, void *psi_out,
                              void *workspace, size_t ws_bytes, void *stream, qw_info *info)
{
    return poly_entry<double>(n, diag, h, J, gamma, c, r, coef, K, basis, psi_in, psi_out, workspace, ws_bytes,
                              stream, info);
}

// One complex64 hypercube pass of a chosen tile shape over caller buffers, for
// timing the shapes a plan is chosen from (the coefficients are fixed, so the
// output is not a Clenshaw term of anything).
qw_status qw_time_pass_c64(int n, int mode, int tb, int nt, int on_the_fly, int L, int g0, int h, int xcd_order,
                           const void *b1, const void *acc, void *dst, void *dst2, const void *psi, const float *d,
                           void *workspace, size_t ws_bytes, void *stream)
{
    if (n < 14 || n > 32) { set_error("n must be in 14..32"); return QW_EINVAL; }
    if (mode != PM_START && mode != PM_ADD && mode != PM_FUSED) { set_error("mode: 0 start, 1 add, 2 fused"); return QW_EINVAL; }
    const bool shape = (tb == TB_NARROW && nt == NT_NARROW) || (tb == Cfg<float>::TB && (nt == NT_MID || nt == Cfg<float>::NT)) ||
                       (tb == TB_WIDE && nt == NT_WIDE);
    if (!shape) { set_error("tile shape must be (12, 1024), (13, 1024), (13, 512) or (14, 1024)"); return QW_EINVAL; }
    const bool otf = on_the_fly != 0 && mode != PM_ADD;
    if (otf && !((tb == Cfg<float>::TB && nt == Cfg<float>::NT) || tb == TB_WIDE)) {
        set_error("the diagonal is rebuilt on (13, 512) and (14, 1024) tiles only");
        return QW_EINVAL;
    }
    if (h < 1 || L < 0 || L + h > tb || (otf && L + h != tb) || g0 + h > n || !(g0 >= L || (g0 == 0 && L == 0))) {
        set_error("bad orientation (L, g0, h) for this tile");
        return QW_EINVAL;
    }
    const bool needs_d = (mode != PM_ADD) && !otf;
    if (!b1 || !dst || (mode != PM_START && !acc) || (mode == PM_FUSED && !dst2) || (mode != PM_ADD && !psi) ||
        (needs_d && !d) || !workspace) {
        set_error("missing buffer for this mode");
        return QW_EINVAL;
    }
    const WsLayout Lw = ws_layout(n, 64, true);
    if (ws_bytes < Lw.total || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        set_error("workspace: qw_workspace_bytes(n, 64, 1) bytes, 256-byte aligned");
        return QW_EINVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    double *qt = reinterpret_cast<double *>(ws + Lw.qt), *ft = reinterpret_cast<double *>(ws + Lw.ft);
    const uint64_t ntiles = (uint64_t(1) << n) >> (L + h);
    if (otf) {
        hipLaunchKernelGGL(k_fill_zero<0>, dim3(64), dim3(256), 0, s, qt, (uint64_t)(1 << TB_WIDE));
        hipLaunchKernelGGL(k_fill_zero<0>, dim3(grid_for(ntiles * TILE_FIELDS, 256, 1 << 16)), dim3(256), 0, s, ft,
                           ntiles * TILE_FIELDS);
    }
    PassArgs<float> a{};
    a.b1 = static_cast<const float2 *>(b1);
    a.acc = static_cast<const float2 *>(mode == PM_START ? nullptr : acc);
    a.dst = static_cast<float2 *>(dst);
    a.dst2 = static_cast<float2 *>(dst2);
    a.psi = static_cast<const float2 *>(psi);
    a.d = d;
    a.Qt = qt;
    a.Ft = otf ? ft : nullptr;
    a.g = 0.01f;
    a.scale = 2.f;
    a.scale2 = 2.f;
    a.cr = 0.1f;
    a.ci = 0.2f;
    a.n = n;
    a.L = L;
    a.g0 = g0;
    a.h = h;
    a.pr = 1.f;   // START and ADD outputs are multiplied by pr + i pi
    a.pi = 0.f;
    a.xcd_order = xcd_order ? 1 : 0;
    launch_pass<float>(a, mode, otf, ntiles, s, TileCfg{tb, nt, true, 0, false});
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// Host-only: the pass sequence for degree K and P orientations as (mode,
// orientation, k, fin) quadruples; returns the number of passes (or the
// capacity needed when cap is too small).
int qw_debug_schedule(int K, int P, int *out, int cap)
{
    const std::vector<SchedPass> S = fused_schedule(K, P);
    if ((int)S.size() <= cap && out)
        for (size_t i = 0; i < S.size(); ++i) {
            out[4 * i] = S[i].mode;
            out[4 * i + 1] = S[i].orient;
            out[4 * i + 2] = S[i].k;
            out[4 * i + 3] = S[i].fin;
        }
    return (int)S.size();
}

// Host-only self check of the pass index maps; returns the number of passes or
// a negative code.  Exported for the CPU test-suite.
int qw_debug_check_plan(int n, int precision) { return check_plan(n, precision); }

}  // extern "C"
