// Batched exp(-i t_i H_i) psi_i for many independent instances of uneven size.
//
// Section III.A of the paper concatenates 2^(24-n) equal-size instances and
// uses one shared polynomial of the largest radius.  Here every instance keeps
// its own shift, bound and coefficients, and sizes may differ:
//
//  * instances with n <= 13 run their whole recurrence inside one workgroup
//    (vector resident in LDS): one persistent launch drains them in
//    descending order of cost N*K;
//  * instances with 14 <= n <= 22 run the fused two-orientation schedule of the
//    single-instance path (one pass per Clenshaw term), grouped: instances are
//    sorted by degree K so that at global step s the still-active ones form a
//    prefix of one tile table, and each step is one launch over that prefix.
//    The launches are captured into a HIP graph.  Optionally the large instances are split into
//    "waves" whose working set (20 bytes per amplitude) fits the 256 MB
//    last-level cache, each wave running all of its steps before the next; the
//    wave size is picked by qw_batched_tune_c64 and stored in a tune file.
//
// Spectral bounds and normalised diagonals are generated on the device from
// the couplings of every instance (section III.A: only the couplings are sent).
#include "qw_kernels.h"

#include <cstdio>
#include <fstream>
#include <numeric>
#include <sstream>

namespace qw {

struct BatchDesc {
    // energy tables
    const double *h, *J;
    double *Q;
    int n, LB;
    int tile0, ntiles;     // range of this instance in the energy tile table
    // recurrence
    const float2 *psi;
    float2 *out;
    float *d;
    float2 *B1, *B2;
    const float2 *coef;    // c_0..c_K
    double c, inv_r;
    float g, pr, pi;
    int K;
};

// Q tables of all instances: grid (chunks of 256 low-bit patterns, instances).
__global__ void k_qtable_batched(BatchDesc *D)
{
    const BatchDesc &b = D[blockIdx.y];
    const uint32_t lo = blockIdx.x * blockDim.x + threadIdx.x;
    if (lo >= (1u << b.LB)) return;
    double acc = 0.0;
    for (int j = 0; j < b.LB; ++j) {
        const double sj = ((lo >> j) & 1) ? -1.0 : 1.0;
        double fj = 0.0;
        for (int k = j + 1; k < b.LB; ++k) {
            const double Jk = b.J[pair_off(b.n, j, k)];
            fj += ((lo >> k) & 1) ? -Jk : Jk;
        }
        acc += sj * fj;
    }
    b.Q[lo] = acc;
}

// One block per energy tile (instance, high bits): block min / max, or (NORM)
// the normalised diagonal (E - c)/r in float.
template <bool NORM>
__global__ void __launch_bounds__(256) k_energy_batched(const BatchDesc *D, const int2 *etiles, double *part)
{
    __shared__ double f[LB_TAB];
    __shared__ double Cc;
    __shared__ double smin[256], smax[256];
    const int2 tt = etiles[blockIdx.x];
    const BatchDesc &b = D[tt.x];
    EnergyTables T{b.h, b.J, b.Q, b.n, b.LB};
    tile_fields(T, (uint64_t)tt.y, f, &Cc);
    __syncthreads();
    const uint32_t TE = 1u << b.LB;
    double mn = INFINITY, mx = -INFINITY;
    for (uint32_t lo = threadIdx.x; lo < TE; lo += blockDim.x) {
        double e = Cc + b.Q[lo];
        for (int j = 0; j < b.LB; ++j) e += ((lo >> j) & 1) ? -f[j] : f[j];
        if constexpr (NORM) {
            b.d[((uint64_t)tt.y << b.LB) | lo] = (float)((e - b.c) * b.inv_r);
        } else {
            mn = fmin(mn, e);
            mx = fmax(mx, e);
        }
    }
    if constexpr (!NORM) {
        smin[threadIdx.x] = mn;
        smax[threadIdx.x] = mx;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
                smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[2 * blockIdx.x] = smin[0];
            part[2 * blockIdx.x + 1] = smax[0];
        }
    }
}

// Per-instance reduction of the tile partials: block i -> emm[2i], emm[2i+1].
__global__ void __launch_bounds__(256) k_minmax_instances(const BatchDesc *D, const double *part, double *emm)
{
    const BatchDesc &b = D[blockIdx.x];
    double mn = INFINITY, mx = -INFINITY;
    for (int i = b.tile0 + threadIdx.x; i < b.tile0 + b.ntiles; i += blockDim.x) {
        mn = fmin(mn, part[2 * i]);
        mx = fmax(mx, part[2 * i + 1]);
    }
    __shared__ double smin[256], smax[256];
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        emm[2 * blockIdx.x] = smin[0];
        emm[2 * blockIdx.x + 1] = smax[0];
    }
}

// b1 = c_K psi over one 2^13 tile of a large instance (b_{K+1} = 0 is never
// read: the first pass takes no accumulator).
__global__ void __launch_bounds__(256) k_init_batched(const BatchDesc *D, const int2 *tiles)
{
    const int2 tt = tiles[blockIdx.x];
    const BatchDesc &b = D[tt.x];
    const float2 cK = b.coef[b.K];
    const uint64_t base = (uint64_t)tt.y << Cfg<float>::TB;
    for (uint32_t e = threadIdx.x; e < (1u << Cfg<float>::TB); e += blockDim.x) {
        const float2 p = b.psi[base + e];
        b.B1[base + e] = make_float2(cK.x * p.x - cK.y * p.y, cK.x * p.y + cK.y * p.x);
    }
}

// Global step `step` of the fused two-orientation schedule for the tile
// (instance, t) of this block.  Every instance with 14 <= n <= 22 runs
// K + 1 passes: step 0 starts term K-1 in the low orientation (MODE START);
// step j (1 <= j < K) completes term K-j and starts term K-j-1 in one fused
// pass; step K completes term 0 and writes the output (MODE ADD).  The
// orientation alternates (even steps: the low 13 bits, odd steps: the n-13
// high bits), so it is the same for every active instance of a step; the
// host launches the fused and the final instances of a step separately.
// 1024 threads per workgroup (16 waves, one workgroup per CU): the per-instance
// arguments live in vector registers here, so fewer amplitudes per thread keep
// the fused pass free of spills (capped at 64 registers for two workgroups per
// CU it spilled and ran 6 % slower).  STREAM: the b vectors carry the
// non-temporal hint and psi and the diagonal stay cacheable, for waves whose
// vectors exceed the memory-side cache (256 instances of 12..22 qubits, 7.7 GB:
// 1093 -> 1020 ms; the hint on psi and the diagonal as well: 1043 ms).
static constexpr int BNT = 1024;

// c_k of an instance, read through a global pointer (one value for the block)
__device__ __forceinline__ float2 coef_at(const float2 *coef, int k)
{
    const QW_GLOBAL float *c = (const QW_GLOBAL float *)(coef + k);
    return make_float2(c[0], c[1]);
}

template <bool HIGH, int MODE, bool STREAM = false>
__global__ void __launch_bounds__(BNT) __attribute__((amdgpu_waves_per_eu(4)))
k_pass_batched(const BatchDesc *D, const int2 *tiles, int step)
{
    constexpr int TB = Cfg<float>::TB, NT = BNT;
    __shared__ float2 lds[1 << TB];
    const int2 tt = wave_uniform(tiles[blockIdx.x]);
    const BatchDesc b = wave_uniform(D[tt.x]);
    const bool swapped = (step >= 1) && ((step - 1) & 1);   // one swap after every fused step
    float2 *X = swapped ? b.B2 : b.B1;
    float2 *Y = swapped ? b.B1 : b.B2;
    PassArgs<float> a{};
    a.b1 = X;
    a.psi = b.psi;
    a.d = b.d;
    a.g = b.g;
    a.n = b.n;
    a.pr = 1.f;
    a.pi = 0.f;
    if (HIGH) {
        a.h = b.n - TB;
        a.L = TB - a.h;
        a.g0 = TB;
    } else {
        a.L = 0;
        a.g0 = 0;
        a.h = TB;
    }
    if constexpr (MODE == PM_START) {
        const int k = b.K - 1;
        const float2 ck = coef_at(b.coef, k);
        a.acc = nullptr;
        a.dst = Y;
        a.scale = (k == 0) ? 1.f : 2.f;
        a.cr = ck.x;
        a.ci = ck.y;
    } else if constexpr (MODE == PM_ADD) {
        a.acc = Y;
        a.dst = b.out;
        a.scale = 1.f;
        a.pr = b.pr;
        a.pi = b.pi;
    } else {
        const int k = b.K - step;   // completed here; k - 1 is started
        const float2 ck = coef_at(b.coef, k - 1);
        a.acc = Y;
        a.dst = Y;
        a.dst2 = X;
        a.scale = 2.f;
        a.scale2 = (k - 1 == 0) ? 1.f : 2.f;
        a.cr = ck.x;
        a.ci = ck.y;
    }
    pass_tile<float, TB, NT, MODE, false, STREAM, STREAM>(a, (uint64_t)tt.y, lds);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static constexpr int BATCH_MAXN = 22;

struct BatchPlan {
    size_t total = 0;
    size_t off_desc, off_etiles, off_tiles, off_part, off_emm, off_hj, off_q, off_coef, off_items, off_order;
    std::vector<size_t> off_b1, off_b2, off_d;
    int n_etiles = 0, n_tiles = 0, coef_slots = 0, hj_count = 0;
};

// Upper bound on the degree from a bound on the radius computable without the
// GPU: |E(z)| <= sum|h| + sum|J|.
static int degree_bound(const qw_batch_item &it, const double *hJ)
{
    const int n = it.n, np = n * (n - 1) / 2;
    double s = 0.0;
    for (int j = 0; j < n + np; ++j) s += std::fabs(hJ[it.off_hJ + j]);
    const double rmax = s + n * std::fabs(it.gamma);
    // single precision may raise r slightly when rounding gamma/r: pad 1%
    return bessel_cutoff(std::fabs(it.t) * rmax * 1.01 + 1.0) + 2;
}

static BatchPlan plan_batch(const qw_batch_item *items, int count, const double *hJ)
{
    BatchPlan P;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    P.off_b1.resize(count);
    P.off_b2.resize(count);
    P.off_d.resize(count);
    for (int i = 0; i < count; ++i) {
        const int n = items[i].n;
        const size_t N = size_t(1) << n;
        P.n_etiles += (n > LB_TAB) ? (int)(N >> LB_TAB) : 1;
        if (n > Cfg<float>::TB) {
            P.off_b1[i] = take(N * 8);
            P.off_b2[i] = take(N * 8);
            P.n_tiles += (int)(N >> Cfg<float>::TB);
        } else {
            P.off_b1[i] = P.off_b2[i] = size_t(-1);
        }
        P.off_d[i] = take(N * 4);
        P.coef_slots += degree_bound(items[i], hJ) + 1;
        P.hj_count += n + n * (n - 1) / 2;
    }
    P.off_desc = take(sizeof(BatchDesc) * count);
    P.off_etiles = take(sizeof(int2) * P.n_etiles);
    P.off_tiles = take(sizeof(int2) * std::max(P.n_tiles, 1));
    P.off_part = take(2 * sizeof(double) * P.n_etiles);
    P.off_emm = take(2 * sizeof(double) * count);
    P.off_hj = take(sizeof(double) * P.hj_count);
    P.off_q = take(sizeof(double) * (size_t(1) << LB_TAB) * count);
    P.off_coef = take(sizeof(float2) * P.coef_slots);
    P.off_items = take(sizeof(OnchipItem<float>) * count);
    P.off_order = take(sizeof(int) * count);
    P.total = off;
    return P;
}

static qw_status validate_batch(const qw_batch_item *items, int count, const double *hJ)
{
    if (!items || count < 1 || !hJ) { set_error("items, count >= 1 and the coupling pool are required"); return QW_EINVAL; }
    for (int i = 0; i < count; ++i) {
        const qw_batch_item &it = items[i];
        if (it.n < 1 || it.n > BATCH_MAXN) { set_error("batched instances need 1 <= n <= 22"); return QW_EINVAL; }
        if (!finite(it.gamma) || !finite(it.t) || !(it.tol > 0.0) || !finite(it.tol)) {
            set_error("instance " + std::to_string(i) + ": gamma, t must be finite and tol > 0");
            return QW_EINVAL;
        }
        if (it.off_hJ < 0 || it.off_psi < 0 || it.off_out < 0) { set_error("negative pool offset"); return QW_EINVAL; }
        const int np = it.n * (it.n - 1) / 2;
        for (int j = 0; j < it.n + np; ++j)
            if (!finite(hJ[it.off_hJ + j])) { set_error("non-finite coupling"); return QW_EINVAL; }
        const int vec = 2;  // complex64 pairs: 16-byte alignment of every state
        if ((it.n > 1 && (it.off_psi % vec || it.off_out % vec))) {
            set_error("state offsets must be even (16-byte aligned)");
            return QW_EINVAL;
        }
    }
    return QW_OK;
}

// Wave size in bytes from the tune file (0 = all large instances together).
static size_t read_tuned_wave(const char *path, const std::string &sig)
{
    if (!path) return 0;
    std::ifstream f(path);
    std::string line;
    size_t best = 0;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string s;
        size_t w;
        if (is >> s >> w && s == sig) best = w;
    }
    return best;
}

static std::string batch_signature(const qw_batch_item *items, int count)
{
    // size histogram: the schedule depends on the sizes only
    int hist[BATCH_MAXN + 1] = {0};
    for (int i = 0; i < count; ++i) hist[items[i].n]++;
    std::ostringstream os;
    os << "c64";
    for (int n = 1; n <= BATCH_MAXN; ++n)
        if (hist[n]) os << "_" << n << "x" << hist[n];
    return os.str();
}

struct BatchRun {
    std::vector<int> large, small;   // instance indices
    std::vector<int> K;
    int maxK = 0;
    long long amp_terms = 0;
    int launches = 0, waves = 0;
};

static qw_status batched_impl(const qw_batch_item *items, int count, const double *hJ, const void *psi_pool,
                              void *out_pool, int method, void *workspace, size_t ws_bytes, size_t wave_bytes,
                              bool use_graph, hipStream_t s, qw_batch_info *info)
{
    qw_status st = validate_batch(items, count, hJ);
    if (st != QW_OK) return st;
    if (method != QW_CHEB && method != QW_CF) { set_error("unknown method"); return QW_EINVAL; }
    if (!psi_pool || !out_pool || !workspace) { set_error("pools and workspace are required"); return QW_EINVAL; }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) || (reinterpret_cast<uintptr_t>(psi_pool) & 15) ||
        (reinterpret_cast<uintptr_t>(out_pool) & 15)) {
        set_error("workspace must be 256-byte and pools 16-byte aligned");
        return QW_EINVAL;
    }
    const BatchPlan P = plan_batch(items, count, hJ);
    if (ws_bytes < P.total) { set_error("workspace too small: need " + std::to_string(P.total)); return QW_ENOMEM; }
    char *ws = static_cast<char *>(workspace);
    const float2 *psi = static_cast<const float2 *>(psi_pool);
    float2 *out = static_cast<float2 *>(out_pool);

    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    const bool timing = info && info->timing;
    if (timing)
        for (auto &e : ev) QW_HIP(hipEventCreate(&e));
    struct EvGuard { hipEvent_t *e; ~EvGuard() { for (int i = 0; i < 3; ++i) if (e[i]) (void)hipEventDestroy(e[i]); } } eg{ev};
    if (timing) QW_HIP(hipEventRecord(ev[0], s));

    // couplings and descriptors (energy part)
    std::vector<double> hjh(P.hj_count);
    std::vector<BatchDesc> desc(count);
    std::vector<int2> etiles;
    etiles.reserve(P.n_etiles);
    double *dhj = reinterpret_cast<double *>(ws + P.off_hj);
    size_t hoff = 0;
    for (int i = 0; i < count; ++i) {
        const qw_batch_item &it = items[i];
        const int n = it.n, np = n * (n - 1) / 2;
        std::memcpy(hjh.data() + hoff, hJ + it.off_hJ, (n + np) * sizeof(double));
        BatchDesc &b = desc[i];
        std::memset(&b, 0, sizeof(b));
        b.h = dhj + hoff;
        b.J = dhj + hoff + n;
        hoff += n + np;
        b.Q = reinterpret_cast<double *>(ws + P.off_q) + (size_t(1) << LB_TAB) * i;
        b.n = n;
        b.LB = std::min(n, LB_TAB);
        b.tile0 = (int)etiles.size();
        const int nt = (n > LB_TAB) ? (1 << (n - LB_TAB)) : 1;
        b.ntiles = nt;
        for (int t = 0; t < nt; ++t) etiles.push_back(make_int2(i, t));
        b.psi = psi + it.off_psi;
        b.out = out + it.off_out;
        b.d = reinterpret_cast<float *>(ws + P.off_d[i]);
        if (P.off_b1[i] != size_t(-1)) {
            b.B1 = reinterpret_cast<float2 *>(ws + P.off_b1[i]);
            b.B2 = reinterpret_cast<float2 *>(ws + P.off_b2[i]);
        }
    }
    BatchDesc *dD = reinterpret_cast<BatchDesc *>(ws + P.off_desc);
    int2 *dE = reinterpret_cast<int2 *>(ws + P.off_etiles);
    double *dpart = reinterpret_cast<double *>(ws + P.off_part);
    double *demm = reinterpret_cast<double *>(ws + P.off_emm);
    QW_HIP(hipMemcpyAsync(dhj, hjh.data(), hjh.size() * sizeof(double), hipMemcpyHostToDevice, s));
    QW_HIP(hipMemcpyAsync(dD, desc.data(), desc.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
    QW_HIP(hipMemcpyAsync(dE, etiles.data(), etiles.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_qtable_batched, dim3((1 << LB_TAB) / 256, count), dim3(256), 0, s, dD);
    hipLaunchKernelGGL(k_energy_batched<false>, dim3(P.n_etiles), dim3(256), 0, s, (const BatchDesc *)dD,
                       (const int2 *)dE, dpart);
    hipLaunchKernelGGL(k_minmax_instances, dim3(count), dim3(256), 0, s, (const BatchDesc *)dD,
                       (const double *)dpart, demm);
    QW_HIP(hipGetLastError());
    std::vector<double> emm(2 * count);
    QW_HIP(hipMemcpyAsync(emm.data(), demm, emm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));

    // per-instance shift, bound, coefficients
    BatchRun run;
    run.K.resize(count);
    std::vector<float2> coefh(P.coef_slots);
    std::vector<OnchipItem<float>> oitems(count);
    float2 *dcoef = reinterpret_cast<float2 *>(ws + P.off_coef);
    int coff = 0;
    for (int i = 0; i < count; ++i) {
        const qw_batch_item &it = items[i];
        BatchDesc &b = desc[i];
        const double emin = emm[2 * i], emax = emm[2 * i + 1];
        if (!finite(emin) || !finite(emax)) { set_error("non-finite energies"); return QW_EINVAL; }
        const double c = 0.5 * (emax + emin);
        double r = 0.5 * (emax - emin) + it.n * std::fabs(it.gamma);
        double g = (r > 0.0) ? it.gamma / r : 0.0;
        if (it.gamma != 0.0 && r > 0.0) {
            float gf = (float)g;
            if (std::fabs((double)gf) > std::fabs(g)) gf = std::nextafter(gf, 0.0f);
            g = (double)gf;
            r = it.gamma / g;
        }
        std::vector<double> alpha;
        int K = 0;
        double err = 0.0;
        if (r > 0.0) {
            if (coefficients(it.t * r, it.tol, method, alpha, &K, &err) != 0) { set_error("coefficients"); return QW_ENOCONV; }
        } else {
            alpha.assign(1, 1.0);  // H = c I: exp(-itc) only
            K = 0;
        }
        if (K == 0 && it.n > Cfg<float>::TB) {
            // the grouped two-pass schedule needs one step: pad with c_1 = 0,
            // so the final step gives H~ 0 - 0 + c_0 psi
            alpha.resize(2);
            alpha[1] = 0.0;
            K = 1;
        }
        const int slots = degree_bound(it, hJ) + 1;
        if (K + 1 > slots) { set_error("internal: degree bound exceeded"); return QW_ENOCONV; }
        for (int k = 0; k <= K; ++k) {
            double cr, ci;
            coef_of(alpha, k, cr, ci);
            coefh[coff + k] = make_float2((float)cr, (float)ci);
        }
        b.coef = dcoef + coff;
        coff += slots;
        b.c = c;
        b.inv_r = (r > 0.0) ? 1.0 / r : 0.0;
        b.g = (float)g;
        b.pr = (float)std::cos(it.t * c);
        b.pi = (float)-std::sin(it.t * c);
        b.K = K;
        run.K[i] = K;
        run.amp_terms += (long long)K << it.n;
        if (it.n <= Cfg<float>::TB) run.small.push_back(i);
        else run.large.push_back(i);
        oitems[i] = OnchipItem<float>{b.psi, b.out, b.d, b.coef, b.g, b.pr, b.pi, it.n, K};
    }
    QW_HIP(hipMemcpyAsync(dcoef, coefh.data(), coefh.size() * sizeof(float2), hipMemcpyHostToDevice, s));
    QW_HIP(hipMemcpyAsync(dD, desc.data(), desc.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_energy_batched<true>, dim3(P.n_etiles), dim3(256), 0, s, (const BatchDesc *)dD,
                       (const int2 *)dE, dpart);
    QW_HIP(hipGetLastError());

    // small class: one persistent launch, costliest first
    std::sort(run.small.begin(), run.small.end(), [&](int a, int b) {
        return ((long long)run.K[a] << items[a].n) > ((long long)run.K[b] << items[b].n);
    });
    OnchipItem<float> *ditems = reinterpret_cast<OnchipItem<float> *>(ws + P.off_items);
    int *dorder = reinterpret_cast<int *>(ws + P.off_order);
    QW_HIP(hipMemcpyAsync(ditems, oitems.data(), oitems.size() * sizeof(OnchipItem<float>), hipMemcpyHostToDevice, s));
    if (!run.small.empty())
        QW_HIP(hipMemcpyAsync(dorder, run.small.data(), run.small.size() * sizeof(int), hipMemcpyHostToDevice, s));

    // large class: waves, each sorted by degree (descending) into the tile table
    std::vector<int> L = run.large;
    std::sort(L.begin(), L.end(), [&](int a, int b) { return run.K[a] > run.K[b]; });
    std::vector<std::vector<int>> waves;
    {
        // greedy packing in degree order up to wave_bytes of working set
        std::vector<int> cur;
        size_t cur_bytes = 0;
        for (int i : L) {
            const size_t bytes = (size_t(20)) << items[i].n;
            if (wave_bytes && !cur.empty() && cur_bytes + bytes > wave_bytes) {
                waves.push_back(cur);
                cur.clear();
                cur_bytes = 0;
            }
            cur.push_back(i);
            cur_bytes += bytes;
        }
        if (!cur.empty()) waves.push_back(cur);
    }
    std::vector<int2> tiles;
    tiles.reserve(P.n_tiles);
    // prefix[j]: tiles of the instances still active at step j (K >= j)
    struct WaveSched { int tile_begin; std::vector<int> prefix; bool stream; };
    std::vector<WaveSched> sched;
    for (auto &w : waves) {
        std::sort(w.begin(), w.end(), [&](int a, int b) { return run.K[a] > run.K[b]; });
        WaveSched ws_{(int)tiles.size(), {}, false};
        std::vector<int> cum;
        double wave_vec_bytes = 0.0;   // b1, b2, psi, out (8 B each) and the diagonal per amplitude
        for (int i : w) {
            wave_vec_bytes += std::ldexp(36.0, items[i].n);
            const int nt = 1 << (items[i].n - Cfg<float>::TB);
            for (int t = 0; t < nt; ++t) tiles.push_back(make_int2(i, t));
            cum.push_back((int)tiles.size() - ws_.tile_begin);
        }
        ws_.stream = wave_vec_bytes > 384.0 * (1 << 20);
        const int maxK = run.K[w.front()];
        ws_.prefix.resize(maxK + 1);
        size_t j = w.size();
        for (int st = 0; st <= maxK; ++st) {
            while (j > 0 && run.K[w[j - 1]] < st) --j;
            ws_.prefix[st] = (j > 0) ? cum[j - 1] : 0;
        }
        sched.push_back(std::move(ws_));
        run.maxK = std::max(run.maxK, maxK);
    }
    int2 *dT = reinterpret_cast<int2 *>(ws + P.off_tiles);
    if (!tiles.empty())
        QW_HIP(hipMemcpyAsync(dT, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    QW_HIP(hipStreamSynchronize(s));   // host staging buffers go out of scope below
    if (timing) QW_HIP(hipEventRecord(ev[1], s));

    if (!run.small.empty()) {
        const int grid = std::min<int>((int)run.small.size(), 512);
        hipLaunchKernelGGL((k_onchip<float, Cfg<float>::TB, ONCHIP_NT>), dim3(grid), dim3(ONCHIP_NT), 0, s,
                           (const OnchipItem<float> *)ditems, (const int *)dorder, (int)run.small.size());
        QW_HIP(hipGetLastError());
        run.launches++;
    }
    if (s == nullptr) use_graph = false;   // the null stream cannot be captured
    if (!sched.empty()) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        if (use_graph) QW_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (const WaveSched &w : sched) {
            const int2 *wt = dT + w.tile_begin;
            hipLaunchKernelGGL(k_init_batched, dim3(w.prefix[0]), dim3(256), 0, s, (const BatchDesc *)dD, wt);
            run.launches++;
            const int last = (int)w.prefix.size() - 1;   // = the largest K of the wave
            auto launch = [&](int mode, bool high, int begin, int count, int st) {
                if (count <= 0) return;
                const dim3 g(count), bl(BNT);
                const int2 *t0 = wt + begin;
                const BatchDesc *dd = dD;
                if (w.stream) {
                    if (mode == PM_START) hipLaunchKernelGGL((k_pass_batched<false, PM_START, true>), g, bl, 0, s, dd, t0, st);
                    else if (mode == PM_FUSED && high) hipLaunchKernelGGL((k_pass_batched<true, PM_FUSED, true>), g, bl, 0, s, dd, t0, st);
                    else if (mode == PM_FUSED) hipLaunchKernelGGL((k_pass_batched<false, PM_FUSED, true>), g, bl, 0, s, dd, t0, st);
                    else if (high) hipLaunchKernelGGL((k_pass_batched<true, PM_ADD, true>), g, bl, 0, s, dd, t0, st);
                    else hipLaunchKernelGGL((k_pass_batched<false, PM_ADD, true>), g, bl, 0, s, dd, t0, st);
                } else {
                    if (mode == PM_START) hipLaunchKernelGGL((k_pass_batched<false, PM_START>), g, bl, 0, s, dd, t0, st);
                    else if (mode == PM_FUSED && high) hipLaunchKernelGGL((k_pass_batched<true, PM_FUSED>), g, bl, 0, s, dd, t0, st);
                    else if (mode == PM_FUSED) hipLaunchKernelGGL((k_pass_batched<false, PM_FUSED>), g, bl, 0, s, dd, t0, st);
                    else if (high) hipLaunchKernelGGL((k_pass_batched<true, PM_ADD>), g, bl, 0, s, dd, t0, st);
                    else hipLaunchKernelGGL((k_pass_batched<false, PM_ADD>), g, bl, 0, s, dd, t0, st);
                }
                run.launches++;
            };
            for (int st = 0; st <= last; ++st) {
                const bool high = (st & 1) != 0;
                if (st == 0) {
                    launch(PM_START, false, 0, w.prefix[0], 0);
                    continue;
                }
                // instances with K > st fuse, those with K == st finish
                const int nfuse = (st + 1 <= last) ? w.prefix[st + 1] : 0;
                launch(PM_FUSED, high, 0, nfuse, st);
                launch(PM_ADD, high, nfuse, w.prefix[st] - nfuse, st);
            }
        }
        if (use_graph) {
            hipError_t e1 = hipStreamEndCapture(s, &graph);
            if (e1 != hipSuccess) { set_error(std::string("graph capture: ") + hipGetErrorString(e1)); return QW_EHIP; }
            hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e2 != hipSuccess) {
                (void)hipGraphDestroy(graph);
                set_error(std::string("graph instantiate: ") + hipGetErrorString(e2));
                return QW_EHIP;
            }
            hipError_t e3 = hipGraphLaunch(exec, s);
            hipError_t e4 = hipStreamSynchronize(s);
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            if (e3 != hipSuccess || e4 != hipSuccess) {
                set_error(std::string("graph launch: ") + hipGetErrorString(e3 != hipSuccess ? e3 : e4));
                return QW_EHIP;
            }
        } else {
            QW_HIP(hipGetLastError());
        }
    }
    if (info) {
        info->count = count;
        info->small_count = (int)run.small.size();
        info->large_count = (int)run.large.size();
        info->max_K = std::max(run.maxK, [&] { int m = 0; for (int i : run.small) m = std::max(m, run.K[i]); return m; }());
        info->launches = run.launches;
        info->waves = (int)waves.size();
        info->amp_terms = run.amp_terms;
        info->wave_bytes = (long long)wave_bytes;
    }
    if (timing) {
        QW_HIP(hipEventRecord(ev[2], s));
        QW_HIP(hipEventSynchronize(ev[2]));
        QW_HIP(hipEventElapsedTime(&info->setup_ms, ev[0], ev[1]));
        QW_HIP(hipEventElapsedTime(&info->loop_ms, ev[1], ev[2]));
    }
    return QW_OK;
}

}  // namespace qw

using namespace qw;

extern "C" {

size_t qw_batched_workspace_bytes_c64(const qw_batch_item *items, int count, const double *hJ_pool)
{
    if (validate_batch(items, count, hJ_pool) != QW_OK) return 0;
    return plan_batch(items, count, hJ_pool).total;
}

qw_status qw_expm_action_batched_c64(const qw_batch_item *items, int count, const double *hJ_pool,
                                     const void *psi_pool, void *out_pool, qw_method method, void *workspace,
                                     size_t ws_bytes, const char *tune_cache, void *stream, qw_batch_info *info)
{
    if (info) {
        const int t = info->timing;
        std::memset(info, 0, sizeof(*info));
        info->timing = t;
    }
    if (!items || count < 1) { set_error("items and count >= 1 are required"); return QW_EINVAL; }
    const size_t wave = read_tuned_wave(tune_cache, batch_signature(items, count));
    return batched_impl(items, count, hJ_pool, psi_pool, out_pool, (int)method, workspace, ws_bytes, wave, true,
                        reinterpret_cast<hipStream_t>(stream), info);
}

qw_status qw_batched_tune_c64(const qw_batch_item *items, int count, const double *hJ_pool, const void *psi_pool,
                              void *out_pool, void *workspace, size_t ws_bytes, const char *tune_cache,
                              void *stream, long long *best_wave_bytes)
{
    if (!items || count < 1) { set_error("items and count >= 1 are required"); return QW_EINVAL; }
    const long long cands[] = {0, 512ll << 20, 256ll << 20, 192ll << 20, 128ll << 20, 64ll << 20};
    float best_ms = INFINITY;
    long long best = 0;
    for (long long w : cands) {
        qw_batch_info bi{};
        bi.timing = 1;
        qw_status st = batched_impl(items, count, hJ_pool, psi_pool, out_pool, QW_CHEB, workspace, ws_bytes,
                                    (size_t)w, true, reinterpret_cast<hipStream_t>(stream), &bi);
        if (st != QW_OK) return st;
        if (bi.loop_ms < best_ms) {
            best_ms = bi.loop_ms;
            best = w;
        }
    }
    if (best_wave_bytes) *best_wave_bytes = best;
    if (tune_cache) {
        FILE *f = std::fopen(tune_cache, "a");
        if (!f) { set_error(std::string("cannot write tune cache ") + tune_cache); return QW_EINVAL; }
        std::fprintf(f, "%s %lld %.3f\n", batch_signature(items, count).c_str(), best, best_ms);
        std::fclose(f);
    }
    return QW_OK;
}

qw_status qw_expm_action_batched_c64_sched(const qw_batch_item *items, int count, const double *hJ_pool,
                                           const void *psi_pool, void *out_pool, qw_method method,
                                           void *workspace, size_t ws_bytes, long long wave_bytes, int use_graph,
                                           void *stream, qw_batch_info *info)
{
    if (info) {
        const int t = info->timing;
        std::memset(info, 0, sizeof(*info));
        info->timing = t;
    }
    if (wave_bytes < 0) { set_error("wave_bytes must be >= 0"); return QW_EINVAL; }
    return batched_impl(items, count, hJ_pool, psi_pool, out_pool, (int)method, workspace, ws_bytes,
                        (size_t)wave_bytes, use_graph != 0, reinterpret_cast<hipStream_t>(stream), info);
}

}  // extern "C"
