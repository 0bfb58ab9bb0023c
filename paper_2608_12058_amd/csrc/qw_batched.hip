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

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
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

// Global step `step` of the fused two-orientation schedule for the tile
// (instance, t) of this block.  Every instance of the multi-pass class runs
// K + 1 passes: step 0 starts term K-1 in the low orientation (MODE START);
// step j (1 <= j < K) completes term K-j and starts term K-j-1 in one fused
// pass; step K completes term 0 and writes the output (MODE ADD).  The
// orientation alternates (even steps: the low TB bits, odd steps: the n - TB
// high bits), so it is the same for every active instance of a step; the
// host launches the fused and the final instances of a step separately.  The
// Clenshaw start b_K = c_K psi is folded into the loads: steps 0 and 1 read
// psi scaled by c_K as b_{k+1}, so b_K is never stored.
//
// Tile classes (chosen per instance size by the tuner): MID = 2^13 tiles with
// 1024 threads (8 amplitudes per thread; the per-instance arguments live in
// vector registers, so fewer amplitudes per thread keep the fused pass free
// of spills), NARROW = 2^12 tiles with 1024 threads (n <= 20), WIDE_T = 2^13
// tiles with 512 threads.  STREAM: the b vectors carry the non-temporal hint
// and psi and the diagonal stay cacheable, for waves whose vectors exceed the
// memory-side cache (256 instances of 12..22 qubits, 7.7 GB: 1093 -> 1020 ms;
// the hint on psi and the diagonal as well: 1043 ms).
enum BatchClass { BC_MID = 0, BC_NARROW = 1, BC_WIDE_T = 2, BC_COUNT = 3 };
template <int C> struct ClassShape;
template <> struct ClassShape<BC_MID> { static constexpr int TB = 13, NT = 1024; };
template <> struct ClassShape<BC_NARROW> { static constexpr int TB = 12, NT = 1024; };
template <> struct ClassShape<BC_WIDE_T> { static constexpr int TB = 13, NT = 512; };
inline int class_tb(int c) { return c == BC_NARROW ? 12 : 13; }

// c_k of an instance, read through a global pointer (one value for the block)
__device__ __forceinline__ float2 coef_at(const float2 *coef, int k)
{
    const QW_GLOBAL float *c = (const QW_GLOBAL float *)(coef + k);
    return make_float2(c[0], c[1]);
}

template <int CLS, bool HIGH, int MODE, bool STREAM = false>
__global__ void __launch_bounds__(ClassShape<CLS>::NT) __attribute__((amdgpu_waves_per_eu(4)))
k_pass_batched(const BatchDesc *D, const int2 *tiles, int step)
{
    constexpr int TB = ClassShape<CLS>::TB, NT = ClassShape<CLS>::NT;
    __shared__ float2 lds[1 << TB];
    const int2 tt = wave_uniform(tiles[blockIdx.x]);
    const BatchDesc b = wave_uniform(D[tt.x]);
    const bool swapped = (step >= 1) && ((step - 1) & 1);   // one swap after every fused step
    float2 *X = swapped ? b.B2 : b.B1;
    float2 *Y = swapped ? b.B1 : b.B2;
    PassArgs<float> a{};
    a.b1 = X;
    if (step <= 1) {
        // b_{k+1} = b_K = c_K psi (b_K itself is never stored)
        const float2 cK = coef_at(b.coef, b.K);
        a.b1 = b.psi;
        a.b1_scaled = 1;
        a.b1r = cK.x;
        a.b1i = cK.y;
    }
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

// Schedule of a batch: the largest size run whole in one workgroup, the tile
// class of every larger size, the working-set cap of a wave, and whether the
// one-workgroup launch runs beside the passes on a side stream.
struct BatchSched {
    long long wave_bytes = 0;
    int onchip_nmax = Cfg<float>::TB;
    int concurrent = 0;
    signed char cls[BATCH_MAXN + 1];
    BatchSched() { std::memset(cls, -1, sizeof(cls)); }
};

// Class actually used for a multi-pass instance of n qubits: the requested
// one, else NARROW for n = 13 (the only class with two orientations there)
// and MID above.
static int class_for(const BatchSched &S, int n)
{
    const int c = S.cls[n];
    if (c >= 0) return c;
    return (n <= 13) ? (int)BC_NARROW : (int)BC_MID;
}

static qw_status validate_sched(const BatchSched &S)
{
    if (S.wave_bytes < 0) { set_error("wave_bytes must be >= 0"); return QW_EINVAL; }
    if (S.onchip_nmax != 12 && S.onchip_nmax != 13) { set_error("onchip_nmax must be 12 or 13"); return QW_EINVAL; }
    for (int n = 1; n <= BATCH_MAXN; ++n) {
        const int c = S.cls[n];
        if (c < -1 || c >= BC_COUNT) { set_error("tile class must be -1, 0, 1 or 2"); return QW_EINVAL; }
        if (n <= S.onchip_nmax || c < 0) continue;
        // two orientations of at most TB bits each, the high one with >= 4 passenger bits
        const int tb = class_tb(c);
        if (n <= tb || n - tb > tb - Cfg<float>::LMIN) {
            set_error("tile class " + std::to_string(c) + " cannot hold " + std::to_string(n) + " qubits");
            return QW_EINVAL;
        }
    }
    return QW_OK;
}

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

// Workspace layout; it does not depend on the schedule: every instance of
// n >= 13 has its two work vectors and room for its tiles in the smallest
// tile class.
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
        if (n >= 13) {
            P.off_b1[i] = take(N * 8);
            P.off_b2[i] = take(N * 8);
            P.n_tiles += (int)(N >> 12);
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

// Tune file: one line per tuning, "<signature> wave=<bytes> onchip=<n>
// conc=<0|1> classes=<one digit per n = 1..22, '-' = default> ms=<time>"; the
// last line of the batch's signature wins.
static std::string sched_fields(const BatchSched &S)
{
    std::ostringstream os;
    os << "wave=" << S.wave_bytes << " onchip=" << S.onchip_nmax << " conc=" << S.concurrent << " classes=";
    for (int n = 1; n <= BATCH_MAXN; ++n) os << (S.cls[n] < 0 ? '-' : (char)('0' + S.cls[n]));
    return os.str();
}

static bool read_tuned_sched(const char *path, const std::string &sig, BatchSched *out)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string s, tok;
        if (!(is >> s) || s != sig) continue;
        BatchSched S;
        bool ok = true;
        while (is >> tok) {
            const size_t eq = tok.find('=');
            if (eq == std::string::npos) { ok = false; break; }
            const std::string k = tok.substr(0, eq), v = tok.substr(eq + 1);
            if (k == "wave") S.wave_bytes = std::atoll(v.c_str());
            else if (k == "onchip") S.onchip_nmax = std::atoi(v.c_str());
            else if (k == "conc") S.concurrent = std::atoi(v.c_str());
            else if (k == "classes") {
                if ((int)v.size() != BATCH_MAXN) { ok = false; break; }
                for (int n = 1; n <= BATCH_MAXN; ++n) S.cls[n] = (v[n - 1] == '-') ? -1 : (signed char)(v[n - 1] - '0');
            }
        }
        if (ok && validate_sched(S) == QW_OK) {
            *out = S;
            found = true;
        }
    }
    return found;
}

// One launch of a batched call.
struct BLaunch {
    int onchip;      // 1: the one-workgroup launch over the small instances
    int cls, mode, high, stream_hint;
    unsigned grid;
    const int2 *tiles;
    int step;
};

template <int C> static void launch_class(const BLaunch &L, const BatchDesc *dD, hipStream_t s)
{
    const dim3 g(L.grid), b(ClassShape<C>::NT);
    const int st = L.step;
    const int2 *t = L.tiles;
    if (L.stream_hint) {
        if (L.mode == PM_START) hipLaunchKernelGGL((k_pass_batched<C, false, PM_START, true>), g, b, 0, s, dD, t, st);
        else if (L.mode == PM_FUSED && L.high) hipLaunchKernelGGL((k_pass_batched<C, true, PM_FUSED, true>), g, b, 0, s, dD, t, st);
        else if (L.mode == PM_FUSED) hipLaunchKernelGGL((k_pass_batched<C, false, PM_FUSED, true>), g, b, 0, s, dD, t, st);
        else if (L.high) hipLaunchKernelGGL((k_pass_batched<C, true, PM_ADD, true>), g, b, 0, s, dD, t, st);
        else hipLaunchKernelGGL((k_pass_batched<C, false, PM_ADD, true>), g, b, 0, s, dD, t, st);
    } else {
        if (L.mode == PM_START) hipLaunchKernelGGL((k_pass_batched<C, false, PM_START>), g, b, 0, s, dD, t, st);
        else if (L.mode == PM_FUSED && L.high) hipLaunchKernelGGL((k_pass_batched<C, true, PM_FUSED>), g, b, 0, s, dD, t, st);
        else if (L.mode == PM_FUSED) hipLaunchKernelGGL((k_pass_batched<C, false, PM_FUSED>), g, b, 0, s, dD, t, st);
        else if (L.high) hipLaunchKernelGGL((k_pass_batched<C, true, PM_ADD>), g, b, 0, s, dD, t, st);
        else hipLaunchKernelGGL((k_pass_batched<C, false, PM_ADD>), g, b, 0, s, dD, t, st);
    }
}

// Side stream of a device (default priority), for the one-workgroup launch
// beside the passes; created once, kept until the process ends.
static qw_status side_stream(hipStream_t *out)
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    QW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) { set_error("device index out of range"); return QW_EINVAL; }
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev]) QW_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
    *out = streams[dev];
    return QW_OK;
}

// Enqueues the launches on s (captured or not).  The one-workgroup launch goes
// first; with `side` it runs on the side stream between a fork and a join
// event, so it overlaps the passes.
static qw_status replay(const std::vector<BLaunch> &Ls, const BatchDesc *dD, const OnchipItem<float> *ditems,
                        const int *dorder, int nsmall, hipStream_t s, hipStream_t side, hipEvent_t fork,
                        hipEvent_t join)
{
    bool joined = true;
    for (const BLaunch &L : Ls) {
        if (L.onchip) {
            hipStream_t os = s;
            if (side) {
                QW_HIP(hipEventRecord(fork, s));
                QW_HIP(hipStreamWaitEvent(side, fork, 0));
                os = side;
                joined = false;
            }
            hipLaunchKernelGGL((k_onchip<float, Cfg<float>::TB, ONCHIP_NT>), dim3(L.grid), dim3(ONCHIP_NT), 0, os,
                               ditems, dorder, nsmall);
            if (side) QW_HIP(hipEventRecord(join, side));
            continue;
        }
        if (L.cls == BC_NARROW) launch_class<BC_NARROW>(L, dD, s);
        else if (L.cls == BC_WIDE_T) launch_class<BC_WIDE_T>(L, dD, s);
        else launch_class<BC_MID>(L, dD, s);
    }
    if (!joined) QW_HIP(hipStreamWaitEvent(s, join, 0));
    QW_HIP(hipGetLastError());
    return QW_OK;
}

// Instantiated graphs of recent calls, keyed by the device, the workspace and
// the exact launch sequence (which fixes every kernel argument: descriptors
// and tile tables are re-uploaded into the same workspace places before each
// replay).  At most GRAPH_CACHE entries; the oldest is destroyed first, after
// its device has finished its work (an eviction waits for the whole device).
static constexpr size_t GRAPH_CACHE = 4;
struct GraphEntry {
    int dev;
    std::string key;
    hipGraphExec_t exec;
};
static std::mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;

static std::string launch_key(const std::vector<BLaunch> &Ls, const void *ws, int conc)
{
    std::ostringstream os;
    os << ws << ':' << conc;
    for (const BLaunch &L : Ls)
        os << ';' << L.onchip << ',' << L.cls << ',' << L.mode << ',' << L.high << ',' << L.stream_hint << ','
           << L.grid << ',' << static_cast<const void *>(L.tiles) << ',' << L.step;
    return os.str();
}

struct BatchRun {
    std::vector<int> large, small;   // instance indices
    std::vector<int> K;
    int maxK = 0;
    long long amp_terms = 0;
    int launches = 0, waves = 0;
    int class_count[BC_COUNT] = {0, 0, 0};
};

static qw_status batched_impl(const qw_batch_item *items, int count, const double *hJ, const void *psi_pool,
                              void *out_pool, int method, void *workspace, size_t ws_bytes, const BatchSched &sch,
                              bool use_graph, hipStream_t s, qw_batch_info *info)
{
    qw_status st = validate_batch(items, count, hJ);
    if (st != QW_OK) return st;
    st = validate_sched(sch);
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

    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // timing 0-2, fork 3, join 4
    const bool timing = info && info->timing;
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int i = 0; i < 5; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } eg{ev};
    if (timing)
        for (int i = 0; i < 3; ++i) QW_HIP(hipEventCreate(&ev[i]));
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
        const bool small = it.n <= sch.onchip_nmax;
        if (K == 0 && !small) {
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
        if (small) run.small.push_back(i);
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

    // large class: waves (greedy in degree order up to wave_bytes of working
    // set), inside a wave one degree-sorted tile table per tile class
    std::vector<int> Lg = run.large;
    std::sort(Lg.begin(), Lg.end(), [&](int a, int b) { return run.K[a] > run.K[b]; });
    std::vector<std::vector<int>> waves;
    {
        std::vector<int> cur;
        size_t cur_bytes = 0;
        for (int i : Lg) {
            const size_t bytes = (size_t(20)) << items[i].n;
            if (sch.wave_bytes && !cur.empty() && cur_bytes + bytes > (size_t)sch.wave_bytes) {
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
    int2 *dT = reinterpret_cast<int2 *>(ws + P.off_tiles);
    std::vector<BLaunch> Ls;
    if (!run.small.empty())
        Ls.push_back({1, 0, 0, 0, 0, (unsigned)std::min<int>((int)run.small.size(), 512), nullptr, 0});
    for (auto &w : waves) {
        double wave_vec_bytes = 0.0;   // b1, b2, psi, out (8 B each) and the diagonal per amplitude
        for (int i : w) wave_vec_bytes += std::ldexp(36.0, items[i].n);
        const int hint = wave_vec_bytes > 384.0 * (1 << 20) ? 1 : 0;
        struct ClassTable { int begin = 0; std::vector<int> prefix; };
        ClassTable ct[BC_COUNT];
        int wave_maxK = 0;
        for (int c = 0; c < BC_COUNT; ++c) {
            std::vector<int> mem;
            for (int i : w)
                if (class_for(sch, items[i].n) == c) mem.push_back(i);
            if (mem.empty()) continue;
            std::sort(mem.begin(), mem.end(), [&](int a, int b) { return run.K[a] > run.K[b]; });
            ct[c].begin = (int)tiles.size();
            std::vector<int> cum;
            const int tb = class_tb(c);
            for (int i : mem) {
                const int nt = 1 << (items[i].n - tb);
                for (int t = 0; t < nt; ++t) tiles.push_back(make_int2(i, t));
                cum.push_back((int)tiles.size() - ct[c].begin);
                run.class_count[c]++;
            }
            const int maxK = run.K[mem.front()];
            wave_maxK = std::max(wave_maxK, maxK);
            ct[c].prefix.resize(maxK + 1);
            size_t j = mem.size();
            for (int stp = 0; stp <= maxK; ++stp) {
                while (j > 0 && run.K[mem[j - 1]] < stp) --j;
                ct[c].prefix[stp] = (j > 0) ? cum[j - 1] : 0;
            }
        }
        for (int stp = 0; stp <= wave_maxK; ++stp) {
            const int high = stp & 1;
            for (int c = 0; c < BC_COUNT; ++c) {
                const std::vector<int> &pre = ct[c].prefix;
                const int last = (int)pre.size() - 1;
                if (stp > last) continue;
                const int2 *t0 = dT + ct[c].begin;
                if (stp == 0) {
                    if (pre[0] > 0) Ls.push_back({0, c, PM_START, 0, hint, (unsigned)pre[0], t0, 0});
                    continue;
                }
                // instances with K > stp fuse, those with K == stp finish
                const int nfuse = (stp + 1 <= last) ? pre[stp + 1] : 0;
                if (nfuse > 0) Ls.push_back({0, c, PM_FUSED, high, hint, (unsigned)nfuse, t0, stp});
                if (pre[stp] - nfuse > 0)
                    Ls.push_back({0, c, PM_ADD, high, hint, (unsigned)(pre[stp] - nfuse), t0 + nfuse, stp});
            }
        }
        run.maxK = std::max(run.maxK, wave_maxK);
    }
    if ((int)tiles.size() > P.n_tiles) { set_error("internal: tile table overflow"); return QW_EINVAL; }
    if (!tiles.empty())
        QW_HIP(hipMemcpyAsync(dT, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    QW_HIP(hipStreamSynchronize(s));   // host staging buffers go out of scope below

    hipStream_t side = nullptr;
    const bool conc = sch.concurrent && !run.small.empty() && !Lg.empty();
    if (conc) {
        st = side_stream(&side);
        if (st != QW_OK) return st;
        QW_HIP(hipEventCreateWithFlags(&ev[3], hipEventDisableTiming));
        QW_HIP(hipEventCreateWithFlags(&ev[4], hipEventDisableTiming));
    }
    if (s == nullptr) use_graph = false;   // the null stream cannot be captured
    int graph_cached = 0;
    float graph_ms = 0.f;
    hipGraphExec_t exec = nullptr;
    if (use_graph && !Ls.empty()) {
        int dev = 0;
        QW_HIP(hipGetDevice(&dev));
        const std::string key = launch_key(Ls, workspace, conc ? 1 : 0);
        std::lock_guard<std::mutex> lock(g_graph_mu);
        for (const GraphEntry &e : g_graphs)
            if (e.dev == dev && e.key == key) exec = e.exec;
        if (exec) {
            graph_cached = 1;
        } else {
            const auto h0 = std::chrono::steady_clock::now();
            hipGraph_t graph = nullptr;
            QW_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            const qw_status rs = replay(Ls, dD, ditems, dorder, (int)run.small.size(), s, side, ev[3], ev[4]);
            hipError_t e1 = hipStreamEndCapture(s, &graph);
            if (rs != QW_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rs;
            }
            if (e1 != hipSuccess) { set_error(std::string("graph capture: ") + hipGetErrorString(e1)); return QW_EHIP; }
            hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e2 != hipSuccess) { set_error(std::string("graph instantiate: ") + hipGetErrorString(e2)); return QW_EHIP; }
            if (g_graphs.size() >= GRAPH_CACHE) {
                // The oldest graph may still run on a stream of an earlier call
                // (the lock covers lookups and launches, not their execution):
                // its device finishes all work before the graph is destroyed.
                const GraphEntry old = g_graphs.front();
                g_graphs.erase(g_graphs.begin());
                if (old.dev != dev) QW_HIP(hipSetDevice(old.dev));
                const hipError_t es = hipDeviceSynchronize();
                if (old.dev != dev) QW_HIP(hipSetDevice(dev));
                QW_HIP(es);
                (void)hipGraphExecDestroy(old.exec);
            }
            g_graphs.push_back({dev, key, exec});
            graph_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - h0).count();
        }
        if (timing) QW_HIP(hipEventRecord(ev[1], s));
        QW_HIP(hipGraphLaunch(exec, s));
    } else {
        if (timing) QW_HIP(hipEventRecord(ev[1], s));
        st = replay(Ls, dD, ditems, dorder, (int)run.small.size(), s, side, ev[3], ev[4]);
        if (st != QW_OK) return st;
    }
    run.launches = (int)Ls.size();
    if (timing) QW_HIP(hipEventRecord(ev[2], s));
    QW_HIP(hipStreamSynchronize(s));
    if (info) {
        info->count = count;
        info->small_count = (int)run.small.size();
        info->large_count = (int)run.large.size();
        info->max_K = std::max(run.maxK, [&] { int m = 0; for (int i : run.small) m = std::max(m, run.K[i]); return m; }());
        info->launches = run.launches;
        info->waves = (int)waves.size();
        info->amp_terms = run.amp_terms;
        info->wave_bytes = sch.wave_bytes;
        info->onchip_nmax = sch.onchip_nmax;
        info->concurrent = conc ? 1 : 0;
        info->graph_cached = graph_cached;
        info->graph_ms = graph_ms;
        for (int c = 0; c < BC_COUNT; ++c) info->class_count[c] = run.class_count[c];
        for (int n = 0; n <= BATCH_MAXN; ++n)
            info->tile_class[n] = (n >= 1 && n > sch.onchip_nmax) ? (signed char)class_for(sch, n) : (signed char)-1;
    }
    if (timing) {
        QW_HIP(hipEventElapsedTime(&info->setup_ms, ev[0], ev[1]));
        QW_HIP(hipEventElapsedTime(&info->loop_ms, ev[1], ev[2]));
    }
    return QW_OK;
}

static BatchSched sched_from(const qw_batch_sched *p)
{
    BatchSched S;
    if (!p) return S;
    S.wave_bytes = p->wave_bytes;
    S.onchip_nmax = p->onchip_nmax ? p->onchip_nmax : Cfg<float>::TB;
    S.concurrent = p->concurrent;
    for (int n = 0; n <= BATCH_MAXN; ++n) S.cls[n] = p->tile_class[n];
    return S;
}

static void sched_to(const BatchSched &S, qw_batch_sched *p)
{
    p->wave_bytes = S.wave_bytes;
    p->onchip_nmax = S.onchip_nmax;
    p->concurrent = S.concurrent;
    for (int n = 0; n <= BATCH_MAXN; ++n) p->tile_class[n] = S.cls[n];
}

}  // namespace qw

using namespace qw;

extern "C" {

size_t qw_batched_workspace_bytes_c64(const qw_batch_item *items, int count, const double *hJ_pool)
{
    if (validate_batch(items, count, hJ_pool) != QW_OK) return 0;
    return plan_batch(items, count, hJ_pool).total;
}

static void clear_info(qw_batch_info *info)
{
    if (info) {
        const int t = info->timing;
        std::memset(info, 0, sizeof(*info));
        info->timing = t;
    }
}

qw_status qw_expm_action_batched_c64(const qw_batch_item *items, int count, const double *hJ_pool,
                                     const void *psi_pool, void *out_pool, qw_method method, void *workspace,
                                     size_t ws_bytes, const char *tune_cache, void *stream, qw_batch_info *info)
{
    clear_info(info);
    if (!items || count < 1) { set_error("items and count >= 1 are required"); return QW_EINVAL; }
    BatchSched S;
    (void)read_tuned_sched(tune_cache, batch_signature(items, count), &S);
    return batched_impl(items, count, hJ_pool, psi_pool, out_pool, (int)method, workspace, ws_bytes, S, true,
                        reinterpret_cast<hipStream_t>(stream), info);
}

qw_status qw_expm_action_batched_c64_sched(const qw_batch_item *items, int count, const double *hJ_pool,
                                           const void *psi_pool, void *out_pool, qw_method method,
                                           void *workspace, size_t ws_bytes, const qw_batch_sched *sched,
                                           int use_graph, void *stream, qw_batch_info *info)
{
    clear_info(info);
    return batched_impl(items, count, hJ_pool, psi_pool, out_pool, (int)method, workspace, ws_bytes, sched_from(sched),
                        use_graph != 0, reinterpret_cast<hipStream_t>(stream), info);
}

// Coordinate search over the schedule, each candidate timed on one call with
// its graph built beforehand (HIP events around the passes only): the tile
// class of each size bucket in turn, then the one-workgroup limit, running the
// one-workgroup launch beside the passes, and the wave size.
qw_status qw_batched_tune_c64(const qw_batch_item *items, int count, const double *hJ_pool, const void *psi_pool,
                              void *out_pool, void *workspace, size_t ws_bytes, const char *tune_cache,
                              void *stream, qw_batch_sched *best_out)
{
    if (!items || count < 1) { set_error("items and count >= 1 are required"); return QW_EINVAL; }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    auto time_of = [&](const BatchSched &S, float *ms) -> qw_status {
        qw_batch_info bi{};
        qw_status st = batched_impl(items, count, hJ_pool, psi_pool, out_pool, QW_CHEB, workspace, ws_bytes, S, true,
                                    s, &bi);   // builds (or finds) the graph
        if (st != QW_OK) return st;
        bi = qw_batch_info{};
        bi.timing = 1;
        st = batched_impl(items, count, hJ_pool, psi_pool, out_pool, QW_CHEB, workspace, ws_bytes, S, true, s, &bi);
        *ms = bi.loop_ms;
        return st;
    };
    int present[BATCH_MAXN + 1] = {0};
    for (int i = 0; i < count; ++i) present[items[i].n] = 1;
    BatchSched best;
    float best_ms = 0.f;
    qw_status st = time_of(best, &best_ms);
    if (st != QW_OK) return st;
    auto consider = [&](const BatchSched &S) -> qw_status {
        if (validate_sched(S) != QW_OK) return QW_OK;   // not a valid candidate for these sizes
        float ms = 0.f;
        const qw_status st2 = time_of(S, &ms);
        if (st2 != QW_OK) return st2;
        if (ms < best_ms) {
            best_ms = ms;
            best = S;
        }
        return QW_OK;
    };
    const int buckets[][2] = {{13, 16}, {17, 18}, {19, 20}, {21, 22}};
    for (const auto &bk : buckets) {
        bool any = false;
        for (int n = bk[0]; n <= bk[1]; ++n) any = any || present[n];
        if (!any) continue;
        for (int c = 0; c < BC_COUNT; ++c) {
            BatchSched S = best;
            for (int n = bk[0]; n <= bk[1]; ++n) S.cls[n] = (signed char)c;
            bool same = true;
            for (int n = bk[0]; n <= bk[1]; ++n)
                if (present[n] && n > S.onchip_nmax && class_for(S, n) != class_for(best, n)) same = false;
            if (same) continue;
            st = consider(S);
            if (st != QW_OK) return st;
        }
    }
    if (present[13]) {
        BatchSched S = best;
        S.onchip_nmax = (best.onchip_nmax == 13) ? 12 : 13;
        if (S.onchip_nmax == 12) S.cls[13] = BC_NARROW;
        st = consider(S);
        if (st != QW_OK) return st;
    }
    {
        BatchSched S = best;
        S.concurrent = !best.concurrent;
        st = consider(S);
        if (st != QW_OK) return st;
    }
    for (long long w : {512ll << 20, 256ll << 20, 128ll << 20}) {
        BatchSched S = best;
        S.wave_bytes = w;
        st = consider(S);
        if (st != QW_OK) return st;
    }
    if (best_out) sched_to(best, best_out);
    if (tune_cache) {
        FILE *f = std::fopen(tune_cache, "a");
        if (!f) { set_error(std::string("cannot write tune cache ") + tune_cache); return QW_EINVAL; }
        std::fprintf(f, "%s %s ms=%.3f\n", batch_signature(items, count).c_str(), sched_fields(best).c_str(), best_ms);
        std::fclose(f);
    }
    return QW_OK;
}

}  // extern "C"
