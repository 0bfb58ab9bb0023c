// Shared device kernels and host helpers of libqwexp (included by every HIP
// translation unit): tile configuration, the Clenshaw pass body, the on-chip
// whole-recurrence kernel, and small host utilities.
#pragma once

#include "qw_device.h"
#include "qw_internal.h"
#include "qwexp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace qw {

// ---------------------------------------------------------------------------
// Compile-time configuration
// ---------------------------------------------------------------------------
template <typename R> struct Cfg;
template <> struct Cfg<float> {
    static constexpr int TB = 13;     // tile bits of a pass (2^13 x 8 B = 64 KB LDS)
    static constexpr int NT = 512;    // threads per pass workgroup
    static constexpr int LMIN = 4;    // passenger bits: rows of >= 128 B
};
template <> struct Cfg<double> {
    static constexpr int TB = 12;     // 2^12 x 16 B = 64 KB LDS
    static constexpr int NT = 512;
    static constexpr int LMIN = 3;
};
static constexpr int ONCHIP_NT = 1024;
static constexpr int MAXPART = 4096;          // reduction partials
static constexpr int KMAX_ONCHIP = 1 << 17;   // coefficient slots for on-chip runs
static constexpr int LB_TAB = 13;             // low bits of the energy tables
static constexpr int KMAX_MON = 1 << 16;      // norm-monitor slots (degree limit when monitoring)

// ---------------------------------------------------------------------------
// Kernels: Ising energies and their range
// ---------------------------------------------------------------------------

// Q[lo] = sum_{j<k<LB} J_jk s_j(lo) s_k(lo).
template <int D = 0>
__global__ void k_qtable(EnergyTables T, double *Q)
{
    const uint32_t lo = blockIdx.x * blockDim.x + threadIdx.x;
    if (lo >= (1u << T.LB)) return;
    double acc = 0.0;
    for (int j = 0; j < T.LB; ++j) {
        const double sj = ((lo >> j) & 1) ? -1.0 : 1.0;
        double fj = 0.0;
        for (int k = j + 1; k < T.LB; ++k) {
            const double Jk = T.J[pair_off(T.n, j, k)];
            fj += ((lo >> k) & 1) ? -Jk : Jk;
        }
        acc += sj * fj;
    }
    Q[lo] = acc;
}

__device__ inline void block_minmax(double lo, double hi, double *part)
{
    __shared__ double smin[256], smax[256];
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
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

// Min / max of E over all z generated from the tables (grid-stride over tiles
// of 2^LB consecutive indices).  256 threads.
template <int D = 0>
__global__ void __launch_bounds__(256) k_minmax_energy(EnergyTables T, double *part)
{
    __shared__ double f[LB_TAB];
    __shared__ double Cc;
    const uint64_t ntiles = uint64_t(1) << (T.n - T.LB);
    const uint32_t TE = 1u << T.LB;
    double mn = INFINITY, mx = -INFINITY;
    for (uint64_t hi = blockIdx.x; hi < ntiles; hi += gridDim.x) {
        __syncthreads();
        tile_fields(T, hi, f, &Cc);
        __syncthreads();
        for (uint32_t lo = threadIdx.x; lo < TE; lo += blockDim.x) {
            double e = Cc + T.Q[lo];
            for (int j = 0; j < T.LB; ++j) e += ((lo >> j) & 1) ? -f[j] : f[j];
            mn = fmin(mn, e);
            mx = fmax(mx, e);
        }
    }
    block_minmax(mn, mx, part);
}

template <int D = 0>
__global__ void __launch_bounds__(256) k_minmax_final(const double *part, int np, double *out)
{
    double mn = INFINITY, mx = -INFINITY;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
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
        out[0] = smin[0];
        out[1] = smax[0];
    }
}

// d[z] = (E(z) - c) / r formed in double, rounded once to R.
template <typename R>
__global__ void __launch_bounds__(256) k_normalize_energy(EnergyTables T, double c, double inv_r, R *d)
{
    __shared__ double f[LB_TAB];
    __shared__ double Cc;
    const uint64_t ntiles = uint64_t(1) << (T.n - T.LB);
    const uint32_t TE = 1u << T.LB;
    for (uint64_t hi = blockIdx.x; hi < ntiles; hi += gridDim.x) {
        __syncthreads();
        tile_fields(T, hi, f, &Cc);
        __syncthreads();
        for (uint32_t lo = threadIdx.x; lo < TE; lo += blockDim.x) {
            double e = Cc + T.Q[lo];
            for (int j = 0; j < T.LB; ++j) e += ((lo >> j) & 1) ? -f[j] : f[j];
            d[(hi << T.LB) | lo] = (R)((e - c) * inv_r);
        }
    }
}

// ---------------------------------------------------------------------------
// Kernels: Clenshaw recurrence
// ---------------------------------------------------------------------------

// A value every lane of the wave holds identically, moved to scalar registers
// word by word (v_readfirstlane).  Used for descriptors loaded from memory, so
// that their fields do not occupy vector registers.
template <typename T> __device__ inline T wave_uniform(const T &v)
{
    static_assert(sizeof(T) % 4 == 0, "4-byte words");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T out = v;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

// Sum of one double per thread over the block, added atomically to *dst by
// thread 0 (vector atomic on global memory).  Every thread must call it.
__device__ inline void block_sum_atomic(double x, double *dst)
{
    __shared__ double wsum[16];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += wsum[i];
        atomicAdd(dst, s);
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_norm2(const CVec<R> *x, uint64_t nvec, double *acc)
{
    double s = 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nvec;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const CVec<R> p = x[i];
#pragma unroll
        for (int v = 0; v < CVec<R>::N; ++v) s += (double)p.v[v].x * p.v[v].x + (double)p.v[v].y * p.v[v].y;
    }
    block_sum_atomic(s, acc);
}

// out = (cr + i ci) psi   (K = 0 or a zero spectral bound)
template <typename R>
__global__ void __launch_bounds__(256) k_scale(const CVec<R> *psi, CVec<R> *out, R cr, R ci, uint64_t nvec)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nvec;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const CVec<R> p = psi[i];
        CVec<R> o;
#pragma unroll
        for (int v = 0; v < CVec<R>::N; ++v) {
            o.v[v].x = cr * p.v[v].x - ci * p.v[v].y;
            o.v[v].y = cr * p.v[v].y + ci * p.v[v].x;
        }
        out[i] = o;
    }
}

enum PassMode { PM_START = 0, PM_ADD = 1, PM_FUSED = 2 };

// 16-byte accesses of the passes.  STREAM adds the non-temporal hint: when a
// call's vectors are far larger than the 256 MB memory-side cache, every pass
// reads and writes each amplitude once and nothing is reused from the caches
// (measured at 28 qubits: 6 % faster in complex64, 10 % in complex128); when
// they fit, the hint costs the reuse between passes (10-15 % slower at 20
// qubits), so small calls and the batched form run without it.  KEEP_PD (with
// STREAM) leaves psi and the diagonal unhinted: while those two (12 B per
// amplitude in complex64, 24 in complex128) take at most 384 MB, they are
// re-read from the cache every term as the b vectors stream past (complex64 24
// qubits: 152.9 -> 140.6 us per term, 25: 395 -> 383, 26: no change, 28: 3186
// -> 3204; complex128 23 qubits: 230.4 -> 207.8, 24: 421.9 -> 415.5).
typedef float qw_f4 __attribute__((ext_vector_type(4)));
// Every access goes through a global-address-space pointer: the passes touch
// device memory only, and pointers that reach a kernel through a descriptor in
// memory (the batched form) would otherwise be accessed with flat instructions,
// which take 64-bit vector addresses and are counted with the LDS operations
// (every LDS wait would then also wait for the loads in flight).
#define QW_GLOBAL __attribute__((address_space(1)))
template <typename R, bool STREAM> __device__ __forceinline__ CVec<R> ld_v(const typename Cplx<R>::T *p)
{
    const QW_GLOBAL qw_f4 *g = (const QW_GLOBAL qw_f4 *)p;
    qw_f4 x;
    if constexpr (STREAM) x = __builtin_nontemporal_load(g);
    else x = *g;
    CVec<R> r;
    __builtin_memcpy(&r, &x, sizeof(r));
    return r;
}
template <typename R, bool STREAM> __device__ __forceinline__ void st_v(typename Cplx<R>::T *p, const CVec<R> &v)
{
    QW_GLOBAL qw_f4 *g = (QW_GLOBAL qw_f4 *)p;
    qw_f4 x;
    __builtin_memcpy(&x, &v, sizeof(x));
    if constexpr (STREAM) __builtin_nontemporal_store(x, g);
    else *g = x;
}
template <bool STREAM, typename T> __device__ __forceinline__ T ld_s(const T *p)
{
    const QW_GLOBAL T *g = (const QW_GLOBAL T *)p;
    if constexpr (STREAM) return __builtin_nontemporal_load(g);
    else return *g;
}

// a * b + c rounded once (v_fma_f32 / v_fma_f64)
template <typename R> __device__ __forceinline__ R fmad(R a, R b, R c)
{
    if constexpr (sizeof(R) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

template <typename R> struct PassArgs {
    using C = typename Cplx<R>::T;
    const C *b1;   // b_{k+1}: its flips over the tile's group are summed
    const C *acc;  // START: b_{k+2} (NULL: zero);  ADD, FUSED: the partial b_k
    C *dst;        // START, ADD: output (may alias acc);  FUSED: the completed b_k
    C *dst2;       // FUSED: the partial b_{k-1} (may alias b1)
    const C *psi;  // START, FUSED: v
    const R *d;    // START, FUSED: normalised diagonal (unless on the fly)
    const double *Qt;  // on the fly: split pair tables of this orientation (k_qsplit_orient)
    const double *Ft;  // on the fly: per tile, f_i / r (i < L + h) and (C - c) / r at TILE_FIELDS - 1
    R dscale = R(1);   // the diagonal used is d * dscale
    R g;           // gamma / r
    R scale;       // START, ADD: 2 inside the recurrence, 1 for the final step; FUSED: for b_k
    R scale2;      // FUSED: the same for b_{k-1}
    R cr, ci;      // START: c_k;  FUSED: c_{k-1}
    R pr, pi;      // START, ADD: multiplier of the result (the global phase on the last pass)
    R sub = R(1);  // START, FUSED: weight of the subtracted b_{k+2} (Clenshaw 1, Horner 0)
    int n, L, g0, h;
    double *norm_acc = nullptr;   // if set: += sum |b|^2 of the completed vector (atomic, one per block)
    int xcd_order = 0;            // 1: blocks take tiles in XCD-major order (xcd_tile)
    int b1_scaled = 0;            // 1: b1 points at psi and b_{k+1} = (b1r + i b1i) psi (the
    R b1r = R(1), b1i = R(0);     //    Clenshaw start b_K = c_K psi, never stored)
};

// Workgroups of a launch are dealt round-robin to the 8 XCDs (block b on XCD
// b mod 8).  xcd_tile gives the blocks of each XCD a contiguous range of
// tiles, so tiles that share DRAM pages (neighbouring rows) run on one XCD.
__host__ __device__ __forceinline__ uint64_t xcd_tile(uint32_t b, uint32_t nb)
{
    return (nb % 8 == 0) ? (uint64_t)(b % 8) * (nb / 8) + b / 8 : b;
}

// Fields of the on-the-fly diagonal for every tile of one orientation: tile
// element bit i stands for index bit vb(i) (i < L: bit i; else g0 + i - L);
// the other index bits are fixed by the tile's base.  With
//   f_i = h_vb(i) + sum_{u fixed} J_{vb(i) u} s_u,
//   C   = sum_{u fixed} h_u s_u + sum_{u<w fixed} J_uw s_u s_w
// and the orientation's pair term Q[e] = sum_{i<j} J_{vb(i) vb(j)} s_i(e) s_j(e),
// E = C + Q[e] + sum_i f_i s_i(e).  One thread per tile writes f_i / r and
// (C - c) / r in double to Ft[tile * TILE_FIELDS ...].
static constexpr int TILE_FIELDS = 16;

template <int D = 0>
__global__ void __launch_bounds__(256) k_tile_fields(const double *hJ, int n, int L, int g0, int h, uint64_t ntiles,
                                                     double c, double inv_r, double *Ft)
{
    const uint64_t tile = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const double *hh = hJ, *J = hJ + n;
    const int nv = L + h;
    const uint64_t base = tile_base(tile, L, g0, h);
    auto isvar = [&](int u) { return u < L || (u >= g0 && u < g0 + h); };
    auto spin = [&](int u) { return ((base >> u) & 1) ? -1.0 : 1.0; };
    double *out = Ft + tile * TILE_FIELDS;
    for (int i = 0; i < nv; ++i) {
        const int j = (i < L) ? i : g0 + (i - L);
        double acc = hh[j];
        for (int u = 0; u < n; ++u) {
            if (isvar(u)) continue;
            acc += spin(u) * J[pair_off(n, j < u ? j : u, j < u ? u : j)];
        }
        out[i] = acc * inv_r;
    }
    double C = 0.0;
    for (int u = 0; u < n; ++u) {
        if (isvar(u)) continue;
        double fu = hh[u];
        for (int w = u + 1; w < n; ++w) {
            if (isvar(w)) continue;
            fu += spin(w) * J[pair_off(n, u, w)];
        }
        C += spin(u) * fu;
    }
    out[TILE_FIELDS - 1] = (C - c) * inv_r;
}

// Pair term of one orientation, split for a block of 2^LOG_NT threads.  Tile
// element bits: T = bits t0..t0+LOG_NT-1 (the thread's), R = the others (the
// element's position among the thread's own): t0 = 1 in complex64 (bit 0 and
// the bits above T), t0 = 0 in complex128 (the bits above T).  With J'(a, b) the coupling
// of the index bits of tile bits a, b divided by r,
//   Q(e) = sum_{a<b} J'(a, b) s_a s_b = QTT(t) + sum_{j in R} s_j G_j(t) + QRR(r),
//   G_j(t) = sum_{i in T} J'(i, j) s_i(t).
// Written in double: QTT[t] at QS_TT, the cross couplings X[j * LOG_NT + i] =
// J'(T_i, R_j) at QS_X and QRR[r] at QS_RR, per orientation.
static constexpr int QS_TT = 0, QS_X = 1024, QS_RR = 1152, QS_MAX_R = 8;

template <int D = 0>
__global__ void __launch_bounds__(256) k_qsplit_orient(const double *hJ, int n, int L, int g0, int h, int log_nt,
                                                       int t0, double inv_r, double *Qs)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const double *J = hJ + n;
    const int nv = L + h, nr = nv - log_nt;
    auto vb = [&](int i) { return (i < L) ? i : g0 + (i - L); };
    auto Jp = [&](int a, int b) {
        const int x = vb(a), y = vb(b);
        return J[pair_off(n, x < y ? x : y, x < y ? y : x)] * inv_r;
    };
    auto rbit = [&](int j) { return (t0 == 1) ? ((j == 0) ? 0 : log_nt + j) : (log_nt + j); };
    if (u < (1 << log_nt)) {
        double q = 0.0;
        for (int a = 0; a < log_nt; ++a)
            for (int b = a + 1; b < log_nt; ++b)
                q += ((((u >> a) ^ (u >> b)) & 1) ? -1.0 : 1.0) * Jp(t0 + a, t0 + b);
        Qs[QS_TT + u] = q;
    }
    if (u < nr * log_nt) Qs[QS_X + u] = Jp(t0 + u % log_nt, rbit(u / log_nt));
    if (u < (1 << nr)) {
        double q = 0.0;
        for (int a = 0; a < nr; ++a)
            for (int b = a + 1; b < nr; ++b)
                q += ((((u >> a) ^ (u >> b)) & 1) ? -1.0 : 1.0) * Jp(rbit(a), rbit(b));
        Qs[QS_RR + u] = q;
    }
}

// One pass over one tile (see tile_base/tile_index); F_group sums the flips of
// the tile's h group bits:
//  START: dst = scale (d .* b1 + g F b1) - sub acc + c_k psi,        then *= (pr + i pi)
//  ADD:   dst = acc + scale g F b1,                                   then *= (pr + i pi)
//  FUSED: b_k = acc + scale g F b1 (completes term k) -> dst;
//         dst2 = scale2 (d .* b_k + g F b_k) - sub b1 + c_{k-1} psi (first part of term k-1)
// The Clenshaw recurrence uses scale 2 (1 on the final step) and sub 1; Horner's
// rule (y_k = H y_{k+1} + a_k psi) the same passes with scale 1 and sub 0.
// FUSED needs b_k of the whole tile, so the tile is re-staged through LDS.
template <typename R, int TB, int NT, int MODE, bool OTF, bool STREAM = false, bool KEEP_PD = false>
__device__ __forceinline__ void pass_tile(const PassArgs<R> &a, uint64_t tile, typename Cplx<R>::T *lds)
{
    using C = typename Cplx<R>::T;
    using V = CVec<R>;
    constexpr int VE = V::N;
    constexpr int PER = (1 << TB) / (NT * VE);
    constexpr bool DIAG = (MODE != PM_ADD);
    static_assert(PER >= 1, "tile smaller than one vector per thread");
    __shared__ double fld[OTF ? TB : 1];
    __shared__ double fbase;

    const int nv = a.L + a.h;
    const uint32_t TE = 1u << nv;
    const uint64_t base = tile_base(tile, a.L, a.g0, a.h);

    if constexpr (OTF) {
        static_assert(TB < TILE_FIELDS, "tile fields and the constant fit one record");
        const double *ft = a.Ft + tile * TILE_FIELDS;
        if ((int)threadIdx.x < nv) fld[threadIdx.x] = ft[threadIdx.x];
        if (threadIdx.x == 0) fbase = ft[TILE_FIELDS - 1];
    }

    V own[PER], accv[PER];
    // Every load of the tile is issued before the first barrier where the
    // registers allow it (requests issued later, between the LDS phases, left
    // HBM idle: loading acc after the barrier cost 4-12 % per pass).  START
    // prefetches psi.  Complex64 FUSED prefetches the diagonal and reads psi
    // where it is used, since psi, d, b_{k+1} and the partial b_k together would
    // exceed the 128 registers of four waves per SIMD, and stores b_k as soon as
    // it is complete (together: 1.5 % per term at 28 qubits); complex128 FUSED
    // prefetches psi, reads d where it is used and stores b_k beside b_{k-1}
    // (the complex64 order made its contiguous pass 10 % slower).  With the
    // on-the-fly diagonal psi is read where it is used.
    constexpr bool C64 = sizeof(R) == 4;
    constexpr bool PD_HINT = STREAM && !KEEP_PD;   // hint on the psi and diagonal loads
    constexpr bool EARLY_PSI = DIAG && !OTF && (MODE != PM_FUSED || !C64);
    constexpr bool EARLY_D = (MODE == PM_FUSED) && !OTF && C64;
    V psiv[EARLY_PSI ? PER : 1];
    R dv[EARLY_D ? PER : 1][VE];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
        if (e < TE) {
            const uint64_t idx = tile_index(base, e, a.L, a.g0);
            own[q] = ld_v<R, STREAM>(a.b1 + idx);
            if (a.b1_scaled) {
#pragma unroll
                for (int v = 0; v < VE; ++v) {
                    const C p = own[q].v[v];
                    own[q].v[v] = C{fmad(a.b1r, p.x, -(a.b1i * p.y)), fmad(a.b1r, p.y, a.b1i * p.x)};
                }
            }
            if (a.acc) {
                accv[q] = ld_v<R, STREAM>(a.acc + idx);
            } else {
#pragma unroll
                for (int v = 0; v < VE; ++v) accv[q].v[v] = C{R(0), R(0)};
            }
            if constexpr (EARLY_PSI) psiv[q] = ld_v<R, PD_HINT>(a.psi + idx);
            if constexpr (EARLY_D) {
#pragma unroll
                for (int v = 0; v < VE; ++v) dv[q][v] = ld_s<PD_HINT>(a.d + idx + v);
            }
#pragma unroll
            for (int v = 0; v < VE; ++v) lds[e + v] = own[q].v[v];
        }
    }
    __syncthreads();

    // Flip sums of the VE consecutive elements e..e+VE-1 of vector q (e a multiple
    // of VE), whose values are arr[q].  Tile element bits split into the vector's
    // own element (bit 0 with VE = 2), the thread (bits up to LOG_NV - 1) and the
    // vector index q (bits LOG_NV and up).  A flipped thread bit maps the group
    // onto another thread's aligned group, read from LDS as one 16-byte vector; a
    // flipped q bit onto another vector of the same thread, already in its
    // registers (arr[q ^ 2^b]: no LDS read); a flip of bit 0 swaps the two
    // elements of arr[q].  The flips are summed in increasing bit order.
    constexpr int LOG_NV = (NT * VE >= 2048) ? 11 : (NT * VE >= 1024) ? 10 : (NT * VE >= 512) ? 9 : 8;
    static_assert((1 << LOG_NV) == NT * VE, "power-of-two vectors per slice");
    constexpr int QB = (PER >= 16) ? 4 : (PER >= 8) ? 3 : (PER >= 4) ? 2 : (PER >= 2) ? 1 : 0;
    static_assert((1 << QB) == PER, "power-of-two vectors per thread");
    // group bits read from LDS: in complex64 those below the q bits; complex128
    // (one element per 16-byte vector) reads every flip from LDS, since keeping
    // the partners in registers spilled its passes
    constexpr bool QREG = (VE == 2);
    const int j_lds = QREG ? max(0, min(a.h, LOG_NV - a.L)) : a.h;
    auto flips = [&](int q, uint32_t e, const V (&arr)[PER], R (&sr)[VE], R (&si)[VE]) {
#pragma unroll
        for (int v = 0; v < VE; ++v) {
            sr[v] = R(0);
            si[v] = R(0);
        }
        const V &self = arr[q];
        const V *lv = reinterpret_cast<const V *>(lds);
        auto step = [&](int j) {
            const uint32_t m = 1u << (a.L + j);
            if (VE == 2 && m == 1u) {
                sr[0] += self.v[VE - 1].x;
                si[0] += self.v[VE - 1].y;
                sr[VE - 1] += self.v[0].x;
                si[VE - 1] += self.v[0].y;
            } else {
                const V nb = lv[(e ^ m) / VE];
#pragma unroll
                for (int v = 0; v < VE; ++v) {
                    sr[v] += nb.v[v].x;
                    si[v] += nb.v[v].y;
                }
            }
        };
        if constexpr (VE == 2) {
            // kept rolled: unrolling a known h hoists every LDS read and spills
#pragma unroll 1
            for (int j = 0; j < j_lds; ++j) step(j);
        } else {
            for (int j = 0; j < j_lds; ++j) step(j);
        }
#pragma unroll
        for (int b = 0; b < (QREG ? QB : 0); ++b) {
            if (LOG_NV + b >= a.L && LOG_NV + b < a.L + a.h) {
                const V &nb = arr[q ^ (1 << b)];
#pragma unroll
                for (int v = 0; v < VE; ++v) {
                    sr[v] += nb.v[v].x;
                    si[v] += nb.v[v].y;
                }
            }
        }
    };
    // Diagonal of element (q, v) (global index idx) for START: loaded from d
    // (after the barrier, to keep it out of the registers held across it) or
    // rebuilt from the tile fields (also in FUSED).  Rebuilt: element bits ee =
    // (q NT + thread) VE + v split into the thread's bits T and the rest R
    // (v and the bits of q: r = v | q << 1 in complex64, r = q in complex128;
    // constants of the unrolled loops).
    // With the tile fields f and the split pair term (k_qsplit_orient),
    //   E/r = C' + sum_{i in T} s_i f_i + QTT(t) + sum_{j in R} s_j (f_j + G_j(t)) + QRR(r),
    // so each thread forms base = C' + sum_T s_i f_i + QTT(t) and H_j = f_j + G_j(t)
    // once, and an element adds its R signs of H_j and QRR(r).  The sums run in
    // double and are rounded to float once, as the stored diagonal is.
    constexpr int LOG_NT = (NT >= 1024) ? 10 : (NT >= 512) ? 9 : (NT >= 256) ? 8 : 7;
    static_assert((1 << LOG_NT) == NT, "power-of-two block");
    constexpr int NR = OTF ? TB - LOG_NT : 1;   // the tile has TB bits (checked on the host)
    static_assert(NR <= QS_MAX_R, "split pair table");
    double base_t = 0.0, Hj[NR];
    // thread bit i is tile bit T0 + i (T0 = 1 in complex64, where bit 0 numbers
    // the pair a thread holds); R bit j is tile bit rbit(j)
    constexpr int T0 = (VE == 2) ? 1 : 0;
    auto rbit = [&](int j) { return (VE == 2) ? ((j == 0) ? 0 : LOG_NT + j) : (LOG_NT + j); };
    if constexpr (OTF) {
        const uint32_t t = threadIdx.x;
        base_t = fbase + a.Qt[QS_TT + t];
#pragma unroll
        for (int i = 0; i < LOG_NT; ++i) base_t += ((t >> i) & 1) ? -fld[T0 + i] : fld[T0 + i];
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            double g = fld[rbit(j)];
#pragma unroll
            for (int i = 0; i < LOG_NT; ++i) {
                const double x = a.Qt[QS_X + j * LOG_NT + i];
                g += ((t >> i) & 1) ? -x : x;
            }
            Hj[j] = g;
        }
    }
    auto diag_of = [&](uint64_t idx, int q, int v) -> R {
        if constexpr (OTF) {
            const int r = (VE == 2) ? (v | (q << 1)) : q;
            double s = base_t;
#pragma unroll
            for (int j = 0; j < NR; ++j) s += ((r >> j) & 1) ? -Hj[j] : Hj[j];
            return (R)(s + a.Qt[QS_RR + r]);
        } else {
            return ld_s<PD_HINT>(a.d + idx) * a.dscale;
        }
    };

    // Element arithmetic with explicit fused multiply-adds, so that the START
    // pass and the second half of FUSED (which compute the same first part of
    // a term) round identically whatever the compiler would contract: the
    // gradient's recomputed windows rely on it.
    //   first part:  scale (d b + g F b) - sub s + c psi
    //   completion:  acc + sg F b
    auto first_part = [&](R dd, const C &b, R sr, R si, const C &sb, const C &ps, R scale) -> C {
        const R hr = fmad(dd, b.x, a.g * sr), hi = fmad(dd, b.y, a.g * si);
        const R tr = fmad(scale, hr, -(a.sub * sb.x)), ti = fmad(scale, hi, -(a.sub * sb.y));
        const R ur = fmad(a.cr, ps.x, -(a.ci * ps.y)), ui = fmad(a.cr, ps.y, a.ci * ps.x);
        return C{tr + ur, ti + ui};
    };

    double nrm = 0.0;
    if constexpr (MODE == PM_FUSED) {
        // complete b_k in registers (complex64: and store it at once)
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
            if (e < TE) {
                R sr[VE], si[VE];
                flips(q, e, own, sr, si);
                const R sg = a.scale * a.g;
#pragma unroll
                for (int v = 0; v < VE; ++v) {
                    accv[q].v[v].x = fmad(sg, sr[v], accv[q].v[v].x);
                    accv[q].v[v].y = fmad(sg, si[v], accv[q].v[v].y);
                }
                if constexpr (C64) st_v<R, STREAM>(a.dst + tile_index(base, e, a.L, a.g0), accv[q]);
            }
        }
        __syncthreads();   // every flip of b_{k+1} has been read
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
            if (e < TE) {
#pragma unroll
                for (int v = 0; v < VE; ++v) lds[e + v] = accv[q].v[v];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
            if (e < TE) {
                const uint64_t idx = tile_index(base, e, a.L, a.g0);
                V out;
                R sr[VE], si[VE];
                V psl;   // one 16-byte load, hinted as the pass
                if constexpr (!EARLY_PSI) psl = ld_v<R, PD_HINT>(a.psi + idx);
                flips(q, e, accv, sr, si);
#pragma unroll
                for (int v = 0; v < VE; ++v) {
                    R dd;
                    if constexpr (EARLY_D) dd = dv[q][v] * a.dscale;
                    else dd = diag_of(idx + v, q, v);
                    const C bk = accv[q].v[v], bp = own[q].v[v];
                    const C ps = EARLY_PSI ? psiv[q].v[v] : psl.v[v];
                    out.v[v] = first_part(dd, bk, sr[v], si[v], bp, ps, a.scale2);
                    if (a.norm_acc) nrm += (double)bk.x * bk.x + (double)bk.y * bk.y;
                }
                if constexpr (!C64) st_v<R, STREAM>(a.dst + idx, accv[q]);
                st_v<R, STREAM>(a.dst2 + idx, out);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
            if (e < TE) {
                const uint64_t idx = tile_index(base, e, a.L, a.g0);
                V out;
                R sr_[VE], si_[VE];
                flips(q, e, own, sr_, si_);
#pragma unroll
                for (int v = 0; v < VE; ++v) {
                    const R sr = sr_[v], si = si_[v];
                    C o;
                    if constexpr (MODE == PM_START) {
                        const R dd = diag_of(idx + v, q, v);
                        const C ps = EARLY_PSI ? psiv[q].v[v] : a.psi[idx + v];
                        o = first_part(dd, own[q].v[v], sr, si, accv[q].v[v], ps, a.scale);
                    } else {
                        const C ac = accv[q].v[v];
                        const R sg = a.scale * a.g;
                        o.x = fmad(sg, sr, ac.x);
                        o.y = fmad(sg, si, ac.y);
                    }
                    // times pr + i pi; exact for 1 + 0i
                    out.v[v].x = fmad(a.pr, o.x, -(a.pi * o.y));
                    out.v[v].y = fmad(a.pr, o.y, a.pi * o.x);
                    if (a.norm_acc) nrm += (double)out.v[v].x * out.v[v].x + (double)out.v[v].y * out.v[v].y;
                }
                st_v<R, STREAM>(a.dst + idx, out);
            }
        }
    }
    if (a.norm_acc) block_sum_atomic(nrm, a.norm_acc);
}

// Two 512-thread workgroups share a CU (64 KB of LDS each): registers are
// capped so that both fit (4 waves per SIMD).
template <typename R, int TB, int NT, int MODE, bool OTF, bool STREAM = false, bool KEEP_PD = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_pass(PassArgs<R> a)
{
    __shared__ typename Cplx<R>::T lds[1 << TB];
    const uint64_t tile = a.xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    pass_tile<R, TB, NT, MODE, OTF, STREAM, KEEP_PD>(a, tile, lds);
}

// Whole recurrence of one small instance (n <= TB) inside one workgroup.
template <typename R> struct OnchipItem {
    using C = typename Cplx<R>::T;
    const C *psi;
    C *out;
    const R *d;
    const C *coef;  // c_0..c_K
    R g;
    R pr, pi;       // global phase
    int n, K;
    R two = R(2), sub = R(1);   // Clenshaw (2, 1); Horner's rule (1, 0)
};

template <typename R, int TB, int NT>
__global__ void __launch_bounds__(NT) k_onchip(const OnchipItem<R> *items, const int *order, int count)
{
    using C = typename Cplx<R>::T;
    constexpr int PER = (1 << TB) / NT;
    static_assert(PER >= 1, "");
    __shared__ C lds[1 << TB];
    for (int it = blockIdx.x; it < count; it += gridDim.x) {
        const OnchipItem<R> I = items[order ? order[it] : it];
        const uint32_t N = 1u << I.n;
        C ps[PER], b1[PER], b2[PER];
        R dd[PER];
        const C cK = I.coef[I.K];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = q * NT + threadIdx.x;
            if (e < N) {
                ps[q] = I.psi[e];
                dd[q] = I.d[e];
                b1[q].x = cK.x * ps[q].x - cK.y * ps[q].y;
                b1[q].y = cK.x * ps[q].y + cK.y * ps[q].x;
                b2[q].x = R(0);
                b2[q].y = R(0);
                lds[e] = b1[q];
            }
        }
        __syncthreads();
        for (int k = I.K - 1; k >= 1; --k) {
            const C ck = I.coef[k];
            C nb[PER];
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const uint32_t e = q * NT + threadIdx.x;
                if (e < N) {
                    R sr = R(0), si = R(0);
                    for (int j = 0; j < I.n; ++j) {
                        const C x = lds[e ^ (1u << j)];
                        sr += x.x;
                        si += x.y;
                    }
                    const R hr = dd[q] * b1[q].x + I.g * sr;
                    const R hi = dd[q] * b1[q].y + I.g * si;
                    nb[q].x = (I.two * hr - I.sub * b2[q].x) + (ck.x * ps[q].x - ck.y * ps[q].y);
                    nb[q].y = (I.two * hi - I.sub * b2[q].y) + (ck.x * ps[q].y + ck.y * ps[q].x);
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const uint32_t e = q * NT + threadIdx.x;
                if (e < N) {
                    b2[q] = b1[q];
                    b1[q] = nb[q];
                    lds[e] = nb[q];
                }
            }
            __syncthreads();
        }
        const C c0 = I.coef[0];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = q * NT + threadIdx.x;
            if (e < N) {
                C y;
                if (I.K == 0) {
                    y.x = c0.x * ps[q].x - c0.y * ps[q].y;
                    y.y = c0.x * ps[q].y + c0.y * ps[q].x;
                } else {
                    R sr = R(0), si = R(0);
                    for (int j = 0; j < I.n; ++j) {
                        const C x = lds[e ^ (1u << j)];
                        sr += x.x;
                        si += x.y;
                    }
                    const R hr = dd[q] * b1[q].x + I.g * sr;
                    const R hi = dd[q] * b1[q].y + I.g * si;
                    y.x = (hr - I.sub * b2[q].x) + (c0.x * ps[q].x - c0.y * ps[q].y);
                    y.y = (hi - I.sub * b2[q].y) + (c0.x * ps[q].y + c0.y * ps[q].x);
                }
                C o;
                o.x = I.pr * y.x - I.pi * y.y;
                o.y = I.pr * y.y + I.pi * y.x;
                I.out[e] = o;
            }
        }
        __syncthreads();  // lds is reused by the next instance
    }
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct PassPlan { int L, g0, h; };

// Orientations of one Clenshaw term for tiles of 2^TB amplitudes: the first
// takes the low min(n, TB0) bits contiguously (TB0 = TB unless given), the rest
// split the high bits as evenly as possible into groups of at most TB - LMIN
// bits, each tile keeping L = TB - h passenger bits for contiguous rows.
inline std::vector<PassPlan> plan_passes(int n, int TB, int LMIN, int TB0 = 0)
{
    std::vector<PassPlan> P;
    const int h0 = std::min(n, TB0 > 0 ? TB0 : TB);
    P.push_back({0, 0, h0});
    const int rem = n - h0;
    if (rem > 0) {
        const int cap = TB - LMIN;
        const int np = (rem + cap - 1) / cap;
        int g = h0;
        for (int p = 0; p < np; ++p) {
            const int hh = rem / np + (p < rem % np ? 1 : 0);
            P.push_back({TB - hh, g, hh});
            g += hh;
        }
    }
    return P;
}

template <typename R> inline std::vector<PassPlan> plan_passes(int n)
{
    return plan_passes(n, Cfg<R>::TB, Cfg<R>::LMIN);
}

// Tile shapes besides the default one.  Wide: complex64 2^14-amplitude tiles
// (128 KB of LDS, 1024 threads, one workgroup per CU), used where they save a
// global pass per term (n = 23, 24, 32) and the vector still has >= 512 tiles.
// Narrow: 2^12-amplitude tiles with 1024 threads, i.e. 4 (complex64) or 4
// (complex128) amplitudes per thread instead of 16 / 8, for small vectors
// (n <= 20 / 21) where one pass would otherwise run too few waves to hide the
// latency of its load, barrier and store; used only where the pass count stays
// the same.  Complex64 at n = 21 keeps 2^13 tiles (two orientations) with 1024
// threads.  Measured per term: n = 21 19.0 us with 1024 threads against 24.7
// with 512; at n = 22 and n = 28 the 512-thread shape is faster (36.3 against
// 38.4 us, 3.62 against 3.75 ms).
// Split: complex64 25 <= n <= 28 takes its contiguous orientation on 2^12
// tiles, and the high bits split into groups of at most 8 (rows of >= 256 B)
// with the same pass count: at 28 qubits 12 + 8 + 8 bits instead of 13 + 8 + 7,
// 3306 -> 3186 us per term (the contiguous fused pass 1095 -> 998 us, the add
// pass 1114 -> 1077); 25, 26, 27 qubits: 405 -> 396, 818 -> 792, 1650 -> 1604 us.
// From 29 qubits one high group takes 9 or 10 bits (128-byte rows): the
// per-orientation plans of action_plan.
static constexpr int TB_WIDE = 14, NT_WIDE = 1024;
static constexpr int TB_NARROW = 12, NT_NARROW = 1024;
static constexpr int NT_MID = 1024;   // complex64 2^13 tiles, 8 amplitudes per thread
static constexpr int SPLIT_NMIN = 25, SPLIT_NMAX = 28;
// Calls without a caller diagonal rebuild it inside the passes: from
// OTF_TOP_NMIN qubits on the fused passes of both end orientations, in
// complex64 (whose middle add pass reads no diagonal, so none is formed) and,
// up to C128_OTF_NMAX qubits, in complex128.  From OTF_NMIN qubits complex64 has no room
// for a stored diagonal at all (storing it would crowd the 288 GB).  Rebuilding costs per-thread set-up and
// double-precision sums: on the strided fused passes of complex64 it pays (28
// qubits, per term: 1114 us with the stored diagonal, 1023 rebuilt), on a
// contiguous complex64 fused pass it did not (999 against 1095); complex128
// saves 8 of its 88 bytes per amplitude on either end.  At 25 qubits psi and
// the diagonal stay in the memory-side cache and the stored one is as fast.
static constexpr int OTF_NMIN = 31, OTF_TOP_NMIN = 26, C128_OTF_NMAX = 30;

struct TileCfg {
    int tb, nt;
    bool stream;           // non-temporal accesses (vectors well beyond the memory-side cache)
    int tb0 = 0;           // > 0: split shape, the contiguous orientation on 2^tb0 tiles
    bool keep_pd = false;  // with stream: psi and the diagonal loaded without the hint
};

// Streaming pays once the call's vectors (b1, b2, psi, out and the diagonal)
// exceed the 256 MB memory-side cache by a margin: complex64 n >= 24,
// complex128 n >= 23.
template <typename R> inline bool stream_for(int n)
{
    const double per_amp = (sizeof(R) == 4) ? 36.0 : 72.0;
    return std::ldexp(per_amp, n) > 384.0 * (1 << 20);
}

template <typename R> inline TileCfg tile_cfg_for_shape(int n)
{
    constexpr int TB = Cfg<R>::TB, LMIN = Cfg<R>::LMIN;
    const bool st = stream_for<R>(n);
    if constexpr (sizeof(R) == 4) {
        if (n >= SPLIT_NMIN && n <= SPLIT_NMAX) return {TB, Cfg<R>::NT, st, TB_NARROW};
        if (n >= TB_WIDE + 9 && plan_passes(n, TB_WIDE, LMIN).size() < plan_passes(n, TB, LMIN).size())
            return {TB_WIDE, NT_WIDE, st};
        if (n > TB && n <= 20 && plan_passes(n, TB_NARROW, LMIN).size() == plan_passes(n, TB, LMIN).size())
            return {TB_NARROW, NT_NARROW, false};
        if (n == 21) return {TB, NT_MID, false};
    } else {
        if (n > TB && n <= 21) return {TB_NARROW, NT_NARROW, false};
    }
    return {TB, Cfg<R>::NT, st};
}

// psi and the diagonal stay cacheable while they take at most 384 MB
// (complex64 n <= 25, complex128 n <= 24).
template <typename R> inline TileCfg tile_cfg_for(int n)
{
    TileCfg c = tile_cfg_for_shape<R>(n);
    c.keep_pd = c.stream && std::ldexp(sizeof(R) == 4 ? 12.0 : 24.0, n) <= 384.0 * (1 << 20);
    return c;
}

// Launch shape of one pass of a call whose tiles are cfg.  Split shape: the
// contiguous orientation runs on 2^tb0-amplitude tiles with 1024 threads (two
// workgroups and 32 waves per CU instead of 16), the strided add passes on the
// 2^13 tiles with 1024 threads (4 amplitudes each: 49 registers, 8 waves per
// SIMD), the strided fused passes in the default shape; every pass streams.
// Otherwise the streaming hint pays on the strided passes (rows gathered from
// far apart) of every shape; on the contiguous first orientation it pays with
// the wide complex64 tiles and in complex128, but not with the default complex64
// tiles (measured per term at 28 qubits: 3544 us with the hint on every pass,
// 3415 us without it on the contiguous pass).
template <typename R> inline TileCfg pass_cfg(const TileCfg &cfg, const PassPlan &pl, int mode)
{
    if (cfg.tb0 > 0) {
        if (pl.L == 0) return {cfg.tb0, NT_NARROW, cfg.stream, 0, cfg.keep_pd};
        if (mode == PM_ADD) return {cfg.tb, NT_MID, cfg.stream, 0, cfg.keep_pd};
        return {cfg.tb, cfg.nt, cfg.stream, 0, cfg.keep_pd};
    }
    TileCfg p = cfg;
    p.stream = cfg.stream && (pl.L > 0 || !(sizeof(R) == 4 && cfg.tb == Cfg<R>::TB));
    return p;
}

// One orientation of an action call's pass plan with its launch shapes.  The
// fused schedule (fused_schedule) runs START / FUSED passes only on the end
// orientations (the first and last of the plan) and an ADD pass on every
// middle one in every term, so where a bit group goes in the plan decides how
// often its kernel runs.
struct OrientSpec {
    PassPlan pl;     // L, g0, h
    TileCfg fused;   // shape of its START / FUSED passes
    TileCfg add;     // shape of its ADD passes
    bool otf;        // START / FUSED rebuild the diagonal from the tile fields
    int xcd;         // blocks take tiles in XCD-major order (xcd_tile)
};

// Complex64 from 25 qubits: the contiguous orientation in the middle (an add
// pass every term, 12 or 13 bits), the two high groups at the ends (one fused
// pass each every other term).  The fused pass of the lower high group runs on
// 2^14-amplitude tiles with rows of >= 512 B (25-28 qubits) or 128 B (30-32
// qubits; 29: 2^13 tiles, 128 B), the top group's on 2^13 tiles (2^14 at 32
// qubits).  Both ends rebuild the diagonal when it comes from (h, J) (from 26
// qubits), so no pass reads a stored one.  At 29-31 qubits this layout took
// 6078, 12297 and 25867 us per term against 6695, 13348 and 27364 for the
// contiguous bits in a fused pass at one end with a stored diagonal.  Measured
// per pass at 28 qubits (same box, microseconds): contiguous add on 2^12 tiles
// 1005 against 1068 for the old middle group (bits 12-19, 2^13 tiles); fused
// pass of bits 12-19 on 2^14 tiles, 512-byte rows, 1765 against 1981 for the
// old contiguous fused pass; top group (bits 20-27) 2030 either way: 2902
// against 3074 per term.  At 32 qubits (13 + 10 + 9 bits): 50.3 against 53.3
// ms per term.  XCD-major order helps the contiguous passes (1005 against
// 1053) and, at 28 qubits, slows the strided fused ones (1765 against 1810);
// from 29 qubits the sweep chose it for the lower high group.
template <typename R> inline std::vector<OrientSpec> action_plan(int n, bool diag_from_tables)
{
    std::vector<OrientSpec> S;
    const bool otf_all = sizeof(R) == 4 && diag_from_tables && n >= OTF_NMIN;
    if constexpr (sizeof(R) == 4) {
        const bool st = stream_for<R>(n);
        const bool kp = st && std::ldexp(12.0, n) <= 384.0 * (1 << 20);
        if (n >= SPLIT_NMIN && n <= SPLIT_NMAX) {
            const int h1 = (n - TB_NARROW + 1) / 2, h2 = n - TB_NARROW - h1;
            const bool otf = diag_from_tables && n >= OTF_TOP_NMIN;
            const TileCfg wide{TB_WIDE, NT_WIDE, st, 0, kp};
            const TileCfg narrow{TB_NARROW, NT_NARROW, st, 0, kp};
            S.push_back({{TB_WIDE - h1, TB_NARROW, h1}, wide, wide, otf, 0});
            S.push_back({{0, 0, TB_NARROW}, narrow, narrow, false, 1});
            S.push_back({{Cfg<R>::TB - h2, TB_NARROW + h1, h2}, {Cfg<R>::TB, Cfg<R>::NT, st, 0, kp},
                         {Cfg<R>::TB, NT_MID, st, 0, kp}, otf, 0});
            return S;
        }
        if (n >= 29 && n <= 31) {
            // the same layout with the fastest shapes of a sweep of pass shapes:
            // 29 qubits 12 + (9, 8), 30 qubits 12 + (10, 8), 31 qubits 13 + (10, 8) bits
            const TileCfg wide{TB_WIDE, NT_WIDE, st, 0, false};
            const TileCfg dflt{Cfg<R>::TB, Cfg<R>::NT, st, 0, false};
            const TileCfg narrow{TB_NARROW, NT_NARROW, st, 0, false};
            const bool otf = diag_from_tables;
            const int c = (n == 31) ? Cfg<R>::TB : TB_NARROW;   // contiguous bits
            const int h1 = (n == 29) ? 9 : 10, h2 = n - c - h1;
            const TileCfg end0 = (h1 == 10) ? wide : dflt;       // rows of 128 B either way
            S.push_back({{end0.tb - h1, c, h1}, end0, end0, otf, 1});
            S.push_back({{0, 0, c}, (c == TB_NARROW) ? narrow : dflt, (c == TB_NARROW) ? narrow : dflt, false, 1});
            S.push_back({{Cfg<R>::TB - h2, c + h1, h2}, dflt, dflt, otf, (n == 29) ? 1 : 0});
            return S;
        }
        if (n == 32) {
            const TileCfg wide{TB_WIDE, NT_WIDE, st, 0, false};
            const TileCfg contig{Cfg<R>::TB, Cfg<R>::NT, st, 0, false};
            S.push_back({{TB_WIDE - 10, Cfg<R>::TB, 10}, wide, wide, otf_all, 1});
            S.push_back({{0, 0, Cfg<R>::TB}, contig, contig, false, 1});
            S.push_back({{TB_WIDE - 9, Cfg<R>::TB + 10, 9}, wide, wide, otf_all, 0});
            return S;
        }
    }
    // otherwise the size's tile configuration: the contiguous orientation first
    const TileCfg cfg = tile_cfg_for<R>(n);
    const std::vector<PassPlan> plan = plan_passes(n, cfg.tb, Cfg<R>::LMIN, cfg.tb0);
    const bool xcd_shape = sizeof(R) == 4 && ((cfg.tb == Cfg<R>::TB && cfg.nt == Cfg<R>::NT) || cfg.tb == TB_WIDE);
    for (const PassPlan &pl : plan)
        S.push_back({pl, pass_cfg<R>(cfg, pl, PM_FUSED), pass_cfg<R>(cfg, pl, PM_ADD), otf_all,
                     (xcd_shape && pl.g0 + pl.h < n) ? 1 : 0});
    if (sizeof(R) == 8 && diag_from_tables && n >= OTF_TOP_NMIN && n <= C128_OTF_NMAX && S.size() >= 2) {
        // complex128 from 26 to 30 qubits: both end orientations (the contiguous
        // one and the top bits) rebuild the diagonal in their fused passes, 80
        // instead of 88 bytes per amplitude, and none is formed (28 qubits: 6.62
        // -> 6.20 ms per term; the top one alone 6.41; 27: 3.56 -> 3.19; 29:
        // 14.00 -> 13.80; 30: 31.78 -> 29.17).  At 31 and 32 qubits complex128
        // keeps its stored diagonal.
        S.front().otf = true;
        S.back().otf = true;
    }
    return S;
}

// Whether a call with this plan reads a stored diagonal: only START and FUSED
// passes read it, and they run on the end orientations.
inline bool plan_reads_diag(const std::vector<OrientSpec> &S)
{
    for (size_t o = 0; o < S.size(); ++o)
        if ((o == 0 || o + 1 == S.size()) && !S[o].otf) return true;
    return false;
}

#define QW_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));              \
            return QW_EHIP;                                                            \
        }                                                                              \
    } while (0)

inline int grid_for(uint64_t work, int per_block, int cap)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

template <typename R> constexpr int prec_of() { return sizeof(R) == 4 ? 64 : 128; }

// Pass sequence of one call.  Term k (K-1 .. 0) visits the P orientations of
// the plan in order 0..P-1 when K-1-k is even and in reverse when it is odd,
// so the last orientation of term k is the first of term k-1 and the two are
// done by one FUSED pass.  P = 1: every term is one START pass.
struct SchedPass {
    int mode;    // PassMode
    int orient;  // index into the pass plan
    int k;       // term completed (FUSED), started (START) or extended (ADD)
    int fin;     // 1 on the pass that writes the final output
};

inline std::vector<SchedPass> fused_schedule(int K, int P)
{
    std::vector<SchedPass> S;
    if (K < 1 || P < 1) return S;
    auto orient = [&](int k, int i) { return (((K - 1 - k) & 1) == 0) ? i : P - 1 - i; };
    if (P == 1) {
        for (int k = K - 1; k >= 0; --k) S.push_back({PM_START, 0, k, k == 0 ? 1 : 0});
        return S;
    }
    S.push_back({PM_START, orient(K - 1, 0), K - 1, 0});
    for (int k = K - 1; k >= 0; --k) {
        for (int i = 1; i <= P - 2; ++i) S.push_back({PM_ADD, orient(k, i), k, 0});
        if (k == 0) S.push_back({PM_ADD, orient(0, P - 1), 0, 1});
        else S.push_back({PM_FUSED, orient(k, P - 1), k, 0});
    }
    return S;
}

// c_k = (-i)^k alpha_k as (re, im).
inline void coef_of(const std::vector<double> &alpha, int k, double &cr, double &ci)
{
    const double al = alpha[k];
    switch (k & 3) {
    case 0: cr = al; ci = 0.0; break;
    case 1: cr = 0.0; ci = -al; break;
    case 2: cr = -al; ci = 0.0; break;
    default: cr = 0.0; ci = al; break;
    }
}

inline bool finite(double x) { return std::isfinite(x); }

}  // namespace qw
