// Energy of a piecewise-constant anneal and its gradient by the adjoint of the
// matrix Clenshaw recurrence (complex64 forward, single-precision adjoint,
// double-precision reductions).
//
// Forward: psi_s = exp(-i t_s c) p_s(H~_s) psi_{s-1}, s = 1..S, with
// H~_s = (E - c)/r_s + (gamma_s/r_s) sum_j X_j and the Chebyshev coefficients
// of exp(-i a_s x), a_s = t_s r_s (Eq. cheb, Alg. 2).  Loss E = <psi_S|H_P|psi_S>.
//
// Reverse mode (derived from Eq. recursion; the paper has no gradient): with
// w = p(H~)v and adjoint ybar of the segment output,
//   beta_0 = conj(phase) ybar, beta_1 = H~ beta_0, beta_{k+1} = 2 H~ beta_k - beta_{k-1};
//   vbar = sum_k conj(c_k) beta_k                (adjoint of the segment input);
//   dL/dd~_i = sum_{k<K} w_k Re(conj(beta_k,i) b_{k+1,i}),  w_0 = 1, w_k = 2;
//   dL/dg~   = sum_{k<K} w_k Re<F beta_k, b_{k+1}>;
//   dL/dt    = sum_k Re(dc_k/dt <beta_k, v>) + Re(-i c <ybar, psi_s>),
//              dc_k/dt = r (-i)^k alpha_k'(a),
// with the shift c, bound r and degree K held fixed.  The b_k are recomputed
// per window of `ckpt_every` terms from checkpointed pairs stored during the
// forward sweep.  dE/dh, dE/dJ follow from G_i = sum_s dL/dd~_{s,i}/r_s +
// |psi_S,i|^2 by a Walsh-type reduction over the basis states.
#include "qw_kernels.h"

namespace qw {

static constexpr int GTB = Cfg<float>::TB;   // tile bits of the element-wise kernels
static constexpr int GNT = Cfg<float>::NT;

// Coefficients of one adjoint step k (see the file comment).
struct AdjStep {
    float scale, ckr, cki, gw;   // scale 2 (1 for k = 0), conj(c_k) applied to beta_k, w_k / r
    double wk, dcr, dci;         // w_k, r dc_k/da
};

struct AdjArgs {
    const float2 *beta;    // beta_k: its flips over the tile group are summed
    const float2 *prev;    // START: beta_{k-1} (NULL for k = 0); ADD, FUSED: partial beta_{k+1}
    float2 *dst;           // beta_{k+1}, partial or complete (may alias prev)
    float2 *dst2;          // FUSED: partial beta_{k+2} (may alias beta)
    const float2 *bnext;   // b_{k+1}
    const float2 *bnext2;  // FUSED: b_{k+2}
    const float2 *v;       // segment input
    float2 *vbar;          // accumulates conj(c_k) beta_k
    float *G;              // accumulates w_k/r Re(conj(beta_k) b_{k+1})
    const float *erel;     // E - c
    double *part;          // per block: [0] += Re(dc_k <beta_k, v>), [1] += w_k Re<F beta_k, b_{k+1}>
    double *part2;         // FUSED: the same for step k + 1
    float dscale, g;
    AdjStep st, st2;       // step k; FUSED: step k + 1
    int L, g0, h;
};

// One element of the first pass of step k: the start of beta_{k+1} and the
// accumulations that use beta_k (b = beta_k, p = beta_{k-1}, bx = b_{k+1},
// x = v, (sr, si) = flips of beta_k over the pass's group).
__device__ __forceinline__ float2 adj_start_elem(const AdjStep &s, float dscale, float g, float er, float2 b,
                                                 float2 p, float2 bx, float2 x, float sr, float si, float2 &vb,
                                                 float &gg, double &dt, double &dg)
{
    dg += s.wk * (double)(sr * bx.x + si * bx.y);
    const float d = er * dscale;
    float2 o;
    o.x = s.scale * (d * b.x + g * sr) - p.x;
    o.y = s.scale * (d * b.y + g * si) - p.y;
    vb.x += s.ckr * b.x + s.cki * b.y;
    vb.y += s.ckr * b.y - s.cki * b.x;
    gg += s.gw * (b.x * bx.x + b.y * bx.y);
    const double pr = (double)b.x * x.x + (double)b.y * x.y;
    const double pi = (double)b.x * x.y - (double)b.y * x.x;
    dt += s.dcr * pr - s.dci * pi;
    return o;
}

// One element of a later pass of step k: p = partial beta_{k+1}.
__device__ __forceinline__ float2 adj_add_elem(const AdjStep &s, float g, float2 p, float2 bx, float sr, float si,
                                               double &dg)
{
    dg += s.wk * (double)(sr * bx.x + si * bx.y);
    float2 o;
    o.x = p.x + s.scale * g * sr;
    o.y = p.y + s.scale * g * si;
    return o;
}

__device__ inline void block_add2(double x, double y, double *out)
{
    __shared__ double sx[64], sy[64];
    for (int o = 32; o > 0; o >>= 1) {
        x += __shfl_xor(x, o);
        y += __shfl_xor(y, o);
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sx[w] = x;
        sy[w] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < nw; ++i) {
            a += sx[i];
            b += sy[i];
        }
        out[0] += a;
        out[1] += b;
    }
}

// One pass of the adjoint step k -> k+1 (see the file comment), on tiles of
// 2^TB amplitudes with NT threads (the shapes of the forward passes):
//  START: first orientation of step k (diagonal, flips, - beta_{k-1}, accumulations);
//  ADD:   a later orientation of step k;
//  FUSED: the last orientation of step k, then in the same orientation the
//         first of step k + 1 from the completed beta_{k+1} re-staged in LDS.
// The per-element arithmetic is the same in all three (adj_start_elem /
// adj_add_elem), so a step gives the same bits fused or not.
enum AdjMode { AM_START = 0, AM_ADD = 1, AM_FUSED = 2 };

template <int MODE, int TB, int NT, bool STREAM>
__global__ void __launch_bounds__(NT) k_adj_pass(AdjArgs a)
{
    using C = float2;
    using V = CVec<float>;
    constexpr int VE = V::N;
    constexpr int PER = (1 << TB) / (NT * VE);
    constexpr bool START = (MODE == AM_START);
    __shared__ C lds[1 << TB];
    const uint32_t TE = 1u << (a.L + a.h);
    const uint64_t base = tile_base(blockIdx.x, a.L, a.g0, a.h);
    V own[PER], pv[PER], bn[PER];
    V vv[START ? PER : 1], vb[START ? PER : 1];
    float er[START ? PER : 1][VE], gg[START ? PER : 1][VE];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
        if (e < TE) {
            const uint64_t idx = tile_index(base, e, a.L, a.g0);
            own[q] = ld_v<float, STREAM>(a.beta + idx);
            if (a.prev) {
                pv[q] = ld_v<float, STREAM>(a.prev + idx);
            } else {
#pragma unroll
                for (int v = 0; v < VE; ++v) pv[q].v[v] = C{0.f, 0.f};
            }
            bn[q] = ld_v<float, STREAM>(a.bnext + idx);
            if constexpr (START) {
                vv[q] = ld_v<float, STREAM>(a.v + idx);
                vb[q] = ld_v<float, STREAM>(a.vbar + idx);
#pragma unroll
                for (int v = 0; v < VE; ++v) {
                    er[q][v] = a.erel[idx + v];
                    gg[q][v] = a.G[idx + v];
                }
            }
#pragma unroll
            for (int v = 0; v < VE; ++v) lds[e + v] = own[q].v[v];
        }
    }
    __syncthreads();
    auto flips = [&](uint32_t ee, float &sr, float &si) {
        sr = 0.f;
        si = 0.f;
        for (int j = 0; j < a.h; ++j) {
            const C nb = lds[ee ^ (1u << (a.L + j))];
            sr += nb.x;
            si += nb.y;
        }
    };
    double acc_dt = 0.0, acc_dg = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
        if (e < TE) {
            const uint64_t idx = tile_index(base, e, a.L, a.g0);
            V out;
#pragma unroll
            for (int v = 0; v < VE; ++v) {
                float sr, si;
                flips(e + v, sr, si);
                if constexpr (START)
                    out.v[v] = adj_start_elem(a.st, a.dscale, a.g, er[q][v], own[q].v[v], pv[q].v[v], bn[q].v[v],
                                              vv[q].v[v], sr, si, vb[q].v[v], gg[q][v], acc_dt, acc_dg);
                else
                    out.v[v] = adj_add_elem(a.st, a.g, pv[q].v[v], bn[q].v[v], sr, si, acc_dg);
            }
            if constexpr (MODE == AM_FUSED) {
                pv[q] = out;   // completed beta_{k+1}, kept for the second half
            } else {
                st_v<float, STREAM>(a.dst + idx, out);
                if constexpr (START) {
                    st_v<float, STREAM>(a.vbar + idx, vb[q]);
#pragma unroll
                    for (int v = 0; v < VE; ++v) a.G[idx + v] = gg[q][v];
                }
            }
        }
    }
    block_add2(acc_dt, acc_dg, a.part + 2 * blockIdx.x);
    if constexpr (MODE == AM_FUSED) {
        // second half: step k + 1 from the completed beta_{k+1} (pv) with
        // beta_k (own) as the subtracted vector
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
            if (e < TE) {
#pragma unroll
                for (int v = 0; v < VE; ++v) lds[e + v] = pv[q].v[v];
            }
        }
        __syncthreads();
        double dt2 = 0.0, dg2 = 0.0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = (uint32_t)(q * NT + threadIdx.x) * VE;
            if (e < TE) {
                const uint64_t idx = tile_index(base, e, a.L, a.g0);
                const V bx = ld_v<float, STREAM>(a.bnext2 + idx);
                const V x = ld_v<float, STREAM>(a.v + idx);
                V vbq = ld_v<float, STREAM>(a.vbar + idx);
                V out;
#pragma unroll
                for (int v = 0; v < VE; ++v) {
                    float sr, si;
                    flips(e + v, sr, si);
                    float gq = a.G[idx + v];
                    out.v[v] = adj_start_elem(a.st2, a.dscale, a.g, a.erel[idx + v], pv[q].v[v], own[q].v[v],
                                              bx.v[v], x.v[v], sr, si, vbq.v[v], gq, dt2, dg2);
                    a.G[idx + v] = gq;
                }
                st_v<float, STREAM>(a.dst + idx, pv[q]);
                st_v<float, STREAM>(a.dst2 + idx, out);
                st_v<float, STREAM>(a.vbar + idx, vbq);
            }
        }
        __syncthreads();   // block_add2's shared sums are reused
        block_add2(dt2, dg2, a.part2 + 2 * blockIdx.x);
    }
}

// Element-wise kernels over tiles of 2^GTB consecutive amplitudes (TE = min(N, 2^GTB)).
struct EwArgs {
    const float2 *x;      // k_adj_last: beta_K;  k_seed: psi_S;  k_beta0: ybar (= vbar buffer)
    const float2 *v;      // k_adj_last: v;  k_beta0: psi_s (segment output)
    float2 *y;            // k_adj_last: vbar;  k_seed: vbar (receives ybar);  k_beta0: beta_0
    float2 *z;            // k_beta0: vbar (zeroed)
    float *G;             // k_seed: |psi_S|^2
    const float *erel;
    double *part;         // per block: [0], [1]
    double c;             // shift
    float cr, ci;         // k_adj_last: c_K;  k_beta0: conj(phase)
    double dcr, dci;      // k_adj_last: dc_K/dt
    uint32_t TE;
};

// vbar += conj(c_K) beta_K;  part[0] += Re(dc_K/dt <beta_K, v>).
__global__ void __launch_bounds__(256) k_adj_last(EwArgs a)
{
    const uint64_t base = (uint64_t)blockIdx.x * a.TE;
    double acc = 0.0;
    for (uint32_t e = threadIdx.x; e < a.TE; e += blockDim.x) {
        const float2 b = a.x[base + e], x = a.v[base + e];
        float2 vb = a.y[base + e];
        vb.x += a.cr * b.x + a.ci * b.y;
        vb.y += a.cr * b.y - a.ci * b.x;
        a.y[base + e] = vb;
        const double pr = (double)b.x * x.x + (double)b.y * x.y;
        const double pi = (double)b.x * x.y - (double)b.y * x.x;
        acc += a.dcr * pr - a.dci * pi;
    }
    block_add2(acc, 0.0, a.part + 2 * blockIdx.x);
}

// ybar = 2 E psi_S into vbar, G = |psi_S|^2, part[0] += sum E |psi_S|^2.
__global__ void __launch_bounds__(256) k_seed(EwArgs a)
{
    const uint64_t base = (uint64_t)blockIdx.x * a.TE;
    double acc = 0.0;
    for (uint32_t e = threadIdx.x; e < a.TE; e += blockDim.x) {
        const float2 p = a.x[base + e];
        const double E = (double)a.erel[base + e] + a.c;
        const double m2 = (double)p.x * p.x + (double)p.y * p.y;
        acc += E * m2;
        a.y[base + e] = make_float2((float)(2.0 * E * p.x), (float)(2.0 * E * p.y));
        a.G[base + e] = (float)m2;
    }
    block_add2(acc, 0.0, a.part + 2 * blockIdx.x);
}

// beta_0 = conj(phase) ybar; vbar = 0; part[0] += c Im<ybar, psi_s> = Re(-i c <ybar, psi_s>).
__global__ void __launch_bounds__(256) k_beta0(EwArgs a)
{
    const uint64_t base = (uint64_t)blockIdx.x * a.TE;
    double acc = 0.0;
    for (uint32_t e = threadIdx.x; e < a.TE; e += blockDim.x) {
        const float2 yb = a.x[base + e], p = a.v[base + e];
        acc += (double)yb.x * p.y - (double)yb.y * p.x;   // Im(conj(ybar) psi)
        a.y[base + e] = make_float2(a.cr * yb.x - a.ci * yb.y, a.cr * yb.y + a.ci * yb.x);
        a.z[base + e] = make_float2(0.f, 0.f);
    }
    block_add2(a.c * acc, 0.0, a.part + 2 * blockIdx.x);
}

__global__ void k_zero_f64(double *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

// Walsh reduction, stage 1: per tile of 2^LB amplitudes (high bits fixed),
//   W0 = sum G, W1_j = sum G s_j, W2_jk = sum G s_j s_k  (j < k < LB),
// combined with the tile's high-bit signs into partial dE/dh_j, dE/dJ_jk.
__global__ void __launch_bounds__(256) k_walsh_tile(const float *G, int n, int LB, double *out)
{
    __shared__ float g[1 << LB_TAB];
    __shared__ double W[1 + LB_TAB + LB_TAB * (LB_TAB - 1) / 2];
    const uint32_t TE = 1u << LB;
    const uint64_t hi = blockIdx.x;
    const uint64_t base = hi << LB;
    for (uint32_t e = threadIdx.x; e < TE; e += blockDim.x) g[e] = G[base + e];
    __syncthreads();
    const int nq = 1 + LB + LB * (LB - 1) / 2;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        int j = -1, k = -1;
        if (q >= 1 && q <= LB) j = q - 1;
        if (q > LB) {   // pair index -> (j, k), j < k < LB
            int r = q - LB - 1;
            j = 0;
            while (r >= LB - 1 - j) { r -= LB - 1 - j; ++j; }
            k = j + 1 + r;
        }
        double acc = 0.0;
        for (uint32_t e = 0; e < TE; ++e) {
            double x = g[e];
            if (j >= 0 && ((e >> j) & 1)) x = -x;
            if (k >= 0 && ((e >> k) & 1)) x = -x;
            acc += x;
        }
        W[q] = acc;
    }
    __syncthreads();
    const int npar = n + n * (n - 1) / 2;
    double *o = out + (size_t)blockIdx.x * npar;
    auto shi = [&](int j) { return ((hi >> (j - LB)) & 1) ? -1.0 : 1.0; };
    auto w2 = [&](int j, int k) { return W[1 + LB + pair_off(LB, j, k)]; };
    for (int p = threadIdx.x; p < npar; p += blockDim.x) {
        double val;
        if (p < n) {
            val = (p < LB) ? W[1 + p] : shi(p) * W[0];
        } else {
            int r = p - n, j = 0;
            while (r >= n - 1 - j) { r -= n - 1 - j; ++j; }
            const int k = j + 1 + r;
            if (k < LB) val = w2(j, k);
            else if (j < LB) val = shi(k) * W[1 + j];
            else val = shi(j) * shi(k) * W[0];
        }
        o[p] = val;
    }
}

// Stage 2: column sums over tiles, one block per parameter.
__global__ void __launch_bounds__(256) k_walsh_reduce(const double *in, int ntiles, int npar, double *res)
{
    double acc = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) acc += in[(size_t)t * npar + blockIdx.x];
    __shared__ double s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) res[blockIdx.x] = s[0];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct SegPlan {
    double r, g, inv_r, a;
    float ph_r, ph_i;
    int K, C, W;
    std::vector<double> alpha, dalpha;   // coefficients and d alpha / d a
    std::vector<int> slot;               // checkpoint slot of b_j (j = 0..K+1), -1 if none
    size_t sbase = 0;                    // store mode: window slot of b_1
};

struct GradLayout {
    size_t states, erel, A, B, vbar, G, win, ckpt, part, partm, walsh, wres, hj, q, red, mpart, total;
    int nwin, nckpt, ntiles_lo, npar;
    bool store;   // every b_k of every segment kept (win holds them all, no recomputation)
};

// Launch helpers over the tile shapes the forward path chooses (tile_cfg_for).
template <int TB, int NT, bool STREAM>
static void grad_pass_shape(const PassArgs<float> &pa, int mode, uint64_t ntiles, hipStream_t s)
{
    if (mode == PM_START) hipLaunchKernelGGL((k_pass<float, TB, NT, PM_START, false, STREAM>), dim3((unsigned)ntiles), dim3(NT), 0, s, pa);
    else if (mode == PM_FUSED) hipLaunchKernelGGL((k_pass<float, TB, NT, PM_FUSED, false, STREAM>), dim3((unsigned)ntiles), dim3(NT), 0, s, pa);
    else hipLaunchKernelGGL((k_pass<float, TB, NT, PM_ADD, false, STREAM>), dim3((unsigned)ntiles), dim3(NT), 0, s, pa);
}

static void launch_grad_pass(const PassArgs<float> &pa, int mode, uint64_t ntiles, TileCfg cfg, hipStream_t s)
{
    if (cfg.tb == TB_NARROW) grad_pass_shape<TB_NARROW, NT_NARROW, false>(pa, mode, ntiles, s);
    else if (cfg.nt == NT_MID) grad_pass_shape<GTB, NT_MID, false>(pa, mode, ntiles, s);
    else if (cfg.stream) grad_pass_shape<GTB, GNT, true>(pa, mode, ntiles, s);
    else grad_pass_shape<GTB, GNT, false>(pa, mode, ntiles, s);
}

template <int TB, int NT, bool STREAM>
static void adj_pass_shape(const AdjArgs &aa, int mode, uint64_t ntiles, hipStream_t s)
{
    const dim3 g((unsigned)ntiles), b(NT);
    if (mode == AM_START) hipLaunchKernelGGL((k_adj_pass<AM_START, TB, NT, STREAM>), g, b, 0, s, aa);
    else if (mode == AM_FUSED) hipLaunchKernelGGL((k_adj_pass<AM_FUSED, TB, NT, STREAM>), g, b, 0, s, aa);
    else hipLaunchKernelGGL((k_adj_pass<AM_ADD, TB, NT, STREAM>), g, b, 0, s, aa);
}

// The adjoint pass holds five vectors per element (256 VGPRs with 512 threads
// on 2^13 tiles): it always runs 1024 threads, 4 or 8 amplitudes per thread.
static void launch_adj_pass(const AdjArgs &aa, int mode, uint64_t ntiles, TileCfg cfg, hipStream_t s)
{
    if (cfg.tb == TB_NARROW) adj_pass_shape<TB_NARROW, NT_NARROW, false>(aa, mode, ntiles, s);
    else if (cfg.stream) adj_pass_shape<GTB, NT_MID, true>(aa, mode, ntiles, s);
    else adj_pass_shape<GTB, NT_MID, false>(aa, mode, ntiles, s);
}

// Tile shape of the gradient's passes: the action's choice, without the wide
// 2^14 tiles (whose adjoint pass would not fit the register file).
static TileCfg grad_cfg(int n)
{
    const TileCfg c = tile_cfg_for<float>(n);
    return (c.tb == TB_WIDE) ? TileCfg{GTB, GNT, c.stream} : c;
}

static int grad_window(int ckpt_every, int K) { return (ckpt_every <= 0 || ckpt_every > K) ? K : ckpt_every; }

static GradLayout grad_layout(int n, int S, const int *Kb, int ckpt_every)
{
    const int tb = grad_cfg(n).tb;
    const size_t N = size_t(1) << n;
    GradLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    L.nwin = 1;
    L.nckpt = 0;
    L.store = ckpt_every < 0;
    if (L.store) {
        // b_1 .. b_K of segment s at slots sum_{s' < s} max(Kb[s'], 1) + j - 1
        L.nwin = 0;
        for (int s = 0; s < S; ++s) L.nwin += std::max(Kb[s], 1);
    }
    for (int s = 0; s < S && !L.store; ++s) {
        const int K = std::max(Kb[s], 1);
        const int C = grad_window(ckpt_every, K);
        const int W = (K + C - 1) / C;
        L.nwin = std::max(L.nwin, C);
        L.nckpt += 2 * (W - 1);
    }
    L.ntiles_lo = (n > tb) ? (int)(N >> tb) : 1;
    L.npar = n + n * (n - 1) / 2;
    L.states = take(N * 8 * (S + 1));
    L.erel = take(N * 4);
    L.A = take(N * 8);
    L.B = take(N * 8);
    L.vbar = take(N * 8);
    L.G = take(N * 4);
    L.win = take(N * 8 * L.nwin);
    L.ckpt = take(N * 8 * std::max(L.nckpt, 1));
    L.part = take(sizeof(double) * 2 * L.ntiles_lo * 4);     // up to 4 passes
    L.partm = take(sizeof(double) * 2 * L.ntiles_lo);
    const int wt = (n > LB_TAB) ? (1 << (n - LB_TAB)) : 1;
    L.walsh = take(sizeof(double) * (size_t)wt * L.npar);
    L.wres = take(sizeof(double) * L.npar);
    L.hj = take(sizeof(double) * (n + n * (n - 1) / 2));
    L.q = take(sizeof(double) * (size_t(1) << LB_TAB));
    L.red = take(2 * sizeof(double));
    L.mpart = take(2 * sizeof(double) * MAXPART);
    L.total = off;
    return L;
}

static int grad_degree_bound(int n, const double *h, const double *J, double gamma, double t)
{
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += std::fabs(h[j]);
    for (int p = 0; p < n * (n - 1) / 2; ++p) s += std::fabs(J[p]);
    const double rmax = s + n * std::fabs(gamma);
    return bessel_cutoff(std::fabs(t) * rmax * 1.01 + 1.0) + 2;
}

static qw_status grad_validate(int n, const double *h, const double *J, int S, const double *gamma,
                               const double *t, double tol)
{
    if (n < 1 || n > 28) { set_error("the gradient supports 1 <= n <= 28"); return QW_EINVAL; }
    if (S < 1 || !gamma || !t || !h || (n > 1 && !J)) { set_error("S >= 1, gamma, t, h, J are required"); return QW_EINVAL; }
    if (!(tol > 0.0) || !finite(tol)) { set_error("tol must be positive"); return QW_EINVAL; }
    for (int s = 0; s < S; ++s)
        if (!finite(gamma[s]) || !finite(t[s])) { set_error("non-finite schedule"); return QW_EINVAL; }
    for (int j = 0; j < n; ++j)
        if (!finite(h[j])) { set_error("non-finite h"); return QW_EINVAL; }
    for (int p = 0; p < n * (n - 1) / 2; ++p)
        if (!finite(J[p])) { set_error("non-finite J"); return QW_EINVAL; }
    return QW_OK;
}

static std::vector<int> grad_bounds(int n, const double *h, const double *J, int S, const double *gamma,
                                    const double *t)
{
    std::vector<int> Kb(S);
    for (int s = 0; s < S; ++s) Kb[s] = grad_degree_bound(n, h, J, gamma[s], t[s]);
    return Kb;
}

static qw_status grad_impl(int n, const double *h, const double *J, int S, const double *gamma, const double *t,
                           const void *psi0, double tol, int ckpt_every, double *E_out, double *dgamma,
                           double *dt, double *dh, double *dJ, void *workspace, size_t ws_bytes, hipStream_t s,
                           void *psiT_out, qw_grad_info *info)
{
    qw_status st = grad_validate(n, h, J, S, gamma, t, tol);
    if (st != QW_OK) return st;
    if (!psi0 || !workspace || !E_out || !dgamma || !dt || !dh || (n > 1 && !dJ)) {
        set_error("psi0, workspace and every output are required");
        return QW_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) || (reinterpret_cast<uintptr_t>(psi0) & 15)) {
        set_error("workspace must be 256-byte and psi0 16-byte aligned");
        return QW_EINVAL;
    }
    const std::vector<int> Kb = grad_bounds(n, h, J, S, gamma, t);
    const GradLayout L = grad_layout(n, S, Kb.data(), ckpt_every);
    if (ws_bytes < L.total) { set_error("workspace too small: need " + std::to_string(L.total)); return QW_ENOMEM; }
    char *ws = static_cast<char *>(workspace);
    const uint64_t N = uint64_t(1) << n;
    using C = float2;
    auto vec = [&](size_t off, size_t i) { return reinterpret_cast<C *>(ws + off) + i * N; };
    C *states = vec(L.states, 0);
    float *erel = reinterpret_cast<float *>(ws + L.erel);
    float *G = reinterpret_cast<float *>(ws + L.G);
    C *vbar = vec(L.vbar, 0);
    double *part = reinterpret_cast<double *>(ws + L.part);
    double *partm = reinterpret_cast<double *>(ws + L.partm);
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timing = info && info->timing;
    if (timing)
        for (auto &e : ev) QW_HIP(hipEventCreate(&e));
    struct EvGuard { hipEvent_t *e; ~EvGuard() { for (int i = 0; i < 2; ++i) if (e[i]) (void)hipEventDestroy(e[i]); } } eg{ev};
    if (timing) QW_HIP(hipEventRecord(ev[0], s));

    // tables, range of E, E - c
    const int np = n * (n - 1) / 2;
    std::vector<double> hj(n + np);
    std::memcpy(hj.data(), h, n * sizeof(double));
    if (np) std::memcpy(hj.data() + n, J, np * sizeof(double));
    double *dhj = reinterpret_cast<double *>(ws + L.hj);
    QW_HIP(hipMemcpyAsync(dhj, hj.data(), hj.size() * sizeof(double), hipMemcpyHostToDevice, s));
    EnergyTables T{dhj, dhj + n, reinterpret_cast<double *>(ws + L.q), n, std::min(n, LB_TAB)};
    hipLaunchKernelGGL(k_qtable<0>, dim3(((1 << T.LB) + 255) / 256), dim3(256), 0, s, T, const_cast<double *>(T.Q));
    const int ntE = (int)(N >> T.LB);
    const int npm = std::min(ntE, MAXPART);
    double *mpart = reinterpret_cast<double *>(ws + L.mpart);
    double *red = reinterpret_cast<double *>(ws + L.red);
    hipLaunchKernelGGL(k_minmax_energy<0>, dim3(npm), dim3(256), 0, s, T, mpart);
    hipLaunchKernelGGL(k_minmax_final<0>, dim3(1), dim3(256), 0, s, (const double *)mpart, npm, red);
    QW_HIP(hipGetLastError());
    double emm[2];
    QW_HIP(hipMemcpyAsync(emm, red, sizeof(emm), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    const double c = 0.5 * (emm[0] + emm[1]), half = 0.5 * (emm[1] - emm[0]);
    hipLaunchKernelGGL(k_normalize_energy<float>, dim3(grid_for(ntE, 1, 1 << 16)), dim3(256), 0, s, T, c, 1.0, erel);
    QW_HIP(hipMemcpyAsync(states, psi0, N * sizeof(C), hipMemcpyDeviceToDevice, s));

    // segment plans
    const TileCfg cfg = grad_cfg(n);
    const std::vector<PassPlan> plan = plan_passes(n, cfg.tb, Cfg<float>::LMIN);
    const int P = (int)plan.size();
    std::vector<SegPlan> seg(S);
    int ck_next = 0;
    size_t store_next = 0;
    for (int q = 0; q < S; ++q) {
        SegPlan &sp = seg[q];
        double r = half + n * std::fabs(gamma[q]);
        double g = (r > 0.0) ? gamma[q] / r : 0.0;
        if (gamma[q] != 0.0 && r > 0.0) {
            float gf = (float)g;
            if (std::fabs((double)gf) > std::fabs(g)) gf = std::nextafter(gf, 0.0f);
            g = (double)gf;
            r = gamma[q] / g;
        }
        if (!(r > 0.0)) { set_error("zero spectral bound in a segment (H = const)"); return QW_EINVAL; }
        sp.r = r;
        sp.g = g;
        sp.inv_r = 1.0 / r;
        sp.a = t[q] * r;
        sp.ph_r = (float)std::cos(t[q] * c);
        sp.ph_i = (float)-std::sin(t[q] * c);
        double err = 0.0;
        if (coefficients(sp.a, tol, QW_CHEB, sp.alpha, &sp.K, &err) != 0) { set_error("coefficients"); return QW_ENOCONV; }
        if (sp.K > Kb[q]) { set_error("internal: degree bound exceeded"); return QW_ENOCONV; }
        std::vector<double> Jm(sp.K + 2);
        bessel_miller(sp.a, sp.K + 1, Jm.data());
        sp.dalpha.resize(sp.K + 1);
        for (int k = 0; k <= sp.K; ++k)
            sp.dalpha[k] = (k == 0) ? -Jm[1] : (Jm[k - 1] - Jm[k + 1]);
        const int K = std::max(sp.K, 1);
        sp.C = L.store ? K : grad_window(ckpt_every, K);
        sp.W = (sp.K == 0) ? 0 : (sp.K + sp.C - 1) / sp.C;
        sp.slot.assign(sp.K + 3, -1);
        sp.sbase = store_next;
        store_next += (size_t)std::max(Kb[q], 1);
        for (int w = 0; w + 1 < sp.W; ++w) {
            const int Tw = (w + 1) * sp.C;
            for (int j = Tw + 1; j <= std::min(Tw + 2, sp.K); ++j)
                if (sp.slot[j] < 0) sp.slot[j] = ck_next++;
        }
        if (ck_next > std::max(L.nckpt, 1)) { set_error("internal: checkpoint slots exceeded"); return QW_ENOCONV; }
    }

    // One pass of the fused schedule (mode START / ADD / FUSED, see pass_tile):
    // b1 = b_{k+1}; acc = partial or b_{k+2}; dst (and dst2 for FUSED).
    auto launch_clenshaw_pass = [&](int mode, int p, const C *b1, const C *acc, C *dst, C *dst2, double cr,
                                    double ci, double scale, double scale2, float pr, float pi, const SegPlan &sp,
                                    const C *v) {
        PassArgs<float> pa{};
        pa.b1 = b1;
        pa.acc = acc;
        pa.dst = dst;
        pa.dst2 = dst2;
        pa.psi = v;
        pa.d = erel;
        pa.g = (float)sp.g;
        pa.scale = (float)scale;
        pa.scale2 = (float)scale2;
        pa.cr = (float)cr;
        pa.ci = (float)ci;
        pa.pr = pr;
        pa.pi = pi;
        pa.n = n;
        pa.L = plan[p].L;
        pa.g0 = plan[p].g0;
        pa.h = plan[p].h;
        pa.dscale = (float)sp.inv_r;
        const uint64_t ntiles = N >> (plan[p].L + plan[p].h);
        launch_grad_pass(pa, mode, ntiles, cfg, s);
    };
    const int eg_grid = grid_for(N / 2, 256 * 4, 1 << 16);
    const uint32_t TEw = (uint32_t)std::min<uint64_t>(N, uint64_t(1) << GTB);
    const int ntw = (int)(N / TEw);

    // forward sweep
    long long amp_terms = 0;
    for (int q = 0; q < S; ++q) {
        const SegPlan &sp = seg[q];
        const C *v = states + (size_t)q * N;
        C *y = states + (size_t)(q + 1) * N;
        amp_terms += (long long)sp.K << n;
        double cr, ci;
        if (sp.K == 0) {
            coef_of(sp.alpha, 0, cr, ci);
            const double pr = cr * sp.ph_r - ci * sp.ph_i, pi = cr * sp.ph_i + ci * sp.ph_r;
            hipLaunchKernelGGL(k_scale<float>, dim3(eg_grid), dim3(256), 0, s, reinterpret_cast<const CVec<float> *>(v),
                               reinterpret_cast<CVec<float> *>(y), (float)pr, (float)pi, (uint64_t)(N / 2));
            continue;
        }
        if (L.store) {
            // every b_j goes to its own slot Wst(j); the partial sums live in B.
            // Same passes and arithmetic as below, so the b_j are bit-identical.
            auto Wst = [&](int j) { return vec(L.win, sp.sbase + (size_t)(j - 1)); };
            C *Y = vec(L.B, 0);
            coef_of(sp.alpha, sp.K, cr, ci);
            hipLaunchKernelGGL(k_scale<float>, dim3(eg_grid), dim3(256), 0, s,
                               reinterpret_cast<const CVec<float> *>(v), reinterpret_cast<CVec<float> *>(Wst(sp.K)),
                               (float)cr, (float)ci, (uint64_t)(N / 2));
            auto scale_of = [](int k) { return k == 0 ? 1.0 : 2.0; };
            for (const SchedPass &ps : fused_schedule(sp.K, P)) {
                const float pr = ps.fin ? sp.ph_r : 1.f, pi = ps.fin ? sp.ph_i : 0.f;
                const C *b1 = Wst(ps.k + 1);
                if (ps.mode == PM_START) {
                    coef_of(sp.alpha, ps.k, cr, ci);
                    const C *acc = (ps.k + 2 <= sp.K) ? (P == 1 ? Wst(ps.k + 2) : nullptr) : nullptr;
                    if (P > 1 && ps.k != sp.K - 1) { set_error("internal: start pass inside a term"); return QW_EINVAL; }
                    C *dst = ps.fin ? y : (P == 1 ? Wst(ps.k) : Y);
                    launch_clenshaw_pass(PM_START, ps.orient, b1, acc, dst, nullptr, cr, ci, scale_of(ps.k), 0.0, pr, pi,
                                         sp, v);
                } else if (ps.mode == PM_ADD) {
                    launch_clenshaw_pass(PM_ADD, ps.orient, b1, Y, ps.fin ? y : Y, nullptr, 0.0, 0.0, scale_of(ps.k),
                                         0.0, pr, pi, sp, v);
                } else {
                    coef_of(sp.alpha, ps.k - 1, cr, ci);
                    launch_clenshaw_pass(PM_FUSED, ps.orient, b1, Y, Wst(ps.k), Y, cr, ci, scale_of(ps.k),
                                         scale_of(ps.k - 1), 1.f, 0.f, sp, v);
                }
            }
            QW_HIP(hipGetLastError());
            continue;
        }
        // fused schedule in two ping-pong buffers; X holds the last completed b_k
        C *X = vec(L.A, 0), *Y = vec(L.B, 0);
        coef_of(sp.alpha, sp.K, cr, ci);
        hipLaunchKernelGGL(k_scale<float>, dim3(eg_grid), dim3(256), 0, s, reinterpret_cast<const CVec<float> *>(v),
                           reinterpret_cast<CVec<float> *>(X), (float)cr, (float)ci, (uint64_t)(N / 2));
        auto save = [&](int k, const C *src) -> qw_status {
            if (k >= 1 && sp.slot[k] >= 0)
                QW_HIP(hipMemcpyAsync(vec(L.ckpt, sp.slot[k]), src, N * sizeof(C), hipMemcpyDeviceToDevice, s));
            return QW_OK;
        };
        if ((st = save(sp.K, X)) != QW_OK) return st;
        auto scale_of = [](int k) { return k == 0 ? 1.0 : 2.0; };
        for (const SchedPass &ps : fused_schedule(sp.K, P)) {
            const float pr = ps.fin ? sp.ph_r : 1.f, pi = ps.fin ? sp.ph_i : 0.f;
            if (ps.mode == PM_START) {
                coef_of(sp.alpha, ps.k, cr, ci);
                launch_clenshaw_pass(PM_START, ps.orient, X, (ps.k == sp.K - 1) ? nullptr : Y, ps.fin ? y : Y,
                                     nullptr, cr, ci, scale_of(ps.k), 0.0, pr, pi, sp, v);
                if (P == 1 && !ps.fin) {
                    std::swap(X, Y);
                    if ((st = save(ps.k, X)) != QW_OK) return st;
                }
            } else if (ps.mode == PM_ADD) {
                launch_clenshaw_pass(PM_ADD, ps.orient, X, Y, ps.fin ? y : Y, nullptr, 0.0, 0.0, scale_of(ps.k), 0.0,
                                     pr, pi, sp, v);
            } else {
                coef_of(sp.alpha, ps.k - 1, cr, ci);
                launch_clenshaw_pass(PM_FUSED, ps.orient, X, Y, Y, X, cr, ci, scale_of(ps.k), scale_of(ps.k - 1),
                                     1.f, 0.f, sp, v);
                std::swap(X, Y);
                if ((st = save(ps.k, X)) != QW_OK) return st;
            }
        }
        QW_HIP(hipGetLastError());
    }
    if (psiT_out)
        QW_HIP(hipMemcpyAsync(psiT_out, states + (size_t)S * N, N * sizeof(C), hipMemcpyDeviceToDevice, s));

    // seed: ybar = 2 H_P psi_S, G = |psi_S|^2, energy
    hipLaunchKernelGGL(k_zero_f64, dim3(64), dim3(256), 0, s, partm, 2 * L.ntiles_lo);
    {
        EwArgs ea{};
        ea.x = states + (size_t)S * N;
        ea.y = vbar;
        ea.G = G;
        ea.erel = erel;
        ea.part = partm;
        ea.c = c;
        ea.TE = TEw;
        hipLaunchKernelGGL(k_seed, dim3(ntw), dim3(256), 0, s, ea);
    }
    QW_HIP(hipGetLastError());
    std::vector<double> hp(2 * std::max(L.ntiles_lo * 4, ntw));
    QW_HIP(hipMemcpyAsync(hp.data(), partm, 2 * ntw * sizeof(double), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    double energy = 0.0;
    for (int i = 0; i < ntw; ++i) energy += hp[2 * i];
    *E_out = energy;

    // backward sweep
    for (int q = S - 1; q >= 0; --q) {
        const SegPlan &sp = seg[q];
        const C *v = states + (size_t)q * N;
        const C *y = states + (size_t)(q + 1) * N;
        hipLaunchKernelGGL(k_zero_f64, dim3(64), dim3(256), 0, s, part, 2 * L.ntiles_lo * 4);
        hipLaunchKernelGGL(k_zero_f64, dim3(64), dim3(256), 0, s, partm, 2 * L.ntiles_lo);
        C *Acur = vec(L.A, 0), *Bnxt = vec(L.B, 0);
        {
            EwArgs ea{};
            ea.x = vbar;           // ybar
            ea.v = y;
            ea.y = Acur;           // beta_0
            ea.z = vbar;           // zeroed
            ea.part = partm;
            ea.c = c;
            ea.cr = sp.ph_r;       // conj(phase) = (ph_r, -ph_i)
            ea.ci = -sp.ph_i;
            ea.TE = TEw;
            hipLaunchKernelGGL(k_beta0, dim3(ntw), dim3(256), 0, s, ea);
        }
        const C *prevp = nullptr;
        for (int w = 0; w < sp.W; ++w) {
            const int Bw = w * sp.C + 1, Tw = std::min((w + 1) * sp.C, sp.K);
            // store mode: one window, b_1 .. b_K already in their slots
            C *win = L.store ? vec(L.win, sp.sbase) : vec(L.win, 0);
            // recompute b_Tw .. b_Bw into win[j - Bw]
            const C *x1 = nullptr, *x2 = nullptr;
            int jstart = 0;
            double cr, ci;
            if (L.store) {
                // nothing to recompute
            } else if (Tw == sp.K) {
                coef_of(sp.alpha, sp.K, cr, ci);
                hipLaunchKernelGGL(k_scale<float>, dim3(eg_grid), dim3(256), 0, s,
                                   reinterpret_cast<const CVec<float> *>(v),
                                   reinterpret_cast<CVec<float> *>(win + (size_t)(sp.K - Bw) * N), (float)cr, (float)ci,
                                   (uint64_t)(N / 2));
                x1 = win + (size_t)(sp.K - Bw) * N;
                x2 = nullptr;
                jstart = sp.K - 1;
            } else {
                x1 = vec(L.ckpt, sp.slot[Tw + 1]);
                x2 = (Tw + 2 <= sp.K) ? vec(L.ckpt, sp.slot[Tw + 2]) : nullptr;
                jstart = Tw;
            }
            // terms j = jstart .. Bw on the fused schedule, b_j kept in win[j - Bw];
            // every term visits the orientations in the order the forward sweep
            // used (mirrored when the window starts on the other parity), so the
            // recomputed b_j equal the forward ones bit for bit
            if (!L.store) {
                auto Wj = [&](int j) { return win + (size_t)(j - Bw) * N; };
                auto Bj = [&](int j) -> const C * {
                    if (j <= jstart) return Wj(j);
                    return (j == jstart + 1) ? x1 : x2;
                };
                const bool mirror = ((sp.K - 1 - jstart) & 1) != 0;
                for (SchedPass ps : fused_schedule(jstart - Bw + 1, P)) {
                    if (mirror) ps.orient = P - 1 - ps.orient;
                    const int j = Bw + ps.k;
                    if (ps.mode == PM_START) {
                        coef_of(sp.alpha, j, cr, ci);
                        launch_clenshaw_pass(PM_START, ps.orient, Bj(j + 1), Bj(j + 2), Wj(j), nullptr, cr, ci, 2.0,
                                             0.0, 1.f, 0.f, sp, v);
                    } else if (ps.mode == PM_ADD) {
                        launch_clenshaw_pass(PM_ADD, ps.orient, Bj(j + 1), Wj(j), Wj(j), nullptr, 0.0, 0.0, 2.0, 0.0,
                                             1.f, 0.f, sp, v);
                    } else {
                        coef_of(sp.alpha, j - 1, cr, ci);
                        launch_clenshaw_pass(PM_FUSED, ps.orient, Bj(j + 1), Wj(j), Wj(j), Wj(j - 1), cr, ci, 2.0,
                                             2.0, 1.f, 0.f, sp, v);
                    }
                }
            }
            // adjoint steps k = Bw-1 .. Tw-1 with b_{k+1} = win[k + 1 - Bw].  Step k
            // visits the orientations in order 0..P-1 (k even) or reversed (k
            // odd), so its last orientation is the first of step k + 1 and the
            // two share one FUSED pass whenever b_{k+2} is in the window.  The
            // order depends on k alone and a partial sum goes to the slot of the
            // pass's position in its step, so the result does not depend on the
            // checkpoint interval.
            {
                auto orient = [&](int k, int i) { return (k & 1) ? P - 1 - i : i; };
                auto step_of = [&](int k) {
                    double ckr, cki, dcr, dci;
                    coef_of(sp.alpha, k, ckr, cki);
                    coef_of(sp.dalpha, k, dcr, dci);
                    const double wk = (k == 0) ? 1.0 : 2.0;
                    AdjStep st;
                    st.scale = (k == 0) ? 1.f : 2.f;
                    st.ckr = (float)ckr;
                    st.cki = (float)cki;
                    st.gw = (float)(wk * sp.inv_r);
                    st.wk = wk;
                    st.dcr = dcr * sp.r;
                    st.dci = dci * sp.r;
                    return st;
                };
                auto bwin = [&](int j) { return win + (size_t)(j - Bw) * N; };
                auto slot = [&](int i) { return part + (size_t)2 * L.ntiles_lo * i; };
                bool started = false;   // step k was started by the previous fused pass
                for (int k = Bw - 1; k <= Tw - 1; ++k) {
                    AdjArgs aa{};
                    aa.v = v;
                    aa.vbar = vbar;
                    aa.G = G;
                    aa.erel = erel;
                    aa.dscale = (float)sp.inv_r;
                    aa.g = (float)sp.g;
                    aa.st = step_of(k);
                    aa.beta = Acur;
                    aa.bnext = bwin(k + 1);
                    auto launch = [&](int mode, int o) {
                        aa.L = plan[o].L;
                        aa.g0 = plan[o].g0;
                        aa.h = plan[o].h;
                        launch_adj_pass(aa, mode, N >> (plan[o].L + plan[o].h), cfg, s);
                    };
                    if (!started) {
                        aa.prev = prevp;
                        aa.dst = Bnxt;
                        aa.part = slot(0);
                        launch(AM_START, orient(k, 0));
                    }
                    started = false;
                    for (int i = 1; i <= P - 2; ++i) {
                        aa.prev = Bnxt;
                        aa.dst = Bnxt;
                        aa.part = slot(i);
                        launch(AM_ADD, orient(k, i));
                    }
                    if (P >= 2) {
                        aa.prev = Bnxt;
                        aa.dst = Bnxt;
                        aa.part = slot(P - 1);
                        if (k + 1 <= Tw - 1) {
                            aa.dst2 = Acur;          // beta_{k+2} over beta_k
                            aa.bnext2 = bwin(k + 2);
                            aa.part2 = slot(0);
                            aa.st2 = step_of(k + 1);
                            launch(AM_FUSED, orient(k, P - 1));
                            started = true;
                        } else {
                            launch(AM_ADD, orient(k, P - 1));
                        }
                    }
                    prevp = Acur;
                    std::swap(Acur, Bnxt);
                }
            }
            QW_HIP(hipGetLastError());
        }
        {
            double ckr, cki, dcr, dci;
            coef_of(sp.alpha, sp.K, ckr, cki);
            coef_of(sp.dalpha, sp.K, dcr, dci);
            EwArgs ea{};
            ea.x = Acur;   // beta_K
            ea.v = v;
            ea.y = vbar;
            ea.part = part;   // pass-0 slots, same tile count
            ea.cr = (float)ckr;
            ea.ci = (float)cki;
            ea.dcr = dcr * sp.r;
            ea.dci = dci * sp.r;
            ea.TE = TEw;
            hipLaunchKernelGGL(k_adj_last, dim3(ntw), dim3(256), 0, s, ea);
            QW_HIP(hipGetLastError());
        }
        const size_t npart = (size_t)2 * L.ntiles_lo * P;
        std::vector<double> pp(npart), pm(2 * ntw);
        QW_HIP(hipMemcpyAsync(pp.data(), part, npart * sizeof(double), hipMemcpyDeviceToHost, s));
        QW_HIP(hipMemcpyAsync(pm.data(), partm, pm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        QW_HIP(hipStreamSynchronize(s));
        double sdt = 0.0, sdg = 0.0, sph = 0.0;
        for (size_t i = 0; i < npart; i += 2) {
            sdt += pp[i];
            sdg += pp[i + 1];
        }
        for (int i = 0; i < ntw; ++i) sph += pm[2 * i];
        dt[q] = sdt + sph;
        dgamma[q] = sdg / sp.r;
    }

    // Walsh reduction of G
    const int wt = (n > LB_TAB) ? (1 << (n - LB_TAB)) : 1;
    double *walsh = reinterpret_cast<double *>(ws + L.walsh);
    double *wres = reinterpret_cast<double *>(ws + L.wres);
    hipLaunchKernelGGL(k_walsh_tile, dim3(wt), dim3(256), 0, s, (const float *)G, n, std::min(n, LB_TAB), walsh);
    hipLaunchKernelGGL(k_walsh_reduce, dim3(L.npar), dim3(256), 0, s, (const double *)walsh, wt, L.npar, wres);
    QW_HIP(hipGetLastError());
    std::vector<double> res(L.npar);
    QW_HIP(hipMemcpyAsync(res.data(), wres, L.npar * sizeof(double), hipMemcpyDeviceToHost, s));
    QW_HIP(hipStreamSynchronize(s));
    std::memcpy(dh, res.data(), n * sizeof(double));
    if (np) std::memcpy(dJ, res.data() + n, np * sizeof(double));
    if (info) {
        info->amp_terms = amp_terms;
        info->passes = P;
        int sk = 0;
        for (auto &x : seg) sk += x.K;
        info->sum_K = sk;
        if (timing) {
            QW_HIP(hipEventRecord(ev[1], s));
            QW_HIP(hipEventSynchronize(ev[1]));
            QW_HIP(hipEventElapsedTime(&info->total_ms, ev[0], ev[1]));
        }
    }
    return QW_OK;
}

}  // namespace qw

using namespace qw;

extern "C" {

size_t qw_anneal_workspace_bytes_c64(int n, const double *h, const double *J, int S, const double *gamma,
                                     const double *t, int ckpt_every)
{
    if (grad_validate(n, h, J, S, gamma, t, 1.0) != QW_OK) return 0;
    const std::vector<int> Kb = grad_bounds(n, h, J, S, gamma, t);
    return grad_layout(n, S, Kb.data(), ckpt_every).total;
}

qw_status qw_anneal_energy_grad_c64(int n, const double *h, const double *J, int S, const double *gamma,
                                    const double *t, const void *psi0, double tol, int ckpt_every, double *E,
                                    double *dgamma, double *dt, double *dh, double *dJ, void *workspace,
                                    size_t ws_bytes, void *stream, void *psiT_out, qw_grad_info *info)
{
    if (info) {
        const int tm = info->timing;
        std::memset(info, 0, sizeof(*info));
        info->timing = tm;
    }
    return grad_impl(n, h, J, S, gamma, t, psi0, tol, ckpt_every, E, dgamma, dt, dh, dJ, workspace, ws_bytes,
                     reinterpret_cast<hipStream_t>(stream), psiT_out, info);
}

}  // extern "C"
