// Device-side building blocks shared by the HIP translation units of libqwexp:
// complex vector types, the tile geometry of a hypercube pass, and the
// per-tile Ising energy tables.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qw {

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

// 16 bytes of consecutive complex values (2 x complex64 or 1 x complex128): the
// unit of every global load and store, so each lane moves 16 B per access.
template <typename R> struct alignas(16) CVec {
    static constexpr int N = 16 / (2 * (int)sizeof(R));
    typename Cplx<R>::T v[N];
};

// ---------------------------------------------------------------------------
// Tile geometry of one global pass over the state (section II.D: the
// hypercube sum is split over groups of bits).  A tile holds 2^(L+h) amplitudes:
// tile element e has its low L bits on index bits 0..L-1 ("passenger" bits
// that keep every memory row contiguous but are not flipped in this pass) and
// its next h bits on index bits g0..g0+h-1 (the flipped group).  The tile id t
// supplies the remaining index bits, L..g0-1 first and then g0+h..n-1.  The
// first pass of a term uses L = 0, g0 = 0 (one contiguous block).
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t tile_base(uint64_t t, int L, int g0, int h)
{
    const int lowcnt = g0 - L;
    const uint64_t tlo = t & ((uint64_t(1) << lowcnt) - 1);
    const uint64_t thi = t >> lowcnt;
    return (tlo << L) | (thi << (g0 + h));
}

__host__ __device__ inline uint64_t tile_index(uint64_t base, uint32_t e, int L, int g0)
{
    const uint32_t lmask = (1u << L) - 1u;
    return base | (uint64_t)(e & lmask) | ((uint64_t)(e >> L) << g0);
}

// Packed row-major upper-triangle offset of J_jk, j < k.
__host__ __device__ inline int pair_off(int n, int j, int k)
{
    return j * n - j * (j + 1) / 2 + (k - j - 1);
}

// Ising energy tables.  Index z splits into lo = z mod 2^LB and hi = z >> LB;
//   E(z) = C(hi) + Q[lo] + sum_{j<LB} f_j(hi) s_j(lo),
//   f_j(hi) = h_j + sum_{k>=LB} J_jk s_k,  C(hi) = sum_{j>=LB} h_j s_j
//             + sum_{LB<=j<k} J_jk s_j s_k,  Q[lo] = sum_{j<k<LB} J_jk s_j s_k.
struct EnergyTables {
    const double *h;  // n
    const double *J;  // n(n-1)/2, packed upper triangle
    const double *Q;  // 2^LB
    int n, LB;
};

// Fields f_j (j < LB) and constant C of the tile with high bits `hi`, computed
// by threads 0..LB of the block into shared memory (caller synchronises).
__device__ inline void tile_fields(const EnergyTables &T, uint64_t hi, double *f, double *C)
{
    const int t = threadIdx.x;
    if (t < T.LB) {
        double acc = T.h[t];
        for (int k = T.LB; k < T.n; ++k) {
            const double Jk = T.J[pair_off(T.n, t, k)];
            acc += ((hi >> (k - T.LB)) & 1) ? -Jk : Jk;
        }
        f[t] = acc;
    } else if (t == T.LB) {
        double acc = 0.0;
        for (int j = T.LB; j < T.n; ++j) {
            const double sj = ((hi >> (j - T.LB)) & 1) ? -1.0 : 1.0;
            double fj = T.h[j];
            for (int k = j + 1; k < T.n; ++k) {
                const double Jk = T.J[pair_off(T.n, j, k)];
                fj += ((hi >> (k - T.LB)) & 1) ? -Jk : Jk;
            }
            acc += sj * fj;
        }
        *C = acc;
    }
}

}  // namespace qw
