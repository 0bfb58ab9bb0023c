// Host-only checks of libqwexp's index maps, pass plans, fused schedule and
// coefficient setup, built with the address and undefined-behaviour sanitizers
// by tests/test_sanitized_host.py (no GPU: only host code runs).
//
// Prints "COEF method a tol K alpha_0 .. alpha_K" and "BESSEL a m J_m" lines
// for the Python side to compare with the oracle; exits non-zero on the first
// failed structural check.
#include "qw_kernels.h"

#include <cstdio>
#include <cstdlib>
#include <vector>

namespace qw {
void set_error(const std::string &msg) { std::fprintf(stderr, "set_error: %s\n", msg.c_str()); }
}  // namespace qw

using namespace qw;

#define CHECK(cond, ...)                                              \
    do {                                                              \
        if (!(cond)) {                                                \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                        \
            std::fprintf(stderr, "\n");                               \
            std::exit(1);                                             \
        }                                                             \
    } while (0)

// Every (tile, element) of every orientation hits each index once, the
// flipped partners stay inside the tile, and the groups cover the n bits once.
template <typename R> static void check_plans(int n, bool full)
{
    const std::vector<OrientSpec> spec = action_plan<R>(n, true);
    uint64_t covered = 0;
    for (size_t o = 0; o < spec.size(); ++o) {
        const PassPlan &p = spec[o].pl;
        for (const TileCfg &pc : {spec[o].fused, spec[o].add})
            CHECK(p.L + p.h <= pc.tb, "n=%d orientation %zu: %d + %d bits exceed the 2^%d tile", n, o, p.L, p.h, pc.tb);
        CHECK(!spec[o].otf || p.L + p.h == spec[o].fused.tb, "n=%d orientation %zu: on-the-fly tile not full", n, o);
        CHECK(p.h >= 1 && p.g0 + p.h <= n, "n=%d orientation %zu: group out of range", n, o);
        for (int j = 0; j < p.h; ++j) {
            const uint64_t bit = uint64_t(1) << (p.g0 + j);
            CHECK(!(covered & bit), "n=%d: bit %d flipped twice", n, p.g0 + j);
            covered |= bit;
        }
        if (!full) continue;
        const uint64_t N = uint64_t(1) << n;
        std::vector<uint8_t> seen(N, 0);
        const uint64_t ntiles = N >> (p.L + p.h);
        const uint32_t TE = 1u << (p.L + p.h);
        for (uint64_t t = 0; t < ntiles; ++t) {
            const uint64_t base = tile_base(t, p.L, p.g0, p.h);
            for (uint32_t e = 0; e < TE; ++e) {
                const uint64_t idx = tile_index(base, e, p.L, p.g0);
                CHECK(idx < N && !seen[idx], "n=%d orientation %zu: index %llu hit twice", n, o,
                      (unsigned long long)idx);
                seen[idx] = 1;
                for (int j = 0; j < p.h; ++j) {
                    const uint32_t pe = e ^ (1u << (p.L + j));
                    CHECK(pe < TE && tile_index(base, pe, p.L, p.g0) == (idx ^ (uint64_t(1) << (p.g0 + j))),
                          "n=%d orientation %zu: flip %d leaves the tile", n, o, j);
                }
            }
        }
    }
    CHECK(covered == ((n == 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1)), "n=%d: groups miss a bit", n);
}

// Term k visits every orientation once; the last orientation of term k is the
// first of term k - 1 (one FUSED pass does both); the final pass is last.
static void check_schedule(int K, int P)
{
    const std::vector<SchedPass> S = fused_schedule(K, P);
    std::vector<std::vector<int>> seen(K, std::vector<int>(P, 0));
    int fins = 0;
    for (size_t i = 0; i < S.size(); ++i) {
        const SchedPass &sp = S[i];
        CHECK(sp.k >= 0 && sp.k < K && sp.orient >= 0 && sp.orient < P, "K=%d P=%d: pass %zu out of range", K, P, i);
        seen[sp.k][sp.orient]++;
        if (sp.mode == PM_FUSED) {
            CHECK(sp.k >= 1, "K=%d P=%d: fused pass completes term 0", K, P);
            seen[sp.k - 1][sp.orient]++;   // starts term k - 1 in the same orientation
        }
        if (sp.fin) {
            ++fins;
            CHECK(i + 1 == S.size() && sp.k == 0, "K=%d P=%d: final pass not last", K, P);
        }
    }
    CHECK(fins == 1, "K=%d P=%d: %d final passes", K, P, fins);
    for (int k = 0; k < K; ++k)
        for (int o = 0; o < P; ++o) CHECK(seen[k][o] == 1, "K=%d P=%d: term %d orientation %d seen %d times", K, P, k, o, seen[k][o]);
}

int main()
{
    for (int n = 1; n <= 32; ++n) {
        check_plans<float>(n, n <= 22);
        check_plans<double>(n, n <= 22);
    }
    for (int P = 1; P <= 4; ++P)
        for (int K = 1; K <= 60; ++K) check_schedule(K, P);
    // XCD-major tile order is a permutation of the launch's blocks
    for (uint32_t nb : {1u, 7u, 8u, 64u, 520u, 4096u, 32768u}) {
        std::vector<uint8_t> hit(nb, 0);
        for (uint32_t b = 0; b < nb; ++b) {
            const uint64_t t = xcd_tile(b, nb);
            CHECK(t < nb && !hit[t], "xcd_tile(%u, %u) = %llu", b, nb, (unsigned long long)t);
            hit[t] = 1;
        }
    }
    std::printf("PLANS OK\n");

    const double as[] = {0.0, 1e-3, 0.7, 5.0, 22.0, 99.0, 300.0, -40.0};
    const double tols[] = {std::ldexp(1.0, -23), 1e-12};
    for (double a : as)
        for (double tol : tols)
            for (int method = 0; method <= 1; ++method) {
                std::vector<double> alpha;
                int K = -1;
                double err = -1.0;
                CHECK(coefficients(a, tol, method, alpha, &K, &err) == 0, "coefficients(%g, %g, %d)", a, tol, method);
                CHECK(K >= 0 && (int)alpha.size() >= K + 1, "coefficients(%g): K = %d", a, K);
                std::printf("COEF %d %.17g %.17g %d", method, a, tol, K);
                for (int k = 0; k <= K; ++k) std::printf(" %.17g", alpha[k]);
                std::printf("\n");
            }
    for (double a : {0.5, 20.0, 150.0}) {
        const int mmax = bessel_cutoff(a) + 5;
        std::vector<double> J(mmax + 1, 0.0);
        CHECK(bessel_miller(a, mmax, J.data()) == 0, "bessel_miller(%g)", a);
        for (int m = 0; m <= mmax; ++m) std::printf("BESSEL %.17g %d %.17g\n", a, m, J[m]);
    }
    return 0;
}
