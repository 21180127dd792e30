// Host-only driver for the sanitizer build of the MPO builders (test
// infrastructure): builds the normal/complementary MPO with every recursion
// basis, compressed and exact, the stacked sub-Hamiltonian MPOs of both
// splits and the affine transform on small random integrals, and feeds the
// argument checks malformed input.  No GPU call is made.
#include <cstdio>
#include <random>
#include <vector>

#include "core.h"

using namespace dmrg;

static void integrals(int K, unsigned seed, std::vector<double>& h, std::vector<double>& v) {
    std::mt19937_64 g(seed);
    std::normal_distribution<double> n(0.0, 1.0);
    h.assign(size_t(K) * K, 0.0);
    v.assign(size_t(K) * K * K * K, 0.0);
    for (int i = 0; i < K; ++i)
        for (int j = i; j < K; ++j) h[i * K + j] = h[j * K + i] = n(g);
    // v = sum_Q L^Q_ij L^Q_kl: the 8-fold symmetry by construction
    for (int Q = 0; Q < K; ++Q) {
        std::vector<double> L(size_t(K) * K);
        for (int i = 0; i < K; ++i)
            for (int j = i; j < K; ++j) L[i * K + j] = L[j * K + i] = 0.3 * n(g);
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j)
                for (int k = 0; k < K; ++k)
                    for (int l = 0; l < K; ++l) v[((size_t(i) * K + j) * K + k) * K + l] += L[i * K + j] * L[k * K + l];
    }
}

int main() {
    int built = 0, rejected = 0;
    for (int K = 2; K <= 6; ++K) {
        std::vector<double> h, v;
        integrals(K, 100 + K, h, v);
        const int N = K, tsz = K % 2;
        for (int basis = 0; basis <= 4; ++basis)
            for (double tol : {0.0, 1e-3}) {
                auto m = build_mpo(h.data(), v.data(), K, N, tsz, -1, tol, basis);
                auto a = affine_mpo(*m, 1.0, -0.1);
                built += 2;
            }
        for (int g = 0; g <= 1; ++g) {
            auto s = build_sum_mpo(h.data(), v.data(), K, N, tsz, g);
            auto a = affine_mpo(*s, 0.5, 2.0);
            built += 2;
        }
        // malformed input: each must throw dmrg::Error
        std::vector<double> hb = h;
        hb[1] += 1.0;  // not symmetric (K >= 2)
        auto expect_throw = [&](auto f) {
            try {
                f();
            } catch (const Error&) {
                ++rejected;
                return;
            }
            std::fprintf(stderr, "malformed input accepted (K=%d)\n", K);
            std::exit(1);
        };
        expect_throw([&] { build_mpo(hb.data(), v.data(), K, N, tsz, -1, 0.0, 0); });
        expect_throw([&] { build_mpo(h.data(), v.data(), K, N, tsz, -1, 0.0, 7); });
        expect_throw([&] { build_mpo(h.data(), v.data(), K, 2 * K + 1, tsz, -1, 0.0, 0); });
        expect_throw([&] { build_sum_mpo(h.data(), v.data(), K, N, tsz, 2); });
        expect_throw([&] { build_sum_mpo(h.data(), v.data(), K, N, tsz + 1, 0); });
    }
    std::printf("host driver: %d MPOs built, %d malformed inputs rejected\n", built, rejected);
    return 0;
}
