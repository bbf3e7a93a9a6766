// Driver of libhe's host arithmetic (prime chain, roots, ChaCha20, secret
// sampler, FP64 encode / decode, the step's and the inference's scale plans)
// under AddressSanitizer and UndefinedBehaviorSanitizer, host code only.  Every
// routine runs over the ring degrees and parameters the library accepts, and
// on inputs it must refuse; a few results are checked so the calls do real
// work.  Exit status 0 with "ok" on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "he_internal.h"

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            std::exit(1);                                                   \
        }                                                                   \
    } while (0)

int main()
{
    using namespace hehost;
    // prime chains of every configuration used, and refusals
    const int cfg[][3] = {{5, 1, 30}, {5, 2, 40}, {20, 4, 40}, {21, 4, 40}, {24, 6, 40}, {8, 2, 40}, {1, 1, 20}};
    for (auto &c : cfg) {
        std::vector<u64> q(c[0] + c[1]);
        CHECK(gen_primes(c[0], c[1], c[2], q.data()) == 0);
        for (u64 p : q) CHECK(p % (1ull << 17) == 1);
        for (int logN = 1; logN <= 16; ++logN) {
            const u64 psi = find_psi(q[0], logN);
            CHECK(powmod(psi, 1ull << logN, q[0]) == q[0] - 1);
        }
        CHECK(mulmod(q[0] - 1, q[0] - 1, q[0]) == 1 && mulmod(invmod(12345, q[0]), 12345, q[0]) == 1);
        CHECK(shoup(q[0] - 1, q[0]) > 0);
    }
    u64 dummy[128];
    (void)gen_primes(0, 1, 40, dummy);  // an empty chain: refused or not, no fault

    // ChaCha20: counter wrap and all-ones key
    uint32_t key[8], nonce[3] = {~0u, ~0u, ~0u}, out[16];
    for (auto &k : key) k = ~0u;
    chacha20_block(key, ~0u, nonce, out);

    // secret sampler: every ring degree, weights 0, 1, 64 and N
    for (int logN = 1; logN <= 16; ++logN) {
        const int N = 1 << logN;
        std::vector<i64> s(N);
        for (int h : {0, 1, 64, N}) {
            if (h > N) continue;
            sample_hwt(99, logN, h, s.data());
            int nz = 0;
            for (i64 v : s) {
                CHECK(v >= -1 && v <= 1);
                nz += v != 0;
            }
            CHECK(nz == h);
        }
    }

    // encode / decode round trip: every ring degree, full and partial slot
    // counts, complex values, scales 2^20 .. 2^50; refusal past 2^62
    for (int logN = 1; logN <= 16; ++logN) {
        const int N = 1 << logN, S = N / 2;
        for (int n : {S, S / 2 > 0 ? S / 2 : 1, 1}) {
            for (double scale : {std::ldexp(1.0, 20), std::ldexp(1.0, 40), std::ldexp(1.0, 50)}) {
                std::vector<double> re(n), im(n), re2(n), im2(n), md(N);
                for (int j = 0; j < n; ++j) {
                    re[j] = std::sin(0.37 * j + logN);
                    im[j] = std::cos(0.11 * j);
                }
                std::vector<i64> m(N);
                CHECK(encode(logN, re.data(), im.data(), n, scale, m.data()) == 0);
                for (int i = 0; i < N; ++i) md[i] = (double)m[i];
                decode(logN, md.data(), scale, n, re2.data(), im2.data());
                double err = 0.0;
                for (int j = 0; j < n; ++j) err = std::fmax(err, std::fabs(re2[j] - re[j]) + std::fabs(im2[j] - im[j]));
                CHECK(err < (double)N / scale * 4.0 + 1e-12);
                decode(logN, md.data(), scale, n, re2.data(), nullptr);
            }
        }
        std::vector<double> big(S > 0 ? S : 1, std::ldexp(1.0, 70));
        std::vector<i64> m(N);
        CHECK(encode(logN, big.data(), nullptr, S > 0 ? S : 1, 1.0, m.data()) != 0);
    }

    // scale plans: both layouts, every level, losses with a2 = 0 and a2 != 0,
    // weight decay, tiny and large eta / n, and refusals
    std::vector<u64> q(24);
    CHECK(gen_primes(20, 4, 40, q.data()) == 0);
    const double coefs[][4] = {{0.5, -0.2, 0.0, 0.002}, {0.5, -0.5, 0.1, -0.01}, {0.0, 0.0, 0.0, 0.0}};
    int ok = 0, refused = 0;
    for (int layout : {(int)HE_LAYOUT_ROWS, (int)HE_LAYOUT_FEATURES, 7}) {
        for (int level = -1; level <= 21; ++level) {
            for (auto &cf : coefs) {
                for (double eta : {1.0 / 6000, 1e-9, 1.0}) {
                    for (double wd : {0.0, 0.05, 1.5}) {
                        he_lr_plan pl;
                        const he_status st = plan_lr_step(q.data(), 20, level, std::ldexp(1.0, 40),
                                                          std::ldexp(1.0, 40), cf, eta, wd, layout, &pl);
                        (st == HE_OK ? ok : refused)++;
                    }
                }
            }
        }
    }
    CHECK(ok > 0 && refused > 0);
    for (int level = -1; level <= 21; ++level) {
        he_infer_plan ip;
        const he_status st = plan_lr_infer(q.data(), 20, level, std::ldexp(1.0, 40), std::ldexp(1.0, 40), coefs[0], &ip);
        CHECK((st == HE_OK) == (level >= 3 && level < 20));
    }
    std::printf("ok\n");
    return 0;
}
