// Driver of libhe's host arithmetic (prime chain, roots, ChaCha20, secret
// sampler, FP64 encode / decode, the step's and the inference's scale plans)
// under AddressSanitizer and UndefinedBehaviorSanitizer, host code only.  Every
// routine runs over the ring degrees and parameters the library accepts, and
// on inputs it must refuse; a few results are checked so the calls do real
// work.  Exit status 0 with "ok" on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sys/wait.h>
#include <thread>
#include <unistd.h>
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

    // the transforms run their loops over a thread pool: the result does not
    // depend on it.  A child forked here has no pool workers and runs every
    // loop on its one thread; its encode and decode equal the parent's bit
    // for bit, and so do those of callers that overlap (all but one of them
    // find the pool busy and run alone).
    {
        const int logN = 16, N = 1 << logN, S = N / 2;
        std::vector<double> re(S), im(S), md(N), dre(S), dim(S);
        for (int j = 0; j < S; ++j) {
            re[j] = std::sin(0.013 * j) * 3.0;
            im[j] = std::cos(0.007 * j);
        }
        std::vector<i64> m(N);
        CHECK(encode(logN, re.data(), im.data(), S, std::ldexp(1.0, 40), m.data()) == 0);
        for (int i = 0; i < N; ++i) md[i] = (double)m[i] + 0.25 * (i % 3);
        decode(logN, md.data(), std::ldexp(1.0, 40), S, dre.data(), dim.data());
        int fd[2];
        CHECK(pipe(fd) == 0);
        const pid_t pid = fork();
        CHECK(pid >= 0);
        if (pid == 0) {
            std::vector<i64> mc(N);
            std::vector<double> cre(S), cim(S);
            int same = encode(logN, re.data(), im.data(), S, std::ldexp(1.0, 40), mc.data()) == 0 && mc == m;
            decode(logN, md.data(), std::ldexp(1.0, 40), S, cre.data(), cim.data());
            same = same && cre == dre && cim == dim;
            const char r = same ? 'y' : 'n';
            (void)!write(fd[1], &r, 1);
            _exit(0);
        }
        char r = 0;
        CHECK(read(fd[0], &r, 1) == 1);
        int st = 0;
        CHECK(waitpid(pid, &st, 0) == pid && WIFEXITED(st));
        CHECK(r == 'y');
        close(fd[0]);
        close(fd[1]);
        std::vector<std::vector<i64>> outs(4, std::vector<i64>(N));
        std::vector<std::thread> th;
        for (int t = 0; t < 4; ++t)
            th.emplace_back([&, t] { CHECK(encode(logN, re.data(), im.data(), S, std::ldexp(1.0, 40), outs[t].data()) == 0); });
        for (auto &t : th) t.join();
        for (auto &o : outs) CHECK(o == m);
    }

    // the decryption's centred CRT of two limbs: residues of known integers w,
    // |w| < q0 q1 / 2 (small, near the bound, random), come back as w rounded
    // to the nearest double
    {
        const u64 q0 = (1ull << 60) - 93, q1 = (1ull << 40) - 87;
        const u128 H = ((u128)q0 * q1) / 2;
        const size_t N = 1 << 14;
        std::vector<u64> r0(N), r1(N);
        std::vector<u128> w(N);
        std::vector<bool> neg(N);
        u64 x = 88172645463325252ull;
        auto next = [&] {
            x ^= x << 13, x ^= x >> 7, x ^= x << 17;
            return x;
        };
        for (size_t i = 0; i < N; ++i) {
            if (i < 4) w[i] = i;
            else if (i < 8) w[i] = H - (i - 4);
            else w[i] = (((u128)next() << 64) | next()) % (H + 1);
            neg[i] = (next() & 1) && w[i] != 0;
            const u128 Q = (u128)q0 * q1, v = neg[i] ? Q - w[i] : w[i];
            r0[i] = (u64)(v % q0);
            r1[i] = (u64)(v % q1);
        }
        std::vector<double> mm(N);
        crt2_centred(r0.data(), r1.data(), N, q0, q1, mm.data());
        for (size_t i = 0; i < N; ++i) CHECK(mm[i] == (neg[i] ? -(double)w[i] : (double)w[i]));
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
