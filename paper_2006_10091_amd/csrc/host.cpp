// host.cpp -- host-side arithmetic of libhe: prime chain, roots, Shoup
// companions, the ChaCha20 stream and the secret sampler (keygen runs it once
// on the host), FP64 canonical-embedding encode/decode, and the FP64 scale
// schedule of the gradient step.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <condition_variable>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <cstring>
#include <unistd.h>
#include <vector>

#include "he_internal.h"

namespace hehost {

// A fixed set of worker threads for the host transforms (the refresh runs
// a decode and an encode back to back).  run(n, f) calls f(0) .. f(n-1) on
// the workers and the calling thread and returns once every worker has
// finished this job, so no worker touches a job after run() returns.  Idle
// workers spin for a short while after a job, then sleep.  A caller that
// finds the pool busy (another thread's transform), or runs in a child
// process forked after the workers started (which has none of them), runs
// its items itself.
class HostPool {
public:
    explicit HostPool(int workers) : pid_(getpid())
    {
        for (int i = 0; i < workers; ++i) th_.emplace_back([this] { loop(); });
    }
    int threads() const { return getpid() == pid_ ? (int)th_.size() + 1 : 1; }
    void run(int n, const std::function<void(int)> &f)
    {
        std::unique_lock<std::mutex> one(run_mu_, std::try_to_lock);
        if (!one.owns_lock() || th_.empty() || n <= 1 || getpid() != pid_) {
            for (int i = 0; i < n; ++i) f(i);
            return;
        }
        fn_ = &f;
        n_ = n;
        next_.store(0);
        done_.store(0);
        {
            std::lock_guard<std::mutex> l(mu_);
            gen_.fetch_add(1);
        }
        cv_.notify_all();
        for (int i; (i = next_.fetch_add(1)) < n;) f(i);
        while (done_.load() < (int)th_.size()) std::this_thread::yield();
    }

private:
    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            const auto t0 = std::chrono::steady_clock::now();
            while (gen_.load() == seen && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(2)) {
            }
            if (gen_.load() == seen) {
                std::unique_lock<std::mutex> l(mu_);
                cv_.wait(l, [&] { return gen_.load() != seen; });
            }
            seen = gen_.load();
            const int n = n_;
            const std::function<void(int)> *f = fn_;
            for (int i; (i = next_.fetch_add(1)) < n;) (*f)(i);
            done_.fetch_add(1);
        }
    }
    const pid_t pid_;
    std::vector<std::thread> th_;
    std::mutex mu_, run_mu_;
    std::condition_variable cv_;
    std::atomic<uint64_t> gen_{0};
    std::atomic<int> next_{0}, done_{0};
    int n_ = 0;
    const std::function<void(int)> *fn_ = nullptr;
};

// the process's pool (never destroyed: its threads wait until the process ends)
static HostPool &pool()
{
    static HostPool *p = new HostPool(std::max(0, std::min(8, (int)std::thread::hardware_concurrency()) - 1));
    return *p;
}

// f(i0, i1) over [0, n) in chunks of the pool
static void parallel_range(size_t n, const std::function<void(size_t, size_t)> &f)
{
    const int T = n >= 4096 ? pool().threads() : 1;
    const size_t step = (n + T - 1) / T;
    pool().run(T, [&](int t) {
        const size_t a = std::min(n, (size_t)t * step), b = std::min(n, a + step);
        if (a < b) f(a, b);
    });
}

u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }

u64 powmod(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
    }
    return r;
}

u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); }  // q prime

u64 shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

static bool miller_rabin(u64 n)
{
    if (n < 2) return false;
    const u64 base[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (u64 p : base) {
        if (n % p == 0) return n == p;
    }
    u64 d = n - 1;
    int s = 0;
    for (; !(d & 1); d >>= 1) ++s;
    for (u64 a : base) {
        u64 x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int i = 1; i < s && witness; ++i) {
            x = mulmod(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

// Prime chain: every prime 1 mod 2^17 (one chain for all N <= 2^16);
// specials = n_special largest below 2^60; q_0 = largest below
// 2^min(60, log_delta+20) that is not special; q_1.. = the primes closest to
// 2^log_delta, by increasing distance, ties to the smaller.
int gen_primes(int nq, int nk, int log_delta, u64 *out)
{
    const u64 step = (u64)1 << 17;
    if (nq < 1 || nk < 0 || nq + nk > HE_MAXP || log_delta < 18 || log_delta > 58) return -1;
    u64 c = ((((u64)1 << 60) - 1) / step) * step + 1;
    for (int got = 0; got < nk; c -= step)
        if (miller_rabin(c)) out[nq + got++] = c;
    int b0 = std::min(60, log_delta + 20);
    c = ((((u64)1 << b0) - 1) / step) * step + 1;
    for (;; c -= step) {
        bool special = false;
        for (int i = 0; i < nk; ++i) special |= out[nq + i] == c;
        if (!special && miller_rabin(c)) break;
    }
    out[0] = c;
    const u64 D = (u64)1 << log_delta;
    u64 below = (D / step) * step + 1;
    if (below > D) below -= step;
    u64 above = below + step;
    for (int k = 1; k < nq; ++k) {
        while (!miller_rabin(below)) below -= step;
        while (!miller_rabin(above)) above += step;
        if (D - below <= above - D) {
            out[k] = below;
            below -= step;
        } else {
            out[k] = above;
            above += step;
        }
    }
    return 0;
}

u64 find_psi(u64 q, int logN)
{
    const u64 N = (u64)1 << logN;
    for (u64 x = 2;; ++x) {
        u64 y = powmod(x, (q - 1) / (2 * N), q);
        if (powmod(y, N, q) == q - 1) return y;
    }
}

static inline uint32_t rotl(uint32_t v, int n) { return (v << n) | (v >> (32 - n)); }

// RFC 8439, Sec. 2.3
void chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16])
{
    uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, key[0], key[1], key[2], key[3],
                      key[4],      key[5],      key[6],      key[7],      counter, nonce[0], nonce[1], nonce[2]};
    uint32_t x[16];
    std::memcpy(x, s, sizeof x);
    auto qr = [&](int a, int b, int c, int d) {
        x[a] += x[b]; x[d] = rotl(x[d] ^ x[a], 16);
        x[c] += x[d]; x[b] = rotl(x[b] ^ x[c], 12);
        x[a] += x[b]; x[d] = rotl(x[d] ^ x[a], 8);
        x[c] += x[d]; x[b] = rotl(x[b] ^ x[c], 7);
    };
    for (int r = 0; r < 10; ++r) {
        qr(0, 4, 8, 12); qr(1, 5, 9, 13); qr(2, 6, 10, 14); qr(3, 7, 11, 15);
        qr(0, 5, 10, 15); qr(1, 6, 11, 12); qr(2, 7, 8, 13); qr(3, 4, 9, 14);
    }
    for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

// 64-bit word w of the stream (seed; type, index, comp): block w/8, words
// 2(w%8) (low) and 2(w%8)+1 (high) of that block.
static void stream_words(u64 seed, uint32_t type, uint32_t index, uint32_t comp, size_t count, u64 *out)
{
    const uint32_t key[8] = {(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0};
    const uint32_t nonce[3] = {type, index, comp};
    uint32_t blk[16];
    for (size_t b = 0; b * 8 < count; ++b) {
        chacha20_block(key, (uint32_t)b, nonce, blk);
        for (int t = 0; t < 8 && b * 8 + t < count; ++t) out[b * 8 + t] = blk[2 * t] | ((u64)blk[2 * t + 1] << 32);
    }
}

// Ternary secret with h nonzero entries: partial Fisher-Yates; step k draws
// word 2k (offset mod N-k) and word 2k+1 (low bit set -> -1).
void sample_hwt(u64 seed, int logN, int h, i64 *out)
{
    const u64 N = (u64)1 << logN;
    std::vector<u64> w(2 * (size_t)h), perm(N);
    stream_words(seed, ST_SECRET, 0, 0, w.size(), w.data());
    for (u64 i = 0; i < N; ++i) {
        perm[i] = i;
        out[i] = 0;
    }
    for (int k = 0; k < h; ++k) {
        u64 j = (u64)k + w[2 * k] % (N - (u64)k);
        std::swap(perm[k], perm[j]);
        out[perm[k]] = (w[2 * k + 1] & 1) ? -1 : 1;
    }
}

// Twiddles of every stage of a size-M FFT, stage len at offset len/2 - 1:
// w[len/2 - 1 + k] = exp(sign 2 pi i k / len), k < len/2.  Computed once per
// (M, sign) and kept for the process (the values are those each call used to
// compute, so results do not change).
static const std::vector<std::complex<double>> &fft_twiddles(size_t M, int sign)
{
    static std::mutex mu;
    static std::map<std::pair<size_t, int>, std::vector<std::complex<double>>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto &w = cache[{M, sign}];
    if (w.empty()) {
        w.resize(M - 1);
        for (size_t len = 2; len <= M; len <<= 1)
            for (size_t k = 0; k < len / 2; ++k)
                w[len / 2 - 1 + k] = std::polar(1.0, sign * 2.0 * M_PI * (double)k / (double)len);
    }
    return w;
}

// One radix-2 butterfly of stage `half` (the complex product written out; the
// library is built without contraction, so it rounds as std::complex's
// operator* does for finite operands)
static inline void butterfly(double *d, const double *w, size_t s, size_t k, size_t half)
{
    double *x = d + 2 * (s + k), *y = d + 2 * (s + k + half);
    const double wr = w[2 * k], wi = w[2 * k + 1];
    const double vr = y[0] * wr - y[1] * wi, vi = y[0] * wi + y[1] * wr;
    const double ur = x[0], ui = x[1];
    x[0] = ur + vr;
    x[1] = ui + vi;
    y[0] = ur - vr;
    y[1] = ui - vi;
}

// Butterflies of the radix-2 stages len = len0 .. len1 (powers of two) on the
// elements [lo, hi) of d (interleaved re, im), a whole number of len1 blocks.
static void fft_stages(double *d, const double *wd, size_t lo, size_t hi, size_t len0, size_t len1)
{
    for (size_t len = len0; len <= len1; len <<= 1) {
        const size_t half = len / 2;
        const double *w = wd + 2 * (half - 1);
        for (size_t s = lo; s < hi; s += len)
            for (size_t k = 0; k < half; ++k) butterfly(d, w, s, k, half);
    }
}

// In-place radix-2 complex FFT of size M (power of two):
// A[k] = sum_n a[n] exp(sign * 2 pi i k n / M).  After the bit reversal the
// stages up to length M / T act on T contiguous blocks of their own, one per
// thread of the pool; each of the last log2 T stages is split by butterflies
// over the threads.  Every butterfly is computed as in a one-thread run, so
// the result does not depend on T.
static void fft(std::vector<std::complex<double>> &a, int sign, bool reversed = false)
{
    const size_t M = a.size();
    if (!reversed)  // callers that write their input to bit-reversed positions skip this pass
        for (size_t i = 1, j = 0; i < M; ++i) {
            size_t bit = M >> 1;
            for (; j & bit; bit >>= 1) j ^= bit;
            j ^= bit;
            if (i < j) std::swap(a[i], a[j]);
        }
    const std::vector<std::complex<double>> &tw = fft_twiddles(M, sign);
    double *d = reinterpret_cast<double *>(a.data());
    const double *wd = reinterpret_cast<const double *>(tw.data());
    size_t T = 1;
    if (M >= ((size_t)1 << 14))
        while (2 * T <= (size_t)pool().threads()) T *= 2;
    if (T == 1) {
        fft_stages(d, wd, 0, M, 2, M);
        return;
    }
    const size_t blk = M / T;
    pool().run((int)T, [&](int t) { fft_stages(d, wd, t * blk, (t + 1) * blk, 2, blk); });
    for (size_t len = 2 * blk; len <= M; len <<= 1) {
        const size_t half = len / 2, per = M / 2 / T;  // butterflies per thread
        const double *w = wd + 2 * (half - 1);
        pool().run((int)T, [&](int t) {
            for (size_t j = t * per; j < (t + 1) * per; ++j) butterfly(d, w, (j / half) * len, j % half, half);
        });
    }
}

// Powers zeta^i, i < N, of zeta = exp(sign i pi / N), kept per (N, sign).
static const std::vector<std::complex<double>> &twist(size_t N, int sign)
{
    static std::mutex mu;
    static std::map<std::pair<size_t, int>, std::vector<std::complex<double>>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto &w = cache[{N, sign}];
    if (w.empty()) {
        w.resize(N);
        for (size_t i = 0; i < N; ++i) w[i] = std::polar(1.0, sign * M_PI * (double)i / (double)N);
    }
    return w;
}

// slot j <-> root zeta^(5^j), zeta = exp(i pi / N); the conjugate slot sits at
// zeta^(-5^j).  Only odd powers of zeta occur, so both directions are N-point
// FFTs over omega = zeta^2 with a twist by zeta^i:
//   encode: m_i = (1/N) Re(zeta^-i sum_k V_k omega^-(k i)), V_k the value at zeta^(2k+1);
//   decode: value at zeta^(2k+1) = sum_i (m_i zeta^i) omega^(k i).
// index i of an N-point transform at its bit-reversed position (N = 2^logN)
static inline size_t brev_idx(size_t i, int logN)
{
    return (size_t)(__builtin_bitreverse32((uint32_t)i) >> (32 - logN));
}

// the working vector of one thread, kept between calls (no fresh page
// faults); its contents are left to the caller
static std::vector<std::complex<double>> &fft_buffer(size_t N)
{
    thread_local std::vector<std::complex<double>> buf;
    buf.resize(N);
    return buf;
}

// 5^j mod M (M a power of two): the exponent of slot j's root
static size_t slot_exp(size_t j, size_t M) { return (size_t)powmod(5, j, M); }

// The loops below run in chunks over the pool; each element is computed as
// in a one-thread run.
int encode(int logN, const double *re, const double *im, int n, double scale, i64 *out)
{
    const size_t N = (size_t)1 << logN, M = 2 * N;
    std::vector<std::complex<double>> &V = fft_buffer(N);
    parallel_range(N, [&](size_t i0, size_t i1) { std::fill(V.begin() + i0, V.begin() + i1, 0.0); });
    // slot j and its conjugate: distinct positions for distinct j
    parallel_range((size_t)n, [&](size_t j0, size_t j1) {
        size_t e = slot_exp(j0, M);
        for (size_t j = j0; j < j1; ++j) {
            std::complex<double> z(re[j], im ? im[j] : 0.0);
            V[brev_idx((e - 1) / 2, logN)] = z * scale;
            V[brev_idx((M - e - 1) / 2, logN)] = std::conj(z) * scale;
            e = (e * 5) % M;
        }
    });
    fft(V, -1, true);
    const std::vector<std::complex<double>> &tw = twist(N, -1);
    std::atomic<int> bad{0};
    parallel_range(N, [&](size_t i0, size_t i1) {
        for (size_t i = i0; i < i1; ++i) {
            const double v = (V[i].real() * tw[i].real() - V[i].imag() * tw[i].imag()) / (double)N;
            const double a = std::fabs(v);
            if (!(a < 4.611686018427388e18)) {  // 2^62
                bad.store(1);
                return;
            }
            // half away from zero: floor(|v| + 0.5) is exact below 2^52; above, v is an integer
            const double r = a < 4503599627370496.0 ? std::floor(a + 0.5) : a;
            out[i] = (i64)(v < 0 ? -r : r);
        }
    });
    return bad.load() ? -1 : 0;
}

void decode(int logN, const double *m, double scale, int n, double *re, double *im)
{
    const size_t N = (size_t)1 << logN, M = 2 * N;
    const std::vector<std::complex<double>> &tw = twist(N, +1);
    std::vector<std::complex<double>> &A = fft_buffer(N);  // every entry written
    parallel_range(N, [&](size_t i0, size_t i1) {
        for (size_t i = i0; i < i1; ++i) A[brev_idx(i, logN)] = m[i] * tw[i];
    });
    fft(A, +1, true);
    parallel_range((size_t)n, [&](size_t j0, size_t j1) {
        size_t e = slot_exp(j0, M);
        for (size_t j = j0; j < j1; ++j) {
            const size_t k = (e - 1) / 2;
            re[j] = A[k].real() / scale;
            if (im) im[j] = A[k].imag() / scale;
            e = (e * 5) % M;
        }
    });
}

// Centred CRT of the first two limbs r0 (mod q0), r1 (mod q1) of N
// coefficients, each rounded to the nearest double: v = r0 + q0 d with
// d = (r1 - r0) q0^-1 mod q1, then v - q0 q1 when v > q0 q1 / 2.
void crt2_centred(const u64 *r0, const u64 *r1, size_t N, u64 q0, u64 q1, double *m)
{
    const u64 q0inv = invmod(q0 % q1, q1);
    const u128 Q = (u128)q0 * q1;
    parallel_range(N, [&](size_t x0, size_t x1) {
        for (size_t x = x0; x < x1; ++x) {
            const u64 d = mulmod((r1[x] + q1 - r0[x] % q1) % q1, q0inv, q1);
            const u128 v = (u128)r0[x] + (u128)q0 * d;
            m[x] = v > Q / 2 ? -(double)(Q - v) : (double)v;
        }
    });
}

// Target scale T of the gradient terms, a power of two: the largest with
// T / (eta/n) <= 2^(floor(log2 q_0) - 10) (10 bits of headroom for the output
// in the last limb), kept between the powers of two with
// T * min(|a1|, |a2|, |a3|) over the nonzero ones in [2^22, 2^23) and in
// [2^30, 2^31).  fm_cap > 0 (feature-major): a further upper bound that keeps
// the gradient mask's plaintext scale at 2^34 or more; false when it cannot
// be met together with the lower bound.
static bool term_scale(const double coef[4], u64 q0, double eta_over_n, double fm_cap, double *T)
{
    double amin = 0.0;
    for (int k : {1, 2, 3}) {
        double a = std::fabs(coef[k]);
        if (a != 0.0 && (amin == 0.0 || a < amin)) amin = a;
    }
    if (amin == 0.0) return false;
    int e, ec;
    std::frexp(amin, &e);
    const double lo = std::ldexp(1.0, 23 - e), hi = std::ldexp(1.0, 31 - e);
    const int qbits = 63 - __builtin_clzll(q0);
    std::frexp(std::ldexp(eta_over_n, qbits - 10), &ec);
    const double cap = std::ldexp(1.0, ec - 1);
    if (fm_cap > 0.0) {
        *T = std::min(hi, std::min(cap, fm_cap));
        return !(*T < lo);
    }
    *T = std::max(lo, std::min(hi, cap));
    return true;
}

static he_status finish_plan(double k0, double k1, double k2, double k3, double kb1, double kw, he_lr_plan *o)
{
    const double kmax = 4.611686018427388e18;  // 2^62
    for (double k : {k0, k1, k2, k3, kb1, kw})
        if (!(std::fabs(k) < kmax)) return HE_ESCALE;
    o->k0 = std::llround(k0);
    o->k2 = std::llround(k2);
    o->k1 = std::llround(k1);
    o->k3 = std::llround(k3);
    o->kb1 = std::llround(kb1);
    o->kw = std::llround(kw);
    return HE_OK;
}

// Feature-major schedule: M = u at level l-1 with no mask, the polynomial one
// level above the row-major one, the summed gradient at level l-3 masked down
// to level l-4 by a plaintext whose scale returns W' (and g) to the data's
// scale s_z, so M's scale at the next step stays near q.
static he_status plan_features(const u64 *q, int level, double s_z, double s_w, const double coef[4],
                               double eta_over_n, double w_decay, he_lr_plan *o)
{
    const double ql = (double)q[level], ql1 = (double)q[level - 1], ql2 = (double)q[level - 2],
                 ql3 = (double)q[level - 3];
    int ef;
    std::frexp(s_z * ql3 * eta_over_n, &ef);
    double T;
    if (!term_scale(coef, q[0], eta_over_n, std::ldexp(1.0, ef - 1 - 34), &T)) return HE_ESCALE;
    o->s1 = s_z * s_w / ql;
    o->s_m = o->s1;
    o->s_a = o->s_m * o->s_m / ql1;
    o->t = T;
    o->s_z3 = T * ql2 / o->s_a * ql1 / o->s_m;
    double k3 = coef[3] * o->s_z3 * ql / s_z;
    o->s_b3 = o->s_m * o->s_z3 / ql1;
    o->s_c = o->s_a * o->s_b3 / ql2;
    o->s_z1 = o->s_c * ql2 / o->s_m;
    double k1 = coef[1] * o->s_z1 * ql1 / s_z;
    o->s_b1 = o->s_m * o->s_z1;
    double kb1 = 0.0;
    double k0 = coef[0] * o->s_c * ql2 / s_z;
    o->s_z2 = o->s_c * ql2 / o->s_a;
    double k2 = coef[2] * o->s_z2 * ql1 / s_z;
    o->s_gsum = o->s_c / eta_over_n;
    o->s_mask = s_z * ql3 / o->s_gsum;
    o->s_g = o->s_gsum * o->s_mask / ql3;
    double kw = (1.0 - w_decay) * o->s_g * ql3 / s_w;
    return finish_plan(k0, k1, k2, k3, kb1, kw, o);
}

// FP64 schedule of one step; each expression is evaluated left to right as
// written (the library is built with floating-point contraction off).
he_status plan_lr_step(const u64 *q, int n_q, int level, double s_z, double s_w, const double coef[4],
                       double eta_over_n, double w_decay, int layout, he_lr_plan *o)
{
    if (layout != HE_LAYOUT_ROWS && layout != HE_LAYOUT_FEATURES) return HE_EINVAL;
    if (level < 4 || level >= n_q) return HE_ELEVEL;
    if (!(eta_over_n > 0.0) || !(s_z > 0.0) || !(s_w > 0.0) || !(w_decay >= 0.0 && w_decay < 1.0)) return HE_ESCALE;
    std::memset(o, 0, sizeof *o);
    o->level_in = level;
    o->level_out = level - 4;
    o->layout = layout;
    if (layout == HE_LAYOUT_FEATURES) return plan_features(q, level, s_z, s_w, coef, eta_over_n, w_decay, o);
    double T;
    if (!term_scale(coef, q[0], eta_over_n, 0.0, &T)) return HE_ESCALE;
    const double ql = (double)q[level], ql1 = (double)q[level - 1], ql2 = (double)q[level - 2],
                 ql3 = (double)q[level - 3];
    o->s1 = s_z * s_w / ql;
    o->s_mask = ql2 * ql1 / o->s1;
    o->s_m = o->s1 * o->s_mask / ql1;
    o->s_a = o->s_m * o->s_m / ql2;
    o->t = T;
    o->s_z3 = T * ql3 / o->s_a * ql2 / o->s_m;
    double k3 = coef[3] * o->s_z3 * ql1 / s_z;
    o->s_b3 = o->s_m * o->s_z3 / ql2;
    o->s_c = o->s_a * o->s_b3 / ql3;
    o->s_z1 = o->s_c * ql3 / o->s_m;
    double k1 = coef[1] * o->s_z1 * ql2 / s_z;
    o->s_b1 = o->s_m * o->s_z1;
    double kb1 = 0.0;
    double k0 = coef[0] * o->s_c * ql3 / s_z;
    o->s_z2 = o->s_c * ql3 / o->s_a;
    double k2 = coef[2] * o->s_z2 * ql2 / s_z;
    o->s_g = o->s_c / eta_over_n;
    o->s_gsum = o->s_g;
    double kw = (1.0 - w_decay) * o->s_g * ql3 / s_w;
    return finish_plan(k0, k1, k2, k3, kb1, kw, o);
}

// Encrypted inference with the polynomial: the margins u (level l-1, scale
// s_u = s_z s_w / q_l) go through p(u) = a0 + a1 u + a2 u^2 + a3 u^3 as
//   U2 = RS(relin(u u))                 level l-2, scale s_u2
//   H  = RS(k3 u) + k2c                 level l-2, declared s_h
//   P  = RS(relin(H U2)) + RS(k1 u) + k0c   level l-3, declared s_p = s_u
// with the integers chosen so that every term carries s_p.  Each expression is
// evaluated left to right as written.
he_status plan_lr_infer(const u64 *q, int n_q, int level, double s_z, double s_w, const double coef[4],
                        he_infer_plan *o)
{
    if (level < 3 || level >= n_q) return HE_ELEVEL;
    if (!(s_z > 0.0) || !(s_w > 0.0)) return HE_ESCALE;
    std::memset(o, 0, sizeof *o);
    o->level_in = level;
    o->level_out = level - 3;
    const double ql = (double)q[level], q1 = (double)q[level - 1], q2 = (double)q[level - 2];
    o->s_u = s_z * s_w / ql;
    o->s_u2 = o->s_u * o->s_u / q1;
    o->s_p = o->s_u;
    o->s_h = o->s_p * q2 / o->s_u2;
    const double k3 = coef[3] * o->s_h * q1 / o->s_u;
    const double k2c = coef[2] * o->s_h;
    const double k1 = coef[1] * o->s_p * q2 / o->s_u;
    const double k0c = coef[0] * o->s_p;
    const double kmax = 4.611686018427388e18;  // 2^62
    for (double k : {k3, k2c, k1, k0c})
        if (!(std::fabs(k) < kmax)) return HE_ESCALE;
    o->k3 = std::llround(k3);
    o->k2c = std::llround(k2c);
    o->k1 = std::llround(k1);
    o->k0c = std::llround(k0c);
    return HE_OK;
}

}  // namespace hehost
