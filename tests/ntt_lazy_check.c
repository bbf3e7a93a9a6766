// Host check of the lazy FP64 NTT arithmetic the GPU transforms use for
// primes below 2^46 (forward) and 2^42 (inverse).  It restates the rule, not
// the kernels: the lazy product r = fma(-floor(hi / q), q, hi) + lo of an
// integer-valued a and a twiddle w < q (hi = a w rounded, lo its exact
// remainder), forward butterflies x +- r with no corrections, inverse
// butterflies x + y and lazy((x - y) w), one reduction at the end of a pass.
// Claims checked for each prime given on the command line:
//   1. at the range extremes of every forward stage s (inputs in
//      [-2(s-1)q, (2s-1)q]) and every inverse stage (|x| <= 2^(s-1) q), with
//      extreme twiddles: r lies in (-q, 2q), r = a w (mod q) exactly, and the
//      butterfly outputs stay in the next stage's range;
//   2. the pass-boundary intermediate (8 forward stages, |v| <= 17q) round
//      trips exactly through the signed 51-bit integer conversion;
//   3. a whole 2^16-point forward transform (16 stages; the ranges tracked
//      stage by stage) and inverse transform (two passes of 8 stages, each
//      reduced) on structured worst-case and random inputs equal the exact
//      128-bit transform residue for residue.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;
typedef __int128 i128;

static double lazy(double a, double w, double q, double qinv)
{
    double hi = a * w;
    double lo = fma(a, w, -hi);
    double qt = floor(hi * qinv);
    return fma(-qt, q, hi) + lo;
}
static double reduce_d(double x, double q, double qinv)
{
    double qt = floor(x * qinv);
    double r = fma(-qt, q, x);
    r = r < 0.0 ? r + q : r;
    return r >= q ? r - q : r;
}
static double d_from_s51(u64 v)
{
    u64 b = v + 0x4338000000000000ull;
    double d;
    memcpy(&d, &b, 8);
    return d - 6755399441055744.0;
}
static u64 s51_from_d(double x)
{
    double y = x + 6755399441055744.0;
    u64 b;
    memcpy(&b, &y, 8);
    return b - 0x4338000000000000ull;
}
static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
static u64 powmod(u64 b, u64 e, u64 q)
{
    u64 r = 1;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}
static u64 st = 0x9E3779B97F4A7C15ull;
static u64 rnd(void)
{
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
}
static i64 smodq(i128 v, u64 q)
{
    i128 r = v % (i128)q;
    return (i64)(r < 0 ? r + q : r);
}
static long bad = 0;
#define CHECK(c, ...)                        \
    do {                                     \
        if (!(c)) {                          \
            if (bad < 8) printf(__VA_ARGS__); \
            ++bad;                           \
        }                                    \
    } while (0)

// 1. operation extremes
static void check_ops(u64 q)
{
    const double qd = (double)q, qinv = 1.0 / qd;
    u64 ws[8] = {0, 1, 2, q - 1, q - 2, (q - 1) / 2, (q + 1) / 2, 0};
    for (int s = 1; s <= 16; ++s) {
        const i64 lo = -2LL * (s - 1) * (i64)q, hi = (2LL * (s - 1) + 1) * (i64)q;
        i64 as[10] = {lo, lo + 1, hi - 1, hi, 0, -1, 1, lo / 2, hi / 2, 0};
        for (int ia = 0; ia < 10; ++ia)
            for (int iw = 0; iw < 8 + 64; ++iw) {
                const i64 a = ia < 9 ? as[ia] : lo + (i64)(rnd() % (u64)(hi - lo + 1));
                const u64 w = iw < 7 ? ws[iw] : rnd() % q;
                const double r = lazy((double)a, (double)w, qd, qinv);
                CHECK(r > -qd && r < 2 * qd && r == floor(r), "fwd s=%d: r out of (-q,2q)\n", s);
                CHECK(smodq((i128)(i64)r, q) == smodq((i128)a * w, q), "fwd s=%d: r != a w mod q\n", s);
                // butterflies with x anywhere in the stage range
                const i64 xs[2] = {lo, hi};
                for (int ix = 0; ix < 2; ++ix) {
                    const double x = (double)xs[ix];
                    CHECK(x + r >= -2.0 * s * qd && x + r <= (2.0 * s + 1) * qd, "fwd s=%d: x + r range\n", s);
                    CHECK(x - r >= -2.0 * s * qd && x - r <= (2.0 * s + 1) * qd, "fwd s=%d: x - r range\n", s);
                }
            }
    }
    if (q < (1ull << 42)) {
        for (int s = 1; s <= 8; ++s) {
            const i64 m = (i64)q << (s - 1);  // |x|, |y| <= 2^(s-1) q, so |x - y| <= 2^s q
            i64 as[7] = {2 * m, 2 * m - 1, -2 * m, -2 * m + 1, 0, 1, -1};
            for (int ia = 0; ia < 7 + 64; ++ia)
                for (int iw = 0; iw < 7; ++iw) {
                    const i64 a = ia < 7 ? as[ia] : (i64)(rnd() % (u64)(4 * m + 1)) - 2 * m;
                    const double r = lazy((double)a, (double)ws[iw], (double)q, 1.0 / (double)q);
                    CHECK(r > -(double)q && r < 2.0 * (double)q, "inv s=%d: r range\n", s);
                    CHECK(smodq((i128)(i64)r, q) == smodq((i128)a * ws[iw], q), "inv s=%d: r != a w\n", s);
                }
            CHECK((double)(2 * m) < 9007199254740992.0, "inv s=%d: sum not exact\n", s);
        }
    }
    // 2. the signed intermediate between the forward passes
    for (i64 v = -16 * (i64)q; v <= 17 * (i64)q; v += (i64)(q / 3) + 1) {
        const i64 vs[3] = {v, -16 * (i64)q, 17 * (i64)q};
        for (int k = 0; k < 3; ++k) {
            u64 bits = s51_from_d((double)vs[k]);
            CHECK((i64)bits == vs[k] && d_from_s51(bits) == (double)vs[k], "s51 round trip %lld\n", (long long)vs[k]);
        }
    }
}

static int brev(int x, int lg)
{
    int r = 0;
    for (int i = 0; i < lg; ++i) r |= ((x >> i) & 1) << (lg - 1 - i);
    return r;
}

// 3. whole transforms: forward CT with twiddles psi^brev(m + i), output in
// bit-reversed order; inverse GS with psi^-brev, two passes of 8 stages
static void check_transforms(u64 q, int lg)
{
    const int N = 1 << lg;
    const double qd = (double)q, qinv = 1.0 / qd;
    // psi: a primitive 2N-th root (q = 1 mod 2N)
    u64 psi = 0;
    for (u64 x = 2;; ++x) {
        u64 y = powmod(x, (q - 1) / (2 * (u64)N), q);
        if (powmod(y, N, q) == q - 1) { psi = y; break; }
    }
    const u64 ipsi = powmod(psi, q - 2, q);
    u64 *tw = malloc(sizeof(u64) * N), *itw = malloc(sizeof(u64) * N);
    for (int k = 0; k < N; ++k) {
        tw[k] = powmod(psi, (u64)brev(k, lg), q);
        itw[k] = powmod(ipsi, (u64)brev(k, lg), q);
    }
    u64 *a = malloc(sizeof(u64) * N), *ex = malloc(sizeof(u64) * N);
    double *v = malloc(sizeof(double) * N);
    for (int pattern = 0; pattern < 6; ++pattern) {
        for (int i = 0; i < N; ++i) {
            switch (pattern) {
            case 0: a[i] = q - 1; break;
            case 1: a[i] = (i & 1) ? q - 1 : 0; break;
            case 2: a[i] = i == 0 ? q - 1 : 0; break;
            case 3: a[i] = (i < N / 2) ? q - 1 : (q - 1) / 2; break;
            case 4: a[i] = (rnd() & 1) ? q - 1 : (q + 1) / 2; break;
            default: a[i] = rnd() % q;
            }
            ex[i] = a[i];
            v[i] = (double)a[i];
        }
        // forward: exact and lazy side by side, ranges tracked per stage
        for (int m = 1, s = 1; m < N; m <<= 1, ++s) {
            const int t = N / (2 * m);
            double mx = 0, mn = 0;
            for (int i = 0; i < m; ++i) {
                const u64 w = tw[m + i];
                for (int j = 2 * i * t; j < 2 * i * t + t; ++j) {
                    u64 u = ex[j], y = mulmod(ex[j + t], w, q);
                    ex[j] = (u + y) % q;
                    ex[j + t] = (u + q - y) % q;
                    const double r = lazy(v[j + t], (double)w, qd, qinv);
                    const double x = v[j];
                    v[j] = x + r;
                    v[j + t] = x - r;
                    mx = fmax(mx, fmax(v[j], v[j + t]));
                    mn = fmin(mn, fmin(v[j], v[j + t]));
                }
            }
            CHECK(mx <= (2.0 * s + 1) * qd && mn >= -2.0 * s * qd, "fwd pattern %d stage %d range\n", pattern, s);
            if (s == lg / 2)  // the pass boundary: stored as a signed integer
                for (int i = 0; i < N; ++i) v[i] = d_from_s51(s51_from_d(v[i]));
        }
        for (int i = 0; i < N; ++i)
            CHECK((u64)reduce_d(v[i], qd, qinv) == ex[i], "fwd pattern %d: residue %d\n", pattern, i);
        if (q >= (1ull << 42)) continue;
        // inverse on the (reduced) forward output: two passes, each reduced at its end
        for (int i = 0; i < N; ++i) v[i] = (double)ex[i];
        for (int m = N / 2, s = 1; m >= 1; m >>= 1, ++s) {
            const int t = N / (2 * m);
            for (int i = 0; i < m; ++i) {
                const u64 w = itw[m + i];
                for (int j = 2 * i * t; j < 2 * i * t + t; ++j) {
                    u64 x = ex[j], y = ex[j + t];
                    ex[j] = (x + y) % q;
                    ex[j + t] = mulmod((x + q - y) % q, w, q);
                    const double xd = v[j], yd = v[j + t];
                    v[j] = xd + yd;
                    v[j + t] = lazy(xd - yd, (double)w, qd, qinv);
                }
            }
            const int in_pass = (s - 1) % (lg / 2) + 1;
            double mx = 0;
            for (int i = 0; i < N; ++i) mx = fmax(mx, fabs(v[i]));
            CHECK(mx <= ldexp(qd, in_pass), "inv pattern %d stage %d range\n", pattern, s);
            if (in_pass == lg / 2)
                for (int i = 0; i < N; ++i) v[i] = reduce_d(v[i], qd, qinv);
        }
        for (int i = 0; i < N; ++i) CHECK((u64)v[i] == ex[i], "inv pattern %d: residue %d\n", pattern, i);
    }
    free(tw); free(itw); free(a); free(ex); free(v);
}

int main(int argc, char **argv)
{
    const int lg = argc > 2 ? atoi(argv[2]) : 16;
    int n = 0;
    for (char *p = argv[1]; *p;) {
        u64 q = strtoull(p, &p, 10);
        if (*p == ',') ++p;
        if (q >= (1ull << 46)) continue;
        check_ops(q);
        check_transforms(q, lg);
        ++n;
    }
    printf("primes %d bad %ld\n", n, bad);
    return bad != 0 || n == 0;
}
