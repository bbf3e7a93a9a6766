// Host check of the FP64 fast basis conversion used by the ModUp and ModDown
// kernels: for every target p below 2^46 that the rule admits, the lazy FP64
// sum of the (whole or split) source products minus the centring term reduces
// to the same canonical residue as exact 128-bit arithmetic.  Sources and
// targets are prime lists on the command line; random and edge residues
// (0, q/2, q/2 + 1, q - 1).  The admission rule restates the one in the
// library (conv_split_bits, conv_whole, conv_fp_ok).
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
typedef uint64_t u64;
typedef unsigned __int128 u128;
static int bits(u64 x) { return 64 - __builtin_clzll(x); }
static int split_bits(int ki) { return (ki + 1) / 2; }
static int whole(int ki, int kp) { return ki <= kp + 4; }
static int fp_ok(int kmax, int kp) { return kp <= 46 && split_bits(kmax) <= kp + 4; }
static double lazy(double a, double w, double q, double qinv) {
    double hi = a * w; double lo = fma(a, w, -hi); double qt = floor(hi * qinv); return fma(-qt, q, hi) + lo;
}
static double reduce_d(double x, double q, double qinv) {
    double qt = floor(x * qinv); double r = fma(-qt, q, x); r = r < 0.0 ? r + q : r; return r >= q ? r - q : r;
}
static u64 s_state = 88172645463325252ull;
static u64 rnd(void) { s_state ^= s_state << 13; s_state ^= s_state >> 7; s_state ^= s_state << 17; return s_state; }
static u64 mulmod(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
int main(int argc, char **argv) {
    // argv: primes of the sources (comma list), then target primes
    int ns = 0, nt = 0; u64 src[16], tgt[64];
    char *p = argv[1];
    while (*p) { src[ns++] = strtoull(p, &p, 10); if (*p == ',') ++p; }
    p = argv[2];
    while (*p) { tgt[nt++] = strtoull(p, &p, 10); if (*p == ',') ++p; }
    long trials = atol(argv[3]);
    int kmax = 0; for (int i = 0; i < ns; ++i) if (bits(src[i]) > kmax) kmax = bits(src[i]);
    long checked = 0, bad = 0, skipped = 0;
    for (int t = 0; t < nt; ++t) {
        u64 pt = tgt[t]; int kp = bits(pt);
        if (!fp_ok(kmax, kp)) { ++skipped; continue; }
        double pd = (double)pt, pinv = 1.0 / pd;
        u64 c[16], ch[16], Qd = 1; int sh[16];
        for (int i = 0; i < ns; ++i) {
            c[i] = rnd() % pt;  // any constants below p (the bounds do not depend on their values)
            if (t % 3 == 0) c[i] = pt - 1 - (rnd() % 4);
            int S = split_bits(bits(src[i]));
            ch[i] = mulmod(c[i], ((u128)1 << S) % pt, pt);
            sh[i] = whole(bits(src[i]), kp) ? 0 : S;
            Qd = mulmod(Qd, src[i] % pt, pt);
        }
        for (long r = 0; r < trials; ++r) {
            u64 v[16];
            for (int i = 0; i < ns; ++i) {
                u64 m = rnd() % 6;
                v[i] = m == 0 ? src[i] - 1 : m == 1 ? src[i] / 2 : m == 2 ? src[i] / 2 + 1 : m == 3 ? 0 : rnd() % src[i];
            }
            // exact
            u128 acc = 0; u64 cnt = 0;
            for (int i = 0; i < ns; ++i) { acc += (u128)v[i] * c[i]; cnt += v[i] > src[i] / 2; }
            u64 ex = (u64)(acc % pt); u64 sub = mulmod(cnt, Qd, pt); ex = ex >= sub ? ex - sub : ex + pt - sub;
            // fp64
            double s = 0.0, cn = 0.0;
            for (int i = 0; i < ns; ++i) {
                cn += v[i] > src[i] / 2 ? 1.0 : 0.0;
                if (sh[i] == 0) s += lazy((double)v[i], (double)c[i], pd, pinv);
                else { s += lazy((double)(v[i] >> sh[i]), (double)ch[i], pd, pinv);
                       s += lazy((double)(v[i] & ((1ull << sh[i]) - 1)), (double)c[i], pd, pinv); }
            }
            double rr = reduce_d(fma(-cn, (double)Qd, s), pd, pinv);
            ++checked;
            if (!(rr >= 0.0 && rr < pd) || (u64)rr != ex) { if (bad < 5) printf("BAD t=%d r=%ld %llu vs %llu\n", t, r, (unsigned long long)rr, (unsigned long long)ex); ++bad; }
        }
    }
    printf("sources %d targets %d (fp %d) checked %ld bad %ld\n", ns, nt, nt - (int)skipped, checked, bad);
    return bad != 0;
}
