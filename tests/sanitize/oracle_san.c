/*
 * Driver of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (CPU only).  The oracle source is compiled into this translation unit; every
 * exported routine runs on a small ring (N = 2^6 .. 2^8, several prime counts
 * and digit widths, every level and digit), including the edge cases of its
 * samplers and conversions, and a few sanity results are checked so that the
 * calls do real work.  Exit status 0 with "ok" on success; the sanitizers
 * abort with a report on the first error.
 */
#include <stdio.h>

#include "../../oracle/he_oracle.c"

#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            exit(1);                                                   \
        }                                                              \
    } while (0)

static void make_params(orc_params *P, int logN, int nq, int nk, int alpha, int log_delta)
{
    memset(P, 0, sizeof *P);
    P->logN = logN;
    P->nq = nq;
    P->nk = nk;
    P->alpha = alpha;
    CHECK(orc_gen_primes(nq, nk, log_delta, P->q) == 0);
    for (int i = 0; i < nq + nk; i++) P->psi[i] = orc_find_psi(P->q[i], logN);
}

static i64 centred(u64 v, u64 q) { return v > q / 2 ? -(i64)(q - v) : (i64)v; }

/* max |dec - m| over the coefficients, on q_0 */
static i64 dec_err(const orc_params *P, int level, const u64 *ct, const i64 *s, const i64 *m)
{
    u64 N = (u64)1 << P->logN;
    u64 *d = malloc((size_t)(level + 1) * N * 8);
    orc_decrypt(P, level, ct, s, d);
    i64 worst = 0;
    for (u64 x = 0; x < N; x++) {
        i64 e = centred(d[x], P->q[0]) - m[x];
        if (e < 0) e = -e;
        if (e > worst) worst = e;
    }
    free(d);
    return worst;
}

static void ring(int logN, int nq, int nk, int alpha, int log_delta)
{
    orc_params P;
    make_params(&P, logN, nq, nk, alpha, log_delta);
    u64 N = (u64)1 << logN;
    int nfull = nq + nk, L = nq - 1, beta = orc_ndigits(&P, L);

    /* NTT round trip and product against the schoolbook negacyclic product */
    u64 *a = malloc(N * 8), *b = malloc(N * 8), *c = malloc(N * 8), *r = malloc(N * 8);
    orc_sample_uniform(7, 6, 1, 0, P.q[1], logN, a);
    orc_sample_uniform(7, 6, 2, 0, P.q[1], logN, b);
    memcpy(c, a, N * 8);
    orc_ntt_fwd(c, logN, P.q[1], P.psi[1]);
    orc_ntt_inv(c, logN, P.q[1], P.psi[1]);
    CHECK(memcmp(a, c, N * 8) == 0);
    orc_polymul(a, b, c, logN, P.q[1], P.psi[1]);
    for (u64 k = 0; k < N; k++) {
        u64 acc = 0;
        for (u64 i = 0; i < N; i++) {
            u64 j = (k + N - i) % N, t = mulmod(a[i], b[j], P.q[1]);
            acc = (i <= k) ? addmod(acc, t, P.q[1]) : submod(acc, t, P.q[1]);
        }
        r[k] = acc;
    }
    CHECK(memcmp(r, c, N * 8) == 0);

    /* samplers: every stream type, edge weights */
    i64 *s = malloc(N * 8), *e = malloc(N * 8), *m = malloc(N * 8), *m2 = malloc(N * 8);
    orc_sample_hwt(3, logN, 0, s);
    orc_sample_hwt(3, logN, (int)N, s);
    for (u64 x = 0; x < N; x++) CHECK(s[x] == 1 || s[x] == -1);
    orc_sample_ternary(3, 8, 0, 0, logN, e);
    orc_sample_cbd(3, 7, 0, 0, logN, e);
    for (u64 x = 0; x < N; x++) CHECK(e[x] >= -21 && e[x] <= 21);
    u64 w[40];
    orc_prng_words(5, 1, 2, 3, 13, 40, w);
    orc_keygen_secret(&P, 11, (int)(N / 4), s);

    /* keys: s^2 evaluation key, public key */
    u64 *sp = malloc((size_t)nfull * N * 8);
    orc_secret_square(&P, s, sp);
    size_t evk_sz = (size_t)beta * 2 * nfull * N;
    u64 *evk = malloc(evk_sz * 8 * 2);
    orc_gen_evk(&P, s, sp, 11, 0, evk);
    orc_gen_evk(&P, s, sp, 11, 2, evk + evk_sz);
    u64 *pk = malloc((size_t)2 * nq * N * 8);
    orc_gen_pk(&P, s, 11, pk);

    /* encryption at every level: sk, seeded sk, pk; decryption bounds */
    for (u64 x = 0; x < N; x++) {
        m[x] = (i64)(x * 37 % 1001) - 500;
        m2[x] = (i64)(x * 11 % 7) - 3;
    }
    size_t ct_sz = (size_t)2 * nq * N;
    u64 *ct = malloc(ct_sz * 8), *ct2 = malloc(ct_sz * 8), *d3 = malloc((size_t)3 * nq * N * 8);
    u64 *ks = malloc(ct_sz * 8), *o = malloc(ct_sz * 8);
    for (int lv = 0; lv <= L; lv++) {
        orc_encrypt_sk(&P, lv, m, s, 13, (u32)lv, ct);
        CHECK(dec_err(&P, lv, ct, s, m) <= 21);
        orc_encrypt_sk_seeded(&P, lv, m, s, 13, (u32)lv, ct);
        CHECK(dec_err(&P, lv, ct, s, m) <= 21);
        orc_encrypt_pk(&P, lv, m, pk, 13, (u32)lv, ct);
        CHECK(dec_err(&P, lv, ct, s, m) <= 21 * (2 * (i64)N + 2));
    }

    /* per level: tensor, key switch (single and summed), ModUp of every digit,
     * ModDown, rescale of 2 and 3 components, automorphisms, elementwise ops */
    int idx[ORC_MAXP];
    for (int i = 0; i < nfull; i++) idx[i] = i;
    u64 *ext = malloc((size_t)(nq + nk) * N * 8), *dn = malloc((size_t)nq * N * 8);
    u64 *acc = malloc((size_t)2 * (nq + nk) * N * 8);
    for (int lv = 1; lv <= L; lv++) {
        size_t n1 = (size_t)(lv + 1) * N;
        orc_encrypt_sk(&P, lv, m, s, 17, 1, ct);
        orc_encrypt_sk(&P, lv, m2, s, 17, 2, ct2);
        orc_tensor(&P, lv, ct, ct2, d3);
        orc_keyswitch(&P, lv, d3 + 2 * n1, evk, ks);
        orc_add(&P, lv + 1, ks, d3, o);
        orc_add(&P, lv + 1, ks + n1, d3 + n1, o + n1);
        orc_keyswitch_sum(&P, lv, 2, d3 + n1, evk, ks);
        for (int j = 0; j < orc_ndigits(&P, lv); j++) orc_modup(&P, lv, j, ct, ext);
        for (size_t t = 0; t < (size_t)(lv + 1 + nk); t++)
            for (u64 x = 0; x < N; x++) acc[t * N + x] = (t * 31 + x * 7) % basis_prime(&P, lv, (int)t, NULL);
        orc_moddown(&P, lv, acc, dn);
        orc_rescale_n(&P, lv, 3, d3, d3);
        orc_rescale(&P, lv, ct, o);
        orc_automorph(&P, lv + 1, idx, 5, ct, o);
        orc_automorph(&P, lv + 1, idx, 2 * N - 1, ct, o);
        orc_mul_int(&P, lv + 1, ct, -(i64)3, o);
        orc_mul_plain(&P, lv + 1, ct, m2, o);
        orc_int_to_rns(&P, m, 0, lv + 1, o);
    }
    /* the uncentred conversion switch and back */
    orc_set_conv_centring(0);
    orc_modup(&P, L, 0, ct, ext);
    orc_set_conv_centring(1);

    /* the tensor_n degree forms */
    orc_encrypt_sk(&P, L, m, s, 19, 1, ct);
    orc_tensor_n(&P, L, 2, ct, 2, ct, d3);

    free(a); free(b); free(c); free(r); free(s); free(e); free(m); free(m2); free(sp); free(evk); free(pk);
    free(ct); free(ct2); free(d3); free(ks); free(o); free(ext); free(dn); free(acc);
}

int main(void)
{
    /* scalar edges */
    CHECK(!orc_is_prime(0) && !orc_is_prime(1) && orc_is_prime(2) && orc_is_prime(18446744073709551557ull));
    CHECK(orc_mulmod(~0ull - 59, ~0ull - 59, 18446744073709551557ull) == 1);
    u32 key[8] = {0}, nonce[3] = {0}, out[16];
    orc_chacha20_block(key, 0xffffffffu, nonce, out);
    orc_set_threads(2);
#ifdef PLANT_OVERREAD
    { /* the test's planted fault: one read past a buffer, which ASan must report */
        volatile u64 *p = malloc(8 * 8);
        u64 v = p[8];
        free((void *)p);
        printf("%llu\n", (unsigned long long)v);
    }
#endif
    ring(6, 3, 1, 1, 30);
    ring(7, 5, 2, 2, 40);
    ring(8, 7, 3, 3, 40);
    ring(6, 4, 2, 4, 40);
    printf("ok\n");
    return 0;
}
