/*
 * he_oracle.c -- plain, slow CPU reference for the RNS-CKKS arithmetic of the
 * encrypted logistic-regression gradient step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file; only tests, the smoke check and the bench's CPU-baseline leg do.
 * It shares no code, header, table or constant generator with the GPU library.
 *
 * Every modular product is (unsigned __int128)a*b % q.  Every polynomial is kept
 * in COEFFICIENT form (residues in [0,q)); a negacyclic product is computed as
 * textbook NTT -> pointwise -> inverse NTT for that one product.  There is no
 * lazy reduction, no Shoup/Barrett, no fusion.
 *
 * The paper (Li & Huang, KDD'20) builds on the approximate-number scheme HEAAN
 * (Sec. 3, "Preliminary": encode/decode, encrypt/decrypt, add, multiply and
 * the rounding ("scaling") operation) and gives no parameters; the RNS form,
 * hybrid key switching, prime rule, sampler and PRNG are the readings listed in
 * the design notes and implemented here from their textbook definitions.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;

#define ORC_MAXP 64

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic                                           */
/* ------------------------------------------------------------------ */
static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }
static u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : (u64)(((u128)a + q - b) % q); }
static u64 powmod(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}
/* q prime: inverse by Fermat's little theorem */
static u64 invmod(u64 a, u64 q) { return powmod(a % q, q - 2, q); }
/* signed integer -> residue in [0,q) */
static u64 smod(i64 v, u64 q)
{
    if (v >= 0) return (u64)v % q;
    u64 m = (u64)(-(v + 1)) + 1; /* |v| without overflow at INT64_MIN */
    m %= q;
    return m == 0 ? 0 : q - m;
}

u64 orc_mulmod(u64 a, u64 b, u64 q) { return mulmod(a, b, q); }

/* threads of the oracle's parallel loops (its timing as a CPU baseline) */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
u64 orc_powmod(u64 b, u64 e, u64 q) { return powmod(b, e, q); }

/* deterministic Miller-Rabin for n < 2^64 (the first 12 primes as bases) */
int orc_is_prime(u64 n)
{
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        u64 x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) {
            x = mulmod(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

/*
 * Prime chain (reading; the paper fixes none).  All primes are 1 mod 2^17,
 * so one chain serves every ring degree N <= 2^16.
 *   out[nq .. nq+nk)  special primes: the nk largest such primes below 2^60
 *   out[0]            q_0 : the largest such prime below 2^min(60, log_delta+20)
 *                     that is not a special prime (20 bits of headroom over the
 *                     scale; keeps q_0 well below P when a digit is one prime)
 *   out[1 .. nq)      q_1..q_{nq-1}: the nq-1 such primes closest to 2^log_delta,
 *                     ordered by increasing distance (ties: smaller first)
 * Returns 0 on success.
 */
int orc_gen_primes(int nq, int nk, int log_delta, u64 *out)
{
    const u64 M = (u64)1 << 17;
    if (nq < 1 || nk < 0 || nq + nk > ORC_MAXP || log_delta < 18 || log_delta > 58) return -1;
    /* special primes: the nk largest below 2^60, descending */
    u64 c = (((u64)1 << 60) - 1) / M * M + 1; /* largest 1 mod M below 2^60 */
    int got = 0;
    while (got < nk) {
        if (orc_is_prime(c)) out[nq + got++] = c;
        c -= M;
    }
    /* q_0: the largest below 2^min(60, log_delta+20) that is not a special prime */
    int b0 = log_delta + 20 < 60 ? log_delta + 20 : 60;
    c = ((((u64)1 << b0) - 1) / M) * M + 1;
    for (;; c -= M) {
        int taken = 0;
        for (int i = 0; i < nk; i++) taken |= (out[nq + i] == c);
        if (!taken && orc_is_prime(c)) break;
    }
    out[0] = c;
    /* scale primes around 2^log_delta: walk outward, below and above */
    u64 D = (u64)1 << log_delta;
    u64 lo = D / M * M + 1;  /* candidates <= D+1 */
    if (lo > D) lo -= M;
    u64 hi = lo + M;         /* candidates > D */
    int need = nq - 1;
    int k = 1;
    while (need > 0) {
        /* next candidate on each side that is prime */
        while (!orc_is_prime(lo)) lo -= M;
        while (!orc_is_prime(hi)) hi += M;
        u64 dl = D - lo, dh = hi - D;
        if (dl <= dh) { out[k++] = lo; lo -= M; }
        else          { out[k++] = hi; hi += M; }
        need--;
    }
    return 0;
}

/* psi: for x = 2,3,...: y = x^((q-1)/2N); the first y with y^N = -1 is taken. */
u64 orc_find_psi(u64 q, int logN)
{
    u64 N = (u64)1 << logN;
    for (u64 x = 2;; x++) {
        u64 y = powmod(x, (q - 1) / (2 * N), q);
        if (powmod(y, N, q) == q - 1) return y;
    }
}

/* ------------------------------------------------------------------ */
/* textbook negacyclic NTT, natural order                               */
/*   forward: A_k = sum_i a_i psi^{(2k+1) i}                            */
/*   inverse: a_i = N^{-1} psi^{-i} sum_k A_k psi^{-2ik}                */
/* implemented as (twist by psi^i) + iterative radix-2 cyclic DFT with   */
/* omega = psi^2 (bit-reversal permutation, then butterflies).          */
/* ------------------------------------------------------------------ */
static void bitrev_perm(u64 *a, u64 N)
{
    for (u64 i = 1, j = 0; i < N; i++) {
        u64 bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
}
static void cyclic_dft(u64 *a, u64 N, u64 omega, u64 q)
{
    bitrev_perm(a, N);
    for (u64 len = 2; len <= N; len <<= 1) {
        u64 wl = powmod(omega, N / len, q);
        for (u64 i = 0; i < N; i += len) {
            u64 w = 1;
            for (u64 j = 0; j < len / 2; j++) {
                u64 u = a[i + j];
                u64 v = mulmod(a[i + j + len / 2], w, q);
                a[i + j] = addmod(u, v, q);
                a[i + j + len / 2] = submod(u, v, q);
                w = mulmod(w, wl, q);
            }
        }
    }
}
void orc_ntt_fwd(u64 *a, int logN, u64 q, u64 psi)
{
    u64 N = (u64)1 << logN;
    u64 p = 1;
    for (u64 i = 0; i < N; i++) { a[i] = mulmod(a[i], p, q); p = mulmod(p, psi, q); }
    cyclic_dft(a, N, mulmod(psi, psi, q), q);
}
void orc_ntt_inv(u64 *a, int logN, u64 q, u64 psi)
{
    u64 N = (u64)1 << logN;
    u64 psi_inv = invmod(psi, q);
    cyclic_dft(a, N, mulmod(psi_inv, psi_inv, q), q);
    u64 ninv = invmod(N % q, q);
    u64 p = ninv;
    for (u64 i = 0; i < N; i++) { a[i] = mulmod(a[i], p, q); p = mulmod(p, psi_inv, q); }
}
/* c = a * b mod (X^N + 1, q); c may alias a or b */
void orc_polymul(const u64 *a, const u64 *b, u64 *c, int logN, u64 q, u64 psi)
{
    u64 N = (u64)1 << logN;
    u64 *ta = (u64 *)malloc(N * 8), *tb = (u64 *)malloc(N * 8);
    memcpy(ta, a, N * 8);
    memcpy(tb, b, N * 8);
    orc_ntt_fwd(ta, logN, q, psi);
    orc_ntt_fwd(tb, logN, q, psi);
    for (u64 i = 0; i < N; i++) ta[i] = mulmod(ta[i], tb[i], q);
    orc_ntt_inv(ta, logN, q, psi);
    memcpy(c, ta, N * 8);
    free(ta);
    free(tb);
}

/* ------------------------------------------------------------------ */
/* ChaCha20 block function (RFC 8439, Sec. 2.3)                         */
/* ------------------------------------------------------------------ */
static u32 rotl32(u32 x, int n) { return (x << n) | (x >> (32 - n)); }
#define QR(a, b, c, d)                      \
    a += b; d ^= a; d = rotl32(d, 16);      \
    c += d; b ^= c; b = rotl32(b, 12);      \
    a += b; d ^= a; d = rotl32(d, 8);       \
    c += d; b ^= c; b = rotl32(b, 7);
void orc_chacha20_block(const u32 key[8], u32 counter, const u32 nonce[3], u32 out[16])
{
    u32 st[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                  key[0], key[1], key[2], key[3], key[4], key[5], key[6], key[7],
                  counter, nonce[0], nonce[1], nonce[2]};
    u32 x[16];
    memcpy(x, st, sizeof x);
    for (int i = 0; i < 10; i++) {
        QR(x[0], x[4], x[8], x[12]);
        QR(x[1], x[5], x[9], x[13]);
        QR(x[2], x[6], x[10], x[14]);
        QR(x[3], x[7], x[11], x[15]);
        QR(x[0], x[5], x[10], x[15]);
        QR(x[1], x[6], x[11], x[12]);
        QR(x[2], x[7], x[8], x[13]);
        QR(x[3], x[4], x[9], x[14]);
    }
    for (int i = 0; i < 16; i++) out[i] = x[i] + st[i];
}

/*
 * Word stream (reading): key = the 64-bit seed in key words 0 (low) and 1
 * (high), all other key words zero; nonce = (type, index, component); the
 * block counter is the block number.  64-bit word t of block b is
 * out[2t] | out[2t+1] << 32, and it is word 8b+t of the stream.
 */
void orc_prng_words(u64 seed, u32 type, u32 index, u32 comp, u64 first, u64 count, u64 *out)
{
    u32 key[8] = {(u32)seed, (u32)(seed >> 32), 0, 0, 0, 0, 0, 0};
    u32 nonce[3] = {type, index, comp};
    u32 blk[16];
    u64 cur_block = ~(u64)0;
    for (u64 w = first; w < first + count; w++) {
        u64 b = w / 8;
        if (b != cur_block) {
            orc_chacha20_block(key, (u32)b, nonce, blk);
            cur_block = b;
        }
        int t = (int)(w % 8);
        out[w - first] = (u64)blk[2 * t] | ((u64)blk[2 * t + 1] << 32);
    }
}

/* stream types (reading) */
enum { ST_SECRET = 1, ST_PK_A = 2, ST_PK_E = 3, ST_EVK_A = 4, ST_EVK_E = 5,
       ST_ENC_A = 6, ST_ENC_E0 = 7, ST_ENC_V = 8, ST_ENC_E1 = 9, ST_SEED_A = 10 };

/* uniform residue mod q: coefficient x takes words 2x (high) and 2x+1 (low) */
void orc_sample_uniform(u64 seed, u32 type, u32 index, u32 comp, u64 q, int logN, u64 *out)
{
    u64 N = (u64)1 << logN;
    u64 *w = (u64 *)malloc(2 * N * 8);
    orc_prng_words(seed, type, index, comp, 0, 2 * N, w);
    for (u64 x = 0; x < N; x++) {
        u128 v = ((u128)w[2 * x] << 64) | w[2 * x + 1];
        out[x] = (u64)(v % q);
    }
    free(w);
}
/* centered binomial, 21 coin pairs: popcount(w & (2^21-1)) - popcount((w>>21) & (2^21-1)) */
void orc_sample_cbd(u64 seed, u32 type, u32 index, u32 comp, int logN, i64 *out)
{
    u64 N = (u64)1 << logN;
    u64 *w = (u64 *)malloc(N * 8);
    orc_prng_words(seed, type, index, comp, 0, N, w);
    for (u64 x = 0; x < N; x++) {
        int a = 0, b = 0;
        for (int k = 0; k < 21; k++) {
            a += (int)((w[x] >> k) & 1);
            b += (int)((w[x] >> (21 + k)) & 1);
        }
        out[x] = a - b;
    }
    free(w);
}
/* ternary secret of Hamming weight h: partial Fisher-Yates over positions;
   step k uses word 2k (offset mod (N-k)) and the low bit of word 2k+1 (sign: 1 -> -1) */
void orc_sample_hwt(u64 seed, int logN, int h, i64 *out)
{
    u64 N = (u64)1 << logN;
    u64 *perm = (u64 *)malloc(N * 8);
    u64 *w = (u64 *)malloc(2 * (u64)h * 8);
    for (u64 i = 0; i < N; i++) { perm[i] = i; out[i] = 0; }
    orc_prng_words(seed, ST_SECRET, 0, 0, 0, 2 * (u64)h, w);
    for (int k = 0; k < h; k++) {
        u64 j = (u64)k + w[2 * k] % (N - (u64)k);
        u64 t = perm[k]; perm[k] = perm[j]; perm[j] = t;
        out[perm[k]] = (w[2 * k + 1] & 1) ? -1 : 1;
    }
    free(perm);
    free(w);
}
/* ternary with P(0)=1/2, P(+-1)=1/4: word x; bit0 = 0 -> 0, else bit1 ? -1 : +1 */
void orc_sample_ternary(u64 seed, u32 type, u32 index, u32 comp, int logN, i64 *out)
{
    u64 N = (u64)1 << logN;
    u64 *w = (u64 *)malloc(N * 8);
    orc_prng_words(seed, type, index, comp, 0, N, w);
    for (u64 x = 0; x < N; x++) out[x] = (w[x] & 1) ? (((w[x] >> 1) & 1) ? -1 : 1) : 0;
    free(w);
}

/* ------------------------------------------------------------------ */
/* RNS-CKKS in coefficient form                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int logN;
    int nq;    /* q_0..q_{nq-1}: ciphertext primes, top level L = nq-1 */
    int nk;    /* special primes p_0..p_{nk-1} */
    int alpha; /* primes per key-switching digit */
    u64 q[ORC_MAXP];   /* q_0..q_{nq-1}, then p_0..p_{nk-1} */
    u64 psi[ORC_MAXP];
} orc_params;

#define LIMB(p, i) ((p) + (size_t)(i) * N)

/* residues of an integer polynomial on primes q[first..first+n) */
void orc_int_to_rns(const orc_params *P, const i64 *m, int first, int n, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    for (int i = 0; i < n; i++)
        for (u64 x = 0; x < N; x++) LIMB(out, i)[x] = smod(m[x], P->q[first + i]);
}

/* limb-wise negacyclic products over primes q[0..n) (same positions) */
static void rns_polymul(const orc_params *P, const u64 *a, const u64 *b, u64 *c, int n)
{
    u64 N = (u64)1 << P->logN;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; i++) orc_polymul(LIMB(a, i), LIMB(b, i), LIMB(c, i), P->logN, P->q[i], P->psi[i]);
}

/* tensor: (x0,x1) x (y0,y1) -> (x0y0, x0y1 + x1y0, x1y1) at level l */
void orc_tensor(const orc_params *P, int level, const u64 *x, const u64 *y, u64 *d)
{
    u64 N = (u64)1 << P->logN;
    int n = level + 1;
    size_t pl = (size_t)n * N;
    const u64 *x0 = x, *x1 = x + pl, *y0 = y, *y1 = y + pl;
    u64 *d0 = d, *d1 = d + pl, *d2 = d + 2 * pl;
    u64 *t = (u64 *)malloc(pl * 8);
    rns_polymul(P, x0, y0, d0, n);
    rns_polymul(P, x0, y1, d1, n);
    rns_polymul(P, x1, y0, t, n);
    rns_polymul(P, x1, y1, d2, n);
    for (int i = 0; i < n; i++)
        for (u64 k = 0; k < N; k++) LIMB(d1, i)[k] = addmod(LIMB(d1, i)[k], LIMB(t, i)[k], P->q[i]);
    free(t);
}

/*
 * tensor of a degree-(nx-1) and a degree-(ny-1) ciphertext at level l (the
 * ciphertext as a polynomial in the secret): d_k = sum_{i+j=k} x_i y_j,
 * k = 0 .. nx+ny-2.  x: [nx][l+1][N], y: [ny][l+1][N], d: [nx+ny-1][l+1][N].
 */
void orc_tensor_n(const orc_params *P, int level, int nx, const u64 *x, int ny, const u64 *y, u64 *d)
{
    u64 N = (u64)1 << P->logN;
    int n = level + 1;
    size_t pl = (size_t)n * N;
    u64 *t = (u64 *)malloc(pl * 8);
    memset(d, 0, (size_t)(nx + ny - 1) * pl * 8);
    for (int i = 0; i < nx; i++)
        for (int j = 0; j < ny; j++) {
            u64 *dk = d + (size_t)(i + j) * pl;
            rns_polymul(P, x + (size_t)i * pl, y + (size_t)j * pl, t, n);
            for (int r = 0; r < n; r++)
                for (u64 k = 0; k < N; k++) LIMB(dk, r)[k] = addmod(LIMB(dk, r)[k], LIMB(t, r)[k], P->q[r]);
        }
    free(t);
}

/*
 * Centring of the fast basis conversion (ModUp and ModDown).  On (the
 * reading used everywhere): each digit y = [x qhat^{-1}]_q enters as its
 * centred representative in (-q/2, q/2).  Off: as its residue in [0, q).  The
 * switch exists only so that a test can plant the uncentred conversion in the
 * oracle and check that the exact pins reject it.
 */
static int conv_centred = 1;
void orc_set_conv_centring(int on) { conv_centred = on != 0; }

/* prime of basis position pos at level l: pos <= l -> q_pos, else special pos-l-1 */
static u64 basis_prime(const orc_params *P, int level, int pos, u64 *psi)
{
    int idx = pos <= level ? pos : P->nq + (pos - level - 1);
    if (psi) *psi = P->psi[idx];
    return P->q[idx];
}

/*
 * ModUp of digit j at level l (approximate fast basis conversion with
 * centered digits): for every basis position t of Q_l u P outside the digit,
 *   ext[t] = sum_{i in D} y_i * (qhat_i mod t)  mod t,
 *   y_i = [d_i * qhat_i^{-1}]_{q_i} taken as its centered representative,
 * qhat_i = prod_{i' in D, i' != i} q_{i'}; positions inside the digit copy d.
 * d: [l+1][N] coefficient form; ext: [l+1+nk][N].
 */
void orc_modup(const orc_params *P, int level, int j, const u64 *d, u64 *ext)
{
    u64 N = (u64)1 << P->logN;
    int lo = j * P->alpha, hi = (j + 1) * P->alpha;
    if (hi > level + 1) hi = level + 1;
    int nb = level + 1 + P->nk;
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < nb; t++) {
        u64 qt = basis_prime(P, level, t, NULL);
        if (t >= lo && t < hi) { memcpy(LIMB(ext, t), LIMB(d, t), N * 8); continue; }
        u64 yinv[ORC_MAXP], qh_t[ORC_MAXP]; /* [qhat_i^{-1}]_{q_i} and qhat_i mod q_t */
        for (int i = lo; i < hi; i++) {
            u64 qi = P->q[i], qhat_i = 1, qhat_t = 1;
            for (int i2 = lo; i2 < hi; i2++)
                if (i2 != i) { qhat_i = mulmod(qhat_i, P->q[i2] % qi, qi); qhat_t = mulmod(qhat_t, P->q[i2] % qt, qt); }
            yinv[i] = invmod(qhat_i, qi);
            qh_t[i] = qhat_t;
        }
        for (u64 x = 0; x < N; x++) {
            u64 acc = 0;
            for (int i = lo; i < hi; i++) {
                u64 qi = P->q[i];
                u64 y = mulmod(LIMB(d, i)[x], yinv[i], qi);
                i64 yc = conv_centred && y > qi / 2 ? -(i64)(qi - y) : (i64)y; /* centered representative */
                acc = addmod(acc, mulmod(smod(yc, qt), qh_t[i], qt), qt);
            }
            LIMB(ext, t)[x] = acc;
        }
    }
}

/*
 * ModDown at level l: c over Q_l u P ([l+1+nk][N], coefficient form) ->
 *   out_i = (c_i - Conv_{P->q_i}(c_P)) * P^{-1} mod q_i,
 *   Conv_{P->q}(v) = sum_p y_p * (phat_p mod q),
 *   y_p = [v_p * phat_p^{-1}]_p taken as its centered representative.
 */
void orc_moddown(const orc_params *P, int level, const u64 *c, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int nk = P->nk;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i <= level; i++) {
        u64 qi = P->q[i];
        u64 Pinv = 1;
        for (int p = 0; p < nk; p++) Pinv = mulmod(Pinv, P->q[P->nq + p] % qi, qi);
        Pinv = invmod(Pinv, qi);
        u64 yinv[ORC_MAXP], ph_i[ORC_MAXP]; /* [phat_p^{-1}]_p and phat_p mod q_i */
        for (int p = 0; p < nk; p++) {
            u64 pp = P->q[P->nq + p], phat_p = 1, phat_i = 1;
            for (int p2 = 0; p2 < nk; p2++)
                if (p2 != p) { phat_p = mulmod(phat_p, P->q[P->nq + p2] % pp, pp); phat_i = mulmod(phat_i, P->q[P->nq + p2] % qi, qi); }
            yinv[p] = invmod(phat_p, pp);
            ph_i[p] = phat_i;
        }
        for (u64 x = 0; x < N; x++) {
            u64 conv = 0;
            for (int p = 0; p < nk; p++) {
                u64 pp = P->q[P->nq + p];
                u64 y = mulmod(LIMB(c, level + 1 + p)[x], yinv[p], pp);
                i64 yc = conv_centred && y > pp / 2 ? -(i64)(pp - y) : (i64)y; /* centered representative */
                conv = addmod(conv, mulmod(smod(yc, qi), ph_i[p], qi), qi);
            }
            LIMB(out, i)[x] = mulmod(submod(LIMB(c, i)[x], conv, qi), Pinv, qi);
        }
    }
}

/* number of key-switching digits at level l */
int orc_ndigits(const orc_params *P, int level) { return (level + 1 + P->alpha - 1) / P->alpha; }

/*
 * Hybrid key switch of d (coefficient form, [l+1][N]) with an evaluation key
 * evk = [beta_top][2][nq+nk][N] (coefficient form, components b then a).
 * out: [2][l+1][N] = ModDown( sum_j ModUp_j(d) * (b_j, a_j) ).
 */
void orc_keyswitch(const orc_params *P, int level, const u64 *d, const u64 *evk, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int nb = level + 1 + P->nk;
    int nfull = P->nq + P->nk;
    int beta = orc_ndigits(P, level);
    size_t ext_sz = (size_t)nb * N;
    u64 *ext = (u64 *)malloc(ext_sz * 8);
    u64 *acc = (u64 *)calloc(2 * ext_sz, 8);
    for (int j = 0; j < beta; j++) {
        orc_modup(P, level, j, d, ext);
        for (int comp = 0; comp < 2; comp++) {
            const u64 *key = evk + ((size_t)j * 2 + comp) * nfull * N;
            u64 *a = acc + comp * ext_sz;
#pragma omp parallel for schedule(dynamic)
            for (int t = 0; t < nb; t++) {
                u64 psi;
                u64 qt = basis_prime(P, level, t, &psi);
                int kpos = t <= level ? t : P->nq + (t - level - 1);
                u64 *prod = (u64 *)malloc(N * 8);
                orc_polymul(LIMB(ext, t), LIMB(key, kpos), prod, P->logN, qt, psi);
                for (u64 x = 0; x < N; x++) LIMB(a, t)[x] = addmod(LIMB(a, t)[x], prod[x], qt);
                free(prod);
            }
        }
    }
    orc_moddown(P, level, acc, out);
    orc_moddown(P, level, acc + ext_sz, out + (size_t)(level + 1) * N);
    free(ext);
    free(acc);
}

/*
 * Sum of n key switches with one ModDown: the inner products of the ModUp of
 * each d_m with its key evk_m are summed in Q_l u P, then the sum is divided
 * by P once.  d: n x [l+1][N] (coefficient form); evk: n x [beta][2][nq+nk][N].
 * For n = 1 this is orc_keyswitch.
 */
void orc_keyswitch_sum(const orc_params *P, int level, int n, const u64 *d, const u64 *evk, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int nb = level + 1 + P->nk;
    int nfull = P->nq + P->nk;
    int beta = orc_ndigits(P, level);
    size_t ext_sz = (size_t)nb * N;
    size_t key_sz = (size_t)orc_ndigits(P, P->nq - 1) * 2 * nfull * N;
    u64 *ext = (u64 *)malloc(ext_sz * 8);
    u64 *acc = (u64 *)calloc(2 * ext_sz, 8);
    for (int m = 0; m < n; m++) {
        const u64 *dm = d + (size_t)m * (level + 1) * N;
        const u64 *km = evk + (size_t)m * key_sz;
        for (int j = 0; j < beta; j++) {
            orc_modup(P, level, j, dm, ext);
            for (int comp = 0; comp < 2; comp++) {
                const u64 *key = km + ((size_t)j * 2 + comp) * nfull * N;
                u64 *a = acc + comp * ext_sz;
#pragma omp parallel for schedule(dynamic)
                for (int t = 0; t < nb; t++) {
                    u64 psi;
                    u64 qt = basis_prime(P, level, t, &psi);
                    int kpos = t <= level ? t : P->nq + (t - level - 1);
                    u64 *prod = (u64 *)malloc(N * 8);
                    orc_polymul(LIMB(ext, t), LIMB(key, kpos), prod, P->logN, qt, psi);
                    for (u64 x = 0; x < N; x++) LIMB(a, t)[x] = addmod(LIMB(a, t)[x], prod[x], qt);
                    free(prod);
                }
            }
        }
    }
    orc_moddown(P, level, acc, out);
    orc_moddown(P, level, acc + ext_sz, out + (size_t)(level + 1) * N);
    free(ext);
    free(acc);
}

/* rescale of ncomp components: [ncomp][l+1][N] -> [ncomp][l][N];
 * c_i <- (c_i - [c_l]_centered) * q_l^{-1} mod q_i, each component on its own */
void orc_rescale_n(const orc_params *P, int level, int ncomp, const u64 *ct, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    u64 ql = P->q[level];
    for (int c = 0; c < ncomp; c++) {
        const u64 *in = ct + (size_t)c * (level + 1) * N;
        u64 *o = out + (size_t)c * level * N;
        for (int i = 0; i < level; i++) {
            u64 qi = P->q[i];
            u64 qlinv = invmod(ql % qi, qi);
            for (u64 x = 0; x < N; x++) {
                u64 v = LIMB(in, level)[x];
                u64 vi = (v > ql / 2) ? smod(-(i64)(ql - v), qi) : v % qi;
                LIMB(o, i)[x] = mulmod(submod(LIMB(in, i)[x], vi, qi), qlinv, qi);
            }
        }
    }
}

void orc_rescale(const orc_params *P, int level, const u64 *ct, u64 *out) { orc_rescale_n(P, level, 2, ct, out); }

/* automorphism X -> X^g (g odd) on n limbs, coefficient form */
void orc_automorph(const orc_params *P, int n, const int *prime_idx, u64 g, const u64 *in, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    for (int i = 0; i < n; i++) {
        u64 q = P->q[prime_idx[i]];
        for (u64 x = 0; x < N; x++) {
            u64 e = (x * g) % (2 * N);
            u64 v = LIMB(in, i)[x];
            if (e < N) LIMB(out, i)[e] = v;
            else LIMB(out, i)[e - N] = v ? q - v : 0;
        }
    }
}

/* elementwise helpers over n limbs of primes q[0..n) */
void orc_add(const orc_params *P, int n, const u64 *a, const u64 *b, u64 *c)
{
    u64 N = (u64)1 << P->logN;
    for (int i = 0; i < n; i++)
        for (u64 x = 0; x < N; x++) LIMB(c, i)[x] = addmod(LIMB(a, i)[x], LIMB(b, i)[x], P->q[i]);
}
void orc_mul_int(const orc_params *P, int n, const u64 *a, i64 k, u64 *c)
{
    u64 N = (u64)1 << P->logN;
    for (int i = 0; i < n; i++) {
        u64 kq = smod(k, P->q[i]);
        for (u64 x = 0; x < N; x++) LIMB(c, i)[x] = mulmod(LIMB(a, i)[x], kq, P->q[i]);
    }
}
/* c = a * m (integer plaintext polynomial) over n limbs */
void orc_mul_plain(const orc_params *P, int n, const u64 *a, const i64 *m, u64 *c)
{
    u64 N = (u64)1 << P->logN;
    u64 *mr = (u64 *)malloc((size_t)n * N * 8);
    orc_int_to_rns(P, m, 0, n, mr);
    rns_polymul(P, a, mr, c, n);
    free(mr);
}

/* ------------------------------------------------------------------ */
/* keys, encryption, decryption                                        */
/* ------------------------------------------------------------------ */
/* b = -a*s + e (+ m) on n limbs of the basis given by prime_idx */
static void rlwe_b(const orc_params *P, int n, const int *prime_idx, const u64 *a, const i64 *s,
                   const i64 *e, const u64 *extra, u64 *b)
{
    u64 N = (u64)1 << P->logN;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; i++) {
        int pi = prime_idx[i];
        u64 q = P->q[pi];
        u64 *sr = (u64 *)malloc(N * 8), *as = (u64 *)malloc(N * 8);
        for (u64 x = 0; x < N; x++) sr[x] = smod(s[x], q);
        orc_polymul(LIMB(a, i), sr, as, P->logN, q, P->psi[pi]);
        for (u64 x = 0; x < N; x++) {
            u64 v = submod(smod(e[x], q), as[x], q);
            if (extra) v = addmod(v, LIMB(extra, i)[x], q);
            LIMB(b, i)[x] = v;
        }
        free(sr);
        free(as);
    }
}

/* secret key: ternary, Hamming weight h */
void orc_keygen_secret(const orc_params *P, u64 seed, int h, i64 *s) { orc_sample_hwt(seed, P->logN, h, s); }

/*
 * Evaluation key for s' (given as residues sp over the full basis
 * [nq+nk][N], coefficient form): for digit j, over every basis prime,
 *   a_j uniform,  b_j = -a_j*s + e_j + [i in D_j] * (P mod q_i) * s'.
 * out: [beta_top][2][nq+nk][N].
 */
void orc_gen_evk(const orc_params *P, const i64 *s, const u64 *sp, u64 seed, u32 key_id, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int nfull = P->nq + P->nk;
    int beta = orc_ndigits(P, P->nq - 1);
    int idx[ORC_MAXP];
    for (int i = 0; i < nfull; i++) idx[i] = i;
    i64 *e = (i64 *)malloc(N * 8);
    u64 *gad = (u64 *)malloc((size_t)nfull * N * 8);
    for (int j = 0; j < beta; j++) {
        u64 *b = out + (size_t)j * 2 * nfull * N;
        u64 *a = b + (size_t)nfull * N;
        for (int i = 0; i < nfull; i++)
            orc_sample_uniform(seed, ST_EVK_A, key_id, (u32)(j * 256 + i), P->q[i], P->logN, LIMB(a, i));
        orc_sample_cbd(seed, ST_EVK_E, key_id, (u32)j, P->logN, e);
        for (int i = 0; i < nfull; i++) {
            u64 q = P->q[i];
            int in_digit = (i < P->nq) && (i >= j * P->alpha) && (i < (j + 1) * P->alpha);
            u64 Pmod = 1;
            for (int p = 0; p < P->nk; p++) Pmod = mulmod(Pmod, P->q[P->nq + p] % q, q);
            for (u64 x = 0; x < N; x++) LIMB(gad, i)[x] = in_digit ? mulmod(Pmod, LIMB(sp, i)[x], q) : 0;
        }
        rlwe_b(P, nfull, idx, a, s, e, gad, b);
    }
    free(e);
    free(gad);
}

/* public key (b, a) on q_0..q_{nq-1}: a uniform, b = -a*s + e */
void orc_gen_pk(const orc_params *P, const i64 *s, u64 seed, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int n = P->nq, idx[ORC_MAXP];
    for (int i = 0; i < n; i++) idx[i] = i;
    u64 *b = out, *a = out + (size_t)n * N;
    for (int i = 0; i < n; i++) orc_sample_uniform(seed, ST_PK_A, 0, (u32)i, P->q[i], P->logN, LIMB(a, i));
    i64 *e = (i64 *)malloc(N * 8);
    orc_sample_cbd(seed, ST_PK_E, 0, 0, P->logN, e);
    rlwe_b(P, n, idx, a, s, e, NULL, b);
    free(e);
}

/* secret-key encryption at level l: (-a*s + e + m, a); stream index = ct_index */
void orc_encrypt_sk(const orc_params *P, int level, const i64 *m, const i64 *s, u64 seed, u32 ct_index, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int n = level + 1, idx[ORC_MAXP];
    for (int i = 0; i < n; i++) idx[i] = i;
    u64 *b = out, *a = out + (size_t)n * N;
    for (int i = 0; i < n; i++) orc_sample_uniform(seed, ST_ENC_A, ct_index, (u32)i, P->q[i], P->logN, LIMB(a, i));
    i64 *e = (i64 *)malloc(N * 8);
    orc_sample_cbd(seed, ST_ENC_E0, ct_index, 0, P->logN, e);
    u64 *mr = (u64 *)malloc((size_t)n * N * 8);
    orc_int_to_rns(P, m, 0, n, mr);
    rlwe_b(P, n, idx, a, s, e, mr, b);
    free(e);
    free(mr);
}

/*
 * Seeded secret-key encryption at level l (reading: the server's sk
 * encryption of Alg. 2 lets the uniform part be sent as a seed).  The uniform
 * part is drawn in the evaluation domain: for limb i its value at the root
 * psi_i^(2k+1) (natural order k) is the uniform residue of coefficient k of
 * stream (seed; ST_SEED_A, index, i); a = its inverse NTT.  Then, as
 * orc_encrypt_sk: (-a*s + e + m, a), e from (seed; ST_ENC_E0, index, 0).
 */
void orc_encrypt_sk_seeded(const orc_params *P, int level, const i64 *m, const i64 *s, u64 seed, u32 ct_index,
                           u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int n = level + 1, idx[ORC_MAXP];
    for (int i = 0; i < n; i++) idx[i] = i;
    u64 *b = out, *a = out + (size_t)n * N;
    for (int i = 0; i < n; i++) {
        orc_sample_uniform(seed, ST_SEED_A, ct_index, (u32)i, P->q[i], P->logN, LIMB(a, i));
        orc_ntt_inv(LIMB(a, i), P->logN, P->q[i], P->psi[i]);
    }
    i64 *e = (i64 *)malloc(N * 8);
    orc_sample_cbd(seed, ST_ENC_E0, ct_index, 0, P->logN, e);
    u64 *mr = (u64 *)malloc((size_t)n * N * 8);
    orc_int_to_rns(P, m, 0, n, mr);
    rlwe_b(P, n, idx, a, s, e, mr, b);
    free(e);
    free(mr);
}

/* public-key encryption at level l: (v*pk_b + e0 + m, v*pk_a + e1) */
void orc_encrypt_pk(const orc_params *P, int level, const i64 *m, const u64 *pk, u64 seed, u32 ct_index, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int n = level + 1, nq = P->nq;
    i64 *v = (i64 *)malloc(N * 8), *e0 = (i64 *)malloc(N * 8), *e1 = (i64 *)malloc(N * 8);
    orc_sample_ternary(seed, ST_ENC_V, ct_index, 0, P->logN, v);
    orc_sample_cbd(seed, ST_ENC_E0, ct_index, 0, P->logN, e0);
    orc_sample_cbd(seed, ST_ENC_E1, ct_index, 0, P->logN, e1);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; i++) {
        u64 q = P->q[i];
        u64 *vr = (u64 *)malloc(N * 8), *t = (u64 *)malloc(N * 8);
        for (u64 x = 0; x < N; x++) vr[x] = smod(v[x], q);
        orc_polymul(vr, pk + (size_t)i * N, t, P->logN, q, P->psi[i]);
        for (u64 x = 0; x < N; x++) LIMB(out, i)[x] = addmod(addmod(t[x], smod(e0[x], q), q), smod(m[x], q), q);
        orc_polymul(vr, pk + (size_t)(nq + i) * N, t, P->logN, q, P->psi[i]);
        for (u64 x = 0; x < N; x++) LIMB(out + (size_t)n * N, i)[x] = addmod(t[x], smod(e1[x], q), q);
        free(vr);
        free(t);
    }
    free(v);
    free(e0);
    free(e1);
}

/* decrypt at level l: residues of b + a*s on q_0..q_l */
void orc_decrypt(const orc_params *P, int level, const u64 *ct, const i64 *s, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int n = level + 1;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; i++) {
        u64 q = P->q[i];
        u64 *sr = (u64 *)malloc(N * 8), *t = (u64 *)malloc(N * 8);
        for (u64 x = 0; x < N; x++) sr[x] = smod(s[x], q);
        orc_polymul(LIMB(ct + (size_t)n * N, i), sr, t, P->logN, q, P->psi[i]);
        for (u64 x = 0; x < N; x++) LIMB(out, i)[x] = addmod(LIMB(ct, i)[x], t[x], q);
        free(sr);
        free(t);
    }
}

/* s' residues for relinearisation: s^2 over the full basis */
void orc_secret_square(const orc_params *P, const i64 *s, u64 *out)
{
    u64 N = (u64)1 << P->logN;
    int nfull = P->nq + P->nk;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < nfull; i++) {
        u64 q = P->q[i];
        u64 *sr = (u64 *)malloc(N * 8);
        for (u64 x = 0; x < N; x++) sr[x] = smod(s[x], q);
        orc_polymul(sr, sr, LIMB(out, i), P->logN, q, P->psi[i]);
        free(sr);
    }
}
