// he_internal.h -- context, tables and launcher interfaces of libhe.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <set>
#include <string>
#include <vector>

#include "he.h"
#include "modarith.h"

typedef unsigned __int128 u128;
typedef int64_t i64;

#define HE_MAXP 64    // primes in a chain (ciphertext + special)
#define HE_MAXDIG 40  // key-switching digits (table bound)
#define HE_MAXBETA 12 // digits a key may have (register bound of the inner product)

struct DeviceTables {
    PrimeInfo *pinfo;        // [np]
    u64 *psi, *psi_sh;       // [np][N] psi^bitrev(k)
    u64 *ipsi, *ipsi_sh;     // [np][N] psi^-bitrev(k)
    double *psi_d, *ipsi_d;  // [np][N] the same as doubles (used for primes below 2^49)
    // ModUp, per level l and digit j: for each member i of the digit:
    //   up_scale[l][i]           = N^{-1} [qhat_i^{-1}]_{q_i} (+ Shoup)   (i < n_q)
    //   up_conv[l][j][ii][t]     = qhat_i mod prime t (+ Shoup)          (t < np)
    //   up_qd[l][j][t]           = Q_D mod prime t (+ Shoup)
    u64 *up_scale;           // [nq][nq][2]
    u64 *up_conv;            // [nq][HE_MAXDIG][alpha][np][2]
    u64 *up_qd;              // [nq][HE_MAXDIG][np][2]
    // FP64 forms for targets below 2^46 (S_i = conv_split_bits(bit length of q_i)):
    //   up_convd[l][j][ii][t]    = (qhat_i mod t, qhat_i 2^S_i mod t)
    //   up_qdd[l][j][t]          = Q_D mod t
    double *up_convd;        // [nq][HE_MAXDIG][alpha][np][2]
    double *up_qdd;          // [nq][HE_MAXDIG][np]
    double *qinv_d;          // [np] 1 / q_t
    // ModDown (independent of the level):
    u64 *dn_scale;           // [nk][2]  N^{-1} [phat_p^{-1}]_p
    u64 *dn_conv;            // [nk][nq][2] phat_p mod q_i
    u64 *dn_p;               // [nq][2]  P mod q_i
    u64 *dn_pinv;            // [nq][2]  P^{-1} mod q_i
    double *dn_convd;        // [nk][nq][2] (phat_p mod q_i, phat_p 2^S_p mod q_i)
    double *dn_pd;           // [nq] P mod q_i
    // Rescale: rs_qinv[l][i] = q_l^{-1} mod q_i, rs_ql[l][i] = q_l mod q_i  (i < l)
    u64 *rs_qinv;            // [nq][nq][2]
    u64 *rs_ql;              // [nq][nq]
    // Rescale as a one-prime ModDown (source q_l, targets q_i, i < l):
    u64 *rs_one;             // [nq][2]  (1, Shoup of 1) mod q_i: the conversion constant
    u64 *rs_ql2;             // [nq][nq][2] q_l mod q_i (+ Shoup): the centring term
    double *rs_oned;         // [nq][nq][2] (1, 2^S_l mod q_i), S_l = conv_split_bits(bit length of q_l)
    double *rs_qld;          // [nq][nq] q_l mod q_i
};

// Persistent two-pass NTT (plain forward / inverse transforms): per XCD,
// PS_SLOTS limb-sized slots hold the intermediates between the passes in that
// XCD's L2.  on = 0 (the default, by measurement: the per-task
// synchronisation costs more than the saved HBM round trip) uses the
// two-launch form.
constexpr int PS_SLOTS = 4;
struct PersistCfg {
    int on = 0;
    int wg_per_xcd = 64;  // workgroups per XCD of a launch
    int lag = 2;          // first passes issued ahead of the second ones (< PS_SLOTS)
    int min_limbs = 1;    // smaller transforms take the two-launch form
    unsigned *ctr = nullptr;
    u64 *slots = nullptr;
    // on = 4 / 5: two launches, the column passes / both passes taking their
    // blocks in XCD-grouped order (every NTT launch, fused passes included).
    // on = 2 / 3: one workgroup of 512 / 1024 threads per limb (both passes),
    // each with a scratch limb; 8 * wg_per_xcd workgroups, at most limb_wgs
    int limb_wgs = 512;
    u64 *limb_scratch = nullptr;  // [limb_wgs][N]
};

// Kernel trace (he_ctx_trace): one record per launch outside capture, its
// events on the context's stream; events are reused once read
struct KRec {
    int kind;
    hipEvent_t a, b;
    double bytes, mm_fp, mm_int;
};
struct KTrace {
    bool on = false;
    bool failed = false;  // an event call failed while recording
    std::vector<KRec> recs;
    std::vector<hipEvent_t> pool;
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t keys_gen = 0;  // generation of the key set the captured launches read
};

struct he_ctx {
    he_params prm;
    int N, logN, nq, nk, np, alpha, dnum;
    std::vector<u64> q, psi;
    hipStream_t stream;
    int device = 0;                  // the HIP device current at creation
    u64 *noalloc = nullptr;          // this device's fixed scratch array (he_rotate_noalloc)
    he_alloc_fn alloc_fn = nullptr;  // caller's device allocator (null: hipMalloc / hipFree)
    he_free_fn free_fn = nullptr;
    void *alloc_user = nullptr;
    DeviceTables t;
    PersistCfg persist;
    std::vector<void *> owned;  // device allocations of the tables (through the allocator)
    void *ws = nullptr;         // scratch workspace
    size_t ws_bytes = 0;
    std::map<std::string, GraphEntry> graphs;
    bool capturing = false;
    hipStream_t gstream = nullptr;  // private stream of the captured step
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // he_batch_submit's operand-table upload: pinned host staging, and the
    // event after its last copy (the buffer is rewritten only once it passed)
    void *sub_host = nullptr;
    size_t sub_host_bytes = 0;
    hipEvent_t sub_ev = nullptr;
    // he_batch_submit's lanes: independent operation groups run on these
    // streams (default priority) between a fork and a join event
    static constexpr int SUBMIT_LANES = 4;
    hipStream_t lane[SUBMIT_LANES] = {};
    hipEvent_t lane_ev[SUBMIT_LANES] = {}, fork_ev = nullptr;
    // key sets this context made and that are not yet released: their
    // back-pointer is cleared when the context goes first
    std::set<he_keys *> keys_made;
    KTrace kt;
};

struct he_keys {
    he_ctx *ctx;                    // the context that made them (its graphs are dropped with them); NULL once it is destroyed
    int logN, nq, nk, alpha;        // the parameter set they are valid for:
    u64 q[HE_MAXP];                 // any context with this ring and chain may use them
    uint64_t gen;                   // unique per key set (graph-cache key; never reused)
    u64 *sk;                        // [np][N] NTT
    u64 *rlk;                       // [dnum][2][np][N] NTT: s^2 -> s
    u64 *rlk3, *rlk4;               // the same for s^3 and s^4 (degree-4 relinearisation)
    u64 *pk;                        // [2][nq][N] NTT: the public key (-a s + e, a)
    std::map<uint64_t, u64 *> rot;  // Galois element -> key
};

// ------------------------------------------------------------------ host math (host.cpp)
namespace hehost {
u64 mulmod(u64 a, u64 b, u64 q);
u64 powmod(u64 b, u64 e, u64 q);
u64 invmod(u64 a, u64 q);
u64 shoup(u64 w, u64 q);
int gen_primes(int nq, int nk, int log_delta, u64 *out);
u64 find_psi(u64 q, int logN);
void chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16]);
void sample_hwt(u64 seed, int logN, int h, i64 *out);
int encode(int logN, const double *re, const double *im, int n, double scale, i64 *out);
void decode(int logN, const double *m, double scale, int n, double *re, double *im);
void crt2_centred(const u64 *r0, const u64 *r1, size_t N, u64 q0, u64 q1, double *m);
he_status plan_lr_step(const u64 *q, int n_q, int level, double s_z, double s_w, const double coef[4],
                       double eta_over_n, double w_decay, int layout, he_lr_plan *o);
he_status plan_lr_infer(const u64 *q, int n_q, int level, double s_z, double s_w, const double coef[4],
                        he_infer_plan *o);
}  // namespace hehost

enum { ST_SECRET = 1, ST_PK_A = 2, ST_PK_E = 3, ST_EVK_A = 4, ST_EVK_E = 5, ST_ENC_A = 6, ST_ENC_E0 = 7,
       ST_ENC_V = 8, ST_ENC_E1 = 9, ST_SEED_A = 10 };

// ------------------------------------------------------------------ launchers (kernels.hip)
// Batched operands are addressed as base + b * (batch stride) + c * (component
// stride) + pos * N; strides are in uint64 elements.
namespace hek {
// NTT in place over positions [pos0, pos0+npos) of nbatch x ncomp polys;
// dir +1 forward, -1 inverse.  Inverse only: post (nullable) is a table of
// (value, shoup) pairs, indexed from pos0, multiplied into the output in place
// of N^{-1}.  skip_digit: component c skips the positions of digit c.
void ntt_batch(he_ctx *c, u64 *base, long long bstride, long long cstride, int nbatch, int ncomp, int pos0,
               int npos, int ell, int dir, const u64 *post, bool skip_digit);
// fused forms (logN >= 12; fused_ok): out-of-place inverse NTT of positions 0..level
// (src -> dst, output scaled by post); forward NTT of the extended digits whose
// first pass computes the ModUp conversion from y; forward NTT of the ModDown
// conversion (from acc's special limbs) whose second pass stores
// base + (acc - conv) P^{-1} into out.
bool fused_ok(const he_ctx *c);
void intt_from(he_ctx *c, const u64 *src, long long sbs, u64 *dst, long long dbs, int B, int level, const u64 *post);
void ntt_moddown(he_ctx *c, int level, int B, const u64 *acc, long long as, u64 *conv, long long cs, const u64 *base,
                 long long bs, long long bcs, int nbase, u64 *out, long long os, long long ocs,
                 const u64 *add = nullptr, long long ads = 0, long long adcs = 0);
void ntt_rescale(he_ctx *c, int level, int B, int ncomp, const u64 *last, const u64 *in, long long is, long long ics,
                 u64 *tmp, u64 *out, long long os, const i64 *kmul);
void intt_last(he_ctx *c, int level, int B, int ncomp, const u64 *in, long long is, long long ics, u64 *last,
               const i64 *kmul);
// op 0 add, 1 sub, 2 multiply by integer k, 3 multiply by plaintext y ([pos][N]), 4 copy,
// 5 add the integer k to every coefficient (a constant polynomial, NTT form);
// positions 0..level of nbatch x ncomp polys.
void ewise(he_ctx *c, int op, int level, int nbatch, int ncomp, const u64 *x, long long xb, long long xc,
           const u64 *y, long long yb, long long yc, u64 *o, long long ob, long long oc, i64 k);
// tensor product of B pairs at a level (output components d0, d1, d2)
void tensor_b(he_ctx *c, int level, int B, const u64 *x, long long xb, long long xc, const u64 *y, long long yb,
              long long yc, u64 *o, long long ob, long long oc);
// ModUp basis conversion of every digit: y [B][l+1][N] scaled iNTT output,
// ext [B][beta][l+1+nk][N] (positions outside each digit written)
// the gradient terms of nb blocks summed (or accumulated) into the degree-4
// G [5][lp+1][N]: sum_b A (x) B3 + M (x) Z1 + k0 Z (+ A (x) Z2 when Z2), with
// A, B3 of degree 2 ([b][3][lp+1][N], batch stride as)
void terms_sum_b(he_ctx *c, int lp, int nb, const u64 *A, const u64 *B3, long long as, const u64 *Z1, const u64 *Z2,
                 long long ps, long long pc, const u64 *M, long long ms, long long mc, const u64 *Z, long long zs,
                 long long zc, i64 k0, u64 *G, bool accumulate);
// baby-step margin products (MAX_BABY = 16 at most): o[blk] = sum_b Zb[blk] (x) Wb[b]
void baby_sum_b(he_ctx *c, int level, int nblk, int nbaby, const u64 *z, long long zb, long long zc, const u64 *zr,
                long long zrb, long long zrs, long long zrc, const u64 *w, long long wc, const u64 *wr, long long wrs,
                long long wrc, u64 *o, long long ob, long long oc);
void modup_b(he_ctx *c, int level, int B, const u64 *y, long long ys, u64 *ext, long long es, long long ds);
// inner product with one key shared by the batch: acc [B][2][l+1+nk][N]
void ks_inner_b(he_ctx *c, int level, int B, const u64 *d2, long long d2s, const u64 *ext, long long es,
                long long ds, const u64 *key, u64 *acc, long long as);
// per-entry evaluation keys / Galois elements for a batch of up to HE_MAXMULTI
// entries (passed by value as kernel arguments)
constexpr int HE_MAXMULTI = 32;
// one entry of a device-side operand table (he_batch_submit, the batched
// step's tail): x, y inputs and o output of one ciphertext-sized elementwise
// operation over `limbs` limbs (primes q_0 ..), component stride limbs * N
// (x's: xl * N when xl > 0); k: the entry's integer for op 2
struct OpDesc {
    const u64 *x, *y;
    u64 *o;
    int limbs, xl;
    i64 k;
};
// op 0: o = x + y (two components); 2: o = k x (two components); 3: o = x y
// with y one plaintext [limbs][N] (both components); 4: o = x (two
// components); 6: the tensor o[3] = (x0 y0, x0 y1 + x1 y0, x1 y1).  One launch
// over n table entries; limbs: the entries' limbs summed (for the kernel
// trace; negative: n * max_limbs).
void desc_ew(he_ctx *c, int op, const OpDesc *tab, int n, int max_limbs, double limbs = -1.0);
struct EntryKeys {
    const u64 *k[HE_MAXMULTI];
};
struct EntryGal {
    u64 g[HE_MAXMULTI];
};
// hoisted rotation sum, inner products: acc [B][2][l+1+nk][N] = sum_g sum_j
// sigma_g(D_j) key_g[j] from ext [B][beta][l+1+nk][N] (NTT form; digit
// positions from x's a-part), and the ModDown base out [B][2][l+1][N] =
// (x0 + sum_g sigma_g(x0), x1); x, out: batch strides xs / os, component
// stride xc.  ng <= HE_MAXMULTI Galois elements and keys.
void giant_sum_b(he_ctx *c, int level, int B, const u64 *ext, long long es, long long ds, const u64 *x, long long xs,
                 long long xc, const EntryGal &gals, const EntryKeys &keys, int ng, u64 *acc, long long as, u64 *out,
                 long long os);
// the limb at q_l of a ModDown's output in coefficient form (from base's and
// acc's limbs l in coefficient form, [b][comp][N], and acc's special limbs)
void md_last_b(he_ctx *c, int level, int B, const u64 *bl, const u64 *al, const u64 *acc, long long as,
               long long acs, u64 *last);
// ModDown and the rescale by q_l after it in one forward transform:
// out [B][2][l][N] = RS(base + ModDown(acc)), last from md_last_b
void ntt_moddown_rescale(he_ctx *c, int level, int B, const u64 *acc, long long as, const u64 *last,
                         const u64 *base, long long bs, long long bcs, u64 *tmp, u64 *out, long long os);
// rotations of one ciphertext sharing its ModUp, inner products: acc
// [n][2][l+1+nk][N] (stride as) = sum_j sigma_g(D_j) key_g[j] from ext
// [beta][l+1+nk][N] (NTT form; digit positions from x's a-part, x component
// stride xc); n <= HE_MAXMULTI
void rot_inner_b(he_ctx *c, int level, int n, const u64 *ext, long long ds, const u64 *x, long long xc,
                 const EntryGal &gals, const EntryKeys &keys, u64 *acc, long long as);
void ks_inner_multi_b(he_ctx *c, int level, int B, const u64 *d2, long long d2s, const u64 *ext, long long es,
                      long long ds, const EntryKeys &keys, u64 *acc, long long as);
void automorph_multi_b(he_ctx *c, int B, int nl, const u64 *in, long long ib, long long ic, u64 *out, long long ob,
                       long long oc, const EntryGal &gals);
// forward NTT of the extended digits (column pass into ext) fused with the
// inner product (row pass accumulating digit x key): acc [B][2][l+1+nk][N];
// keys: per-entry keys (nullptr: `key` shared by the batch)
void ks_ntt_inner(he_ctx *c, int level, int B, const u64 *d2, long long d2s, u64 *ext, long long es, long long ds,
                  const u64 *key, const EntryKeys *keys, u64 *acc, long long as);
// ModDown conversion from the special primes: conv [B][2][l+1][N] (coefficient)
void moddown_conv_b(he_ctx *c, int level, int B, const u64 *acc, long long as, u64 *conv, long long cs);
// out = base + (acc - conv) P^{-1} on the first nbase components (else no base)
void moddown_finish_b(he_ctx *c, int level, int B, const u64 *acc, long long as, const u64 *conv, long long cs,
                      const u64 *base, long long bs, long long bcs, int nbase, u64 *out, long long os,
                      long long ocs, const u64 *add = nullptr, long long ads = 0, long long adcs = 0);
// rescale pieces: lastc [B][2][N] (coefficient) -> tmp [B][2][l][N]; finish
void rescale_bcast_b(he_ctx *c, int level, int B, const u64 *lastc, u64 *tmp, int ncomp = 2);
void rescale_finish_b(he_ctx *c, int level, int B, const u64 *in, long long is, const u64 *tmp, u64 *out,
                      long long os, int ncomp = 2);
// NTT-order automorphism X -> X^g of B two-component entries of nl limbs
void automorph_b(he_ctx *c, int B, int nl, const u64 *in, long long ib, long long ic, u64 *out, long long ob,
                 long long oc, u64 g);
// out[c] (+)= sum over B entries of in[b][c], positions 0..level, both components
void batch_sum(he_ctx *c, int level, int B, const u64 *in, long long ib, long long ic, u64 *out, long long oc,
               bool accumulate, int ncomp = 2);
// PRNG and samplers (coefficient form), positions -> primes given on the host
void sample_uniform(he_ctx *c, u64 seed, uint32_t type, uint32_t index, uint32_t comp_base, int n_pos,
                    const int *prime_of_pos, u64 *out);
void sample_cbd(he_ctx *c, u64 seed, uint32_t type, uint32_t index, uint32_t comp, int n_pos,
                const int *prime_of_pos, u64 *out);
void int_to_rns(he_ctx *c, const i64 *m, int n_pos, const int *prime_of_pos, u64 *out);
// the uniform part of seeded ciphertexts, drawn in the evaluation domain:
// entry e (stream index index0 + e), limb i: the value at root psi_i^(2k+1) is
// the uniform residue of coefficient k of stream (seed; ST_SEED_A, index0 + e,
// i), stored at NTT position bitrev(k); out + e * os, limbs 0..level
void seeded_a(he_ctx *c, u64 seed, uint32_t index0, int nent, int level, u64 *out, long long os);
// measured butterflies per second of the NTT's FP64 (fp) or 64-bit integer
// butterfly with operands in registers (the VALU roofline of the transform);
// scratch: 256 * 8 * 4 * 256 uint64 of device memory
double valu_bfly_rate(he_ctx *c, bool fp, int pidx, u64 *scratch);
// ternary v: word x of the stream, bit 0 clear -> 0, else bit 1 ? -1 : +1
void sample_ternary(he_ctx *c, u64 seed, uint32_t type, uint32_t index, uint32_t comp, int n_pos,
                    const int *prime_of_pos, u64 *out);
// public-key encryption combine (NTT): b = v pk_b + e0 + m, a = v pk_a + e1 on limbs 0..level
void encpk_combine(he_ctx *c, int level, const u64 *v, const u64 *pk, const u64 *e0, const u64 *e1, const u64 *m,
                   u64 *b, u64 *a);
// key generation / encryption / decryption combines (NTT domain)
void evk_combine(he_ctx *c, const u64 *a, const u64 *s, const u64 *e, const u64 *sp, int digit, u64 *b);
// b = -a s + e + m (m nullable: the public key's b)
void enc_combine(he_ctx *c, int level, const u64 *a, const u64 *s, const u64 *e, const u64 *m, u64 *b);
void dec_combine(he_ctx *c, int level, const u64 *ct, const u64 *s, u64 *out);
}  // namespace hek

#define HIPCHK(x)                                        \
    do {                                                 \
        hipError_t e_ = (x);                             \
        if (e_ != hipSuccess) return HE_EDEVICE;         \
    } while (0)
