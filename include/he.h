/*
 * he.h -- C ABI of libhe: RNS-CKKS arithmetic and the encrypted logistic-
 * regression gradient step on one AMD Instinct MI355X (gfx950).
 *
 * What it implements.  The paper (Li & Huang, "Faster Secure Data Mining via
 * Distributed Homomorphic Encryption", KDD'20) trains linear models on data
 * that a parameter server encrypted with HEAAN; each worker evaluates the
 * linearised gradient step of eq. (appr) + eq. (update) on its encrypted shard
 * (Alg. 1) and sends the encrypted weights back for a refresh every l steps
 * (Alg. 2).  The library provides the operations Sec. 3 ("Preliminary") lists --
 * encode/decode, key generation, encrypt/decrypt, add, multiply, rescale --
 * plus the rotation the block packing needs, and the whole step of eq. (appr)
 * on one worker's shard.
 *
 * Conventions shared by every entry point.
 *   Memory.   Ciphertexts, plaintexts and key buffers are device memory OWNED
 *             BY THE CALLER (allocated, for example, with torch); the library
 *             never frees them.  The context owns only its precomputed tables
 *             and a scratch workspace, and takes both from the allocator the
 *             caller gives he_ctx_create (grown on demand outside any graph
 *             capture, given back by he_ctx_trim / he_ctx_destroy).
 *   Layout.   A ciphertext at level l is uint64 [2][l+1][N], limb-major (limb i
 *             of component c at element offset (c*(l+1)+i)*N), values in
 *             [0, q_i), in the library's private NTT order.  A plaintext at
 *             level l is uint64 [l+1][N] in the same order.  The canonical
 *             exchange form (he_ct_download / he_ct_upload) is coefficient
 *             order, residues in [0, q_i).
 *   Streams.  Every call is asynchronous on the context's HIP stream
 *             (he_ctx_set_stream); outputs are valid after that stream is
 *             synchronised.  Calls that return host data synchronise it.
 *   Threads.  One context per stream; a context is not thread-safe.
 *   Errors.   No exception crosses the ABI.  Every metadata check (levels,
 *             scales, keys, sizes) is made on the host BEFORE any launch, so a
 *             call that returns an error has launched nothing.
 *   In place. he_rescale and he_add accept out == in.
 */
#ifndef HE_H
#define HE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HE_OK = 0,
    HE_EINVAL = 1,  /* bad argument, size or layout */
    HE_ENOMEM = 2,  /* device or host allocation failed */
    HE_ELEVEL = 3,  /* not enough levels / level mismatch */
    HE_ESCALE = 4,  /* scale mismatch or scale plan out of range */
    HE_EKEY = 5,    /* required evaluation key absent, or keys of another parameter set */
    HE_EDEVICE = 6  /* HIP runtime error */
} he_status;

/*
 * Scheme parameters (the paper fixes none; it names only the ring order N and
 * the modulus magnitude M and their trade-off, Sec. 3).
 *   log_n      ring degree N = 2^log_n, 10 <= log_n <= 16
 *   n_q        ciphertext primes q_0..q_{n_q-1} (top level L = n_q-1), 2..40
 *   n_special  special primes for key switching, 1..12
 *   alpha      primes per key-switching digit (dnum = ceil(n_q/alpha)), alpha <= n_special
 *   log_delta  log2 of the default scale, 20..50
 * Prime rule: every prime is 1 mod 2^17; specials are the n_special largest
 * below 2^60; q_0 the largest below 2^min(60, log_delta+20); q_1.. the n_q-1
 * closest to 2^log_delta by increasing distance (ties: smaller first).
 */
typedef struct {
    int32_t log_n;
    int32_t n_q;
    int32_t n_special;
    int32_t alpha;
    int32_t log_delta;
} he_params;

typedef struct he_ctx he_ctx;
typedef struct he_keys he_keys;

/* Ciphertext (Sec. 3: a pair of ring elements).  data: device [2][level+1][N]. */
typedef struct {
    uint64_t *data;
    int32_t level;
    int32_t reserved;
    double scale;
} he_ct;

/* Plaintext: device [level+1][N], NTT order, with its encoding scale. */
typedef struct {
    uint64_t *data;
    int32_t level;
    int32_t reserved;
    double scale;
} he_pt;

/* Seeded ciphertext: the b component in device memory, the uniform a
 * component given by (seed, index) and regenerated on use (half the bytes of
 * an he_ct).  b: device [level+1][N], NTT order. */
typedef struct {
    uint64_t *b;
    int32_t level;
    int32_t reserved;
    double scale;
    uint64_t seed;
    uint32_t index;
    uint32_t reserved2;
} he_ct_seeded;

/* Degree-2 ciphertext (d0, d1, d2) of a product before relinearisation. */
typedef struct {
    uint64_t *data; /* device [3][level+1][N] */
    int32_t level;
    int32_t reserved;
    double scale;
} he_ct3;

/* Block layouts of the gradient step (c = 2^ceil(log2 d) columns, r = N/(2c) rows).
 * HE_LAYOUT_ROWS: row-major, slot i*c + j holds y_i x_ij (block packing of the
 * encrypted-LR literature the paper builds on, Sec. 3); W holds w in every row.
 * HE_LAYOUT_FEATURES: feature-major, slot j*r + i holds y_i x_ij; W holds w_j in
 * every slot of feature block j.  Same gradient, fewer key switches per block. */
enum { HE_LAYOUT_ROWS = 0, HE_LAYOUT_FEATURES = 1 };

/* Most baby steps a feature-major margin sum may take (he_lr_grad_step). */
#define HE_MAXBABY 16

/* Scale schedule of one gradient step (pure host; see he_plan_lr_step).
 * The polynomial's terms are formed unrescaled at one level with scale
 * s_c * q (C = A B3, B1 = M Z1 with Z1 at scale s_z1, k0 Z, B2 = A Z2),
 * summed over the blocks and relinearised and rescaled once: s_b1 is the
 * scale of M Z1 and kb1 is unused (0).
 * s_gsum: scale of the summed gradient before its mask (feature-major; equal to
 * s_g for row-major). */
typedef struct {
    int32_t level_in, level_out;
    double s1, s_mask, s_m, s_a, t, s_z3, s_b3, s_c, s_z1, s_b1, s_g;
    int64_t k0, k1, k3, kb1, kw;
    double s_z2;
    int64_t k2;
    double s_gsum;
    int32_t layout, reserved;
} he_lr_plan;

/* Scale schedule of an encrypted inference with the polynomial (pure host;
 * he_plan_lr_infer).  The margins u (scale s_u) go through
 * U2 = RS(relin(u u)) (scale s_u2), H = RS(k3 u) + k2c (declared s_h) and
 * p(u) = RS(relin(H U2)) + RS(k1 u) + k0c at scale s_p; k3 and k1 multiply,
 * k2c and k0c are added as constants. */
typedef struct {
    int32_t level_in, level_out;
    double s_u, s_u2, s_h, s_p;
    int64_t k3, k2c, k1, k0c;
} he_infer_plan;

/* ---------------------------------------------------------------- context */

/* Device memory provider of a context.  alloc(user, bytes) returns `bytes` of
 * device memory on the context's device, 256-byte aligned, or NULL when none
 * is left (the call that needed it then returns HE_ENOMEM); release(user, p)
 * gives back a pointer alloc returned.  The library calls them only from
 * inside its own calls, on the calling thread, and never while a HIP graph is
 * being captured.  The Python binding backs them with torch.empty, so all of
 * the library's device memory is torch's. */
typedef void *(*he_alloc_fn)(void *user, size_t bytes);
typedef void (*he_free_fn)(void *user, void *ptr);

/* Create a context: prime chain, roots, twiddle and basis-conversion tables
 * (device memory from `alloc`; alloc = NULL: hipMalloc / hipFree, release
 * then ignored).  alloc_user is passed back to both callbacks unchanged.
 * hip_stream: a hipStream_t (NULL = default stream).  Errors: HE_EINVAL on
 * parameters out of range, HE_ENOMEM when the allocator fails, HE_EDEVICE
 * from HIP.  On error nothing stays allocated. */
he_status he_ctx_create(const he_params *prm, he_alloc_fn alloc, he_free_fn release, void *alloc_user,
                        void *hip_stream, he_ctx **out);
he_status he_ctx_destroy(he_ctx *ctx);
he_status he_ctx_set_stream(he_ctx *ctx, void *hip_stream);
/* Copy the prime chain (q_0..q_{n_q-1}, then the specials) to host memory;
 * n must be >= n_q + n_special. */
he_status he_ctx_primes(const he_ctx *ctx, uint64_t *out, int n);
/* Pure host (no device): the prime chain the parameters select, as above;
 * n must be >= n_q + n_special.  HE_EINVAL on parameters out of range. */
he_status he_params_primes(const he_params *prm, uint64_t *out, int n);
/* Launch shape of the context's plain forward and inverse NTTs (a tuning
 * knob; results are bit-identical for every setting).  persistent = 1: both
 * passes in one persistent launch of 8 * wg_per_xcd workgroups, each XCD
 * transforming its own limbs with the intermediate kept in its L2 and `lag`
 * first passes issued ahead of the second ones (1 <= lag <= 3), for
 * transforms of at least min_limbs limbs (smaller ones take the two-launch
 * form); 2 / 3: one workgroup of 512 / 1024 threads per limb doing both
 * passes through a scratch limb of its own (8 * wg_per_xcd workgroups, at
 * most 512; the scratch kept in L2 / Infinity Cache; lag unused; ring
 * degrees whose passes do not split evenly fall back to two launches);
 * 0: one launch per pass (the intermediate goes through HBM); 4 / 5: the
 * same with the column passes / both passes taking their workgroups in an
 * XCD-grouped order (XCD k runs the k-th eighth of the blocks, so the strips
 * of one limb run on one XCD together), for every transform of the context,
 * fused ones included; wg_per_xcd, lag and min_limbs unused.  Drops
 * the captured graphs.  HE_EINVAL for values out of range, during capture,
 * or persistent on a ring below 2^12.  Default: the two-launch form
 * (paper_2006_10091_amd/autotune.py measures the choices and writes the
 * table the binding applies). */
he_status he_ctx_set_ntt(he_ctx *ctx, int persistent, int wg_per_xcd, int lag, int min_limbs);
/* Give the context's scratch workspace back to its allocator (it is re-grown
 * on demand); graphs captured over it are dropped. */
he_status he_ctx_trim(he_ctx *ctx);

/* Bytes of a ciphertext / plaintext / degree-2 ciphertext at a level. */
size_t he_ct_bytes(const he_ctx *ctx, int level);
size_t he_pt_bytes(const he_ctx *ctx, int level);
size_t he_ct3_bytes(const he_ctx *ctx, int level);

/* ---------------------------------------------------------------- keys */

/* A key set is valid for every context of its parameter set (ring degree,
 * prime chain and digit width, as he_ctx_create derives them from
 * he_params): contexts of one parameter set may share one key set, as
 * serving lanes on their own streams do.  Every call that takes keys returns
 * HE_EKEY for a key set of another parameter set. */

/* Bytes of the key buffer for n_rot rotation keys (secret key, the keys for
 * s^2, s^3 and s^4, the public key [2][n_q][N] and the rotation keys, each
 * evaluation key [dnum][2][n_q+n_special][N]). */
size_t he_keys_bytes(const he_ctx *ctx, int n_rot);

/* Key generation (Alg. 2, initialisation: the server generates the keys).
 * The secret is ternary with 64 nonzero coefficients; the relinearisation key
 * is for s^2, two more switch s^3 and s^4 to s (the gradient step relinearises
 * a degree-4 sum), and one rotation key is made per entry of rot_steps (a left
 * rotation of the slot vector by that many slots, Galois element 5^t mod 2N).
 * The public key (-a*s + e, a) over q_0..q_{n_q-1} is made too (Alg. 1: the
 * worker's pk).  Randomness: ChaCha20 keyed by seed.  key_buf: caller device
 * memory of at least he_keys_bytes(ctx, n_rot) bytes; *out is a host handle referencing it
 * (free with he_keys_destroy; the buffer stays the caller's). */
he_status he_keygen(he_ctx *ctx, uint64_t seed, const int32_t *rot_steps, int n_rot,
                    void *key_buf, size_t key_buf_bytes, he_keys **out);
/* Release a key handle; graphs its context captured with it are dropped (the
 * buffer stays the caller's).  Keys and the context that made them may be
 * released in either order.  Graphs that other contexts captured with them are never replayed
 * again (their cache entries name the key set's generation) and go with
 * those contexts or their next he_ctx_trim. */
he_status he_keys_destroy(he_keys *keys);
/* Download a key for inspection, coefficient order: which = -2 secret
 * ([n_q+n_special][N]), -5 the public key ([2][n_q][N]), -1 relinearisation
 * key (s^2), -3 / -4 the keys for s^3 / s^4, else the Galois element of a
 * rotation key ([dnum][2][n_q+n_special][N]).  host must hold the size. */
he_status he_keys_download(he_ctx *ctx, const he_keys *keys, int64_t which, uint64_t *host);

/* ---------------------------------------------------------------- encoding (host FP64) */

/* Canonical-embedding encode (Sec. 3, encode/decode): slot j of the complex
 * vector (re[j] + i*im[j], j < n_slots <= N/2, the rest zero) is the value at
 * the root zeta^(5^j), zeta = exp(i*pi/N); coefficients are scale*m rounded half
 * away from zero into coeffs[N] (host).  im may be NULL.  HE_EINVAL when a
 * coefficient does not fit in int64. */
he_status he_encode(he_ctx *ctx, const double *re, const double *im, int n_slots, double scale,
                    int64_t *coeffs);
/* Decode host integer coefficients (as doubles) at a scale into n_slots slots. */
he_status he_decode(he_ctx *ctx, const double *coeffs, double scale, int n_slots, double *re,
                    double *im);

/* Integer coefficients (host int64[N]) -> plaintext at a level (device, NTT). */
he_status he_pt_load(he_ctx *ctx, const int64_t *coeffs, int level, double scale, he_pt *out);

/* ---------------------------------------------------------------- encryption */

/* Encryption of a plaintext at its level (output level = pt level).
 *   use_sk != 0: secret-key encryption (Alg. 2: the server encrypts data and
 *     weights with sk): (-a*s + e + m, a), a uniform, e centred binomial (21
 *     pairs).
 *   use_sk == 0: public-key encryption (Alg. 1: a worker holds pk):
 *     (v*pk_b + e0 + m, v*pk_a + e1), v ternary (P(0) = 1/2), e0 and e1
 *     centred binomial; pk = (-a*s + e, a) is made by he_keygen.
 * Randomness: ChaCha20 keyed by seed; stream index `index` separates
 * ciphertexts made with one seed.  out: caller memory for a ciphertext at
 * pt's level.  Errors: HE_EINVAL. */
he_status he_encrypt(he_ctx *ctx, const he_pt *pt, const he_keys *keys, int use_sk, uint64_t seed,
                     uint32_t index, he_ct *out);
/* Seeded secret-key encryption (Alg. 2: the server encrypts the data with
 * sk, so the uniform part can travel, and stay in HBM, as a seed): out->b =
 * -a*s + e + m with a drawn in the evaluation domain -- limb i's value at
 * the root psi_i^(2k+1) is the uniform residue of coefficient k of ChaCha20
 * stream (seed; type 10, index, i) -- and e as he_encrypt.  out->b: caller
 * memory [pt level + 1][N]; out->seed, out->index are set.  HE_EINVAL. */
he_status he_encrypt_seeded(he_ctx *ctx, const he_pt *pt, const he_keys *keys, uint64_t seed, uint32_t index,
                            he_ct_seeded *out);
/* Materialise seeded ciphertexts: out[i] = (in[i].b, a(in[i].seed,
 * in[i].index)) at in[i]'s level (caller memory).  HE_EINVAL. */
he_status he_ct_expand(he_ctx *ctx, const he_ct_seeded *in, int n, he_ct *out);

/* Decrypt (Alg. 2: the server decrypts the worker's weights): residues of
 * b + a*s at every limb, coefficient order, to host [level+1][N]. */
he_status he_decrypt(he_ctx *ctx, const he_ct *ct, const he_keys *keys, uint64_t *host_residues);
/* Decrypt and decode n_slots slots (host).  The message's coefficients must
 * satisfy |m| < q_0*q_1/2 (lifted from limbs 0 and 1; 0 alone at level 0). */
he_status he_decrypt_decode(he_ctx *ctx, const he_ct *ct, const he_keys *keys, int n_slots,
                            double *re, double *im);

/* Ciphertext <-> canonical coefficient form (host [2][level+1][N]). */
he_status he_ct_download(he_ctx *ctx, const he_ct *ct, uint64_t *host);
he_status he_ct_upload(he_ctx *ctx, const uint64_t *host, int level, double scale, he_ct *out);

/* ---------------------------------------------------------------- homomorphic operations */

/* Tensor product of two ciphertexts at one level (Sec. 3, multiplication):
 * (b1 b2, b1 a2 + a1 b2, a1 a2); scale = product of scales. */
he_status he_mul(he_ctx *ctx, const he_ct *x, const he_ct *y, he_ct3 *out);
/* Relinearisation: hybrid key switch of d2 from s^2 to s (ModUp per digit,
 * inner product with the relinearisation key, ModDown by the special primes). */
he_status he_relin(he_ctx *ctx, const he_ct3 *in, const he_keys *keys, he_ct *out);
/* Rescale (Sec. 3, "scaling": the homomorphic rounding): divide by q_l with
 * rounding and drop limb l; scale /= q_l.  HE_ELEVEL at level 0. */
he_status he_rescale(he_ctx *ctx, const he_ct *in, he_ct *out);
/* Left rotation of the slots by `steps` (automorphism X -> X^(5^steps) and a key
 * switch back to s).  HE_EKEY if that rotation key was not generated. */
he_status he_rotate(he_ctx *ctx, const he_ct *in, int steps, const he_keys *keys, he_ct *out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): he_rotate
 * with its scratch taken from a fixed array of HE_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device until the process ends, so the call
 * allocates nothing (no hipMalloc, no allocator callback).  Arguments,
 * layout and results as he_rotate (bit-identical), out distinct from in.
 * HE_ENOMEM when the rotation needs more scratch than the array holds
 * (he_rotate_noalloc_bytes(ctx, level) > HE_NOALLOC_SCRATCH_BYTES; at
 * N = 2^16 with 4 special primes in 4-prime digits, levels up to 9).  No
 * buffer of the array needs to start at zero.  Every call on one device
 * shares that device's array: calls that overlap on one device (other
 * streams, other threads, other contexts) race and give wrong results;
 * serialise them. */
#define HE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
he_status he_rotate_noalloc(he_ctx *ctx, const he_ct *in, int steps, const he_keys *keys, he_ct *out);
size_t he_rotate_noalloc_bytes(const he_ctx *ctx, int level);

/* out = x + y (same level; HE_ESCALE unless the scales are equal). */
he_status he_add(he_ctx *ctx, const he_ct *x, const he_ct *y, he_ct *out);
/* out = k * x for an integer k, |k| < 2^62; out->scale = out_scale (the caller
 * states how the integer is interpreted). */
he_status he_mul_int(he_ctx *ctx, const he_ct *x, int64_t k, double out_scale, he_ct *out);
/* out = x * pt (plaintext at x's level); scale multiplies. */
he_status he_mul_plain(he_ctx *ctx, const he_ct *x, const he_pt *pt, he_ct *out);
/* out = x restricted to its first level+1 limbs (same scale). */
he_status he_drop_level(he_ctx *ctx, const he_ct *x, int level, he_ct *out);

/* ---------------------------------------------------------------- the gradient step */

/* Pure host scale schedule of one gradient step at W's level (no device use).
 * w_decay = eta * lambda of an L2 regulariser R(w) = lambda/2 |w|^2 (eq. (obj);
 * 0 for none), in [0, 1).  layout: HE_LAYOUT_ROWS or HE_LAYOUT_FEATURES.
 * HE_ELEVEL when fewer than 4 levels remain, HE_ESCALE when an integer
 * constant leaves |k| < 2^62 or no coefficient a1..a3 is nonzero, HE_EINVAL
 * for an unknown layout.  q: the prime chain (he_ctx_primes). */
he_status he_plan_lr_step(const uint64_t *q, int n_q, int level, double s_z, double s_w,
                          const double coef[4], double eta_over_n, double w_decay, int layout,
                          he_lr_plan *out);

/*
 * One encrypted gradient step on one worker's shard: eq. (appr) with a Table 2
 * polynomial p(m) = coef[0] + coef[1] m + coef[2] m^2 + coef[3] m^3 followed by
 * eq. (update) with an optional L2 regulariser, written as
 *   W' = (1 - w_decay) W + g,   g = (eta/n) sum_i p(y_i w.x_i) y_i x_i
 * (p approximates -L'; w_decay = eta lambda; a nonzero coef[2] adds one
 * product per block).
 * Inputs: Z[0..n_blocks) -- the data blocks in `layout` (c*r = N/2), all at one
 * level >= W's and one scale, one uniform stride apart in memory; W -- the
 * weights in the same layout; mask -- a plaintext at the scale
 * he_plan_lr_step gives as s_mask: for HE_LAYOUT_ROWS the column-0 indicator
 * (slots i*c) at W's level - 1, for HE_LAYOUT_FEATURES the indicator of
 * slots j*r at W's level - 3; keys with the relinearisation key and the
 * rotations the slot sums below take (he_lr_grad_step checks them all before
 * any launch, HE_EKEY when one is absent).
 * Row-major: per block, the column sum, mask and replication over the row,
 * polynomial; the row sum once per step.  Feature-major: per block, a cyclic
 * sum over the feature blocks leaves m_i in every slot of sample i, then the
 * polynomial; once per step, the sum inside each feature block, the mask and
 * the replication over the block.  A slot sum of 2^k rotations by multiples
 * of a unit u (row-major: column sum u = n_baby over c / n_baby terms,
 * replication u = -1 over c, row sum u = c over r; feature-major: sample sum
 * u = 1 and replication u = -1 over r) is taken as one hoisted sum (one
 * ModUp, one ModDown) per group of index bits: the k bits in ceil(k/3) groups
 * of sizes differing by at most one, smaller groups on the low bits; a group
 * of s bits from bit b adds the rotations j*2^b*u, j = 1 .. 2^s - 1 (2^k = 128:
 * {1,2,3}, {4,8,12}, {16,..,112} times u).  The keys are those rotations.  In
 * the polynomial, A = M^2 and
 * B3 = M (a3 Z) are rescaled but not relinearised; the terms (degree 4 in the
 * secret) are summed over the blocks and relinearised once per step with the
 * keys for s^2, s^3 and s^4, then rescaled.
 * Baby steps (n_baby a power of two, 1 <= n_baby <= min(c, HE_MAXBABY);
 * 1 = none): the margin sum, a cyclic sum of c rotations by multiples of a
 * unit u (u = r feature-major, 1 row-major), is split as
 * sum_{g} Rot(sum_{j < n_baby} Rot(Z, j u) (x) Rot(W, j u), g n_baby u).
 * The caller keeps Zrot[b * (n_baby - 1) + j - 1] = Rot(Z[b], j u) for
 * j = 1 .. n_baby - 1 (he_rotate_many; one level >= W's, Z's scale, uniform
 * strides in that order; NULL when n_baby = 1); the step rotates W by j u once
 * for all blocks, sums the n_baby products per block without relinearising,
 * and relinearises and rescales once; the column or giant sum then runs over
 * c / n_baby terms instead of c.  keys then also hold the rotations j u
 * (j < n_baby).
 * Feature-major with 1 < n_baby < c and c / n_baby <= 16, the giant steps
 * g n_baby r (0 < g < c / n_baby; they form a group of rotations, c r = N/2)
 * are taken as one hoisted sum, x + sum_g Rot(x, g n_baby r): one ModUp of
 * x's a-part, every rotation's inner product summed in Q u P, one ModDown;
 * keys then hold every g n_baby r.  Otherwise the feature-major giant sum is
 * a grouped sum of unit n_baby r over c / n_baby terms, as the slot sums.
 * Zk (nullable): the step's data terms precomputed by he_lr_data_terms for
 * the same Z, W level and scale, coef, eta_over_n, w_decay and layout
 * (checked: levels, scales and uniform strides; HE_ESCALE when a scale differs);
 * the step then skips their rescales.  NULL: computed in the step.
 * Outputs (caller memory, W's level - 4): W_out, and G_out (nullable) = g.
 * mode 0: plain form (one he_* operation per block per step, one kernel
 * sequence each); mode 1: batched form (every block in one launch per
 * operation, key streams shared across blocks); mode 2: batched form replayed
 * from a captured HIP graph (captured on first use for these buffers).
 * All modes give bit-identical ciphertexts.
 */
he_status he_lr_grad_step(he_ctx *ctx, const he_ct *Z, int n_blocks, const he_ct *W,
                          const he_pt *mask, const double coef[4], double eta_over_n,
                          double w_decay, int c, int r, int layout, const he_ct *Zrot, int n_baby,
                          const he_ct *Zk, const he_keys *keys, int mode, he_ct *W_out, he_ct *G_out);

/*
 * Several independent gradient steps (eq. (appr) + eq. (update), one per
 * request: workers' shards, or serving requests) that share the context, the
 * packing, c, r and their weights' level; each request has its own blocks,
 * weights, mask, Table 2 coefficients, eta/n, regulariser and outputs, with
 * the arguments and meaning of he_lr_grad_step (no baby steps, no data terms).
 * mode 1: each request's per-block part runs on its own blocks, then the
 * once-per-step tail (the relinearisation of the summed degree-4 terms, the
 * rescale, the slot sums, mask and replication, the W update) runs once for
 * all requests, every kernel over all of them together; mode 0: each request
 * as he_lr_grad_step's plain form.  Each request's W' and g are bit-identical
 * to its own he_lr_grad_step.  Errors before any launch: those of
 * he_lr_grad_step for any request, HE_ELEVEL when the weights' levels
 * differ.
 */
typedef struct {
    const he_ct *Z;      /* the request's blocks (uniform stride) */
    int32_t n_blocks;
    const he_ct *W;      /* weights; every request's at one level */
    const he_pt *mask;   /* its step mask (scale from he_plan_lr_step with its eta/n) */
    const double *coef;  /* [4] */
    double eta_over_n, w_decay;
    he_ct *W_out, *G_out;  /* G_out may be NULL */
} he_lr_request;
he_status he_lr_grad_step_multi(he_ctx *ctx, const he_lr_request *reqs, int n_req, int c, int r, int layout,
                                const he_keys *keys, int mode);
/* Device workspace (bytes) of he_lr_grad_step_multi for n_req requests of at
 * most max_blocks blocks each, weights at `level`; 0 for invalid arguments. */
size_t he_lr_grad_step_multi_bytes(const he_ctx *ctx, int level, int max_blocks, int n_req, int layout, int mode);

/*
 * he_lr_grad_step on seeded data blocks (the shard that does not fit in HBM as
 * full ciphertexts: 2^20 samples x 512 features at N = 2^16 is 16384 blocks,
 * 384 GiB in full, 192 GiB seeded).  The blocks are taken `chunk` at a time:
 * each chunk's uniform parts are regenerated into the workspace, then the
 * chunk runs as he_lr_grad_step's batched form (no baby steps, no
 * precomputed data terms) and its gradient terms join the step's sum; the
 * once-per-step part follows the last chunk.  Bit-identical to
 * he_lr_grad_step (mode 1) on the expanded blocks.  Z[b]: one level >= W's,
 * one scale and seed, b-parts one uniform stride apart, index Z[0].index + b.
 * 1 <= chunk <= n_blocks; the workspace holds one chunk
 * (he_lr_step_bytes for `chunk` blocks plus the expanded chunk).  Other
 * arguments and errors as he_lr_grad_step.
 */
he_status he_lr_grad_step_seeded(he_ctx *ctx, const he_ct_seeded *Z, int n_blocks, const he_ct *W, const he_pt *mask,
                                 const double coef[4], double eta_over_n, double w_decay, int c, int r, int layout,
                                 int chunk, const he_keys *keys, he_ct *W_out, he_ct *G_out);
/* Workspace bytes he_lr_grad_step_seeded takes for weights at `level`, data
 * at data_level and `chunk` blocks per chunk (0 for invalid arguments). */
size_t he_lr_step_seeded_bytes(const he_ctx *ctx, int level, int data_level, int chunk, int layout);

/*
 * The data terms of a gradient step (eq. (appr): the a3 and a1 (and a2)
 * coefficients times the data, each an integer multiple of Z rescaled once),
 * which depend on the weights only through their level and scale: a worker
 * whose weights return to the same level and scale every refresh period
 * computes them once per level and passes them to he_lr_grad_step as Zk.
 *   out[b]                = RS(k3 Z[b])   at level l - 1 (features) / l - 2 (rows)
 *   out[n_blocks + b]     = RS(k1 Z[b])   at level l - 2 / l - 3
 *   out[2 n_blocks + b]   = RS(k2 Z[b])   same level, only when coef[2] != 0
 * with k1, k2, k3 from the step's plan (he_plan_lr_step(q, l, Z's scale,
 * w_scale, ...)); l = w_level.  Z as for he_lr_grad_step; out: caller memory,
 * each group of n_blocks at one uniform stride (the k2 group at the k1
 * group's stride).  Errors before any launch: HE_EINVAL, HE_ELEVEL, HE_ESCALE.
 */
he_status he_lr_data_terms(he_ctx *ctx, const he_ct *Z, int n_blocks, int w_level, double w_scale,
                           const double coef[4], double eta_over_n, double w_decay, int layout, he_ct *out);

/*
 * Encrypted inference on one worker's blocks: the margins m_i = w.x_i of
 * eq. (appr) (the first half of the step, for scoring data with the current
 * weights).  Per block: u = RS(relin(Z_b (x) W)), then the margin sum
 * u = sum_{j < c} Rot(u, j unit) -- row major: unit 1 (m_i at slot i*c);
 * feature major: unit r (m_i at every slot j*r + i) -- as grouped hoisted
 * sums, the grouping of he_lr_grad_step's slot sums (keys: j*2^b*unit for
 * each group).  Z, W, c, r, layout as for
 * he_lr_grad_step (W at any level >= 1, Z at a level >= W's); out[0..n_blocks)
 * caller memory for ciphertexts at W's level - 1, one uniform stride apart;
 * scale Z.scale * W.scale / q_level.  mode 0 / 1 / 2 as for he_lr_grad_step
 * (bit-identical).  Errors before any launch: HE_EINVAL, HE_ELEVEL, HE_EKEY.
 */
he_status he_lr_margins(he_ctx *ctx, const he_ct *Z, int n_blocks, const he_ct *W, int c, int r, int layout,
                        const he_keys *keys, int mode, he_ct *out);

/* Pure host schedule of he_lr_infer with a polynomial (no device use): W at
 * `level` (>= 3), data scale s_z, weight scale s_w, coef = a0..a3.  HE_ELEVEL
 * below level 3, HE_ESCALE when a constant leaves |k| < 2^62.  q: the prime
 * chain (he_ctx_primes). */
he_status he_plan_lr_infer(const uint64_t *q, int n_q, int level, double s_z, double s_w, const double coef[4],
                           he_infer_plan *out);

/*
 * Encrypted inference (the serving call; Alg. 1's worker scores its data with
 * the current encrypted weights): the margins m_i = w.x_i of eq. (appr), as
 * he_lr_margins computes them, and, when coef is given, the Table 2
 * polynomial applied slot by slot, p(m) = coef[0] + coef[1] m + coef[2] m^2 +
 * coef[3] m^3 (with p approximating -L', p(m) scores each sample; for the
 * binomial deviance it approximates sigma(-m)).
 *   coef == NULL: out[b] = the margins, exactly he_lr_margins (level W - 1).
 *   coef != NULL: out[b] = p(margins) at W's level - 3 with scale s_p of
 *     he_plan_lr_infer (W at level >= 3).
 * Row-major blocks hold m_i (and p(m_i)) at slot i*c, feature-major ones at
 * every slot j*r + i.  Z, W, c, r, layout, keys, mode as for he_lr_margins;
 * out[0..n_blocks): caller memory at the output level, one uniform stride
 * apart.  Errors before any launch: HE_EINVAL, HE_ELEVEL, HE_ESCALE, HE_EKEY.
 */
he_status he_lr_infer(he_ctx *ctx, const he_ct *Z, int n_blocks, const he_ct *W, int c, int r, int layout,
                      const double *coef, const he_keys *keys, int mode, he_ct *out);

/* Device workspace (bytes) that he_lr_grad_step / he_lr_margins take for
 * n_blocks blocks with weights at `level` in `mode` (with n_baby baby steps for
 * the step; the context keeps and grows one workspace; callers doing
 * admission control budget with this).  0 for invalid arguments. */
size_t he_lr_step_bytes(const he_ctx *ctx, int level, int n_blocks, int layout, int n_baby, int mode);
size_t he_lr_margins_bytes(const he_ctx *ctx, int level, int n_blocks, int mode);

/* ---------------------------------------------------------------- batched operations */

/*
 * Batched multiply -> relinearise -> rescale -> rotate over n independent
 * ciphertext pairs of one context, at any mix of levels 1..L (the ciphertext
 * products, key switches and rescalings of Sec. 3 that the step is made of,
 * as a standalone batch):
 *   out[i] = Rot(RS(relin(x[i] (x) y[i])), steps[i])   at level(x[i]) - 1,
 *   out[i].scale = x[i].scale * y[i].scale / q_level.
 * x[i], y[i]: device ciphertexts of one level each (any addresses); out[i]:
 * caller memory holding a ciphertext at level(x[i]) - 1, distinct from every
 * input.  Entries of one level run together, up to 32 per launch, each with
 * its own rotation key; keys needs the relinearisation key and every step.
 * In modes 1 and 2 the groups are dealt to 4 streams of the context, each
 * with a workspace region of its own, forked from and joined back to the
 * context's stream.
 * mode 0: one entry at a time; 1: grouped by level; 2: grouped, captured
 * into a HIP graph on first use for these buffers and replayed.  All modes
 * give bit-identical outputs.  Errors (before any launch): HE_EINVAL,
 * HE_ELEVEL (level 0 or x/y levels differ), HE_EKEY (a rotation key absent).
 */
he_status he_batch_mul_rotate(he_ctx *ctx, const he_ct *x, const he_ct *y, const int *steps, int n,
                              const he_keys *keys, int mode, he_ct *out);

/*
 * A batch of independent operations described one by one (Sec. 3's
 * homomorphic operations: multiplication with relinearisation, the rounding
 * "scaling" step, rotation, addition), of any mix of kinds and levels:
 *   HE_OP_MUL         out = RS(relin(x (x) y))            level(x) - 1
 *   HE_OP_MUL_ROTATE  out = Rot(RS(relin(x (x) y)), steps) level(x) - 1
 *   HE_OP_ROTATE      out = Rot(x, steps)                   level(x)
 *   HE_OP_RESCALE     out = RS(x)                           level(x) - 1
 *   HE_OP_ADD         out = x + y                           level(x)
 * Rot is a left rotation of the slots by `steps` (Galois element 5^steps).
 * Scales: MUL* x.scale * y.scale / q_level, RESCALE x.scale / q_level, else
 * x.scale; every op's out.level and out.scale are written on return.
 * y is read by MUL, MUL_ROTATE and ADD (same level as x; ADD: same scale) and
 * ignored otherwise.  out.data: caller memory of a ciphertext at the output
 * level; no output may overlap another output or any input of the batch (the
 * operations are independent: none reads another's result).
 * How it runs: a device-side table of the operations' operands drives the
 * elementwise phases -- the tensor products of every MUL / MUL_ROTATE, the
 * staging of ROTATE / RESCALE inputs, every ADD and the copy of every result
 * to its out -- each one launch over all operations of all levels; the key
 * switches and rescalings run per level, all operations of one level
 * together (rotations up to 32 per launch, each with its own key).  In modes
 * 1 and 2 the level groups, which share no data, are dealt to 4 streams of
 * the context (largest first, to the least loaded), each with a scratch area
 * of its own, between a fork from and a join back to the context's stream.
 * mode 0: one operation per launch group; 1: grouped; 2: grouped and
 * captured into a HIP graph on first use for these operations and buffers,
 * replayed afterwards (the table is uploaded before each replay).  All modes
 * give bit-identical outputs, equal to the single-operation calls.
 * Errors, before any launch: HE_EINVAL (bad op code or pointers, overlapping
 * outputs), HE_ELEVEL (level below what the op consumes, x / y levels
 * differ), HE_ESCALE (ADD of different scales), HE_EKEY (a rotation key or
 * the relinearisation key's parameter set).
 */
enum { HE_OP_MUL = 1, HE_OP_MUL_ROTATE = 2, HE_OP_ROTATE = 3, HE_OP_RESCALE = 4, HE_OP_ADD = 5 };
typedef struct {
    int32_t op;     /* HE_OP_* */
    int32_t steps;  /* rotation steps (MUL_ROTATE, ROTATE) */
    he_ct x, y;     /* operands (device) */
    he_ct out;      /* result (device, caller memory); level and scale set on return */
} he_op;
he_status he_batch_submit(he_ctx *ctx, he_op *ops, int n, const he_keys *keys, int mode);
/* Device workspace (bytes) he_batch_submit takes for these operations in
 * `mode` (admission control); 0 for invalid arguments. */
size_t he_batch_submit_bytes(const he_ctx *ctx, const he_op *ops, int n, int mode);

/*
 * Hoisted sum of rotations (Sec. 3 rotations; the feature-major giant steps of
 * he_lr_grad_step): out[i] = x[i] + sum_s Rot(x[i], steps[s]) for n
 * ciphertexts, as one key switch each: x's a-part is raised to Q_l u P once,
 * every rotation's inner product with its key is summed there, and the sum is
 * divided by P once (so the rounding differs from a chain of rotate-and-adds;
 * the slots agree).  1 <= n_steps <= 32.  The gathers are local when the
 * steps' Galois elements form a small group (as the giant steps do); any steps
 * are accepted.  x[0..n): one level and scale, uniform stride; out: caller
 * memory for n ciphertexts at that level, uniform stride, not overlapping x.
 * Errors before any launch: HE_EINVAL, HE_ELEVEL, HE_EKEY.
 */
he_status he_rotate_sum(he_ctx *ctx, const he_ct *x, int n, const int *steps, int n_steps, const he_keys *keys,
                        he_ct *out);

/*
 * Rotations of n ciphertexts by each of n_steps steps (Sec. 3 rotations; the
 * baby-step copies of a shard's data for he_lr_grad_step):
 *   out[i * n_steps + s] = Rot(x[i], steps[s]).
 * x[0..n): one level and scale, one uniform stride apart; out: caller memory
 * for n * n_steps ciphertexts at that level, one allocation with a uniform
 * stride in that order, distinct from x.  With two or more steps each input
 * is raised to Q u P once and rotated every way from there (its digits
 * automorphed per step, one ModDown per output; the same ciphertexts as one
 * key switch per rotation); with one step all n ciphertexts rotate as one
 * batch.  Errors before any launch: HE_EINVAL, HE_ELEVEL, HE_EKEY (a rotation
 * key absent).
 */
he_status he_rotate_many(he_ctx *ctx, const he_ct *x, int n, const int *steps, int n_steps, const he_keys *keys,
                         he_ct *out);

/* ---------------------------------------------------------------- NTT (measurement) */

/* Forward (dir=+1) or inverse (dir=-1) NTT in place over n_limbs consecutive
 * limbs of `data` (device, [n_limbs][N]); limb i uses prime index
 * prime_idx0 + (i % prime_period) of the chain.  Exposed for benchmarking. */
he_status he_ntt(he_ctx *ctx, uint64_t *data, int n_limbs, int prime_idx0, int prime_period, int dir);

/* The VALU roofline of the NTT (measurement): butterflies per second of the
 * transform's butterfly on prime prime_idx with its operands in registers
 * and no memory traffic, fp64 = 1 the lazy FP64 form (primes below 2^46),
 * 0 the 64-bit Shoup form; timed with HIP events on the context's stream
 * (synchronises it).  A transform's VALU fraction is its (N/2) log2 N
 * butterflies per limb times limbs per second over this rate.  HE_EINVAL. */
he_status he_valu_peak(he_ctx *ctx, int prime_idx, int fp64, double *bfly_per_s);

/* ---------------------------------------------------------------- kernel trace (measurement) */

/* Kernel kinds of the trace.  The NTT's two passes are kept apart by their
 * fused prologue or epilogue: MD_CONV is a forward column pass whose prologue
 * forms a ModDown or rescale conversion (Sec. 3's ModDown and rescale),
 * MD_FINISH the row pass storing (base + acc - conversion) P^-1; KS_COLS and
 * KS_ROWS are the key switch's digit transform and the row pass fused with
 * the key inner product. */
enum {
    HE_K_NTT_FWD_COLS = 0, HE_K_NTT_FWD_ROWS, HE_K_NTT_INV_ROWS, HE_K_NTT_INV_COLS, HE_K_NTT_ONE_LAUNCH,
    HE_K_MD_CONV, HE_K_MD_FINISH, HE_K_MD_LAST, HE_K_KS_COLS, HE_K_KS_ROWS, HE_K_MODUP,
    HE_K_GIANT_FP64, HE_K_GIANT_INT, HE_K_ROT_INNER, HE_K_BABY_SUM, HE_K_TERMS_SUM, HE_K_TENSOR,
    HE_K_ELEMENTWISE, HE_K_AUTOMORPH, HE_K_GIANT_GATHER, HE_K_OTHER, HE_K_COUNT
};

/* One kernel kind's launches since the trace was switched on. */
typedef struct {
    int kind;          /* HE_K_* */
    int launches;
    double ms;         /* summed HIP-event time of its launches */
    double bytes;      /* summed algorithmic bytes: each operand of a launch
                        * read or written once; the intermediate between the
                        * two passes of a transform is not counted, so a
                        * plain transform's passes move 16 N bytes a limb */
    double mm_fp64;    /* modular products (butterflies count one each) at
                        * primes below 2^46, done in FP64 */
    double mm_int;     /* the same at wider primes (64-bit integer forms) */
} he_kernel_stat;

/* on != 0: from now on every launch of the context (outside graph capture,
 * where nothing is recorded) is bracketed by two HIP events on the
 * context's stream and recorded with its kind and work; earlier records are
 * dropped.  on = 0: recording stops (records are kept for he_ctx_trace_read).
 * The events add a few microseconds per launch: the trace is for
 * measurement runs, not for timing the whole.  HE_EINVAL. */
he_status he_ctx_trace(he_ctx *ctx, int on);

/* Waits for every recorded launch (and the context's stream), sums the
 * records per kind into out (caller's host array of max entries; kinds with
 * no launch are left out, in kind order) and clears them; *n = the entries
 * written.  HE_EDEVICE when an event failed while recording; HE_EINVAL. */
he_status he_ctx_trace_read(he_ctx *ctx, he_kernel_stat *out, int max, int *n);

/* Name of a kernel kind ("?" when out of range). */
const char *he_kernel_kind_name(int kind);

const char *he_strerror(he_status s);

#ifdef __cplusplus
}
#endif
#endif /* HE_H */
