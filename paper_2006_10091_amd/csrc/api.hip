// api.hip -- the C ABI of libhe (include/he.h): context and tables, keys,
// encryption, the homomorphic operations and the encrypted gradient step.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <map>
#include <functional>
#include <sstream>

#include "he_internal.h"

#define TRY(x)                          \
    do {                                \
        he_status st_ = (x);            \
        if (st_ != HE_OK) return st_;   \
    } while (0)

namespace {

// ------------------------------------------------------------------ helpers
struct Arena {
    char *base = nullptr;
    size_t cap = 0, off = 0;
    u64 *take(size_t n_u64)
    {
        size_t bytes = (n_u64 * 8 + 255) & ~(size_t)255;
        if (off + bytes > cap) return nullptr;
        u64 *p = (u64 *)(base + off);
        off += bytes;
        return p;
    }
};

inline size_t al(size_t n_u64) { return ((n_u64 * 8 + 255) & ~(size_t)255) / 8; }

// Fixed device scratch of he_rotate_noalloc: one array per device, held until
// the process ends.  Host code never names it: it uses the device address
// hipGetSymbolAddress returned on that device (noalloc_ptr).
static __device__ __align__(256) u64 noalloc_scratch[HE_NOALLOC_SCRATCH_BYTES / 8];
constexpr int HE_MAXDEV = 64;
std::mutex noalloc_mu;
u64 *noalloc_ptr[HE_MAXDEV] = {};

// the scratch array's address on device `dev` (current), looked up once per device
he_status noalloc_setup(int dev, u64 **out)
{
    if (dev < 0 || dev >= HE_MAXDEV) return HE_EDEVICE;
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !p) return HE_EDEVICE;
        noalloc_ptr[dev] = (u64 *)p;
    }
    *out = noalloc_ptr[dev];
    return HE_OK;
}

// Device memory comes from the caller's allocator when one was given (the
// Python binding backs it with torch), else from hipMalloc.
void *dev_alloc(he_ctx *c, size_t bytes)
{
    if (c->alloc_fn) return c->alloc_fn(c->alloc_user, bytes);
    void *p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
void dev_free(he_ctx *c, void *p)
{
    if (!p) return;
    if (c->alloc_fn) {
        if (c->free_fn) c->free_fn(c->alloc_user, p);
        return;
    }
    (void)hipFree(p);
}

// Drop the captured graphs that read key set `keys_gen` (0: every graph).
// Called when that key set is destroyed and whenever the workspace moves: a
// graph holds the device addresses it was captured with.
he_status drop_graphs(he_ctx *c, uint64_t keys_gen)
{
    bool any = false;
    for (auto &kv : c->graphs) any |= keys_gen == 0 || kv.second.keys_gen == keys_gen;
    if (!any) return HE_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->gstream) HIPCHK(hipStreamSynchronize(c->gstream));
    for (auto it = c->graphs.begin(); it != c->graphs.end();) {
        if (keys_gen == 0 || it->second.keys_gen == keys_gen) {
            if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
            if (it->second.graph) (void)hipGraphDestroy(it->second.graph);
            it = c->graphs.erase(it);
        } else {
            ++it;
        }
    }
    return HE_OK;
}

he_status ensure_ws(he_ctx *c, size_t bytes)
{
    if (c->ws_bytes >= bytes) return HE_OK;
    if (c->capturing) return HE_ENOMEM;
    if (c->ws) {
        TRY(drop_graphs(c, 0));
        HIPCHK(hipStreamSynchronize(c->stream));
        dev_free(c, c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    c->ws = dev_alloc(c, bytes);
    if (!c->ws) return HE_ENOMEM;
    c->ws_bytes = bytes;
    return HE_OK;
}

Arena arena(he_ctx *c)
{
    Arena a;
    a.base = (char *)c->ws;
    a.cap = c->ws_bytes;
    return a;
}

inline int beta_at(const he_ctx *c, int level) { return (level + 1 + c->alpha - 1) / c->alpha; }

// scratch (uint64 elements) of one key switch of B entries at a level
size_t ks_scratch(const he_ctx *c, int l, int B)
{
    const size_t N = c->N;
    const int nb = l + 1 + c->nk;
    return al(B * (l + 1) * N) + al((size_t)B * beta_at(c, l) * nb * N) + al((size_t)B * 2 * nb * N) +
           al((size_t)B * 2 * (l + 1) * N);
}
size_t rescale_scratch(const he_ctx *c, int l, int B, int ncomp = 2)
{
    // the unfused form copies a scaled or strided input to a plain one first
    const size_t y = hek::fused_ok(c) ? 0 : al((size_t)B * ncomp * (l + 1) * c->N);
    return al((size_t)B * ncomp * c->N) + al((size_t)B * ncomp * l * c->N) + y;
}
size_t rotate_scratch(const he_ctx *c, int l, int B) { return al((size_t)B * 2 * (l + 1) * c->N) + ks_scratch(c, l, B); }
// relin_rescale_apply: the key switch's buffers and three limbs per component
// (fused); else the relinearised intermediate and the larger of the two steps
size_t relin_rescale_scratch(const he_ctx *c, int l, int B)
{
    if (hek::fused_ok(c)) return ks_scratch(c, l, B) + 3 * al((size_t)B * 2 * c->N);
    return al((size_t)B * 2 * (l + 1) * c->N) + std::max(ks_scratch(c, l, B), rescale_scratch(c, l, B));
}

he_status last_error()
{
    return hipGetLastError() == hipSuccess ? HE_OK : HE_EDEVICE;
}

// ------------------------------------------------------------------ core batched operations
// Key switch of d2 (B entries, NTT, limbs 0..l, batch stride d2s) with key;
// out = base + KS(d2) on the first nbase components, plus add (optional, every
// component; may be out itself).
he_status ks_apply(he_ctx *c, Arena &ar, int l, int B, const u64 *d2, long long d2s, const u64 *key,
                   const u64 *base, long long bs, long long bcs, int nbase, u64 *out, long long os, long long ocs,
                   const hek::EntryKeys *keys = nullptr, const u64 *add = nullptr, long long ads = 0,
                   long long adcs = 0)
{
    const size_t N = c->N;
    const int nb = l + 1 + c->nk, beta = beta_at(c, l);
    const size_t mark = ar.off;
    u64 *y = ar.take((size_t)B * (l + 1) * N);
    u64 *ext = ar.take((size_t)B * beta * nb * N);
    u64 *acc = ar.take((size_t)B * 2 * nb * N);
    u64 *conv = ar.take((size_t)B * 2 * (l + 1) * N);
    if (!y || !ext || !acc || !conv) return HE_ENOMEM;
    const long long ys = (long long)(l + 1) * N, ds = (long long)nb * N, es = (long long)beta * ds;
    const long long as = 2LL * nb * N, cs = 2LL * (l + 1) * N;
    const u64 *up_post = c->t.up_scale + (size_t)l * c->nq * 2;
    if (hek::fused_ok(c)) {
        // digits to coefficient form, scaled by N^{-1} [qhat_i^{-1}]_{q_i} (read from d2)
        hek::intt_from(c, d2, d2s, y, ys, B, l, up_post);
        // ModUp conversion (its own kernel: fused into the first forward pass it
        // measured no faster, also with each digit's targets grouped on one XCD
        // so that the sources are read from L2 -- that pass then waits on the
        // conversion's loads and arithmetic), then the forward NTT of the
        // extended digits
        hek::modup_b(c, l, B, y, ys, ext, es, ds);
        // forward NTT of the extended digits with the key inner product fused into its row pass
        hek::ks_ntt_inner(c, l, B, d2, d2s, ext, es, ds, key, keys, acc, as);
        // special-prime limbs to coefficient form, scaled by N^{-1} [phat_p^{-1}]_p
        hek::ntt_batch(c, acc, as, ds, B, 2, l + 1, c->nk, l, -1, c->t.dn_scale, false);
        // ModDown conversion inside the first pass, base + (acc - conv) P^{-1} stored by the second
        hek::ntt_moddown(c, l, B, acc, as, conv, cs, base, bs, bcs, nbase, out, os, ocs, add, ads, adcs);
    } else {
        hek::ewise(c, 4, l, B, 1, d2, d2s, 0, nullptr, 0, 0, y, ys, 0, 0);
        hek::ntt_batch(c, y, ys, 0, B, 1, 0, l + 1, l, -1, up_post, false);
        hek::modup_b(c, l, B, y, ys, ext, es, ds);
        hek::ntt_batch(c, ext, es, ds, B, beta, 0, nb, l, +1, nullptr, true);
        if (keys)
            hek::ks_inner_multi_b(c, l, B, d2, d2s, ext, es, ds, *keys, acc, as);
        else
            hek::ks_inner_b(c, l, B, d2, d2s, ext, es, ds, key, acc, as);
        hek::ntt_batch(c, acc, as, ds, B, 2, l + 1, c->nk, l, -1, c->t.dn_scale, false);
        hek::moddown_conv_b(c, l, B, acc, as, conv, cs);
        hek::ntt_batch(c, conv, cs, (long long)(l + 1) * N, B, 2, 0, l + 1, l, +1, nullptr, false);
        hek::moddown_finish_b(c, l, B, acc, as, conv, cs, base, bs, bcs, nbase, out, os, ocs, add, ads, adcs);
    }
    ar.off = mark;
    return last_error();
}

// relinearise B degree-2 ciphertexts d3 [B][3][l+1][N] (batch stride d3s) -> out [B][2][l+1][N]
he_status relin_apply(he_ctx *c, Arena &ar, int l, int B, const u64 *d3, long long d3s, const u64 *rlk, u64 *out,
                      long long os)
{
    const long long lc = (long long)(l + 1) * c->N;
    return ks_apply(c, ar, l, B, d3 + 2 * lc, d3s, rlk, d3, d3s, lc, 2, out, os, lc);
}

// relinearise and rescale B degree-2 ciphertexts d3 [B][3][l+1][N] (batch
// stride d3s) -> out [B][2][l][N] (batch stride os): the key switch's ModDown
// and the rescale by q_l share one forward transform (the same integers as
// relin_apply then rescale_apply); unfused contexts take those two
he_status rescale_apply(he_ctx *c, Arena &ar, int l, int B, const u64 *in, long long is, u64 *out, long long os,
                        int ncomp = 2, const i64 *kmul = nullptr, long long ics = 0);
he_status relin_rescale_apply(he_ctx *c, Arena &ar, int l, int B, const u64 *d3, long long d3s, const u64 *rlk,
                              u64 *out, long long os)
{
    const size_t N = c->N;
    const long long lc = (long long)(l + 1) * N;
    const size_t mark = ar.off;
    if (!hek::fused_ok(c)) {
        u64 *u0 = ar.take((size_t)B * 2 * lc);
        if (!u0) return HE_ENOMEM;
        he_status st = relin_apply(c, ar, l, B, d3, d3s, rlk, u0, 2 * lc);
        if (st == HE_OK) st = rescale_apply(c, ar, l, B, u0, 2 * lc, out, os, 2, nullptr, 0);
        ar.off = mark;
        return st;
    }
    const int nb = l + 1 + c->nk, beta = beta_at(c, l);
    u64 *y = ar.take((size_t)B * (l + 1) * N);
    u64 *ext = ar.take((size_t)B * beta * nb * N);
    u64 *acc = ar.take((size_t)B * 2 * nb * N);
    u64 *tmp = ar.take((size_t)B * 2 * (l + 1) * N);
    u64 *tb = ar.take((size_t)B * 2 * N), *ta = ar.take((size_t)B * 2 * N), *last = ar.take((size_t)B * 2 * N);
    if (!y || !ext || !acc || !tmp || !tb || !ta || !last) return HE_ENOMEM;
    const long long ys = lc, ds = (long long)nb * N, es = (long long)beta * ds, as = 2LL * nb * N;
    const u64 *d2 = d3 + 2 * lc;
    hek::intt_from(c, d2, d3s, y, ys, B, l, c->t.up_scale + (size_t)l * c->nq * 2);
    hek::modup_b(c, l, B, y, ys, ext, es, ds);
    hek::ks_ntt_inner(c, l, B, d2, d3s, ext, es, ds, rlk, nullptr, acc, as);
    hek::ntt_batch(c, acc, as, ds, B, 2, l + 1, c->nk, l, -1, c->t.dn_scale, false);
    // limb l of base and acc in coefficient form, then the ModDown output's limb l
    hek::intt_last(c, l, B, 2, d3, d3s, lc, tb, nullptr);
    hek::intt_last(c, l, B, 2, acc, as, ds, ta, nullptr);
    hek::md_last_b(c, l, B, tb, ta, acc, as, ds, last);
    hek::ntt_moddown_rescale(c, l, B, acc, as, last, d3, d3s, lc, tmp, out, os);
    ar.off = mark;
    return last_error();
}

// rescale B ciphertexts of ncomp components at level l -> level l-1 (each
// component on its own; out may equal in only for B == 1)
he_status rescale_apply(he_ctx *c, Arena &ar, int l, int B, const u64 *in, long long is, u64 *out, long long os,
                        int ncomp, const i64 *kmul, long long ics)
{
    // out = RS(k in) with k = *kmul when given; in's component stride is ics
    // (default (l+1) N: a ciphertext at level l, or a higher-level one read on
    // its first l+1 limbs)
    const size_t N = c->N;
    const size_t mark = ar.off;
    const long long lc = (long long)(l + 1) * N;
    if (ics == 0) ics = lc;
    u64 *lastc = ar.take((size_t)B * ncomp * N);
    u64 *tmp = ar.take((size_t)B * ncomp * l * N);
    if (!lastc || !tmp) return HE_ENOMEM;
    // the fused form reads limb i of the input and writes limb i of the output
    // from different workgroups: it needs them apart (he_rescale allows out == in)
    const u64 *in_end = in + (long long)(B - 1) * is + (ncomp - 1) * ics + lc;
    const u64 *out_end = out + (long long)(B - 1) * os + (long long)ncomp * l * N;
    const bool apart = out >= in_end || in >= out_end;
    if (hek::fused_ok(c) && apart) {
        // a one-prime ModDown: the last limbs to coefficient form, then the
        // centred conversion to q_0..q_{l-1} inside the first forward pass and
        // (c_i - x) q_l^{-1} stored by the second
        hek::intt_last(c, l, B, ncomp, in, is, ics, lastc, kmul);
        hek::ntt_rescale(c, l, B, ncomp, lastc, in, is, ics, tmp, out, os, kmul);
    } else {
        if (kmul || ics != lc) {
            // the unfused kernels take a plain level-l input: k in, or a copy
            u64 *y = ar.take((size_t)B * ncomp * lc);
            if (!y) return HE_ENOMEM;
            hek::ewise(c, kmul ? 2 : 4, l, B, ncomp, in, is, ics, nullptr, 0, 0, y, ncomp * lc, lc, kmul ? *kmul : 0);
            in = y;
            is = ncomp * lc;
        }
        hek::ewise(c, 4, 0, B, ncomp, in + (long long)l * N, is, lc, nullptr, 0, 0, lastc, (long long)ncomp * N,
                   (long long)N, 0);
        // the limbs use prime q_l: address them as position l of a shifted base
        hek::ntt_batch(c, lastc - (long long)l * N, (long long)ncomp * N, (long long)N, B, ncomp, l, 1, l, -1,
                       nullptr, false);
        hek::rescale_bcast_b(c, l, B, lastc, tmp, ncomp);
        hek::ntt_batch(c, tmp, (long long)ncomp * l * N, (long long)l * N, B, ncomp, 0, l, l - 1, +1, nullptr,
                       false);
        hek::rescale_finish_b(c, l, B, in, is, tmp, out, os, ncomp);
    }
    ar.off = mark;
    return last_error();
}

// rotate B ciphertexts at level l by the Galois element g
// out = Rot_g(in) (+ add, component stride (l+1) N, batch stride os; may be out)
he_status rotate_apply(he_ctx *c, Arena &ar, int l, int B, const u64 *in, long long is, u64 g, const u64 *key,
                       u64 *out, long long os, const u64 *add = nullptr)
{
    const size_t N = c->N;
    const size_t mark = ar.off;
    const long long lc = (long long)(l + 1) * N;
    u64 *rot = ar.take((size_t)B * 2 * lc);
    if (!rot) return HE_ENOMEM;
    hek::automorph_b(c, B, l + 1, in, is, lc, rot, 2 * lc, lc, g);
    he_status st = ks_apply(c, ar, l, B, rot + lc, 2 * lc, key, rot, 2 * lc, lc, 1, out, os, lc, nullptr, add, os, lc);
    ar.off = mark;
    return st;
}

// rotate B <= HE_MAXMULTI ciphertexts at level l, entry b by Galois element
// gals.g[b] with key keys.k[b]
he_status rotate_multi_apply(he_ctx *c, Arena &ar, int l, int B, const u64 *in, long long is,
                             const hek::EntryGal &gals, const hek::EntryKeys &keys, u64 *out, long long os)
{
    const size_t N = c->N;
    const size_t mark = ar.off;
    const long long lc = (long long)(l + 1) * N;
    u64 *rot = ar.take((size_t)B * 2 * lc);
    if (!rot) return HE_ENOMEM;
    hek::automorph_multi_b(c, B, l + 1, in, is, lc, rot, 2 * lc, lc, gals);
    if (is != 0 || B < 2 || !hek::fused_ok(c)) {
        he_status st = ks_apply(c, ar, l, B, rot + lc, 2 * lc, nullptr, rot, 2 * lc, lc, 1, out, os, lc, &keys);
        ar.off = mark;
        return st;
    }
    // one input rotated B ways: its a-part raised to Q_l u P and transformed
    // once, each rotation's inner product taken from the automorphed digits
    // (the automorphism commutes with the scaling, ModUp and the NTT, so the
    // result is the same as B separate key switches), one ModDown per rotation
    const int nb = l + 1 + c->nk, beta = beta_at(c, l);
    u64 *y = ar.take((size_t)(l + 1) * N);
    u64 *ext = ar.take((size_t)beta * nb * N);
    u64 *acc = ar.take((size_t)B * 2 * nb * N);
    u64 *conv = ar.take((size_t)B * 2 * (l + 1) * N);
    if (!y || !ext || !acc || !conv) return HE_ENOMEM;
    const long long ds = (long long)nb * N, es = (long long)beta * ds, as = 2LL * nb * N, cs = 2LL * (l + 1) * N;
    hek::intt_from(c, in + lc, 0, y, lc, 1, l, c->t.up_scale + (size_t)l * c->nq * 2);
    hek::modup_b(c, l, 1, y, lc, ext, es, ds);
    hek::ntt_batch(c, ext, es, ds, 1, beta, 0, nb, l, +1, nullptr, true);
    hek::rot_inner_b(c, l, B, ext, ds, in, lc, gals, keys, acc, as);
    hek::ntt_batch(c, acc, as, ds, B, 2, l + 1, c->nk, l, -1, c->t.dn_scale, false);
    hek::ntt_moddown(c, l, B, acc, as, conv, cs, rot, 2 * lc, lc, 1, out, os, lc);
    ar.off = mark;
    return last_error();
}

// x + sum_g Rot(x, g) for B ciphertexts at level l (in, batch stride is) as
// one key switch: the a-part's ModUp once, every rotation's inner product
// (automorphism applied to the extended digits, which commutes with ModUp)
// summed in Q_l u P, one ModDown; the b-parts are automorphed and added
// directly.  out [B][2][l+1][N] (batch stride os) must not overlap in.
he_status rotate_sum_hoisted_apply(he_ctx *c, Arena &ar, int l, int B, const u64 *in, long long is,
                                   const hek::EntryGal &gals, const hek::EntryKeys &keys, int ng, u64 *out,
                                   long long os)
{
    const size_t N = c->N;
    const int nb = l + 1 + c->nk, beta = beta_at(c, l);
    const size_t mark = ar.off;
    u64 *y = ar.take((size_t)B * (l + 1) * N);
    u64 *ext = ar.take((size_t)B * beta * nb * N);
    u64 *acc = ar.take((size_t)B * 2 * nb * N);
    u64 *conv = ar.take((size_t)B * 2 * (l + 1) * N);
    if (!y || !ext || !acc || !conv) return HE_ENOMEM;
    const long long lc = (long long)(l + 1) * N, ds = (long long)nb * N, es = (long long)beta * ds;
    const long long as = 2LL * nb * N, cs = 2LL * (l + 1) * N;
    const u64 *up_post = c->t.up_scale + (size_t)l * c->nq * 2;
    if (hek::fused_ok(c)) {
        hek::intt_from(c, in + lc, is, y, lc, B, l, up_post);
    } else {
        hek::ewise(c, 4, l, B, 1, in + lc, is, 0, nullptr, 0, 0, y, lc, 0, 0);
        hek::ntt_batch(c, y, lc, 0, B, 1, 0, l + 1, l, -1, up_post, false);
    }
    hek::modup_b(c, l, B, y, lc, ext, es, ds);
    hek::ntt_batch(c, ext, es, ds, B, beta, 0, nb, l, +1, nullptr, true);
    hek::giant_sum_b(c, l, B, ext, es, ds, in, is, lc, gals, keys, ng, acc, as, out, os);
    hek::ntt_batch(c, acc, as, ds, B, 2, l + 1, c->nk, l, -1, c->t.dn_scale, false);
    if (hek::fused_ok(c)) {
        hek::ntt_moddown(c, l, B, acc, as, conv, cs, out, os, lc, 2, out, os, lc);
    } else {
        hek::moddown_conv_b(c, l, B, acc, as, conv, cs);
        hek::ntt_batch(c, conv, cs, lc, B, 2, 0, l + 1, l, +1, nullptr, false);
        hek::moddown_finish_b(c, l, B, acc, as, conv, cs, out, os, lc, 2, out, os, lc);
    }
    ar.off = mark;
    return last_error();
}

// feature-major giant steps taken as one hoisted sum (the rotations by
// g n_baby rows, g < cols / n_baby, form a group: cols rows = N/2)
constexpr int HE_GIANT_MAX = 16;
bool giant_hoisted(int layout, int cols, int n_baby)
{
    return layout == HE_LAYOUT_FEATURES && n_baby > 1 && n_baby < cols && cols / n_baby <= HE_GIANT_MAX;
}

u64 galois_of(const he_ctx *c, long long steps)
{
    const long long S = c->N / 2;
    long long t = ((steps % S) + S) % S;
    return hehost::powmod(5, (u64)t, 2 * (u64)c->N);
}

const u64 *find_rot_key(const he_keys *k, u64 g)
{
    auto it = k->rot.find(g);
    return it == k->rot.end() ? nullptr : it->second;
}

bool ct_ok(const he_ctx *c, const he_ct *x) { return x && x->data && x->level >= 0 && x->level < c->nq; }

// ------------------------------------------------------------------ tables
template <class T>
T *dev_upload(he_ctx *c, const std::vector<T> &h)
{
    void *p = dev_alloc(c, h.size() * sizeof(T));
    if (!p) return nullptr;
    c->owned.push_back(p);
    if (hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return (T *)p;
}

he_status build_tables(he_ctx *c)
{
    using namespace hehost;
    const int np = c->np, nq = c->nq, nk = c->nk, N = c->N, A = c->alpha;
    std::vector<PrimeInfo> pi(np);
    for (int i = 0; i < np; ++i) {
        u64 q = c->q[i];
        PrimeInfo &p = pi[i];
        p.q = q;
        p.k = 64 - __builtin_clzll(q);
        p.mu = (u64)(((u128)1 << (2 * p.k)) / q);
        p.ninv = invmod((u64)N % q, q);
        p.ninv_sh = shoup(p.ninv, q);
        p.r64 = (u64)(((u128)1 << 64) % q);
        p.r64_sh = shoup(p.r64, q);
        p.one_sh = shoup(1, q);
        p.pad = 0;
    }
    std::vector<u64> psi((size_t)np * N), psis((size_t)np * N), ipsi((size_t)np * N), ipsis((size_t)np * N);
    for (int i = 0; i < np; ++i) {
        u64 q = c->q[i], w = c->psi[i], wi = invmod(w, q);
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (int k = 1; k < N; ++k) {
            pw[k] = mulmod(pw[k - 1], w, q);
            ipw[k] = mulmod(ipw[k - 1], wi, q);
        }
        for (int k = 0; k < N; ++k) {
            unsigned r = 0;
            for (int b = 0; b < c->logN; ++b)
                if (k >> b & 1) r |= 1u << (c->logN - 1 - b);
            size_t o = (size_t)i * N + k;
            psi[o] = pw[r];
            psis[o] = shoup(pw[r], q);
            ipsi[o] = ipw[r];
            ipsis[o] = shoup(ipw[r], q);
        }
    }
    std::vector<u64> up_scale((size_t)nq * nq * 2, 0), up_conv((size_t)nq * HE_MAXDIG * A * np * 2, 0),
        up_qd((size_t)nq * HE_MAXDIG * np * 2, 0);
    for (int l = 0; l < nq; ++l) {
        for (int j = 0; j < beta_at(c, l); ++j) {
            int d0 = j * A, d1 = std::min(d0 + A, l + 1);
            for (int i = d0; i < d1; ++i) {
                u64 qi = c->q[i], qhat = 1;
                for (int i2 = d0; i2 < d1; ++i2)
                    if (i2 != i) qhat = mulmod(qhat, c->q[i2] % qi, qi);
                u64 sc = mulmod(invmod((u64)N % qi, qi), invmod(qhat, qi), qi);
                up_scale[((size_t)l * nq + i) * 2] = sc;
                up_scale[((size_t)l * nq + i) * 2 + 1] = shoup(sc, qi);
                for (int t = 0; t < np; ++t) {
                    u64 qt = c->q[t], v = 1;
                    for (int i2 = d0; i2 < d1; ++i2)
                        if (i2 != i) v = mulmod(v, c->q[i2] % qt, qt);
                    size_t o = ((((size_t)l * HE_MAXDIG + j) * A + (i - d0)) * np + t) * 2;
                    up_conv[o] = v;
                    up_conv[o + 1] = shoup(v, qt);
                }
            }
            for (int t = 0; t < np; ++t) {
                u64 qt = c->q[t], v = 1;
                for (int i2 = d0; i2 < d1; ++i2) v = mulmod(v, c->q[i2] % qt, qt);
                size_t o = (((size_t)l * HE_MAXDIG + j) * np + t) * 2;
                up_qd[o] = v;
                up_qd[o + 1] = shoup(v, qt);
            }
        }
    }
    std::vector<u64> dn_scale((size_t)nk * 2), dn_conv((size_t)nk * nq * 2), dn_p((size_t)nq * 2),
        dn_pinv((size_t)nq * 2);
    for (int k = 0; k < nk; ++k) {
        u64 pk = c->q[nq + k], phat = 1;
        for (int k2 = 0; k2 < nk; ++k2)
            if (k2 != k) phat = mulmod(phat, c->q[nq + k2] % pk, pk);
        u64 sc = mulmod(invmod((u64)N % pk, pk), invmod(phat, pk), pk);
        dn_scale[2 * k] = sc;
        dn_scale[2 * k + 1] = shoup(sc, pk);
        for (int i = 0; i < nq; ++i) {
            u64 qi = c->q[i], v = 1;
            for (int k2 = 0; k2 < nk; ++k2)
                if (k2 != k) v = mulmod(v, c->q[nq + k2] % qi, qi);
            dn_conv[((size_t)k * nq + i) * 2] = v;
            dn_conv[((size_t)k * nq + i) * 2 + 1] = shoup(v, qi);
        }
    }
    for (int i = 0; i < nq; ++i) {
        u64 qi = c->q[i], P = 1;
        for (int k = 0; k < nk; ++k) P = mulmod(P, c->q[nq + k] % qi, qi);
        dn_p[2 * i] = P;
        dn_p[2 * i + 1] = shoup(P, qi);
        u64 Pi = invmod(P, qi);
        dn_pinv[2 * i] = Pi;
        dn_pinv[2 * i + 1] = shoup(Pi, qi);
    }
    // FP64 forms of the conversion constants (used for targets below 2^46)
    auto bits = [](u64 x) { return 64 - __builtin_clzll(x); };
    auto pow2mod = [&](int e, u64 m) {
        u64 r = 1 % m;
        for (int k = 0; k < e; ++k) r = mulmod(r, 2, m);
        return r;
    };
    std::vector<double> up_convd(up_conv.size(), 0.0), up_qdd((size_t)nq * HE_MAXDIG * np, 0.0),
        dn_convd(dn_conv.size(), 0.0), dn_pd(nq, 0.0), qinv_d(np, 0.0);
    for (int t = 0; t < np; ++t) qinv_d[t] = 1.0 / (double)c->q[t];
    for (int l = 0; l < nq; ++l)
        for (int j = 0; j < beta_at(c, l); ++j) {
            int d0 = j * A, d1 = std::min(d0 + A, l + 1);
            for (int i = d0; i < d1; ++i) {
                const int S = conv_split_bits(bits(c->q[i]));
                for (int t = 0; t < np; ++t) {
                    size_t o = ((((size_t)l * HE_MAXDIG + j) * A + (i - d0)) * np + t) * 2;
                    up_convd[o] = (double)up_conv[o];
                    up_convd[o + 1] = (double)mulmod(up_conv[o], pow2mod(S, c->q[t]), c->q[t]);
                }
            }
            for (int t = 0; t < np; ++t)
                up_qdd[((size_t)l * HE_MAXDIG + j) * np + t] = (double)up_qd[(((size_t)l * HE_MAXDIG + j) * np + t) * 2];
        }
    for (int k = 0; k < nk; ++k) {
        const int S = conv_split_bits(bits(c->q[nq + k]));
        for (int i = 0; i < nq; ++i) {
            size_t o = ((size_t)k * nq + i) * 2;
            dn_convd[o] = (double)dn_conv[o];
            dn_convd[o + 1] = (double)mulmod(dn_conv[o], pow2mod(S, c->q[i]), c->q[i]);
        }
    }
    for (int i = 0; i < nq; ++i) dn_pd[i] = (double)dn_p[2 * i];
    std::vector<u64> rs_qinv((size_t)nq * nq * 2, 0), rs_ql((size_t)nq * nq, 0);
    std::vector<u64> rs_one((size_t)nq * 2), rs_ql2((size_t)nq * nq * 2, 0);
    std::vector<double> rs_oned((size_t)nq * nq * 2, 0.0), rs_qld((size_t)nq * nq, 0.0);
    for (int i = 0; i < nq; ++i) {
        rs_one[2 * i] = 1;
        rs_one[2 * i + 1] = shoup(1, c->q[i]);
    }
    for (int l = 1; l < nq; ++l) {
        const int S = conv_split_bits(bits(c->q[l]));
        for (int i = 0; i < l; ++i) {
            u64 qi = c->q[i], v = invmod(c->q[l] % qi, qi);
            rs_qinv[((size_t)l * nq + i) * 2] = v;
            rs_qinv[((size_t)l * nq + i) * 2 + 1] = shoup(v, qi);
            rs_ql[(size_t)l * nq + i] = c->q[l] % qi;
            rs_ql2[((size_t)l * nq + i) * 2] = c->q[l] % qi;
            rs_ql2[((size_t)l * nq + i) * 2 + 1] = shoup(c->q[l] % qi, qi);
            rs_oned[((size_t)l * nq + i) * 2] = 1.0;
            rs_oned[((size_t)l * nq + i) * 2 + 1] = (double)pow2mod(S, qi);
            rs_qld[(size_t)l * nq + i] = (double)(c->q[l] % qi);
        }
    }
    DeviceTables &t = c->t;
    t.pinfo = dev_upload(c, pi);
    t.psi = dev_upload(c, psi);
    t.psi_sh = dev_upload(c, psis);
    t.ipsi = dev_upload(c, ipsi);
    t.ipsi_sh = dev_upload(c, ipsis);
    std::vector<double> psid(psi.begin(), psi.end()), ipsid(ipsi.begin(), ipsi.end());
    t.psi_d = dev_upload(c, psid);
    t.ipsi_d = dev_upload(c, ipsid);
    t.up_scale = dev_upload(c, up_scale);
    t.up_conv = dev_upload(c, up_conv);
    t.up_qd = dev_upload(c, up_qd);
    t.dn_scale = dev_upload(c, dn_scale);
    t.dn_conv = dev_upload(c, dn_conv);
    t.dn_p = dev_upload(c, dn_p);
    t.dn_pinv = dev_upload(c, dn_pinv);
    t.up_convd = dev_upload(c, up_convd);
    t.up_qdd = dev_upload(c, up_qdd);
    t.qinv_d = dev_upload(c, qinv_d);
    t.dn_convd = dev_upload(c, dn_convd);
    t.dn_pd = dev_upload(c, dn_pd);
    t.rs_one = dev_upload(c, rs_one);
    t.rs_ql2 = dev_upload(c, rs_ql2);
    t.rs_oned = dev_upload(c, rs_oned);
    t.rs_qld = dev_upload(c, rs_qld);
    t.rs_qinv = dev_upload(c, rs_qinv);
    t.rs_ql = dev_upload(c, rs_ql);
    if (!t.pinfo || !t.psi || !t.psi_sh || !t.ipsi || !t.ipsi_sh || !t.psi_d || !t.ipsi_d || !t.up_scale || !t.up_conv || !t.up_qd ||
        !t.dn_scale || !t.dn_conv || !t.dn_p || !t.dn_pinv || !t.rs_qinv || !t.rs_ql || !t.up_convd || !t.up_qdd ||
        !t.qinv_d || !t.dn_convd || !t.dn_pd || !t.rs_one || !t.rs_ql2 || !t.rs_oned || !t.rs_qld)
        return HE_ENOMEM;
    // the persistent NTT's slots (8 XCDs x PS_SLOTS limbs) and counters; contents
    // need no initial value (the counters are zeroed before every launch)
    if (hek::fused_ok(c)) {
        c->persist.slots = (u64 *)dev_alloc(c, (size_t)8 * PS_SLOTS * N * 8);
        if (c->persist.slots) c->owned.push_back(c->persist.slots);
        c->persist.ctr = (unsigned *)dev_alloc(c, 4096);
        if (c->persist.ctr) c->owned.push_back(c->persist.ctr);
        if (!c->persist.slots || !c->persist.ctr) return HE_ENOMEM;
    } else {
        c->persist.on = 0;
    }
    return HE_OK;
}

std::vector<int> identity_positions(int n)
{
    std::vector<int> v(n);
    for (int i = 0; i < n; ++i) v[i] = i;
    return v;
}

// one evaluation key for s' (NTT, [np][N]) into dst [dnum][2][np][N]
he_status make_evk(he_ctx *c, Arena &ar, u64 seed, uint32_t key_id, const u64 *sk, const u64 *sp, u64 *dst)
{
    const size_t N = c->N;
    const int np = c->np;
    const size_t mark = ar.off;
    u64 *e = ar.take((size_t)np * N);
    if (!e) return HE_ENOMEM;
    std::vector<int> ids = identity_positions(np);
    for (int j = 0; j < c->dnum; ++j) {
        u64 *b = dst + (size_t)j * 2 * np * N;
        u64 *a = b + (size_t)np * N;
        hek::sample_uniform(c, seed, ST_EVK_A, key_id, (uint32_t)(j * 256), np, ids.data(), a);
        hek::ntt_batch(c, a, 0, 0, 1, 1, 0, np, c->nq - 1, +1, nullptr, false);
        hek::sample_cbd(c, seed, ST_EVK_E, key_id, (uint32_t)j, np, ids.data(), e);
        hek::ntt_batch(c, e, 0, 0, 1, 1, 0, np, c->nq - 1, +1, nullptr, false);
        hek::evk_combine(c, a, sk, e, sp, j, b);
    }
    ar.off = mark;
    return last_error();
}

// ------------------------------------------------------------------ the gradient step
struct StepBufs {
    u64 *T3, *U0, *U, *R, *M, *Z3, *Z1, *A, *B3, *G, *Rg, *Z2, *Gm, *G5;
    u64 *Wr;  // feature-major baby steps: Rot(W, b r), b = 1 .. n_baby - 1
};

// Per-block intermediates sit one level higher in the feature-major circuit
// (no mask level between the margins and the polynomial): e = 1 there.  A and
// B3 are rescaled but not relinearised (three components); the block's
// gradient terms C = A B3 (and B1, B2, k0 Z) are summed unrescaled and
// unrelinearised (degree 4, five components) at level l-3+e, across the
// blocks too, and the sum is relinearised and rescaled once per step.
size_t step_bytes(const he_ctx *c, int l, int nb, int layout, int n_baby = 1)
{
    const size_t N = c->N;
    const int e = layout == HE_LAYOUT_FEATURES ? 1 : 0;
    size_t n = 0;
    n += al((size_t)nb * 3 * (l + 1) * N);                 // T3
    n += al((size_t)nb * 2 * (l + 1) * N);                 // U0
    n += 2 * al((size_t)nb * 2 * l * N);                   // U, R
    n += al((size_t)nb * 2 * (l - 1) * N);                 // M
    n += 2 * al((size_t)nb * 2 * (l - 1 + e) * N);         // Z3, Z1
    n += 2 * al((size_t)nb * 3 * (l - 2 + e) * N);         // A, B3
    n += al((size_t)nb * 2 * (l - 2 + e) * N);             // Z2
    n += al((size_t)5 * (l - 2 + e) * N);                  // G5
    n += 2 * al((size_t)2 * (l - 3 + e) * N);              // G, Rg
    n += al((size_t)2 * (l - 3) * N);                      // Gm
    size_t scratch = std::max(rotate_scratch(c, l, nb), rescale_scratch(c, l, nb));
    scratch = std::max(scratch, rescale_scratch(c, l - 1, nb, 3));  // A, B3: degree 2
    scratch = std::max(scratch, relin_rescale_scratch(c, l, nb));     // the margins' products
    if (n_baby > 1) {
        n += al((size_t)(n_baby - 1) * 2 * (l + 1) * N);  // Wr
        scratch = std::max(scratch, rotate_scratch(c, l, n_baby - 1));
    }
    // per step: the rotations at level l-3+e, or the degree-4 relinearisation's
    // three-entry key switch and its three outputs
    n += std::max(scratch, std::max(rotate_scratch(c, l - 3 + e, 1),
                                    al((size_t)6 * (l - 2 + e) * N) + ks_scratch(c, l - 3 + e, 3)));
    return n * 8 + 4096;
}

he_status step_alloc(he_ctx *c, Arena &ar, int l, int nb, int layout, int n_baby, StepBufs &s)
{
    const size_t N = c->N;
    const int e = layout == HE_LAYOUT_FEATURES ? 1 : 0;
    s.T3 = ar.take((size_t)nb * 3 * (l + 1) * N);
    s.U0 = ar.take((size_t)nb * 2 * (l + 1) * N);
    s.U = ar.take((size_t)nb * 2 * l * N);
    s.R = ar.take((size_t)nb * 2 * l * N);
    s.M = ar.take((size_t)nb * 2 * (l - 1) * N);
    s.Z3 = ar.take((size_t)nb * 2 * (l - 1 + e) * N);
    s.Z1 = ar.take((size_t)nb * 2 * (l - 1 + e) * N);
    s.A = ar.take((size_t)nb * 3 * (l - 2 + e) * N);
    s.B3 = ar.take((size_t)nb * 3 * (l - 2 + e) * N);
    s.Z2 = ar.take((size_t)nb * 2 * (l - 2 + e) * N);
    s.G5 = ar.take((size_t)5 * (l - 2 + e) * N);
    s.G = ar.take((size_t)2 * (l - 3 + e) * N);
    s.Rg = ar.take((size_t)2 * (l - 3 + e) * N);
    s.Gm = ar.take((size_t)2 * (l - 3) * N);
    s.Wr = n_baby > 1 ? ar.take((size_t)(n_baby - 1) * 2 * (l + 1) * N) : nullptr;
    u64 *all[] = {s.T3, s.U0, s.U, s.R, s.M, s.Z3, s.Z1, s.A, s.B3, s.Z2, s.G5, s.G, s.Rg, s.Gm};
    for (u64 *p : all)
        if (!p) return HE_ENOMEM;
    if (n_baby > 1 && !s.Wr) return HE_ENOMEM;
    return HE_OK;
}

// ct x ct -> relin -> rescale for nb entries at level l (inputs [nb][2][*] with
// batch/component strides), output [nb][2][l][N]
he_status mul_relin_rescale(he_ctx *c, Arena &ar, StepBufs &s, int l, int nb, const u64 *x, long long xb,
                            long long xc, const u64 *y, long long yb, long long yc, const u64 *rlk, u64 *out)
{
    const long long N = c->N, lc = (l + 1) * N;
    hek::tensor_b(c, l, nb, x, xb, xc, y, yb, yc, s.T3, 3 * lc, lc);
    return relin_rescale_apply(c, ar, l, nb, s.T3, 3 * lc, rlk, out, 2LL * l * N);
}

// ct x ct -> rescale, not relinearised, for nb entries at level l: output
// [nb][3][l][N] (degree 2)
he_status mul_rescale3(he_ctx *c, Arena &ar, StepBufs &s, int l, int nb, const u64 *x, long long xb, long long xc,
                       const u64 *y, long long yb, long long yc, u64 *out)
{
    const long long N = c->N, lc = (l + 1) * N;
    hek::tensor_b(c, l, nb, x, xb, xc, y, yb, yc, s.T3, 3 * lc, lc);
    return rescale_apply(c, ar, l, nb, s.T3, 3 * lc, out, 3LL * l * N, 3);
}

// per-block part of the step for blocks [b0, b0+nb); G (+)= sum of their terms
// Baby-step copies of the data for the margins: block b's copy for baby step
// j (1 <= j < n_baby) at zr + b * zrb + (j - 1) * zrs, component stride zrc.
struct BabyData {
    const u64 *zr = nullptr;
    long long zrb = 0, zrs = 0, zrc = 0;
    int n_baby = 1;
};

// The step's data terms precomputed by he_lr_data_terms: Z3 = RS(k3 Z) and
// Z1 = RS(k1 Z) (and Z2 = RS(k2 Z) for k2 != 0, with Z1's batch stride),
// block b at z3 + b z3s etc.; nullptr: the step computes them.
struct TermData {
    const u64 *z3 = nullptr, *z1 = nullptr, *z2 = nullptr;
    long long z3s = 0, z1s = 0;
};

he_status slot_sum_hoisted(he_ctx *c, Arena &ar, int level, int B, u64 *x, long long xs, u64 *tmp, long long ts,
                           long long unit, int count, const he_keys *keys);

he_status step_blocks(he_ctx *c, Arena &ar, StepBufs &s, const he_lr_plan &pl, const he_ct *Z, long long zbs, int b0,
                      int nb, const he_ct *W, const he_pt *mask, int cols, const he_keys *keys, bool accumulate,
                      const BabyData &bd, const TermData &td)
{
    const long long N = c->N;
    const int l = W->level;
    const int lz = Z[b0].level;
    const u64 *zp = Z[b0].data;
    const long long zc = (lz + 1) * N;
    const long long wc = (l + 1) * N;
    const long long u1 = (long long)l * N;  // component stride at level l-1
    int t0 = 1;
    if (bd.n_baby > 1) {
        // D1 by baby steps: u = RS(relin(sum_j Rot(Z, j) (x) Rot(W, j))), level l-1
        const long long lc = (l + 1) * N;
        hek::baby_sum_b(c, l, nb, bd.n_baby, zp, zbs, zc, bd.zr + b0 * bd.zrb, bd.zrb, bd.zrs, bd.zrc, W->data, wc,
                        s.Wr, 2 * lc, lc, s.T3, 3 * lc, lc);
        TRY(relin_rescale_apply(c, ar, l, nb, s.T3, 3 * lc, keys->rlk, s.U, 2 * u1));
        t0 = bd.n_baby;
    } else {
        // D1: u = RS(relin(Z (x) W)), level l-1
        TRY(mul_relin_rescale(c, ar, s, l, nb, zp, zbs, zc, W->data, 0, wc, keys->rlk, s.U));
    }
    // column sum: u = sum_{j < cols / t0} Rot(u, j t0), grouped hoisted sums
    // (s.R, unused by this layout, holds every other partial sum)
    TRY(slot_sum_hoisted(c, ar, l - 1, nb, s.U, 2 * u1, s.R, 2 * u1, t0, cols / t0, keys));
    // mask column 0, rescale: M at level l-2
    hek::ewise(c, 3, l - 1, nb, 2, s.U, 2 * u1, u1, mask->data, 0, 0, s.U, 2 * u1, u1, 0);
    TRY(rescale_apply(c, ar, l - 1, nb, s.U, 2 * u1, s.M, 2 * (l - 1) * N));
    const long long m1 = (long long)(l - 1) * N;
    // replicate column 0 over the row: M = sum_{j < cols} Rot(M, -j)
    TRY(slot_sum_hoisted(c, ar, l - 2, nb, s.M, 2 * m1, s.R, 2 * m1, -1, cols, keys));
    // A = RS(M^2) ; Z3 = RS(k3 Z), B3 = RS(M Z3), degree 2 ; Z1 = RS(k1 Z)   (level l-3)
    TRY(mul_rescale3(c, ar, s, l - 2, nb, s.M, 2 * m1, m1, s.M, 2 * m1, m1, s.A));
    const u64 *z3p = s.Z3;
    long long z3s = 2 * m1;
    if (td.z3) {
        z3p = td.z3 + (long long)b0 * td.z3s;
        z3s = td.z3s;
    } else {
        TRY(rescale_apply(c, ar, l - 1, nb, zp, zbs, s.Z3, 2 * m1, 2, &pl.k3, zc));
    }
    TRY(mul_rescale3(c, ar, s, l - 2, nb, s.M, 2 * m1, m1, z3p, z3s, m1, s.B3));
    // Z1 = RS(k1 Z) and, for a2 != 0, Z2 = RS(k2 Z), both at level l-3
    const long long a1 = (long long)(l - 2) * N;
    const u64 *z1p = s.Z1, *z2p = pl.k2 != 0 ? s.Z2 : nullptr;
    long long z1s = 2 * a1;
    if (td.z1) {
        z1p = td.z1 + (long long)b0 * td.z1s;
        z2p = pl.k2 != 0 ? td.z2 + (long long)b0 * td.z1s : nullptr;
        z1s = td.z1s;
    } else {
        TRY(rescale_apply(c, ar, l - 2, nb, zp, zbs, s.Z1, 2 * a1, 2, &pl.k1, zc));
        if (pl.k2 != 0) TRY(rescale_apply(c, ar, l - 2, nb, zp, zbs, s.Z2, 2 * a1, 2, &pl.k2, zc));
    }
    // the blocks' terms at level l-3 (unrescaled, degree 4), summed straight into G5
    hek::terms_sum_b(c, l - 3, nb, s.A, s.B3, 3 * a1, z1p, z2p, z1s, a1, s.M, 2 * m1, m1, zp, zbs, zc, pl.k0, s.G5,
                     accumulate);
    return last_error();
}

// Feature-major per-block part for blocks [b0, b0+nb): margins by a cyclic sum
// over the feature blocks (every slot of sample i ends with m_i), then the
// polynomial one level above the row-major circuit; G (+)= sum of the terms
// at level l-3.
he_status step_blocks_features(he_ctx *c, Arena &ar, StepBufs &s, const he_lr_plan &pl, const he_ct *Z,
                               long long zbs, int b0, int nb, const he_ct *W, int cols, int rows,
                               const he_keys *keys, bool accumulate, const BabyData &bd, const TermData &td)
{
    const long long N = c->N;
    const int l = W->level;
    const int lz = Z[b0].level;
    const u64 *zp = Z[b0].data;
    const long long zc = (lz + 1) * N;
    const long long wc = (l + 1) * N;
    const long long u1 = (long long)l * N;  // component stride at level l-1
    int t0 = 1;
    if (bd.n_baby > 1) {
        // D1 by baby steps: u = RS(relin(sum_j Rot(Z, j r) (x) Rot(W, j r))), level l-1
        const long long lc = (l + 1) * N;
        hek::baby_sum_b(c, l, nb, bd.n_baby, zp, zbs, zc, bd.zr + b0 * bd.zrb, bd.zrb, bd.zrs, bd.zrc, W->data, wc,
                        s.Wr, 2 * lc, lc, s.T3, 3 * lc, lc);
        TRY(relin_rescale_apply(c, ar, l, nb, s.T3, 3 * lc, keys->rlk, s.U, 2 * u1));
        t0 = bd.n_baby;
    } else {
        // D1: u = RS(relin(Z (x) W)), level l-1
        TRY(mul_relin_rescale(c, ar, s, l, nb, zp, zbs, zc, W->data, 0, wc, keys->rlk, s.U));
    }
    u64 *M = s.U;
    if (giant_hoisted(HE_LAYOUT_FEATURES, cols, bd.n_baby)) {
        // the giant steps g n_baby rows (0 < g < cols / n_baby) as one key switch: M = U + sum_g Rot(U)
        hek::EntryGal eg;
        hek::EntryKeys ek;
        const int ng = cols / bd.n_baby - 1;
        for (int g = 1; g <= ng; ++g) {
            eg.g[g - 1] = galois_of(c, (long long)g * bd.n_baby * rows);
            ek.k[g - 1] = find_rot_key(keys, eg.g[g - 1]);
            if (!ek.k[g - 1]) return HE_EKEY;
        }
        TRY(rotate_sum_hoisted_apply(c, ar, l - 1, nb, s.U, 2 * u1, eg, ek, ng, s.R, 2 * u1));
        M = s.R;
    } else {
        // U = sum_{j < cols / t0} Rot(U, j t0 rows), grouped hoisted sums (s.R: the other partial sums)
        TRY(slot_sum_hoisted(c, ar, l - 1, nb, s.U, 2 * u1, s.R, 2 * u1, (long long)t0 * rows, cols / t0, keys));
    }
    // A = RS(M^2) ; Z3 = RS(k3 Z), B3 = RS(M Z3), degree 2 ; Z1 = RS(k1 Z)   (level l-2)
    TRY(mul_rescale3(c, ar, s, l - 1, nb, M, 2 * u1, u1, M, 2 * u1, u1, s.A));
    const u64 *z3p = s.Z3;
    long long z3s = 2 * u1;
    if (td.z3) {
        z3p = td.z3 + (long long)b0 * td.z3s;
        z3s = td.z3s;
    } else {
        TRY(rescale_apply(c, ar, l, nb, zp, zbs, s.Z3, 2 * u1, 2, &pl.k3, zc));
    }
    TRY(mul_rescale3(c, ar, s, l - 1, nb, M, 2 * u1, u1, z3p, z3s, u1, s.B3));
    // Z1 = RS(k1 Z) and, for a2 != 0, Z2 = RS(k2 Z), both at level l-2
    const long long a1 = (long long)(l - 1) * N;
    const u64 *z1p = s.Z1, *z2p = pl.k2 != 0 ? s.Z2 : nullptr;
    long long z1s = 2 * a1;
    if (td.z1) {
        z1p = td.z1 + (long long)b0 * td.z1s;
        z2p = pl.k2 != 0 ? td.z2 + (long long)b0 * td.z1s : nullptr;
        z1s = td.z1s;
    } else {
        TRY(rescale_apply(c, ar, l - 1, nb, zp, zbs, s.Z1, 2 * a1, 2, &pl.k1, zc));
        if (pl.k2 != 0) TRY(rescale_apply(c, ar, l - 1, nb, zp, zbs, s.Z2, 2 * a1, 2, &pl.k2, zc));
    }
    // the block's terms at level l-2 (unrescaled, degree 4); G5 (+)= their sum
    hek::terms_sum_b(c, l - 2, nb, s.A, s.B3, 3 * a1, z1p, z2p, z1s, a1, M, 2 * u1, u1, zp, zbs, zc, pl.k0, s.G5,
                     accumulate);
    return last_error();
}

// The rotation-index groups of a slot sum over count = 2^k slots: the k bits
// of the index in ceil(k / 3) groups, sizes as even as possible (the smaller
// ones first), low bits first.  Group i is {b0, s}: it adds the rotations by
// j 2^b0, j = 1 .. 2^s - 1.  Returns the number of groups (at most 11).
static int slot_sum_groups(int count, int (*g)[2])
{
    int k = 0;
    while ((1 << k) < count) ++k;
    if (k == 0) return 0;
    const int ng = (k + 2) / 3, q = k / ng, rem = k % ng;
    int b0 = 0;
    for (int i = 0; i < ng; ++i) {
        const int sz = q + (i >= ng - rem ? 1 : 0);
        g[i][0] = b0;
        g[i][1] = sz;
        b0 += sz;
    }
    return ng;
}

// x <- sum_{i < count} Rot(x, i unit) on B ciphertexts at `level` (batch
// stride xs; count a power of two; unit may be negative), one hoisted sum per
// index group of slot_sum_groups: the group's rotations share one ModUp and
// one ModDown.  The running sum alternates between x and tmp (B ciphertexts,
// batch stride ts) and ends in x.
he_status slot_sum_hoisted(he_ctx *c, Arena &ar, int level, int B, u64 *x, long long xs, u64 *tmp, long long ts,
                           long long unit, int count, const he_keys *keys)
{
    int grp[11][2];
    const int ng = slot_sum_groups(count, grp);
    u64 *in = x, *out = tmp;
    long long is = xs, os = ts;
    for (int i = 0; i < ng; ++i) {
        const int n = (1 << grp[i][1]) - 1;
        hek::EntryGal eg;
        hek::EntryKeys ek;
        for (int j = 1; j <= n; ++j) {
            eg.g[j - 1] = galois_of(c, unit * ((long long)j << grp[i][0]));
            ek.k[j - 1] = find_rot_key(keys, eg.g[j - 1]);
            if (!ek.k[j - 1]) return HE_EKEY;
        }
        TRY(rotate_sum_hoisted_apply(c, ar, level, B, in, is, eg, ek, n, out, os));
        std::swap(in, out);
        std::swap(is, os);
    }
    if (in != x) {
        const long long lc = (long long)(level + 1) * c->N;
        hek::ewise(c, 4, level, B, 2, in, is, lc, nullptr, 0, 0, x, xs, lc, 0);
    }
    return last_error();
}

// the rotations slot_sum_hoisted(unit, count) takes, all present in k
static bool slot_sum_keys(he_ctx *c, const he_keys *k, long long unit, int count)
{
    int grp[11][2];
    const int ng = slot_sum_groups(count, grp);
    for (int i = 0; i < ng; ++i)
        for (int j = 1; j < 1 << grp[i][1]; ++j)
            if (!find_rot_key(k, galois_of(c, unit * ((long long)j << grp[i][0])))) return false;
    return true;
}

// Every rotation key a gradient step of this layout and baby-step count
// takes.  Feature-major: the margins' baby steps j rows (j < n_baby) and
// giant steps (one hoisted sum of g n_baby rows, else a grouped sum of unit
// n_baby rows over cols / n_baby terms), the sample sum over the rows and the
// replication (grouped sums of unit +1 and -1).  Row-major: baby steps j
// (j < n_baby), the column sum (grouped, unit n_baby, cols / n_baby terms),
// the replication (unit -1, cols terms) and the once-per-step row sum (unit
// cols, rows terms).
he_status step_keys(he_ctx *c, const he_keys *k, int layout, int cols, int rows, int n_baby)
{
    const bool fm = layout == HE_LAYOUT_FEATURES;
    const long long mu = fm ? rows : 1;
    for (int j = 1; j < n_baby; ++j)
        if (!find_rot_key(k, galois_of(c, (long long)j * mu))) return HE_EKEY;
    bool ok;
    if (fm) {
        ok = slot_sum_keys(c, k, 1, rows) && slot_sum_keys(c, k, -1, rows);
        if (giant_hoisted(layout, cols, n_baby)) {
            for (int g = 1; g < cols / n_baby; ++g)
                ok = ok && find_rot_key(k, galois_of(c, (long long)g * n_baby * rows));
        } else {
            ok = ok && slot_sum_keys(c, k, (long long)n_baby * rows, cols / n_baby);
        }
    } else {
        ok = slot_sum_keys(c, k, n_baby, cols / n_baby) && slot_sum_keys(c, k, -1, cols) &&
             slot_sum_keys(c, k, cols, rows);
    }
    return ok ? HE_OK : HE_EKEY;
}

// Run `body` captured into a HIP graph on first use of `key` and replayed
// after that, on the context's private stream ordered after and before the
// caller's stream by events.  Buffers must not move between replays (the key
// names every pointer the body uses, the workspace included).
template <class F>
he_status run_graph(he_ctx *c, const std::string &key, uint64_t keys_gen, F body)
{
    if (!c->gstream) {
        HIPCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    }
    GraphEntry &ge = c->graphs[key];
    hipStream_t user = c->stream;
    HIPCHK(hipEventRecord(c->ev_in, user));
    HIPCHK(hipStreamWaitEvent(c->gstream, c->ev_in, 0));
    if (!ge.exec) {
        c->stream = c->gstream;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) {
            c->stream = user;
            c->graphs.erase(key);
            return HE_EDEVICE;
        }
        c->capturing = true;
        he_status st = body();
        c->capturing = false;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->stream, &g);
        c->stream = user;
        if (st != HE_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            c->graphs.erase(key);
            return st != HE_OK ? st : HE_EDEVICE;
        }
        ge.graph = g;
        ge.keys_gen = keys_gen;
        if (hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            c->graphs.erase(key);
            return HE_EDEVICE;
        }
    }
    HIPCHK(hipGraphLaunch(ge.exec, c->gstream));
    HIPCHK(hipEventRecord(c->ev_out, c->gstream));
    HIPCHK(hipStreamWaitEvent(user, c->ev_out, 0));
    return HE_OK;
}

// ------------------------------------------------------------------ batched mul -> relin -> rescale -> rotate
// Entries of one level run together, up to HE_MAXMULTI per launch, each with
// its own rotation key; inputs are read in place, outputs staged and copied.
// ------------------------------------------------------------------ lanes of independent groups
// Batches whose groups share no data run them on the context's lane streams
// (default priority), forked from and joined back to the context's stream;
// inside a capture the lanes become parallel branches of the graph.
static he_status lanes_ready(he_ctx *c)
{
    if (c->fork_ev) return HE_OK;
    if (c->capturing) return HE_EINVAL;  // made once, outside any capture
    HIPCHK(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    for (int i = 0; i < he_ctx::SUBMIT_LANES; ++i) {
        HIPCHK(hipStreamCreateWithFlags(&c->lane[i], hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->lane_ev[i], hipEventDisableTiming));
    }
    return HE_OK;
}

static he_status lanes_fork(he_ctx *c, int K)
{
    if (K < 2) return HE_OK;
    HIPCHK(hipEventRecord(c->fork_ev, c->stream));
    for (int i = 0; i < K; ++i) HIPCHK(hipStreamWaitEvent(c->lane[i], c->fork_ev, 0));
    return HE_OK;
}

static he_status lanes_join(he_ctx *c, int K)
{
    if (K < 2) return HE_OK;
    for (int i = 0; i < K; ++i) {
        HIPCHK(hipEventRecord(c->lane_ev[i], c->lane[i]));
        HIPCHK(hipStreamWaitEvent(c->stream, c->lane_ev[i], 0));
    }
    return HE_OK;
}

// Runs tasks (cost, body(lane)) on K lanes: largest first, each to the least
// loaded lane; body runs with c->stream set to its lane's stream (the
// context's own stream when K = 1).  The lanes are joined even after an error.
static he_status lanes_run(he_ctx *c, int K, std::vector<std::pair<double, std::function<he_status(int)>>> &tasks)
{
    std::vector<int> order(tasks.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return tasks[a].first > tasks[b].first; });
    TRY(lanes_fork(c, K));
    hipStream_t main = c->stream;
    std::vector<double> load(K, 0.0);
    he_status st = HE_OK;
    for (int t : order) {
        const int i = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[i] += tasks[t].first;
        c->stream = K > 1 ? c->lane[i] : main;
        st = tasks[t].second(i);
        c->stream = main;
        if (st != HE_OK) break;
    }
    TRY(lanes_join(c, K));
    return st;
}

size_t batch_bytes(const he_ctx *c, int l, int B)
{
    const size_t N = c->N;
    size_t n = al((size_t)B * 3 * (l + 1) * N) + 2 * al((size_t)B * 2 * l * N);
    n += std::max(relin_rescale_scratch(c, l, B), rotate_scratch(c, l - 1, B));
    return n * 8 + 4096;
}

// The level groups (in chunks) of he_batch_mul_rotate as tasks on K lanes,
// lane i with the scratch [i * per, (i + 1) * per) of the workspace.
he_status batch_impl(he_ctx *c, const he_ct *x, const he_ct *y, const u64 *gal, const he_keys *k, int chunk,
                     const std::map<int, std::vector<int>> &groups, he_ct *out, int K, size_t per)
{
    const long long N = c->N;
    std::vector<std::pair<double, std::function<he_status(int)>>> tasks;
    for (const auto &gr : groups) {
        const int l = gr.first;
        const std::vector<int> *idx = &gr.second;
        for (size_t s0 = 0; s0 < idx->size(); s0 += chunk) {
            const int B = (int)std::min<size_t>(chunk, idx->size() - s0);
            tasks.push_back({(double)B * (l + 1 + c->nk), [=](int lane) -> he_status {
                const long long lc = (long long)(l + 1) * N, rc = (long long)l * N;
                Arena ar;
                ar.base = (char *)c->ws + (size_t)lane * per;
                ar.cap = per;
                u64 *T3 = ar.take((size_t)B * 3 * lc);
                u64 *R = ar.take((size_t)B * 2 * rc);
                u64 *Ob = ar.take((size_t)B * 2 * rc);
                if (!T3 || !R || !Ob) return HE_ENOMEM;
                hek::EntryKeys keys;
                hek::EntryGal gals;
                for (int b = 0; b < B; ++b) {
                    const int i = (*idx)[s0 + b];
                    hek::tensor_b(c, l, 1, x[i].data, 0, lc, y[i].data, 0, lc, T3 + b * 3 * lc, 3 * lc, lc);
                    keys.k[b] = find_rot_key(k, gal[i]);
                    gals.g[b] = gal[i];
                }
                TRY(relin_rescale_apply(c, ar, l, B, T3, 3 * lc, k->rlk, R, 2 * rc));
                TRY(rotate_multi_apply(c, ar, l - 1, B, R, 2 * rc, gals, keys, Ob, 2 * rc));
                for (int b = 0; b < B; ++b)
                    hek::ewise(c, 4, l - 1, 1, 2, Ob + b * 2 * rc, 0, rc, nullptr, 0, 0, out[(*idx)[s0 + b]].data, 0,
                               rc, 0);
                return HE_OK;
            }});
        }
    }
    TRY(lanes_run(c, K, tasks));
    return last_error();
}

// ------------------------------------------------------------------ encrypted inference (margins)
size_t margins_bytes(const he_ctx *c, int l, int nb)
{
    const size_t N = c->N;
    size_t n = al((size_t)nb * 3 * (l + 1) * N) + al((size_t)nb * 2 * l * N);
    n += std::max(relin_rescale_scratch(c, l, nb), rotate_scratch(c, l - 1, nb));
    return n * 8 + 4096;
}

// u = RS(relin(Z_b (x) W)) written straight into out (uniform batch stride
// obs), then the margin sum in place: u = sum_{j < count} Rot(u, j unit) as
// grouped hoisted sums (R holds every other partial sum)
he_status margins_impl(he_ctx *c, const he_ct *Z, int n_blocks, long long zbs, const he_ct *W, long long unit,
                       int count, const he_keys *keys, int chunk, u64 *out, long long obs, size_t ws_off = 0)
{
    const long long N = c->N;
    const int l = W->level;
    const long long zc = (long long)(Z[0].level + 1) * N, wc = (long long)(l + 1) * N, lc = wc, u1 = (long long)l * N;
    for (int b0 = 0; b0 < n_blocks; b0 += chunk) {
        const int nb = std::min(chunk, n_blocks - b0);
        Arena ar = arena(c);
        ar.off = ws_off;  // the workspace below ws_off belongs to the caller
        u64 *T3 = ar.take((size_t)nb * 3 * lc);
        u64 *R = ar.take((size_t)nb * 2 * u1);
        if (!T3 || !R) return HE_ENOMEM;
        u64 *u = out + b0 * obs;
        hek::tensor_b(c, l, nb, Z[b0].data, chunk == 1 ? 0 : zbs, zc, W->data, 0, wc, T3, 3 * lc, lc);
        TRY(relin_rescale_apply(c, ar, l, nb, T3, 3 * lc, keys->rlk, u, obs));
        TRY(slot_sum_hoisted(c, ar, l - 1, nb, u, obs, R, 2 * u1, unit, count, keys));
    }
    return last_error();
}

// the whole step; nchunk = 1 (plain: per-block operations) or n_blocks (batched)
// Seeded data blocks (he_lr_grad_step_seeded): b-parts b + blk * bs at one
// level and scale, uniform parts from (seed, index0 + blk).
struct SeedData {
    const u64 *b = nullptr;
    long long bs = 0;
    u64 seed = 0;
    uint32_t index0 = 0;
    int level = 0;
    double scale = 0.0;
};

// full ciphertexts of seeded blocks [b0, b0 + nb) into E (stride 2 (level+1) N)
void expand_seeded(he_ctx *c, const SeedData &sd, int b0, int nb, u64 *E)
{
    const long long lc = (long long)(sd.level + 1) * c->N;
    hek::ewise(c, 4, sd.level, nb, 1, sd.b + b0 * sd.bs, sd.bs, 0, nullptr, 0, 0, E, 2 * lc, 0, 0);
    hek::seeded_a(c, sd.seed, sd.index0 + (uint32_t)b0, nb, sd.level, E + lc, 2 * lc);
}

he_status step_impl(he_ctx *c, const he_lr_plan &pl, const he_ct *Z, int n_blocks, long long zbs, const BabyData &bd,
                    const TermData &td, const he_ct *W, const he_pt *mask, int cols, int rows, const he_keys *keys,
                    int chunk, he_ct *W_out, he_ct *G_out, const SeedData *sd = nullptr)
{
    const long long N = c->N;
    const int l = W->level;
    Arena ar = arena(c);
    StepBufs s;
    const bool fm = pl.layout == HE_LAYOUT_FEATURES;
    u64 *E = nullptr;  // one chunk of seeded blocks, expanded
    if (sd) {
        E = ar.take((size_t)chunk * 2 * (sd->level + 1) * N);
        if (!E) return HE_ENOMEM;
    }
    TRY(step_alloc(c, ar, l, chunk, pl.layout, bd.n_baby, s));
    if (bd.n_baby > 1) {
        // the baby steps of W, once per step for every block: Rot(W, j u), j = 1 .. n_baby - 1
        // (u = rows feature-major, 1 row-major)
        const long long lc = (l + 1) * N;
        const long long unit = fm ? rows : 1;
        hek::EntryKeys ek;
        hek::EntryGal eg;
        for (int j = 1; j < bd.n_baby; ++j) {
            eg.g[j - 1] = galois_of(c, (long long)j * unit);
            ek.k[j - 1] = find_rot_key(keys, eg.g[j - 1]);
        }
        TRY(rotate_multi_apply(c, ar, l, bd.n_baby - 1, W->data, 0, eg, ek, s.Wr, 2 * lc));
    }
    for (int b0 = 0; b0 < n_blocks; b0 += chunk) {
        int nb = std::min(chunk, n_blocks - b0);
        long long bs = zbs;
        if (chunk == 1) bs = 0;
        if (sd) {
            // this chunk's blocks as full ciphertexts, then the same per-block kernels
            expand_seeded(c, *sd, b0, nb, E);
            const he_ct ze{E, sd->level, 0, sd->scale};
            const long long es = 2LL * (sd->level + 1) * N;
            if (fm)
                TRY(step_blocks_features(c, ar, s, pl, &ze, es, 0, nb, W, cols, rows, keys, b0 > 0, bd, td));
            else
                TRY(step_blocks(c, ar, s, pl, &ze, es, 0, nb, W, mask, cols, keys, b0 > 0, bd, td));
            continue;
        }
        if (fm)
            TRY(step_blocks_features(c, ar, s, pl, Z, bs, b0, nb, W, cols, rows, keys, b0 > 0, bd, td));
        else
            TRY(step_blocks(c, ar, s, pl, Z, bs, b0, nb, W, mask, cols, keys, b0 > 0, bd, td));
    }
    const long long g1 = (long long)(l - 3) * N;  // component stride at level l-4
    {
        // one relinearisation of the summed degree-4 terms: (g0, g1) plus the
        // key switches of g2, g3, g4 from s^2, s^3, s^4; then one rescale
        const int lg = fm ? l - 2 : l - 3;
        const long long x1 = (long long)(lg + 1) * N;
        // the three key switches as one batch of three entries (per-entry keys),
        // then (g0, g1) plus their sum
        hek::EntryKeys ek;
        ek.k[0] = keys->rlk;
        ek.k[1] = keys->rlk3;
        ek.k[2] = keys->rlk4;
        const size_t mark = ar.off;
        u64 *ksx = ar.take((size_t)6 * x1);
        if (!ksx) return HE_ENOMEM;
        TRY(ks_apply(c, ar, lg, 3, s.G5 + 2 * x1, x1, nullptr, nullptr, 0, 0, 0, ksx, 2 * x1, x1, &ek));
        hek::ewise(c, 0, lg, 1, 2, s.G5, 0, x1, ksx, 0, x1, s.U0, 0, x1, 0);
        for (int e = 1; e < 3; ++e)
            hek::ewise(c, 0, lg, 1, 2, s.U0, 0, x1, ksx + 2 * e * x1, 0, x1, s.U0, 0, x1, 0);
        ar.off = mark;
        TRY(rescale_apply(c, ar, lg, 1, s.U0, 2 * x1, s.G, 2LL * lg * N));
    }
    u64 *g = s.G;
    if (fm) {
        // sum inside each feature block (level l-3), mask slots j r, rescale to
        // level l-4, replicate over the block
        const long long h1 = (long long)(l - 2) * N;
        TRY(slot_sum_hoisted(c, ar, l - 3, 1, s.G, 2 * h1, s.Rg, 2 * h1, +1, rows, keys));
        hek::ewise(c, 3, l - 3, 1, 2, s.G, 2 * h1, h1, mask->data, 0, 0, s.G, 2 * h1, h1, 0);
        TRY(rescale_apply(c, ar, l - 3, 1, s.G, 2 * h1, s.Gm, 2 * g1));
        TRY(slot_sum_hoisted(c, ar, l - 4, 1, s.Gm, 2 * g1, s.Rg, 2 * g1, -1, rows, keys));
        g = s.Gm;
    } else {
        // row sum: G = sum_{j < rows} Rot(G, j cols), grouped hoisted sums   (level l-4)
        const long long o1 = (long long)(l - 3) * N;
        TRY(slot_sum_hoisted(c, ar, l - 4, 1, s.G, 2 * o1, s.Rg, 2 * o1, cols, rows, keys));
    }
    if (G_out) hek::ewise(c, 4, l - 4, 1, 2, g, 2 * g1, g1, nullptr, 0, 0, G_out->data, 2 * g1, g1, 0);
    // W' = RS(kW W) + g
    TRY(rescale_apply(c, ar, l - 3, 1, W->data, 0, W_out->data, 2 * g1, 2, &pl.kw, (l + 1) * N));
    hek::ewise(c, 0, l - 4, 1, 2, W_out->data, 2 * g1, g1, g, 2 * g1, g1, W_out->data, 2 * g1, g1, 0);
    return last_error();
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *he_strerror(he_status s)
{
    switch (s) {
    case HE_OK: return "ok";
    case HE_EINVAL: return "invalid argument";
    case HE_ENOMEM: return "out of memory";
    case HE_ELEVEL: return "level out of range or mismatched";
    case HE_ESCALE: return "scale mismatch or scale plan out of range";
    case HE_EKEY: return "required evaluation key absent";
    case HE_EDEVICE: return "HIP runtime error";
    }
    return "unknown status";
}

he_status he_ctx_create(const he_params *prm, he_alloc_fn alloc, he_free_fn release, void *alloc_user,
                        void *hip_stream, he_ctx **out)
{
    if (!prm || !out) return HE_EINVAL;
    *out = nullptr;
    if (prm->log_n < 10 || prm->log_n > 16 || prm->n_q < 2 || prm->n_q > 40 || prm->n_special < 1 ||
        prm->n_special > 12 || prm->alpha < 1 || prm->alpha > prm->n_special || prm->log_delta < 20 ||
        prm->log_delta > 50 || prm->n_q + prm->n_special > HE_MAXP)
        return HE_EINVAL;
    int dnum = (prm->n_q + prm->alpha - 1) / prm->alpha;
    if (dnum > HE_MAXBETA) return HE_EINVAL;
    std::unique_ptr<he_ctx> c(new (std::nothrow) he_ctx());
    if (!c) return HE_ENOMEM;
    c->prm = *prm;
    c->logN = prm->log_n;
    c->N = 1 << prm->log_n;
    c->nq = prm->n_q;
    c->nk = prm->n_special;
    c->np = c->nq + c->nk;
    c->alpha = prm->alpha;
    c->dnum = dnum;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) return HE_EDEVICE;
    TRY(noalloc_setup(c->device, &c->noalloc));
    c->alloc_fn = alloc;
    c->free_fn = release;
    c->alloc_user = alloc_user;
    c->q.assign(c->np, 0);
    if (hehost::gen_primes(c->nq, c->nk, prm->log_delta, c->q.data()) != 0) return HE_EINVAL;
    c->psi.resize(c->np);
    for (int i = 0; i < c->np; ++i) c->psi[i] = hehost::find_psi(c->q[i], c->logN);
    he_status st = build_tables(c.get());
    if (st != HE_OK) {
        he_ctx_destroy(c.release());
        return st;
    }
    *out = c.release();
    return HE_OK;
}

he_status he_params_primes(const he_params *prm, uint64_t *out, int n)
{
    if (!prm || !out || prm->n_q < 1 || prm->n_special < 0 || n < prm->n_q + prm->n_special) return HE_EINVAL;
    return hehost::gen_primes(prm->n_q, prm->n_special, prm->log_delta, out) == 0 ? HE_OK : HE_EINVAL;
}

he_status he_ctx_destroy(he_ctx *c)
{
    if (!c) return HE_EINVAL;
    (void)hipDeviceSynchronize();
    for (auto &kv : c->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    for (void *p : c->owned) dev_free(c, p);
    dev_free(c, c->ws);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->sub_ev) {
        (void)hipEventSynchronize(c->sub_ev);
        (void)hipEventDestroy(c->sub_ev);
    }
    if (c->sub_host) (void)hipHostFree(c->sub_host);
    for (int i = 0; i < he_ctx::SUBMIT_LANES; ++i) {
        if (c->lane[i]) (void)hipStreamDestroy(c->lane[i]);
        if (c->lane_ev[i]) (void)hipEventDestroy(c->lane_ev[i]);
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    for (he_keys *k : c->keys_made) k->ctx = nullptr;  // released later, they no longer reach this context
    for (const KRec &r : c->kt.recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : c->kt.pool) (void)hipEventDestroy(e);
    delete c;
    return HE_OK;
}

he_status he_ctx_set_ntt(he_ctx *c, int persistent, int wg_per_xcd, int lag, int min_limbs)
{
    if (!c || persistent < 0 || persistent > 5 || wg_per_xcd < 1 || wg_per_xcd > 1024 || lag < 1 || lag >= PS_SLOTS ||
        min_limbs < 1)
        return HE_EINVAL;
    if (persistent == 1 && !c->persist.slots) return HE_EINVAL;
    if (c->capturing) return HE_EINVAL;
    if ((persistent == 2 || persistent == 3) && !c->persist.limb_scratch) {
        // the one-workgroup-per-limb form's scratch limbs, made on first use
        if (!c->persist.slots || c->logN < 12) return HE_EINVAL;
        c->persist.limb_scratch = (u64 *)dev_alloc(c, (size_t)c->persist.limb_wgs * c->N * 8);
        if (!c->persist.limb_scratch) return HE_ENOMEM;
        c->owned.push_back(c->persist.limb_scratch);
    }
    // captured graphs hold the launch shapes of the old setting
    TRY(drop_graphs(c, 0));
    c->persist.on = persistent;
    c->persist.wg_per_xcd = wg_per_xcd;
    c->persist.lag = lag;
    c->persist.min_limbs = min_limbs;
    return HE_OK;
}

he_status he_ctx_set_stream(he_ctx *c, void *s)
{
    if (!c) return HE_EINVAL;
    c->stream = (hipStream_t)s;
    return HE_OK;
}

he_status he_ctx_primes(const he_ctx *c, uint64_t *out, int n)
{
    if (!c || !out || n < c->np) return HE_EINVAL;
    std::copy(c->q.begin(), c->q.end(), out);
    return HE_OK;
}

he_status he_ctx_trim(he_ctx *c)
{
    if (!c) return HE_EINVAL;
    TRY(drop_graphs(c, 0));
    if (c->ws) {
        HIPCHK(hipStreamSynchronize(c->stream));
        dev_free(c, c->ws);
    }
    c->ws = nullptr;
    c->ws_bytes = 0;
    return HE_OK;
}

size_t he_ct_bytes(const he_ctx *c, int level) { return c ? (size_t)2 * (level + 1) * c->N * 8 : 0; }
size_t he_pt_bytes(const he_ctx *c, int level) { return c ? (size_t)(level + 1) * c->N * 8 : 0; }
size_t he_ct3_bytes(const he_ctx *c, int level) { return c ? (size_t)3 * (level + 1) * c->N * 8 : 0; }

size_t he_keys_bytes(const he_ctx *c, int n_rot)
{
    if (!c || n_rot < 0) return 0;
    const size_t evk = (size_t)c->dnum * 2 * c->np * c->N * 8;
    const size_t pk = (size_t)2 * c->nq * c->N * 8;
    return (size_t)c->np * c->N * 8 + evk * (3 + (size_t)n_rot) + pk;
}

// Keys are valid for every context of their parameter set (ring degree,
// prime chain, digit width): their layout and residues depend on nothing else.
static bool keys_ok(const he_ctx *c, const he_keys *k)
{
    if (k->logN != c->logN || k->nq != c->nq || k->nk != c->nk || k->alpha != c->alpha) return false;
    for (int i = 0; i < c->np; ++i)
        if (k->q[i] != c->q[i]) return false;
    return true;
}

he_status he_keygen(he_ctx *c, uint64_t seed, const int32_t *rot_steps, int n_rot, void *key_buf,
                    size_t key_buf_bytes, he_keys **out)
{
    if (!c || !out || !key_buf || n_rot < 0 || (n_rot > 0 && !rot_steps)) return HE_EINVAL;
    if (key_buf_bytes < he_keys_bytes(c, n_rot)) return HE_EINVAL;
    *out = nullptr;
    const size_t N = c->N;
    const int np = c->np;
    const size_t evk_n = (size_t)c->dnum * 2 * np * N;
    TRY(ensure_ws(c, (al((size_t)np * N) * 4) * 8 + 4096));
    std::unique_ptr<he_keys> k(new (std::nothrow) he_keys());
    if (!k) return HE_ENOMEM;
    static std::atomic<uint64_t> next_gen{1};
    k->ctx = c;
    k->logN = c->logN;
    k->nq = c->nq;
    k->nk = c->nk;
    k->alpha = c->alpha;
    for (int i = 0; i < c->np; ++i) k->q[i] = c->q[i];
    k->gen = next_gen++;
    k->sk = (u64 *)key_buf;
    k->rlk = k->sk + (size_t)np * N;
    k->rlk3 = k->rlk + evk_n;
    k->rlk4 = k->rlk3 + evk_n;
    // secret: ternary, 64 nonzero coefficients (host ChaCha20), residues, NTT
    std::vector<i64> s(N);
    hehost::sample_hwt(seed, c->logN, std::min(64, (int)N), s.data());
    Arena ar = arena(c);
    u64 *sd = ar.take(N);
    u64 *sp = ar.take((size_t)np * N);
    u64 *sq = ar.take((size_t)np * N);
    if (!sd || !sp || !sq) return HE_ENOMEM;
    HIPCHK(hipMemcpyAsync(sd, s.data(), N * 8, hipMemcpyHostToDevice, c->stream));
    std::vector<int> ids = identity_positions(np);
    hek::int_to_rns(c, (const i64 *)sd, np, ids.data(), k->sk);
    hek::ntt_batch(c, k->sk, 0, 0, 1, 1, 0, np, c->nq - 1, +1, nullptr, false);
    // relinearisation key: s' = s^2
    hek::ewise(c, 3, np - 1, 1, 1, k->sk, 0, 0, k->sk, 0, 0, sp, 0, 0, 0);
    TRY(make_evk(c, ar, seed, 0, k->sk, sp, k->rlk));
    // keys for s^3 = s^2 s and s^4 = s^2 s^2 (key ids 2 and 4: even, so apart
    // from every Galois element)
    hek::ewise(c, 3, np - 1, 1, 1, sp, 0, 0, k->sk, 0, 0, sq, 0, 0, 0);
    TRY(make_evk(c, ar, seed, 2, k->sk, sq, k->rlk3));
    hek::ewise(c, 3, np - 1, 1, 1, sp, 0, 0, sp, 0, 0, sq, 0, 0, 0);
    TRY(make_evk(c, ar, seed, 4, k->sk, sq, k->rlk4));
    // public key (-a s + e, a) over q_0 .. q_{nq-1} (Alg. 1's worker key)
    k->pk = k->rlk4 + evk_n;
    {
        u64 *pb = k->pk, *pa = k->pk + (size_t)c->nq * N;
        std::vector<int> qi = identity_positions(c->nq);
        hek::sample_uniform(c, seed, ST_PK_A, 0, 0, c->nq, qi.data(), pa);
        hek::ntt_batch(c, pa, 0, 0, 1, 1, 0, c->nq, c->nq - 1, +1, nullptr, false);
        hek::sample_cbd(c, seed, ST_PK_E, 0, 0, c->nq, qi.data(), sq);
        hek::ntt_batch(c, sq, 0, 0, 1, 1, 0, c->nq, c->nq - 1, +1, nullptr, false);
        hek::enc_combine(c, c->nq - 1, pa, k->sk, sq, nullptr, pb);
    }
    u64 *next = k->pk + (size_t)2 * c->nq * N;
    for (int r = 0; r < n_rot; ++r) {
        u64 g = galois_of(c, rot_steps[r]);
        if (g == 1 || k->rot.count(g)) continue;
        hek::automorph_b(c, 1, np, k->sk, 0, 0, sp, 0, 0, g);  // s(X^g): one component only is used
        TRY(make_evk(c, ar, seed, (uint32_t)g, k->sk, sp, next));
        k->rot[g] = next;
        next += evk_n;
    }
    HIPCHK(hipStreamSynchronize(c->stream));  // the host secret buffer is released below
    TRY(last_error());
    c->keys_made.insert(k.get());
    *out = k.release();
    return HE_OK;
}

he_status he_keys_destroy(he_keys *k)
{
    if (!k) return HE_EINVAL;
    // graphs captured with these keys hold their device addresses: a later key
    // set may be given the same host handle or buffer
    he_status st = HE_OK;
    if (k->ctx) {  // the making context is still alive (its destroy clears ctx)
        st = drop_graphs(k->ctx, k->gen);
        k->ctx->keys_made.erase(k);
    }
    delete k;
    if (st != HE_OK) return st;
    return HE_OK;
}

he_status he_keys_download(he_ctx *c, const he_keys *k, int64_t which, uint64_t *host)
{
    if (!c || !k || !host) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    const size_t N = c->N;
    const int np = c->np;
    const u64 *src;
    int npoly;
    int nlimb = np;
    if (which == -2) {
        src = k->sk;
        npoly = 1;
    } else if (which == -5) {
        src = k->pk;
        npoly = 2;
        nlimb = c->nq;
    } else {
        src = which == -1 ? k->rlk : which == -3 ? k->rlk3 : which == -4 ? k->rlk4 : find_rot_key(k, (u64)which);
        if (!src) return HE_EKEY;
        npoly = c->dnum * 2;
    }
    const size_t n = (size_t)npoly * nlimb * N;
    TRY(ensure_ws(c, al(n) * 8 + 4096));
    Arena ar = arena(c);
    u64 *t = ar.take(n);
    HIPCHK(hipMemcpyAsync(t, src, n * 8, hipMemcpyDeviceToDevice, c->stream));
    hek::ntt_batch(c, t, (long long)nlimb * N, 0, npoly, 1, 0, nlimb, c->nq - 1, -1, nullptr, false);
    HIPCHK(hipMemcpyAsync(host, t, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return last_error();
}

he_status he_encode(he_ctx *c, const double *re, const double *im, int n, double scale, int64_t *coeffs)
{
    if (!c || !re || !coeffs || n < 0 || n > c->N / 2 || !(scale > 0)) return HE_EINVAL;
    return hehost::encode(c->logN, re, im, n, scale, coeffs) == 0 ? HE_OK : HE_EINVAL;
}

he_status he_decode(he_ctx *c, const double *coeffs, double scale, int n, double *re, double *im)
{
    if (!c || !coeffs || !re || n < 0 || n > c->N / 2 || !(scale > 0)) return HE_EINVAL;
    hehost::decode(c->logN, coeffs, scale, n, re, im);
    return HE_OK;
}

he_status he_pt_load(he_ctx *c, const int64_t *coeffs, int level, double scale, he_pt *out)
{
    if (!c || !coeffs || !out || !out->data || level < 0 || level >= c->nq) return HE_EINVAL;
    const size_t N = c->N;
    TRY(ensure_ws(c, al(N) * 8 + 4096));
    Arena ar = arena(c);
    u64 *m = ar.take(N);
    HIPCHK(hipMemcpyAsync(m, coeffs, N * 8, hipMemcpyHostToDevice, c->stream));
    std::vector<int> ids = identity_positions(level + 1);
    hek::int_to_rns(c, (const i64 *)m, level + 1, ids.data(), out->data);
    hek::ntt_batch(c, out->data, 0, 0, 1, 1, 0, level + 1, level, +1, nullptr, false);
    HIPCHK(hipStreamSynchronize(c->stream));
    out->level = level;
    out->scale = scale;
    return last_error();
}

he_status he_encrypt(he_ctx *c, const he_pt *pt, const he_keys *k, int use_sk, uint64_t seed, uint32_t index,
                     he_ct *out)
{
    if (!c || !pt || !k || !out || !pt->data || !out->data || pt->level < 0 || pt->level >= c->nq) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    const int l = pt->level;
    const size_t N = c->N;
    const size_t n = (size_t)(l + 1) * N;
    u64 *b = out->data, *a = out->data + n;
    std::vector<int> ids = identity_positions(l + 1);
    if (!use_sk) {
        // (v pk_b + e0 + m, v pk_a + e1), v ternary, e0 and e1 centred binomial
        TRY(ensure_ws(c, 3 * al(n) * 8 + 4096));
        Arena ar = arena(c);
        u64 *v = ar.take(n), *e0 = ar.take(n), *e1 = ar.take(n);
        if (!v || !e0 || !e1) return HE_ENOMEM;
        hek::sample_ternary(c, seed, ST_ENC_V, index, 0, l + 1, ids.data(), v);
        hek::sample_cbd(c, seed, ST_ENC_E0, index, 0, l + 1, ids.data(), e0);
        hek::sample_cbd(c, seed, ST_ENC_E1, index, 0, l + 1, ids.data(), e1);
        hek::ntt_batch(c, v, 0, 0, 1, 1, 0, l + 1, l, +1, nullptr, false);
        hek::ntt_batch(c, e0, 0, 0, 1, 1, 0, l + 1, l, +1, nullptr, false);
        hek::ntt_batch(c, e1, 0, 0, 1, 1, 0, l + 1, l, +1, nullptr, false);
        hek::encpk_combine(c, l, v, k->pk, e0, e1, pt->data, b, a);
        out->level = l;
        out->scale = pt->scale;
        return last_error();
    }
    TRY(ensure_ws(c, al(n) * 8 + 4096));
    Arena ar = arena(c);
    u64 *e = ar.take(n);
    hek::sample_uniform(c, seed, ST_ENC_A, index, 0, l + 1, ids.data(), a);
    hek::ntt_batch(c, a, 0, 0, 1, 1, 0, l + 1, l, +1, nullptr, false);
    hek::sample_cbd(c, seed, ST_ENC_E0, index, 0, l + 1, ids.data(), e);
    hek::ntt_batch(c, e, 0, 0, 1, 1, 0, l + 1, l, +1, nullptr, false);
    hek::enc_combine(c, l, a, k->sk, e, pt->data, b);
    out->level = l;
    out->scale = pt->scale;
    return last_error();
}

he_status he_encrypt_seeded(he_ctx *c, const he_pt *pt, const he_keys *k, uint64_t seed, uint32_t index,
                            he_ct_seeded *out)
{
    if (!c || !pt || !k || !out || !pt->data || !out->b || pt->level < 0 || pt->level >= c->nq) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    const int l = pt->level;
    const size_t n = (size_t)(l + 1) * c->N;
    TRY(ensure_ws(c, 2 * al(n) * 8 + 4096));
    Arena ar = arena(c);
    u64 *a = ar.take(n), *e = ar.take(n);
    if (!a || !e) return HE_ENOMEM;
    std::vector<int> ids = identity_positions(l + 1);
    hek::seeded_a(c, seed, index, 1, l, a, 0);  // already in the evaluation domain
    hek::sample_cbd(c, seed, ST_ENC_E0, index, 0, l + 1, ids.data(), e);
    hek::ntt_batch(c, e, 0, 0, 1, 1, 0, l + 1, l, +1, nullptr, false);
    hek::enc_combine(c, l, a, k->sk, e, pt->data, out->b);
    out->level = l;
    out->scale = pt->scale;
    out->seed = seed;
    out->index = index;
    return last_error();
}

he_status he_ct_expand(he_ctx *c, const he_ct_seeded *in, int n, he_ct *out)
{
    if (!c || !in || !out || n < 0) return HE_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!in[i].b || !out[i].data || in[i].level < 0 || in[i].level >= c->nq) return HE_EINVAL;
    for (int i = 0; i < n; ++i) {
        SeedData sd;
        sd.b = in[i].b;
        sd.seed = in[i].seed;
        sd.index0 = in[i].index;
        sd.level = in[i].level;
        expand_seeded(c, sd, 0, 1, out[i].data);
        out[i].level = in[i].level;
        out[i].scale = in[i].scale;
    }
    return last_error();
}

// the first nl limbs (coefficient form) of the decryption, to host
static he_status decrypt_limbs(he_ctx *c, const he_ct *ct, const he_keys *k, int nl, uint64_t *host)
{
    const int l = ct->level;
    const size_t N = c->N;
    TRY(ensure_ws(c, al((size_t)(l + 1) * N) * 8 + 4096));
    Arena ar = arena(c);
    u64 *m = ar.take((size_t)(l + 1) * N);
    hek::dec_combine(c, l, ct->data, k->sk, m);
    hek::ntt_batch(c, m, 0, 0, 1, 1, 0, nl, l, -1, nullptr, false);
    HIPCHK(hipMemcpyAsync(host, m, (size_t)nl * N * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return last_error();
}

he_status he_decrypt(he_ctx *c, const he_ct *ct, const he_keys *k, uint64_t *host)
{
    if (!c || !ct_ok(c, ct) || !k || !host) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    return decrypt_limbs(c, ct, k, ct->level + 1, host);
}

he_status he_decrypt_decode(he_ctx *c, const he_ct *ct, const he_keys *k, int n, double *re, double *im)
{
    if (!c || !ct_ok(c, ct) || !k || !re || n < 0 || n > c->N / 2) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    const size_t N = c->N;
    // the message is centred below q0 q1 / 2: the first two limbs determine it
    const int nl = std::min(2, ct->level + 1);
    thread_local std::vector<u64> res;
    thread_local std::vector<double> m;
    res.resize((size_t)nl * N);
    m.resize(N);
    TRY(decrypt_limbs(c, ct, k, nl, res.data()));
    const u64 q0 = c->q[0];
    if (nl == 1) {
        for (size_t x = 0; x < N; ++x) m[x] = res[x] > q0 / 2 ? -(double)(q0 - res[x]) : (double)res[x];
    } else {
        hehost::crt2_centred(res.data(), res.data() + N, N, q0, c->q[1], m.data());
    }
    hehost::decode(c->logN, m.data(), ct->scale, n, re, im);
    return HE_OK;
}

he_status he_ct_download(he_ctx *c, const he_ct *ct, uint64_t *host)
{
    if (!c || !ct_ok(c, ct) || !host) return HE_EINVAL;
    const size_t n = (size_t)2 * (ct->level + 1) * c->N;
    TRY(ensure_ws(c, al(n) * 8 + 4096));
    Arena ar = arena(c);
    u64 *t = ar.take(n);
    HIPCHK(hipMemcpyAsync(t, ct->data, n * 8, hipMemcpyDeviceToDevice, c->stream));
    const long long lc = (long long)(ct->level + 1) * c->N;
    hek::ntt_batch(c, t, 0, lc, 1, 2, 0, ct->level + 1, ct->level, -1, nullptr, false);
    HIPCHK(hipMemcpyAsync(host, t, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return last_error();
}

he_status he_ct_upload(he_ctx *c, const uint64_t *host, int level, double scale, he_ct *out)
{
    if (!c || !host || !out || !out->data || level < 0 || level >= c->nq) return HE_EINVAL;
    const size_t n = (size_t)2 * (level + 1) * c->N;
    HIPCHK(hipMemcpyAsync(out->data, host, n * 8, hipMemcpyHostToDevice, c->stream));
    const long long lc = (long long)(level + 1) * c->N;
    hek::ntt_batch(c, out->data, 0, lc, 1, 2, 0, level + 1, level, +1, nullptr, false);
    HIPCHK(hipStreamSynchronize(c->stream));
    out->level = level;
    out->scale = scale;
    return last_error();
}

he_status he_mul(he_ctx *c, const he_ct *x, const he_ct *y, he_ct3 *out)
{
    if (!c || !ct_ok(c, x) || !ct_ok(c, y) || !out || !out->data) return HE_EINVAL;
    if (x->level != y->level) return HE_ELEVEL;
    const int l = x->level;
    const long long lc = (long long)(l + 1) * c->N;
    hek::tensor_b(c, l, 1, x->data, 0, lc, y->data, 0, lc, out->data, 0, lc);
    out->level = l;
    out->scale = x->scale * y->scale;
    return last_error();
}

he_status he_relin(he_ctx *c, const he_ct3 *in, const he_keys *k, he_ct *out)
{
    if (!c || !in || !in->data || !k || !out || !out->data || in->level < 0 || in->level >= c->nq) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    const int l = in->level;
    TRY(ensure_ws(c, ks_scratch(c, l, 1) * 8 + 4096));
    Arena ar = arena(c);
    TRY(relin_apply(c, ar, l, 1, in->data, 0, k->rlk, out->data, 0));
    out->level = l;
    out->scale = in->scale;
    return HE_OK;
}

he_status he_rescale(he_ctx *c, const he_ct *in, he_ct *out)
{
    if (!c || !ct_ok(c, in)) return HE_EINVAL;
    if (in->level < 1) return HE_ELEVEL;
    if (!out || !out->data) return HE_EINVAL;
    const int l = in->level;
    const double sc = in->scale / (double)c->q[l];
    TRY(ensure_ws(c, rescale_scratch(c, l, 1) * 8 + 4096));
    Arena ar = arena(c);
    TRY(rescale_apply(c, ar, l, 1, in->data, 0, out->data, 0));
    out->level = l - 1;
    out->scale = sc;
    return HE_OK;
}

he_status he_rotate(he_ctx *c, const he_ct *in, int steps, const he_keys *k, he_ct *out)
{
    if (!c || !ct_ok(c, in) || !k || !out || !out->data || out->data == in->data) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    const int l = in->level;
    const u64 g = galois_of(c, steps);
    const double sc = in->scale;
    if (g == 1) {
        const long long lc = (long long)(l + 1) * c->N;
        hek::ewise(c, 4, l, 1, 2, in->data, 0, lc, nullptr, 0, 0, out->data, 0, lc, 0);
    } else {
        const u64 *key = find_rot_key(k, g);
        if (!key) return HE_EKEY;
        TRY(ensure_ws(c, rotate_scratch(c, l, 1) * 8 + 4096));
        Arena ar = arena(c);
        TRY(rotate_apply(c, ar, l, 1, in->data, 0, g, key, out->data, 0));
    }
    out->level = l;
    out->scale = sc;
    return last_error();
}

he_status he_rotate_noalloc(he_ctx *c, const he_ct *in, int steps, const he_keys *k, he_ct *out)
{
    if (!c || !ct_ok(c, in) || !k || !out || !out->data || out->data == in->data) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    if (!c->noalloc) return HE_EDEVICE;
    const int l = in->level;
    const u64 g = galois_of(c, steps);
    const double sc = in->scale;
    if (g == 1) {
        const long long lc = (long long)(l + 1) * c->N;
        hek::ewise(c, 4, l, 1, 2, in->data, 0, lc, nullptr, 0, 0, out->data, 0, lc, 0);
    } else {
        const u64 *key = find_rot_key(k, g);
        if (!key) return HE_EKEY;
        // the same kernels as he_rotate, their buffers carved from the fixed array
        if (rotate_scratch(c, l, 1) * 8 > HE_NOALLOC_SCRATCH_BYTES) return HE_ENOMEM;
        Arena ar;
        ar.base = (char *)c->noalloc;
        ar.cap = HE_NOALLOC_SCRATCH_BYTES;
        TRY(rotate_apply(c, ar, l, 1, in->data, 0, g, key, out->data, 0));
    }
    out->level = l;
    out->scale = sc;
    return last_error();
}

size_t he_rotate_noalloc_bytes(const he_ctx *c, int level)
{
    if (!c || level < 0 || level >= c->nq) return 0;
    return rotate_scratch(c, level, 1) * 8;
}

he_status he_add(he_ctx *c, const he_ct *x, const he_ct *y, he_ct *out)
{
    if (!c || !ct_ok(c, x) || !ct_ok(c, y) || !out || !out->data) return HE_EINVAL;
    if (x->level != y->level) return HE_ELEVEL;
    if (x->scale != y->scale) return HE_ESCALE;
    const int l = x->level;
    const double sc = x->scale;
    const long long lc = (long long)(l + 1) * c->N;
    hek::ewise(c, 0, l, 1, 2, x->data, 0, lc, y->data, 0, lc, out->data, 0, lc, 0);
    out->level = l;
    out->scale = sc;
    return last_error();
}

he_status he_mul_int(he_ctx *c, const he_ct *x, int64_t k, double out_scale, he_ct *out)
{
    if (!c || !ct_ok(c, x) || !out || !out->data) return HE_EINVAL;
    if (k >= ((int64_t)1 << 62) || k <= -((int64_t)1 << 62)) return HE_ESCALE;
    const int l = x->level;
    const long long lc = (long long)(l + 1) * c->N;
    hek::ewise(c, 2, l, 1, 2, x->data, 0, lc, nullptr, 0, 0, out->data, 0, lc, k);
    out->level = l;
    out->scale = out_scale;
    return last_error();
}

he_status he_mul_plain(he_ctx *c, const he_ct *x, const he_pt *pt, he_ct *out)
{
    if (!c || !ct_ok(c, x) || !pt || !pt->data || !out || !out->data) return HE_EINVAL;
    if (pt->level != x->level) return HE_ELEVEL;
    const int l = x->level;
    const double sc = x->scale * pt->scale;
    const long long lc = (long long)(l + 1) * c->N;
    hek::ewise(c, 3, l, 1, 2, x->data, 0, lc, pt->data, 0, 0, out->data, 0, lc, 0);
    out->level = l;
    out->scale = sc;
    return last_error();
}

he_status he_drop_level(he_ctx *c, const he_ct *x, int level, he_ct *out)
{
    if (!c || !ct_ok(c, x) || !out || !out->data) return HE_EINVAL;
    if (level < 0 || level > x->level) return HE_ELEVEL;
    const long long xc = (long long)(x->level + 1) * c->N, oc = (long long)(level + 1) * c->N;
    const double sc = x->scale;
    if (out->data == x->data && level != x->level) {
        // component 1 moves down; one thread per coefficient walks limbs upward
        TRY(ensure_ws(c, al((size_t)(level + 1) * c->N) * 8 + 4096));
        Arena ar = arena(c);
        u64 *t = ar.take((size_t)(level + 1) * c->N);
        hek::ewise(c, 4, level, 1, 1, x->data + xc, 0, 0, nullptr, 0, 0, t, 0, 0, 0);
        hek::ewise(c, 4, level, 1, 1, t, 0, 0, nullptr, 0, 0, out->data + oc, 0, 0, 0);
    } else {
        hek::ewise(c, 4, level, 1, 2, x->data, 0, xc, nullptr, 0, 0, out->data, 0, oc, 0);
    }
    out->level = level;
    out->scale = sc;
    return last_error();
}

he_status he_plan_lr_step(const uint64_t *q, int n_q, int level, double s_z, double s_w, const double coef[4],
                          double eta_over_n, double w_decay, int layout, he_lr_plan *out)
{
    if (!q || !coef || !out || n_q < 1) return HE_EINVAL;
    return hehost::plan_lr_step(q, n_q, level, s_z, s_w, coef, eta_over_n, w_decay, layout, out);
}

// levels of the step's data terms Z3 and Z1 / Z2 for weights at level l
inline int z3_level(int l, bool fm) { return fm ? l - 1 : l - 2; }
inline int z1_level(int l, bool fm) { return fm ? l - 2 : l - 3; }

// n ciphertexts x[0..n) at one level and scale with one uniform stride (0 for n = 1)
he_status uniform_group(const he_ctx *c, const he_ct *x, int n, int level, double scale, long long &stride)
{
    stride = 0;
    for (int b = 0; b < n; ++b) {
        if (!ct_ok(c, &x[b])) return HE_EINVAL;
        if (x[b].level != level) return HE_ELEVEL;
        if (x[b].scale != scale) return HE_ESCALE;
        if (b == 1) stride = x[1].data - x[0].data;
        if (b > 1 && x[b].data - x[b - 1].data != stride) return HE_EINVAL;
    }
    if (n > 1 && stride < 2LL * (level + 1) * c->N) return HE_EINVAL;
    return HE_OK;
}

// The step's arguments checked before any launch (level, scale, stride and
// key errors), with its plan, block stride and baby / term data.
struct StepArgs {
    he_lr_plan pl;
    long long zbs = 0;
    BabyData bd;
    TermData td;
};

static he_status step_args(he_ctx *c, const he_ct *Z, int n_blocks, const he_ct *W, const he_pt *mask,
                           const double coef[4], double eta_over_n, double w_decay, int cols, int rows, int layout,
                           const he_ct *Zrot, int n_baby, const he_ct *Zk, const he_keys *k, int mode,
                           const he_ct *W_out, const he_ct *G_out, StepArgs &sa)
{
    if (!c || !Z || n_blocks < 1 || !ct_ok(c, W) || !mask || !mask->data || !coef || !k || mode < 0 || mode > 2)
        return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    if (layout != HE_LAYOUT_ROWS && layout != HE_LAYOUT_FEATURES) return HE_EINVAL;
    const bool fm = layout == HE_LAYOUT_FEATURES;
    if (n_baby < 1 || n_baby > HE_MAXBABY || (n_baby & (n_baby - 1)) || (n_baby > 1 && (n_baby > cols || !Zrot)))
        return HE_EINVAL;
    if (W->level < 4) return HE_ELEVEL;
    if (!W_out || !W_out->data || (G_out && !G_out->data)) return HE_EINVAL;
    if (cols < 1 || rows < 1 || (cols & (cols - 1)) || (rows & (rows - 1)) || (long long)cols * rows != c->N / 2)
        return HE_EINVAL;
    const int l = W->level;
    if (l < 4) return HE_ELEVEL;
    if (mask->level != (fm ? l - 3 : l - 1)) return HE_ELEVEL;
    const int lz = Z[0].level;
    const double sz = Z[0].scale;
    long long zbs = 0;
    for (int b = 0; b < n_blocks; ++b) {
        if (!ct_ok(c, &Z[b]) || Z[b].level != lz || Z[b].scale != sz) return Z[b].level != lz ? HE_ELEVEL : HE_EINVAL;
        if (b == 1) zbs = Z[1].data - Z[0].data;
        if (b > 1 && Z[b].data - Z[b - 1].data != zbs) return HE_EINVAL;  // one uniform block stride
    }
    if (lz < l) return HE_ELEVEL;
    if (mode > 0 && n_blocks > 1 && zbs < 2LL * (lz + 1) * c->N) return HE_EINVAL;
    sa.zbs = zbs;
    // baby-step copies: Zrot[b * (n_baby - 1) + j - 1] = Rot(Z[b], j rows), one level, one scale, uniform strides
    BabyData &bd = sa.bd;
    bd.n_baby = n_baby;
    if (n_baby > 1) {
        const int m = n_baby - 1, lr = Zrot[0].level;
        if (lr < l) return HE_ELEVEL;
        bd.zr = Zrot[0].data;
        bd.zrc = (long long)(lr + 1) * c->N;
        bd.zrs = m > 1 ? Zrot[1].data - Zrot[0].data : 0;
        bd.zrb = n_blocks > 1 ? Zrot[m].data - Zrot[0].data : 0;
        for (int b = 0; b < n_blocks; ++b)
            for (int j = 0; j < m; ++j) {
                const he_ct &z = Zrot[b * m + j];
                if (!ct_ok(c, &z) || z.level != lr || z.scale != sz) return z.level != lr ? HE_ELEVEL : HE_EINVAL;
                if (z.data != bd.zr + b * bd.zrb + j * bd.zrs) return HE_EINVAL;  // uniform strides
            }
        if (m > 1 && bd.zrs < 2 * bd.zrc) return HE_EINVAL;
        if (n_blocks > 1 && bd.zrb < (long long)m * 2 * bd.zrc) return HE_EINVAL;
    }
    he_lr_plan &pl = sa.pl;
    TRY(hehost::plan_lr_step(c->q.data(), c->nq, l, sz, W->scale, coef, eta_over_n, w_decay, layout, &pl));
    if (mask->scale != pl.s_mask) return HE_ESCALE;
    // precomputed data terms (he_lr_data_terms for this plan): Z3 group, Z1 group, Z2 group when k2 != 0
    TermData &td = sa.td;
    if (Zk) {
        long long s3, s1, s2;
        TRY(uniform_group(c, Zk, n_blocks, z3_level(l, fm), pl.s_z3, s3));
        TRY(uniform_group(c, Zk + n_blocks, n_blocks, z1_level(l, fm), pl.s_z1, s1));
        td.z3 = Zk[0].data;
        td.z3s = s3;
        td.z1 = Zk[n_blocks].data;
        td.z1s = s1;
        if (pl.k2 != 0) {
            TRY(uniform_group(c, Zk + 2 * n_blocks, n_blocks, z1_level(l, fm), pl.s_z2, s2));
            if (s2 != s1) return HE_EINVAL;
            td.z2 = Zk[2 * n_blocks].data;
        }
    }
    // every key the step needs, checked before any launch
    return step_keys(c, k, layout, cols, rows, n_baby);
}

he_status he_lr_grad_step(he_ctx *c, const he_ct *Z, int n_blocks, const he_ct *W, const he_pt *mask,
                          const double coef[4], double eta_over_n, double w_decay, int cols, int rows, int layout,
                          const he_ct *Zrot, int n_baby, const he_ct *Zk, const he_keys *k, int mode, he_ct *W_out,
                          he_ct *G_out)
{
    StepArgs sa;
    TRY(step_args(c, Z, n_blocks, W, mask, coef, eta_over_n, w_decay, cols, rows, layout, Zrot, n_baby, Zk, k, mode,
                  W_out, G_out, sa));
    const he_lr_plan &pl = sa.pl;
    const long long zbs = sa.zbs;
    const BabyData &bd = sa.bd;
    const TermData &td = sa.td;
    const int l = W->level;
    const int lz = Z[0].level;
    const int chunk = mode == 0 ? 1 : n_blocks;
    TRY(ensure_ws(c, step_bytes(c, l, chunk, layout, n_baby)));
    if (mode == 2) {
        std::ostringstream key;
        key << "step:" << (const void *)Z[0].data << ':' << zbs << ':' << n_blocks << ':' << lz << ':'
            << (const void *)W->data << ':' << l << ':' << (const void *)mask->data << ':' << cols << ':'
            << k->gen << ':' << (const void *)k->sk << ':' << (const void *)W_out->data << ':'
            << (const void *)(G_out ? G_out->data : nullptr) << ':' << pl.k0 << ':' << pl.k1 << ':' << pl.k2 << ':'
            << pl.k3 << ':' << pl.kb1 << ':' << pl.kw << ':' << (const void *)c->ws << ':' << layout << ':' << n_baby
            << ':' << (const void *)bd.zr << ':' << bd.zrb << ':' << bd.zrs << ':' << bd.zrc << ':'
            << (const void *)td.z3 << ':' << td.z3s << ':' << (const void *)td.z1 << ':' << td.z1s << ':'
            << (const void *)td.z2;
        TRY(run_graph(c, key.str(), k->gen, [&] {
            return step_impl(c, pl, Z, n_blocks, zbs, bd, td, W, mask, cols, rows, k, chunk, W_out, G_out);
        }));
    } else {
        TRY(step_impl(c, pl, Z, n_blocks, zbs, bd, td, W, mask, cols, rows, k, chunk, W_out, G_out));
    }
    W_out->level = l - 4;
    W_out->scale = pl.s_g;
    if (G_out) {
        G_out->level = l - 4;
        G_out->scale = pl.s_g;
    }
    return last_error();
}

he_status he_lr_grad_step_seeded(he_ctx *c, const he_ct_seeded *Z, int n_blocks, const he_ct *W, const he_pt *mask,
                                 const double coef[4], double eta_over_n, double w_decay, int cols, int rows,
                                 int layout, int chunk, const he_keys *k, he_ct *W_out, he_ct *G_out)
{
    if (!c || !Z || n_blocks < 1 || !ct_ok(c, W) || !mask || !mask->data || !coef || !k || chunk < 1 ||
        chunk > n_blocks)
        return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    if (layout != HE_LAYOUT_ROWS && layout != HE_LAYOUT_FEATURES) return HE_EINVAL;
    const bool fm = layout == HE_LAYOUT_FEATURES;
    if (!W_out || !W_out->data || (G_out && !G_out->data)) return HE_EINVAL;
    if (cols < 1 || rows < 1 || (cols & (cols - 1)) || (rows & (rows - 1)) || (long long)cols * rows != c->N / 2)
        return HE_EINVAL;
    const int l = W->level;
    if (l < 4) return HE_ELEVEL;
    if (mask->level != (fm ? l - 3 : l - 1)) return HE_ELEVEL;
    SeedData sd;
    sd.b = Z[0].b;
    sd.level = Z[0].level;
    sd.scale = Z[0].scale;
    sd.seed = Z[0].seed;
    sd.index0 = Z[0].index;
    for (int b = 0; b < n_blocks; ++b) {
        const he_ct_seeded &z = Z[b];
        if (!z.b || z.level != sd.level) return z.b ? HE_ELEVEL : HE_EINVAL;
        if (z.scale != sd.scale || z.seed != sd.seed || z.index != sd.index0 + (uint32_t)b) return HE_EINVAL;
        if (b == 1) sd.bs = Z[1].b - Z[0].b;
        if (b > 1 && Z[b].b - Z[b - 1].b != sd.bs) return HE_EINVAL;
    }
    if (sd.level < l || sd.level >= c->nq) return HE_ELEVEL;
    if (n_blocks > 1 && sd.bs < (long long)(sd.level + 1) * c->N) return HE_EINVAL;
    he_lr_plan pl;
    TRY(hehost::plan_lr_step(c->q.data(), c->nq, l, sd.scale, W->scale, coef, eta_over_n, w_decay, layout, &pl));
    if (mask->scale != pl.s_mask) return HE_ESCALE;
    TRY(step_keys(c, k, layout, cols, rows, 1));
    TRY(ensure_ws(c, step_bytes(c, l, chunk, layout, 1) + al((size_t)chunk * 2 * (sd.level + 1) * c->N) * 8));
    BabyData bd;
    TermData td;
    TRY(step_impl(c, pl, nullptr, n_blocks, 0, bd, td, W, mask, cols, rows, k, chunk, W_out, G_out, &sd));
    W_out->level = l - 4;
    W_out->scale = pl.s_g;
    if (G_out) {
        G_out->level = l - 4;
        G_out->scale = pl.s_g;
    }
    return last_error();
}

size_t he_lr_step_seeded_bytes(const he_ctx *c, int level, int data_level, int chunk, int layout)
{
    if (!c || level < 4 || level >= c->nq || data_level < level || data_level >= c->nq || chunk < 1) return 0;
    return step_bytes(c, level, chunk, layout, 1) + al((size_t)chunk * 2 * (data_level + 1) * c->N) * 8;
}

he_status he_lr_data_terms(he_ctx *c, const he_ct *Z, int n_blocks, int w_level, double w_scale, const double coef[4],
                           double eta_over_n, double w_decay, int layout, he_ct *out)
{
    if (!c || !Z || n_blocks < 1 || !coef || !out) return HE_EINVAL;
    if (layout != HE_LAYOUT_ROWS && layout != HE_LAYOUT_FEATURES) return HE_EINVAL;
    const bool fm = layout == HE_LAYOUT_FEATURES;
    const int l = w_level;
    if (l < 4) return HE_ELEVEL;
    const int lz = Z[0].level;
    const double sz = Z[0].scale;
    long long zbs;
    TRY(uniform_group(c, Z, n_blocks, lz, sz, zbs));
    if (lz < l) return HE_ELEVEL;
    he_lr_plan pl;
    TRY(hehost::plan_lr_step(c->q.data(), c->nq, l, sz, w_scale, coef, eta_over_n, w_decay, layout, &pl));
    const int ng = pl.k2 != 0 ? 3 : 2;
    const int lev[3] = {z3_level(l, fm), z1_level(l, fm), z1_level(l, fm)};
    const i64 kk[3] = {pl.k3, pl.k1, pl.k2};
    const double sc[3] = {pl.s_z3, pl.s_z1, pl.s_z2};
    long long os[3];
    for (int g = 0; g < ng; ++g) {
        const long long lc = (long long)(lev[g] + 1) * c->N;
        os[g] = 0;
        for (int b = 0; b < n_blocks; ++b) {
            const he_ct &o = out[g * n_blocks + b];
            if (!o.data) return HE_EINVAL;
            if (b == 1) os[g] = o.data - out[g * n_blocks].data;
            if (b > 1 && o.data - out[g * n_blocks + b - 1].data != os[g]) return HE_EINVAL;
        }
        if (n_blocks > 1 && os[g] < 2 * lc) return HE_EINVAL;
    }
    if (ng == 3 && os[2] != os[1]) return HE_EINVAL;
    TRY(ensure_ws(c, rescale_scratch(c, l, n_blocks) * 8 + 4096));
    const long long zc = (long long)(lz + 1) * c->N;
    for (int g = 0; g < ng; ++g) {
        Arena ar = arena(c);
        TRY(rescale_apply(c, ar, lev[g] + 1, n_blocks, Z[0].data, zbs, out[g * n_blocks].data, os[g], 2, &kk[g], zc));
        for (int b = 0; b < n_blocks; ++b) {
            out[g * n_blocks + b].level = lev[g];
            out[g * n_blocks + b].scale = sc[g];
        }
    }
    return last_error();
}

he_status he_rotate_many(he_ctx *c, const he_ct *x, int n, const int *steps, int n_steps, const he_keys *k,
                         he_ct *out)
{
    if (!c || !x || n < 1 || !steps || n_steps < 1 || !k || !out) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    const int l = x[0].level;
    const long long N = c->N, lc = (long long)(l + 1) * N;
    long long xs = 0, os = 0;
    for (int i = 0; i < n; ++i) {
        if (!ct_ok(c, &x[i]) || x[i].scale != x[0].scale) return HE_EINVAL;
        if (x[i].level != l) return HE_ELEVEL;
        if (i == 1) xs = x[1].data - x[0].data;
        if (i > 1 && x[i].data - x[i - 1].data != xs) return HE_EINVAL;
    }
    if (n > 1 && xs < 2 * lc) return HE_EINVAL;
    const int m = n * n_steps;
    for (int i = 0; i < m; ++i) {
        if (!out[i].data) return HE_EINVAL;
        if (i == 1) os = out[1].data - out[0].data;
        if (i > 1 && out[i].data - out[i - 1].data != os) return HE_EINVAL;
    }
    if (m > 1 && os < 2 * lc) return HE_EINVAL;
    // outputs apart from the inputs
    const u64 *x_end = x[0].data + (long long)(n - 1) * xs + 2 * lc;
    const u64 *o_end = out[0].data + (long long)(m - 1) * os + 2 * lc;
    if (!(o_end <= x[0].data || out[0].data >= x_end)) return HE_EINVAL;
    std::vector<u64> gal(n_steps);
    std::vector<const u64 *> key(n_steps);
    for (int s = 0; s < n_steps; ++s) {
        gal[s] = galois_of(c, steps[s]);
        key[s] = find_rot_key(k, gal[s]);
        if (!key[s]) return HE_EKEY;
    }
    if (n_steps >= 2 && hek::fused_ok(c)) {
        // each input rotated every way at once, sharing its ModUp (bit-identical
        // to one rotation per step), in groups of at most HE_MAXMULTI steps
        const int G = std::min(n_steps, hek::HE_MAXMULTI);
        TRY(ensure_ws(c, rotate_scratch(c, l, G) * 8 + 4096));
        for (int i = 0; i < n; ++i)
            for (int s0 = 0; s0 < n_steps; s0 += G) {
                const int g = std::min(G, n_steps - s0);
                hek::EntryGal eg;
                hek::EntryKeys ek;
                for (int s = 0; s < g; ++s) {
                    eg.g[s] = gal[s0 + s];
                    ek.k[s] = key[s0 + s];
                }
                Arena ar = arena(c);
                TRY(rotate_multi_apply(c, ar, l, g, x[0].data + (long long)i * xs, 0, eg, ek,
                                       out[(long long)i * n_steps + s0].data, os));
            }
    } else {
        TRY(ensure_ws(c, rotate_scratch(c, l, n) * 8 + 4096));
        for (int s = 0; s < n_steps; ++s) {
            Arena ar = arena(c);
            TRY(rotate_apply(c, ar, l, n, x[0].data, xs, gal[s], key[s], out[s].data, (long long)n_steps * os));
        }
    }
    for (int i = 0; i < m; ++i) {
        out[i].level = l;
        out[i].scale = x[0].scale;
    }
    return last_error();
}

he_status he_rotate_sum(he_ctx *c, const he_ct *x, int n, const int *steps, int n_steps, const he_keys *k,
                        he_ct *out)
{
    if (!c || !x || n < 1 || !steps || n_steps < 1 || n_steps > hek::HE_MAXMULTI || !k || !out) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    const int l = x[0].level;
    const long long N = c->N, lc = (long long)(l + 1) * N;
    long long xs = 0, os = 0;
    for (int i = 0; i < n; ++i) {
        if (!ct_ok(c, &x[i]) || x[i].scale != x[0].scale || !out[i].data) return HE_EINVAL;
        if (x[i].level != l) return HE_ELEVEL;
        if (i == 1) {
            xs = x[1].data - x[0].data;
            os = out[1].data - out[0].data;
        }
        if (i > 1 && (x[i].data - x[i - 1].data != xs || out[i].data - out[i - 1].data != os)) return HE_EINVAL;
    }
    if (n > 1 && (xs < 2 * lc || os < 2 * lc)) return HE_EINVAL;
    const u64 *x_end = x[0].data + (long long)(n - 1) * xs + 2 * lc;
    const u64 *o_end = out[0].data + (long long)(n - 1) * os + 2 * lc;
    if (!(o_end <= x[0].data || out[0].data >= x_end)) return HE_EINVAL;
    hek::EntryGal eg;
    hek::EntryKeys ek;
    for (int s = 0; s < n_steps; ++s) {
        eg.g[s] = galois_of(c, steps[s]);
        ek.k[s] = find_rot_key(k, eg.g[s]);
        if (!ek.k[s]) return HE_EKEY;
    }
    TRY(ensure_ws(c, ks_scratch(c, l, n) * 8 + 4096));
    Arena ar = arena(c);
    TRY(rotate_sum_hoisted_apply(c, ar, l, n, x[0].data, xs, eg, ek, n_steps, out[0].data, os));
    for (int i = 0; i < n; ++i) {
        out[i].level = l;
        out[i].scale = x[0].scale;
    }
    return last_error();
}

he_status he_batch_mul_rotate(he_ctx *c, const he_ct *x, const he_ct *y, const int *steps, int n, const he_keys *k,
                              int mode, he_ct *out)
{
    if (!c || !x || !y || !steps || !k || !out || n < 1 || mode < 0 || mode > 2) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    std::vector<u64> gal(n);
    std::map<int, std::vector<int>> groups;
    for (int i = 0; i < n; ++i) {
        if (!ct_ok(c, &x[i]) || !ct_ok(c, &y[i]) || !out[i].data) return HE_EINVAL;
        if (x[i].level != y[i].level || x[i].level < 1) return HE_ELEVEL;
        gal[i] = galois_of(c, steps[i]);
        if (!find_rot_key(k, gal[i])) return HE_EKEY;
        groups[x[i].level].push_back(i);
    }
    const int chunk = mode == 0 ? 1 : hek::HE_MAXMULTI;
    size_t need = 0;
    int ntask = 0;
    for (const auto &g : groups) {
        need = std::max(need, batch_bytes(c, g.first, std::min(chunk, (int)g.second.size())));
        ntask += ((int)g.second.size() + chunk - 1) / chunk;
    }
    // modes 1 and 2: the groups on up to 4 lanes, each with a scratch region of its own
    const int K = mode == 0 ? 1 : std::max(1, std::min(he_ctx::SUBMIT_LANES, ntask));
    const size_t per = (need + 255) & ~(size_t)255;
    TRY(ensure_ws(c, K * per));
    if (K > 1) TRY(lanes_ready(c));
    if (mode == 2) {
        std::ostringstream key;
        key << "batch:" << n << ':' << k->gen << ':' << (const void *)k->sk << ':' << (const void *)c->ws;
        for (int i = 0; i < n; ++i)
            key << ':' << (const void *)x[i].data << ',' << (const void *)y[i].data << ',' << (const void *)out[i].data
                << ',' << x[i].level << ',' << gal[i];
        TRY(run_graph(c, key.str(), k->gen,
                      [&] { return batch_impl(c, x, y, gal.data(), k, chunk, groups, out, K, per); }));
    } else {
        TRY(batch_impl(c, x, y, gal.data(), k, chunk, groups, out, K, per));
    }
    for (int i = 0; i < n; ++i) {
        out[i].level = x[i].level - 1;
        out[i].scale = x[i].scale * y[i].scale / (double)c->q[x[i].level];
    }
    return last_error();
}

// ------------------------------------------------------------------ descriptor batches (he_batch_submit)
// The plan of one submission: operations grouped by kind and input level, the
// staging regions of each group (uniform strides, so the batched key
// switches and rescalings take them) and the device operand tables of the
// elementwise phases.
struct SubmitPlan {
    int chunk = 1;
    std::vector<u64> gal;                   // per op: Galois element of its rotation (1: none)
    std::map<int, std::vector<int>> mul;    // x level -> MUL_ROTATE ops, then MUL ops
    std::map<int, int> mul_rot;             // x level -> how many MUL_ROTATE ops lead the group
    std::map<int, std::vector<int>> rot;    // x level -> ROTATE ops with a key switch
    std::map<int, std::vector<int>> resc;   // x level -> RESCALE ops
    std::vector<int> add, copy;             // ADD ops; ROTATE ops by a multiple of the slot count
    size_t table_u64 = 0, staging_u64 = 0, scratch_u64 = 0;
    int lanes = 1;                          // streams the groups are spread over, each with its own scratch
};

static int out_level(const he_op &o)
{
    return (o.op == HE_OP_MUL || o.op == HE_OP_MUL_ROTATE || o.op == HE_OP_RESCALE) ? o.x.level - 1 : o.x.level;
}

// k = NULL: sizing only (the rotation keys are not checked)
static he_status submit_plan(const he_ctx *c, const he_op *ops, int n, const he_keys *k, int mode, SubmitPlan &pl)
{
    if (!c || !ops || n < 1 || mode < 0 || mode > 2) return HE_EINVAL;
    pl.chunk = mode == 0 ? 1 : 1 << 30;
    pl.gal.assign(n, 1);
    struct Span {
        uintptr_t lo, hi;
        bool out;
    };
    std::vector<Span> spans;
    const size_t N = c->N;
    for (int i = 0; i < n; ++i) {
        const he_op &o = ops[i];
        if (o.op < HE_OP_MUL || o.op > HE_OP_ADD || !ct_ok(c, &o.x) || !o.out.data) return HE_EINVAL;
        const int l = o.x.level;
        const bool two = o.op == HE_OP_MUL || o.op == HE_OP_MUL_ROTATE || o.op == HE_OP_ADD;
        if (two && !ct_ok(c, &o.y)) return HE_EINVAL;
        if (two && o.y.level != l) return HE_ELEVEL;
        if (o.op == HE_OP_ADD && o.x.scale != o.y.scale) return HE_ESCALE;
        if (out_level(o) < 0) return HE_ELEVEL;
        if (o.op == HE_OP_MUL_ROTATE || o.op == HE_OP_ROTATE) {
            pl.gal[i] = galois_of(c, o.steps);
            if (k && pl.gal[i] != 1 && !find_rot_key(k, pl.gal[i])) return HE_EKEY;
        }
        const size_t in_b = (size_t)2 * (l + 1) * N * 8, out_b = (size_t)2 * (out_level(o) + 1) * N * 8;
        spans.push_back({(uintptr_t)o.x.data, (uintptr_t)o.x.data + in_b, false});
        if (two) spans.push_back({(uintptr_t)o.y.data, (uintptr_t)o.y.data + in_b, false});
        spans.push_back({(uintptr_t)o.out.data, (uintptr_t)o.out.data + out_b, true});
        if (o.op == HE_OP_MUL || o.op == HE_OP_MUL_ROTATE) pl.mul_rot.emplace(l, 0);
        switch (o.op) {
        case HE_OP_MUL_ROTATE:
            if (pl.gal[i] != 1) {
                pl.mul[l].insert(pl.mul[l].begin() + pl.mul_rot[l], i);
                ++pl.mul_rot[l];
                break;
            }
            // a rotation by a multiple of the slot count is the product alone
            pl.mul[l].push_back(i);
            break;
        case HE_OP_MUL: pl.mul[l].push_back(i); break;
        case HE_OP_ROTATE:
            if (pl.gal[i] != 1) pl.rot[l].push_back(i);
            else pl.copy.push_back(i);
            break;
        case HE_OP_RESCALE: pl.resc[l].push_back(i); break;
        default: pl.add.push_back(i); break;
        }
    }
    // no output overlaps another output or an input (inputs may be shared)
    std::sort(spans.begin(), spans.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    uintptr_t all_end = 0, out_end = 0;
    for (const Span &sp : spans) {
        if (sp.out ? sp.lo < all_end : sp.lo < out_end) return HE_EINVAL;
        all_end = std::max(all_end, sp.hi);
        if (sp.out) out_end = std::max(out_end, sp.hi);
    }
    // sizes: operand tables, staging, and the largest group's scratch
    size_t ntab = pl.add.size() + pl.copy.size();
    size_t stg = 0, scr = 0;
    for (const auto &g : pl.mul) {
        const int l = g.first, B = (int)g.second.size(), Br = pl.mul_rot[l];
        ntab += 2 * B;  // tensor, copy out
        stg += al((size_t)B * 3 * (l + 1) * N) + al((size_t)B * 2 * l * N) + al((size_t)Br * 2 * l * N);
        scr = std::max(scr, relin_rescale_scratch(c, l, std::min(B, pl.chunk)));
        if (Br) scr = std::max(scr, rotate_scratch(c, l - 1, std::min({Br, pl.chunk, hek::HE_MAXMULTI})));
    }
    for (const auto &g : pl.rot) {
        const int l = g.first, B = (int)g.second.size();
        ntab += 2 * B;  // stage in, copy out
        stg += 2 * al((size_t)B * 2 * (l + 1) * N);
        scr = std::max(scr, rotate_scratch(c, l, std::min({B, pl.chunk, hek::HE_MAXMULTI})));
    }
    for (const auto &g : pl.resc) {
        const int l = g.first, B = (int)g.second.size();
        ntab += 2 * B;
        stg += al((size_t)B * 2 * (l + 1) * N) + al((size_t)B * 2 * l * N);
        scr = std::max(scr, rescale_scratch(c, l, std::min(B, pl.chunk)));
    }
    pl.table_u64 = al(ntab * sizeof(hek::OpDesc) / 8);
    pl.staging_u64 = stg;
    pl.scratch_u64 = scr;
    const int groups = (int)(pl.mul.size() + pl.rot.size() + pl.resc.size());
    pl.lanes = mode == 0 ? 1 : std::max(1, std::min(he_ctx::SUBMIT_LANES, groups));
    return HE_OK;
}

static size_t submit_bytes(const SubmitPlan &pl)
{
    return (pl.table_u64 + pl.staging_u64 + (size_t)pl.lanes * al(pl.scratch_u64)) * 8 + 4096;
}

// The staging regions and operand tables of a plan laid out in the workspace
// (the tables first, at its start, then the staging, then the scratch arena).
struct SubmitLayout {
    std::vector<hek::OpDesc> tab;  // host copy: tensor | stage in | add | copy out
    int n_tensor = 0, n_in = 0, n_add = 0, n_out = 0, max_limbs = 0;
    std::map<int, u64 *> T3, R, RO, Rin, Rout, Sin, Sout;
};

static he_status submit_layout(he_ctx *c, const he_op *ops, const SubmitPlan &pl, Arena &ar, SubmitLayout &ly)
{
    const long long N = c->N;
    ar.off = pl.table_u64 * 8;
    for (const auto &g : pl.mul) {
        const int l = g.first, B = (int)g.second.size(), Br = pl.mul_rot.at(l);
        ly.T3[l] = ar.take((size_t)B * 3 * (l + 1) * N);
        ly.R[l] = ar.take((size_t)B * 2 * l * N);
        ly.RO[l] = Br ? ar.take((size_t)Br * 2 * l * N) : nullptr;
        if (!ly.T3[l] || !ly.R[l] || (Br && !ly.RO[l])) return HE_ENOMEM;
    }
    for (const auto &g : pl.rot) {
        const int l = g.first, B = (int)g.second.size();
        ly.Rin[l] = ar.take((size_t)B * 2 * (l + 1) * N);
        ly.Rout[l] = ar.take((size_t)B * 2 * (l + 1) * N);
        if (!ly.Rin[l] || !ly.Rout[l]) return HE_ENOMEM;
    }
    for (const auto &g : pl.resc) {
        const int l = g.first, B = (int)g.second.size();
        ly.Sin[l] = ar.take((size_t)B * 2 * (l + 1) * N);
        ly.Sout[l] = ar.take((size_t)B * 2 * l * N);
        if (!ly.Sin[l] || !ly.Sout[l]) return HE_ENOMEM;
    }
    std::vector<hek::OpDesc> tensor, in, add, out;
    auto lim = [&](int limbs) { ly.max_limbs = std::max(ly.max_limbs, limbs); return limbs; };
    for (const auto &g : pl.mul) {
        const int l = g.first, Br = pl.mul_rot.at(l);
        for (size_t b = 0; b < g.second.size(); ++b) {
            const he_op &o = ops[g.second[b]];
            tensor.push_back({o.x.data, o.y.data, ly.T3[l] + b * 3 * (l + 1) * N, lim(l + 1), 0});
            const u64 *res = (int)b < Br ? ly.RO[l] + b * 2 * l * N : ly.R[l] + b * 2 * l * N;
            out.push_back({res, nullptr, o.out.data, lim(l), 0});
        }
    }
    for (const auto &g : pl.rot) {
        const int l = g.first;
        for (size_t b = 0; b < g.second.size(); ++b) {
            const he_op &o = ops[g.second[b]];
            in.push_back({o.x.data, nullptr, ly.Rin[l] + b * 2 * (l + 1) * N, lim(l + 1), 0});
            out.push_back({ly.Rout[l] + b * 2 * (l + 1) * N, nullptr, o.out.data, l + 1, 0});
        }
    }
    for (const auto &g : pl.resc) {
        const int l = g.first;
        for (size_t b = 0; b < g.second.size(); ++b) {
            const he_op &o = ops[g.second[b]];
            in.push_back({o.x.data, nullptr, ly.Sin[l] + b * 2 * (l + 1) * N, lim(l + 1), 0});
            out.push_back({ly.Sout[l] + b * 2 * l * N, nullptr, o.out.data, l, 0});
        }
    }
    for (int i : pl.add) add.push_back({ops[i].x.data, ops[i].y.data, ops[i].out.data, lim(ops[i].x.level + 1), 0});
    for (int i : pl.copy) out.push_back({ops[i].x.data, nullptr, ops[i].out.data, lim(ops[i].x.level + 1), 0});
    ly.n_tensor = (int)tensor.size();
    ly.n_in = (int)in.size();
    ly.n_add = (int)add.size();
    ly.n_out = (int)out.size();
    ly.tab = tensor;
    ly.tab.insert(ly.tab.end(), in.begin(), in.end());
    ly.tab.insert(ly.tab.end(), add.begin(), add.end());
    ly.tab.insert(ly.tab.end(), out.begin(), out.end());
    return HE_OK;
}

static he_status submit_impl(he_ctx *c, const he_op *ops, const SubmitPlan &pl, const SubmitLayout &ly,
                             const he_keys *k, size_t scratch_off)
{
    const long long N = c->N;
    const hek::OpDesc *tab = (const hek::OpDesc *)c->ws;
    auto limbs = [&](int i0, int n) {
        double s = 0.0;
        for (int i = i0; i < i0 + n; ++i) s += ly.tab[i].limbs;
        return s;
    };
    const int o_in = ly.n_tensor, o_add = o_in + ly.n_in, o_out = o_add + ly.n_add;
    // elementwise phases over every operation of every level: one launch each
    hek::desc_ew(c, 6, tab, ly.n_tensor, ly.max_limbs, limbs(0, ly.n_tensor));
    hek::desc_ew(c, 4, tab + o_in, ly.n_in, ly.max_limbs, limbs(o_in, ly.n_in));
    hek::desc_ew(c, 0, tab + o_add, ly.n_add, ly.max_limbs, limbs(o_add, ly.n_add));
    const int rchunk = std::min(pl.chunk, hek::HE_MAXMULTI);
    // The level groups share no data: each is one task, and the tasks are
    // dealt to pl.lanes streams (largest first, each to the least loaded
    // lane), each lane with a scratch arena of its own.  A lane runs its tasks
    // in order, so its arena is reused as on one stream.
    std::vector<Arena> lane_ar(pl.lanes, arena(c));
    const size_t sb = al(pl.scratch_u64) * 8;  // 256-byte multiples: every lane's arena starts aligned
    for (int i = 0; i < pl.lanes; ++i) {
        lane_ar[i].off = scratch_off + i * sb;
        lane_ar[i].cap = scratch_off + (i + 1) * sb;
    }
    std::vector<std::pair<double, std::function<he_status(int)>>> tasks;
    // products: relinearise and rescale per level, then the MUL_ROTATE rotations
    for (const auto &g : pl.mul) {
        const int l = g.first, B = (int)g.second.size(), Br = pl.mul_rot.at(l);
        const std::vector<int> *idx = &g.second;
        tasks.push_back({(double)(B + Br) * (l + 1 + c->nk), [&, l, B, Br, idx](int lane) -> he_status {
            Arena &ar = lane_ar[lane];
            const long long t3 = 3LL * (l + 1) * N, r2 = 2LL * l * N;
            for (int s0 = 0; s0 < B; s0 += pl.chunk) {
                const int b = std::min(pl.chunk, B - s0);
                TRY(relin_rescale_apply(c, ar, l, b, ly.T3.at(l) + s0 * t3, t3, k->rlk, ly.R.at(l) + s0 * r2, r2));
            }
            for (int s0 = 0; s0 < Br; s0 += rchunk) {
                const int b = std::min(rchunk, Br - s0);
                hek::EntryGal eg;
                hek::EntryKeys ek;
                for (int j = 0; j < b; ++j) {
                    eg.g[j] = pl.gal[(*idx)[s0 + j]];
                    ek.k[j] = find_rot_key(k, eg.g[j]);
                }
                TRY(rotate_multi_apply(c, ar, l - 1, b, ly.R.at(l) + s0 * r2, r2, eg, ek, ly.RO.at(l) + s0 * r2,
                                       r2));
            }
            return HE_OK;
        }});
    }
    for (const auto &g : pl.rot) {
        const int l = g.first, B = (int)g.second.size();
        const std::vector<int> *idx = &g.second;
        tasks.push_back({(double)B * (l + 1 + c->nk), [&, l, B, idx](int lane) -> he_status {
            Arena &ar = lane_ar[lane];
            const long long c2 = 2LL * (l + 1) * N;
            for (int s0 = 0; s0 < B; s0 += rchunk) {
                const int b = std::min(rchunk, B - s0);
                hek::EntryGal eg;
                hek::EntryKeys ek;
                for (int j = 0; j < b; ++j) {
                    eg.g[j] = pl.gal[(*idx)[s0 + j]];
                    ek.k[j] = find_rot_key(k, eg.g[j]);
                }
                TRY(rotate_multi_apply(c, ar, l, b, ly.Rin.at(l) + s0 * c2, c2, eg, ek, ly.Rout.at(l) + s0 * c2,
                                       c2));
            }
            return HE_OK;
        }});
    }
    for (const auto &g : pl.resc) {
        const int l = g.first, B = (int)g.second.size();
        tasks.push_back({0.25 * B * (l + 1), [&, l, B](int lane) -> he_status {
            Arena &ar = lane_ar[lane];
            const long long c2 = 2LL * (l + 1) * N, r2 = 2LL * l * N;
            for (int s0 = 0; s0 < B; s0 += pl.chunk) {
                const int b = std::min(pl.chunk, B - s0);
                TRY(rescale_apply(c, ar, l, b, ly.Sin.at(l) + s0 * c2, c2, ly.Sout.at(l) + s0 * r2, r2));
            }
            return HE_OK;
        }});
    }
    TRY(lanes_run(c, pl.lanes, tasks));
    // every result to its out: one launch
    hek::desc_ew(c, 4, tab + o_out, ly.n_out, ly.max_limbs, limbs(o_out, ly.n_out));
    return last_error();
}

size_t he_batch_submit_bytes(const he_ctx *c, const he_op *ops, int n, int mode)
{
    SubmitPlan pl;
    return submit_plan(c, ops, n, nullptr, mode, pl) == HE_OK ? submit_bytes(pl) : 0;
}

he_status he_batch_submit(he_ctx *c, he_op *ops, int n, const he_keys *k, int mode)
{
    if (!c || !ops || n < 1 || !k) return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    SubmitPlan pl;
    TRY(submit_plan(c, ops, n, k, mode, pl));
    TRY(ensure_ws(c, submit_bytes(pl)));
    Arena ar = arena(c);
    SubmitLayout ly;
    TRY(submit_layout(c, ops, pl, ar, ly));
    const size_t scratch_off = ar.off;
    // the operand tables, uploaded before the work (and before a replay) from
    // the context's pinned staging buffer, which the previous upload must have
    // left first
    const size_t tb = ly.tab.size() * sizeof(hek::OpDesc);
    if (!c->sub_ev) HIPCHK(hipEventCreateWithFlags(&c->sub_ev, hipEventDisableTiming));
    HIPCHK(hipEventSynchronize(c->sub_ev));
    if (c->sub_host_bytes < tb) {
        if (c->sub_host) (void)hipHostFree(c->sub_host);
        c->sub_host = nullptr;
        c->sub_host_bytes = 0;
        HIPCHK(hipHostMalloc(&c->sub_host, tb, hipHostMallocDefault));
        c->sub_host_bytes = tb;
    }
    std::memcpy(c->sub_host, ly.tab.data(), tb);
    HIPCHK(hipMemcpyAsync(c->ws, c->sub_host, tb, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipEventRecord(c->sub_ev, c->stream));
    if (pl.lanes > 1) TRY(lanes_ready(c));
    if (mode == 2) {
        std::ostringstream key;
        key << "submit:" << n << ':' << k->gen << ':' << (const void *)k->sk << ':' << (const void *)c->ws;
        for (int i = 0; i < n; ++i)
            key << ':' << ops[i].op << ',' << pl.gal[i] << ',' << (const void *)ops[i].x.data << ','
                << (const void *)ops[i].y.data << ',' << (const void *)ops[i].out.data << ',' << ops[i].x.level;
        TRY(run_graph(c, key.str(), k->gen, [&] { return submit_impl(c, ops, pl, ly, k, scratch_off); }));
    } else {
        TRY(submit_impl(c, ops, pl, ly, k, scratch_off));
    }
    for (int i = 0; i < n; ++i) {
        he_op &o = ops[i];
        const int l = o.x.level;
        o.out.level = out_level(o);
        if (o.op == HE_OP_MUL || o.op == HE_OP_MUL_ROTATE) o.out.scale = o.x.scale * o.y.scale / (double)c->q[l];
        else if (o.op == HE_OP_RESCALE) o.out.scale = o.x.scale / (double)c->q[l];
        else o.out.scale = o.x.scale;
    }
    return last_error();
}

// ------------------------------------------------------------------ several requests' steps, tails batched
// Per request the per-block part of the step runs as in he_lr_grad_step (its
// own plan, mask and blocks), into its own degree-4 term sum; the once-per-step
// tail then runs once for all requests: the three relinearisation key switches
// (one batched call per key), the rescale, the grouped slot sums of every
// request together, the masks and W updates through a device operand table.
// Every kernel treats each entry on its own, so each request's W' and g are
// bit-identical to its own he_lr_grad_step in mode 1.
struct MultiBufs {
    u64 *G5, *ksx, *U0, *G, *Gm, *Wk, *Wr;
    hek::OpDesc *tab;
};

static size_t multi_tail_u64(const he_ctx *c, int l, int n, int layout, size_t *tab_u64 = nullptr)
{
    const size_t N = c->N;
    const bool fm = layout == HE_LAYOUT_FEATURES;
    const int lg = fm ? l - 2 : l - 3;
    const size_t x1 = (size_t)(lg + 1) * N;
    const size_t tb = al((size_t)4 * n * sizeof(hek::OpDesc) / 8 + 1);
    if (tab_u64) *tab_u64 = tb;
    size_t u = tb + al((size_t)n * 5 * x1) + al((size_t)3 * n * 2 * x1) + al((size_t)n * 2 * x1);
    u += al((size_t)n * 2 * lg * N) + (fm ? al((size_t)n * 2 * (l - 3) * N) : 0);
    u += al((size_t)n * 2 * (l - 2) * N) + al((size_t)n * 2 * (l - 3) * N);
    // the batched tail's scratch: a key switch of n entries at lg, rotations and rescales of n
    size_t scr = std::max(ks_scratch(c, lg, n), rescale_scratch(c, lg, n));
    scr = std::max(scr, rotate_scratch(c, lg - 1, n));
    scr = std::max(scr, rescale_scratch(c, l - 3, n));
    return u + scr;
}

static size_t multi_bytes(const he_ctx *c, int l, int max_blocks, int n, int layout, int mode)
{
    return step_bytes(c, l, mode == 0 ? 1 : max_blocks, layout, 1) + multi_tail_u64(c, l, n, layout) * 8 + 4096;
}

static he_status multi_impl(he_ctx *c, const he_lr_request *rq, int n, const std::vector<StepArgs> &sa, int cols,
                            int rows, int layout, const he_keys *k, int max_blocks)
{
    const long long N = c->N;
    const int l = rq[0].W->level;
    const bool fm = layout == HE_LAYOUT_FEATURES;
    const int lg = fm ? l - 2 : l - 3;
    const long long x1 = (long long)(lg + 1) * N, r1 = (long long)lg * N, g1 = (long long)(l - 3) * N;
    const long long w1 = (long long)(l - 2) * N;
    Arena ar = arena(c);
    StepBufs s;
    TRY(step_alloc(c, ar, l, max_blocks, layout, 1, s));
    MultiBufs m;
    size_t tab_u64 = 0;
    (void)multi_tail_u64(c, l, n, layout, &tab_u64);
    m.tab = (hek::OpDesc *)ar.take(tab_u64);
    m.G5 = ar.take((size_t)n * 5 * x1);
    m.ksx = ar.take((size_t)3 * n * 2 * x1);
    m.U0 = ar.take((size_t)n * 2 * x1);
    m.G = ar.take((size_t)n * 2 * r1);
    m.Gm = fm ? ar.take((size_t)n * 2 * g1) : nullptr;
    m.Wk = ar.take((size_t)n * 2 * w1);
    m.Wr = ar.take((size_t)n * 2 * g1);
    if (!m.tab || !m.G5 || !m.ksx || !m.U0 || !m.G || (fm && !m.Gm) || !m.Wk || !m.Wr) return HE_ENOMEM;
    // per request: the per-block part into its own term sum
    for (int i = 0; i < n; ++i) {
        s.G5 = m.G5 + (long long)i * 5 * x1;
        const BabyData bd;
        const TermData td;
        if (fm)
            TRY(step_blocks_features(c, ar, s, sa[i].pl, rq[i].Z, sa[i].zbs, 0, rq[i].n_blocks, rq[i].W, cols, rows, k,
                                     false, bd, td));
        else
            TRY(step_blocks(c, ar, s, sa[i].pl, rq[i].Z, sa[i].zbs, 0, rq[i].n_blocks, rq[i].W, rq[i].mask, cols, k,
                            false, bd, td));
    }
    // the operand tables of the tail: masks (feature-major), G copies, kW W, W' = RS(kW W) + g
    std::vector<hek::OpDesc> tab;
    u64 *gfin = fm ? m.Gm : m.G;
    const long long gs = fm ? 2 * g1 : 2 * r1;  // batch stride of the final g (level l-4 either way)
    if (fm)
        for (int i = 0; i < n; ++i) tab.push_back({m.G + i * 2 * r1, rq[i].mask->data, m.G + i * 2 * r1, l - 2, 0, 0});
    const int t_mask = 0, t_copy = (int)tab.size();
    int n_copy = 0;
    for (int i = 0; i < n; ++i)
        if (rq[i].G_out) {
            tab.push_back({gfin + i * gs, nullptr, rq[i].G_out->data, l - 3, 0, 0});
            ++n_copy;
        }
    const int t_kw = (int)tab.size();
    for (int i = 0; i < n; ++i) tab.push_back({rq[i].W->data, nullptr, m.Wk + i * 2 * w1, l - 2, l + 1, sa[i].pl.kw});
    const int t_add = (int)tab.size();
    for (int i = 0; i < n; ++i) tab.push_back({m.Wr + i * 2 * g1, gfin + i * gs, rq[i].W_out->data, l - 3, 0, 0});
    const size_t tb = tab.size() * sizeof(hek::OpDesc);
    if (!c->sub_ev) HIPCHK(hipEventCreateWithFlags(&c->sub_ev, hipEventDisableTiming));
    HIPCHK(hipEventSynchronize(c->sub_ev));
    if (c->sub_host_bytes < tb) {
        if (c->sub_host) (void)hipHostFree(c->sub_host);
        c->sub_host = nullptr;
        c->sub_host_bytes = 0;
        HIPCHK(hipHostMalloc(&c->sub_host, tb, hipHostMallocDefault));
        c->sub_host_bytes = tb;
    }
    std::memcpy(c->sub_host, tab.data(), tb);
    HIPCHK(hipMemcpyAsync(m.tab, c->sub_host, tb, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipEventRecord(c->sub_ev, c->stream));
    // one relinearisation of every request's degree-4 sum: the key switches of
    // g2, g3, g4 (one batched call per key), then (g0, g1) plus their sum
    const u64 *rk[3] = {k->rlk, k->rlk3, k->rlk4};
    for (int e = 0; e < 3; ++e)
        TRY(ks_apply(c, ar, lg, n, m.G5 + (2 + e) * x1, 5 * x1, rk[e], nullptr, 0, 0, 0, m.ksx + (long long)e * n * 2 * x1,
                     2 * x1, x1));
    hek::ewise(c, 0, lg, n, 2, m.G5, 5 * x1, x1, m.ksx, 2 * x1, x1, m.U0, 2 * x1, x1, 0);
    for (int e = 1; e < 3; ++e)
        hek::ewise(c, 0, lg, n, 2, m.U0, 2 * x1, x1, m.ksx + (long long)e * n * 2 * x1, 2 * x1, x1, m.U0, 2 * x1, x1,
                   0);
    TRY(rescale_apply(c, ar, lg, n, m.U0, 2 * x1, m.G, 2 * r1));
    if (fm) {
        // sum inside each feature block, mask slots j r, rescale, replicate
        // (m.Wk, written only by the W update below, holds the sums' other half)
        TRY(slot_sum_hoisted(c, ar, l - 3, n, m.G, 2 * r1, m.Wk, 2 * r1, +1, rows, k));
        hek::desc_ew(c, 3, m.tab + t_mask, n, l - 2);
        TRY(rescale_apply(c, ar, l - 3, n, m.G, 2 * r1, m.Gm, 2 * g1));
        TRY(slot_sum_hoisted(c, ar, l - 4, n, m.Gm, 2 * g1, m.Wk, 2 * g1, -1, rows, k));
    } else {
        TRY(slot_sum_hoisted(c, ar, l - 4, n, m.G, 2 * r1, m.Wk, 2 * r1, cols, rows, k));  // row sum
    }
    hek::desc_ew(c, 4, m.tab + t_copy, n_copy, l - 3);
    // W' = RS(kW W) + g
    hek::desc_ew(c, 2, m.tab + t_kw, n, l - 2);
    TRY(rescale_apply(c, ar, l - 3, n, m.Wk, 2 * w1, m.Wr, 2 * g1));
    hek::desc_ew(c, 0, m.tab + t_add, n, l - 3);
    return last_error();
}

size_t he_lr_grad_step_multi_bytes(const he_ctx *c, int level, int max_blocks, int n_req, int layout, int mode)
{
    if (!c || level < 4 || level >= c->nq || max_blocks < 1 || n_req < 1 || mode < 0 || mode > 1 ||
        (layout != HE_LAYOUT_ROWS && layout != HE_LAYOUT_FEATURES))
        return 0;
    if (mode == 0) return step_bytes(c, level, 1, layout, 1);
    return multi_bytes(c, level, max_blocks, n_req, layout, mode);
}

he_status he_lr_grad_step_multi(he_ctx *c, const he_lr_request *rq, int n_req, int cols, int rows, int layout,
                                const he_keys *k, int mode)
{
    if (!c || !rq || n_req < 1 || !k || mode < 0 || mode > 1) return HE_EINVAL;
    std::vector<StepArgs> sa(n_req);
    int max_blocks = 1;
    for (int i = 0; i < n_req; ++i) {
        if (!rq[i].W) return HE_EINVAL;
        TRY(step_args(c, rq[i].Z, rq[i].n_blocks, rq[i].W, rq[i].mask, rq[i].coef, rq[i].eta_over_n, rq[i].w_decay,
                      cols, rows, layout, nullptr, 1, nullptr, k, 1, rq[i].W_out, rq[i].G_out, sa[i]));
        if (rq[i].W->level != rq[0].W->level) return HE_ELEVEL;
        max_blocks = std::max(max_blocks, rq[i].n_blocks);
    }
    const int l = rq[0].W->level;
    if (mode == 0) {  // each request on its own (the reference form)
        TRY(ensure_ws(c, step_bytes(c, l, 1, layout, 1)));
        for (int i = 0; i < n_req; ++i) {
            const BabyData bd;
            const TermData td;
            TRY(step_impl(c, sa[i].pl, rq[i].Z, rq[i].n_blocks, sa[i].zbs, bd, td, rq[i].W, rq[i].mask, cols, rows,
                          k, 1, rq[i].W_out, rq[i].G_out));
        }
    } else {
        TRY(ensure_ws(c, multi_bytes(c, l, max_blocks, n_req, layout, mode)));
        TRY(multi_impl(c, rq, n_req, sa, cols, rows, layout, k, max_blocks));
    }
    for (int i = 0; i < n_req; ++i) {
        rq[i].W_out->level = l - 4;
        rq[i].W_out->scale = sa[i].pl.s_g;
        if (rq[i].G_out) {
            rq[i].G_out->level = l - 4;
            rq[i].G_out->scale = sa[i].pl.s_g;
        }
    }
    return last_error();
}

size_t he_lr_step_bytes(const he_ctx *c, int level, int n_blocks, int layout, int n_baby, int mode)
{
    if (!c || level < 4 || level >= c->nq || n_blocks < 1 || (layout != HE_LAYOUT_ROWS && layout != HE_LAYOUT_FEATURES))
        return 0;
    if (n_baby < 1 || n_baby > HE_MAXBABY || (n_baby & (n_baby - 1))) return 0;
    return step_bytes(c, level, mode == 0 ? 1 : n_blocks, layout, n_baby);
}

size_t he_lr_margins_bytes(const he_ctx *c, int level, int n_blocks, int mode)
{
    if (!c || level < 1 || level >= c->nq || n_blocks < 1) return 0;
    return margins_bytes(c, level, mode == 0 ? 1 : n_blocks);
}

// Argument checks shared by he_lr_margins and he_lr_infer (before any launch):
// Z and out uniform strides (out at level out_level), levels, the margin keys.
he_status margins_args(he_ctx *c, const he_ct *Z, int n_blocks, const he_ct *W, int cols, int rows, int layout,
                       const he_keys *k, int mode, const he_ct *out, int min_level, int out_level, long long &zbs,
                       long long &obs)
{
    if (!c || !Z || n_blocks < 1 || !ct_ok(c, W) || !k || !out || !out[0].data || mode < 0 || mode > 2)
        return HE_EINVAL;
    if (!keys_ok(c, k)) return HE_EKEY;
    if (layout != HE_LAYOUT_ROWS && layout != HE_LAYOUT_FEATURES) return HE_EINVAL;
    if (cols < 1 || rows < 1 || (cols & (cols - 1)) || (rows & (rows - 1)) || (long long)cols * rows != c->N / 2)
        return HE_EINVAL;
    const int l = W->level;
    if (l < min_level) return HE_ELEVEL;
    const int lz = Z[0].level;
    const double sz = Z[0].scale;
    zbs = 0;
    obs = 0;
    for (int b = 0; b < n_blocks; ++b) {
        if (!ct_ok(c, &Z[b]) || Z[b].level != lz || Z[b].scale != sz) return Z[b].level != lz ? HE_ELEVEL : HE_EINVAL;
        if (!out[b].data) return HE_EINVAL;
        if (b == 1) {
            zbs = Z[1].data - Z[0].data;
            obs = out[1].data - out[0].data;
        }
        if (b > 1 && (Z[b].data - Z[b - 1].data != zbs || out[b].data - out[b - 1].data != obs)) return HE_EINVAL;
    }
    if (lz < l) return HE_ELEVEL;
    if (n_blocks > 1 && (zbs < 2LL * (lz + 1) * c->N || obs < 2LL * (out_level + 1) * c->N)) return HE_EINVAL;
    return slot_sum_keys(c, k, layout == HE_LAYOUT_FEATURES ? rows : 1, cols) ? HE_OK : HE_EKEY;
}

// p(u) of he_lr_infer for nb blocks: u [nb][2][l][N] (level l-1, batch stride
// us) -> out [nb][2][l-2][N] (level l-3, batch stride os); see he_plan_lr_infer
he_status infer_poly(he_ctx *c, Arena &ar, const he_infer_plan &pl, int nb, const u64 *u, long long us, u64 *out,
                     long long os, const u64 *rlk)
{
    const long long N = c->N;
    const int l1 = pl.level_in - 1, l2 = l1 - 1;  // u's level, then U2's and H's
    const long long c1 = (long long)(l1 + 1) * N, c2 = (long long)(l2 + 1) * N, c3 = (long long)l2 * N;
    const size_t mark = ar.off;
    u64 *T3 = ar.take((size_t)nb * 3 * c1);
    u64 *U2 = ar.take((size_t)nb * 2 * c2);
    u64 *Hb = ar.take((size_t)nb * 2 * c2);
    u64 *Lb = ar.take((size_t)nb * 2 * c3);
    if (!T3 || !U2 || !Hb || !Lb) return HE_ENOMEM;
    // U2 = RS(relin(u u))
    hek::tensor_b(c, l1, nb, u, us, c1, u, us, c1, T3, 3 * c1, c1);
    TRY(relin_rescale_apply(c, ar, l1, nb, T3, 3 * c1, rlk, U2, 2 * c2));
    // H = RS(k3 u) + k2c
    TRY(rescale_apply(c, ar, l1, nb, u, us, Hb, 2 * c2, 2, &pl.k3));
    if (pl.k2c != 0) hek::ewise(c, 5, l2, nb, 1, Hb, 2 * c2, 0, nullptr, 0, 0, Hb, 2 * c2, 0, pl.k2c);
    // out = RS(relin(H U2)) + RS(k1 u) + k0c
    hek::tensor_b(c, l2, nb, Hb, 2 * c2, c2, U2, 2 * c2, c2, T3, 3 * c2, c2);
    TRY(relin_rescale_apply(c, ar, l2, nb, T3, 3 * c2, rlk, out, os));
    TRY(rescale_apply(c, ar, l2, nb, u, us, Lb, 2 * c3, 2, &pl.k1, c1));
    hek::ewise(c, 0, l2 - 1, nb, 2, out, os, c3, Lb, 2 * c3, c3, out, os, c3, 0);
    if (pl.k0c != 0) hek::ewise(c, 5, l2 - 1, nb, 1, out, os, 0, nullptr, 0, 0, out, os, 0, pl.k0c);
    ar.off = mark;
    return last_error();
}

size_t infer_bytes(const he_ctx *c, int l, int nb)
{
    const size_t N = c->N;
    size_t n = al((size_t)nb * 2 * l * N);  // the margins
    const size_t poly = al((size_t)nb * 3 * l * N) + 2 * al((size_t)nb * 2 * (l - 1) * N) +
                        al((size_t)nb * 2 * (l - 2) * N) +
                        std::max(relin_rescale_scratch(c, l - 1, nb), rescale_scratch(c, l - 1, nb));
    return n * 8 + std::max(margins_bytes(c, l, nb), poly * 8 + 4096);
}

he_status infer_impl(he_ctx *c, const he_infer_plan &pl, const he_ct *Z, int n_blocks, long long zbs, const he_ct *W,
                     long long unit, int count, const he_keys *keys, int chunk, u64 *out, long long obs)
{
    const long long N = c->N;
    const int l = W->level;
    for (int b0 = 0; b0 < n_blocks; b0 += chunk) {
        const int nb = std::min(chunk, n_blocks - b0);
        Arena ar = arena(c);
        u64 *U = ar.take((size_t)nb * 2 * l * N);
        if (!U) return HE_ENOMEM;
        TRY(margins_impl(c, Z + b0, nb, zbs, W, unit, count, keys, nb, U, 2LL * l * N, ar.off));
        TRY(infer_poly(c, ar, pl, nb, U, 2LL * l * N, out + b0 * obs, obs, keys->rlk));
    }
    return last_error();
}

he_status he_lr_margins(he_ctx *c, const he_ct *Z, int n_blocks, const he_ct *W, int cols, int rows, int layout,
                        const he_keys *k, int mode, he_ct *out)
{
    long long zbs = 0, obs = 0;
    TRY(margins_args(c, Z, n_blocks, W, cols, rows, layout, k, mode, out, 1, W ? W->level - 1 : 0, zbs, obs));
    const int l = W->level;
    const int lz = Z[0].level;
    const double sz = Z[0].scale;
    const bool fm = layout == HE_LAYOUT_FEATURES;
    const long long unit = fm ? rows : 1;
    const int count = cols;
    const int chunk = mode == 0 ? 1 : n_blocks;
    TRY(ensure_ws(c, margins_bytes(c, l, chunk)));
    if (mode == 2) {
        std::ostringstream key;
        key << "margins:" << (const void *)Z[0].data << ':' << zbs << ':' << n_blocks << ':' << lz << ':'
            << (const void *)W->data << ':' << l << ':' << cols << ':' << layout << ':' << k->gen << ':'
            << (const void *)k->sk << ':' << (const void *)out[0].data << ':' << obs << ':' << (const void *)c->ws;
        TRY(run_graph(c, key.str(), k->gen,
                      [&] { return margins_impl(c, Z, n_blocks, zbs, W, unit, count, k, chunk, out[0].data, obs); }));
    } else {
        TRY(margins_impl(c, Z, n_blocks, zbs, W, unit, count, k, chunk, out[0].data, obs));
    }
    const double so = sz * W->scale / (double)c->q[l];
    for (int b = 0; b < n_blocks; ++b) {
        out[b].level = l - 1;
        out[b].scale = so;
    }
    return last_error();
}

// ---------------------------------------------------------------- kernel trace

he_status he_ctx_trace(he_ctx *c, int on)
{
    if (!c || c->capturing) return HE_EINVAL;
    if (on) {
        for (const KRec &r : c->kt.recs) {
            c->kt.pool.push_back(r.a);
            c->kt.pool.push_back(r.b);
        }
        c->kt.recs.clear();
        c->kt.failed = false;
    }
    c->kt.on = on != 0;
    return HE_OK;
}

he_status he_ctx_trace_read(he_ctx *c, he_kernel_stat *out, int max, int *n)
{
    if (!c || !n || max < 0 || (max > 0 && !out)) return HE_EINVAL;
    HIPCHK(hipStreamSynchronize(c->stream));
    he_kernel_stat acc[HE_K_COUNT];
    for (int k = 0; k < HE_K_COUNT; ++k) acc[k] = he_kernel_stat{k, 0, 0.0, 0.0, 0.0, 0.0};
    bool failed = c->kt.failed;
    for (const KRec &r : c->kt.recs) {
        float ms = 0.0f;
        // records made on an earlier stream of the context complete on their own
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) failed = true;
        he_kernel_stat &a = acc[r.kind >= 0 && r.kind < HE_K_COUNT ? r.kind : HE_K_OTHER];
        a.launches += 1;
        a.ms += ms;
        a.bytes += r.bytes;
        a.mm_fp64 += r.mm_fp;
        a.mm_int += r.mm_int;
        c->kt.pool.push_back(r.a);
        c->kt.pool.push_back(r.b);
    }
    c->kt.recs.clear();
    c->kt.failed = false;
    int w = 0;
    for (int k = 0; k < HE_K_COUNT && w < max; ++k)
        if (acc[k].launches) out[w++] = acc[k];
    *n = w;
    return failed ? HE_EDEVICE : HE_OK;
}

const char *he_kernel_kind_name(int kind)
{
    static const char *names[HE_K_COUNT] = {
        "ntt forward column pass", "ntt forward row pass", "ntt inverse row pass", "ntt inverse column pass",
        "ntt, both passes in one launch", "moddown/rescale conversion + forward column pass",
        "forward row pass + moddown/rescale finish", "moddown last limb", "key-switch digits' column pass",
        "key-switch row pass + key inner product", "modup conversion", "hoisted rotation sum, FP64 positions",
        "hoisted rotation sum, 60-bit positions", "rotation inner products (shared modup)", "baby-step products",
        "gradient terms sum", "tensor product", "elementwise", "automorphism",
        "hoisted rotation sum, gathered (steps not tile-local)", "other"};
    return kind >= 0 && kind < HE_K_COUNT ? names[kind] : "?";
}

he_status he_valu_peak(he_ctx *c, int prime_idx, int fp64, double *bfly_per_s)
{
    if (!c || !bfly_per_s || prime_idx < 0 || prime_idx >= c->np) return HE_EINVAL;
    if (fp64 && c->q[prime_idx] >= (1ull << 46)) return HE_EINVAL;
    const size_t n = (size_t)256 * 8 * 4 * 256;
    TRY(ensure_ws(c, al(n) * 8 + 4096));
    *bfly_per_s = hek::valu_bfly_rate(c, fp64 != 0, prime_idx, (u64 *)c->ws);
    return *bfly_per_s > 0.0 ? last_error() : HE_EDEVICE;
}

he_status he_plan_lr_infer(const uint64_t *q, int n_q, int level, double s_z, double s_w, const double coef[4],
                           he_infer_plan *out)
{
    if (!q || !coef || !out || n_q < 1) return HE_EINVAL;
    return hehost::plan_lr_infer(q, n_q, level, s_z, s_w, coef, out);
}

he_status he_lr_infer(he_ctx *c, const he_ct *Z, int n_blocks, const he_ct *W, int cols, int rows, int layout,
                      const double *coef, const he_keys *k, int mode, he_ct *out)
{
    if (!coef) return he_lr_margins(c, Z, n_blocks, W, cols, rows, layout, k, mode, out);
    long long zbs = 0, obs = 0;
    TRY(margins_args(c, Z, n_blocks, W, cols, rows, layout, k, mode, out, 3, W ? W->level - 3 : 0, zbs, obs));
    const int l = W->level;
    he_infer_plan pl;
    TRY(hehost::plan_lr_infer(c->q.data(), c->nq, l, Z[0].scale, W->scale, coef, &pl));
    const long long unit = layout == HE_LAYOUT_FEATURES ? rows : 1;
    const int chunk = mode == 0 ? 1 : n_blocks;
    TRY(ensure_ws(c, infer_bytes(c, l, chunk)));
    if (mode == 2) {
        std::ostringstream key;
        key << "infer:" << (const void *)Z[0].data << ':' << zbs << ':' << n_blocks << ':' << Z[0].level << ':'
            << (const void *)W->data << ':' << l << ':' << cols << ':' << layout << ':' << k->gen << ':'
            << (const void *)k->sk << ':' << (const void *)out[0].data << ':' << obs << ':' << (const void *)c->ws
            << ':' << pl.k3 << ':' << pl.k2c << ':' << pl.k1 << ':' << pl.k0c;
        TRY(run_graph(c, key.str(), k->gen, [&] {
            return infer_impl(c, pl, Z, n_blocks, zbs, W, unit, cols, k, chunk, out[0].data, obs);
        }));
    } else {
        TRY(infer_impl(c, pl, Z, n_blocks, zbs, W, unit, cols, k, chunk, out[0].data, obs));
    }
    for (int b = 0; b < n_blocks; ++b) {
        out[b].level = l - 3;
        out[b].scale = pl.s_p;
    }
    return last_error();
}

he_status he_ntt(he_ctx *c, uint64_t *data, int n_limbs, int prime_idx0, int prime_period, int dir)
{
    if (!c || !data || n_limbs < 1 || prime_period < 1 || prime_idx0 < 0 || prime_idx0 + prime_period > c->np ||
        (dir != 1 && dir != -1))
        return HE_EINVAL;
    // limbs [n_limbs] = batches of prime_period consecutive positions
    if (n_limbs % prime_period) return HE_EINVAL;
    const int nbatch = n_limbs / prime_period;
    // positions prime_idx0 .. +period of a poly whose prime map is the identity
    hek::ntt_batch(c, data - (long long)prime_idx0 * c->N, (long long)prime_period * c->N, 0, nbatch, 1, prime_idx0,
                   prime_period, c->nq - 1, dir, nullptr, false);
    return last_error();
}

}  // extern "C"
