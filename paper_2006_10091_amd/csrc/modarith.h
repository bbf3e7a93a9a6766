// modarith.h -- 64-bit modular arithmetic for gfx950 (primes q < 2^60).
//
// gfx950 has no 64x64->128 multiply; __umul64hi and the 64-bit low product
// lower to chains of 32-bit v_mad_u64_u32 / v_mul_hi_u32.  Two reductions:
//   * Shoup (V. Shoup, NTL): a * w mod q for a constant w < q with the
//     precomputed w' = floor(w 2^64 / q); one high and two low products,
//     any a < 2^64, result in [0, 2q) before the final correction.
//   * Barrett (Handbook of Applied Cryptography, Alg. 14.42, base 2):
//     x mod q for x < 2^(2k), k = bitlen(q), mu = floor(2^(2k) / q).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;

// FP64 fast basis conversion (the centred conversion of the key switch, every
// target prime p below 2^46).  Each source residue v < q_i enters one exact
// lazy FP64 product with a constant below p, which needs |v| <= 33p: a source
// of at most kp + 4 bits (kp = bit length of p) enters whole, a wider one as
// two halves v = vh 2^S + vl with S = ceil(ki / 2), each half of at most
// kp + 4 bits.
__host__ __device__ constexpr int conv_split_bits(int ki) { return (ki + 1) / 2; }
__host__ __device__ constexpr bool conv_whole(int ki, int kp) { return ki <= kp + 4; }
__host__ __device__ constexpr bool conv_fp_ok(int ki_max, int kp)
{
    return kp <= 46 && conv_split_bits(ki_max) <= kp + 4;
}

// Per-prime constants (device table, one entry per prime of the chain).
struct PrimeInfo {
    u64 q;
    u64 mu;        // floor(2^(2k) / q)
    u64 ninv;      // N^{-1} mod q
    u64 ninv_sh;   // Shoup companion of ninv
    u64 r64;       // 2^64 mod q
    u64 r64_sh;    // Shoup companion of r64
    u64 one_sh;    // floor(2^64 / q): Shoup companion of 1 (reduces any u64)
    u32 k;         // bit length of q
    u32 pad;
};

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q)
{
    u64 s = a + b;
    return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
__device__ __forceinline__ u64 neg_mod(u64 a, u64 q) { return a ? q - a : 0; }

// a * w mod q, w < q, wp = floor(w 2^64 / q); a any 64-bit value.
__device__ __forceinline__ u64 mul_shoup(u64 a, u64 w, u64 wp, u64 q)
{
    u64 qh = __umul64hi(a, wp);
    u64 r = a * w - qh * q;
    return r >= q ? r - q : r;
}
// a mod q for any 64-bit a (Shoup with w = 1).
__device__ __forceinline__ u64 reduce64(u64 a, const PrimeInfo &p) { return mul_shoup(a, 1, p.one_sh, p.q); }

// (hi 2^64 + lo) mod q for x < 2^(2k).
__device__ __forceinline__ u64 barrett128(u64 hi, u64 lo, const PrimeInfo &p)
{
    const u32 k = p.k;
    u64 x1 = (hi << (65 - k)) | (lo >> (k - 1));     // floor(x / 2^(k-1)) < 2^(k+1)
    u64 h2 = __umul64hi(x1, p.mu);
    u64 l2 = x1 * p.mu;
    u64 qhat = (h2 << (63 - k)) | (l2 >> (k + 1));    // floor(x1 mu / 2^(k+1))
    u64 r = lo - qhat * p.q;                           // x - qhat q < 3q
    if (r >= p.q) r -= p.q;
    if (r >= p.q) r -= p.q;
    return r;
}
// a * b mod q for a, b < q.
__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const PrimeInfo &p)
{
    return barrett128(__umul64hi(a, b), a * b, p);
}
// (hi 2^64 + lo) mod q for ANY 128-bit value: hi is reduced first.
__device__ __forceinline__ u64 reduce128(u64 hi, u64 lo, const PrimeInfo &p)
{
    u64 h = reduce64(hi, p);                            // < q
    u64 t = mul_shoup(h, p.r64, p.r64_sh, p.q);         // hi 2^64 mod q
    return add_mod(t, reduce64(lo, p), p.q);
}
