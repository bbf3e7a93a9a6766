// kernels.hip -- HIP kernels of libhe for gfx950 (CDNA4, wave64).
//
// All arithmetic is exact modular integer arithmetic on uint64 limbs (no
// MFMA: there is no dense floating-point contraction on this path).
// Layout: a limb is N consecutive uint64; limbs of a polynomial are
// consecutive; launches address limbs through LimbBatch / (pointer, stride).
#include <algorithm>

#include "he_internal.h"

namespace {

constexpr int NTT_THREADS = 256;
constexpr int NTT_TILE = 4096;  // uint64 elements staged in LDS per workgroup (32 KiB)

__device__ __forceinline__ int prime_of(int pos, int ell, int nq) { return pos <= ell ? pos : nq + pos - ell - 1; }

__device__ __forceinline__ unsigned brev_n(unsigned x, int bits) { return __brev(x) >> (32 - bits); }

// v < k q with small k (v < 2^64): v mod q by repeated conditional subtraction of
// the largest fitting power-of-two multiple of q
__device__ __forceinline__ u64 reduce_small(u64 v, u64 q, int k)
{
    for (u64 m = q << (31 - __clz(k > 1 ? k - 1 : 1)); m >= q; m >>= 1)
        if (v >= m) v -= m;
    return v;
}

struct NttArgs {
    u64 *base;
    long long bstride;  // between batch entries
    long long cstride;  // between components within an entry
    int ncomp;
    int pos0;
    int skip_digit;  // 1: component c skips positions [c*alpha, min(c*alpha+alpha, ell+1))
    int alpha;
    int ell, nq;
    int logN, logN1;
    int zoff;  // first batch x component entry of this launch (chunked launches)
    int xcd;   // 1: column passes, 2: both passes take their blocks XCD-grouped (vb_xcd)
};

// Block index of a pass: blockIdx for the one-pass-per-launch kernels, a
// virtual one when a persistent kernel runs both passes (ntt_persist_t).
struct VB {
    int x, y, z;
};
__device__ __forceinline__ VB vb_here() { return VB{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z}; }
// Workgroups are dealt to the 8 XCDs in turn by linear id.  This bijection
// gives XCD k the contiguous eighth k of the (x fastest) block order, so the
// x-neighbours of one limb -- its 16 column strips -- run on one XCD one after
// another and fetch each row of the limb close together in time.  Grids whose
// size is not a multiple of 8 keep their order.
__device__ __forceinline__ VB vb_xcd()
{
    const unsigned gx = gridDim.x, gy = gridDim.y, total = gx * gy * gridDim.z;
    if (total & 7u) return vb_here();
    const unsigned id = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned j = (id & 7u) * (total >> 3) + (id >> 3);
    return VB{(int)(j % gx), (int)((j / gx) % gy), (int)(j / (gx * gy))};
}

__device__ __forceinline__ bool ntt_locate(const NttArgs &a, VB vb, u64 *&limb, int &pidx)
{
    const int pos = a.pos0 + vb.y;
    const int z = vb.z + a.zoff;
    const int b = z / a.ncomp, c = z % a.ncomp;
    if (a.skip_digit) {
        int s0 = c * a.alpha, s1 = min(s0 + a.alpha, a.ell + 1);
        if (pos >= s0 && pos < s1) return false;
    }
    limb = a.base + (long long)b * a.bstride + (long long)c * a.cstride + ((long long)pos << a.logN);
    pidx = prime_of(pos, a.ell, a.nq);
    return true;
}
__device__ __forceinline__ bool ntt_locate(const NttArgs &a, u64 *&limb, int &pidx)
{
    return ntt_locate(a, vb_here(), limb, pidx);
}

// Pass over the N1 "rows" (stride N2 = N/N1) for a tile of C consecutive
// columns: the stages m = 1 .. N1/2 of the Cooley-Tukey forward transform
// (inverse: Gentleman-Sande stages m = N1/2 .. 1, then the output scaling).
template <bool INV>
__global__ __launch_bounds__(NTT_THREADS) void ntt_cols(NttArgs a, const PrimeInfo *__restrict__ pinfo,
                                                        const u64 *__restrict__ tw, const u64 *__restrict__ tws,
                                                        const u64 *__restrict__ post)
{
    __shared__ u64 lds[NTT_TILE];
    u64 *limb;
    int pidx;
    if (!ntt_locate(a, limb, pidx)) return;
    const int N = 1 << a.logN, N1 = 1 << a.logN1, N2 = N >> a.logN1;
    const int C = min(NTT_TILE >> a.logN1, N2);
    const int col0 = blockIdx.x * C;
    const PrimeInfo p = pinfo[pidx];
    const u64 q = p.q;
    const u64 *W = tw + ((long long)pidx << a.logN);
    const u64 *Ws = tws + ((long long)pidx << a.logN);
    const int tot = N1 * C;
    for (int e = threadIdx.x; e < tot; e += NTT_THREADS) {
        int h = e / C, cc = e - h * C;
        lds[e] = limb[(long long)h * N2 + col0 + cc];
    }
    __syncthreads();
    if (!INV) {
        for (int m = 1; m < N1; m <<= 1) {
            const int th = N1 / (2 * m);
            for (int bf = threadIdx.x; bf < tot / 2; bf += NTT_THREADS) {
                int cc = bf % C, bi = bf / C;
                int g = bi / th, jj = bi - g * th;
                int h = g * 2 * th + jj;
                u64 w = W[m + g], ws = Ws[m + g];
                u64 u = lds[h * C + cc];
                u64 v = mul_shoup(lds[(h + th) * C + cc], w, ws, q);
                lds[h * C + cc] = add_mod(u, v, q);
                lds[(h + th) * C + cc] = sub_mod(u, v, q);
            }
            __syncthreads();
        }
    } else {
        for (int m = N1 / 2; m >= 1; m >>= 1) {
            const int th = N1 / (2 * m);
            for (int bf = threadIdx.x; bf < tot / 2; bf += NTT_THREADS) {
                int cc = bf % C, bi = bf / C;
                int g = bi / th, jj = bi - g * th;
                int h = g * 2 * th + jj;
                u64 w = W[m + g], ws = Ws[m + g];
                u64 x = lds[h * C + cc], y = lds[(h + th) * C + cc];
                lds[h * C + cc] = add_mod(x, y, q);
                lds[(h + th) * C + cc] = mul_shoup(sub_mod(x, y, q), w, ws, q);
            }
            __syncthreads();
        }
    }
    u64 sc = 0, scs = 0;
    if (INV) {
        if (post) {  // indexed from the first position of the launch
            sc = post[2 * blockIdx.y];
            scs = post[2 * blockIdx.y + 1];
        } else {
            sc = p.ninv;
            scs = p.ninv_sh;
        }
    }
    for (int e = threadIdx.x; e < tot; e += NTT_THREADS) {
        int h = e / C, cc = e - h * C;
        u64 v = lds[e];
        if (INV) v = mul_shoup(v, sc, scs, q);
        limb[(long long)h * N2 + col0 + cc] = v;
    }
}

// Pass over R consecutive rows of N2 contiguous elements: forward stages
// m = N1 .. N/2 (inverse: N/2 .. N1).  Stage m = N1 m', half-width t = N2/(2m'),
// twiddle index N1 m' + h m' + l/(2t) for row h, column l.
template <bool INV>
__global__ __launch_bounds__(NTT_THREADS) void ntt_rows(NttArgs a, const PrimeInfo *__restrict__ pinfo,
                                                        const u64 *__restrict__ tw, const u64 *__restrict__ tws)
{
    __shared__ u64 lds[NTT_TILE];
    u64 *limb;
    int pidx;
    if (!ntt_locate(a, limb, pidx)) return;
    const int N = 1 << a.logN, N1 = 1 << a.logN1, N2 = N >> a.logN1;
    const int R = min(NTT_TILE / N2, N1);
    const int h0 = blockIdx.x * R;
    const u64 q = pinfo[pidx].q;
    const u64 *W = tw + ((long long)pidx << a.logN);
    const u64 *Ws = tws + ((long long)pidx << a.logN);
    const int tot = R * N2;
    u64 *src = limb + (long long)h0 * N2;
    for (int e = threadIdx.x; e < tot; e += NTT_THREADS) lds[e] = src[e];
    __syncthreads();
    const int half = N2 / 2;
    if (!INV) {
        for (int mp = 1; mp < N2; mp <<= 1) {
            const int t = N2 / (2 * mp);
            for (int bf = threadIdx.x; bf < tot / 2; bf += NTT_THREADS) {
                int rr = bf / half, bi = bf - rr * half;
                int g = bi / t, jj = bi - g * t;
                int l = g * 2 * t + jj;
                int idx = N1 * mp + (h0 + rr) * mp + g;
                u64 *row = lds + rr * N2;
                u64 u = row[l];
                u64 v = mul_shoup(row[l + t], W[idx], Ws[idx], q);
                row[l] = add_mod(u, v, q);
                row[l + t] = sub_mod(u, v, q);
            }
            __syncthreads();
        }
    } else {
        for (int mp = N2 / 2; mp >= 1; mp >>= 1) {
            const int t = N2 / (2 * mp);
            for (int bf = threadIdx.x; bf < tot / 2; bf += NTT_THREADS) {
                int rr = bf / half, bi = bf - rr * half;
                int g = bi / t, jj = bi - g * t;
                int l = g * 2 * t + jj;
                int idx = N1 * mp + (h0 + rr) * mp + g;
                u64 *row = lds + rr * N2;
                u64 x = row[l], y = row[l + t];
                row[l] = add_mod(x, y, q);
                row[l + t] = mul_shoup(sub_mod(x, y, q), W[idx], Ws[idx], q);
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < tot; e += NTT_THREADS) src[e] = lds[e];
}

// ------------------------------------------------------------------ register-tiled NTT
// One pass transforms lines of M = 2^LM elements (pass A: the N1 "rows" of a
// column, stride N2; pass B: a contiguous row of N2).  A line is held by
// T = 2^LT threads with E = 2^LE elements each.  Stages whose butterfly
// half-width t >= T run with the strided layout x = tau + T k; stages with
// t < T run with the contiguous layout x = E tau + k; one padded LDS exchange
// switches between them.  Harvey's lazy butterflies keep forward values in
// [0, 4q) and inverse values in [0, 2q) until the last pass.
constexpr int LINE_THREADS = 256;

template <int LM>
struct LineShape {
    static constexpr int LE = (LM + 1) / 2 < 4 ? (LM + 1) / 2 : 4;
    static constexpr int LT = LM - LE;
    static constexpr int E = 1 << LE, T = 1 << LT, M = 1 << LM;
    static constexpr int LINES = LINE_THREADS / T;
    static constexpr int PADDED = M + M / E;  // one pad word per E elements
};

__device__ __forceinline__ u64 shoup_lazy(u64 a, u64 w, u64 wp, u64 q) { return a * w - __umul64hi(a, wp) * q; }

// forward (Cooley-Tukey) butterfly, inputs in [0, 4q), outputs in [0, 4q)
__device__ __forceinline__ void ct_bfly(u64 &x, u64 &y, u64 w, u64 wp, u64 q, u64 q2)
{
    u64 a = x >= q2 ? x - q2 : x;
    u64 t = shoup_lazy(y, w, wp, q);
    x = a + t;
    y = a - t + q2;
}
// inverse (Gentleman-Sande) butterfly, inputs in [0, 2q), outputs in [0, 2q)
__device__ __forceinline__ void gs_bfly(u64 &x, u64 &y, u64 w, u64 wp, u64 q, u64 q2)
{
    u64 s = x + y;
    s = s >= q2 ? s - q2 : s;
    u64 d = x - y + q2;
    y = shoup_lazy(d, w, wp, q);
    x = s;
}

__device__ __forceinline__ int lds_pad(int x, int LE) { return x + (x >> LE); }

// Twiddle index of a butterfly in line-stage s (m' = 2^s) for line element x:
// pass A: m' + x/(2t); pass B: N1 m' + h m' + x/(2t), with 2t = M / m'.
template <int LM, bool PASS_B>
__device__ __forceinline__ int tw_index(int s, int x, int h, int N1)
{
    const int g = x >> (LM - s);
    return PASS_B ? (N1 << s) + (h << s) + g : (1 << s) + g;
}

// forward stages s0..s1-1 on the strided layout (x = tau + T k)
template <int LM, bool PASS_B>
__device__ __forceinline__ void fwd_strided(u64 (&v)[LineShape<LM>::E], int tau, int h, int N1, const u64 *W,
                                            const u64 *Ws, u64 q, u64 q2)
{
    using S = LineShape<LM>;
#pragma unroll
    for (int s = 0; s < S::LE; ++s) {
        const int hk = 1 << (S::LE - 1 - s);
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            if (k & hk) continue;
            const int idx = tw_index<LM, PASS_B>(s, tau + S::T * k, h, N1);
            ct_bfly(v[k], v[k + hk], W[idx], Ws[idx], q, q2);
        }
    }
}
// forward stages LE..LM-1 on the contiguous layout (x = E tau + k)
template <int LM, bool PASS_B>
__device__ __forceinline__ void fwd_contig(u64 (&v)[LineShape<LM>::E], int tau, int h, int N1, const u64 *W,
                                           const u64 *Ws, u64 q, u64 q2)
{
    using S = LineShape<LM>;
#pragma unroll
    for (int s = S::LE; s < LM; ++s) {
        const int hk = 1 << (LM - 1 - s);
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            if (k & hk) continue;
            const int idx = tw_index<LM, PASS_B>(s, S::E * tau + k, h, N1);
            ct_bfly(v[k], v[k + hk], W[idx], Ws[idx], q, q2);
        }
    }
}
// inverse stages LM-1..LE on the contiguous layout
template <int LM, bool PASS_B>
__device__ __forceinline__ void inv_contig(u64 (&v)[LineShape<LM>::E], int tau, int h, int N1, const u64 *W,
                                           const u64 *Ws, u64 q, u64 q2)
{
    using S = LineShape<LM>;
#pragma unroll
    for (int s = LM - 1; s >= S::LE; --s) {
        const int hk = 1 << (LM - 1 - s);
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            if (k & hk) continue;
            const int idx = tw_index<LM, PASS_B>(s, S::E * tau + k, h, N1);
            gs_bfly(v[k], v[k + hk], W[idx], Ws[idx], q, q2);
        }
    }
}
// inverse stages LE-1..0 on the strided layout
template <int LM, bool PASS_B>
__device__ __forceinline__ void inv_strided(u64 (&v)[LineShape<LM>::E], int tau, int h, int N1, const u64 *W,
                                            const u64 *Ws, u64 q, u64 q2)
{
    using S = LineShape<LM>;
#pragma unroll
    for (int s = S::LE - 1; s >= 0; --s) {
        const int hk = 1 << (S::LE - 1 - s);
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            if (k & hk) continue;
            const int idx = tw_index<LM, PASS_B>(s, tau + S::T * k, h, N1);
            gs_bfly(v[k], v[k + hk], W[idx], Ws[idx], q, q2);
        }
    }
}

// ---- exact FP64 variant for primes below 2^49 (values stay integers < 2^51).
// a*w = hi + lo exactly (FMA); quotient floor(hi / q) is off by at most one,
// so the remainder hi - Q q + lo lies in [-q, 2q) and is corrected once each way.
__device__ __forceinline__ double mulmod_d(double a, double w, double q, double qinv)
{
    double hi = a * w;
    double lo = __fma_rn(a, w, -hi);
    double qt = floor(hi * qinv);
    double r = __fma_rn(-qt, q, hi) + lo;
    r = r < 0.0 ? r + q : r;
    return r >= q ? r - q : r;
}
__device__ __forceinline__ void ct_bfly_d(double &x, double &y, double w, double q, double q2, double qinv)
{
    double a = x >= q2 ? x - q2 : x;
    double t = mulmod_d(y, w, q, qinv);
    x = a + t;
    y = a - t + q2;
}
__device__ __forceinline__ void gs_bfly_d(double &x, double &y, double w, double q, double q2, double qinv)
{
    double s = x + y;
    s = s >= q2 ? s - q2 : s;
    double d = x - y + q2;
    y = mulmod_d(d, w, q, qinv);
    x = s;
}
template <int LM, bool PASS_B, bool INV, bool STRIDED>
__device__ __forceinline__ void stages_d(double (&v)[LineShape<LM>::E], int tau, int h, int N1, const double *W,
                                         double q, double qinv)
{
    using S = LineShape<LM>;
    const double q2 = 2.0 * q;
    constexpr int s_lo = STRIDED ? 0 : S::LE, s_hi = STRIDED ? S::LE : LM;
#pragma unroll
    for (int si = 0; si < s_hi - s_lo; ++si) {
        const int s = INV ? s_hi - 1 - si : s_lo + si;
        const int hk = STRIDED ? 1 << (S::LE - 1 - s) : 1 << (LM - 1 - s);
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            if (k & hk) continue;
            const int x = STRIDED ? tau + S::T * k : S::E * tau + k;
            const double w = W[tw_index<LM, PASS_B>(s, x, h, N1)];
            if (INV) gs_bfly_d(v[k], v[k + hk], w, q, q2, qinv);
            else ct_bfly_d(v[k], v[k + hk], w, q, q2, qinv);
        }
    }
}
// ---- signed lazy FP64 forward path for primes below 2^46.  For an integer-
// valued |a| <= 33q and 0 <= w < q, a*w = hi + lo exactly (FMA), the estimate
// Q = floor(hi / q) is within one of the true quotient (its FP64 error is below
// 3 * 2^-53 * 33q < 1), and fma(-Q, q, hi) + lo is exact and lies in (-q, 2q).
// The forward butterfly x +- t then needs no correction: each stage widens the
// range by 2q on each side, so the 16 stages of both passes keep every value
// inside [-32q, 33q], exact in FP64.  The row pass reduces at the end; the
// intermediate between the passes is stored as a signed integer.
__device__ __forceinline__ double mulmod_lazy_d(double a, double w, double q, double qinv)
{
    double hi = a * w;
    double lo = __fma_rn(a, w, -hi);
    double qt = floor(hi * qinv);
    return __fma_rn(-qt, q, hi) + lo;
}
// Exact conversions between FP64 and integers through the exponent bits (two
// operations each): an unsigned value below 2^52 is the mantissa of
// 2^52 + v; a signed one of magnitude below 2^51 (two's complement bits) that
// of 1.5 * 2^52 + v.  Every lazy path keeps its values inside these ranges.
__device__ __forceinline__ double d_from_u52(u64 v)
{
    return __longlong_as_double((long long)(v | 0x4330000000000000ull)) - 4503599627370496.0;
}
__device__ __forceinline__ double d_from_s51(u64 v)
{
    return __longlong_as_double((long long)(v + 0x4338000000000000ull)) - 6755399441055744.0;
}
__device__ __forceinline__ u64 u52_from_d(double x)
{
    return (u64)__double_as_longlong(x + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}
__device__ __forceinline__ u64 s51_from_d(double x)
{
    return (u64)__double_as_longlong(x + 6755399441055744.0) - 0x4338000000000000ull;
}
__device__ __forceinline__ double reduce_d(double x, double q, double qinv)
{
    double qt = floor(x * qinv);
    double r = __fma_rn(-qt, q, x);
    r = r < 0.0 ? r + q : r;
    return r >= q ? r - q : r;
}
template <int LM, bool PASS_B, bool STRIDED>
__device__ __forceinline__ void fwd_stages_ds(double (&v)[LineShape<LM>::E], int tau, int h, int N1, const double *W,
                                              double q, double qinv)
{
    using S = LineShape<LM>;
    constexpr int s_lo = STRIDED ? 0 : S::LE, s_hi = STRIDED ? S::LE : LM;
#pragma unroll
    for (int s = s_lo; s < s_hi; ++s) {
        const int hk = STRIDED ? 1 << (S::LE - 1 - s) : 1 << (LM - 1 - s);
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            if (k & hk) continue;
            const int x = STRIDED ? tau + S::T * k : S::E * tau + k;
            const double t = mulmod_lazy_d(v[k + hk], W[tw_index<LM, PASS_B>(s, x, h, N1)], q, qinv);
            v[k + hk] = v[k] - t;
            v[k] = v[k] + t;
        }
    }
}

// Inverse (Gentleman-Sande) counterpart for primes below 2^42: x' = x + y and
// y' = lazy((x - y) w), no corrections.  Sums double the range each stage, so
// one 8-stage pass from [0, q) stays inside |v| <= 2^8 q <= 2^50 (exact, and the
// quotient estimate of every product within one); each pass reduces at its end.
template <int LM, bool PASS_B, bool STRIDED>
__device__ __forceinline__ void inv_stages_ds(double (&v)[LineShape<LM>::E], int tau, int h, int N1, const double *W,
                                              double q, double qinv)
{
    using S = LineShape<LM>;
    constexpr int s_lo = STRIDED ? 0 : S::LE, s_hi = STRIDED ? S::LE : LM;
#pragma unroll
    for (int si = 0; si < s_hi - s_lo; ++si) {
        const int s = s_hi - 1 - si;
        const int hk = STRIDED ? 1 << (S::LE - 1 - s) : 1 << (LM - 1 - s);
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            if (k & hk) continue;
            const int x = STRIDED ? tau + S::T * k : S::E * tau + k;
            const double a = v[k], b = v[k + hk];
            v[k] = a + b;
            v[k + hk] = mulmod_lazy_d(a - b, W[tw_index<LM, PASS_B>(s, x, h, N1)], q, qinv);
        }
    }
}

template <int LM>
__device__ __forceinline__ void exch_d(double (&v)[LineShape<LM>::E], double *line, int tau, bool to_contig)
{
    using S = LineShape<LM>;
#pragma unroll
    for (int k = 0; k < S::E; ++k) line[lds_pad(to_contig ? tau + S::T * k : S::E * tau + k, S::LE)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < S::E; ++k) v[k] = line[lds_pad(to_contig ? S::E * tau + k : tau + S::T * k, S::LE)];
}

// strided <-> contiguous through LDS (line-private region of PADDED words)
template <int LM>
__device__ __forceinline__ void to_contig(u64 (&v)[LineShape<LM>::E], u64 *line, int tau)
{
    using S = LineShape<LM>;
#pragma unroll
    for (int k = 0; k < S::E; ++k) line[lds_pad(tau + S::T * k, S::LE)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < S::E; ++k) v[k] = line[lds_pad(S::E * tau + k, S::LE)];
}
template <int LM>
__device__ __forceinline__ void to_strided(u64 (&v)[LineShape<LM>::E], u64 *line, int tau)
{
    using S = LineShape<LM>;
#pragma unroll
    for (int k = 0; k < S::E; ++k) line[lds_pad(S::E * tau + k, S::LE)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < S::E; ++k) v[k] = line[lds_pad(tau + S::T * k, S::LE)];
}

__device__ __forceinline__ u64 reduce4q(u64 v, u64 q, u64 q2)
{
    v = v >= q2 ? v - q2 : v;
    return v >= q ? v - q : v;
}

// Fusion around the two passes (all optional, chosen per launch):
//   pass A prologue  PRO_MODDOWN : input = centred conversion of the source residues to the
//                                  limb's prime (ModDown: the special primes; rescale: q_l)
//   pass B (inverse) PRO_SRC     : read the limb from another buffer (out-of-place)
//   pass B epilogue  EPI_FINISH  : store base + (acc - x) P^{-1} instead of x
//   pass B epilogue  EPI_FIN_ACC : the same with no base and no addend (rescales):
//                                  fewer loads and registers
enum { PRO_NONE = 0, PRO_MODDOWN = 2, PRO_SRC = 3, PRO_MDRS = 5 };
enum { EPI_NONE = 0, EPI_FINISH = 1, EPI_FIN_ACC = 2 };

struct Fuse {
    const u64 *src;      // conversion sources (acc / last limbs) or source limbs (PRO_SRC)
    long long sbs, scs;  // batch / component strides of src
    long long soff;      // conversion: limb offset of the first source in src[b][c]
    int nsrc, sp0;       // conversion: number of sources, prime index of the first
    const u64 *cvt;      // conversion constants [source][target][2]: dn_conv / rs_one
    const u64 *cnt;      // centring term [target][2]: dn_p / rs_ql2 of the level
    const double *cvtd;  // FP64 forms: dn_convd / rs_oned of the level
    const double *cntd;  // dn_pd / rs_qld of the level
    int alpha, np, nk;
    const u64 *acc;      // finish: acc [b][comp][pos], strides as / acs
    long long as, acs;
    const u64 *base;     // finish: base [b][comp][pos] on the first nbase components
    long long bs, bcs;
    int nbase;
    u64 *out;            // finish: out [b][comp][pos]
    long long os, ocs;
    const u64 *pinv;     // finish: P^{-1} mod q_pos (+ Shoup)
    const u64 *add;      // finish: optional addend [b][comp][pos] on every component (may be out)
    long long ads, adcs;
    int has_kmul;        // PRO_SRC: multiply the source by kmul (mod each prime) as it is read
    i64 kmul;
    int has_kacc;        // finish: multiply acc by kacc (mod each prime) as it is read
    i64 kacc;
    const u64 *post;     // finish: final multiplier per target position (+ Shoup), or null
    const u64 *last;     // PRO_MDRS: the ModDown output's limb at q_l in coefficient form, [b][comp][N]
    int lpos;            // PRO_MDRS: l, the position of q_l
};

// k mod p for a signed 64-bit integer k
__device__ __forceinline__ u64 int_mod(i64 k, const PrimeInfo &p)
{
    const u64 mag = k < 0 ? (u64)(-(k + 1)) + 1 : (u64)k;
    const u64 r = reduce64(mag, p);
    return k < 0 ? neg_mod(r, p.q) : r;
}

constexpr int MAXW = 8;  // special primes the ModDown prologue reads (and the fused path's digit-width bound)

// per-workgroup constants of a conversion prologue
struct ConvConst {
    u64 c[MAXW], cs[MAXW], half[MAXW];
    u64 k, ks;
    int n;
    const u64 *src;
    // FP64 path (target below 2^46): per source the constant, its 2^S multiple
    // and split point (S = 0: the source enters whole), and Q mod p
    bool fp;
    double cd[MAXW], ch[MAXW], kd;
    int sh[MAXW];
};

// FP64 constants of a conversion to a target of bit length kp, sources
// s0 .. s0 + cc.n - 1 (their constant pairs e[i * es], e[i * es + 1])
__device__ __forceinline__ void conv_setup_fp(ConvConst &cc, const PrimeInfo *pinfo, int s0, const double *e,
                                              long long es, double kd, int kp)
{
    int kmax = 0;
#pragma unroll
    for (int i = 0; i < MAXW; ++i) {
        if (i < cc.n) {
            const int ki = (int)pinfo[s0 + i].k;
            kmax = max(kmax, ki);
            cc.cd[i] = e[i * es];
            cc.ch[i] = e[i * es + 1];
            cc.sh[i] = conv_whole(ki, kp) ? 0 : conv_split_bits(ki);
        }
    }
    cc.kd = kd;
    cc.fp = conv_fp_ok(kmax, kp);
}

// conversion prologue constants: sources are primes sp0 .. sp0 + nsrc - 1
// (ModDown: the special primes; rescale: q_l), the target is q_pos of this
// workgroup
__device__ __forceinline__ void conv_setup(const NttArgs &a, const Fuse &f, const PrimeInfo *pinfo, int tp,
                                           ConvConst &cc, VB vb)
{
    const int z = vb.z + a.zoff;
    const int b = z / a.ncomp, c = z % a.ncomp;
    const int pos = a.pos0 + vb.y;  // target q_pos
    cc.n = f.nsrc;
    cc.src = f.src + b * f.sbs + c * f.scs + (f.soff << a.logN);
#pragma unroll
    for (int i = 0; i < MAXW; ++i) {
        if (i < cc.n) {
            const u64 *e = f.cvt + ((long long)i * a.nq + pos) * 2;
            cc.c[i] = e[0];
            cc.cs[i] = e[1];
            cc.half[i] = pinfo[f.sp0 + i].q >> 1;
        }
    }
    cc.k = f.cnt[2 * pos];
    cc.ks = f.cnt[2 * pos + 1];
    conv_setup_fp(cc, pinfo, f.sp0, f.cvtd + (long long)pos * 2, 2LL * a.nq, f.cntd[pos], (int)pinfo[tp].k);
}

// centred fast basis conversion of one coefficient (offset off in the limb) to
// the prime p: exact 128-bit sum of the products, one reduction, then the
// centring correction cnt * Q mod p
__device__ __forceinline__ u64 conv_value(const ConvConst &cc, long long off, const PrimeInfo &p, int logN)
{
    u64 lo = 0, hi = 0, cnt = 0;
#pragma unroll
    for (int i = 0; i < MAXW; ++i) {
        if (i < cc.n) {
            const u64 v = cc.src[((long long)i << logN) + off];
            cnt += v > cc.half[i];
            const u64 pl = v * cc.c[i], ph = __umul64hi(v, cc.c[i]);
            lo += pl;
            hi += ph + (lo < pl);
        }
    }
    const u64 acc = reduce128(hi, lo, p);
    return sub_mod(acc, mul_shoup(cnt, cc.k, cc.ks, p.q), p.q);
}

// The conversion in FP64 (cc.fp: target p below 2^46) for the E elements of
// one column-pass thread (offsets
// off0 + k * step), source by source: the E loads of one source limb are
// issued together before their products, so a thread keeps E loads in flight
template <int E>
__device__ __forceinline__ void conv_column_d(const ConvConst &cc, long long off0, long long step, double (&d)[E],
                                              double pd, double pinv, int logN)
{
    u32 cnt[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        d[k] = 0.0;
        cnt[k] = 0;
    }
#pragma unroll
    for (int i = 0; i < MAXW; ++i) {
        if (i < cc.n) {
            const u64 *src = cc.src + ((long long)i << logN) + off0;
            u64 v[E];
#pragma unroll
            for (int k = 0; k < E; ++k) v[k] = src[k * step];
            const int sh = cc.sh[i];
            const double c0 = cc.cd[i], c1 = cc.ch[i];
            const u64 half = cc.half[i];
            if (sh == 0) {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    cnt[k] += v[k] > half;
                    d[k] += mulmod_lazy_d(d_from_u52(v[k]), c0, pd, pinv);
                }
            } else {
                const u64 m = (1ull << sh) - 1;
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    cnt[k] += v[k] > half;
                    d[k] += mulmod_lazy_d((double)(u32)(v[k] >> sh), c1, pd, pinv) +
                            mulmod_lazy_d((double)(u32)(v[k] & m), c0, pd, pinv);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) d[k] = reduce_d(__fma_rn(-(double)cnt[k], cc.kd, d[k]), pd, pinv);
}

// pass A: columns.  Thread (tau, cc) with cc fastest; LINES consecutive columns per workgroup.
// xbuf (plain forward / inverse only): where the intermediate between the two
// passes lives (the persistent kernel's L2-resident slot); null: in place.
template <int LOGN, bool INV, int PRO>
__device__ __forceinline__ void ntt_cols_body(const NttArgs &a, const PrimeInfo *__restrict__ pinfo,
                                              const u64 *__restrict__ tw, const u64 *__restrict__ tws,
                                              const u64 *__restrict__ post, const double *__restrict__ twd,
                                              const Fuse &f, VB vb, u64 *lds, u64 *xbuf, int tid)
{
    constexpr int LM = (LOGN + 1) / 2, N2 = 1 << (LOGN - LM);
    using S = LineShape<LM>;
    u64 *limb;
    int pidx;
    if (!ntt_locate(a, vb, limb, pidx)) return;
    u64 *xl = xbuf ? xbuf : limb;  // the intermediate's side of this pass
    const int cc = tid % S::LINES, tau = tid / S::LINES;
    const int col = vb.x * S::LINES + cc;
    const PrimeInfo p = pinfo[pidx];
    const u64 q = p.q, q2 = 2 * q;
    const u64 *W = tw + ((long long)pidx << LOGN);
    const u64 *Ws = tws + ((long long)pidx << LOGN);
    u64 *line = lds + cc * S::PADDED;
    ConvConst cv;
    constexpr bool CONV = PRO == PRO_MODDOWN || PRO == PRO_MDRS;
    if (CONV) conv_setup(a, f, pinfo, pidx, cv, vb);
    // PRO_MDRS (a ModDown and the rescale by q_l after it, in one transform):
    // the input is the ModDown conversion plus [P] times the rescale's centred
    // conversion of the ModDown output's last limb, conv + P x; both are
    // linear before the forward transform.  cv.k / cv.kd hold [P] here.
    const u64 *lastp = nullptr;
    u64 lq = 0;
    if (PRO == PRO_MDRS) {
        lastp = f.last + ((long long)(vb.z + a.zoff) << LOGN);
        lq = pinfo[f.lpos].q;
    }
    auto mdrs_d = [&](double conv, long long off, double qd, double qinv) -> double {
        const u64 v = lastp[off];
        const double x = (double)v - (v > (lq >> 1) ? (double)lq : 0.0);  // centred, |x| < q_l / 2
        return reduce_d(conv + mulmod_lazy_d(x, cv.kd, qd, qinv), qd, qinv);
    };
    auto load = [&](int row) -> u64 {
        const long long off = (long long)row * N2 + col;
        if (PRO == PRO_MDRS) {
            const u64 v = lastp[off];
            const u64 xm = v > (lq >> 1) ? sub_mod(reduce64(v, p), reduce64(lq, p), q) : reduce64(v, p);
            return add_mod(conv_value(cv, off, p, LOGN), mul_shoup(xm, cv.k, cv.ks, q), q);
        }
        if (PRO == PRO_MODDOWN) return conv_value(cv, off, p, LOGN);
        return limb[off];
    };
    if (q < (1ull << 49)) {  // exact FP64 path (quotient estimate off by at most one)
        const double qd = (double)q, qinv = 1.0 / qd;
        const double *Wd = twd + ((long long)pidx << LOGN);
        double *dl = reinterpret_cast<double *>(line);
        double d[S::E];
        if (!INV && q < (1ull << 46)) {  // signed lazy: the row pass reads a signed intermediate
            if (CONV && cv.fp) {
                conv_column_d<S::E>(cv, (long long)tau * N2 + col, (long long)S::T * N2, d, qd, qinv, LOGN);
                if (PRO == PRO_MDRS) {
#pragma unroll
                    for (int k = 0; k < S::E; ++k) d[k] = mdrs_d(d[k], (long long)(tau + S::T * k) * N2 + col, qd, qinv);
                }
            } else if (CONV) {
#pragma unroll
                for (int k = 0; k < S::E; ++k) d[k] = d_from_u52(load(tau + S::T * k));
            } else {
#pragma unroll
                for (int k = 0; k < S::E; ++k)
                    d[k] = d_from_u52(__builtin_nontemporal_load(limb + (long long)(tau + S::T * k) * N2 + col));
            }
            fwd_stages_ds<LM, false, true>(d, tau, 0, 0, Wd, qd, qinv);
            exch_d<LM>(d, dl, tau, true);
            fwd_stages_ds<LM, false, false>(d, tau, 0, 0, Wd, qd, qinv);
            if (xbuf) {  // L2-resident intermediate: a normal store, kept in the cache
#pragma unroll
                for (int k = 0; k < S::E; ++k) xl[(long long)(S::E * tau + k) * N2 + col] = s51_from_d(d[k]);
            } else {
#pragma unroll
                for (int k = 0; k < S::E; ++k)
                    __builtin_nontemporal_store(s51_from_d(d[k]), limb + (long long)(S::E * tau + k) * N2 + col);
            }
        } else if (!INV) {
#pragma unroll
            for (int k = 0; k < S::E; ++k) d[k] = (double)load(tau + S::T * k);
            stages_d<LM, false, false, true>(d, tau, 0, 0, Wd, qd, qinv);
            exch_d<LM>(d, dl, tau, true);
            stages_d<LM, false, false, false>(d, tau, 0, 0, Wd, qd, qinv);
#pragma unroll
            for (int k = 0; k < S::E; ++k) xl[(long long)(S::E * tau + k) * N2 + col] = (u64)d[k];
        } else if (q < (1ull << 42)) {  // lazy inverse: input reduced by the row pass
            if (xbuf) {
#pragma unroll
                for (int k = 0; k < S::E; ++k) d[k] = d_from_u52(xl[(long long)(S::E * tau + k) * N2 + col]);
            } else {
#pragma unroll
                for (int k = 0; k < S::E; ++k)
                    d[k] = d_from_u52(__builtin_nontemporal_load(limb + (long long)(S::E * tau + k) * N2 + col));
            }
            inv_stages_ds<LM, false, false>(d, tau, 0, 0, Wd, qd, qinv);
            exch_d<LM>(d, dl, tau, false);
            inv_stages_ds<LM, false, true>(d, tau, 0, 0, Wd, qd, qinv);
            u64 sc = post ? post[2 * vb.y] : p.ninv;
            const double scd = (double)sc;
#pragma unroll
            for (int k = 0; k < S::E; ++k)
                __builtin_nontemporal_store(u52_from_d(reduce_d(mulmod_lazy_d(d[k], scd, qd, qinv), qd, qinv)),
                                            limb + (long long)(tau + S::T * k) * N2 + col);
        } else {
#pragma unroll
            for (int k = 0; k < S::E; ++k) d[k] = (double)xl[(long long)(S::E * tau + k) * N2 + col];
            stages_d<LM, false, true, false>(d, tau, 0, 0, Wd, qd, qinv);
            exch_d<LM>(d, dl, tau, false);
            stages_d<LM, false, true, true>(d, tau, 0, 0, Wd, qd, qinv);
            u64 sc = post ? post[2 * vb.y] : p.ninv;
            const double scd = (double)sc;
#pragma unroll
            for (int k = 0; k < S::E; ++k)
                limb[(long long)(tau + S::T * k) * N2 + col] = (u64)mulmod_d(d[k], scd, qd, qinv);
        }
        return;
    }
    u64 v[S::E];
    if (!INV) {
#pragma unroll
        for (int k = 0; k < S::E; ++k) v[k] = load(tau + S::T * k);
        fwd_strided<LM, false>(v, tau, 0, 0, W, Ws, q, q2);
        to_contig<LM>(v, line, tau);
        fwd_contig<LM, false>(v, tau, 0, 0, W, Ws, q, q2);
#pragma unroll
        for (int k = 0; k < S::E; ++k) xl[(long long)(S::E * tau + k) * N2 + col] = v[k];
    } else {
#pragma unroll
        for (int k = 0; k < S::E; ++k) v[k] = xl[(long long)(S::E * tau + k) * N2 + col];
        inv_contig<LM, false>(v, tau, 0, 0, W, Ws, q, q2);
        to_strided<LM>(v, line, tau);
        inv_strided<LM, false>(v, tau, 0, 0, W, Ws, q, q2);
        u64 sc, scs;
        if (post) {
            sc = post[2 * vb.y];
            scs = post[2 * vb.y + 1];
        } else {
            sc = p.ninv;
            scs = p.ninv_sh;
        }
#pragma unroll
        for (int k = 0; k < S::E; ++k) limb[(long long)(tau + S::T * k) * N2 + col] = mul_shoup(v[k], sc, scs, q);
    }
}
// 4 waves per SIMD, the LDS bound of the 2^14..2^16 shapes: the ModDown
// prologue variants would take 137-140 VGPRs (3 waves) and fit in 128 with a
// 40-byte spill, measured 3% faster; the row pass's finish epilogue is not
// capped (166 VGPRs; at 128 it spills 132 bytes and ran 27% slower)
template <int LOGN, bool INV, int PRO>
__global__ __launch_bounds__(LINE_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void ntt_cols_t(
    NttArgs a, const PrimeInfo *__restrict__ pinfo, const u64 *__restrict__ tw, const u64 *__restrict__ tws,
    const u64 *__restrict__ post, const double *__restrict__ twd, Fuse f)
{
    using S = LineShape<(LOGN + 1) / 2>;
    __shared__ u64 lds[S::LINES * S::PADDED];
    ntt_cols_body<LOGN, INV, PRO>(a, pinfo, tw, tws, post, twd, f, a.xcd ? vb_xcd() : vb_here(), lds, nullptr,
                                  (int)threadIdx.x);
}

// pass B: rows.  Thread (line, tau) with tau fastest; LINES consecutive rows per workgroup.
// MODE: forward EPI_NONE / EPI_FINISH / EPI_FIN_ACC; inverse PRO_NONE / PRO_SRC.
// xbuf (plain forward / inverse only): the intermediate's location (read by
// the forward pass, written by the inverse one); null: in place.
template <int LOGN, bool INV, int MODE>
__device__ __forceinline__ void ntt_rows_body(const NttArgs &a, const PrimeInfo *__restrict__ pinfo,
                                              const u64 *__restrict__ tw, const u64 *__restrict__ tws,
                                              const double *__restrict__ twd, const Fuse &f, VB vb, u64 *lds,
                                              u64 *xbuf, int tid)
{
    constexpr int LM = LOGN - (LOGN + 1) / 2, N1 = 1 << ((LOGN + 1) / 2);
    constexpr bool FIN = !INV && (MODE == EPI_FINISH || MODE == EPI_FIN_ACC);
    constexpr bool BASE = MODE == EPI_FINISH;  // base and addend may be present
    constexpr bool SRC = INV && MODE == PRO_SRC;
    using S = LineShape<LM>;
    u64 *limb;
    int pidx;
    if (!ntt_locate(a, vb, limb, pidx)) return;
    const int tau = tid % S::T, ln = tid / S::T;
    const int h = vb.x * S::LINES + ln;
    const PrimeInfo p = pinfo[pidx];
    const u64 q = p.q, q2 = 2 * q;
    const u64 *W = tw + ((long long)pidx << LOGN);
    const u64 *Ws = tws + ((long long)pidx << LOGN);
    u64 *row = limb + (long long)h * S::M;
    u64 *line = lds + ln * S::PADDED;
    const int z = vb.z + a.zoff;
    const int b = z / a.ncomp, c = z % a.ncomp;
    const int pos = a.pos0 + vb.y;
    const long long roff = ((long long)pos << LOGN) + (long long)h * S::M;
    const u64 *in = row;
    if (SRC) in = f.src + b * f.sbs + c * f.scs + roff;
    // the persistent kernel's intermediate: read it (forward) or write it (inverse) through the cache
    u64 *xrow = xbuf ? xbuf + (long long)h * S::M : nullptr;
    if (!INV && xbuf) in = xrow;
    // finish epilogue: out = base + (acc - x) P^{-1}
    auto store = [&](int k, u64 x) {
        const int e = tau + S::T * k;
        if (FIN) {
            u64 av = f.acc[b * f.as + c * f.acs + roff + e];
            if (f.has_kacc) av = mul_mod(av, int_mod(f.kacc, p), p);
            u64 r = mul_shoup(sub_mod(av, x, q), f.pinv[2 * pos], f.pinv[2 * pos + 1], q);
            if (BASE && c < f.nbase) r = add_mod(r, f.base[b * f.bs + c * f.bcs + roff + e], q);
            if (BASE && f.add) r = add_mod(r, f.add[b * f.ads + c * f.adcs + roff + e], q);
            if (f.post) r = mul_shoup(r, f.post[2 * pos], f.post[2 * pos + 1], q);
            f.out[b * f.os + c * f.ocs + roff + e] = r;
        } else {
            __builtin_nontemporal_store(x, row + e);
        }
    };
    if (q < (1ull << 49)) {  // exact FP64 path (quotient estimate off by at most one)
        const double qd = (double)q, qinv = 1.0 / qd;
        const double *Wd = twd + ((long long)pidx << LOGN);
        double *dl = reinterpret_cast<double *>(line);
        double d[S::E];
        if (!INV && q < (1ull << 46)) {  // signed lazy: input is the column pass's signed intermediate
            if (xbuf) {
#pragma unroll
                for (int k = 0; k < S::E; ++k) d[k] = d_from_s51(in[tau + S::T * k]);
            } else {
#pragma unroll
                for (int k = 0; k < S::E; ++k) d[k] = d_from_s51(__builtin_nontemporal_load(in + tau + S::T * k));
            }
            // finish operands are loaded before the stages, so their latency overlaps them
            u64 fa[FIN ? S::E : 1], fb[BASE ? S::E : 1];
            if (FIN) {
                // fb = base + addend (each below q, so the sum is below 2q)
                const u64 *ap = f.acc + b * f.as + c * f.acs + roff + tau;
                const u64 *bp = f.base + b * f.bs + c * f.bcs + roff + tau;
                const u64 *dp = f.add + b * f.ads + c * f.adcs + roff + tau;
#pragma unroll
                for (int k = 0; k < S::E; ++k) {
                    fa[k] = ap[S::T * k];
                    if (BASE) fb[k] = (c < f.nbase ? bp[S::T * k] : 0) + (f.add ? dp[S::T * k] : 0);
                }
            }
            fwd_stages_ds<LM, true, true>(d, tau, h, N1, Wd, qd, qinv);
            exch_d<LM>(d, dl, tau, true);
            fwd_stages_ds<LM, true, false>(d, tau, h, N1, Wd, qd, qinv);
            __syncthreads();
            exch_d<LM>(d, dl, tau, false);
            if (FIN) {
                // base (+ addend) + (acc - x) P^{-1}: the lazy product is in (-q, 2q), the sum in (-q, 4q)
                const double pinv = d_from_u52(f.pinv[2 * pos]);
                const double postd = f.post ? d_from_u52(f.post[2 * pos]) : 0.0;
                u64 *op = f.out + b * f.os + c * f.ocs + roff + tau;
                const double ka = f.has_kacc ? d_from_u52(int_mod(f.kacc, p)) : 0.0;
#pragma unroll
                for (int k = 0; k < S::E; ++k) {
                    const double x = reduce_d(d[k], qd, qinv);
                    // kacc acc is a lazy product in (-q, 2q); minus x it stays within (-2q, 2q)
                    const double av = f.has_kacc ? mulmod_lazy_d(d_from_u52(fa[k]), ka, qd, qinv) : d_from_u52(fa[k]);
                    double r = mulmod_lazy_d(av - x, pinv, qd, qinv);
                    if (BASE) r += d_from_u52(fb[k]);
                    if (f.post)
                        op[S::T * k] = u52_from_d(reduce_d(mulmod_lazy_d(r, postd, qd, qinv), qd, qinv));
                    else
                        op[S::T * k] = u52_from_d(reduce_d(r, qd, qinv));
                }
            } else {
#pragma unroll
                for (int k = 0; k < S::E; ++k) store(k, u52_from_d(reduce_d(d[k], qd, qinv)));
            }
            return;
        }
        if (!INV && xbuf) {
#pragma unroll
            for (int k = 0; k < S::E; ++k) d[k] = d_from_u52(in[tau + S::T * k]);
        } else {
#pragma unroll
            for (int k = 0; k < S::E; ++k) d[k] = d_from_u52(__builtin_nontemporal_load(in + tau + S::T * k));
        }
        if (SRC && f.has_kmul) {  // the source times kmul, reduced to [0, q)
            const double kd = d_from_u52(int_mod(f.kmul, p));
#pragma unroll
            for (int k = 0; k < S::E; ++k) d[k] = mulmod_d(d[k], kd, qd, qinv);
        }
        if (!INV) {
            stages_d<LM, true, false, true>(d, tau, h, N1, Wd, qd, qinv);
            exch_d<LM>(d, dl, tau, true);
            stages_d<LM, true, false, false>(d, tau, h, N1, Wd, qd, qinv);
            __syncthreads();
            exch_d<LM>(d, dl, tau, false);
            const double q2d = 2.0 * qd;
#pragma unroll
            for (int k = 0; k < S::E; ++k) {
                double x = d[k] >= q2d ? d[k] - q2d : d[k];
                store(k, (u64)(x >= qd ? x - qd : x));
            }
        } else if (q < (1ull << 42)) {  // lazy inverse, reduced for the column pass
            exch_d<LM>(d, dl, tau, true);
            inv_stages_ds<LM, true, false>(d, tau, h, N1, Wd, qd, qinv);
            __syncthreads();
            exch_d<LM>(d, dl, tau, false);
            inv_stages_ds<LM, true, true>(d, tau, h, N1, Wd, qd, qinv);
            if (xbuf) {
#pragma unroll
                for (int k = 0; k < S::E; ++k) xrow[tau + S::T * k] = u52_from_d(reduce_d(d[k], qd, qinv));
            } else {
#pragma unroll
                for (int k = 0; k < S::E; ++k)
                    __builtin_nontemporal_store(u52_from_d(reduce_d(d[k], qd, qinv)), row + tau + S::T * k);
            }
        } else {
            exch_d<LM>(d, dl, tau, true);
            stages_d<LM, true, true, false>(d, tau, h, N1, Wd, qd, qinv);
            __syncthreads();
            exch_d<LM>(d, dl, tau, false);
            stages_d<LM, true, true, true>(d, tau, h, N1, Wd, qd, qinv);
            u64 *wr = xbuf ? xrow : row;
#pragma unroll
            for (int k = 0; k < S::E; ++k) wr[tau + S::T * k] = (u64)d[k];
        }
        return;
    }
    u64 v[S::E];
    if (!INV && xbuf) {
#pragma unroll
        for (int k = 0; k < S::E; ++k) v[k] = in[tau + S::T * k];
    } else {
#pragma unroll
        for (int k = 0; k < S::E; ++k) v[k] = __builtin_nontemporal_load(in + tau + S::T * k);
    }
    if (SRC && f.has_kmul) {
        const u64 kq = int_mod(f.kmul, p);
#pragma unroll
        for (int k = 0; k < S::E; ++k) v[k] = mul_mod(v[k], kq, p);
    }
    if (!INV) {
        fwd_strided<LM, true>(v, tau, h, N1, W, Ws, q, q2);
        to_contig<LM>(v, line, tau);
        fwd_contig<LM, true>(v, tau, h, N1, W, Ws, q, q2);
        __syncthreads();
        to_strided<LM>(v, line, tau);
#pragma unroll
        for (int k = 0; k < S::E; ++k) store(k, reduce4q(v[k], q, q2));
    } else {
        to_contig<LM>(v, line, tau);
        inv_contig<LM, true>(v, tau, h, N1, W, Ws, q, q2);
        __syncthreads();
        to_strided<LM>(v, line, tau);
        inv_strided<LM, true>(v, tau, h, N1, W, Ws, q, q2);
        if (xbuf) {
#pragma unroll
            for (int k = 0; k < S::E; ++k) xrow[tau + S::T * k] = v[k];
        } else {
#pragma unroll
            for (int k = 0; k < S::E; ++k) __builtin_nontemporal_store(v[k], row + tau + S::T * k);
        }
    }
}
template <int LOGN, bool INV, int MODE>
__global__ __launch_bounds__(LINE_THREADS) void ntt_rows_t(NttArgs a, const PrimeInfo *__restrict__ pinfo,
                                                           const u64 *__restrict__ tw, const u64 *__restrict__ tws,
                                                           const double *__restrict__ twd, Fuse f)
{
    using S = LineShape<LOGN - (LOGN + 1) / 2>;
    __shared__ u64 lds[S::LINES * S::PADDED];
    ntt_rows_body<LOGN, INV, MODE>(a, pinfo, tw, tws, twd, f, a.xcd == 2 ? vb_xcd() : vb_here(), lds, nullptr,
                                   (int)threadIdx.x);
}

// Row pass of the extended digits' forward NTT fused with the key-switch
// inner product: for position t of entry b, each digit j's rows go through
// the last NTT stages (or are read from d2 when t lies inside digit j, already
// in NTT form), are multiplied by key_j[0] and key_j[1] and accumulated in
// registers; only acc[b][comp][t] is written.  Entries are the fastest grid
// index, so consecutive workgroups share key rows in L2.
struct KsArgs {
    const u64 *d2;
    long long d2s;
    const u64 *ext;  // column-pass intermediates [b][j][pos][N]
    long long es, ds;
    const u64 *key;  // [j][2][np][N], shared by the batch unless per_entry
    hek::EntryKeys ek;
    int per_entry;
    u64 *acc;  // [b][2][nb][N]
    long long as;
    int alpha, beta, ell, nq, np, nb;
    int nent;  // entries B
};

template <int LOGN>
__global__ __launch_bounds__(LINE_THREADS) void ntt_rows_ks_t(KsArgs a, const PrimeInfo *__restrict__ pinfo,
                                                              const u64 *__restrict__ tw, const u64 *__restrict__ tws,
                                                              const double *__restrict__ twd)
{
    constexpr int LM = LOGN - (LOGN + 1) / 2, N1 = 1 << ((LOGN + 1) / 2);
    using S = LineShape<LM>;
    __shared__ u64 lds[S::LINES * S::PADDED];
    // one-dimensional grid over (entry, row block, position).  Workgroups are
    // dealt to the 8 XCDs in turn; when the (row block, position) pairs split
    // evenly, every entry of one pair lands on the same XCD, so that pair's
    // key rows are fetched into one L2 once instead of once per XCD.
    constexpr int NRB = N1 / S::LINES;
    const int w = blockIdx.x, npair = NRB * a.nb;
    int b, pr;
    if ((npair & 7) == 0) {
        const int sidx = w >> 3;
        b = sidx % a.nent;
        pr = (sidx / a.nent) * 8 + (w & 7);
    } else {
        b = w % a.nent;
        pr = w / a.nent;
    }
    const int t = pr / NRB;
    const int tau = threadIdx.x % S::T, ln = threadIdx.x / S::T;
    const int h = (pr % NRB) * S::LINES + ln;
    const int tp = prime_of(t, a.ell, a.nq);
    const PrimeInfo p = pinfo[tp];
    const u64 q = p.q;
    const long long roff = ((long long)t << LOGN) + (long long)h * S::M;
    const long long keylimb = (long long)a.np << LOGN;
    const u64 *key = (a.per_entry ? a.ek.k[b] : a.key) + ((long long)tp << LOGN) + (long long)h * S::M;
    u64 *line = lds + ln * S::PADDED;
    u64 *o = a.acc + b * a.as + roff;
    if (q < (1ull << 46)) {  // lazy FP64: products in (-q, 2q), sums of beta <= 12 exact
        const double qd = (double)q, qinv = 1.0 / qd;
        const double *Wd = twd + ((long long)tp << LOGN);
        double *dl = reinterpret_cast<double *>(line);
        double s0[S::E], s1[S::E];
#pragma unroll
        for (int k = 0; k < S::E; ++k) s0[k] = s1[k] = 0.0;
        for (int j = 0; j < a.beta; ++j) {
            const int d0 = j * a.alpha, d1 = min(d0 + a.alpha, a.ell + 1);
            double d[S::E];
            if (t >= d0 && t < d1) {
                const u64 *src = a.d2 + b * a.d2s + roff;
#pragma unroll
                for (int k = 0; k < S::E; ++k) d[k] = d_from_u52(src[tau + S::T * k]);
            } else {
                const u64 *src = a.ext + b * a.es + j * a.ds + roff;
#pragma unroll
                for (int k = 0; k < S::E; ++k)
                    d[k] = d_from_s51(__builtin_nontemporal_load(src + tau + S::T * k));
                fwd_stages_ds<LM, true, true>(d, tau, h, N1, Wd, qd, qinv);
                exch_d<LM>(d, dl, tau, true);
                fwd_stages_ds<LM, true, false>(d, tau, h, N1, Wd, qd, qinv);
                __syncthreads();
                exch_d<LM>(d, dl, tau, false);
                __syncthreads();  // the next digit's exchange rewrites the line
            }
            const u64 *kj = key + (long long)j * 2 * keylimb;
#pragma unroll
            for (int k = 0; k < S::E; ++k) {
                const int e = tau + S::T * k;
                s0[k] += mulmod_lazy_d(d[k], d_from_u52(kj[e]), qd, qinv);
                s1[k] += mulmod_lazy_d(d[k], d_from_u52(kj[keylimb + e]), qd, qinv);
            }
        }
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            const int e = tau + S::T * k;
            o[e] = u52_from_d(reduce_d(s0[k], qd, qinv));
            o[((long long)a.nb << LOGN) + e] = u52_from_d(reduce_d(s1[k], qd, qinv));
        }
        return;
    }
    // larger primes: Harvey-lazy Shoup stages, canonical values, 128-bit products
    const u64 *W = tw + ((long long)tp << LOGN);
    const u64 *Ws = tws + ((long long)tp << LOGN);
    const u64 q2 = 2 * q;
    u64 s0[S::E], s1[S::E];
#pragma unroll
    for (int k = 0; k < S::E; ++k) s0[k] = s1[k] = 0;
    for (int j = 0; j < a.beta; ++j) {
        const int d0 = j * a.alpha, d1 = min(d0 + a.alpha, a.ell + 1);
        u64 v[S::E];
        if (t >= d0 && t < d1) {
            const u64 *src = a.d2 + b * a.d2s + roff;
#pragma unroll
            for (int k = 0; k < S::E; ++k) v[k] = src[tau + S::T * k];
        } else {
            const u64 *src = a.ext + b * a.es + j * a.ds + roff;
#pragma unroll
            for (int k = 0; k < S::E; ++k) v[k] = __builtin_nontemporal_load(src + tau + S::T * k);
            fwd_strided<LM, true>(v, tau, h, N1, W, Ws, q, q2);
            to_contig<LM>(v, line, tau);
            fwd_contig<LM, true>(v, tau, h, N1, W, Ws, q, q2);
            __syncthreads();
            to_strided<LM>(v, line, tau);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < S::E; ++k) v[k] = reduce4q(v[k], q, q2);
        }
        const u64 *kj = key + (long long)j * 2 * keylimb;
#pragma unroll
        for (int k = 0; k < S::E; ++k) {
            const int e = tau + S::T * k;
            s0[k] = add_mod(s0[k], mul_mod(v[k], kj[e], p), q);
            s1[k] = add_mod(s1[k], mul_mod(v[k], kj[keylimb + e], p), q);
        }
    }
#pragma unroll
    for (int k = 0; k < S::E; ++k) {
        const int e = tau + S::T * k;
        o[e] = s0[k];
        o[((long long)a.nb << LOGN) + e] = s1[k];
    }
}

// ------------------------------------------------------------------ elementwise
struct EwArgs {
    u64 *x, *y, *o;
    long long xb, xc, yb, yc, ob, oc;  // batch / component strides
    int ncomp, pos0, ell, nq, logN;
};

__device__ __forceinline__ long long ew_off(long long bs, long long cs, int b, int c, int pos, int logN)
{
    return (long long)b * bs + (long long)c * cs + ((long long)pos << logN);
}

// op: 0 add, 1 sub, 2 mul by integer, 3 mul by plaintext (y: [pos][N], no batch/comp), 4 copy,
// 5 add the integer k to every coefficient (NTT form: a constant polynomial)
template <int OP>
__global__ __launch_bounds__(256) void ew_kernel(EwArgs a, const PrimeInfo *__restrict__ pinfo, i64 k)
{
    const int pos = a.pos0 + (int)blockIdx.y;
    const int z = (int)blockIdx.z;
    const int b = z / a.ncomp, c = z % a.ncomp;
    const int N = 1 << a.logN;
    const PrimeInfo p = pinfo[prime_of(pos, a.ell, a.nq)];
    const u64 *x = a.x + ew_off(a.xb, a.xc, b, c, pos, a.logN);
    u64 *o = a.o + ew_off(a.ob, a.oc, b, c, pos, a.logN);
    const u64 *y = nullptr;
    if (OP == 0 || OP == 1) y = a.y + ew_off(a.yb, a.yc, b, c, pos, a.logN);
    if (OP == 3) y = a.y + ((long long)pos << a.logN);
    u64 kq = 0;
    if (OP == 2 || OP == 5) {
        u64 mag = k < 0 ? (u64)(-(k + 1)) + 1 : (u64)k;
        kq = reduce64(mag, p);
        if (k < 0) kq = neg_mod(kq, p.q);
    }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256) {
        u64 v;
        if (OP == 0) v = add_mod(x[i], y[i], p.q);
        else if (OP == 1) v = sub_mod(x[i], y[i], p.q);
        else if (OP == 2) v = mul_mod(x[i], kq, p);
        else if (OP == 3) v = mul_mod(x[i], y[i], p);
        else if (OP == 5) v = add_mod(x[i], kq, p.q);
        else v = x[i];
        o[i] = v;
    }
}

// tensor: out0 = x0 y0, out1 = x0 y1 + x1 y0, out2 = x1 y1 (limbs 0..l)
__global__ __launch_bounds__(256) void tensor_kernel(const u64 *__restrict__ x, long long xb, long long xc,
                                                     const u64 *__restrict__ y, long long yb, long long yc,
                                                     u64 *__restrict__ o, long long ob, long long oc,
                                                     const PrimeInfo *__restrict__ pinfo, int logN)
{
    const int i = blockIdx.y, b = blockIdx.z;
    const PrimeInfo p = pinfo[i];
    const long long li = (long long)i << logN;
    const u64 *x0 = x + b * xb + li, *x1 = x0 + xc;
    const u64 *y0 = y + b * yb + li, *y1 = y0 + yc;
    u64 *o0 = o + b * ob + li, *o1 = o0 + oc, *o2 = o1 + oc;
    const int N = 1 << logN;
    for (int t = blockIdx.x * 256 + threadIdx.x; t < N; t += gridDim.x * 256) {
        u64 a0 = x0[t], a1 = x1[t], b0 = y0[t], b1 = y1[t];
        o0[t] = mul_mod(a0, b0, p);
        o1[t] = add_mod(mul_mod(a0, b1, p), mul_mod(a1, b0, p), p.q);
        o2[t] = mul_mod(a1, b1, p);
    }
}

// Elementwise operations driven by a device-side operand table: workgroup
// (x, limb, entry) reads entry blockIdx.z's pointers and limb count, so one
// launch covers operations of any mix of levels (workgroups past an entry's
// limbs return at once).  OP 0 add, 4 copy, 6 tensor (see OpDesc).
template <int OP>
__global__ __launch_bounds__(256) void desc_ew_kernel(const hek::OpDesc *__restrict__ tab,
                                                      const PrimeInfo *__restrict__ pinfo, int logN)
{
    const hek::OpDesc d = tab[blockIdx.z];
    const int i = blockIdx.y;
    if (i >= d.limbs) return;
    const PrimeInfo p = pinfo[i];
    const long long li = (long long)i << logN, lc = (long long)d.limbs << logN;
    const long long xc = d.xl > 0 ? (long long)d.xl << logN : lc;
    const int N = 1 << logN;
    const u64 *x0 = d.x + li, *x1 = x0 + xc;
    u64 *o0 = d.o + li, *o1 = o0 + lc;
    const u64 kq = OP == 2 ? int_mod(d.k, p) : 0;
    for (int t = blockIdx.x * 256 + threadIdx.x; t < N; t += gridDim.x * 256) {
        if (OP == 4) {
            o0[t] = x0[t];
            o1[t] = x1[t];
        } else if (OP == 2) {
            o0[t] = mul_mod(x0[t], kq, p);
            o1[t] = mul_mod(x1[t], kq, p);
        } else if (OP == 3) {
            const u64 m = d.y[li + t];
            o0[t] = mul_mod(x0[t], m, p);
            o1[t] = mul_mod(x1[t], m, p);
        } else {
            const u64 *y0 = d.y + li, *y1 = y0 + lc;
            if (OP == 0) {
                o0[t] = add_mod(x0[t], y0[t], p.q);
                o1[t] = add_mod(x1[t], y1[t], p.q);
            } else {
                const u64 a0 = x0[t], a1 = x1[t], b0 = y0[t], b1 = y1[t];
                o0[t] = mul_mod(a0, b0, p);
                o1[t] = add_mod(mul_mod(a0, b1, p), mul_mod(a1, b0, p), p.q);
                o1[t + lc] = mul_mod(a1, b1, p);
            }
        }
    }
}

// The gradient terms of nb blocks summed into one degree-4 ciphertext at level
// lp (limbs 0..lp), straight into g (accumulated onto g when acc):
//   g += sum_b A_b (x) B3_b + M_b (x) Z1_b + k0 Z_b  (+ A_b (x) Z2_b when z2)
// where (x) is the tensor product of polynomials in the secret: A and B3 are
// of degree 2 (three components, not relinearised), M, Z1, Z2 and Z of
// degree 1, and d_k of a product sums the component products of degrees
// i + j = k.  No block's terms are stored.  Primes below 2^46: lazy FP64
// products (at most 6 in (-q, 2q) per component and block), one reduction per
// block; wider primes: Barrett products and modular sums.
struct TermArgs {
    const u64 *a, *b3;  // level lp, [b][3][lp+1][N]: batch stride as, component stride pc
    long long as;
    const u64 *z1, *z2;  // level lp, [b][2][lp+1][N]: batch stride ps, component stride pc
    long long ps, pc;
    const u64 *m;  // M: batch stride ms, component stride mc (first lp+1 limbs read)
    long long ms, mc;
    const u64 *z;  // data: batch stride zs, component stride zc
    long long zs, zc;
    u64 *g;  // [5][lp+1][N], component stride pc
    i64 k0;
    int nb, acc, logN;
};

__global__ __launch_bounds__(256) void terms_sum_kernel(TermArgs a, const PrimeInfo *__restrict__ pinfo)
{
    const int i = blockIdx.y;
    const PrimeInfo p = pinfo[i];
    const long long off = ((long long)i << a.logN) + blockIdx.x * 256 + threadIdx.x;
    const long long pc = a.pc;
    const u64 mag = a.k0 < 0 ? (u64)(-(a.k0 + 1)) + 1 : (u64)a.k0;
    u64 kq = reduce64(mag, p);
    if (a.k0 < 0) kq = neg_mod(kq, p.q);
    u64 *g = a.g + off;
    if (p.q < (1ull << 46)) {
        const double qd = (double)p.q, qinv = 1.0 / qd, kd = d_from_u52(kq);
        double gk[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) gk[k] = a.acc ? d_from_u52(g[k * pc]) : 0.0;
        auto mm = [&](double x, double y) { return mulmod_lazy_d(x, y, qd, qinv); };
        for (int b = 0; b < a.nb; ++b) {
            const long long ab = b * a.as + off, pb = b * a.ps + off;
            double x[3], y[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                x[k] = d_from_u52(a.a[ab + k * pc]);
                y[k] = d_from_u52(a.b3[ab + k * pc]);
            }
            const double m0 = d_from_u52(a.m[b * a.ms + off]), m1 = d_from_u52(a.m[b * a.ms + a.mc + off]);
            const double u0 = d_from_u52(a.z1[pb]), u1 = d_from_u52(a.z1[pb + pc]);
            const double z0 = d_from_u52(a.z[b * a.zs + off]), z1 = d_from_u52(a.z[b * a.zs + a.zc + off]);
            double t0 = mm(x[0], y[0]) + mm(m0, u0) + mm(z0, kd);
            double t1 = mm(x[0], y[1]) + mm(x[1], y[0]) + mm(m0, u1) + mm(m1, u0) + mm(z1, kd);
            double t2 = mm(x[0], y[2]) + mm(x[1], y[1]) + mm(x[2], y[0]) + mm(m1, u1);
            double t3 = mm(x[1], y[2]) + mm(x[2], y[1]);
            double t4 = mm(x[2], y[2]);
            if (a.z2) {
                const double w0 = d_from_u52(a.z2[pb]), w1 = d_from_u52(a.z2[pb + pc]);
                t0 += mm(x[0], w0);
                t1 += mm(x[0], w1) + mm(x[1], w0);
                t2 += mm(x[1], w1) + mm(x[2], w0);
                t3 += mm(x[2], w1);
            }
            gk[0] = reduce_d(gk[0] + t0, qd, qinv);
            gk[1] = reduce_d(gk[1] + t1, qd, qinv);
            gk[2] = reduce_d(gk[2] + t2, qd, qinv);
            gk[3] = reduce_d(gk[3] + t3, qd, qinv);
            gk[4] = reduce_d(gk[4] + t4, qd, qinv);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) g[k * pc] = u52_from_d(gk[k]);
        return;
    }
    u64 gk[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) gk[k] = a.acc ? g[k * pc] : 0;
    auto mm = [&](u64 x, u64 y) { return mul_mod(x, y, p); };
    auto ad = [&](u64 x, u64 y) { return add_mod(x, y, p.q); };
    for (int b = 0; b < a.nb; ++b) {
        const long long ab = b * a.as + off, pb = b * a.ps + off;
        u64 x[3], y[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            x[k] = a.a[ab + k * pc];
            y[k] = a.b3[ab + k * pc];
        }
        const u64 m0 = a.m[b * a.ms + off], m1 = a.m[b * a.ms + a.mc + off];
        const u64 u0 = a.z1[pb], u1 = a.z1[pb + pc];
        const u64 z0 = a.z[b * a.zs + off], z1 = a.z[b * a.zs + a.zc + off];
        gk[0] = ad(gk[0], ad(ad(mm(x[0], y[0]), mm(m0, u0)), mm(z0, kq)));
        gk[1] = ad(gk[1], ad(ad(ad(mm(x[0], y[1]), mm(x[1], y[0])), ad(mm(m0, u1), mm(m1, u0))), mm(z1, kq)));
        gk[2] = ad(gk[2], ad(ad(mm(x[0], y[2]), mm(x[1], y[1])), ad(mm(x[2], y[0]), mm(m1, u1))));
        gk[3] = ad(gk[3], ad(mm(x[1], y[2]), mm(x[2], y[1])));
        gk[4] = ad(gk[4], mm(x[2], y[2]));
        if (a.z2) {
            const u64 w0 = a.z2[pb], w1 = a.z2[pb + pc];
            gk[0] = ad(gk[0], mm(x[0], w0));
            gk[1] = ad(gk[1], ad(mm(x[0], w1), mm(x[1], w0)));
            gk[2] = ad(gk[2], ad(mm(x[1], w1), mm(x[2], w0)));
            gk[3] = ad(gk[3], mm(x[2], w1));
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) g[k * pc] = gk[k];
}

// Baby-step margin products: o[blk] = sum_{b < nbaby} Zb[blk] (x) Wb[b], one
// degree-2 ciphertext per block (NTT domain, limbs 0..l).  Zb[blk] is the block
// itself for b = 0 and its rotated copy zr[blk][b-1] otherwise; Wb[0] = w and
// Wb[b] = wr[b-1].  A thread keeps the W values of its coefficient in
// registers and streams every block's data once.  Primes below 2^46: exact
// lazy FP64 products, each in (-q, 2q), at most 2 * MAX_BABY = 32 of them per
// sum, so every sum stays inside (-32q, 64q) and one reduction ends it; wider
// primes: Barrett products and modular sums.
constexpr int MAX_BABY = 16;
struct BabyArgs {
    const u64 *z;
    long long zb, zc;  // blocks: block stride, component stride
    const u64 *zr;
    long long zrb, zrs, zrc;  // rotated data: block stride, baby-step stride, component stride
    const u64 *w;
    long long wc;  // W: component stride
    const u64 *wr;
    long long wrs, wrc;  // rotated W: baby-step stride, component stride
    u64 *o;
    long long ob, oc;  // output: block stride, component stride
    int nbaby, nblk, logN;
};

// NB (compile time) baby steps, so the 2 NB loads of a block are issued
// together; blockIdx.z selects a chunk of BABY_CHUNK blocks.
constexpr int BABY_CHUNK = 24;
template <int NB>
__global__ __launch_bounds__(256) void baby_sum_kernel(BabyArgs a, const PrimeInfo *__restrict__ pinfo)
{
    const int i = blockIdx.y;
    const PrimeInfo p = pinfo[i];
    const long long off = ((long long)i << a.logN) + blockIdx.x * 256 + threadIdx.x;
    const int blk0 = blockIdx.z * BABY_CHUNK, blk1 = min(blk0 + BABY_CHUNK, a.nblk);
    if (p.q < (1ull << 46)) {
        const double qd = (double)p.q, qinv = 1.0 / qd;
        double w0[NB], w1[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const u64 *wp = b == 0 ? a.w + off : a.wr + (b - 1) * a.wrs + off;
            w0[b] = d_from_u52(wp[0]);
            w1[b] = d_from_u52(wp[b == 0 ? a.wc : a.wrc]);
        }
        for (int blk = blk0; blk < blk1; ++blk) {
            u64 z0[NB], z1[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const u64 *zp = b == 0 ? a.z + blk * a.zb + off : a.zr + blk * a.zrb + (b - 1) * a.zrs + off;
                z0[b] = __builtin_nontemporal_load(zp);  // streamed once per step: keep W's rows in cache
                z1[b] = __builtin_nontemporal_load(zp + (b == 0 ? a.zc : a.zrc));
            }
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const double x0 = d_from_u52(z0[b]), x1 = d_from_u52(z1[b]);
                d0 += mulmod_lazy_d(x0, w0[b], qd, qinv);
                d1 += mulmod_lazy_d(x0, w1[b], qd, qinv) + mulmod_lazy_d(x1, w0[b], qd, qinv);
                d2 += mulmod_lazy_d(x1, w1[b], qd, qinv);
            }
            u64 *o = a.o + blk * a.ob + off;
            o[0] = u52_from_d(reduce_d(d0, qd, qinv));
            o[a.oc] = u52_from_d(reduce_d(d1, qd, qinv));
            o[2 * a.oc] = u52_from_d(reduce_d(d2, qd, qinv));
        }
        return;
    }
    u64 w0[NB], w1[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const u64 *wp = b == 0 ? a.w + off : a.wr + (b - 1) * a.wrs + off;
        w0[b] = wp[0];
        w1[b] = wp[b == 0 ? a.wc : a.wrc];
    }
    for (int blk = blk0; blk < blk1; ++blk) {
        u64 d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const u64 *zp = b == 0 ? a.z + blk * a.zb + off : a.zr + blk * a.zrb + (b - 1) * a.zrs + off;
            const u64 x0 = zp[0], x1 = zp[b == 0 ? a.zc : a.zrc];
            d0 = add_mod(d0, mul_mod(x0, w0[b], p), p.q);
            d1 = add_mod(d1, add_mod(mul_mod(x0, w1[b], p), mul_mod(x1, w0[b], p), p.q), p.q);
            d2 = add_mod(d2, mul_mod(x1, w1[b], p), p.q);
        }
        u64 *o = a.o + blk * a.ob + off;
        o[0] = d0;
        o[a.oc] = d1;
        o[2 * a.oc] = d2;
    }
}

// ModUp conversion: ext[b][j][t] for positions t outside digit j.
// y[b][i] holds [d_i qhat_i^{-1}]_{q_i} (coefficient form).  A thread reads
// the digit's residues of two neighbouring coefficients once (16-byte loads)
// and writes every target.  Targets below 2^46 take the FP64 path (exact lazy
// products, one reduction); wider ones an exact 128-bit sum and one Barrett
// reduction.  Both give the canonical residue of the same integer.  A bounds
// the digit width at compile time (registers); nd <= A is the digit's width.
constexpr int MAX_ALPHA = 12;
template <int A>
__global__ __launch_bounds__(256) void modup_kernel(const u64 *__restrict__ y, long long ys, u64 *__restrict__ ext,
                                                    long long es, long long ds, const PrimeInfo *__restrict__ pinfo,
                                                    const u64 *__restrict__ conv, const u64 *__restrict__ qd,
                                                    const double *__restrict__ convd, const double *__restrict__ qdd,
                                                    const double *__restrict__ qinv_d, int level, int alpha, int nq,
                                                    int np, int nk, int beta, int logN)
{
    typedef __attribute__((ext_vector_type(2))) unsigned long long u64x2;
    const int z = blockIdx.y;
    const int b = z / beta, j = z % beta;
    const int d0 = j * alpha, d1 = min(d0 + alpha, level + 1);
    const int nd = d1 - d0;
    const int N = 1 << logN;
    const int x = 2 * (blockIdx.x * 256 + threadIdx.x);
    if (x >= N) return;
    const u64 *yb = y + b * ys;
    u64 v[A][2];
    u64 cnt[2] = {0, 0};
    int kmax = 0;
#pragma unroll
    for (int i = 0; i < A; ++i) {
        if (i < nd) {
            const PrimeInfo pi = pinfo[d0 + i];
            const u64x2 w = *reinterpret_cast<const u64x2 *>(yb + ((long long)(d0 + i) << logN) + x);
            v[i][0] = w.x;
            v[i][1] = w.y;
            cnt[0] += w.x > (pi.q >> 1);
            cnt[1] += w.y > (pi.q >> 1);
            kmax = max(kmax, (int)pi.k);
        }
    }
    // conv layout: [level][HE_MAXDIG][alpha][np][2]; qd: [level][HE_MAXDIG][np][2]
    const long long cbase = (((long long)level * HE_MAXDIG + j) * alpha) * np;
    const u64 *cv = conv + cbase * 2;
    const double *cvd = convd + cbase * 2;
    const u64 *qq = qd + (((long long)level * HE_MAXDIG + j) * np) * 2;
    const double *qqd = qdd + ((long long)level * HE_MAXDIG + j) * np;
    u64 *o = ext + b * es + j * ds + x;
    const int nb = level + 1 + nk;
    for (int t = 0; t < nb; ++t) {
        if (t >= d0 && t < d1) continue;
        const int tp = prime_of(t, level, nq);
        const PrimeInfo pt = pinfo[tp];
        const int kp = (int)pt.k;
        u64x2 r;
        if (conv_fp_ok(kmax, kp)) {
            const double pd = (double)pt.q, pinv = qinv_d[tp];
            const double kd = qqd[tp];
            double s0 = -(double)cnt[0] * kd, s1 = -(double)cnt[1] * kd;
#pragma unroll
            for (int i = 0; i < A; ++i) {
                if (i < nd) {
                    const double *e = cvd + ((long long)i * np + tp) * 2;
                    const int ki = (int)pinfo[d0 + i].k;
                    if (conv_whole(ki, kp)) {
                        s0 += mulmod_lazy_d(d_from_u52(v[i][0]), e[0], pd, pinv);
                        s1 += mulmod_lazy_d(d_from_u52(v[i][1]), e[0], pd, pinv);
                    } else {
                        const int S = conv_split_bits(ki);
                        const u64 m = (1ull << S) - 1;
                        s0 += mulmod_lazy_d((double)(u32)(v[i][0] >> S), e[1], pd, pinv) +
                              mulmod_lazy_d((double)(u32)(v[i][0] & m), e[0], pd, pinv);
                        s1 += mulmod_lazy_d((double)(u32)(v[i][1] >> S), e[1], pd, pinv) +
                              mulmod_lazy_d((double)(u32)(v[i][1] & m), e[0], pd, pinv);
                    }
                }
            }
            r.x = u52_from_d(reduce_d(s0, pd, pinv));
            r.y = u52_from_d(reduce_d(s1, pd, pinv));
        } else {
            // exact 128-bit sum of the products (each < 2^120), one reduction
            u64 lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
#pragma unroll
            for (int i = 0; i < A; ++i) {
                if (i < nd) {
                    const u64 ci = cv[((long long)i * np + tp) * 2];
                    u64 pl = v[i][0] * ci, ph = __umul64hi(v[i][0], ci);
                    lo0 += pl;
                    hi0 += ph + (lo0 < pl);
                    pl = v[i][1] * ci;
                    ph = __umul64hi(v[i][1], ci);
                    lo1 += pl;
                    hi1 += ph + (lo1 < pl);
                }
            }
            const u64 kq = qq[2 * tp], kqs = qq[2 * tp + 1];
            r.x = sub_mod(reduce128(hi0, lo0, pt), mul_shoup(cnt[0], kq, kqs, pt.q), pt.q);
            r.y = sub_mod(reduce128(hi1, lo1, pt), mul_shoup(cnt[1], kq, kqs, pt.q), pt.q);
        }
        *reinterpret_cast<u64x2 *>(o + ((long long)t << logN)) = r;
    }
}

// Key-switching inner product for B entries sharing one key: each thread keeps
// the key coefficients of two neighbouring positions in registers (16-byte
// accesses) and loops over the batch.
__global__ __launch_bounds__(256) void ks_inner_kernel(const u64 *__restrict__ d2, long long d2s,
                                                       const u64 *__restrict__ ext, long long es, long long ds,
                                                       const u64 *__restrict__ key, u64 *__restrict__ acc,
                                                       long long as, const PrimeInfo *__restrict__ pinfo, int B,
                                                       int level, int alpha, int nq, int np, int beta, int logN)
{
    typedef __attribute__((ext_vector_type(2))) unsigned long long u64x2;
    const int t = blockIdx.y;
    const int tp = prime_of(t, level, nq);
    const PrimeInfo p = pinfo[tp];
    const int N = 1 << logN;
    const int nb = level + 1 + (np - nq);
    const long long keylimb = (long long)np << logN;  // one key component
    const long long lt = (long long)t << logN;
    for (int x = 2 * (blockIdx.x * 256 + threadIdx.x); x < N; x += 2 * gridDim.x * 256) {
        u64x2 kb[HE_MAXBETA], ka[HE_MAXBETA];
        for (int j = 0; j < beta; ++j) {
            const u64 *kj = key + (long long)j * 2 * keylimb + ((long long)tp << logN) + x;
            kb[j] = *reinterpret_cast<const u64x2 *>(kj);
            ka[j] = *reinterpret_cast<const u64x2 *>(kj + keylimb);
        }
        for (int b = 0; b < B; ++b) {
            u64 s0a = 0, s1a = 0, s0b = 0, s1b = 0;
            for (int j = 0; j < beta; ++j) {
                const int d0 = j * alpha, d1 = min(d0 + alpha, level + 1);
                const u64 *src = (t >= d0 && t < d1) ? d2 + b * d2s + lt + x : ext + b * es + j * ds + lt + x;
                const u64x2 X = *reinterpret_cast<const u64x2 *>(src);
                s0a = add_mod(s0a, mul_mod(X.x, kb[j].x, p), p.q);
                s1a = add_mod(s1a, mul_mod(X.x, ka[j].x, p), p.q);
                s0b = add_mod(s0b, mul_mod(X.y, kb[j].y, p), p.q);
                s1b = add_mod(s1b, mul_mod(X.y, ka[j].y, p), p.q);
            }
            u64 *o = acc + b * as + lt + x;
            u64x2 r0, r1;
            r0.x = s0a;
            r0.y = s0b;
            r1.x = s1a;
            r1.y = s1b;
            *reinterpret_cast<u64x2 *>(o) = r0;
            *reinterpret_cast<u64x2 *>(o + ((long long)nb << logN)) = r1;
        }
    }
}

// Inner product with a different evaluation key per entry (rotations by
// different steps in one launch): entry b = blockIdx.z uses keys.k[b]; the key
// is read once per entry (no reuse across entries to keep in registers).
__global__ __launch_bounds__(256) void ks_inner_multi_kernel(const u64 *__restrict__ d2, long long d2s,
                                                             const u64 *__restrict__ ext, long long es, long long ds,
                                                             hek::EntryKeys keys, u64 *__restrict__ acc, long long as,
                                                             const PrimeInfo *__restrict__ pinfo, int level,
                                                             int alpha, int nq, int np, int beta, int logN)
{
    typedef __attribute__((ext_vector_type(2))) unsigned long long u64x2;
    const int t = blockIdx.y;
    const int b = blockIdx.z;
    const int tp = prime_of(t, level, nq);
    const PrimeInfo p = pinfo[tp];
    const int N = 1 << logN;
    const int nb = level + 1 + (np - nq);
    const long long keylimb = (long long)np << logN;
    const long long lt = (long long)t << logN;
    const u64 *key = keys.k[b];
    for (int x = 2 * (blockIdx.x * 256 + threadIdx.x); x < N; x += 2 * gridDim.x * 256) {
        u64 s0a = 0, s1a = 0, s0b = 0, s1b = 0;
        for (int j = 0; j < beta; ++j) {
            const u64 *kj = key + (long long)j * 2 * keylimb + ((long long)tp << logN) + x;
            const u64x2 kb = *reinterpret_cast<const u64x2 *>(kj);
            const u64x2 ka = *reinterpret_cast<const u64x2 *>(kj + keylimb);
            const int d0 = j * alpha, d1 = min(d0 + alpha, level + 1);
            const u64 *src = (t >= d0 && t < d1) ? d2 + b * d2s + lt + x : ext + b * es + j * ds + lt + x;
            const u64x2 X = *reinterpret_cast<const u64x2 *>(src);
            s0a = add_mod(s0a, mul_mod(X.x, kb.x, p), p.q);
            s1a = add_mod(s1a, mul_mod(X.x, ka.x, p), p.q);
            s0b = add_mod(s0b, mul_mod(X.y, kb.y, p), p.q);
            s1b = add_mod(s1b, mul_mod(X.y, ka.y, p), p.q);
        }
        u64 *o = acc + b * as + lt + x;
        u64x2 r0, r1;
        r0.x = s0a;
        r0.y = s0b;
        r1.x = s1a;
        r1.y = s1b;
        *reinterpret_cast<u64x2 *>(o) = r0;
        *reinterpret_cast<u64x2 *>(o + ((long long)nb << logN)) = r1;
    }
}

// ModDown conversion: acc[b][comp] positions level+1.. hold scaled iNTT
// outputs y_p (coefficient); conv[b][comp][i] = sum_p y~_p (phat_p mod q_i).
// A thread reads the k special residues of one coefficient once.
__global__ __launch_bounds__(256) void moddown_conv_kernel(const u64 *__restrict__ acc, long long as,
                                                           u64 *__restrict__ conv, long long cs,
                                                           const PrimeInfo *__restrict__ pinfo,
                                                           const u64 *__restrict__ dconv, const u64 *__restrict__ dp,
                                                           int level, int nq, int nk, int logN)
{
    const int z = blockIdx.y;  // b*2 + comp
    const int b = z >> 1, comp = z & 1;
    const int N = 1 << logN;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= N) return;
    const int nb = level + 1 + nk;
    const u64 *src = acc + b * as + ((long long)comp * nb << logN) + x;
    u64 *o = conv + b * cs + ((long long)comp * (level + 1) << logN) + x;
    u64 v[MAX_ALPHA];
    u64 cnt = 0;
    for (int k = 0; k < nk; ++k) {
        v[k] = src[(long long)(level + 1 + k) << logN];
        cnt += v[k] > (pinfo[nq + k].q >> 1);
    }
    for (int i = 0; i <= level; ++i) {
        const u64 q = pinfo[i].q;
        u64 s = 0;
        for (int k = 0; k < nk; ++k) {
            const u64 *c2 = dconv + ((long long)k * nq + i) * 2;
            s += mul_shoup(v[k], c2[0], c2[1], q);
        }
        s = reduce_small(s, q, nk);
        o[(long long)i << logN] = sub_mod(s, mul_shoup(cnt, dp[2 * i], dp[2 * i + 1], q), q);
    }
}

// out[b][comp][i] = base + (acc - conv) P^{-1}   (NTT domain)
__global__ __launch_bounds__(256) void moddown_finish_kernel(const u64 *__restrict__ acc, long long as,
                                                             const u64 *__restrict__ conv, long long cs,
                                                             const u64 *__restrict__ base, long long bs,
                                                             long long bcs, int nbase, u64 *out, long long os,
                                                             long long ocs, const u64 *add, long long ads,
                                                             long long adcs, const PrimeInfo *__restrict__ pinfo,
                                                             const u64 *__restrict__ pinv, int level, int nk,
                                                             int logN)
{
    const int i = blockIdx.y;
    const int z = blockIdx.z;
    const int b = z >> 1, comp = z & 1;
    const int N = 1 << logN;
    const int nb = level + 1 + nk;
    const u64 q = pinfo[i].q;
    const u64 w = pinv[2 * i], ws = pinv[2 * i + 1];
    const long long li = (long long)i << logN;
    const u64 *a = acc + b * as + ((long long)comp * nb << logN) + li;
    const u64 *c = conv + b * cs + ((long long)comp * (level + 1) << logN) + li;
    const u64 *bb = (comp < nbase) ? base + b * bs + comp * bcs + li : nullptr;
    u64 *o = out + b * os + comp * ocs + li;
    const u64 *ad = add ? add + b * ads + comp * adcs + li : nullptr;  // may be o itself: read before the write
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256) {
        u64 v = mul_shoup(sub_mod(a[x], c[x], q), w, ws, q);
        if (bb) v = add_mod(v, bb[x], q);
        if (ad) v = add_mod(v, ad[x], q);
        o[x] = v;
    }
}

// tmp[b][c][i] = [last]_centered mod q_i  (coefficient) for i < level
__global__ __launch_bounds__(256) void rescale_bcast_kernel(const u64 *__restrict__ lastc, u64 *__restrict__ tmp,
                                                            const PrimeInfo *__restrict__ pinfo,
                                                            const u64 *__restrict__ rs_ql, int level, int nq,
                                                            int logN)
{
    const int i = blockIdx.y;
    const int z = blockIdx.z;  // b*2+c
    const int N = 1 << logN;
    const PrimeInfo p = pinfo[i];
    const u64 ql = pinfo[level].q;
    const u64 qlmod = rs_ql[(long long)level * nq + i];
    const u64 *src = lastc + ((long long)z << logN);
    u64 *o = tmp + ((long long)(z * level + i) << logN);
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256) {
        u64 v = src[x];
        u64 r = reduce64(v, p);
        if (v > (ql >> 1)) r = sub_mod(r, qlmod, p.q);
        o[x] = r;
    }
}

// out[b][c][i] = (in[b][c][i] - tmp[b][c][i]) q_l^{-1}; one thread walks the
// limbs of one coefficient in order, so out may alias in (it trails by N).
__global__ __launch_bounds__(256) void rescale_finish_kernel(const u64 *in, long long is, const u64 *__restrict__ tmp,
                                                             u64 *out, long long os,
                                                             const PrimeInfo *__restrict__ pinfo,
                                                             const u64 *__restrict__ rs_qinv, int level, int nq,
                                                             int logN, int ncomp)
{
    const int b = blockIdx.y;
    const int N = 1 << logN;
    const u64 *qi_tab = rs_qinv + (long long)level * nq * 2;
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256) {
        for (int c = 0; c < ncomp; ++c) {
            const u64 *src = in + b * is + ((long long)c * (level + 1) << logN);
            const u64 *tp = tmp + ((long long)(b * ncomp + c) * level << logN);
            u64 *dst = out + b * os + ((long long)c * level << logN);
            for (int i = 0; i < level; ++i) {
                const u64 q = pinfo[i].q;
                long long off = ((long long)i << logN) + x;
                u64 v = sub_mod(src[off], tp[off], q);
                dst[off] = mul_shoup(v, qi_tab[2 * i], qi_tab[2 * i + 1], q);
            }
        }
    }
}

// NTT-order automorphism: output index k holds the value at the root
// psi^(2 br(k) + 1); sigma_g(a) there equals a at psi^((2 br(k)+1) g).
__global__ __launch_bounds__(256) void automorph_kernel(const u64 *__restrict__ in, long long ib, long long ic,
                                                        u64 *__restrict__ out, long long ob, long long oc, u64 g,
                                                        int logN)
{
    const int limb = blockIdx.y;
    const int b = blockIdx.z >> 1, c = blockIdx.z & 1;
    const int N = 1 << logN;
    const u64 mask2n = 2 * (u64)N - 1;
    const u64 *src = in + b * ib + c * ic + ((long long)limb << logN);
    u64 *dst = out + b * ob + c * oc + ((long long)limb << logN);
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
        u64 e = 2 * (u64)brev_n(k, logN) + 1;
        u64 e2 = (e * g) & mask2n;
        unsigned k2 = brev_n((unsigned)((e2 - 1) >> 1), logN);
        dst[k] = src[k2];
    }
}

// Hoisted sum of rotations, the inner-product step: for every entry b,
// position t of Q_l u P and coefficient k (NTT order),
//   acc[b][comp][t][k] = sum_{g < ng} sum_{j < beta} D_j[t][s_g(k)] key_g[j][comp][t][k]
// where D_j is digit j's ModUp in NTT form (ext, or the input's own a-part on
// the digit's positions) and s_g the index map of the automorphism X -> X^g
// (sigma_g(a) at k = a at s_g(k); the automorphism commutes with ModUp).  For
// t <= l it also writes out[b][0][t][k] = x0[k] + sum_g x0[s_g(k)] and
// out[b][1][t][k] = x1[k], the base of the one ModDown that follows.  When the
// Galois elements form a group of order ng + 1 <= 16 whose elements are 1 mod
// 2^m, s_g(k) stays inside k's aligned run of 2N / 2^m coefficients: the
// gathers stay within a few cache lines.  Each thread serves up to GIANT_EPT
// entries, so each key value is loaded once for all of them; the entry groups
// of one (t, k-tile) are dealt to one XCD, so the keys are fetched into one L2.
constexpr int GIANT_EPT = 4;
struct GiantArgs {
    const u64 *ext;  // [b][beta][nb][N]
    long long es, ds;
    const u64 *x;  // input [b][2][l+1][N]: batch stride xs, component stride xc
    long long xs, xc;
    hek::EntryKeys keys;  // key_g [beta][2][np][N]
    hek::EntryGal gals;
    int ng, gc;  // rotations; rotations per staged key chunk (tile kernel)
    u64 *acc;  // [b][2][nb][N]
    long long as;
    u64 *out;  // [b][2][l+1][N]: batch stride os, component stride xc
    long long os;
    int alpha, beta, ell, nq, np, nb, nent, ngroups, logN;
};

__device__ __forceinline__ long long giant_index(u64 e, u64 g, u64 mask2n, int logN)
{
    // only the low logN + 1 bits of e g are used: a 32-bit product suffices
    const unsigned e2 = ((unsigned)e * (unsigned)g) & (unsigned)mask2n;
    return brev_n((e2 - 1) >> 1, logN);
}

__global__ __launch_bounds__(256) void giant_gather_kernel(GiantArgs a, const PrimeInfo *__restrict__ pinfo)
{
    const int ntile = (1 << a.logN) / 256;
    const int npair = ntile * a.nb;
    const int w = blockIdx.x;
    int grp, pr;
    if ((npair & 7) == 0) {
        const int sidx = w >> 3;
        grp = sidx % a.ngroups;
        pr = (sidx / a.ngroups) * 8 + (w & 7);
    } else {
        grp = w % a.ngroups;
        pr = w / a.ngroups;
    }
    const int t = pr / ntile;
    const int k = (pr % ntile) * 256 + threadIdx.x;
    const int b0 = grp * GIANT_EPT;
    const int ne = min(GIANT_EPT, a.nent - b0);
    const int tp = prime_of(t, a.ell, a.nq);
    const PrimeInfo p = pinfo[tp];
    const long long N = 1ll << a.logN;
    const u64 mask2n = 2 * (u64)N - 1;
    const u64 e = 2 * (u64)brev_n((unsigned)k, a.logN) + 1;
    const long long keylimb = ((long long)tp << a.logN) + k;
    const long long np_n = (long long)a.np << a.logN;
    const long long toff = (long long)t << a.logN;
    // the digit holding position t (inside Q_l), whose D_j[t] is the input's a-part
    const int jt = t <= a.ell ? t / a.alpha : -1;
    if (p.q < (1ull << 46)) {
        const double qd = (double)p.q, qinv = 1.0 / qd;
        double s0[GIANT_EPT], s1[GIANT_EPT];
#pragma unroll
        for (int i = 0; i < GIANT_EPT; ++i) s0[i] = s1[i] = 0.0;
        for (int g = 0; g < a.ng; ++g) {
            const u64 e2 = (e * a.gals.g[g]) & mask2n;
            const long long k2 = brev_n((unsigned)((e2 - 1) >> 1), a.logN);
            const u64 *key = a.keys.k[g] + keylimb;
            double p0[GIANT_EPT], p1[GIANT_EPT];
#pragma unroll
            for (int i = 0; i < GIANT_EPT; ++i) p0[i] = p1[i] = 0.0;
            for (int j = 0; j < a.beta; ++j) {
                const double k0 = d_from_u52(key[(2 * j) * np_n]), k1 = d_from_u52(key[(2 * j + 1) * np_n]);
#pragma unroll
                for (int i = 0; i < GIANT_EPT; ++i) {
                    if (i < ne) {
                        const int b = b0 + i;
                        const u64 v = j == jt ? a.x[b * a.xs + a.xc + toff + k2]
                                              : a.ext[b * a.es + j * a.ds + toff + k2];
                        const double dv = d_from_u52(v);
                        p0[i] += mulmod_lazy_d(dv, k0, qd, qinv);
                        p1[i] += mulmod_lazy_d(dv, k1, qd, qinv);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < GIANT_EPT; ++i) {
                s0[i] = reduce_d(s0[i] + p0[i], qd, qinv);
                s1[i] = reduce_d(s1[i] + p1[i], qd, qinv);
            }
        }
#pragma unroll
        for (int i = 0; i < GIANT_EPT; ++i) {
            if (i < ne) {
                u64 *o = a.acc + (b0 + i) * a.as + toff + k;
                o[0] = u52_from_d(s0[i]);
                o[(long long)a.nb << a.logN] = u52_from_d(s1[i]);
            }
        }
    } else {
        u64 s0[GIANT_EPT], s1[GIANT_EPT];
#pragma unroll
        for (int i = 0; i < GIANT_EPT; ++i) s0[i] = s1[i] = 0;
        for (int g = 0; g < a.ng; ++g) {
            const u64 e2 = (e * a.gals.g[g]) & mask2n;
            const long long k2 = brev_n((unsigned)((e2 - 1) >> 1), a.logN);
            const u64 *key = a.keys.k[g] + keylimb;
            for (int j = 0; j < a.beta; ++j) {
                const u64 k0 = key[(2 * j) * np_n], k1 = key[(2 * j + 1) * np_n];
#pragma unroll
                for (int i = 0; i < GIANT_EPT; ++i) {
                    if (i < ne) {
                        const int b = b0 + i;
                        const u64 v = j == jt ? a.x[b * a.xs + a.xc + toff + k2]
                                              : a.ext[b * a.es + j * a.ds + toff + k2];
                        s0[i] = add_mod(s0[i], mul_mod(v, k0, p), p.q);
                        s1[i] = add_mod(s1[i], mul_mod(v, k1, p), p.q);
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < GIANT_EPT; ++i) {
            if (i < ne) {
                u64 *o = a.acc + (b0 + i) * a.as + toff + k;
                o[0] = s0[i];
                o[(long long)a.nb << a.logN] = s1[i];
            }
        }
    }
    if (t > a.ell) return;
    // the base: b-parts automorphed and summed, the a-part copied
    for (int i = 0; i < ne; ++i) {
        const int b = b0 + i;
        const u64 *x0 = a.x + b * a.xs + toff;
        u64 v = x0[k];
        for (int g = 0; g < a.ng; ++g) {
            const u64 e2 = (e * a.gals.g[g]) & mask2n;
            v = add_mod(v, x0[brev_n((unsigned)((e2 - 1) >> 1), a.logN)], p.q);
        }
        u64 *o = a.out + b * a.os + toff + k;
        o[0] = v;
        o[a.xc] = x0[a.xc + k];
    }
}

// The same sum when every s_g keeps k inside its aligned tile of 64
// coefficients (g = 1 mod 2^(logN - 5)): the 64 lanes of a wave hold one tile,
// each lane loads its own coefficient of every digit once (coalesced).  A
// workgroup takes one position t and one tile for the entries (wave w serves
// entries w, w + 4, ..); the tile's keys are staged in LDS a chunk of rotations
// at a time and read there by every entry.  FP (positions whose prime is below
// 2^46): key_g[j][k] is staged at lane m = s_g(k), so lane m forms
// sum_j D_j[m] key_g[j][k] from its own digits and lane k pulls that partial
// sum (ds_bpermute, two 32-bit halves); lazy FP64 products, the running sum
// reduced every 48 / beta rotations.  Otherwise lane k pulls every
// D_j[s_g(k)] and keeps exact 128-bit sums reduced once per chunk (at most 40
// products below 2^120 each), for two entries per pass.
constexpr int GP_TK = 64, GP_LANES = 4, GP_MAXB = 8;
constexpr int GP_LDS = 40 * 1024;  // bytes of staged keys per workgroup

__device__ __forceinline__ u64 lane_take(u64 v, int src)
{
    const int addr = src << 2;
    const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(v >> 32));
    return ((u64)hi << 32) | lo;
}

template <bool FP, int BETA>
__global__ __launch_bounds__(GP_TK *GP_LANES) void giant_perm_kernel(GiantArgs a, const PrimeInfo *__restrict__ pinfo)
{
    extern __shared__ u64 keys_lds[];
    const int ntile = (1 << a.logN) / GP_TK;
    const int t = blockIdx.x / ntile;
    const int L = threadIdx.x % GP_TK, lane = threadIdx.x / GP_TK;
    const int k = (blockIdx.x % ntile) * GP_TK + L;
    const int tp = prime_of(t, a.ell, a.nq);
    const PrimeInfo p = pinfo[tp];
    if ((p.q < (1ull << 46)) != FP) return;  // the other instantiation's position (uniform per workgroup)
    const long long N = 1ll << a.logN;
    const u64 mask2n = 2 * (u64)N - 1;
    const u64 e = 2 * (u64)brev_n((unsigned)k, a.logN) + 1;
    const long long toff = (long long)t << a.logN;
    const long long np_n = (long long)a.np << a.logN;
    const long long comp1 = (long long)a.nb << a.logN;
    const int jt = t <= a.ell ? t / a.alpha : -1;
    const double qd = (double)p.q, qinv = 1.0 / qd;
    constexpr int per = BETA * 2 * GP_TK;  // staged values per rotation
    for (int g0 = 0; g0 < a.ng; g0 += a.gc) {
        const int gn = min(a.gc, a.ng - g0);
        __syncthreads();
        for (int v = threadIdx.x; v < gn * per; v += blockDim.x) {
            const int gi = v / per, r = v % per, jc = r / GP_TK, kk = r % GP_TK;
            const u64 kv = a.keys.k[g0 + gi][jc * np_n + ((long long)tp << a.logN) + (k - L) + kk];
            if (FP) {  // stored at the lane whose digits coefficient kk takes
                const u64 ek = 2 * (u64)brev_n((unsigned)((k - L) + kk), a.logN) + 1;
                const int m = (int)(giant_index(ek, a.gals.g[g0 + gi], mask2n, a.logN) & (GP_TK - 1));
                keys_lds[v - kk + m] = (u64)__double_as_longlong(d_from_u52(kv));
            } else {
                keys_lds[v] = kv;
            }
        }
        __syncthreads();
        // 60-bit positions: two entries per pass (b and b + GP_LANES, uniform
        // per wave), sharing the staged keys' reads and the source lane (the
        // FP64 positions measured slower that way)
        constexpr int GP_EP = FP ? 1 : 2;
        for (int b = lane; b < a.nent; b += GP_EP * GP_LANES) {
            const int ne = GP_EP == 2 && b + GP_LANES < a.nent ? 2 : 1;
            u64 d[GP_EP][BETA];
#pragma unroll
            for (int i = 0; i < GP_EP; ++i) {
                const int bi = b + i * GP_LANES;
#pragma unroll
                for (int j = 0; j < BETA; ++j) {
                    u64 x = 0;
                    if (i < ne) x = j == jt ? a.x[bi * a.xs + a.xc + toff + k] : a.ext[bi * a.es + j * a.ds + toff + k];
                    d[i][j] = FP ? (u64)__double_as_longlong(d_from_u52(x)) : x;
                }
            }
            double s0[GP_EP], s1[GP_EP];
            u64 lo0[GP_EP], hi0[GP_EP], lo1[GP_EP], hi1[GP_EP];
#pragma unroll
            for (int i = 0; i < GP_EP; ++i) {
                s0[i] = s1[i] = 0.0;
                lo0[i] = hi0[i] = lo1[i] = hi1[i] = 0;
                if (g0 > 0 && i < ne) {  // the running sums of the earlier chunks
                    const u64 *o = a.acc + (b + i * GP_LANES) * a.as + toff + k;
                    if (FP) {
                        s0[i] = d_from_u52(o[0]);
                        s1[i] = d_from_u52(o[comp1]);
                    } else {
                        lo0[i] = o[0];
                        lo1[i] = o[comp1];
                    }
                }
            }
            constexpr int GP_RED = 48 / BETA;
            int nred = 0;
            for (int gi = 0; gi < gn; ++gi) {
                const int src = (int)(giant_index(e, a.gals.g[g0 + gi], mask2n, a.logN) & (GP_TK - 1));
                const u64 *kl = keys_lds + gi * per + L;
                if constexpr (FP) {
                    // this lane's own digits times the keys staged at it: the
                    // rotation's partial sum for the lane that takes these
                    // digits, which pulls it (2 pulls per component instead of
                    // 2 per digit); every sum is an exact integer below 2^52
                    double p0[GP_EP], p1[GP_EP];
#pragma unroll
                    for (int i = 0; i < GP_EP; ++i) p0[i] = p1[i] = 0.0;
#pragma unroll
                    for (int j = 0; j < BETA; ++j) {
                        const double k0 = __longlong_as_double((long long)kl[(2 * j) * GP_TK]);
                        const double k1 = __longlong_as_double((long long)kl[(2 * j + 1) * GP_TK]);
#pragma unroll
                        for (int i = 0; i < GP_EP; ++i) {
                            const double dv = __longlong_as_double((long long)d[i][j]);
                            p0[i] += mulmod_lazy_d(dv, k0, qd, qinv);
                            p1[i] += mulmod_lazy_d(dv, k1, qd, qinv);
                        }
                    }
#pragma unroll
                    for (int i = 0; i < GP_EP; ++i) {
                        s0[i] += __longlong_as_double((long long)lane_take((u64)__double_as_longlong(p0[i]), src));
                        s1[i] += __longlong_as_double((long long)lane_take((u64)__double_as_longlong(p1[i]), src));
                    }
                    // back into (-q, 2q) every GP_RED rotations: from there the
                    // sum takes at most 48 lazy products, each below 2q + 2^39
                    // < 2^47.1 in magnitude (q < 2^46: the product's low part is
                    // at most half an ulp of a value below 2^92), and stays an
                    // exact integer below 2^52.6
                    if (++nred == GP_RED) {
                        nred = 0;
#pragma unroll
                        for (int i = 0; i < GP_EP; ++i) {
                            s0[i] = __fma_rn(-floor(s0[i] * qinv), qd, s0[i]);
                            s1[i] = __fma_rn(-floor(s1[i] * qinv), qd, s1[i]);
                        }
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < BETA; ++j) {
                        const u64 k0 = kl[(2 * j) * GP_TK], k1 = kl[(2 * j + 1) * GP_TK];
#pragma unroll
                        for (int i = 0; i < GP_EP; ++i) {
                            const u64 v = lane_take(d[i][j], src);
                            u64 pl = v * k0, ph = __umul64hi(v, k0);
                            lo0[i] += pl;
                            hi0[i] += ph + (lo0[i] < pl);
                            pl = v * k1;
                            ph = __umul64hi(v, k1);
                            lo1[i] += pl;
                            hi1[i] += ph + (lo1[i] < pl);
                        }
                    }
                }
            }
            // FP: one full reduction; 128-bit sums of at most 40 products below 2^120 per chunk: reduced once
#pragma unroll
            for (int i = 0; i < GP_EP; ++i) {
                if (i < ne) {
                    u64 *o = a.acc + (b + i * GP_LANES) * a.as + toff + k;
                    o[0] = FP ? u52_from_d(reduce_d(s0[i], qd, qinv)) : reduce128(hi0[i], lo0[i], p);
                    o[comp1] = FP ? u52_from_d(reduce_d(s1[i], qd, qinv)) : reduce128(hi1[i], lo1[i], p);
                }
            }
        }
    }
    if (t > a.ell) return;
    // the base: b-parts automorphed and summed, the a-part copied
    for (int b = lane; b < a.nent; b += GP_LANES) {
        const u64 *x0 = a.x + b * a.xs + toff;
        const u64 own = x0[k];
        u64 v = own;
        for (int g = 0; g < a.ng; ++g)
            v = add_mod(v, lane_take(own, (int)(giant_index(e, a.gals.g[g], mask2n, a.logN) & (GP_TK - 1))), p.q);
        u64 *o = a.out + b * a.os + toff + k;
        o[0] = v;
        o[a.xc] = x0[a.xc + k];
    }
}

// Rotations of one ciphertext sharing its ModUp, the inner-product step: for
// rotation g < n, position t of Q_l u P and coefficient k (NTT order),
//   acc[g][comp][t][k] = sum_{j < beta} D_j[t][s_g(k)] key_g[j][comp][t][k]
// with D_j and s_g as in the hoisted sum above (the digits of the one input
// raised once; the automorphism commutes with ModUp), each rotation kept
// apart for its own ModDown.  One thread per (g, t, k); the gathers are
// global (the steps need not form a group).
__global__ __launch_bounds__(256) void rot_inner_kernel(GiantArgs a, const PrimeInfo *__restrict__ pinfo)
{
    const int ntile = (1 << a.logN) / 256;
    const int w = blockIdx.x;
    const int g = w / (ntile * a.nb), r = w % (ntile * a.nb);
    const int t = r / ntile;
    const int k = (r % ntile) * 256 + threadIdx.x;
    const int tp = prime_of(t, a.ell, a.nq);
    const PrimeInfo p = pinfo[tp];
    const long long N = 1ll << a.logN;
    const u64 mask2n = 2 * (u64)N - 1;
    const u64 e = 2 * (u64)brev_n((unsigned)k, a.logN) + 1;
    const long long k2 = giant_index(e, a.gals.g[g], mask2n, a.logN);
    const long long toff = (long long)t << a.logN;
    const long long np_n = (long long)a.np << a.logN;
    const int jt = t <= a.ell ? t / a.alpha : -1;
    const u64 *key = a.keys.k[g] + ((long long)tp << a.logN) + k;
    u64 *o = a.acc + g * a.as + toff + k;
    if (p.q < (1ull << 46)) {
        const double qd = (double)p.q, qinv = 1.0 / qd;
        double s0 = 0.0, s1 = 0.0;
        for (int j = 0; j < a.beta; ++j) {
            const u64 v = j == jt ? a.x[a.xc + toff + k2] : a.ext[j * a.ds + toff + k2];
            const double dv = d_from_u52(v);
            s0 += mulmod_lazy_d(dv, d_from_u52(key[(2 * j) * np_n]), qd, qinv);
            s1 += mulmod_lazy_d(dv, d_from_u52(key[(2 * j + 1) * np_n]), qd, qinv);
        }
        o[0] = u52_from_d(reduce_d(s0, qd, qinv));
        o[(long long)a.nb << a.logN] = u52_from_d(reduce_d(s1, qd, qinv));
    } else {
        u64 lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
        for (int j = 0; j < a.beta; ++j) {
            const u64 v = j == jt ? a.x[a.xc + toff + k2] : a.ext[j * a.ds + toff + k2];
            const u64 k0 = key[(2 * j) * np_n], k1 = key[(2 * j + 1) * np_n];
            u64 pl = v * k0, ph = __umul64hi(v, k0);
            lo0 += pl;
            hi0 += ph + (lo0 < pl);
            pl = v * k1;
            ph = __umul64hi(v, k1);
            lo1 += pl;
            hi1 += ph + (lo1 < pl);
        }
        o[0] = reduce128(hi0, lo0, p);
        o[(long long)a.nb << a.logN] = reduce128(hi1, lo1, p);
    }
}

// The limb at q_l of a ModDown's output, in coefficient form, for the rescale
// by q_l that follows: last = base + (acc - conv) P^{-1} mod q_l from the
// coefficient forms of base's and acc's limbs l (bl, al: [b][comp][N]) and the
// special limbs of acc (coefficient form, scaled as the ModDown reads them),
// conv their centred conversion to q_l -- the same integers as the inverse
// transform of the ModDown output's limb l.
__global__ __launch_bounds__(256) void md_last_kernel(const u64 *__restrict__ bl, const u64 *__restrict__ al,
                                                      const u64 *__restrict__ acc, long long as, long long acs,
                                                      u64 *__restrict__ last, const PrimeInfo *__restrict__ pinfo,
                                                      const u64 *__restrict__ dn_conv, const u64 *__restrict__ dn_p,
                                                      const u64 *__restrict__ dn_pinv, int level, int nq, int nk,
                                                      int logN)
{
    const int bc = blockIdx.y;
    const int b = bc >> 1, c = bc & 1;
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    const PrimeInfo p = pinfo[level];
    const u64 *src = acc + b * as + c * acs + ((long long)(level + 1) << logN) + k;
    u64 lo = 0, hi = 0, cnt = 0;
    for (int i = 0; i < nk; ++i) {
        const u64 v = src[(long long)i << logN];
        cnt += v > (pinfo[nq + i].q >> 1);
        const u64 ci = dn_conv[((long long)i * nq + level) * 2];
        const u64 pl = v * ci, ph = __umul64hi(v, ci);
        lo += pl;
        hi += ph + (lo < pl);
    }
    const u64 conv = sub_mod(reduce128(hi, lo, p), mul_shoup(cnt, dn_p[2 * level], dn_p[2 * level + 1], p.q), p.q);
    const long long o = ((long long)bc << logN) + k;
    last[o] = add_mod(bl[o], mul_shoup(sub_mod(al[o], conv, p.q), dn_pinv[2 * level], dn_pinv[2 * level + 1], p.q),
                      p.q);
}

// automorph_kernel with a Galois element per entry b (blockIdx.z = 2 b + c)
__global__ __launch_bounds__(256) void automorph_multi_kernel(const u64 *__restrict__ in, long long ib, long long ic,
                                                              u64 *__restrict__ out, long long ob, long long oc,
                                                              hek::EntryGal gals, int logN)
{
    const int limb = blockIdx.y;
    const int b = blockIdx.z >> 1, c = blockIdx.z & 1;
    const int N = 1 << logN;
    const u64 mask2n = 2 * (u64)N - 1;
    const u64 g = gals.g[b];
    const u64 *src = in + b * ib + c * ic + ((long long)limb << logN);
    u64 *dst = out + b * ob + c * oc + ((long long)limb << logN);
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
        u64 e = 2 * (u64)brev_n(k, logN) + 1;
        u64 e2 = (e * g) & mask2n;
        unsigned k2 = brev_n((unsigned)((e2 - 1) >> 1), logN);
        dst[k] = src[k2];
    }
}

// out[c][i] = sum_b in[b][c][i]  (mod q_i), positions 0..level
__global__ __launch_bounds__(256) void batch_sum_kernel(const u64 *__restrict__ in, long long ib, long long ic,
                                                        int B, u64 *__restrict__ out, long long oc, int accumulate,
                                                        const PrimeInfo *__restrict__ pinfo, int logN)
{
    const int i = blockIdx.y, c = blockIdx.z;
    const int N = 1 << logN;
    const u64 q = pinfo[i].q;
    const long long li = (long long)i << logN;
    u64 *o = out + c * oc + li;
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256) {
        u64 s = accumulate ? o[x] : 0;
        for (int b = 0; b < B; ++b) s = add_mod(s, in[b * ib + c * ic + li + x], q);
        o[x] = s;
    }
}

// ------------------------------------------------------------------ ChaCha20 (RFC 8439, Sec. 2.3)
__device__ __forceinline__ uint32_t rotl32(uint32_t v, int n) { return (v << n) | (v >> (32 - n)); }

__device__ void chacha_block(uint32_t seed_lo, uint32_t seed_hi, uint32_t counter, uint32_t n0, uint32_t n1,
                             uint32_t n2, uint32_t out[16])
{
    uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, seed_lo, seed_hi, 0, 0,
                      0,           0,           0,           0,           counter, n0,      n1, n2};
    uint32_t x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = s[i];
#define QR(a, b, c, d)                                   \
    x[a] += x[b]; x[d] = rotl32(x[d] ^ x[a], 16);        \
    x[c] += x[d]; x[b] = rotl32(x[b] ^ x[c], 12);        \
    x[a] += x[b]; x[d] = rotl32(x[d] ^ x[a], 8);         \
    x[c] += x[d]; x[b] = rotl32(x[b] ^ x[c], 7);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        QR(0, 4, 8, 12) QR(1, 5, 9, 13) QR(2, 6, 10, 14) QR(3, 7, 11, 15)
        QR(0, 5, 10, 15) QR(1, 6, 11, 12) QR(2, 7, 8, 13) QR(3, 4, 9, 14)
    }
#undef QR
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

struct PosPrimes {
    int n;
    int prime[HE_MAXP];
};

// uniform residues: coefficient x of position pos uses words 2x (high) and
// 2x+1 (low) of stream (seed; type, index, comp_base + pos).
__global__ __launch_bounds__(256) void uniform_kernel(u64 seed, uint32_t type, uint32_t index, uint32_t comp_base,
                                                      PosPrimes pp, const PrimeInfo *__restrict__ pinfo,
                                                      u64 *__restrict__ out, int logN)
{
    const int pos = blockIdx.y;
    const int N = 1 << logN;
    const PrimeInfo p = pinfo[pp.prime[pos]];
    u64 *o = out + ((long long)pos << logN);
    const int nblk = N / 4;  // 4 coefficients per ChaCha block
    for (int blk = blockIdx.x * 256 + threadIdx.x; blk < nblk; blk += gridDim.x * 256) {
        uint32_t w[16];
        chacha_block((uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)blk, type, index, comp_base + pos, w);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            u64 hi = w[4 * c] | ((u64)w[4 * c + 1] << 32);
            u64 lo = w[4 * c + 2] | ((u64)w[4 * c + 3] << 32);
            o[4 * blk + c] = reduce128(hi, lo, p);
        }
    }
}

// centered binomial (21 pairs) from word x; residues on every position
__global__ __launch_bounds__(256) void cbd_kernel(u64 seed, uint32_t type, uint32_t index, uint32_t comp, PosPrimes pp,
                                                  const PrimeInfo *__restrict__ pinfo, u64 *__restrict__ out,
                                                  int logN)
{
    const int N = 1 << logN;
    const int nblk = N / 8;
    for (int blk = blockIdx.x * 256 + threadIdx.x; blk < nblk; blk += gridDim.x * 256) {
        uint32_t w[16];
        chacha_block((uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)blk, type, index, comp, w);
        for (int c = 0; c < 8; ++c) {
            u64 v = w[2 * c] | ((u64)w[2 * c + 1] << 32);
            int e = __popcll(v & 0x1FFFFFull) - __popcll((v >> 21) & 0x1FFFFFull);
            for (int pos = 0; pos < pp.n; ++pos) {
                u64 q = pinfo[pp.prime[pos]].q;
                out[((long long)pos << logN) + 8 * blk + c] = e >= 0 ? (u64)e : q - (u64)(-e);
            }
        }
    }
}

// Uniform part of seeded ciphertexts in the evaluation domain.  Thread j0 <
// N/4 computes ChaCha20 block b = bitrev_{logN-2}(j0), i.e. the coefficients
// k = 4b + u (u < 4) of the stream, whose NTT positions bitrev_logN(k) =
// bitrev_2(u) N/4 + j0 are four coalesced streams across the threads.
__global__ __launch_bounds__(256) void seeded_a_kernel(u64 seed, uint32_t index0, const PrimeInfo *__restrict__ pinfo,
                                                       u64 *__restrict__ out, long long os, int logN)
{
    const int i = blockIdx.y, e = blockIdx.z;
    const int Q = 1 << (logN - 2);
    const PrimeInfo p = pinfo[i];
    u64 *o = out + (long long)e * os + ((long long)i << logN);
    for (int j0 = blockIdx.x * 256 + threadIdx.x; j0 < Q; j0 += gridDim.x * 256) {
        const uint32_t b = __brev((uint32_t)j0) >> (34 - logN);
        uint32_t w[16];
        chacha_block((uint32_t)seed, (uint32_t)(seed >> 32), b, ST_SEED_A, index0 + (uint32_t)e, (uint32_t)i, w);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const u64 hi = w[4 * u] | ((u64)w[4 * u + 1] << 32);
            const u64 lo = w[4 * u + 2] | ((u64)w[4 * u + 3] << 32);
            const int bu = (u >> 1) | ((u & 1) << 1);  // bitrev_2(u)
            o[j0 + bu * Q] = reduce128(hi, lo, p);
        }
    }
}

// ternary with P(0) = 1/2, P(+-1) = 1/4 from word x: bit 0 clear -> 0, else bit 1 ? -1 : +1
__global__ __launch_bounds__(256) void ternary_kernel(u64 seed, uint32_t type, uint32_t index, uint32_t comp,
                                                      PosPrimes pp, const PrimeInfo *__restrict__ pinfo,
                                                      u64 *__restrict__ out, int logN)
{
    const int N = 1 << logN;
    const int nblk = N / 8;
    for (int blk = blockIdx.x * 256 + threadIdx.x; blk < nblk; blk += gridDim.x * 256) {
        uint32_t w[16];
        chacha_block((uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)blk, type, index, comp, w);
        for (int c = 0; c < 8; ++c) {
            const uint32_t lo = w[2 * c];
            const int t = (lo & 1) ? ((lo & 2) ? -1 : 1) : 0;
            for (int pos = 0; pos < pp.n; ++pos) {
                const u64 q = pinfo[pp.prime[pos]].q;
                out[((long long)pos << logN) + 8 * blk + c] = t >= 0 ? (u64)t : q - 1;
            }
        }
    }
}

__global__ __launch_bounds__(256) void int_to_rns_kernel(const i64 *__restrict__ m, PosPrimes pp,
                                                         const PrimeInfo *__restrict__ pinfo, u64 *__restrict__ out,
                                                         int logN)
{
    const int pos = blockIdx.y;
    const int N = 1 << logN;
    const PrimeInfo p = pinfo[pp.prime[pos]];
    u64 *o = out + ((long long)pos << logN);
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256) {
        i64 v = m[x];
        u64 mag = v < 0 ? (u64)(-(v + 1)) + 1 : (u64)v;
        u64 r = reduce64(mag, p);
        o[x] = v < 0 ? neg_mod(r, p.q) : r;
    }
}

// evaluation key: b = -a s + e + [pos in digit] (P mod q_pos) s'
__global__ __launch_bounds__(256) void evk_kernel(const u64 *__restrict__ a, const u64 *__restrict__ s,
                                                  const u64 *__restrict__ e, const u64 *__restrict__ sp,
                                                  const u64 *__restrict__ dp, const PrimeInfo *__restrict__ pinfo,
                                                  int d0, int d1, u64 *__restrict__ b, int logN)
{
    const int pos = blockIdx.y;
    const int N = 1 << logN;
    const PrimeInfo p = pinfo[pos];
    const long long off = (long long)pos << logN;
    const bool gad = pos >= d0 && pos < d1;
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256) {
        u64 v = sub_mod(e[off + x], mul_mod(a[off + x], s[off + x], p), p.q);
        if (gad) v = add_mod(v, mul_shoup(sp[off + x], dp[2 * pos], dp[2 * pos + 1], p.q), p.q);
        b[off + x] = v;
    }
}

__global__ __launch_bounds__(256) void enc_kernel(const u64 *__restrict__ a, const u64 *__restrict__ s,
                                                  const u64 *__restrict__ e, const u64 *__restrict__ m,
                                                  const PrimeInfo *__restrict__ pinfo, u64 *__restrict__ b, int logN)
{
    const int i = blockIdx.y;
    const int N = 1 << logN;
    const PrimeInfo p = pinfo[i];
    const long long off = (long long)i << logN;
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256)
        b[off + x] = add_mod(sub_mod(e[off + x], mul_mod(a[off + x], s[off + x], p), p.q), m ? m[off + x] : 0, p.q);
}

// public-key encryption: b = v pk_b + e0 + m, a = v pk_a + e1 (pk component stride pkc)
__global__ __launch_bounds__(256) void encpk_kernel(const u64 *__restrict__ v, const u64 *__restrict__ pk,
                                                    long long pkc, const u64 *__restrict__ e0,
                                                    const u64 *__restrict__ e1, const u64 *__restrict__ m,
                                                    const PrimeInfo *__restrict__ pinfo, u64 *__restrict__ b,
                                                    u64 *__restrict__ a, int logN)
{
    const int i = blockIdx.y;
    const int N = 1 << logN;
    const PrimeInfo p = pinfo[i];
    const long long off = (long long)i << logN;
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256) {
        const u64 vx = v[off + x];
        b[off + x] = add_mod(add_mod(mul_mod(vx, pk[off + x], p), e0[off + x], p.q), m[off + x], p.q);
        a[off + x] = add_mod(mul_mod(vx, pk[pkc + off + x], p), e1[off + x], p.q);
    }
}

__global__ __launch_bounds__(256) void dec_kernel(const u64 *__restrict__ ct, const u64 *__restrict__ s,
                                                  const PrimeInfo *__restrict__ pinfo, u64 *__restrict__ out,
                                                  int level, int logN)
{
    const int i = blockIdx.y;
    const int N = 1 << logN;
    const PrimeInfo p = pinfo[i];
    const long long off = (long long)i << logN;
    const long long a_off = (long long)(level + 1) << logN;
    for (int x = blockIdx.x * 256 + threadIdx.x; x < N; x += gridDim.x * 256)
        out[off + x] = add_mod(ct[off + x], mul_mod(ct[a_off + off + x], s[off + x], p), p.q);
}

inline int xblocks(int N, int per_thread = 4)
{
    int blocks = N / (256 * per_thread);
    return blocks < 1 ? 1 : blocks;
}

PosPrimes make_pp(int n, const int *prime_of_pos)
{
    PosPrimes pp;
    pp.n = n;
    for (int i = 0; i < n; ++i) pp.prime[i] = prime_of_pos[i];
    return pp;
}

}  // namespace

namespace hek {

// Launches are split only past this size (grid-z bound); measured: splitting
// into cache-sized chunks costs more in kernel boundaries than it saves.
constexpr long long NTT_CHUNK_BYTES = 1ll << 40;

// ------------------------------------------------------------------ kernel trace
// A launch's record while the context's trace is on (never under capture):
// an event before the launch on the context's stream, one after it (at the
// end of the scope), and the launch's algorithmic work.
struct KSpan {
    he_ctx *c;
    long idx = -1;
    KSpan(he_ctx *cx, int kind, double bytes, double mm_fp = 0.0, double mm_int = 0.0) : c(cx)
    {
        KTrace &t = c->kt;
        if (!t.on || c->capturing) return;
        hipEvent_t e[2];
        for (int i = 0; i < 2; ++i) {
            if (!t.pool.empty()) {
                e[i] = t.pool.back();
                t.pool.pop_back();
            } else if (hipEventCreate(&e[i]) != hipSuccess) {
                if (i == 1) t.pool.push_back(e[0]);
                t.failed = true;
                return;
            }
        }
        if (hipEventRecord(e[0], c->stream) != hipSuccess) t.failed = true;
        t.recs.push_back(KRec{kind, e[0], e[1], bytes, mm_fp, mm_int});
        idx = (long)t.recs.size() - 1;
    }
    ~KSpan()
    {
        if (idx >= 0 && hipEventRecord(c->kt.recs[idx].b, c->stream) != hipSuccess) c->kt.failed = true;
    }
    KSpan(const KSpan &) = delete;
    KSpan &operator=(const KSpan &) = delete;
};

// positions [pos0, pos0 + npos) of the basis at level ell (q_0..q_ell, then
// the special primes) whose prime is below 2^46 (FP64 arithmetic)
static int fp_pos(const he_ctx *c, int ell, int pos0, int npos)
{
    int n = 0;
    for (int t = pos0; t < pos0 + npos; ++t) {
        const int p = t <= ell ? t : c->nq + t - ell - 1;
        if (p >= 0 && p < c->np && c->q[p] < (1ull << 46)) ++n;
    }
    return n;
}

// limbs that nzc batch x component entries (from a.zoff) of a transform over
// npos positions take, and the FP64 ones among them (skip_digit: component c
// leaves out the positions of digit c)
static void ntt_limbs(const he_ctx *c, const NttArgs &a, int npos, int nzc, double *limbs, double *fpl)
{
    *limbs = *fpl = 0.0;
    if (!c->kt.on || c->capturing) return;  // only a recorded launch needs them
    const int f = fp_pos(c, a.ell, a.pos0, npos);
    double l = 0.0, fl = 0.0;
    for (int z = 0; z < nzc; ++z) {
        int ns = 0, nsf = 0;
        if (a.skip_digit) {
            const int comp = (a.zoff + z) % a.ncomp;
            const int s0 = std::max(comp * a.alpha, a.pos0);
            const int s1 = std::min(std::min(comp * a.alpha + a.alpha, a.ell + 1), a.pos0 + npos);
            if (s1 > s0) {
                ns = s1 - s0;
                nsf = fp_pos(c, a.ell, s0, ns);
            }
        }
        l += npos - ns;
        fl += f - nsf;
    }
    *limbs = l;
    *fpl = fl;
}

// ------------------------------------------------------------------ VALU roofline of the butterflies
// The NTT's two butterfly forms with operands in registers and no memory
// traffic: FP = 1 the signed lazy FP64 form (primes below 2^46), FP = 0 the
// Harvey-lazy Shoup form on 64-bit integers (wider primes).  Each thread runs
// 8 independent butterfly chains for `iters` rounds; the result is stored so
// nothing is dead code.  Butterflies per second over the launch is the
// measured VALU peak of that instruction mix.
template <bool FP>
__global__ __launch_bounds__(256) void valu_bfly_kernel(const PrimeInfo *__restrict__ pinfo, int pidx, int iters,
                                                        u64 *__restrict__ out)
{
    const PrimeInfo p = pinfo[pidx];
    const u64 q = p.q, q2 = 2 * q;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (FP) {
        const double qd = (double)q, qinv = 1.0 / qd;
        double x[8], y[8];
        const double w = (double)(q / 3 + t % 97);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            x[k] = (double)((t * 8 + k) % 1000);
            y[k] = (double)((t * 8 + k) % 777);
        }
        for (int it = 0; it < iters; it += 16) {
            // 16 stages of the transform's butterfly x +- lazy(y w), then one
            // reduction per value: the transform's own mix (ranges within [-32q, 33q])
            for (int st = 0; st < 16; ++st) {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const double r = mulmod_lazy_d(y[k], w, qd, qinv);
                    const double a = x[k];
                    x[k] = a + r;
                    y[k] = a - r;
                }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                x[k] = reduce_d(x[k], qd, qinv);
                y[k] = reduce_d(y[k], qd, qinv);
            }
        }
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += x[k] + y[k];
        out[t] = (u64)acc;
    } else {
        u64 x[8], y[8];
        const u64 w = q / 3 + (u64)(t % 97);
        const u64 ws = (u64)(((u128)w << 64) / q);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            x[k] = (u64)((t * 8 + k) % 1000);
            y[k] = (u64)((t * 8 + k) % 777);
        }
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < 8; ++k) ct_bfly(x[k], y[k], w, ws, q, q2);
        }
        u64 acc = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += x[k] ^ y[k];
        out[t] = acc;
    }
}

// ------------------------------------------------------------------ persistent two-pass NTT
// Both passes of a plain forward or inverse transform in one launch, with the
// intermediate between them kept in the L2 of the XCD that computes it.  A
// workgroup reads the XCD it runs on (hardware register XCC_ID) and takes
// tasks from that XCD's ticket counter; limb g of the batch belongs to XCD
// g mod 8.  A task is one workgroup's share (`part`) of one pass over one
// limb; per XCD the tickets run through phases of P tasks: the first pass of
// limbs 0 .. D-1, then alternately the second pass of limb j and the first
// pass of limb j + D, then the remaining second passes.  Limb k's
// intermediate lives in slot k mod PS_SLOTS of the XCD's slot buffer, so it
// never leaves that XCD's L2 unless evicted.  A second pass waits until its
// limb's first pass has completed (P tasks counted on the slot), a first pass
// waits until the slot's previous limb has finished its second pass.  Every
// wait is on tasks whose tickets were taken earlier by running workgroups of
// the same XCD, so the waits always end: no co-residency is assumed, and one
// workgroup per XCD alone would also finish.  Counters are zeroed by a kernel
// before every launch (graph-safe).
#define HWREG_XCC_ID ((20) | (0 << 6) | ((4 - 1) << 11))  // hwreg(HW_REG_XCC_ID, 0, 4)

struct PersistArgs {
    unsigned *ctr;  // per XCD a 256-byte block: ticket counter, then PS_SLOTS x (first, second) completions
    u64 *slots;     // [8][PS_SLOTS][N]
    int nlimb;      // limbs of the launch (npos x entries x components)
    int npos;
    int lag;        // D: first passes issued ahead of the second ones (1 .. PS_SLOTS - 1)
};

__global__ void persist_reset_kernel(unsigned *ctr, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0u;
}

// Wait until *p reaches need.  Every lane of the calling wave polls (one
// request per wave) and the loop condition is made wave-uniform, so no lane
// diverges.  Bounded: after 2^22 polls (well over a second) it gives up and
// raises the flag word, so a wait that could not end (it cannot, by the
// schedule's construction) ends the kernel with wrong values instead of
// hanging the device.
constexpr int PS_FLAG = 8 * 64;  // word index of the flag after the 8 XCDs' counter blocks
__device__ __forceinline__ void wait_count(unsigned *p, unsigned need, unsigned *flag)
{
    for (unsigned it = 0;; ++it) {
        const unsigned v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (v >= need) return;
        if (it >= (1u << 22)) {
            __hip_atomic_fetch_or(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// The control flow below is wave-uniform everywhere outside the pass bodies:
// tickets and counts are read into scalars (readfirstlane), and the counter
// updates and polls are made by wave 0 (a wave-uniform condition), every lane
// with a nonzero increment on one lane only; so each wave executes the same
// barriers.
template <int LOGN, bool INV>
__global__ __launch_bounds__(LINE_THREADS) void ntt_persist_t(NttArgs a, const PrimeInfo *__restrict__ pinfo,
                                                              const u64 *__restrict__ tw, const u64 *__restrict__ tws,
                                                              const u64 *__restrict__ post,
                                                              const double *__restrict__ twd, PersistArgs ps)
{
    constexpr int LA = (LOGN + 1) / 2, LB = LOGN - LA;
    using SA = LineShape<LA>;
    using SB = LineShape<LB>;
    constexpr int PA = (1 << LB) / SA::LINES;  // column-pass workgroups per limb
    constexpr int PB = (1 << LA) / SB::LINES;  // row-pass workgroups per limb
    constexpr int P = PA > PB ? PA : PB;
    constexpr int WA = SA::LINES * SA::PADDED, WB = SB::LINES * SB::PADDED;
    __shared__ u64 lds[WA > WB ? WA : WB];
    __shared__ unsigned tk;
    const int x = (int)(__builtin_amdgcn_s_getreg(HWREG_XCC_ID) & 7u);
    // this XCD's counter block (its own 256 bytes): [0] tickets, [1 + 2 slot] first-pass
    // completions, [2 + 2 slot] second-pass completions
    unsigned *blk = ps.ctr + 64 * x;
    const int tid = (int)threadIdx.x;
    const unsigned one = threadIdx.x == 0 ? 1u : 0u;
    // wave 0 alone touches the counters (a wave-uniform condition)
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64;
    const int nk = ps.nlimb > x ? (ps.nlimb - x + 7) / 8 : 0;  // this XCD's limbs: g = 8 k + x
    const int D = nk < ps.lag ? nk : ps.lag;
    const unsigned total = 2u * (unsigned)nk * P;
    Fuse f{};
    for (;;) {
        if (wave0) {
            const unsigned got = atomicAdd(blk, one);  // lane 0 takes the ticket
            if (threadIdx.x == 0) tk = got;
        }
        __syncthreads();
        const unsigned t = __builtin_amdgcn_readfirstlane(tk);
        __syncthreads();  // every wave has read tk before the next ticket overwrites it
        if (t >= total) break;
        const int ph = (int)(t / P), part = (int)(t % P);
        bool first;  // the transform's first pass (forward: columns; inverse: rows)
        int k;
        if (ph < D) {
            first = true;
            k = ph;
        } else if (ph - D < 2 * (nk - D)) {
            const int r = ph - D;
            first = (r & 1) != 0;
            k = (r >> 1) + (first ? D : 0);
        } else {
            first = false;
            k = nk - D + (ph - D - 2 * (nk - D));
        }
        const int slot = k % PS_SLOTS;
        const unsigned gen = (unsigned)(k / PS_SLOTS);
        unsigned *d1 = blk + 1 + 2 * slot, *d2 = d1 + 1;
        if (wave0) {
            if (first) {
                if (gen > 0) wait_count(d2, gen * P, ps.ctr + PS_FLAG);  // the slot's previous limb has left it
            } else {
                wait_count(d1, (gen + 1) * P, ps.ctr + PS_FLAG);  // this limb's first pass is complete
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // no stale L1 lines of the slot
        const int g = 8 * k + x;
        const VB vb{part, g % ps.npos, g / ps.npos};
        u64 *xb = ps.slots + ((long long)(x * PS_SLOTS + slot) << LOGN);
        if (!INV) {
            if (first) {
                if (part < PA) ntt_cols_body<LOGN, false, PRO_NONE>(a, pinfo, tw, tws, nullptr, twd, f, vb, lds, xb, tid);
            } else if (part < PB) {
                ntt_rows_body<LOGN, false, EPI_NONE>(a, pinfo, tw, tws, twd, f, vb, lds, xb, tid);
            }
        } else {
            if (first) {
                if (part < PB) ntt_rows_body<LOGN, true, PRO_NONE>(a, pinfo, tw, tws, twd, f, vb, lds, xb, tid);
            } else if (part < PA) {
                ntt_cols_body<LOGN, true, PRO_NONE>(a, pinfo, tw, tws, post, twd, f, vb, lds, xb, tid);
            }
        }
        // the barrier waits for every wave's stores: the task's output is in L2
        __syncthreads();
        if (wave0) atomicAdd(first ? d1 : d2, one);
    }
}

// ------------------------------------------------------------------ one workgroup per limb
// Both passes of a plain transform by one workgroup of G x 256 threads: the G
// 256-thread groups take the first pass's line groups in turns, write the
// intermediate to the workgroup's own scratch limb, meet at a barrier, and
// take the second pass from it.  No workgroup waits for another; the scratch
// limb (N words per workgroup) is rewritten limb after limb, so it stays in
// L2 or the Infinity Cache instead of making a round trip through HBM.  Both
// passes need a multiple of G line groups, so every group executes the same
// barriers.  G = 2 (512 threads) keeps 256 VGPRs per lane; G = 4 (1024
// threads) caps them at 128 and spills.
template <int LOGN, int G>
struct LimbShape {
    static constexpr int LA = (LOGN + 1) / 2, LB = LOGN - LA;
    static constexpr int PA = (1 << LB) / LineShape<LA>::LINES, PB = (1 << LA) / LineShape<LB>::LINES;
    static constexpr int WA = LineShape<LA>::LINES * LineShape<LA>::PADDED, WB = LineShape<LB>::LINES * LineShape<LB>::PADDED;
    static constexpr int W = WA > WB ? WA : WB;
    static constexpr bool OK = PA % G == 0 && PB % G == 0;
};

template <int LOGN, bool INV, int G>
__global__ __launch_bounds__(256 * G) void ntt_limb_t(NttArgs a, const PrimeInfo *__restrict__ pinfo,
                                                      const u64 *__restrict__ tw, const u64 *__restrict__ tws,
                                                      const u64 *__restrict__ post, const double *__restrict__ twd,
                                                      u64 *scratch, int nlimb, int npos)
{
    using LS = LimbShape<LOGN, G>;
    static_assert(LS::OK, "line groups per pass must be a multiple of G");
    __shared__ u64 lds[G * LS::W];
    const int sub = (int)threadIdx.x >> 8, tid = (int)threadIdx.x & 255;
    u64 *sl = lds + sub * LS::W;
    u64 *xb = scratch + ((long long)blockIdx.x << LOGN);
    Fuse f{};
    for (int g = (int)blockIdx.x; g < nlimb; g += (int)gridDim.x) {
        const int y = g % npos, z = g / npos;
        // A body's last LDS read follows its last barrier, so every body call
        // ends with a barrier before the next one writes the same LDS slice.
        // The barrier after a pass's last call also completes the intermediate
        // (one CU: no cache maintenance needed), and the one after the second
        // pass keeps the scratch limb until it has been read.
        if (!INV) {
            for (int it = 0; it < LS::PA / G; ++it) {
                ntt_cols_body<LOGN, false, PRO_NONE>(a, pinfo, tw, tws, nullptr, twd, f, VB{G * it + sub, y, z}, sl,
                                                     xb, tid);
                __syncthreads();
            }
            for (int it = 0; it < LS::PB / G; ++it) {
                ntt_rows_body<LOGN, false, EPI_NONE>(a, pinfo, tw, tws, twd, f, VB{G * it + sub, y, z}, sl, xb, tid);
                __syncthreads();
            }
        } else {
            for (int it = 0; it < LS::PB / G; ++it) {
                ntt_rows_body<LOGN, true, PRO_NONE>(a, pinfo, tw, tws, twd, f, VB{G * it + sub, y, z}, sl, xb, tid);
                __syncthreads();
            }
            for (int it = 0; it < LS::PA / G; ++it) {
                ntt_cols_body<LOGN, true, PRO_NONE>(a, pinfo, tw, tws, post, twd, f, VB{G * it + sub, y, z}, sl, xb,
                                                    tid);
                __syncthreads();
            }
        }
    }
}

template <int LOGN, int G>
static bool limb_launch(he_ctx *c, const NttArgs &a, int nlimb, int npos, int dir, const u64 *post)
{
    if constexpr (!LimbShape<LOGN, G>::OK) {
        return false;
    } else {
        const int grid = std::min(nlimb, std::min(8 * c->persist.wg_per_xcd, c->persist.limb_wgs));
        double l, fl;
        ntt_limbs(c, a, npos, nlimb / npos, &l, &fl);
        const double bf = (double)(1 << (LOGN - 1)) * LOGN;
        KSpan ks(c, HE_K_NTT_ONE_LAUNCH, 2.0 * l * (8 << LOGN), fl * bf, (l - fl) * bf);
        if (dir > 0)
            ntt_limb_t<LOGN, false, G><<<grid, 256 * G, 0, c->stream>>>(a, c->t.pinfo, c->t.psi, c->t.psi_sh,
                                                                        nullptr, c->t.psi_d,
                                                                        c->persist.limb_scratch, nlimb, npos);
        else
            ntt_limb_t<LOGN, true, G><<<grid, 256 * G, 0, c->stream>>>(a, c->t.pinfo, c->t.ipsi, c->t.ipsi_sh, post,
                                                                       c->t.ipsi_d, c->persist.limb_scratch, nlimb,
                                                                       npos);
        return true;
    }
}

template <int LOGN>
static void ntt_launch_t(he_ctx *c, NttArgs a, int nbatch, int npos, int dir, const u64 *post, int pro, int epi,
                         const Fuse &f)
{
    constexpr int LA = (LOGN + 1) / 2, LB = LOGN - LA;
    const int nz = nbatch * a.ncomp;
    if (pro == PRO_NONE && epi == EPI_NONE && (c->persist.on == 2 || c->persist.on == 3) &&
        c->persist.limb_scratch && npos * nz >= c->persist.min_limbs) {
        a.zoff = 0;
        const bool done = c->persist.on == 2 ? limb_launch<LOGN, 2>(c, a, npos * nz, npos, dir, post)
                                             : limb_launch<LOGN, 4>(c, a, npos * nz, npos, dir, post);
        if (done) return;
    }
    if (pro == PRO_NONE && epi == EPI_NONE && c->persist.on == 1 && c->persist.slots &&
        npos * nz >= c->persist.min_limbs) {
        PersistArgs ps;
        ps.ctr = c->persist.ctr;
        ps.slots = c->persist.slots;
        ps.nlimb = npos * nz;
        ps.npos = npos;
        ps.lag = c->persist.lag;
        a.zoff = 0;
        persist_reset_kernel<<<1, 256, 0, c->stream>>>(ps.ctr, PS_FLAG);  // counters (the flag word stays raised)
        const dim3 grid(8 * c->persist.wg_per_xcd);
        double l, fl;
        ntt_limbs(c, a, npos, nz, &l, &fl);
        const double bf = (double)(1 << (LOGN - 1)) * LOGN;
        KSpan ks(c, HE_K_NTT_ONE_LAUNCH, 2.0 * l * (8 << LOGN), fl * bf, (l - fl) * bf);
        if (dir > 0)
            ntt_persist_t<LOGN, false><<<grid, LINE_THREADS, 0, c->stream>>>(a, c->t.pinfo, c->t.psi, c->t.psi_sh,
                                                                            nullptr, c->t.psi_d, ps);
        else
            ntt_persist_t<LOGN, true><<<grid, LINE_THREADS, 0, c->stream>>>(a, c->t.pinfo, c->t.ipsi, c->t.ipsi_sh,
                                                                           post, c->t.ipsi_d, ps);
        return;
    }
    a.xcd = c->persist.on >= 4 ? c->persist.on - 3 : 0;
    const long long per_z = (long long)npos << (LOGN + 3);
    int zc = (int)std::max(1LL, NTT_CHUNK_BYTES / per_z);
    if (zc > nz) zc = nz;
    const PrimeInfo *pi = c->t.pinfo;
    for (int z0 = 0; z0 < nz; z0 += zc) {
        const int nzc = std::min(zc, nz - z0);
        a.zoff = z0;
        dim3 gc((1 << (LOGN - LA)) / LineShape<LA>::LINES, npos, nzc);
        dim3 gr((1 << LA) / LineShape<LB>::LINES, npos, nzc);
        hipStream_t st = c->stream;
        // each pass's algorithmic work: its operands read or written once,
        // the intermediate between the two passes excluded (so the two
        // passes of a plain transform move 16 N bytes a limb together), its
        // butterflies and the products of its fused prologue / epilogue
        double l, fl;
        ntt_limbs(c, a, npos, nzc, &l, &fl);
        const double L8 = 8.0 * (1 << LOGN), NN = (double)(1 << LOGN), HB = NN / 2;
        const int nsrc = pro == PRO_MDRS ? f.nsrc + 1 : f.nsrc;
        const bool conv = dir > 0 && (pro == PRO_MODDOWN || pro == PRO_MDRS);
        const double pro_b = conv ? (double)nzc * nsrc * L8 : l * L8;  // sources, or the input
        const double pro_m = conv ? NN * nsrc : 0.0;
        double epi_b = l * L8, epi_m = 0.0;  // the output
        if (epi == EPI_FINISH) {
            epi_b = 2.0 * l * L8;  // acc, out
            if (f.nbase > 0) epi_b += l * L8 * std::min(f.nbase, a.ncomp) / a.ncomp;
            if (f.add) epi_b += l * L8;
            epi_m = NN * (1 + (f.post ? 1 : 0) + (f.has_kacc ? 1 : 0));
        }
        if (dir > 0) {
            KSpan k1(c, conv ? HE_K_MD_CONV : HE_K_NTT_FWD_COLS, pro_b, fl * (HB * LA + pro_m),
                     (l - fl) * (HB * LA + pro_m));
            if (pro == PRO_MODDOWN)
                ntt_cols_t<LOGN, false, PRO_MODDOWN><<<gc, LINE_THREADS, 0, st>>>(a, pi, c->t.psi, c->t.psi_sh,
                                                                                 nullptr, c->t.psi_d, f);
            else if (pro == PRO_MDRS)
                ntt_cols_t<LOGN, false, PRO_MDRS><<<gc, LINE_THREADS, 0, st>>>(a, pi, c->t.psi, c->t.psi_sh,
                                                                              nullptr, c->t.psi_d, f);
            else
                ntt_cols_t<LOGN, false, PRO_NONE><<<gc, LINE_THREADS, 0, st>>>(a, pi, c->t.psi, c->t.psi_sh, nullptr,
                                                                              c->t.psi_d, f);
        }
        if (dir > 0) {
            KSpan k2(c, epi == EPI_FINISH ? HE_K_MD_FINISH : HE_K_NTT_FWD_ROWS, epi_b, fl * (HB * LB + epi_m),
                     (l - fl) * (HB * LB + epi_m));
            if (epi == EPI_FINISH && f.nbase == 0 && !f.add)
                ntt_rows_t<LOGN, false, EPI_FIN_ACC><<<gr, LINE_THREADS, 0, st>>>(a, pi, c->t.psi, c->t.psi_sh,
                                                                                 c->t.psi_d, f);
            else if (epi == EPI_FINISH)
                ntt_rows_t<LOGN, false, EPI_FINISH><<<gr, LINE_THREADS, 0, st>>>(a, pi, c->t.psi, c->t.psi_sh,
                                                                                c->t.psi_d, f);
            else
                ntt_rows_t<LOGN, false, EPI_NONE><<<gr, LINE_THREADS, 0, st>>>(a, pi, c->t.psi, c->t.psi_sh,
                                                                              c->t.psi_d, f);
        } else {
            {
                const double km = f.has_kmul ? NN : 0.0;
                KSpan k1(c, HE_K_NTT_INV_ROWS, l * L8, fl * (HB * LB + km), (l - fl) * (HB * LB + km));
                if (pro == PRO_SRC)
                    ntt_rows_t<LOGN, true, PRO_SRC><<<gr, LINE_THREADS, 0, st>>>(a, pi, c->t.ipsi, c->t.ipsi_sh,
                                                                                c->t.ipsi_d, f);
                else
                    ntt_rows_t<LOGN, true, PRO_NONE><<<gr, LINE_THREADS, 0, st>>>(a, pi, c->t.ipsi, c->t.ipsi_sh,
                                                                                 c->t.ipsi_d, f);
            }
            const double pm = post ? NN : 0.0;
            KSpan k2(c, HE_K_NTT_INV_COLS, l * L8, fl * (HB * LA + pm), (l - fl) * (HB * LA + pm));
            ntt_cols_t<LOGN, true, PRO_NONE><<<gc, LINE_THREADS, 0, st>>>(a, pi, c->t.ipsi, c->t.ipsi_sh, post,
                                                                         c->t.ipsi_d, f);
        }
    }
}

static void ntt_launch(he_ctx *c, NttArgs a, int nbatch, int npos, int dir, const u64 *post, int pro = PRO_NONE,
                       int epi = EPI_NONE, const Fuse *fp = nullptr)
{
    Fuse f{};
    if (fp) f = *fp;
    switch (a.logN) {
    case 12: return ntt_launch_t<12>(c, a, nbatch, npos, dir, post, pro, epi, f);
    case 13: return ntt_launch_t<13>(c, a, nbatch, npos, dir, post, pro, epi, f);
    case 14: return ntt_launch_t<14>(c, a, nbatch, npos, dir, post, pro, epi, f);
    case 15: return ntt_launch_t<15>(c, a, nbatch, npos, dir, post, pro, epi, f);
    case 16: return ntt_launch_t<16>(c, a, nbatch, npos, dir, post, pro, epi, f);
    default: break;
    }
    // small rings: the stage-per-barrier kernels (no fusion)
    const int N1 = 1 << a.logN1, N2 = 1 << (a.logN - a.logN1);
    const int C = std::min(NTT_TILE >> a.logN1, N2);
    const int R = std::min(NTT_TILE / N2, N1);
    dim3 gc(N2 / C, npos, nbatch * a.ncomp), gr(N1 / R, npos, nbatch * a.ncomp);
    KSpan ks(c, HE_K_OTHER, 0.0);
    if (dir > 0) {
        ntt_cols<false><<<gc, NTT_THREADS, 0, c->stream>>>(a, c->t.pinfo, c->t.psi, c->t.psi_sh, nullptr);
        ntt_rows<false><<<gr, NTT_THREADS, 0, c->stream>>>(a, c->t.pinfo, c->t.psi, c->t.psi_sh);
    } else {
        ntt_rows<true><<<gr, NTT_THREADS, 0, c->stream>>>(a, c->t.pinfo, c->t.ipsi, c->t.ipsi_sh);
        ntt_cols<true><<<gc, NTT_THREADS, 0, c->stream>>>(a, c->t.pinfo, c->t.ipsi, c->t.ipsi_sh, post);
    }
}

void ntt_batch(he_ctx *c, u64 *base, long long bstride, long long cstride, int nbatch, int ncomp, int pos0,
               int npos, int ell, int dir, const u64 *post, bool skip_digit)
{
    NttArgs a;
    a.base = base;
    a.bstride = bstride;
    a.cstride = cstride;
    a.ncomp = ncomp;
    a.pos0 = pos0;
    a.skip_digit = skip_digit ? 1 : 0;
    a.alpha = c->alpha;
    a.ell = ell;
    a.nq = c->nq;
    a.logN = c->logN;
    a.logN1 = (c->logN + 1) / 2;
    a.zoff = 0;
    a.xcd = 0;  // set by the launcher from the context
    ntt_launch(c, a, nbatch, npos, dir, post);
}

static NttArgs make_args(he_ctx *c, u64 *base, long long bstride, long long cstride, int ncomp, int pos0, int ell,
                         bool skip_digit)
{
    NttArgs a;
    a.base = base;
    a.bstride = bstride;
    a.cstride = cstride;
    a.ncomp = ncomp;
    a.pos0 = pos0;
    a.skip_digit = skip_digit ? 1 : 0;
    a.alpha = c->alpha;
    a.ell = ell;
    a.nq = c->nq;
    a.logN = c->logN;
    a.logN1 = (c->logN + 1) / 2;
    a.zoff = 0;
    a.xcd = c->persist.on >= 4 ? c->persist.on - 3 : 0;
    return a;
}

bool fused_ok(const he_ctx *c) { return c->logN >= 12 && c->alpha <= MAXW && c->nk <= MAXW; }

template <int LOGN>
static void ks_fused_t(he_ctx *c, NttArgs a, int B, int beta, int nb, const KsArgs &k)
{
    constexpr int LA = (LOGN + 1) / 2, LB = LOGN - LA;
    Fuse f{};
    a.zoff = 0;
    dim3 gc((1 << (LOGN - LA)) / LineShape<LA>::LINES, nb, B * beta);
    // the digits' transformed limbs (each digit's own positions are already
    // in NTT form and skipped): the column pass reads them, the row pass
    // (the intermediate between them excluded) reads those own positions
    // from d2 and the keys, and writes acc
    double l, fl;
    ntt_limbs(c, a, nb, B * beta, &l, &fl);
    const double L8 = 8.0 * (1 << LOGN), NN = (double)(1 << LOGN), HB = NN / 2;
    {
        KSpan ks(c, HE_K_KS_COLS, l * L8, fl * HB * LA, (l - fl) * HB * LA);
        ntt_cols_t<LOGN, false, PRO_NONE><<<gc, LINE_THREADS, 0, c->stream>>>(a, c->t.pinfo, c->t.psi, c->t.psi_sh,
                                                                              nullptr, c->t.psi_d, f);
    }
    KsArgs kk = k;
    kk.nent = B;
    dim3 gr(B * ((1 << LA) / LineShape<LB>::LINES) * nb, 1, 1);
    const double keys = (k.per_entry ? B : 1) * 2.0 * beta * nb;
    const int fpn = fp_pos(c, k.ell, 0, nb);
    const double ip = (double)B * NN * 2 * beta;  // inner-product products per position
    KSpan ks(c, HE_K_KS_ROWS, ((double)B * (k.ell + 1) + keys + 2.0 * B * nb) * L8, fl * HB * LB + fpn * ip,
             (l - fl) * HB * LB + (nb - fpn) * ip);
    ntt_rows_ks_t<LOGN><<<gr, LINE_THREADS, 0, c->stream>>>(kk, c->t.pinfo, c->t.psi, c->t.psi_sh, c->t.psi_d);
}

void ks_ntt_inner(he_ctx *c, int level, int B, const u64 *d2, long long d2s, u64 *ext, long long es, long long ds,
                  const u64 *key, const EntryKeys *keys, u64 *acc, long long as)
{
    const int beta = (level + 1 + c->alpha - 1) / c->alpha;
    const int nb = level + 1 + c->nk;
    KsArgs k{};
    k.d2 = d2;
    k.d2s = d2s;
    k.ext = ext;
    k.es = es;
    k.ds = ds;
    k.key = key;
    if (keys) k.ek = *keys;
    k.per_entry = keys ? 1 : 0;
    k.acc = acc;
    k.as = as;
    k.alpha = c->alpha;
    k.beta = beta;
    k.ell = level;
    k.nq = c->nq;
    k.np = c->np;
    k.nb = nb;
    NttArgs a = make_args(c, ext, es, ds, beta, 0, level, true);
    switch (c->logN) {
    case 12: return ks_fused_t<12>(c, a, B, beta, nb, k);
    case 13: return ks_fused_t<13>(c, a, B, beta, nb, k);
    case 14: return ks_fused_t<14>(c, a, B, beta, nb, k);
    case 15: return ks_fused_t<15>(c, a, B, beta, nb, k);
    default: return ks_fused_t<16>(c, a, B, beta, nb, k);
    }
}

void intt_from(he_ctx *c, const u64 *src, long long sbs, u64 *dst, long long dbs, int B, int level, const u64 *post)
{
    Fuse f{};
    f.src = src;
    f.sbs = sbs;
    f.scs = 0;
    NttArgs a = make_args(c, dst, dbs, 0, 1, 0, level, false);
    ntt_launch(c, a, B, level + 1, -1, post, PRO_SRC, EPI_NONE, &f);
}

void ntt_moddown(he_ctx *c, int level, int B, const u64 *acc, long long as, u64 *conv, long long cs, const u64 *base,
                 long long bs, long long bcs, int nbase, u64 *out, long long os, long long ocs, const u64 *add,
                 long long ads, long long adcs)
{
    const long long N = c->N, nb = level + 1 + c->nk;
    Fuse f{};
    f.src = acc;
    f.sbs = as;
    f.scs = nb * N;
    f.soff = level + 1;
    f.nsrc = c->nk;
    f.sp0 = c->nq;
    f.cvt = c->t.dn_conv;
    f.cnt = c->t.dn_p;
    f.cvtd = c->t.dn_convd;
    f.cntd = c->t.dn_pd;
    f.nk = c->nk;
    f.np = c->np;
    f.acc = acc;
    f.as = as;
    f.acs = nb * N;
    f.base = base;
    f.bs = bs;
    f.bcs = bcs;
    f.nbase = nbase;
    f.out = out;
    f.os = os;
    f.ocs = ocs;
    f.add = add;
    f.ads = ads;
    f.adcs = adcs;
    f.pinv = c->t.dn_pinv;
    NttArgs a = make_args(c, conv, cs, (level + 1) * N, 2, 0, level, false);
    ntt_launch(c, a, B, level + 1, +1, nullptr, PRO_MODDOWN, EPI_FINISH, &f);
}

// Rescale of B ciphertexts of ncomp components at level l as a one-prime
// ModDown: the last limbs, already in coefficient form in last [b][comp][N],
// are converted (centred) to q_0 .. q_{l-1} inside the first forward pass, and
// the second pass stores (in - x) q_l^{-1} into out (in read with component
// stride ics, times *kmul when kmul is given).  tmp [b][comp][l][N] holds the
// intermediate between the passes.
void ntt_rescale(he_ctx *c, int level, int B, int ncomp, const u64 *last, const u64 *in, long long is, long long ics,
                 u64 *tmp, u64 *out, long long os, const i64 *kmul)
{
    const long long N = c->N, lc_in = ics, lc_out = (long long)level * N;
    Fuse f{};
    f.src = last;
    f.sbs = ncomp * N;
    f.scs = N;
    f.soff = 0;
    f.nsrc = 1;
    f.sp0 = level;
    f.cvt = c->t.rs_one;
    f.cnt = c->t.rs_ql2 + (long long)level * c->nq * 2;
    f.cvtd = c->t.rs_oned + (long long)level * c->nq * 2;
    f.cntd = c->t.rs_qld + (long long)level * c->nq;
    f.acc = in;
    f.as = is;
    f.acs = lc_in;
    f.nbase = 0;
    f.out = out;
    f.os = os;
    f.ocs = lc_out;
    f.pinv = c->t.rs_qinv + (long long)level * c->nq * 2;
    if (kmul) {
        f.has_kacc = 1;
        f.kacc = *kmul;
    }
    NttArgs a = make_args(c, tmp, ncomp * lc_out, lc_out, ncomp, 0, level - 1, false);
    ntt_launch(c, a, B, level, +1, nullptr, PRO_MODDOWN, EPI_FINISH, &f);
}

// inverse NTT of the last limb (position l) of B ciphertexts of ncomp
// components (component stride ics), read in place from in (times *kmul when
// given), written to last [b][comp][N]
void intt_last(he_ctx *c, int level, int B, int ncomp, const u64 *in, long long is, long long ics, u64 *last,
               const i64 *kmul)
{
    const long long N = c->N;
    Fuse f{};
    f.src = in;
    f.sbs = is;
    f.scs = ics;
    if (kmul) {
        f.has_kmul = 1;
        f.kmul = *kmul;
    }
    NttArgs a = make_args(c, last - (long long)level * N, ncomp * N, N, ncomp, level, level, false);
    ntt_launch(c, a, B, 1, -1, nullptr, PRO_SRC, EPI_NONE, &f);
}

static void ew(he_ctx *c, int op, const EwArgs &a, int npos, int nbatch, i64 k)
{
    dim3 g(xblocks(c->N), npos, nbatch * a.ncomp);
    // operands once: x and o per component; y per component (sums), one
    // plaintext per entry (op 3; once when it is shared), none otherwise
    const double lim = (double)npos * nbatch * a.ncomp, L8 = 8.0 * c->N;
    double yl = 0.0;
    if (op == 0 || op == 1) yl = lim;
    else if (op == 3) yl = (double)npos * (a.yb ? nbatch : 1);
    const double fl = (double)fp_pos(c, a.ell, a.pos0, npos) / npos;
    const double mm = (op == 2 || op == 3) ? lim * c->N : 0.0;
    KSpan ks(c, HE_K_ELEMENTWISE, (2.0 * lim + yl) * L8, mm * fl, mm * (1.0 - fl));
    switch (op) {
    case 0: ew_kernel<0><<<g, 256, 0, c->stream>>>(a, c->t.pinfo, k); break;
    case 1: ew_kernel<1><<<g, 256, 0, c->stream>>>(a, c->t.pinfo, k); break;
    case 2: ew_kernel<2><<<g, 256, 0, c->stream>>>(a, c->t.pinfo, k); break;
    case 3: ew_kernel<3><<<g, 256, 0, c->stream>>>(a, c->t.pinfo, k); break;
    case 5: ew_kernel<5><<<g, 256, 0, c->stream>>>(a, c->t.pinfo, k); break;
    default: ew_kernel<4><<<g, 256, 0, c->stream>>>(a, c->t.pinfo, k); break;
    }
}

void ewise(he_ctx *c, int op, int level, int nbatch, int ncomp, const u64 *x, long long xb, long long xc,
           const u64 *y, long long yb, long long yc, u64 *o, long long ob, long long oc, i64 k)
{
    EwArgs a;
    a.x = const_cast<u64 *>(x);
    a.y = const_cast<u64 *>(y);
    a.o = o;
    a.xb = xb; a.xc = xc; a.yb = yb; a.yc = yc; a.ob = ob; a.oc = oc;
    a.ncomp = ncomp;
    a.pos0 = 0;
    a.ell = level;
    a.nq = c->nq;
    a.logN = c->logN;
    ew(c, op, a, level + 1, nbatch, k);
}

void tensor_b(he_ctx *c, int level, int B, const u64 *x, long long xb, long long xc, const u64 *y, long long yb,
              long long yc, u64 *o, long long ob, long long oc)
{
    dim3 g(xblocks(c->N), level + 1, B);
    const double lim = (double)(level + 1) * B, fl = fp_pos(c, level, 0, level + 1) / (double)(level + 1);
    KSpan ks(c, HE_K_TENSOR, 7.0 * lim * 8.0 * c->N, 4.0 * lim * c->N * fl, 4.0 * lim * c->N * (1.0 - fl));
    tensor_kernel<<<g, 256, 0, c->stream>>>(x, xb, xc, y, yb, yc, o, ob, oc, c->t.pinfo, c->logN);
}

void desc_ew(he_ctx *c, int op, const OpDesc *tab, int n, int max_limbs, double limbs)
{
    if (n < 1) return;
    dim3 g(xblocks(c->N), max_limbs, n);
    // operand limbs per entry limb: x, o (two components each; the tensor's
    // o three), y two (sum, tensor) or one (plaintext)
    const double per = op == 0 ? 6.0 : op == 3 ? 5.0 : op == 6 ? 7.0 : 4.0;
    const double mper = op == 2 || op == 3 ? 2.0 : op == 6 ? 4.0 : 0.0;
    const double lim = limbs >= 0.0 ? limbs : (double)n * max_limbs;
    const double fl = (double)fp_pos(c, max_limbs - 1, 0, max_limbs) / max_limbs;
    KSpan ks(c, HE_K_ELEMENTWISE, per * lim * 8.0 * c->N, mper * lim * c->N * fl, mper * lim * c->N * (1.0 - fl));
    switch (op) {
    case 0: desc_ew_kernel<0><<<g, 256, 0, c->stream>>>(tab, c->t.pinfo, c->logN); break;
    case 2: desc_ew_kernel<2><<<g, 256, 0, c->stream>>>(tab, c->t.pinfo, c->logN); break;
    case 3: desc_ew_kernel<3><<<g, 256, 0, c->stream>>>(tab, c->t.pinfo, c->logN); break;
    case 4: desc_ew_kernel<4><<<g, 256, 0, c->stream>>>(tab, c->t.pinfo, c->logN); break;
    default: desc_ew_kernel<6><<<g, 256, 0, c->stream>>>(tab, c->t.pinfo, c->logN); break;
    }
}

void terms_sum_b(he_ctx *c, int lp, int nb, const u64 *A, const u64 *B3, long long as, const u64 *Z1, const u64 *Z2,
                 long long ps, long long pc, const u64 *M, long long ms, long long mc, const u64 *Z, long long zs,
                 long long zc, i64 k0, u64 *G, bool accumulate)
{
    TermArgs a{A, B3, as, Z1, Z2, ps, pc, M, ms, mc, Z, zs, zc, G, k0, nb, accumulate ? 1 : 0, c->logN};
    dim3 g(c->N / 256, lp + 1, 1);
    // per block: A, B3 (3 components each), Z1, Z (2), Z2 (2, when given), M
    // (2, per block or shared); G's 5 components written (and read when accumulating)
    const double per_blk = 10.0 + (Z2 ? 2.0 : 0.0) + (ms ? 2.0 : 0.0);
    const double lim = (lp + 1.0) * (per_blk * nb + (ms ? 0.0 : 2.0) + (accumulate ? 10.0 : 5.0));
    const double fl = fp_pos(c, lp, 0, lp + 1) / (lp + 1.0);
    const double mm = (lp + 1.0) * nb * c->N * (15.0 + (Z2 ? 6.0 : 0.0));
    KSpan ks(c, HE_K_TERMS_SUM, lim * 8.0 * c->N, mm * fl, mm * (1.0 - fl));
    terms_sum_kernel<<<g, 256, 0, c->stream>>>(a, c->t.pinfo);
}

void baby_sum_b(he_ctx *c, int level, int nblk, int nbaby, const u64 *z, long long zb, long long zc, const u64 *zr,
                long long zrb, long long zrs, long long zrc, const u64 *w, long long wc, const u64 *wr, long long wrs,
                long long wrc, u64 *o, long long ob, long long oc)
{
    BabyArgs a{z, zb, zc, zr, zrb, zrs, zrc, w, wc, wr, wrs, wrc, o, ob, oc, nbaby, nblk, c->logN};
    dim3 g(c->N / 256, level + 1, (nblk + BABY_CHUNK - 1) / BABY_CHUNK);
    // every block's nbaby data copies (2 components) and W's nbaby rotations
    // read once, each block's degree-2 product written
    const double lim = (level + 1.0) * (2.0 * nbaby * nblk + 2.0 * nbaby + 3.0 * nblk);
    const double fl = fp_pos(c, level, 0, level + 1) / (level + 1.0);
    const double mm = (level + 1.0) * nblk * nbaby * 4.0 * c->N;
    KSpan ks(c, HE_K_BABY_SUM, lim * 8.0 * c->N, mm * fl, mm * (1.0 - fl));
    switch (nbaby) {
    case 2: baby_sum_kernel<2><<<g, 256, 0, c->stream>>>(a, c->t.pinfo); break;
    case 4: baby_sum_kernel<4><<<g, 256, 0, c->stream>>>(a, c->t.pinfo); break;
    case 8: baby_sum_kernel<8><<<g, 256, 0, c->stream>>>(a, c->t.pinfo); break;
    default: baby_sum_kernel<MAX_BABY><<<g, 256, 0, c->stream>>>(a, c->t.pinfo); break;
    }
}

void modup_b(he_ctx *c, int level, int B, const u64 *y, long long ys, u64 *ext, long long es, long long ds)
{
    const int beta = (level + 1 + c->alpha - 1) / c->alpha;
    dim3 g((c->N / 2 + 255) / 256, B * beta, 1);
    // y read once, every digit's positions outside it written; digit j of
    // alpha_j members takes alpha_j products per target
    const int nb = level + 1 + c->nk;
    double mf = 0.0, mi = 0.0;
    for (int j = 0; j < beta; ++j) {
        const int j0 = j * c->alpha, aj = std::min(c->alpha, level + 1 - j0);
        const int f = fp_pos(c, level, 0, nb) - fp_pos(c, level, j0, aj);
        mf += (double)aj * f;
        mi += (double)aj * (nb - aj - f);
    }
    KSpan ks(c, HE_K_MODUP, (double)B * ((level + 1) + (double)beta * nb - (level + 1)) * 8.0 * c->N,
             mf * B * c->N, mi * B * c->N);
#define HE_MODUP(A)                                                                                                     \
    modup_kernel<A><<<g, 256, 0, c->stream>>>(y, ys, ext, es, ds, c->t.pinfo, c->t.up_conv, c->t.up_qd, c->t.up_convd, \
                                              c->t.up_qdd, c->t.qinv_d, level, c->alpha, c->nq, c->np, c->nk, beta,     \
                                              c->logN)
    if (c->alpha <= 1)
        HE_MODUP(1);
    else if (c->alpha <= 2)
        HE_MODUP(2);
    else if (c->alpha <= 4)
        HE_MODUP(4);
    else if (c->alpha <= 6)
        HE_MODUP(6);
    else if (c->alpha <= 8)
        HE_MODUP(8);
    else
        HE_MODUP(MAX_ALPHA);
#undef HE_MODUP
}

void ks_inner_b(he_ctx *c, int level, int B, const u64 *d2, long long d2s, const u64 *ext, long long es,
                long long ds, const u64 *key, u64 *acc, long long as)
{
    const int beta = (level + 1 + c->alpha - 1) / c->alpha;
    dim3 g(xblocks(c->N, 2), level + 1 + c->nk, 1);
    const int nb = level + 1 + c->nk, f = fp_pos(c, level, 0, nb);
    const double ip = (double)B * c->N * 2 * beta;
    KSpan ks(c, HE_K_OTHER, ((double)B * beta * nb + 2.0 * beta * nb + 2.0 * B * nb) * 8.0 * c->N, f * ip,
             (nb - f) * ip);
    ks_inner_kernel<<<g, 256, 0, c->stream>>>(d2, d2s, ext, es, ds, key, acc, as, c->t.pinfo, B, level, c->alpha,
                                              c->nq, c->np, beta, c->logN);
}

void ks_inner_multi_b(he_ctx *c, int level, int B, const u64 *d2, long long d2s, const u64 *ext, long long es,
                      long long ds, const EntryKeys &keys, u64 *acc, long long as)
{
    const int beta = (level + 1 + c->alpha - 1) / c->alpha;
    dim3 g(xblocks(c->N, 2), level + 1 + c->nk, B);
    const int nb = level + 1 + c->nk, f = fp_pos(c, level, 0, nb);
    const double ip = (double)B * c->N * 2 * beta;
    KSpan ks(c, HE_K_OTHER, ((double)B * beta * nb * 3.0 + 2.0 * B * nb) * 8.0 * c->N, f * ip, (nb - f) * ip);
    ks_inner_multi_kernel<<<g, 256, 0, c->stream>>>(d2, d2s, ext, es, ds, keys, acc, as, c->t.pinfo, level,
                                                    c->alpha, c->nq, c->np, beta, c->logN);
}

void moddown_conv_b(he_ctx *c, int level, int B, const u64 *acc, long long as, u64 *conv, long long cs)
{
    dim3 g((c->N + 255) / 256, B * 2, 1);
    KSpan ks(c, HE_K_OTHER, 2.0 * B * (c->nk + level + 1.0) * 8.0 * c->N);
    moddown_conv_kernel<<<g, 256, 0, c->stream>>>(acc, as, conv, cs, c->t.pinfo, c->t.dn_conv, c->t.dn_p, level,
                                                  c->nq, c->nk, c->logN);
}

void moddown_finish_b(he_ctx *c, int level, int B, const u64 *acc, long long as, const u64 *conv, long long cs,
                      const u64 *base, long long bs, long long bcs, int nbase, u64 *out, long long os,
                      long long ocs, const u64 *add, long long ads, long long adcs)
{
    dim3 g(xblocks(c->N), level + 1, B * 2);
    KSpan ks(c, HE_K_OTHER, 2.0 * B * (level + 1.0) * (3.0 + (nbase > 0 ? nbase / 2.0 : 0.0) + (add ? 1.0 : 0.0)) *
                                8.0 * c->N);
    moddown_finish_kernel<<<g, 256, 0, c->stream>>>(acc, as, conv, cs, base, bs, bcs, nbase, out, os, ocs, add, ads,
                                                    adcs, c->t.pinfo, c->t.dn_pinv, level, c->nk, c->logN);
}

void rescale_bcast_b(he_ctx *c, int level, int B, const u64 *lastc, u64 *tmp, int ncomp)
{
    dim3 g(xblocks(c->N), level, B * ncomp);
    KSpan ks(c, HE_K_OTHER, (double)B * ncomp * (1.0 + level) * 8.0 * c->N);
    rescale_bcast_kernel<<<g, 256, 0, c->stream>>>(lastc, tmp, c->t.pinfo, c->t.rs_ql, level, c->nq, c->logN);
}

void rescale_finish_b(he_ctx *c, int level, int B, const u64 *in, long long is, const u64 *tmp, u64 *out,
                      long long os, int ncomp)
{
    dim3 g(xblocks(c->N, 1), B, 1);
    KSpan ks(c, HE_K_OTHER, 3.0 * B * ncomp * level * 8.0 * c->N);
    rescale_finish_kernel<<<g, 256, 0, c->stream>>>(in, is, tmp, out, os, c->t.pinfo, c->t.rs_qinv, level, c->nq,
                                                    c->logN, ncomp);
}

void automorph_b(he_ctx *c, int B, int nl, const u64 *in, long long ib, long long ic, u64 *out, long long ob,
                 long long oc, u64 g)
{
    dim3 gr(xblocks(c->N), nl, B * 2);
    KSpan ks(c, HE_K_AUTOMORPH, 4.0 * B * nl * 8.0 * c->N);
    automorph_kernel<<<gr, 256, 0, c->stream>>>(in, ib, ic, out, ob, oc, g, c->logN);
}

// the hoisted sum's algorithmic work over the positions whose prime is (fp)
// or is not below 2^46: per position, every entry's beta digits read once,
// the ng keys' beta digits of both components once, the two accumulator
// components written; on q_0..q_l also the input's b part read and the
// base's two components written (the digit at the position's own digit is
// the input's a part, counted with the digits)
static void giant_work(const he_ctx *c, int level, int B, int ng, bool fp, double *bytes, double *mm)
{
    const int beta = (level + 1 + c->alpha - 1) / c->alpha, nb = level + 1 + c->nk;
    double lim = 0.0, pos = 0.0;
    for (int t = 0; t < nb; ++t) {
        if ((fp_pos(c, level, t, 1) == 1) != fp) continue;
        lim += (double)B * beta + 2.0 * beta * ng + 2.0 * B + (t <= level ? 3.0 * B : 0.0);
        pos += 1.0;
    }
    *bytes = lim * 8.0 * c->N;
    *mm = pos * B * c->N * ng * beta * 2.0;
}

static void giant_gather_b(he_ctx *c, int level, int B, const u64 *ext, long long es, long long ds, const u64 *x,
                           long long xs, long long xc, const EntryGal &gals, const EntryKeys &keys, int ng, u64 *acc,
                           long long as, u64 *out, long long os)
{
    GiantArgs a{};
    a.ext = ext;
    a.es = es;
    a.ds = ds;
    a.x = x;
    a.xs = xs;
    a.xc = xc;
    a.keys = keys;
    a.gals = gals;
    a.ng = ng;
    a.acc = acc;
    a.as = as;
    a.out = out;
    a.os = os;
    a.alpha = c->alpha;
    a.beta = (level + 1 + c->alpha - 1) / c->alpha;
    a.ell = level;
    a.nq = c->nq;
    a.np = c->np;
    a.nb = level + 1 + c->nk;
    a.nent = B;
    a.ngroups = (B + GIANT_EPT - 1) / GIANT_EPT;
    a.logN = c->logN;
    const long long nwg = (long long)a.ngroups * (c->N / 256) * a.nb;
    double bf, mf, bi, mi;
    giant_work(c, level, B, ng, true, &bf, &mf);
    giant_work(c, level, B, ng, false, &bi, &mi);
    KSpan ks(c, HE_K_GIANT_GATHER, bf + bi, mf, mi);
    giant_gather_kernel<<<dim3((unsigned)nwg, 1, 1), 256, 0, c->stream>>>(a, c->t.pinfo);
}

void giant_sum_b(he_ctx *c, int level, int B, const u64 *ext, long long es, long long ds, const u64 *x, long long xs,
                 long long xc, const EntryGal &gals, const EntryKeys &keys, int ng, u64 *acc, long long as, u64 *out,
                 long long os)
{
    const int beta = (level + 1 + c->alpha - 1) / c->alpha;
    // tile-local permutations: every Galois element 1 mod 2^(logN - 5)
    bool local = c->logN >= 6 && beta <= GP_MAXB;
    for (int g = 0; g < ng; ++g) local = local && ((gals.g[g] - 1) & ((2ull << (c->logN - 6)) - 1)) == 0;
    if (!local) {
        giant_gather_b(c, level, B, ext, es, ds, x, xs, xc, gals, keys, ng, acc, as, out, os);
        return;
    }
    GiantArgs a{};
    a.es = es;
    a.ds = ds;
    a.xs = xs;
    a.xc = xc;
    a.keys = keys;
    a.gals = gals;
    a.ng = ng;
    a.as = as;
    a.os = os;
    a.alpha = c->alpha;
    a.beta = beta;
    a.ell = level;
    a.nq = c->nq;
    a.np = c->np;
    a.nb = level + 1 + c->nk;
    a.logN = c->logN;
    const int per = beta * 2 * GP_TK * 8;  // staged key bytes per rotation
    // rotations per staged chunk: balanced chunks of at most GP_LDS bytes
    const int nchunk = (ng * per + GP_LDS - 1) / GP_LDS;
    a.gc = (ng + nchunk - 1) / nchunk;
    const size_t lds = (size_t)a.gc * per;
    const unsigned nwg = (unsigned)((c->N / GP_TK) * a.nb);
    a.ext = ext;
    a.x = x;
    a.acc = acc;
    a.out = out;
    a.nent = B;
    double bf, mf, bi, mi;
    giant_work(c, level, B, ng, true, &bf, &mf);
    giant_work(c, level, B, ng, false, &bi, &mi);
    switch (beta) {
#define HE_GIANT(BT)                                                                                      \
    case BT: {                                                                                            \
        {                                                                                                 \
            KSpan ks(c, HE_K_GIANT_FP64, bf, mf, 0.0);                                                    \
            giant_perm_kernel<true, BT><<<nwg, GP_TK * GP_LANES, lds, c->stream>>>(a, c->t.pinfo);        \
        }                                                                                                 \
        KSpan ks(c, HE_K_GIANT_INT, bi, 0.0, mi);                                                         \
        giant_perm_kernel<false, BT><<<nwg, GP_TK * GP_LANES, lds, c->stream>>>(a, c->t.pinfo);           \
        break;                                                                                            \
    }
        HE_GIANT(1);
        HE_GIANT(2);
        HE_GIANT(3);
        HE_GIANT(4);
        HE_GIANT(5);
        HE_GIANT(6);
        HE_GIANT(7);
        HE_GIANT(8);
#undef HE_GIANT
    }
}

void rot_inner_b(he_ctx *c, int level, int n, const u64 *ext, long long ds, const u64 *x, long long xc,
                 const EntryGal &gals, const EntryKeys &keys, u64 *acc, long long as)
{
    GiantArgs a{};
    a.ext = ext;
    a.ds = ds;
    a.x = x;
    a.xc = xc;
    a.keys = keys;
    a.gals = gals;
    a.ng = n;
    a.acc = acc;
    a.as = as;
    a.alpha = c->alpha;
    a.beta = (level + 1 + c->alpha - 1) / c->alpha;
    a.ell = level;
    a.nq = c->nq;
    a.np = c->np;
    a.nb = level + 1 + c->nk;
    a.logN = c->logN;
    const long long nwg = (long long)n * a.nb * (c->N / 256);
    // the one input's digits read once, n rotations' keys, n accumulators written
    const int f = fp_pos(c, level, 0, a.nb);
    const double ip = (double)n * c->N * 2 * a.beta;
    KSpan ks(c, HE_K_ROT_INNER, ((double)a.beta * a.nb + n * 2.0 * a.beta * a.nb + n * 2.0 * a.nb) * 8.0 * c->N,
             f * ip, (a.nb - f) * ip);
    rot_inner_kernel<<<dim3((unsigned)nwg, 1, 1), 256, 0, c->stream>>>(a, c->t.pinfo);
}

void md_last_b(he_ctx *c, int level, int B, const u64 *bl, const u64 *al, const u64 *acc, long long as,
               long long acs, u64 *last)
{
    dim3 g(c->N / 256, B * 2, 1);
    // per component: base's and acc's limbs l, acc's special limbs, the output limb
    const double mm = 2.0 * B * c->N * (c->nk + 1.0);
    const bool fq = c->q[level] < (1ull << 46);
    KSpan ks(c, HE_K_MD_LAST, 2.0 * B * (3.0 + c->nk) * 8.0 * c->N, fq ? mm : 0.0, fq ? 0.0 : mm);
    md_last_kernel<<<g, 256, 0, c->stream>>>(bl, al, acc, as, acs, last, c->t.pinfo, c->t.dn_conv, c->t.dn_p,
                                            c->t.dn_pinv, level, c->nq, c->nk, c->logN);
}

// ModDown of acc by P and the rescale by q_l after it as one forward
// transform: out = (base + (acc - Y) P^{-1}) q_l^{-1} on positions 0..l-1,
// Y the transform of conv_P(acc) + [P] conv_{q_l}(last) (PRO_MDRS); tmp
// [B][2][l][N] holds the transform's intermediate.
void ntt_moddown_rescale(he_ctx *c, int level, int B, const u64 *acc, long long as, const u64 *last,
                         const u64 *base, long long bs, long long bcs, u64 *tmp, u64 *out, long long os)
{
    const long long N = c->N, nb = level + 1 + c->nk;
    Fuse f{};
    f.src = acc;
    f.sbs = as;
    f.scs = nb * N;
    f.soff = level + 1;
    f.nsrc = c->nk;
    f.sp0 = c->nq;
    f.cvt = c->t.dn_conv;
    f.cnt = c->t.dn_p;
    f.cvtd = c->t.dn_convd;
    f.cntd = c->t.dn_pd;
    f.nk = c->nk;
    f.np = c->np;
    f.acc = acc;
    f.as = as;
    f.acs = nb * N;
    f.base = base;
    f.bs = bs;
    f.bcs = bcs;
    f.nbase = 2;
    f.out = out;
    f.os = os;
    f.ocs = (long long)level * N;
    f.pinv = c->t.dn_pinv;
    f.post = c->t.rs_qinv + (long long)level * c->nq * 2;
    f.last = last;
    f.lpos = level;
    NttArgs a = make_args(c, tmp, 2LL * level * N, (long long)level * N, 2, 0, level - 1, false);
    ntt_launch(c, a, B, level, +1, nullptr, PRO_MDRS, EPI_FINISH, &f);
}

void automorph_multi_b(he_ctx *c, int B, int nl, const u64 *in, long long ib, long long ic, u64 *out, long long ob,
                       long long oc, const EntryGal &gals)
{
    dim3 gr(xblocks(c->N), nl, B * 2);
    KSpan ks(c, HE_K_AUTOMORPH, 4.0 * B * nl * 8.0 * c->N);
    automorph_multi_kernel<<<gr, 256, 0, c->stream>>>(in, ib, ic, out, ob, oc, gals, c->logN);
}

void batch_sum(he_ctx *c, int level, int B, const u64 *in, long long ib, long long ic, u64 *out, long long oc,
               bool accumulate, int ncomp)
{
    dim3 g(xblocks(c->N), level + 1, ncomp);
    KSpan ks(c, HE_K_ELEMENTWISE, (B + (accumulate ? 2.0 : 1.0)) * ncomp * (level + 1.0) * 8.0 * c->N);
    batch_sum_kernel<<<g, 256, 0, c->stream>>>(in, ib, ic, B, out, oc, accumulate ? 1 : 0, c->t.pinfo, c->logN);
}

void sample_uniform(he_ctx *c, u64 seed, uint32_t type, uint32_t index, uint32_t comp_base, int n_pos,
                    const int *prime_of_pos, u64 *out)
{
    dim3 g(std::max(1, c->N / 4 / 256), n_pos, 1);
    KSpan ks(c, HE_K_OTHER, ((double)n_pos) * 8.0 * c->N);
    uniform_kernel<<<g, 256, 0, c->stream>>>(seed, type, index, comp_base, make_pp(n_pos, prime_of_pos), c->t.pinfo,
                                             out, c->logN);
}

void sample_cbd(he_ctx *c, u64 seed, uint32_t type, uint32_t index, uint32_t comp, int n_pos,
                const int *prime_of_pos, u64 *out)
{
    dim3 g(std::max(1, c->N / 8 / 256), 1, 1);
    KSpan ks(c, HE_K_OTHER, ((double)n_pos) * 8.0 * c->N);
    cbd_kernel<<<g, 256, 0, c->stream>>>(seed, type, index, comp, make_pp(n_pos, prime_of_pos), c->t.pinfo, out,
                                         c->logN);
}

void int_to_rns(he_ctx *c, const i64 *m, int n_pos, const int *prime_of_pos, u64 *out)
{
    dim3 g(xblocks(c->N), n_pos, 1);
    KSpan ks(c, HE_K_OTHER, (1.0 + n_pos) * 8.0 * c->N);
    int_to_rns_kernel<<<g, 256, 0, c->stream>>>(m, make_pp(n_pos, prime_of_pos), c->t.pinfo, out, c->logN);
}

void evk_combine(he_ctx *c, const u64 *a, const u64 *s, const u64 *e, const u64 *sp, int digit, u64 *b)
{
    int d0 = digit * c->alpha, d1 = std::min(d0 + c->alpha, c->nq);
    dim3 g(xblocks(c->N), c->np, 1);
    KSpan ks(c, HE_K_OTHER, (5.0 * c->np) * 8.0 * c->N);
    evk_kernel<<<g, 256, 0, c->stream>>>(a, s, e, sp, c->t.dn_p, c->t.pinfo, d0, d1, b, c->logN);
}

double valu_bfly_rate(he_ctx *c, bool fp, int pidx, u64 *scratch)
{
    const int blocks = 256 * 8 * 4, iters = 4096;  // 4 workgroups per CU, enough waves to fill every SIMD
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 0.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 0.0;
    }
    float ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
        (void)hipEventRecord(e0, c->stream);
        if (fp)
            valu_bfly_kernel<true><<<blocks, 256, 0, c->stream>>>(c->t.pinfo, pidx, iters, scratch);
        else
            valu_bfly_kernel<false><<<blocks, 256, 0, c->stream>>>(c->t.pinfo, pidx, iters, scratch);
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms > 0.0f ? (double)blocks * 256 * 8 * iters / (ms * 1e-3) : 0.0;
}

void seeded_a(he_ctx *c, u64 seed, uint32_t index0, int nent, int level, u64 *out, long long os)
{
    dim3 g(std::max(1, c->N / 4 / 256), level + 1, nent);
    KSpan ks(c, HE_K_OTHER, ((double)nent * (level + 1)) * 8.0 * c->N);
    seeded_a_kernel<<<g, 256, 0, c->stream>>>(seed, index0, c->t.pinfo, out, os, c->logN);
}

void sample_ternary(he_ctx *c, u64 seed, uint32_t type, uint32_t index, uint32_t comp, int n_pos,
                    const int *prime_of_pos, u64 *out)
{
    dim3 g(std::max(1, c->N / 8 / 256), 1, 1);
    KSpan ks(c, HE_K_OTHER, ((double)n_pos) * 8.0 * c->N);
    ternary_kernel<<<g, 256, 0, c->stream>>>(seed, type, index, comp, make_pp(n_pos, prime_of_pos), c->t.pinfo, out,
                                             c->logN);
}

void encpk_combine(he_ctx *c, int level, const u64 *v, const u64 *pk, const u64 *e0, const u64 *e1, const u64 *m,
                   u64 *b, u64 *a)
{
    dim3 g(xblocks(c->N), level + 1, 1);
    KSpan ks(c, HE_K_OTHER, (8.0 * (level + 1)) * 8.0 * c->N);
    encpk_kernel<<<g, 256, 0, c->stream>>>(v, pk, (long long)c->nq * c->N, e0, e1, m, c->t.pinfo, b, a, c->logN);
}

void enc_combine(he_ctx *c, int level, const u64 *a, const u64 *s, const u64 *e, const u64 *m, u64 *b)
{
    dim3 g(xblocks(c->N), level + 1, 1);
    KSpan ks(c, HE_K_OTHER, (5.0 * (level + 1)) * 8.0 * c->N);
    enc_kernel<<<g, 256, 0, c->stream>>>(a, s, e, m, c->t.pinfo, b, c->logN);
}

void dec_combine(he_ctx *c, int level, const u64 *ct, const u64 *s, u64 *out)
{
    dim3 g(xblocks(c->N), level + 1, 1);
    KSpan ks(c, HE_K_OTHER, (4.0 * (level + 1)) * 8.0 * c->N);
    dec_kernel<<<g, 256, 0, c->stream>>>(ct, s, c->t.pinfo, out, level, c->logN);
}

}  // namespace hek
