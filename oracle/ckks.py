"""Oracle RNS-CKKS: ctypes marshalling around he_oracle.c plus the FP64/big-int
parts (encode/decode, CRT).  Coefficient form everywhere.

TEST INFRASTRUCTURE ONLY (see package docstring).

The scheme is the approximate-number HE the paper builds on (Sec. 3,
"Preliminary": encode/decode by the canonical embedding, RLWE
encrypt/decrypt, addition, multiplication and rescaling); the paper gives no
parameters, so ring degree, prime chain, key-switching digits, sampler and
PRNG are readings, each implemented from its textbook definition.
"""
import ctypes
import math
from ctypes import c_int, c_uint32, c_uint64, c_int64, c_void_p, POINTER

import numpy as np

from . import build as _build

MAXP = 64
HWT = 64  # Hamming weight of the ternary secret (reading: sparse HEAAN-style secret)


class _CParams(ctypes.Structure):
    _fields_ = [("logN", c_int), ("nq", c_int), ("nk", c_int), ("alpha", c_int),
                ("q", c_uint64 * MAXP), ("psi", c_uint64 * MAXP)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    L = ctypes.CDLL(_build.build(force=False))
    P = POINTER(_CParams)
    u64p = POINTER(c_uint64)
    i64p = POINTER(c_int64)
    sig = {
        "orc_mulmod": (c_uint64, [c_uint64, c_uint64, c_uint64]),
        "orc_powmod": (c_uint64, [c_uint64, c_uint64, c_uint64]),
        "orc_is_prime": (c_int, [c_uint64]),
        "orc_gen_primes": (c_int, [c_int, c_int, c_int, u64p]),
        "orc_find_psi": (c_uint64, [c_uint64, c_int]),
        "orc_ntt_fwd": (None, [u64p, c_int, c_uint64, c_uint64]),
        "orc_ntt_inv": (None, [u64p, c_int, c_uint64, c_uint64]),
        "orc_polymul": (None, [u64p, u64p, u64p, c_int, c_uint64, c_uint64]),
        "orc_chacha20_block": (None, [POINTER(c_uint32), c_uint32, POINTER(c_uint32), POINTER(c_uint32)]),
        "orc_prng_words": (None, [c_uint64, c_uint32, c_uint32, c_uint32, c_uint64, c_uint64, u64p]),
        "orc_sample_uniform": (None, [c_uint64, c_uint32, c_uint32, c_uint32, c_uint64, c_int, u64p]),
        "orc_sample_cbd": (None, [c_uint64, c_uint32, c_uint32, c_uint32, c_int, i64p]),
        "orc_sample_hwt": (None, [c_uint64, c_int, c_int, i64p]),
        "orc_sample_ternary": (None, [c_uint64, c_uint32, c_uint32, c_uint32, c_int, i64p]),
        "orc_int_to_rns": (None, [P, i64p, c_int, c_int, u64p]),
        "orc_tensor": (None, [P, c_int, u64p, u64p, u64p]),
        "orc_modup": (None, [P, c_int, c_int, u64p, u64p]),
        "orc_moddown": (None, [P, c_int, u64p, u64p]),
        "orc_ndigits": (c_int, [P, c_int]),
        "orc_keyswitch": (None, [P, c_int, u64p, u64p, u64p]),
        "orc_keyswitch_sum": (None, [P, c_int, c_int, u64p, u64p, u64p]),
        "orc_rescale": (None, [P, c_int, u64p, u64p]),
        "orc_rescale_n": (None, [P, c_int, c_int, u64p, u64p]),
        "orc_tensor_n": (None, [P, c_int, c_int, u64p, c_int, u64p, u64p]),
        "orc_automorph": (None, [P, c_int, POINTER(c_int), c_uint64, u64p, u64p]),
        "orc_add": (None, [P, c_int, u64p, u64p, u64p]),
        "orc_mul_int": (None, [P, c_int, u64p, c_int64, u64p]),
        "orc_mul_plain": (None, [P, c_int, u64p, i64p, u64p]),
        "orc_keygen_secret": (None, [P, c_uint64, c_int, i64p]),
        "orc_gen_evk": (None, [P, i64p, u64p, c_uint64, c_uint32, u64p]),
        "orc_gen_pk": (None, [P, i64p, c_uint64, u64p]),
        "orc_encrypt_sk": (None, [P, c_int, i64p, i64p, c_uint64, c_uint32, u64p]),
        "orc_encrypt_pk": (None, [P, c_int, i64p, u64p, c_uint64, c_uint32, u64p]),
        "orc_decrypt": (None, [P, c_int, u64p, i64p, u64p]),
        "orc_secret_square": (None, [P, i64p, u64p]),
        "orc_set_conv_centring": (None, [c_int]),
        "orc_encrypt_sk_seeded": (None, [P, c_int, i64p, i64p, c_uint64, c_uint32, u64p]),
        "orc_set_threads": (None, [c_int]),
        "orc_max_threads": (c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _u(a):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(POINTER(c_uint64))


def _i(a):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(POINTER(c_int64))


# ---------------------------------------------------------------- parameters
class Params:
    """Ring degree 2^logN; ciphertext primes q_0..q_{nq-1} (top level L=nq-1);
    nk special primes; alpha primes per key-switching digit."""

    def __init__(self, logN, nq, nk, alpha, log_delta):
        self.logN, self.nq, self.nk, self.alpha, self.log_delta = logN, nq, nk, alpha, log_delta
        self.N = 1 << logN
        self.S = self.N // 2
        self.L = nq - 1
        buf = np.zeros(MAXP, dtype=np.uint64)
        if lib().orc_gen_primes(nq, nk, log_delta, _u(buf)) != 0:
            raise ValueError("bad prime-chain request")
        self.q = [int(v) for v in buf[: nq + nk]]
        self.psi = [int(lib().orc_find_psi(q, logN)) for q in self.q]
        self.c = _CParams()
        self.c.logN, self.c.nq, self.c.nk, self.c.alpha = logN, nq, nk, alpha
        for i, (q, p) in enumerate(zip(self.q, self.psi)):
            self.c.q[i] = q
            self.c.psi[i] = p
        self.cp = ctypes.pointer(self.c)

    @classmethod
    def custom(cls, logN, primes, nq, nk, alpha, log_delta=20):
        """Parameters over an explicit prime list (q_0..q_{nq-1}, p_0..): tiny
        rings for brute-force checks.  Every prime must be 1 mod 2N."""
        self = cls.__new__(cls)
        self.logN, self.nq, self.nk, self.alpha, self.log_delta = logN, nq, nk, alpha, log_delta
        self.N = 1 << logN
        self.S = self.N // 2
        self.L = nq - 1
        self.q = [int(v) for v in primes]
        assert len(self.q) == nq + nk and all(q % (2 * self.N) == 1 for q in self.q)
        self.psi = [int(lib().orc_find_psi(q, logN)) for q in self.q]
        self.c = _CParams()
        self.c.logN, self.c.nq, self.c.nk, self.c.alpha = logN, nq, nk, alpha
        for i, (q, p) in enumerate(zip(self.q, self.psi)):
            self.c.q[i] = q
            self.c.psi[i] = p
        self.cp = ctypes.pointer(self.c)
        return self

    @property
    def delta(self):
        return float(2 ** self.log_delta)

    def ndigits(self, level):
        return (level + 1 + self.alpha - 1) // self.alpha

    def special(self):
        return self.q[self.nq:]


class CT:
    """Ciphertext: data uint64 [2][level+1][N] in coefficient form, plus FP64 scale."""

    def __init__(self, data, level, scale):
        self.data = np.ascontiguousarray(data, dtype=np.uint64)
        self.level = level
        self.scale = float(scale)
        assert self.data.shape[0] == 2 and self.data.shape[1] == level + 1

    def copy(self):
        return CT(self.data.copy(), self.level, self.scale)


# ---------------------------------------------------------------- encoding
def _pow5(N):
    e = np.empty(N // 2, dtype=np.int64)
    v = 1
    for j in range(N // 2):
        e[j] = v
        v = (v * 5) % (2 * N)
    return e


def round_half_away(x):
    """Round half away from zero, exactly, on an FP64 array."""
    x = np.asarray(x, dtype=np.float64)
    r = np.floor(x)
    f = x - r
    up = (f > 0.5) | ((f == 0.5) & (x > 0))
    return (r + up).astype(np.float64)


def encode(z, scale, N):
    """Canonical-embedding encode (Sec. 3, "Encode/Decode"): slot j <-> the
    root zeta^(5^j), zeta = exp(i*pi/N); m_i = (2/N) Re sum_j scale*z_j
    zeta^(-5^j i), evaluated with a 2N-point FFT, rounded half away from zero."""
    S = N // 2
    zz = np.zeros(S, dtype=np.complex128)
    z = np.asarray(z)
    zz[: z.shape[0]] = z
    e = _pow5(N)
    V = np.zeros(2 * N, dtype=np.complex128)
    V[e] = zz * scale
    V[(2 * N - e) % (2 * N)] = np.conj(zz) * scale
    m = np.fft.fft(V)[:N].real / N
    m = round_half_away(m)
    if np.max(np.abs(m)) >= 2.0 ** 62:
        raise ValueError("encoded coefficient out of int64 range")
    return m.astype(np.int64)


def decode(m, scale, N):
    """Evaluate m at zeta^(5^j) (j < N/2) and divide by scale; m holds integers
    (Python ints or an int/float array)."""
    mf = np.array([float(v) for v in m], dtype=np.float64) if isinstance(m, list) else np.asarray(m, dtype=np.float64)
    E = np.fft.ifft(np.concatenate([mf, np.zeros(N)])) * (2 * N)
    return E[_pow5(N)] / scale


def crt_centered(res, primes):
    """Exact centered CRT lift of residues res[i][x] mod primes[i] (Python ints)."""
    Q = 1
    for q in primes:
        Q *= q
    acc = np.zeros(res.shape[1], dtype=object)
    for i, q in enumerate(primes):
        Qi = Q // q
        ci = Qi * pow(Qi, -1, q)
        acc = acc + res[i].astype(object) * ci
    out = []
    half = Q // 2
    for v in acc:
        v = int(v) % Q
        out.append(v - Q if v > half else v)
    return out


# ---------------------------------------------------------------- keys
class Keys:
    def __init__(self, P, seed, rot_steps=(), with_pk=False, h=HWT):
        L = lib()
        N = P.N
        self.P = P
        self.seed = seed
        self.s = np.zeros(N, dtype=np.int64)
        if not 0 < h <= N:
            raise ValueError("Hamming weight must be in (0, N]")
        L.orc_keygen_secret(P.cp, seed, h, _i(self.s))
        nfull = P.nq + P.nk
        sp = np.zeros((nfull, N), dtype=np.uint64)
        L.orc_secret_square(P.cp, _i(self.s), _u(sp))
        self.rlk = self._evk(sp, 0)
        # keys for s^3 and s^4 (relinearising degree-3 and degree-4
        # ciphertexts), key ids 2 and 4: even, so apart from every Galois
        # element; s^3 = s^2 s and s^4 = s^2 s^2, negacyclic, per prime
        sp3 = np.zeros_like(sp)
        sp4 = np.zeros_like(sp)
        for i in range(nfull):
            q = P.q[i]
            si = np.ascontiguousarray(np.where(self.s < 0, self.s + q, self.s).astype(np.uint64))
            L.orc_polymul(_u(sp[i]), _u(si), _u(sp3[i]), P.logN, q, P.psi[i])
            L.orc_polymul(_u(sp[i]), _u(sp[i]), _u(sp4[i]), P.logN, q, P.psi[i])
        self.rlk_pow = {2: self.rlk, 3: self._evk(sp3, 2), 4: self._evk(sp4, 4)}
        self.rot = {}
        for t in rot_steps:
            self.add_rotation(t)
        self.pk = None
        if with_pk:
            self.pk = np.zeros((2, P.nq, N), dtype=np.uint64)
            L.orc_gen_pk(P.cp, _i(self.s), seed, _u(self.pk))

    def _evk(self, sp, key_id):
        P = self.P
        beta = P.ndigits(P.L)
        out = np.zeros((beta, 2, P.nq + P.nk, P.N), dtype=np.uint64)
        lib().orc_gen_evk(P.cp, _i(self.s), _u(np.ascontiguousarray(sp)), self.seed, key_id, _u(out))
        return out

    def add_rotation(self, t):
        P = self.P
        g = galois(P, t)
        if g in self.rot:
            return
        nfull = P.nq + P.nk
        srns = np.zeros((nfull, P.N), dtype=np.uint64)
        lib().orc_int_to_rns(P.cp, _i(self.s), 0, nfull, _u(srns))
        sp = automorph_limbs(P, srns, list(range(nfull)), g)
        self.rot[g] = self._evk(sp, g)


def galois(P, t):
    """Galois element of a left rotation by t slots: 5^t mod 2N."""
    return pow(5, t % P.S, 2 * P.N)


def automorph_limbs(P, limbs, prime_idx, g):
    n = limbs.shape[0]
    out = np.zeros_like(limbs)
    idx = (c_int * n)(*prime_idx)
    lib().orc_automorph(P.cp, n, idx, g, _u(np.ascontiguousarray(limbs)), _u(out))
    return out


# ---------------------------------------------------------------- encryption
def encrypt_sk(P, keys, m, level, scale, seed, index):
    """Secret-key encryption (the parameter server encrypts with sk, Alg. 2)."""
    out = np.zeros((2, level + 1, P.N), dtype=np.uint64)
    lib().orc_encrypt_sk(P.cp, level, _i(np.ascontiguousarray(m, dtype=np.int64)), _i(keys.s), seed, index, _u(out))
    return CT(out, level, scale)


def encrypt_sk_seeded(P, keys, m, level, scale, seed, index):
    """Secret-key encryption whose uniform part is a function of (seed, index):
    drawn in the evaluation domain, so a holder of the seed regenerates it."""
    out = np.zeros((2, level + 1, P.N), dtype=np.uint64)
    lib().orc_encrypt_sk_seeded(P.cp, level, _i(np.ascontiguousarray(m, dtype=np.int64)), _i(keys.s), seed, index,
                                _u(out))
    return CT(out, level, scale)


def encrypt_pk(P, keys, m, level, scale, seed, index):
    out = np.zeros((2, level + 1, P.N), dtype=np.uint64)
    lib().orc_encrypt_pk(P.cp, level, _i(np.ascontiguousarray(m, dtype=np.int64)), _u(keys.pk), seed, index, _u(out))
    return CT(out, level, scale)


def decrypt_residues(P, keys, ct):
    out = np.zeros((ct.level + 1, P.N), dtype=np.uint64)
    lib().orc_decrypt(P.cp, ct.level, _u(ct.data), _i(keys.s), _u(out))
    return out


def decrypt(P, keys, ct):
    """Decrypt and decode: complex slot values."""
    res = decrypt_residues(P, keys, ct)
    m = crt_centered(res, P.q[: ct.level + 1])
    return decode(m, ct.scale, P.N)


# ---------------------------------------------------------------- operations
def drop(ct, level):
    assert level <= ct.level
    return CT(ct.data[:, : level + 1], level, ct.scale)


def add(P, x, y):
    assert x.level == y.level
    n = x.level + 1
    out = np.zeros((2, n, P.N), dtype=np.uint64)
    for c in range(2):
        o = np.zeros((n, P.N), dtype=np.uint64)
        lib().orc_add(P.cp, n, _u(np.ascontiguousarray(x.data[c])), _u(np.ascontiguousarray(y.data[c])), _u(o))
        out[c] = o
    return CT(out, x.level, x.scale)


def mul_int(P, x, k, scale=None):
    n = x.level + 1
    out = np.zeros_like(x.data)
    for c in range(2):
        o = np.zeros_like(x.data[c])
        lib().orc_mul_int(P.cp, n, _u(np.ascontiguousarray(x.data[c])), int(k), _u(o))
        out[c] = o
    return CT(out, x.level, x.scale if scale is None else scale)


def mul_plain(P, x, m, pt_scale):
    n = x.level + 1
    out = np.zeros_like(x.data)
    mm = np.ascontiguousarray(m, dtype=np.int64)
    for c in range(2):
        o = np.zeros_like(x.data[c])
        lib().orc_mul_plain(P.cp, n, _u(np.ascontiguousarray(x.data[c])), _i(mm), _u(o))
        out[c] = o
    return CT(out, x.level, x.scale * pt_scale)


def tensor(P, x, y):
    """(d0, d1, d2) of a ciphertext product; returns (array [3][l+1][N], scale)."""
    assert x.level == y.level
    d = np.zeros((3, x.level + 1, P.N), dtype=np.uint64)
    lib().orc_tensor(P.cp, x.level, _u(np.ascontiguousarray(x.data)), _u(np.ascontiguousarray(y.data)), _u(d))
    return d, x.scale * y.scale


def keyswitch(P, level, d, evk):
    out = np.zeros((2, level + 1, P.N), dtype=np.uint64)
    lib().orc_keyswitch(P.cp, level, _u(np.ascontiguousarray(d)), _u(evk), _u(out))
    return out


def keyswitch_sum(P, level, ds, evks):
    """sum_m KS(d_m, evk_m) with the inner products summed before one ModDown."""
    assert len(ds) == len(evks) >= 1
    d = np.ascontiguousarray(np.stack(ds), dtype=np.uint64)
    k = np.ascontiguousarray(np.stack(evks), dtype=np.uint64)
    out = np.zeros((2, level + 1, P.N), dtype=np.uint64)
    lib().orc_keyswitch_sum(P.cp, level, len(ds), _u(d), _u(k), _u(out))
    return out


def relin(P, d, scale, level, keys):
    ks = keyswitch(P, level, d[2], keys.rlk)
    out = np.zeros((2, level + 1, P.N), dtype=np.uint64)
    n = level + 1
    o0 = np.zeros((n, P.N), dtype=np.uint64)
    o1 = np.zeros((n, P.N), dtype=np.uint64)
    lib().orc_add(P.cp, n, _u(np.ascontiguousarray(d[0])), _u(ks[0]), _u(o0))
    lib().orc_add(P.cp, n, _u(np.ascontiguousarray(d[1])), _u(ks[1]), _u(o1))
    out[0], out[1] = o0, o1
    return CT(out, level, scale)


def tensor_n(P, level, x, y):
    """Tensor of two ciphertexts of any degree at level l, each an array
    [deg+1][l+1][N] (a polynomial in the secret): d_k = sum_{i+j=k} x_i y_j."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    y = np.ascontiguousarray(y, dtype=np.uint64)
    assert x.shape[1:] == (level + 1, P.N) and y.shape[1:] == (level + 1, P.N)
    d = np.zeros((x.shape[0] + y.shape[0] - 1, level + 1, P.N), dtype=np.uint64)
    lib().orc_tensor_n(P.cp, level, x.shape[0], _u(x), y.shape[0], _u(y), _u(d))
    return d


def rescale_n(P, level, d):
    """Rescale of every component of an array [n][l+1][N] -> [n][l][N]."""
    d = np.ascontiguousarray(d, dtype=np.uint64)
    out = np.zeros((d.shape[0], level, P.N), dtype=np.uint64)
    lib().orc_rescale_n(P.cp, level, d.shape[0], _u(d), _u(out))
    return out


def add_n(P, level, x, y):
    """Sum of two ciphertext arrays of any degrees (the shorter one padded)."""
    n = level + 1
    if x.shape[0] < y.shape[0]:
        x, y = y, x
    out = np.array(x, dtype=np.uint64, copy=True)
    for k in range(y.shape[0]):
        o = np.zeros((n, P.N), dtype=np.uint64)
        lib().orc_add(P.cp, n, _u(np.ascontiguousarray(x[k])), _u(np.ascontiguousarray(y[k])), _u(o))
        out[k] = o
    return out


def relin_n(P, d, scale, level, keys):
    """Relinearisation of a degree-k ciphertext (k <= 4): (d_0, d_1) plus the
    key switch of each d_j (j >= 2) from s^j to s, each on its own."""
    assert 2 <= d.shape[0] - 1 <= 4
    n = level + 1
    o = [np.ascontiguousarray(d[0]), np.ascontiguousarray(d[1])]
    for j in range(2, d.shape[0]):
        ks = keyswitch(P, level, d[j], keys.rlk_pow[j])
        for c in range(2):
            t = np.zeros((n, P.N), dtype=np.uint64)
            lib().orc_add(P.cp, n, _u(o[c]), _u(ks[c]), _u(t))
            o[c] = t
    return CT(np.stack(o), level, scale)


def mul(P, x, y, keys):
    d, s = tensor(P, x, y)
    return relin(P, d, s, x.level, keys)


def rescale(P, x, scale=None):
    l = x.level
    out = np.zeros((2, l, P.N), dtype=np.uint64)
    lib().orc_rescale(P.cp, l, _u(np.ascontiguousarray(x.data)), _u(out))
    return CT(out, l - 1, x.scale / float(P.q[l]) if scale is None else scale)


def rotate_sum_hoisted(P, x, steps, keys):
    """x + sum_{t in steps} Rot(x, t) as one key switch: each rotation's
    automorphed a-part is switched back to s by its own key, the inner
    products are summed in Q_l u P and divided by P once; the b-parts are
    automorphed and added directly."""
    n = x.level + 1
    idx = list(range(n))
    b = np.ascontiguousarray(x.data[0])
    a_parts, evks = [], []
    for t in steps:
        g = galois(P, t)
        if g not in keys.rot:
            raise KeyError("no rotation key for step %d" % t)
        o = np.zeros((n, P.N), dtype=np.uint64)
        lib().orc_add(P.cp, n, _u(b), _u(automorph_limbs(P, x.data[0], idx, g)), _u(o))
        b = o
        a_parts.append(automorph_limbs(P, x.data[1], idx, g))
        evks.append(keys.rot[g])
    ks = keyswitch_sum(P, x.level, a_parts, evks)
    o0 = np.zeros((n, P.N), dtype=np.uint64)
    o1 = np.zeros((n, P.N), dtype=np.uint64)
    lib().orc_add(P.cp, n, _u(b), _u(ks[0]), _u(o0))
    lib().orc_add(P.cp, n, _u(np.ascontiguousarray(x.data[1])), _u(ks[1]), _u(o1))
    return CT(np.stack([o0, o1]), x.level, x.scale)


def rotate(P, x, t, keys):
    """Left rotation of the slot vector by t (automorphism X -> X^(5^t)),
    then key switch of the automorphed a-part back to s."""
    g = galois(P, t)
    if g == 1:
        return x.copy()
    if g not in keys.rot:
        raise KeyError("no rotation key for step %d" % t)
    idx = list(range(x.level + 1))
    b = automorph_limbs(P, x.data[0], idx, g)
    a = automorph_limbs(P, x.data[1], idx, g)
    ks = keyswitch(P, x.level, a, keys.rot[g])
    n = x.level + 1
    o0 = np.zeros((n, P.N), dtype=np.uint64)
    lib().orc_add(P.cp, n, _u(b), _u(ks[0]), _u(o0))
    return CT(np.stack([o0, ks[1]]), x.level, x.scale)


def add_const(P, x, k):
    """x + k for an integer k: the constant polynomial k added to the b-part
    (coefficient 0), which adds k to every slot at x's scale."""
    out = x.data.copy()
    for i in range(x.level + 1):
        q = P.q[i]
        out[0, i, 0] = np.uint64((int(out[0, i, 0]) + int(k)) % q)
    return CT(out, x.level, x.scale)
