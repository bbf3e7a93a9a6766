"""Pins of the CPU oracle against values fixed by the paper, by textbook
definitions and by brute force on tiny rings (Python big integers).

No expected value here is produced by the GPU library.
"""
import ctypes
import math
import os
import random

import numpy as np
import pytest

from oracle import ckks as O
from oracle import lr as LR
from paper_2006_10091_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ independent helpers
def is_prime_py(n):
    """Deterministic Miller-Rabin for n < 3.3e24 (Python ints, written here)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(count, bits, two_n, start_offset=0):
    """`count` primes 1 mod two_n just below 2^bits."""
    out = []
    c = ((1 << bits) - 1) // two_n * two_n + 1 - start_offset * two_n
    while len(out) < count:
        if is_prime_py(c):
            out.append(c)
        c -= two_n
    return out


def schoolbook_negacyclic(a, b, q):
    N = len(a)
    c = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                c[k] += a[i] * b[j]
            else:
                c[k - N] -= a[i] * b[j]
    return [v % q for v in c]


def crt_py(res_cols, primes):
    """Centered integer with the given residues (brute CRT by Python pow)."""
    Q = math.prod(primes)
    x = 0
    for r, q in zip(res_cols, primes):
        Qi = Q // q
        x += int(r) * Qi * pow(Qi, -1, q)
    x %= Q
    return x - Q if x > Q // 2 else x


def tiny_params(logN=4, nq=4, nk=2, alpha=2, bits=26):
    two_n = 2 << logN
    qs = ntt_primes(nq, bits, two_n)
    ps = ntt_primes(nk, bits + 4, two_n)
    return O.Params.custom(logN, qs + ps, nq, nk, alpha)


def limbs_of_int(xs, primes):
    return np.array([[int(x) % q for x in xs] for q in primes], dtype=np.uint64)


# ------------------------------------------------------------ PRNG
def test_chacha20_rfc8439_block():
    vals = {}
    for line in open(os.path.join(GOLDEN, "chacha20_block.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        vals[k] = v
    key = (ctypes.c_uint32 * 8)(*[int(x, 16) for x in vals["key"]])
    nonce = (ctypes.c_uint32 * 3)(*[int(x, 16) for x in vals["nonce"]])
    out = (ctypes.c_uint32 * 16)()
    O.lib().orc_chacha20_block(key, int(vals["counter"][0]), nonce, out)
    assert [int(x, 16) for x in vals["out"]] == list(out)


def test_prng_word_stream_layout():
    # word t of block b is out[2t] | out[2t+1] << 32 of block counter b
    seed = 0x0123456789ABCDEF
    words = np.zeros(24, dtype=np.uint64)
    O.lib().orc_prng_words(seed, 6, 7, 8, 0, 24, words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    key = (ctypes.c_uint32 * 8)(seed & 0xFFFFFFFF, seed >> 32, 0, 0, 0, 0, 0, 0)
    nonce = (ctypes.c_uint32 * 3)(6, 7, 8)
    for b in range(3):
        out = (ctypes.c_uint32 * 16)()
        O.lib().orc_chacha20_block(key, b, nonce, out)
        for t in range(8):
            assert int(words[8 * b + t]) == out[2 * t] | (out[2 * t + 1] << 32)


# ------------------------------------------------------------ primes and roots
@pytest.mark.parametrize("cfg", [(13, 5, 1, 1, 30), (16, 20, 4, 4, 40), (16, 24, 6, 6, 40)])
def test_prime_chain_rule(cfg):
    logN, nq, nk, alpha, ld = cfg
    P = O.Params(logN, nq, nk, alpha, ld)
    M = 1 << 17
    for q in P.q:
        assert q % M == 1 and q < (1 << 60) and is_prime_py(q)
    assert len(set(P.q)) == len(P.q)
    # special primes: the nk largest admissible primes below 2^60
    spec = P.q[nq:]
    c = ((1 << 60) - 1) // M * M + 1
    expect = []
    while len(expect) < nk:
        if is_prime_py(c):
            expect.append(c)
        c -= M
    assert spec == expect
    # q_0: largest admissible prime below 2^min(60, ld+20), not special
    b0 = min(60, ld + 20)
    c = ((1 << b0) - 1) // M * M + 1
    while not (is_prime_py(c) and c not in spec):
        c -= M
    assert P.q[0] == c
    # scale primes: the nq-1 admissible primes closest to 2^ld, by distance
    D = 1 << ld
    chosen = P.q[1:nq]
    dist = [abs(q - D) for q in chosen]
    assert dist == sorted(dist)
    far = max(dist)
    lo = (D - far) // M * M + 1
    cand = [x for x in range(lo, D + far + 1, M) if abs(x - D) < far and is_prime_py(x)]
    assert set(cand) <= set(chosen)


def test_psi_primitive_and_first():
    P = O.Params(13, 5, 1, 1, 30)
    N = P.N
    for q, psi in zip(P.q, P.psi):
        assert pow(psi, N, q) == q - 1
        for x in range(2, 50):
            y = pow(x, (q - 1) // (2 * N), q)
            if pow(y, N, q) == q - 1:
                assert y == psi
                break


# ------------------------------------------------------------ NTT / products
def _u64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


@pytest.mark.parametrize("logN", [3, 4, 5])
def test_ntt_matches_definition(logN):
    N = 1 << logN
    q = ntt_primes(1, 30, 2 * N)[0]
    psi = int(O.lib().orc_find_psi(q, logN))
    rnd = random.Random(logN)
    a = [rnd.randrange(q) for _ in range(N)]
    arr = np.array(a, dtype=np.uint64)
    O.lib().orc_ntt_fwd(_u64p(arr), logN, q, psi)
    want = [sum(a[i] * pow(psi, (2 * k + 1) * i, q) for i in range(N)) % q for k in range(N)]
    assert [int(v) for v in arr] == want
    O.lib().orc_ntt_inv(_u64p(arr), logN, q, psi)
    assert [int(v) for v in arr] == a


def test_ntt_of_delta_is_all_ones():
    logN, N = 6, 64
    q = ntt_primes(1, 40, 2 * N)[0]
    psi = int(O.lib().orc_find_psi(q, logN))
    a = np.zeros(N, dtype=np.uint64)
    a[0] = 1
    O.lib().orc_ntt_fwd(_u64p(a), logN, q, psi)
    assert np.all(a == 1)


@pytest.mark.parametrize("logN,bits", [(3, 20), (4, 40), (6, 59)])
def test_polymul_vs_schoolbook(logN, bits):
    N = 1 << logN
    q = ntt_primes(1, bits, 2 * N)[0]
    psi = int(O.lib().orc_find_psi(q, logN))
    rnd = random.Random(bits)
    a = [rnd.randrange(q) for _ in range(N)]
    b = [rnd.randrange(q) for _ in range(N)]
    A, B, C = (np.array(a, dtype=np.uint64), np.array(b, dtype=np.uint64), np.zeros(N, dtype=np.uint64))
    O.lib().orc_polymul(_u64p(A), _u64p(B), _u64p(C), logN, q, psi)
    assert [int(v) for v in C] == schoolbook_negacyclic(a, b, q)


def test_rns_product_is_bigint_product_mod_Q():
    P = tiny_params(logN=4, nq=3, nk=1, alpha=1)
    rnd = random.Random(5)
    N, Q = P.N, math.prod(P.q[:3])
    a = [rnd.randrange(-1000, 1000) for _ in range(N)]
    b = [rnd.randrange(-(1 << 40), 1 << 40) for _ in range(N)]
    x = O.CT(np.stack([limbs_of_int(a, P.q[:3]), limbs_of_int([0] * N, P.q[:3])]), 2, 1.0)
    y = O.CT(np.stack([limbs_of_int(b, P.q[:3]), limbs_of_int([0] * N, P.q[:3])]), 2, 1.0)
    d, _ = O.tensor(P, x, y)
    want = schoolbook_negacyclic(a, b, Q)
    got = [crt_py(d[0][:, k], P.q[:3]) % Q for k in range(N)]
    assert got == want


def test_crt_centered_bigint():
    primes = ntt_primes(4, 50, 1 << 17)
    Q = math.prod(primes)
    rnd = random.Random(9)
    xs = [rnd.randrange(-(Q // 2), Q // 2) for _ in range(64)]
    res = limbs_of_int(xs, primes)
    assert O.crt_centered(res, primes) == xs


# ------------------------------------------------------------ basis conversion, rescale
def test_modup_exact_relation():
    P = tiny_params(logN=4, nq=4, nk=2, alpha=2)
    N, level = P.N, 3
    rnd = random.Random(11)
    Q = math.prod(P.q[:4])
    xs = [rnd.randrange(Q) for _ in range(N)]
    d = limbs_of_int(xs, P.q[:4])
    for j in range(P.ndigits(level)):
        ext = np.zeros((level + 1 + P.nk, N), dtype=np.uint64)
        O.lib().orc_modup(P.cp, level, j, _u64p(d), _u64p(ext))
        D = list(range(j * P.alpha, min((j + 1) * P.alpha, level + 1)))
        QD = math.prod(P.q[i] for i in D)
        basis = P.q[: level + 1] + P.special()
        for k in range(N):
            X = crt_py(ext[:, k], basis)  # the integer the converted digit represents
            xD = xs[k] % QD
            e, rem = divmod(X - xD, QD)
            assert rem == 0                              # X = x mod Q_D
            assert -len(D) // 2 - 1 <= e <= len(D) // 2  # centered digits: small overflow


def test_moddown_is_division_by_P():
    P = tiny_params(logN=4, nq=4, nk=2, alpha=2)
    N, level = P.N, 3
    rnd = random.Random(12)
    basis = P.q[: level + 1] + P.special()
    QP = math.prod(basis)
    Pm = math.prod(P.special())
    Q = math.prod(P.q[: level + 1])
    xs = [rnd.randrange(QP) for _ in range(N)]
    c = limbs_of_int(xs, basis)
    out = np.zeros((level + 1, N), dtype=np.uint64)
    O.lib().orc_moddown(P.cp, level, _u64p(c), _u64p(out))
    for k in range(N):
        y = crt_py(out[:, k], P.q[: level + 1])
        xc = xs[k] if xs[k] <= QP // 2 else xs[k] - QP
        # y = (x - conv)/P with conv = x mod P (centered digits, overflow <= k/2+1)
        diff = (y * Pm - xc) % Q
        diff = diff - Q if diff > Q // 2 else diff
        assert abs(diff) <= (P.nk // 2 + 1) * Pm


def test_rescale_is_rounded_division():
    P = tiny_params(logN=4, nq=4, nk=1, alpha=1)
    N, level = P.N, 3
    rnd = random.Random(13)
    Q = math.prod(P.q[:4])
    xs = [[rnd.randrange(-(Q // 2), Q // 2) for _ in range(N)] for _ in range(2)]
    ct = O.CT(np.stack([limbs_of_int(x, P.q[:4]) for x in xs]), level, 1.0)
    out = O.rescale(P, ct)
    ql = P.q[level]
    for c in range(2):
        for k in range(N):
            want = (2 * xs[c][k] + ql) // (2 * ql)  # round(x/q_l); q_l odd: no ties
            assert crt_py(out.data[c][:, k], P.q[:3]) == want


def test_automorphism_is_substitution():
    P = tiny_params(logN=4, nq=2, nk=1, alpha=1)
    N = P.N
    rnd = random.Random(14)
    a = [rnd.randrange(P.q[0]) for _ in range(N)]
    for g in (5, 25, 2 * N - 1, 3):
        out = O.automorph_limbs(P, np.array([a], dtype=np.uint64), [0], g)
        want = [0] * N
        for i, v in enumerate(a):  # a(X^g) reduced mod X^N + 1
            e = (i * g) % (2 * N)
            if e < N:
                want[e] = (want[e] + v) % P.q[0]
            else:
                want[e - N] = (want[e - N] - v) % P.q[0]
        assert [int(v) for v in out[0]] == want


# ------------------------------------------------------------ keys, encryption, key switching
def test_sampler_properties():
    P = O.Params(13, 5, 1, 1, 30)
    N = P.N
    s = np.zeros(N, dtype=np.int64)
    O.lib().orc_sample_hwt(77, 13, 64, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    assert np.count_nonzero(s) == 64 and set(np.unique(s)) <= {-1, 0, 1}
    e = np.zeros(N, dtype=np.int64)
    O.lib().orc_sample_cbd(77, 3, 0, 0, 13, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    assert np.abs(e).max() <= 21 and abs(e.mean()) < 0.2 and 9.0 < e.var() < 12.0
    u = np.zeros(N, dtype=np.uint64)
    O.lib().orc_sample_uniform(77, 2, 0, 0, P.q[1], 13, _u64p(u))
    assert int(u.max()) < P.q[1] and abs(u.astype(np.float64).mean() / P.q[1] - 0.5) < 0.02


def test_encrypt_decrypt_exact_noise_bound():
    P = O.Params(13, 5, 1, 1, 30)
    keys = O.Keys(P, 2001, with_pk=True)
    m = synth.small_poly(3, P.N, 1 << 40)
    for level in (P.L, 2):
        ct = O.encrypt_sk(P, keys, m, level, 1.0, 3001, 0)
        got = O.crt_centered(O.decrypt_residues(P, keys, ct), P.q[: level + 1])
        err = np.array(got, dtype=object) - m.astype(object)
        assert max(abs(int(v)) for v in err) <= 21  # e is centered binomial(21)
    ct = O.encrypt_pk(P, keys, m, P.L, 1.0, 3001, 1)
    got = O.crt_centered(O.decrypt_residues(P, keys, ct), P.q[: P.L + 1])
    err = np.array(got, dtype=object) - m.astype(object)
    assert max(abs(int(v)) for v in err) < 2 ** 12  # v*e + e0 + e1*s, h = 64


def test_keyswitch_decrypts_to_d_times_sprime():
    P = tiny_params(logN=5, nq=4, nk=2, alpha=2, bits=28)
    keys = O.Keys(P, 21, rot_steps=[1], h=8)
    N, level = P.N, 3
    rnd = random.Random(15)
    Q = math.prod(P.q[:4])
    dx = [rnd.randrange(Q) for _ in range(N)]
    d = limbs_of_int(dx, P.q[:4])
    ks = O.keyswitch(P, level, d, keys.rlk)
    ct = O.CT(ks, level, 1.0)
    got = O.crt_centered(O.decrypt_residues(P, keys, ct), P.q[:4])
    s = [int(v) for v in keys.s]
    s2 = schoolbook_negacyclic(s, s, Q)
    want = schoolbook_negacyclic(dx, s2, Q)
    for k in range(N):
        diff = (got[k] - want[k]) % Q
        diff = diff - Q if diff > Q // 2 else diff
        assert abs(diff) < 2 ** 12


def _poly_in_secret(comps, s, Q):
    """sum_k comps[k] s^k in Z_Q[X]/(X^N + 1), by schoolbook products."""
    N = len(s)
    acc, sk = [0] * N, [1] + [0] * (N - 1)
    for k, ck in enumerate(comps):
        if k:
            sk = schoolbook_negacyclic(sk, s, Q)
        acc = [(a + b) % Q for a, b in zip(acc, schoolbook_negacyclic(ck, sk, Q))]
    return acc


def test_tensor_of_degree_two_ciphertexts_decrypts_to_the_product():
    # a ciphertext of degree k is a polynomial in s: the tensor must be the
    # product of the two polynomials, so its value at s is the product of values
    P = tiny_params(logN=3, nq=3, nk=1, alpha=1, bits=24)
    N, level = P.N, 2
    Q = math.prod(P.q[:3])
    rnd = random.Random(31)
    s = [rnd.choice((-1, 0, 1)) for _ in range(N)]
    for nx, ny in ((3, 3), (3, 2), (2, 2)):
        xs = [[rnd.randrange(Q) for _ in range(N)] for _ in range(nx)]
        ys = [[rnd.randrange(Q) for _ in range(N)] for _ in range(ny)]
        d = O.tensor_n(P, level, np.stack([limbs_of_int(x, P.q[:3]) for x in xs]),
                       np.stack([limbs_of_int(y, P.q[:3]) for y in ys]))
        assert d.shape[0] == nx + ny - 1
        got = _poly_in_secret([[crt_py(d[k][:, i], P.q[:3]) % Q for i in range(N)] for k in range(d.shape[0])], s, Q)
        vx, vy = _poly_in_secret(xs, s, Q), _poly_in_secret(ys, s, Q)
        assert got == schoolbook_negacyclic(vx, vy, Q)


def test_rescale_of_three_components_is_rounded_division():
    P = tiny_params(logN=4, nq=4, nk=1, alpha=1)
    N, level = P.N, 3
    rnd = random.Random(32)
    Q = math.prod(P.q[:4])
    xs = [[rnd.randrange(-(Q // 2), Q // 2) for _ in range(N)] for _ in range(3)]
    out = O.rescale_n(P, level, np.stack([limbs_of_int(x, P.q[:4]) for x in xs]))
    ql = P.q[level]
    for c in range(3):
        for k in range(N):
            assert crt_py(out[c][:, k], P.q[:3]) == (2 * xs[c][k] + ql) // (2 * ql)


def test_relinearisation_of_degree_four_decrypts_to_its_value_at_s():
    # (d0..d4) -> (d0', d1') with d0' + d1' s = sum_k d_k s^k + small: pins
    # the keys for s^2, s^3 and s^4 (a wrong power leaves an error of size Q)
    P = tiny_params(logN=5, nq=4, nk=2, alpha=2, bits=28)
    keys = O.Keys(P, 22, h=8)
    N, level = P.N, 3
    Q = math.prod(P.q[:4])
    rnd = random.Random(33)
    s = [int(v) for v in keys.s]
    for deg in (2, 3, 4):
        ds = [[rnd.randrange(Q) for _ in range(N)] for _ in range(deg + 1)]
        ct = O.relin_n(P, np.stack([limbs_of_int(x, P.q[:4]) for x in ds]), 1.0, level, keys)
        got = O.crt_centered(O.decrypt_residues(P, keys, ct), P.q[:4])
        want = _poly_in_secret(ds, s, Q)
        for k in range(N):
            diff = (got[k] - want[k]) % Q
            diff = diff - Q if diff > Q // 2 else diff
            assert abs(diff) < (deg - 1) * 2 ** 12


def test_keyswitch_sum_decrypts_to_the_sum_of_products():
    # sum_m KS(d_m, evk_m) with one ModDown: decrypts to sum_m d_m s'_m + small
    P = tiny_params(logN=5, nq=4, nk=2, alpha=2, bits=28)
    keys = O.Keys(P, 23, rot_steps=[1, 3], h=8)
    N, level = P.N, 3
    Q = math.prod(P.q[:4])
    rnd = random.Random(34)
    s = [int(v) for v in keys.s]
    ds = [[rnd.randrange(Q) for _ in range(N)] for _ in range(3)]
    evks = [keys.rlk, keys.rot[O.galois(P, 1)], keys.rot[O.galois(P, 3)]]
    ks = O.keyswitch_sum(P, level, [limbs_of_int(x, P.q[:4]) for x in ds], evks)
    got = O.crt_centered(O.decrypt_residues(P, keys, O.CT(ks, level, 1.0)), P.q[:4])
    s2 = schoolbook_negacyclic(s, s, Q)
    want = [0] * N
    for dm, sp in zip(ds, [s2, _subst(s, O.galois(P, 1), Q), _subst(s, O.galois(P, 3), Q)]):
        want = [(a + b) % Q for a, b in zip(want, schoolbook_negacyclic(dm, sp, Q))]
    for k in range(N):
        diff = (got[k] - want[k]) % Q
        diff = diff - Q if diff > Q // 2 else diff
        assert abs(diff) < 2 ** 12


def _subst(a, g, Q):
    """a(X^g) mod X^N + 1 (brute force)."""
    N = len(a)
    out = [0] * N
    for i, v in enumerate(a):
        e = (i * g) % (2 * N)
        if e < N:
            out[e] = (out[e] + v) % Q
        else:
            out[e - N] = (out[e - N] - v) % Q
    return out


def test_hoisted_rotation_sum():
    P = O.Params(13, 5, 1, 1, 30)
    steps = [512, 1024, 1536]  # three of the rotations by multiples of S / 8
    keys = O.Keys(P, 2001, rot_steps=steps)
    a = np.random.default_rng(5).uniform(-1, 1, P.S)
    ct = O.encrypt_sk(P, keys, O.encode(a, P.delta, P.N), P.L, P.delta, 3001, 0)
    # one step: exactly the rotate-and-add (one key switch, one ModDown)
    one = O.rotate_sum_hoisted(P, ct, [512], keys)
    assert np.array_equal(one.data, O.add(P, ct, O.rotate(P, ct, 512, keys)).data)
    # several: the slot sum of the rotations
    got = O.decrypt(P, keys, O.rotate_sum_hoisted(P, ct, steps, keys)).real
    want = a + sum(np.roll(a, -t) for t in steps)
    assert np.max(np.abs(got - want)) < 2.0 ** -14


# ------------------------------------------------------------ encode / decode
def test_encode_constant_is_exact():
    N = 1 << 13
    for c, scale in ((0.7, 2.0 ** 30), (-1.25, 2.0 ** 40)):
        m = O.encode(np.full(N // 2, c), scale, N)
        assert m[0] == round(c * scale) and not np.any(m[1:])


def test_encode_matches_direct_canonical_embedding():
    N, scale = 16, 2.0 ** 20
    rnd = np.random.default_rng(3)
    z = rnd.uniform(-1, 1, N // 2) + 1j * rnd.uniform(-1, 1, N // 2)
    m = O.encode(z, scale, N)
    zeta = np.exp(1j * np.pi / N)
    for i in range(N):
        v = 0.0
        for j in range(N // 2):
            v += (z[j] * zeta ** (-(pow(5, j, 2 * N)) * i)).real
        v *= 2 * scale / N
        assert abs(m[i] - v) <= 0.5 + 1e-6
    back = O.decode(m, scale, N)
    assert np.max(np.abs(back - z)) < N / scale


def test_rotation_is_slot_roll():
    P = O.Params(13, 5, 1, 1, 30)
    keys = O.Keys(P, 2001, rot_steps=[4, -1])
    a = np.random.default_rng(1).uniform(-1, 1, P.S)
    ct = O.encrypt_sk(P, keys, O.encode(a, P.delta, P.N), P.L, P.delta, 3001, 0)
    for t in (4, -1):
        got = O.decrypt(P, keys, O.rotate(P, ct, t, keys)).real
        assert np.max(np.abs(got - np.roll(a, -t))) < 2.0 ** -16


def test_mult_decrypts_to_product():
    P = O.Params(13, 5, 1, 1, 30)
    keys = O.Keys(P, 2001)
    g = np.random.default_rng(0)
    a, b = g.uniform(-1, 1, P.S), g.uniform(-1, 1, P.S)
    ca = O.encrypt_sk(P, keys, O.encode(a, P.delta, P.N), P.L, P.delta, 3001, 0)
    cb = O.encrypt_sk(P, keys, O.encode(b, P.delta, P.N), P.L, P.delta, 3001, 1)
    got = O.decrypt(P, keys, O.rescale(P, O.mul(P, ca, cb, keys))).real
    assert np.max(np.abs(got - a * b)) < 2.0 ** -(30 - 12)


# ------------------------------------------------------------ least squares, plaintext gradient
def _table2():
    rows = {}
    for line in open(os.path.join(GOLDEN, "table2_gradient_polynomials.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        rows[k] = [float(x) for x in v]
    return rows


def test_ls_fit_symmetry_and_table2_binomial():
    c8 = LR.grad_poly_binomial(8.0)
    assert abs(c8[0] - 0.5) < 1e-13 and abs(c8[2]) < 1e-13
    c16 = LR.grad_poly_binomial(16.0)
    t2 = _table2()["binomial"]
    # printed to 4 decimals (Table 2)
    assert [round(v, 4) for v in c16] == pytest.approx(t2, abs=1e-12)


def test_ls_fit_table2_hinge_magnitudes():
    h = LR.ls_fit(lambda x: np.maximum(1.0 - x, 0.0), 16.0, 4, nodes=4000)
    grad = [-h[1], -2 * h[2], -3 * h[3], -4 * h[4]]  # -d/dx of the 4-order fit
    t2 = _table2()["hinge"]
    assert round(grad[0], 4) == t2[0] and round(grad[1], 4) == t2[1]
    # magnitudes match; the printed x^2 and x^3 signs are the opposite ones
    assert round(abs(grad[2]), 4) == abs(t2[2]) and round(abs(grad[3]), 5) == abs(t2[3])


def test_ls_fit_is_limit_of_random_sampling():
    rnd = np.random.default_rng(4)
    x = rnd.uniform(-8, 8, 400000)
    V = np.stack([x ** k for k in range(4)], 1)
    mc = np.linalg.lstsq(V, 1 / (1 + np.exp(x)), rcond=None)[0]
    assert np.allclose(mc, LR.grad_poly_binomial(8.0), atol=2e-3 * np.abs(LR.grad_poly_binomial(8.0)).max())


def test_plain_gradient_finite_difference():
    X, y = synth.small_data(n=256, d=8)
    w = np.random.default_rng(2).normal(size=8) * 0.3
    n = X.shape[0]

    def loss(w):
        return np.mean(np.log1p(np.exp(-y * (X @ w))))

    # with the exact -L' = sigma(-m) in place of the polynomial
    z = y[:, None] * X
    g = (1.0 / n) * ((1 / (1 + np.exp(z @ w)))[:, None] * z).sum(0)
    fd = np.array([(loss(w - 1e-6 * e) - loss(w + 1e-6 * e)) / 2e-6 for e in np.eye(8)])
    assert np.allclose(g, fd, atol=1e-8)
    # w = 0: g = (eta/n) a0 sum_i z_i
    coef = [0.5, -0.15, 0.0, 0.0016]
    g0 = LR.lr_gradient_fp64(X, y, np.zeros(8), coef, 1.0 / n)
    assert np.allclose(g0, 0.5 * z.mean(0), rtol=0, atol=1e-15)


# ------------------------------------------------------------ scale plan and the whole step
def test_plan_consistency():
    P = O.Params(16, 20, 4, 4, 40)
    coef = [0.5, -0.15012041, 0.0, 0.00159302]
    for sW in (P.delta, 2.0 ** 44.55):
        pl = LR.plan_lr_step(P.q, 19, P.delta, sW, coef, 1 / 6000)
        for k in ("k0", "k1", "k3", "kW"):
            assert 2 ** 20 <= abs(pl[k]) < 2 ** 62
        assert pl["kB1"] == 0
        # every unrescaled term lands on the same scale sC q_{l-3}: C = A B3,
        # B1 = M Z1 (Z1's actual scale from its integer k1), k0 Z
        ql3, ql2 = float(P.q[16]), float(P.q[17])
        assert abs(pl["sA"] * pl["sB3"] / ql3 / pl["sC"] - 1) < 2 ** -40
        assert abs(pl["sM"] * (P.delta * pl["k1"] / ql2) / ql3 / pl["sC"] / coef[1] - 1) < 2 ** -20
        assert abs(P.delta * pl["k0"] / ql3 / pl["sC"] / coef[0] - 1) < 2 ** -20
    with pytest.raises(LR.LevelError):
        LR.plan_lr_step(P.q, 3, P.delta, P.delta, coef, 1 / 6000)


@pytest.mark.parametrize("n_baby", [1, 4, 16])
def test_encrypted_step_matches_fp64_gradient(n_baby):
    """Whole circuit on the small workload: decrypted g within 2^-20 of the FP64
    gradient with the same polynomial at the decrypted input weights; with
    n_baby > 1 the column sum takes baby steps over the rotated data (16 = c:
    no giant step)."""
    W = synth.WORKLOADS["small"]
    P = O.Params(W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"])
    X, y = synth.small_data()
    w0 = synth.initial_weights("small", 16, W["seed_w"])
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    keys = O.Keys(P, W["seed_keys"], rot_steps=LR.rotation_steps(c, r, LR.ROWS, n_baby))
    coef = LR.grad_poly_binomial(8.0)
    coef[0], coef[2] = 0.5, 0.0
    eta_n = 1.0 / X.shape[0]
    Z = [O.encrypt_sk(P, keys, O.encode(blocks[i], P.delta, P.N), P.L, P.delta, W["seed_enc"], i)
         for i in range(blocks.shape[0])]
    Wc = O.encrypt_sk(P, keys, O.encode(LR.pack_weights(w0, P.S, c), P.delta, P.N), P.L, P.delta,
                      W["seed_enc"], 100000)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n)
    mask = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    Zrot = LR.rotate_data(P, keys, Z, 1, n_baby) if n_baby > 1 else None
    Wn, g = LR.lr_grad_step(P, keys, Z, Wc, mask, coef, eta_n, c, r, plan=pl, Zrot=Zrot, n_baby=n_baby)
    wdec = O.decrypt(P, keys, Wc).real[:16]
    gref = LR.lr_gradient_fp64(X, y, wdec, coef, eta_n)
    gd = O.decrypt(P, keys, g).real.reshape(r, c)[:, :16]
    for row in (0, r // 2, r - 1):
        assert np.max(np.abs(gd[row] - gref)) / np.max(np.abs(gref)) < 2.0 ** -20
    wn = O.decrypt(P, keys, Wn).real.reshape(r, c)[0, :16]
    assert np.max(np.abs(wn - (wdec + gref))) / np.max(np.abs(wdec + gref)) < 2.0 ** -20


def _table2_row(name):
    return _table2()[name]


@pytest.mark.parametrize("loss,w_decay", [("hinge", 0.0), ("binomial", 0.05)])
def test_encrypted_step_other_losses_and_regulariser(loss, w_decay):
    """Table 2's hinge row (nonzero x^2 term) and an L2-regularised binomial
    step: decrypted g within 2^-20 of FP64, and W' = (1 - eta lambda) W + g."""
    W = synth.WORKLOADS["small"]
    P = O.Params(W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"])
    X, y = synth.small_data(n=512)
    w0 = synth.initial_weights("small", 16, W["seed_w"])
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    keys = O.Keys(P, W["seed_keys"], rot_steps=LR.rotation_steps(c, r))
    coef = _table2_row(loss)
    eta_n = 1.0 / X.shape[0]
    Z = [O.encrypt_sk(P, keys, O.encode(blocks[i], P.delta, P.N), P.L, P.delta, 7, i) for i in range(len(blocks))]
    Wc = O.encrypt_sk(P, keys, O.encode(LR.pack_weights(w0, P.S, c), P.delta, P.N), P.L, P.delta, 7, 999)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n, w_decay)
    assert (pl["k2"] != 0) == (coef[2] != 0)
    mask = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    Wn, g = LR.lr_grad_step(P, keys, Z, Wc, mask, coef, eta_n, c, r, plan=pl)
    wdec = O.decrypt(P, keys, Wc).real[:16]
    gref = LR.lr_gradient_fp64(X, y, wdec, coef, eta_n)
    gd = O.decrypt(P, keys, g).real[:16]
    assert np.max(np.abs(gd - gref)) / np.max(np.abs(gref)) < 2.0 ** -20
    wn = O.decrypt(P, keys, Wn).real[:16]
    want = (1.0 - w_decay) * wdec + gref
    assert np.max(np.abs(wn - want)) / np.max(np.abs(want)) < 2.0 ** -20


def test_feature_major_packing_is_the_transpose():
    X, y = synth.small_data(n=700)
    rb, c, r = LR.pack_blocks(X, y, 4096)
    fb, c2, r2 = LR.pack_blocks_features(X, y, 4096)
    assert (c, r) == (c2, r2) == (16, 256)
    for b in (0, 2):
        for i, j in ((0, 0), (3, 5), (255, 15), (17, 1)):
            assert fb[b, j * r + i] == rb[b, i * c + j]
    w = np.arange(1.0, 11.0)
    pw = LR.pack_weights_features(w, 4096, 16)
    assert pw[0 * r + 7] == 1.0 and pw[9 * r + 200] == 10.0 and pw[12 * r] == 0.0
    assert np.flatnonzero(LR.feature_mask(4096, r)).tolist() == [j * r for j in range(16)]
    st = LR.rotation_steps(c, r, LR.FEATURES)
    # the slot sums over r = 256 = 2^8 slots: index bits in groups of 2, 3, 3
    slot = [1, 2, 3, 4, 8, 12, 16, 20, 24, 28, 32, 64, 96, 128, 160, 192, 224]
    # the margin sum over c = 16 feature blocks: groups {1, 2, 3}, {4, 8, 12} times r
    assert st == sorted({t * r for t in (1, 2, 3, 4, 8, 12)} | {t * s for t in slot for s in (1, -1)})
    assert LR.slot_sum_groups(16) == [[1, 2, 3], [4, 8, 12]]
    assert LR.slot_sum_groups(256) == [slot[:3], slot[3:10], slot[10:]]
    # baby steps b r for every b < n_baby, giant steps g n_baby r for every g < c / n_baby (hoisted)
    st8 = LR.rotation_steps(c, r, LR.FEATURES, 8)
    assert {b * r for b in range(1, 8)} <= set(st8) and 8 * r in st8 and len(st8) == len(set(st8)) == 7 + 1 + 34
    st4 = LR.rotation_steps(c, r, LR.FEATURES, 4)
    assert {b * r for b in range(1, 4)} | {g * 4 * r for g in range(1, 4)} <= set(st4)
    assert len(st4) == len(set(st4)) == 3 + 3 + 34
    assert LR.giant_hoisted(c, LR.FEATURES, 4) and not LR.giant_hoisted(c, LR.FEATURES, 16)
    assert not LR.giant_hoisted(c, LR.ROWS, 4) and not LR.giant_hoisted(256, LR.FEATURES, 8)


def test_slot_sum_groups_cover_every_index_once():
    """Reading 28's grouping: for r = 2^k, summing Rot(., t) over each
    group in turn adds every rotation index i < r exactly once (each i is
    one combination of the groups' digits), the groups' sizes differ by at
    most one with the smaller groups on the low bits, and there are
    ceil(k / 3) of them."""
    for k in range(0, 12):
        r = 1 << k
        groups = LR.slot_sum_groups(r)
        assert len(groups) == -(-k // 3)
        counts = {0: 1}
        for g in groups:
            nxt = {}
            for i, m in counts.items():
                for t in [0] + g:
                    nxt[i + t] = nxt.get(i + t, 0) + m
            counts = nxt
        assert counts == {i: 1 for i in range(r)}, k
        sizes = [len(g).bit_length() for g in groups]
        assert sizes == sorted(sizes) and (not sizes or max(sizes) - min(sizes) <= 1)


def test_grouped_slot_sums_decrypt_to_the_block_sums():
    """The feature-major step's slot sum as grouped hoisted sums (reading 28)
    decrypts to the same values as the plain rotate-and-add doubling: in
    every slot, the sum of the next r slots (cyclically), within the key
    switch noise; and the replication (negative steps) the same backwards."""
    P = O.Params(*SMALL40)
    r = 64
    keys = O.Keys(P, 11, rot_steps=sorted({t * s for g in LR.slot_sum_groups(r) for t in g for s in (1, -1)}))
    g0 = np.random.default_rng(5)
    v = g0.uniform(-1, 1, P.S)
    x = O.encrypt_sk(P, keys, O.encode(v, P.delta, P.N), 3, P.delta, 9, 0)
    for sign in (1, -1):
        y = x
        for grp in LR.slot_sum_groups(r):
            y = O.rotate_sum_hoisted(P, y, [sign * t for t in grp], keys)
        got = O.decrypt(P, keys, y).real
        want = sum(np.roll(v, -sign * i) for i in range(r))
        assert np.max(np.abs(got - want)) < 1e-6, sign


def test_baby_giant_margins_equal_the_rotation_sum():
    """Sum_b Rot(Z, b r) (x) Rot(W, b r), relinearised and rescaled, decrypts to
    the sum of Rot(Z (x) W, b r) (a rotation is a ring automorphism): checked
    slot by slot against the plain sum of the rolled products."""
    P = O.Params(*SMALL40)
    r, n_baby = 256, 4
    keys = O.Keys(P, 5, rot_steps=[b * r for b in range(1, n_baby)])
    g = np.random.default_rng(3)
    z, w = g.uniform(-1, 1, P.S), g.uniform(-1, 1, P.S)
    Zc = O.encrypt_sk(P, keys, O.encode(z, P.delta, P.N), P.L, P.delta, 1, 1)
    Wc = O.encrypt_sk(P, keys, O.encode(w, P.delta, P.N), P.L, P.delta, 1, 2)
    Zr = LR.rotate_data(P, keys, [Zc], r, n_baby)[0]
    Wr = [Wc] + [O.rotate(P, Wc, b * r, keys) for b in range(1, n_baby)]
    s1 = P.delta * P.delta / P.q[P.L]
    u = LR._margin_products(P, keys, [Zc] + Zr, Wr, P.L, s1)
    want = sum(np.roll(z * w, -b * r) for b in range(n_baby))
    got = O.decrypt(P, keys, u).real
    assert u.level == P.L - 1 and np.max(np.abs(got - want)) < 2.0 ** -18


SMALL40 = (13, 5, 2, 2, 40)  # the small ring at scale 2^40 (feature-major needs a larger data scale)


def test_feature_major_refused_where_the_mask_would_lose_precision():
    W = synth.WORKLOADS["small"]
    P = O.Params(W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"])
    coef = LR.grad_poly_binomial(8.0)
    coef[0], coef[2] = 0.5, 0.0
    with pytest.raises(LR.ScaleError):
        LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, 1 / 2048, 0.0, LR.FEATURES)
    LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, 1 / 2048, 0.0, LR.ROWS)


@pytest.mark.parametrize("loss,w_decay,n_baby", [("binomial-ls", 0.0, 1), ("hinge", 0.0, 1), ("binomial-ls", 0.05, 1),
                                                 ("binomial-ls", 0.0, 4), ("hinge", 0.0, 8)])
def test_encrypted_step_feature_major(loss, w_decay, n_baby):
    """Feature-major circuit: the decrypted g, in every slot of each feature
    block, within 2^-20 of the FP64 gradient; W' = (1 - eta lambda) W + g
    likewise; 4 levels used.  n_baby > 1: margins by baby and giant steps from
    the rotated data."""
    W = synth.WORKLOADS["small"]
    P = O.Params(*SMALL40)
    X, y = synth.small_data(n=700)
    w0 = synth.initial_weights("small", 16, W["seed_w"])
    blocks, c, r = LR.pack_blocks_features(X, y, P.S)
    keys = O.Keys(P, W["seed_keys"], rot_steps=LR.rotation_steps(c, r, LR.FEATURES, n_baby))
    if loss == "hinge":
        coef = _table2_row("hinge")
    else:
        coef = LR.grad_poly_binomial(8.0)
        coef[0], coef[2] = 0.5, 0.0
    eta_n = 1.0 / X.shape[0]
    Z = [O.encrypt_sk(P, keys, O.encode(blocks[i], P.delta, P.N), P.L, P.delta, 7, i) for i in range(len(blocks))]
    Wc = O.encrypt_sk(P, keys, O.encode(LR.pack_weights_features(w0, P.S, c), P.delta, P.N), P.L, P.delta, 7, 999)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n, w_decay, LR.FEATURES)
    mask = O.encode(LR.feature_mask(P.S, r), pl["s_mask"], P.N)
    Zrot = LR.rotate_data(P, keys, Z, r, n_baby) if n_baby > 1 else None
    Wn, g = LR.lr_grad_step(P, keys, Z, Wc, mask, coef, eta_n, c, r, plan=pl, layout=LR.FEATURES, Zrot=Zrot,
                            n_baby=n_baby)
    assert Wn.level == g.level == P.L - 4
    wdec = O.decrypt(P, keys, Wc).real.reshape(c, r)[:16, 0]
    gref = LR.lr_gradient_fp64(X, y, wdec, coef, eta_n)
    gd = O.decrypt(P, keys, g).real.reshape(c, r)
    for i in (0, 1, r // 2, r - 1):
        assert np.max(np.abs(gd[:16, i] - gref)) / np.max(np.abs(gref)) < 2.0 ** -20
    # W' slot by slot against the same slot of W (each slot carries its own
    # encryption noise, about 2^-22 absolute at this scale)
    wfull = O.decrypt(P, keys, Wc).real.reshape(c, r)
    wn = O.decrypt(P, keys, Wn).real.reshape(c, r)
    for i in (0, 5, r - 1):
        want = (1.0 - w_decay) * wfull[:16, i] + gref
        assert np.max(np.abs(wn[:16, i] - want)) / np.max(np.abs(want)) < 2.0 ** -20


def test_seeded_encryption_decrypts_and_its_a_is_the_stream_in_the_evaluation_domain():
    """orc_encrypt_sk_seeded: decrypts to m within the error bound (as sk
    encryption), its uniform part's forward NTT is the (seed, index) stream's
    uniform residues in natural evaluation order, and another index gives
    another a."""
    P = O.Params(13, 5, 1, 1, 30)
    keys = O.Keys(P, 2001)
    m = synth.small_poly(4, P.N, 1 << 40)
    for level in (P.L, 1):
        ct = O.encrypt_sk_seeded(P, keys, m, level, 1.0, 77, 12)
        got = O.crt_centered(O.decrypt_residues(P, keys, ct), P.q[: level + 1])
        err = np.array(got, dtype=object) - m.astype(object)
        assert max(abs(int(v)) for v in err) <= 21
        for i in range(level + 1):
            a = np.ascontiguousarray(ct.data[1, i])
            O.lib().orc_ntt_fwd(_u64p(a), P.logN, P.q[i], P.psi[i])
            u = np.zeros(P.N, dtype=np.uint64)
            O.lib().orc_sample_uniform(77, 10, 12, i, P.q[i], P.logN, _u64p(u))
            assert np.array_equal(a, u)
    other = O.encrypt_sk_seeded(P, keys, m, 1, 1.0, 77, 13)
    assert not np.array_equal(other.data[1], O.encrypt_sk_seeded(P, keys, m, 1, 1.0, 77, 12).data[1])
