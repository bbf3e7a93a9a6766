"""Exact pins of the oracle's centred fast basis conversion (ModUp and
ModDown of the hybrid key switch) and of its ternary sampler.

The conversion is the reading the design notes state: each digit
y_i = [x qhat_i^{-1}]_{q_i} enters as its centred representative, so the
converted integer is v = sum_i y_i qhat_i with every |y_i| < q_i / 2.  Three
independent pins:
  * brute force on primes below 2^9: y_i found by searching the centred range
    for the integer with y_i qhat_i = x (mod q_i), no modular inverse, edge
    digits (0, 1, (q-1)/2, (q+1)/2, q-1) included;
  * on the 40/60-bit chains, the output's big integer is checked to be such a
    sum (its centred digits rebuild it exactly, which an uncentred sum with
    any digit above q/2 does not);
  * oddness: negating the input negates the output (true of the centred
    conversion, false of the uncentred one since sum_i q_i qhat_i = alpha Q_D).
A planted uncentred conversion (the oracle's test switch) fails all three.
"""
import ctypes
import math
import random

import numpy as np
import pytest

from oracle import ckks as O

TINY = [17, 97, 113, 193, 241, 257]  # primes 1 mod 16 (N = 8): q_0..q_3, then two special primes


def _u(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def tiny():
    return O.Params.custom(3, TINY, 4, 2, 2)


def chain(name):
    """Real prime chains on a ring of 16 coefficients (every prime is 1 mod 2^17)."""
    cfg = {"image": (16, 20, 4, 4, 40), "large": (16, 24, 6, 6, 40), "small": (13, 5, 1, 1, 30)}[name]
    P = O.Params(*cfg)
    return O.Params.custom(4, P.q, cfg[1], cfg[2], cfg[3], cfg[4])


def centred(v, q):
    v %= q
    return v - q if v > q // 2 else v


def crt(res, primes):
    Q = math.prod(primes)
    x = sum(int(r) * (Q // q) * pow(Q // q, -1, q) for r, q in zip(res, primes)) % Q
    return x - Q if x > Q // 2 else x


def brute_digit(x, q, qhat):
    """The integer y with |y| < q/2 and y * qhat = x (mod q), by search."""
    hits = [y for y in range(-(q // 2), q // 2 + 1) if (y * qhat - x) % q == 0]
    assert len(hits) == 1
    return hits[0]


def edge_inputs(primes, count, rnd):
    """Integers x mod prod(primes) whose digits [x qhat_i^{-1}]_{q_i} sweep the
    edge values and random ones."""
    Q = math.prod(primes)
    xs = []
    for k in range(count):
        x = 0
        for i, q in enumerate(primes):
            edges = [0, 1, (q - 1) // 2, (q + 1) // 2, q - 1]
            u = edges[(k + 2 * i) % 5] if k < 10 else rnd.randrange(q)
            qh = Q // q
            x += u * qh  # digit i of x is u: x qhat_i^{-1} = u (mod q_i)
        xs.append(x % Q)
    return xs


def modup(P, level, j, xs_full):
    """orc_modup on integer coefficients given on the full level basis."""
    N = P.N
    d = np.array([[x % q for x in xs_full] for q in P.q[: level + 1]], dtype=np.uint64)
    ext = np.zeros((level + 1 + P.nk, N), dtype=np.uint64)
    O.lib().orc_modup(P.cp, level, j, _u(d), _u(ext))
    return ext


def moddown(P, level, c):
    out = np.zeros((level + 1, P.N), dtype=np.uint64)
    O.lib().orc_moddown(P.cp, level, _u(np.ascontiguousarray(c)), _u(out))
    return out


# ------------------------------------------------------------------ checks (count mismatches)
def modup_brute_mismatches(rnd):
    P = tiny()
    level, bad = 3, 0
    basis = P.q[: level + 1] + P.special()
    for j in range(P.ndigits(level)):
        D = P.q[j * P.alpha:(j + 1) * P.alpha]
        QD = math.prod(D)
        for rep in range(3):
            xd = edge_inputs(D, P.N, rnd) if rep < 2 else [rnd.randrange(QD) for _ in range(P.N)]
            # the input's other limbs are arbitrary: only the digit's residues are converted
            xs = [x + QD * rnd.randrange(1000) for x in xd]
            ext = modup(P, level, j, xs)
            for k in range(P.N):
                v = sum(brute_digit(xs[k], q, QD // q) * (QD // q) for q in D)
                for t, p in enumerate(basis):
                    want = xs[k] % p if p in D else v % p
                    bad += int(ext[t][k]) != want
    return bad


def moddown_brute_mismatches(rnd):
    P = tiny()
    level, bad = 3, 0
    basis = P.q[: level + 1] + P.special()
    Pm = math.prod(P.special())
    QP = math.prod(basis)
    for rep in range(3):
        xP = edge_inputs(P.special(), P.N, rnd) if rep < 2 else [rnd.randrange(Pm) for _ in range(P.N)]
        xs = [(x + Pm * rnd.randrange(QP // Pm)) % QP for x in xP]
        c = np.array([[x % p for x in xs] for p in basis], dtype=np.uint64)
        out = moddown(P, level, c)
        for k in range(P.N):
            v = sum(brute_digit(xs[k], p, Pm // p) * (Pm // p) for p in P.special())
            assert (xs[k] - v) % Pm == 0
            y = (xs[k] - v) // Pm
            for i, q in enumerate(P.q[: level + 1]):
                bad += int(out[i][k]) != y % q
    return bad


def is_centred_sum(v, primes):
    """v = sum_i y_i qhat_i with every |y_i| < q_i/2 (the digits are unique)."""
    Q = math.prod(primes)
    return v == sum(centred(v * pow(Q // q, -1, q), q) * (Q // q) for q in primes)


def modup_char_mismatches(name, rnd):
    P = chain(name)
    level, bad = P.L, 0
    basis = P.q[: level + 1] + P.special()
    for j in range(P.ndigits(level)):
        D = P.q[j * P.alpha:min((j + 1) * P.alpha, level + 1)]
        QD = math.prod(D)
        xs = [rnd.randrange(math.prod(P.q[: level + 1])) for _ in range(P.N)]
        ext = modup(P, level, j, xs)
        for k in range(P.N):
            # the digit's residues are the input's; the whole output is one integer v
            v = crt([x if p not in D else xs[k] % p for p, x in zip(basis, ext[:, k])], basis)
            ok = all(int(ext[t][k]) == xs[k] % p for t, p in enumerate(basis) if p in D)
            ok = ok and (v - xs[k]) % QD == 0 and abs(v) < len(D) * QD // 2 and is_centred_sum(v, D)
            bad += not ok
    return bad


def moddown_char_mismatches(name, rnd):
    P = chain(name)
    level, bad = P.L, 0
    basis = P.q[: level + 1] + P.special()
    Q, Pm = math.prod(P.q[: level + 1]), math.prod(P.special())
    xs = [rnd.randrange(-(Q * Pm) // 4, (Q * Pm) // 4) for _ in range(P.N)]
    c = np.array([[x % p for x in xs] for p in basis], dtype=np.uint64)
    out = moddown(P, level, c)
    for k in range(P.N):
        y = crt(out[:, k], P.q[: level + 1])
        v = xs[k] - y * Pm  # the converted value the ModDown subtracted
        bad += not (abs(v) < P.nk * Pm // 2 and is_centred_sum(v, P.special()))
    return bad


def oddness_mismatches(rnd):
    bad = 0
    for P in (tiny(), chain("image")):
        level = P.L
        basis = P.q[: level + 1] + P.special()
        Qf = math.prod(P.q[: level + 1])
        xs = [rnd.randrange(Qf) for _ in range(P.N)]
        for j in range(P.ndigits(level)):
            a, b = modup(P, level, j, xs), modup(P, level, j, [(-x) % Qf for x in xs])
            for t, p in enumerate(basis):
                bad += sum(int(b[t][k]) != (-int(a[t][k])) % p for k in range(P.N))
        c = np.array([[rnd.randrange(p) for _ in range(P.N)] for p in basis], dtype=np.uint64)
        cn = np.array([[(-int(v)) % p for v in row] for p, row in zip(basis, c)], dtype=np.uint64)
        a, b = moddown(P, level, c), moddown(P, level, cn)
        for i, q in enumerate(P.q[: level + 1]):
            bad += sum(int(b[i][k]) != (-int(a[i][k])) % q for k in range(P.N))
    return bad


# ------------------------------------------------------------------ tests
def test_modup_equals_brute_force_centred_conversion():
    assert modup_brute_mismatches(random.Random(1)) == 0


def test_moddown_equals_brute_force_centred_division():
    assert moddown_brute_mismatches(random.Random(2)) == 0


@pytest.mark.parametrize("name", ["small", "image", "large"])
def test_modup_output_is_a_centred_digit_sum(name):
    assert modup_char_mismatches(name, random.Random(3)) == 0


@pytest.mark.parametrize("name", ["small", "image", "large"])
def test_moddown_subtracts_a_centred_digit_sum(name):
    assert moddown_char_mismatches(name, random.Random(4)) == 0


def test_conversions_are_odd():
    assert oddness_mismatches(random.Random(5)) == 0


def test_planted_uncentred_conversion_fails_every_pin():
    O.lib().orc_set_conv_centring(0)
    try:
        assert modup_brute_mismatches(random.Random(1)) > 0
        assert moddown_brute_mismatches(random.Random(2)) > 0
        assert modup_char_mismatches("image", random.Random(3)) > 0
        assert moddown_char_mismatches("image", random.Random(4)) > 0
        assert oddness_mismatches(random.Random(5)) > 0
    finally:
        O.lib().orc_set_conv_centring(1)
    assert modup_brute_mismatches(random.Random(1)) == 0


def test_ternary_sampler_distribution():
    """orc_sample_ternary (the pk-encryption mask v): P(0) = 1/2,
    P(+1) = P(-1) = 1/4, independent across coefficients and streams."""
    N = 1 << 16
    s = np.zeros(N, dtype=np.int64)
    t = np.zeros(N, dtype=np.int64)
    ip = ctypes.POINTER(ctypes.c_int64)
    O.lib().orc_sample_ternary(9, 8, 0, 0, 16, s.ctypes.data_as(ip))
    O.lib().orc_sample_ternary(9, 8, 1, 0, 16, t.ctypes.data_as(ip))
    assert set(np.unique(s)) == {-1, 0, 1}
    n0, n1, nm = (s == 0).sum(), (s == 1).sum(), (s == -1).sum()
    # five standard deviations of the binomial counts
    assert abs(n0 - N / 2) < 5 * math.sqrt(N / 4)
    assert abs(n1 - N / 4) < 5 * math.sqrt(N * 3 / 16) and abs(nm - N / 4) < 5 * math.sqrt(N * 3 / 16)
    # neighbours and the second stream are independent: the joint zero rate is 1/4
    both = ((s[:-1] == 0) & (s[1:] == 0)).sum()
    assert abs(both - (N - 1) / 4) < 5 * math.sqrt(N * 3 / 16)
    assert abs(((s == 0) & (t == 0)).sum() - N / 4) < 5 * math.sqrt(N * 3 / 16)
    assert abs(float(np.mean(s * t))) < 5 / math.sqrt(N) and abs(float(np.mean(s))) < 5 * math.sqrt(0.5 / N)
