"""The lazy FP64 NTT arithmetic of the GPU transforms (primes below 2^46
forward, 2^42 inverse), checked on the host against exact 128-bit
arithmetic: operation extremes of every stage's range, the signed 51-bit
intermediate between the passes, and whole 2^16-point transforms on
worst-case inputs (all q-1, alternating 0/q-1, a single q-1, halves at
(q-1)/2, random q-1/(q+1)/2) residue for residue.  Covers every prime of the
chains the tests and the bench use, plus the largest admissible primes below
2^46 and 2^42, where the range arguments are tightest."""
import os
import shutil
import subprocess

import pytest

from paper_2006_10091_amd import he as H

HERE = os.path.dirname(os.path.abspath(__file__))
CHAINS = {
    "small": (13, 5, 1, 1, 30), "small40": (13, 5, 2, 2, 40), "image": (16, 20, 4, 4, 40),
    "large": (16, 24, 6, 6, 40), "batch": (16, 21, 4, 4, 40), "serve": (16, 8, 2, 2, 40),
}


def _is_prime(n):
    if n < 2:
        return False
    bases = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    for p in bases:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in bases:
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


def _largest_below(bits):
    m = 1 << 17
    c = ((1 << bits) - 1) // m * m + 1
    while not _is_prime(c):
        c -= m
    return c


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("ntt") / "ntt_lazy_check")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", exe, os.path.join(HERE, "ntt_lazy_check.c"), "-lm"],
                   check=True)
    return exe


def test_lazy_ntt_rule_on_every_chain_prime(checker):
    primes = set()
    for cfg in CHAINS.values():
        primes |= {q for q in H.params_primes(*cfg) if q < 2 ** 46}
    primes |= {_largest_below(46), _largest_below(42)}
    r = subprocess.run([checker, ",".join(map(str, sorted(primes))), "16"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    assert "bad 0" in r.stdout and int(r.stdout.split()[1]) == len(primes)
