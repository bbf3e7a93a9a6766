"""The FP64 basis-conversion rule of the key switch (ModUp and ModDown for
target primes below 2^46), checked on the host against exact 128-bit
arithmetic over every prime chain the tests and the bench use.  The GPU
parity tests check the kernels themselves bit for bit against the oracle;
this test covers the rule's range argument, including edge residues that
random ciphertexts rarely produce."""
import os
import shutil
import subprocess

import pytest

from paper_2006_10091_amd import he as H

HERE = os.path.dirname(os.path.abspath(__file__))
CHAINS = {
    "small": (13, 5, 1, 1, 30), "small40": (13, 5, 2, 2, 40), "image": (16, 20, 4, 4, 40),
    "large": (16, 24, 6, 6, 40), "batch": (16, 21, 4, 4, 40), "serve": (16, 8, 2, 2, 40),
    "refresh1": (16, 5, 1, 1, 40), "wide digits": (16, 24, 2, 12, 40),
}


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("conv") / "fp64_conv_check")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", exe, os.path.join(HERE, "fp64_conv_check.c"), "-lm"],
                   check=True)
    return exe


@pytest.mark.parametrize("name", sorted(CHAINS))
def test_fp64_conversion_matches_exact(checker, name):
    lg, nq, nk, al, ld = CHAINS[name]
    q = H.params_primes(lg, nq, nk, al, ld)
    cq, sp = q[:nq], q[nq:]
    jobs = [(cq[j * al:(j + 1) * al], [t for t in q if t not in cq[j * al:(j + 1) * al]])
            for j in range((nq + al - 1) // al)]  # ModUp: each digit to every other prime
    jobs.append((sp, cq))  # ModDown: the special primes to the ciphertext primes
    n_fp = 0
    for src, tgt in jobs:
        r = subprocess.run([checker, ",".join(map(str, src)), ",".join(map(str, tgt)), "3000"],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stdout
        n_fp += int(r.stdout.split("(fp ")[1].split(")")[0])
    assert n_fp > 0  # the FP64 path is exercised on every chain
