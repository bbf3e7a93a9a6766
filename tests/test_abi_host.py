"""Host-only checks of the C-ABI library: it loads, exports every symbol that
include/he.h declares, and its pure-host parts (prime chain, scale plan,
packing) agree with the oracle.  No device call is made."""
import math
import os
import re

import numpy as np
import pytest

from oracle import ckks as O
from oracle import lr as LR
from paper_2006_10091_amd import he as H
from paper_2006_10091_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "he.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_symbols()
    assert len(names) >= 30
    for n in names:
        assert hasattr(H._lib, n), n
    assert set(names) == set(H.EXPORTS)


@pytest.mark.parametrize("cfg", [(13, 5, 1, 1, 30), (16, 20, 4, 4, 40), (16, 24, 6, 6, 40),
                                 (14, 21, 4, 4, 40), (15, 8, 2, 2, 40)])
def test_prime_chain_matches_oracle(cfg):
    assert H.params_primes(*cfg) == O.Params(*cfg).q


def test_prime_chain_rejects_bad_params():
    with pytest.raises(H.HEError):
        H.params_primes(13, 5, 1, 1, 70)


COEF = [0.5, -0.1501204134, 0.0, 0.0015930174]
HINGE = [0.5875, -0.1005, 0.0008, -0.00039]  # Table 2, hinge row as printed


@pytest.mark.parametrize("name", ["small", "image", "large"])
@pytest.mark.parametrize("coef,w_decay", [(COEF, 0.0), (HINGE, 0.0), (COEF, 0.01)])
def test_scale_plan_matches_oracle_bit_for_bit(name, coef, w_decay):
    W = synth.WORKLOADS[name]
    q = O.Params(W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"]).q
    delta = float(2 ** W["log_delta"])
    eta_n = 1.0 / W["n"]
    s_w = delta
    for level in range(W["nq"] - 1, 3, -4):
        a = LR.plan_lr_step(q, level, delta, s_w, coef, eta_n, w_decay)
        b = H.plan_lr_step(q, W["nq"], level, delta, s_w, coef, eta_n, w_decay)
        for k in ("s1", "s_mask", "sM", "sA", "T", "sZ3", "sB3", "sC", "sZ1", "sB1", "sZ2", "s_g"):
            kk = {"sM": "s_m", "sA": "s_a", "T": "t", "sZ3": "s_z3", "sB3": "s_b3", "sC": "s_c", "sZ1": "s_z1",
                  "sB1": "s_b1", "sZ2": "s_z2"}.get(k, k)
            assert a[k] == b[kk], (level, k)
        for k in ("k0", "k1", "k2", "k3", "kB1", "kW"):
            assert a[k] == b[k.lower()], (level, k)
        s_w = a["s_g"]  # the next step starts from the previous output scale


def test_scale_plan_errors():
    q = O.Params(13, 5, 1, 1, 30).q
    with pytest.raises(H.HEError) as e:
        H.plan_lr_step(q, 5, 3, 2.0 ** 30, 2.0 ** 30, COEF, 1 / 2048)
    assert e.value.status == 3  # HE_ELEVEL
    with pytest.raises(H.HEError) as e:
        H.plan_lr_step(q, 5, 4, 2.0 ** 30, 2.0 ** 30, [0.5, 0.0, 0.0, 0.0], 1 / 2048)
    assert e.value.status == 4  # HE_ESCALE: no a1..a3
    with pytest.raises(H.HEError) as e:
        H.plan_lr_step(q, 5, 4, 2.0 ** 30, 2.0 ** 30, COEF, 1 / 2048, 1.0)
    assert e.value.status == 4  # HE_ESCALE: w_decay outside [0, 1)
    with pytest.raises(H.HEError) as e:
        H.plan_lr_step(q, 5, 4, 2.0 ** 30, 1.0, COEF, 1 / 2048)
    assert e.value.status == 4  # HE_ESCALE: constant out of range


def test_packing_matches_oracle_layout():
    X, y = synth.small_data(n=300, d=11)
    a, c1, r1 = H.pack_blocks(X, y, 4096)
    b, c2, r2 = LR.pack_blocks(X, y, 4096)
    assert (c1, r1) == (c2, r2) == (16, 256)
    assert np.array_equal(a, b)
    w = np.arange(11.0)
    assert np.array_equal(H.pack_weights(w, 4096, 16), LR.pack_weights(w, 4096, 16))
    assert np.array_equal(H.column0_mask(4096, 16), LR.column_mask(4096, 16))
