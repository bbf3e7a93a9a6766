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
                                 (14, 21, 4, 4, 40), (15, 8, 2, 2, 40), (15, 8, 4, 4, 40)])
def test_prime_chain_matches_oracle(cfg):
    assert H.params_primes(*cfg) == O.Params(*cfg).q


def test_prime_chain_rejects_bad_params():
    with pytest.raises(H.HEError):
        H.params_primes(13, 5, 1, 1, 70)


COEF = [0.5, -0.1501204134, 0.0, 0.0015930174]
HINGE = [0.5875, -0.1005, 0.0008, -0.00039]  # Table 2, hinge row as printed


@pytest.mark.parametrize("name,n", [("small", None), ("image", None), ("large", None), ("image", 128)])
@pytest.mark.parametrize("coef,w_decay", [(COEF, 0.0), (HINGE, 0.0), (COEF, 0.01)])
@pytest.mark.parametrize("layout", [LR.ROWS, LR.FEATURES])
def test_scale_plan_matches_oracle_bit_for_bit(name, n, coef, w_decay, layout):
    W = synth.WORKLOADS[name]
    q = O.Params(W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"]).q
    delta = float(2 ** W["log_delta"])
    eta_n = 1.0 / (n or W["n"])
    s_w = delta
    for level in range(W["nq"] - 1, 3, -4):
        try:
            a = LR.plan_lr_step(q, level, delta, s_w, coef, eta_n, w_decay, layout)
        except LR.ScaleError:
            # refused (feature-major at a data scale too small for n/eta): the library agrees
            assert layout == LR.FEATURES
            with pytest.raises(H.HEError) as e:
                H.plan_lr_step(q, W["nq"], level, delta, s_w, coef, eta_n, w_decay, layout)
            assert e.value.status == 4
            return
        b = H.plan_lr_step(q, W["nq"], level, delta, s_w, coef, eta_n, w_decay, layout)
        assert b["layout"] == layout
        for k in ("s1", "s_mask", "sM", "sA", "T", "sZ3", "sB3", "sC", "sZ1", "sB1", "sZ2", "s_g", "s_gsum"):
            kk = {"sM": "s_m", "sA": "s_a", "T": "t", "sZ3": "s_z3", "sB3": "s_b3", "sC": "s_c", "sZ1": "s_z1",
                  "sB1": "s_b1", "sZ2": "s_z2"}.get(k, k)
            assert a[k] == b[kk], (level, k)
        for k in ("k0", "k1", "k2", "k3", "kB1", "kW"):
            assert a[k] == b[k.lower()], (level, k)
        s_w = a["s_g"]  # the next step starts from the previous output scale


def test_term_scale_headroom_rule():
    """T: the largest power of two keeping 10 bits of headroom for the output in
    q_0, between the two coefficient-resolution bounds."""
    q = O.Params(16, 20, 4, 4, 40).q
    assert q[0].bit_length() == 60
    assert LR.term_scale(COEF, q[0], 1 / 6000) == 2.0 ** 36   # 2^49 / 6000 -> 2^36
    assert LR.term_scale(COEF, q[0], 1 / 128) == 2.0 ** 40     # capped: T a3 in [2^30, 2^31)
    assert LR.term_scale(COEF, q[0], 2.0 ** -20) == 2.0 ** 32  # floored: T a3 in [2^22, 2^23)
    for eta_n in (1 / 6000, 1 / 128, 2.0 ** -20):
        pl = H.plan_lr_step(q, 20, 19, 2.0 ** 40, 2.0 ** 40, COEF, eta_n)
        assert pl["t"] == LR.term_scale(COEF, q[0], eta_n)
    # feature-major: the mask's plaintext scale stays >= 2^34
    for eta_n, t in ((1 / 6000, 2.0 ** 33), (1 / 128, 2.0 ** 38)):
        pl = H.plan_lr_step(q, 20, 19, 2.0 ** 40, 2.0 ** 40, COEF, eta_n, 0.0, H.LAYOUT_FEATURES)
        assert pl["t"] == t and pl["s_mask"] >= 2.0 ** 34
        assert abs(pl["s_g"] / 2.0 ** 40 - 1) < 1e-12  # W' returns at the data's scale


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
    with pytest.raises(H.HEError) as e:
        H.plan_lr_step(q, 5, 4, 2.0 ** 30, 2.0 ** 30, COEF, 1 / 2048, 0.0, 2)
    assert e.value.status == 1  # HE_EINVAL: unknown layout


def test_packing_matches_oracle_layout():
    X, y = synth.small_data(n=300, d=11)
    a, c1, r1 = H.pack_blocks(X, y, 4096)
    b, c2, r2 = LR.pack_blocks(X, y, 4096)
    assert (c1, r1) == (c2, r2) == (16, 256)
    assert np.array_equal(a, b)
    w = np.arange(11.0)
    assert np.array_equal(H.pack_weights(w, 4096, 16), LR.pack_weights(w, 4096, 16))
    assert np.array_equal(H.column0_mask(4096, 16), LR.column_mask(4096, 16))
    a, _, _ = H.pack_blocks(X, y, 4096, H.LAYOUT_FEATURES)
    b, _, _ = LR.pack_blocks_features(X, y, 4096)
    assert np.array_equal(a, b)
    assert np.array_equal(H.pack_weights(w, 4096, 16, H.LAYOUT_FEATURES), LR.pack_weights_features(w, 4096, 16))
    assert np.array_equal(H.step_mask(4096, 16, H.LAYOUT_FEATURES), LR.feature_mask(4096, 256))
    assert np.array_equal(H.step_mask(4096, 16), LR.column_mask(4096, 16))
    for lay in (LR.ROWS, LR.FEATURES):
        for nb in (1, 2, 4, 8, 16):
            assert sorted(H.rotation_steps(16, 256, lay, nb)) == sorted(LR.rotation_steps(16, 256, lay, nb))
            assert sorted(H.rotation_steps(256, 128, lay, nb)) == sorted(LR.rotation_steps(256, 128, lay, nb))
        assert np.array_equal(H.unpack_weights(H.pack_weights(w, 4096, 16, lay), 16, 11, lay), w)


@pytest.mark.parametrize("name", ["small", "image", "large"])
@pytest.mark.parametrize("coef", [COEF, HINGE, [0.1, 0.2, 0.3, 0.0]])
def test_inference_plan_matches_oracle_bit_for_bit(name, coef):
    W = synth.WORKLOADS[name]
    q = O.Params(W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"]).q
    delta = float(2 ** W["log_delta"])
    for level in range(W["nq"] - 1, 2, -3):
        for s_w in (delta, delta * 1.37):
            a = LR.plan_lr_infer(q, level, delta, s_w, coef)
            b = H.plan_lr_infer(q, W["nq"], level, delta, s_w, coef)
            assert (b["level_in"], b["level_out"]) == (level, level - 3)
            for k in ("s_u", "s_u2", "s_h", "s_p", "k3", "k2c", "k1", "k0c"):
                assert a[k] == b[k], (level, k)
    with pytest.raises(H.HEError) as e:
        H.plan_lr_infer(q, W["nq"], 2, delta, delta, coef)
    assert e.value.status == 3
    with pytest.raises(LR.LevelError):
        LR.plan_lr_infer(q, 2, delta, delta, coef)


def test_noalloc_scratch_size_matches_header():
    import re
    src = open(os.path.join(ROOT, "include", "he.h")).read()
    m = re.search(r"#define HE_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == H.NOALLOC_SCRATCH_BYTES


def test_kernel_trace_names_and_argument_checks():
    """Every kernel kind of the trace has a distinct name; out-of-range kinds
    and a missing context are refused without a device call."""
    names = [H._lib.he_kernel_kind_name(k).decode() for k in range(H.K_COUNT)]
    assert len(set(names)) == H.K_COUNT and "?" not in names
    assert H._lib.he_kernel_kind_name(H.K_COUNT).decode() == "?"
    assert H._lib.he_kernel_kind_name(-1).decode() == "?"
    assert H._lib.he_ctx_trace(None, 1) != 0
    n = H.ctypes.c_int()
    assert H._lib.he_ctx_trace_read(None, None, 0, H.ctypes.byref(n)) != 0
