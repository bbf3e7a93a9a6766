"""Pins of the oracle's encrypted inference (the serving call): the constant
addition and the polynomial applied to the margins, against the FP64 values
p(w.z_i) of the same samples."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import lr as LR
from paper_2006_10091_amd import synth

SMALL40 = (13, 5, 2, 2, 40)


def test_add_const_adds_to_every_slot():
    P = O.Params(*SMALL40)
    keys = O.Keys(P, 3)
    z = np.random.default_rng(1).uniform(-1, 1, P.S)
    ct = O.encrypt_sk(P, keys, O.encode(z, P.delta, P.N), P.L, P.delta, 1, 1)
    k = -123456789012
    got = O.decrypt(P, keys, O.add_const(P, ct, k)).real
    base = O.decrypt(P, keys, ct).real
    # exact up to the FP64 decode: k / scale in every slot
    assert np.max(np.abs(got - base - k / P.delta)) < 2.0 ** -30
    # the residues differ in coefficient 0 only, by k mod q_i
    d = O.add_const(P, ct, k).data.astype(object) - ct.data.astype(object)
    for i, q in enumerate(P.q[: P.L + 1]):
        assert int(d[0, i, 0]) % q == k % q and not np.any(d[0, i, 1:]) and not np.any(d[1, i])


@pytest.mark.parametrize("layout", [LR.ROWS, LR.FEATURES])
@pytest.mark.parametrize("loss", ["ls", "hinge"])
def test_inference_decrypts_to_the_polynomial_of_the_margins(layout, loss):
    P = O.Params(*SMALL40)
    X, y = synth.small_data(n=300)
    w = np.random.default_rng(4).uniform(-0.3, 0.3, 16)
    pack = LR.pack_blocks_features if layout == LR.FEATURES else LR.pack_blocks
    pw = LR.pack_weights_features if layout == LR.FEATURES else LR.pack_weights
    blocks, c, r = pack(X, y, P.S)
    unit = r if layout == LR.FEATURES else 1
    keys = O.Keys(P, 5, rot_steps=[t * unit for g in LR.slot_sum_groups(c) for t in g])  # grouped margin sum
    if loss == "hinge":
        coef = [0.5875, -0.1005, 0.0008, -0.00039]  # Table 2's hinge row (nonzero m^2 term)
    else:
        coef = list(LR.grad_poly_binomial(8.0))
        coef[0], coef[2] = 0.5, 0.0
    Z = [O.encrypt_sk(P, keys, O.encode(blocks[i], P.delta, P.N), P.L, P.delta, 2, i) for i in range(len(blocks))]
    Wc = O.encrypt_sk(P, keys, O.encode(pw(w, P.S, c), P.delta, P.N), P.L, P.delta, 2, 99)
    out = LR.lr_infer(P, keys, Z, Wc, c, r, layout, coef)
    pl = LR.plan_lr_infer(P.q, P.L, P.delta, P.delta, coef)
    assert out[0].level == P.L - 3 and out[0].scale == pl["s_p"]
    m = (y[:, None] * X) @ w
    want = coef[0] + coef[1] * m + coef[2] * m * m + coef[3] * m ** 3
    for b in range(len(blocks)):
        dec = O.decrypt(P, keys, out[b]).real
        grid = dec.reshape(c, r).T if layout == LR.FEATURES else dec.reshape(r, c)
        rows = min(r, X.shape[0] - b * r)
        assert np.max(np.abs(grid[:rows, 0] - want[b * r: b * r + rows])) < 2.0 ** -20
    # coef None: the margins themselves
    mg = LR.lr_infer(P, keys, Z, Wc, c, r, layout)
    dec = O.decrypt(P, keys, mg[0]).real
    grid = dec.reshape(c, r).T if layout == LR.FEATURES else dec.reshape(r, c)
    assert np.max(np.abs(grid[:, 0] - m[:r])) < 2.0 ** -20
