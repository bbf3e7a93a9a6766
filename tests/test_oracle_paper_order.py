"""The oracle's step (lr_grad_step: baby steps, a hoisted giant sum, products
left unrelinearised and terms summed before one relinearisation) pinned
against the same step in the order of Sec. 3 and Sec. 4 (lr_grad_step_plain:
every product relinearised and rescaled, every slot sum a chain of
rotate-and-adds, per-block rescales).

Both circuits use one scale plan, so their decrypted outputs compute the same
slots and differ only by where they round.  The bound per case is stated
below from that noise: each circuit alone sits about 2^-22 (scale 2^30, and
feature-major, whose gradient mask limits it) or 2^-30 (row-major at scale
2^40) from the FP64 gradient, and the two noises are independent.  Every
slot of g and W' is compared, not only the data slots.
"""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import lr as LR
from paper_2006_10091_amd import synth

SMALL = (13, 5, 1, 1, 30)
SMALL40 = (13, 5, 2, 2, 40)

# (ring, layout, n_baby, loss, w_decay, n, log2 bound on |g_fused - g_plain| / max |g|)
CASES = [
    (SMALL, LR.ROWS, 1, "ls", 0.0, 700, -22.0),
    (SMALL, LR.ROWS, 4, "ls", 0.0, 700, -22.0),
    (SMALL, LR.ROWS, 16, "ls", 0.0, 700, -22.0),
    (SMALL40, LR.ROWS, 1, "ls", 0.0, 700, -28.0),
    (SMALL40, LR.ROWS, 16, "hinge", 0.0, 700, -28.0),
    (SMALL40, LR.ROWS, 4, "ls", 0.05, 300, -28.0),
    (SMALL40, LR.FEATURES, 1, "ls", 0.0, 700, -21.0),
    (SMALL40, LR.FEATURES, 2, "ls", 0.0, 256, -21.0),
    (SMALL40, LR.FEATURES, 4, "hinge", 0.0, 700, -21.0),
    (SMALL40, LR.FEATURES, 16, "ls", 0.05, 700, -21.0),
]


def _coef(loss):
    if loss == "hinge":
        # Table 2's hinge row (nonzero x^2 term), as tests/golden holds it
        rows = {}
        import os
        for line in open(os.path.join(os.path.dirname(__file__), "golden", "table2_gradient_polynomials.txt")):
            if line.startswith("#") or not line.strip():
                continue
            name, *v = line.split()
            rows[name] = [float(x) for x in v]
        return rows["hinge"]
    c = LR.grad_poly_binomial(8.0)
    c[0], c[2] = 0.5, 0.0
    return c


@pytest.mark.parametrize("ring,layout,n_baby,loss,w_decay,n,bound", CASES)
def test_fused_step_matches_paper_order_step(ring, layout, n_baby, loss, w_decay, n, bound):
    W = synth.WORKLOADS["small"]
    P = O.Params(*ring)
    X, y = synth.small_data(n=n)
    w0 = synth.initial_weights("small", 16, W["seed_w"])
    pack = LR.pack_blocks_features if layout == LR.FEATURES else LR.pack_blocks
    pw = LR.pack_weights_features if layout == LR.FEATURES else LR.pack_weights
    blocks, c, r = pack(X, y, P.S)
    steps = sorted(set(LR.rotation_steps(c, r, layout, n_baby)) | set(LR.rotation_steps(c, r, layout, 1)))
    keys = O.Keys(P, W["seed_keys"], rot_steps=steps)
    coef = _coef(loss)
    eta_n = 1.0 / n
    Z = [O.encrypt_sk(P, keys, O.encode(blocks[i], P.delta, P.N), P.L, P.delta, 7, i) for i in range(len(blocks))]
    Wc = O.encrypt_sk(P, keys, O.encode(pw(w0, P.S, c), P.delta, P.N), P.L, P.delta, 7, 999)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n, w_decay, layout)
    msk = LR.feature_mask(P.S, r) if layout == LR.FEATURES else LR.column_mask(P.S, c)
    mask = O.encode(msk, pl["s_mask"], P.N)
    unit = r if layout == LR.FEATURES else 1
    Zrot = LR.rotate_data(P, keys, Z, unit, n_baby) if n_baby > 1 else None
    Wf, gf = LR.lr_grad_step(P, keys, Z, Wc, mask, coef, eta_n, c, r, plan=pl, w_decay=w_decay, layout=layout,
                             Zrot=Zrot, n_baby=n_baby)
    Wp, gp = LR.lr_grad_step_plain(P, keys, Z, Wc, mask, coef, eta_n, c, r, plan=pl, w_decay=w_decay, layout=layout)
    assert (Wf.level, gf.level, Wf.scale, gf.scale) == (Wp.level, gp.level, Wp.scale, gp.scale) == \
        (P.L - 4, P.L - 4, pl["s_g"], pl["s_g"])
    df, dp = O.decrypt(P, keys, gf).real, O.decrypt(P, keys, gp).real
    wf, wp = O.decrypt(P, keys, Wf).real, O.decrypt(P, keys, Wp).real
    gmax = np.max(np.abs(dp))
    assert gmax > 0
    assert np.max(np.abs(df - dp)) / gmax < 2.0 ** bound
    assert np.max(np.abs(wf - wp)) / np.max(np.abs(wp)) < 2.0 ** bound
    # the paper-order step itself against FP64 (the same check the fused one has)
    wdec = O.decrypt(P, keys, Wc).real
    wd = wdec.reshape(c, r)[:16, 0] if layout == LR.FEATURES else wdec[:16]
    gref = LR.lr_gradient_fp64(X, y, wd, coef, eta_n)
    gd = dp.reshape(c, r)[:16, :].T if layout == LR.FEATURES else dp.reshape(r, c)[:, :16]
    assert np.max(np.abs(gd - gref)) / np.max(np.abs(gref)) < 2.0 ** -20
