"""he_lr_grad_step_multi: several requests' gradient steps with their
once-per-step tails batched.  Each request's W' and g equal its own
he_lr_grad_step bit for bit (both packings, shard sizes, weights and eta/n
differing per request, in both modes), one request is checked against the
oracle directly, and the errors come before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ckks as O  # noqa: E402
from oracle import lr as LR  # noqa: E402
from paper_2006_10091_amd import he as H  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402

SMALL40 = (13, 5, 2, 2, 40)
SERVE = (15, 8, 4, 4, 40)  # the serving chain (paper_2006_10091_amd.serve.CHAIN)
COEF = [0.5, -0.1501204134, 0.0, 0.0015930174]


def _requests(ctx, keys, layout, sizes, seed, d=16):
    fm = layout == H.LAYOUT_FEATURES
    L = ctx.n_q - 1
    reqs, raw = [], []
    for i, n in enumerate(sizes):
        g = synth.rng(seed + i)
        X = g.uniform(0.0, 1.0, size=(n, d))
        y = np.where(g.uniform(size=n) < 0.5, 1.0, -1.0)
        blocks, c, r = (LR.pack_blocks_features if fm else LR.pack_blocks)(X, y, ctx.S)
        Z = ctx.ct_block(len(blocks), L)
        for b in range(len(blocks)):
            ctx.encrypt(ctx.pt_load(ctx.encode(blocks[b], ctx.delta), L, ctx.delta), keys, seed, 100 * i + b, out=Z[b])
        w = g.uniform(-0.1, 0.1, size=d)
        pw = (LR.pack_weights_features if fm else LR.pack_weights)(w, ctx.S, c)
        mw = ctx.encode(pw, ctx.delta)
        W = ctx.encrypt(ctx.pt_load(mw, L, ctx.delta), keys, seed, 100 * i + 99)
        pl = ctx.plan_lr_step(L, ctx.delta, ctx.delta, COEF, 1.0 / n, layout=layout)
        msk = LR.feature_mask(ctx.S, r) if fm else LR.column_mask(ctx.S, c)
        mm = ctx.encode(msk, pl["s_mask"])
        mask = ctx.pt_load(mm, H.mask_level(L, layout), pl["s_mask"])
        reqs.append(dict(Z=Z, W=W, mask=mask, coef=COEF, eta_over_n=1.0 / n))
        raw.append(dict(blocks=blocks, mw=mw, mm=mm, pl=pl, n=n, c=c, r=r))
    return reqs, raw


@pytest.mark.parametrize("cfg,layout,sizes", [
    (SMALL40, H.LAYOUT_ROWS, (300, 700, 1500, 256)),
    (SMALL40, H.LAYOUT_FEATURES, (300, 700, 1500)),
    (SERVE, H.LAYOUT_FEATURES, (600, 2500, 4000, 900, 5000)),
    (SERVE, H.LAYOUT_ROWS, (600, 2500, 1200)),
])
def test_multi_step_equals_single_steps(cfg, layout, sizes):
    ctx = H.Context(*cfg)
    d = 16 if cfg == SMALL40 else 24
    c = 16 if cfg == SMALL40 else 32
    r = ctx.S // c
    keys = ctx.keygen(7, H.rotation_steps(c, r, layout))
    reqs, _ = _requests(ctx, keys, layout, sizes, 40, d)
    print("%s, layout %d: %s" % (cfg, layout, [len(q["Z"]) for q in reqs]), flush=True)
    want = []
    for q in reqs:
        Wn, g = ctx.lr_grad_step(q["Z"], q["W"], q["mask"], COEF, q["eta_over_n"], c, r, keys, mode=1, layout=layout)
        want.append((ctx.download(Wn), ctx.download(g), Wn.level, Wn.scale))
    for mode in (1, 0, 1):
        got = ctx.lr_grad_step_multi(reqs, c, r, keys, mode=mode, layout=layout)
        for (Wn, g), (wW, wg, lv, sc) in zip(got, want):
            assert (Wn.level, Wn.scale, g.level, g.scale) == (lv, sc, lv, sc)
            assert np.array_equal(ctx.download(Wn), wW) and np.array_equal(ctx.download(g), wg), mode
    # G_out omitted for some requests: W' unchanged
    reqs2 = [dict(q, G_out=False) if i % 2 else q for i, q in enumerate(reqs)]
    got = ctx.lr_grad_step_multi(reqs2, c, r, keys, mode=1, layout=layout)
    for i, ((Wn, g), (wW, wg, _, _)) in enumerate(zip(got, want)):
        assert np.array_equal(ctx.download(Wn), wW)
        assert (g is None) == bool(i % 2)


def test_multi_step_request_against_oracle():
    ctx = H.Context(*SMALL40)
    P = O.Params(*SMALL40)
    c, r = 16, ctx.S // 16
    steps = LR.rotation_steps(c, r, LR.FEATURES)
    keys, okeys = ctx.keygen(9, steps), O.Keys(P, 9, rot_steps=steps)
    reqs, raw = _requests(ctx, keys, H.LAYOUT_FEATURES, (700, 300), 60)
    got = ctx.lr_grad_step_multi(reqs, c, r, keys, mode=1, layout=H.LAYOUT_FEATURES)
    # the oracle from the same ciphertexts (downloaded: the encryption itself is checked elsewhere)
    q0, r0 = reqs[0], raw[0]
    oZ = [O.CT(ctx.download(z), z.level, z.scale) for z in q0["Z"]]
    oW = O.CT(ctx.download(q0["W"]), q0["W"].level, q0["W"].scale)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, COEF, 1.0 / r0["n"], 0.0, LR.FEATURES)
    assert pl["s_mask"] == r0["pl"]["s_mask"]  # the library's plan, evaluated by the oracle
    oWn, og = LR.lr_grad_step(P, okeys, oZ, oW, r0["mm"], COEF, 1.0 / r0["n"], c, r, plan=pl, layout=LR.FEATURES)
    assert np.array_equal(ctx.download(got[0][0]), oWn.data) and np.array_equal(ctx.download(got[0][1]), og.data)


def test_multi_step_errors():
    ctx = H.Context(*SMALL40)
    c, r = 16, ctx.S // 16
    keys = ctx.keygen(3, H.rotation_steps(c, r, H.LAYOUT_ROWS))
    reqs, _ = _requests(ctx, keys, H.LAYOUT_ROWS, (300, 300), 80)
    low = ctx.encrypt(ctx.pt_load(ctx.encode(np.zeros(ctx.S), ctx.delta), ctx.n_q - 2, ctx.delta), keys, 1, 1)
    bad = [reqs[0], dict(reqs[1], W=low)]
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step_multi(bad, c, r, keys, mode=1)
    assert e.value.status == 3  # HE_ELEVEL: the weights' levels differ (or the mask's level)
    with pytest.raises(H.HEError):
        ctx.lr_grad_step_multi(reqs, c, r, keys, mode=2)
    assert ctx.step_multi_bytes(ctx.n_q - 1, 2, 2) > ctx.step_bytes(ctx.n_q - 1, 2)
