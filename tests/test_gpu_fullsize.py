"""Parity at the headline size (N = 2^16, 20 + 4 primes, dnum 5) in the
launch configuration the bench times.

* every key-switching operation of the step, bit for bit against the oracle,
  at the levels the step uses;
* one-block steps (the whole circuit, the once-per-step sums included) bit for
  bit against the oracle, in the batched form, in both block layouts, with
  and without 16 baby steps;
* the full 47-block shard in both layouts, with and without 16 baby steps:
  the plain, batched and graph-replayed forms agree bit for bit, and the
  decrypted gradient is within 2^-20 of the FP64 one;
* 10 training steps with a refresh every 4, both layouts, against FP64.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ckks as O  # noqa: E402
from oracle import lr as LR  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402

W = synth.WORKLOADS["image"]
CFG = (W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"])


def _coef():
    c = LR.grad_poly_binomial(8.0)
    return [0.5, float(c[1]), 0.0, float(c[3])]


@pytest.fixture(scope="module")
def env():
    from paper_2006_10091_amd import he as H
    P = O.Params(*CFG)
    ctx = H.Context(*CFG)
    X, y = synth.image_data(W["seed_data"], W["n"])
    blocks, c, r = H.pack_blocks(X, y, ctx.S)
    steps = sorted({t for lay in (LR.ROWS, LR.FEATURES) for nb in (1, 16) for t in LR.rotation_steps(c, r, lay, nb)})
    gk = ctx.keygen(W["seed_keys"], steps)
    return dict(H=H, P=P, ctx=ctx, X=X, y=y, blocks=blocks, c=c, r=r, steps=steps, gk=gk)


@pytest.fixture(scope="module")
def okeys(env):
    return O.Keys(env["P"], W["seed_keys"], rot_steps=env["steps"])


def _rct(env, level, seed):
    P = env["P"]
    d = np.stack([synth.uniform_residues(seed, P.q[: level + 1], P.N),
                  synth.uniform_residues(seed + 1, P.q[: level + 1], P.N)])
    return d, env["ctx"].upload(d, level, 1.0)


def test_full_size_keyswitch_ops_bit_exact(env, okeys):
    ctx, P, gk = env["ctx"], env["P"], env["gk"]
    L = P.L
    xd, x = _rct(env, L, 101)
    yd, y = _rct(env, L, 103)
    got = ctx.rescale(ctx.relin(ctx.mul(x, y), gk))
    want = O.rescale(P, O.mul(P, O.CT(xd, L, 1.0), O.CT(yd, L, 1.0), okeys))
    assert np.array_equal(ctx.download(got), want.data)
    for level, t in ((L - 1, 1), (L - 2, -env["c"] // 2), (L - 4, env["c"] * 64)):
        zd, z = _rct(env, level, 200 + level)
        assert np.array_equal(ctx.download(ctx.rotate(z, t, gk)), O.rotate(P, O.CT(zd, level, 1.0), t, okeys).data)


def _edge_ct(env, level, seed):
    """Residues drawn only from {0, 1, (q-1)/2, (q+1)/2, q-1}: the centring
    boundaries of the rescale and basis conversions and the extremes of the
    lazy ranges."""
    P = env["P"]
    g = np.random.default_rng(seed)
    d = np.zeros((2, level + 1, P.N), dtype=np.uint64)
    for i, q in enumerate(P.q[: level + 1]):
        edges = np.array([0, 1, (q - 1) // 2, (q + 1) // 2, q - 1], dtype=np.uint64)
        d[:, i, :] = edges[g.integers(0, 5, size=(2, P.N))]
    return d, env["ctx"].upload(d, level, 1.0)


def test_full_size_edge_residues_bit_exact(env, okeys):
    """mul -> relin -> rescale, a rotation and a hoisted rotation sum at N = 2^16
    with 20 + 4 primes on edge-valued residues, bit for bit against the oracle."""
    ctx, P, gk = env["ctx"], env["P"], env["gk"]
    L = P.L
    xd, x = _edge_ct(env, L, 1)
    yd, y = _edge_ct(env, L, 2)
    got = ctx.rescale(ctx.relin(ctx.mul(x, y), gk))
    want = O.rescale(P, O.mul(P, O.CT(xd, L, 1.0), O.CT(yd, L, 1.0), okeys))
    assert np.array_equal(ctx.download(got), want.data)
    zd, z = _edge_ct(env, L - 1, 3)
    t = env["c"] // 2
    assert np.array_equal(ctx.download(ctx.rotate(z, t, gk)), O.rotate(P, O.CT(zd, L - 1, 1.0), t, okeys).data)
    steps = [16 * env["r"] * g for g in (1, 2, 3)]  # giant steps of the feature-major margin sum
    out = ctx.rotate_sum([z], steps, gk)
    want = O.rotate_sum_hoisted(P, O.CT(zd, L - 1, 1.0), steps, okeys)
    assert np.array_equal(ctx.download(out[0]), want.data)


def _as_grid(H, slots, c, r, layout):
    """Decoded slots as [sample row, feature column]."""
    v = np.asarray(slots)
    return v.reshape(c, r).T if layout == H.LAYOUT_FEATURES else v.reshape(r, c)


@pytest.mark.parametrize("layout,n_baby", [(0, 1), (1, 1), (1, 16), (0, 16)])
def test_full_size_one_block_step_bit_exact(env, okeys, layout, n_baby):
    """One block of the shard through the whole circuit, GPU batched form vs
    oracle, in both layouts, and feature-major with baby steps."""
    ctx, P, gk = env["ctx"], env["P"], env["gk"]
    c, r = env["c"], env["r"]
    assert set(LR.rotation_steps(c, r, layout, n_baby)) <= set(env["steps"])
    coef = _coef()
    eta_n = 1.0 / 128
    blk = (LR.pack_blocks_features if layout else LR.pack_blocks)(env["X"], env["y"], P.S)[0][5]
    m = O.encode(blk, P.delta, P.N)
    oZ = O.encrypt_sk(P, okeys, m, P.L, P.delta, 9, 5)
    gZ = ctx.ct_block(1, P.L)
    ctx.encrypt(ctx.pt_load(m, P.L, P.delta), gk, 9, 5, out=gZ[0])
    w = np.random.default_rng(5).uniform(-0.05, 0.05, 196)
    pw = LR.pack_weights_features(w, P.S, c) if layout else LR.pack_weights(w, P.S, c)
    mw = O.encode(pw, P.delta, P.N)
    oW = O.encrypt_sk(P, okeys, mw, P.L, P.delta, 9, 999)
    gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), gk, 9, 999)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n, 0.0, layout)
    mm = O.encode(LR.feature_mask(P.S, r) if layout else LR.column_mask(P.S, c), pl["s_mask"], P.N)
    unit = r if layout else 1
    oZr = LR.rotate_data(P, okeys, [oZ], unit, n_baby) if n_baby > 1 else None
    oWn, og = LR.lr_grad_step(P, okeys, [oZ], oW, mm, coef, eta_n, c, r, plan=pl, layout=layout, Zrot=oZr,
                              n_baby=n_baby)
    H = env["H"]
    mask = ctx.pt_load(mm, H.mask_level(P.L, layout), pl["s_mask"])
    gZr = ctx.rotate_data(gZ, unit, n_baby, gk)
    Wn, g = ctx.lr_grad_step(gZ, gW, mask, coef, eta_n, c, r, gk, mode=1, layout=layout, Zrot=gZr, n_baby=n_baby)
    assert np.array_equal(ctx.download(Wn), oWn.data)
    assert np.array_equal(ctx.download(g), og.data)


@pytest.mark.parametrize("layout,n_baby", [(0, 1), (1, 1), (1, 16), (0, 16)])
def test_full_shard_forms_agree_and_gradient_within_tolerance(env, layout, n_baby):
    ctx, gk, H = env["ctx"], env["gk"], env["H"]
    L, S = ctx.n_q - 1, ctx.S
    X, y = env["X"], env["y"]
    blocks, c, r = H.pack_blocks(X, y, S, layout)
    d = X.shape[1]
    Z = ctx.ct_block(blocks.shape[0], L)
    for i in range(blocks.shape[0]):
        ctx.encrypt(ctx.pt_load(ctx.encode(blocks[i], ctx.delta), L, ctx.delta), gk, W["seed_enc"], i, out=Z[i])
    w0 = np.random.default_rng(8).uniform(-0.02, 0.02, d)
    Wc = ctx.encrypt(ctx.pt_load(ctx.encode(H.pack_weights(w0, S, c, layout), ctx.delta), L, ctx.delta), gk, 3,
                     77777)
    coef, eta_n = _coef(), 1.0 / X.shape[0]
    pl = ctx.plan_lr_step(L, ctx.delta, ctx.delta, coef, eta_n, layout=layout)
    mask = ctx.pt_load(ctx.encode(H.step_mask(S, c, layout), pl["s_mask"]), H.mask_level(L, layout), pl["s_mask"])
    Zr = ctx.rotate_data(Z, H.baby_unit(layout, r), n_baby, gk)
    outs = []
    for mode in (0, 1, 2, 2):
        Wn, g = ctx.lr_grad_step(Z, Wc, mask, coef, eta_n, c, r, gk, mode=mode, layout=layout, Zrot=Zr,
                                 n_baby=n_baby)
        outs.append((ctx.download(Wn), ctx.download(g)))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    wgrid = _as_grid(H, ctx.decrypt_decode(Wc, gk).real, c, r, layout)
    gref = LR.lr_gradient_fp64(X, y, wgrid[0, :d], coef, eta_n)
    gd = _as_grid(H, ctx.decrypt_decode(g, gk).real, c, r, layout)
    for row in (0, r // 2, r - 1):
        assert np.max(np.abs(gd[row, :d] - gref)) / np.max(np.abs(gref)) < 2.0 ** -20
        assert np.max(np.abs(gd[row, d:])) < 2.0 ** -20 * np.max(np.abs(gref))  # padded features stay 0
    wn = _as_grid(H, ctx.decrypt_decode(Wn, gk).real, c, r, layout)
    for row in (0, r - 1):  # each slot of W carries its own encryption noise
        want = wgrid[row, :d] + gref
        assert np.max(np.abs(wn[row, :d] - want)) / np.max(np.abs(want)) < 2.0 ** -20


@pytest.mark.parametrize("layout,n_baby", [(0, 1), (1, 1), (1, 16), (0, 16)])
def test_full_size_training_ten_steps_refresh_every_four(env, layout, n_baby):
    """The image shard's 10 steps with a refresh every 4 (Alg. 1 / Alg. 2),
    graph-replayed batched form, against FP64 plaintext training."""
    from paper_2006_10091_amd import train as T
    ctx, gk = env["ctx"], env["gk"]
    X, y = env["X"], env["y"]
    coef = _coef()
    rec = []
    w_final = T.train(ctx, gk, X, y, coef, 1.0, 10, 4, np.zeros(X.shape[1]), 3004, mode=2, record=rec,
                      layout=layout, n_baby=n_baby)
    w = np.zeros(X.shape[1])
    for k in range(10):
        w = w + LR.lr_gradient_fp64(X, y, w, coef, 1.0 / X.shape[0])
        assert np.max(np.abs(rec[k] - w)) / np.max(np.abs(w)) < 2.0 ** -20, k
    assert np.max(np.abs(w_final - w)) / np.max(np.abs(w)) < 2.0 ** -20
