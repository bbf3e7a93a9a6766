"""Parity at the large-shard parameters (N = 2^16, 24 + 6 primes, dnum 4,
512 dense Gaussian features: c = 512, r = 64), on a subset of the shard's
blocks (the full 2^20 samples are 16384 blocks).

* one block through the whole row-major circuit, GPU batched form bit for bit
  against the oracle at the top level;
* 8 blocks: plain, batched and graph forms agree bit for bit and the
  decrypted gradient is within 2^-20 of FP64;
* the shard's schedule on those 8 blocks: 5 steps from level 23 with no
  refresh (23 -> 19 -> 15 -> 11 -> 7 -> 3), each step's output within 2^-20 of
  the FP64 step taken from the decrypted input weights;
* the feature-major layout is refused at the full shard's n = 2^20.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ckks as O  # noqa: E402
from oracle import lr as LR  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402

W = synth.WORKLOADS["large"]
CFG = (W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"])
NB = 8


def _coef():
    c = LR.grad_poly_binomial(8.0)
    return [0.5, float(c[1]), 0.0, float(c[3])]


@pytest.fixture(scope="module")
def env():
    from paper_2006_10091_amd import he as H
    ctx = H.Context(*CFG)
    S = ctx.S
    Xs, ys = zip(*[synth.large_block(W["seed_data"], b, S // 512, 512) for b in range(NB)])
    X, y = np.concatenate(Xs), np.concatenate(ys)
    blocks, c, r = H.pack_blocks(X, y, S)
    assert (c, r) == (512, 64) and blocks.shape[0] == NB
    steps = H.rotation_steps(c, r)
    gk = ctx.keygen(W["seed_keys"], steps)
    L = ctx.n_q - 1
    Z = ctx.ct_block(NB, L)
    for i in range(NB):
        ctx.encrypt(ctx.pt_load(ctx.encode(blocks[i], ctx.delta), L, ctx.delta), gk, W["seed_enc"], i, out=Z[i])
    return dict(H=H, ctx=ctx, X=X, y=y, blocks=blocks, c=c, r=r, steps=steps, gk=gk, Z=Z, L=L)


def test_large_params_one_block_bit_exact(env):
    ctx, gk, c, r, L = env["ctx"], env["gk"], env["c"], env["r"], env["L"]
    P = O.Params(*CFG)
    assert ctx.primes == P.q and P.ndigits(P.L) == 4
    okeys = O.Keys(P, W["seed_keys"], rot_steps=env["steps"])
    coef, eta_n = _coef(), 1.0 / 64
    m = O.encode(env["blocks"][3], P.delta, P.N)
    oZ = O.encrypt_sk(P, okeys, m, L, P.delta, 11, 3)
    gZ = ctx.ct_block(1, L)
    ctx.encrypt(ctx.pt_load(m, L, P.delta), gk, 11, 3, out=gZ[0])
    w = np.random.default_rng(7).standard_normal(512) / np.sqrt(512)
    mw = O.encode(LR.pack_weights(w, P.S, c), P.delta, P.N)
    oW = O.encrypt_sk(P, okeys, mw, L, P.delta, 11, 999)
    gW = ctx.encrypt(ctx.pt_load(mw, L, P.delta), gk, 11, 999)
    pl = LR.plan_lr_step(P.q, L, P.delta, P.delta, coef, eta_n)
    mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, okeys, [oZ], oW, mm, coef, eta_n, c, r, plan=pl)
    Wn, g = ctx.lr_grad_step(gZ, gW, ctx.pt_load(mm, L - 1, pl["s_mask"]), coef, eta_n, c, r, gk, mode=1)
    assert np.array_equal(ctx.download(Wn), oWn.data)
    assert np.array_equal(ctx.download(g), og.data)


def _grad_check(env, W_in, g, coef, eta_n):
    H, ctx, gk, c, r = env["H"], env["ctx"], env["gk"], env["c"], env["r"]
    X, y = env["X"], env["y"]
    wdec = ctx.decrypt_decode(W_in, gk).real.reshape(r, c)[0]
    gref = LR.lr_gradient_fp64(X, y, wdec, coef, eta_n)
    gd = ctx.decrypt_decode(g, gk).real.reshape(r, c)
    for row in (0, r - 1):
        assert np.max(np.abs(gd[row] - gref)) / np.max(np.abs(gref)) < 2.0 ** -20
    return wdec, gref


def test_large_params_eight_blocks_forms_and_tolerance(env):
    H, ctx, gk, c, r, L = env["H"], env["ctx"], env["gk"], env["c"], env["r"], env["L"]
    coef, eta_n = _coef(), 1.0 / env["X"].shape[0]
    w0 = np.random.default_rng(8).standard_normal(512) * 0.05
    Wc = ctx.encrypt(ctx.pt_load(ctx.encode(H.pack_weights(w0, ctx.S, c), ctx.delta), L, ctx.delta), gk, 5, 4242)
    pl = ctx.plan_lr_step(L, ctx.delta, ctx.delta, coef, eta_n)
    mask = ctx.pt_load(ctx.encode(H.column0_mask(ctx.S, c), pl["s_mask"]), L - 1, pl["s_mask"])
    outs = []
    for mode in (0, 1, 2, 2):
        Wn, g = ctx.lr_grad_step(env["Z"], Wc, mask, coef, eta_n, c, r, gk, mode=mode)
        outs.append((ctx.download(Wn), ctx.download(g)))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    _grad_check(env, Wc, g, coef, eta_n)


def test_large_params_five_steps_without_refresh(env):
    """Levels 23 -> 3 in 5 graph-replayed steps; every step's g against FP64
    at its decrypted input weights."""
    from paper_2006_10091_amd import train as T
    H, ctx, gk, c, r, L = env["H"], env["ctx"], env["gk"], env["c"], env["r"], env["L"]
    coef, eta_n = _coef(), 1.0 / env["X"].shape[0]
    ps = T.ParameterServer(ctx, gk, 512, c, W["seed_enc"])
    worker = T.Worker(ctx, gk, env["Z"], coef, eta_n, c, r, mode=2)
    Wc = ps.encrypt_weights(np.zeros(512))
    for k in range(5):
        assert Wc.level == L - 4 * k
        Wn, g = worker.step(Wc, want_g=True)
        _grad_check(env, Wc, g, coef, eta_n)
        Wc = Wn
    assert Wc.level == 3


def test_feature_major_refused_at_full_large_shard(env):
    H, ctx = env["H"], env["ctx"]
    with pytest.raises(H.HEError) as e:
        ctx.plan_lr_step(env["L"], ctx.delta, ctx.delta, _coef(), 2.0 ** -20, layout=H.LAYOUT_FEATURES)
    assert e.value.status == 4
