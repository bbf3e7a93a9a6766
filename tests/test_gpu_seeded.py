"""Seeded ciphertexts (the uniform part regenerated from (seed, index), drawn
in the evaluation domain) and the chunked step over them: bit for bit against
the oracle's seeded encryption and step, and against he_lr_grad_step on the
expanded blocks, at the small size and at the large-shard parameters
(N = 2^16, 24 + 6 primes)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ckks as O  # noqa: E402
from oracle import lr as LR  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402


def _coef():
    c = LR.grad_poly_binomial(8.0)
    return [0.5, float(c[1]), 0.0, float(c[3])]


@pytest.mark.parametrize("cfg", [(13, 5, 1, 1, 30), (16, 24, 6, 6, 40)])
def test_seeded_encryption_bit_exact(cfg):
    from paper_2006_10091_amd import he as H
    P = O.Params(*cfg)
    ctx = H.Context(*cfg)
    ok = O.Keys(P, 41)
    gk = ctx.keygen(41, [])
    z = np.random.default_rng(1).uniform(-1, 1, P.S)
    m = O.encode(z, P.delta, P.N)
    for level, idx in ((P.L, 7), (1, 123456)):
        sc = ctx.encrypt_seeded(ctx.pt_load(m, level, P.delta), gk, 99, idx)
        assert (sc.level, sc.seed, sc.index) == (level, 99, idx)
        full = ctx.expand([sc])[0]
        want = O.encrypt_sk_seeded(P, ok, m, level, P.delta, 99, idx)
        assert np.array_equal(ctx.download(full), want.data)
    assert np.max(np.abs(ctx.decrypt_decode(full, gk).real - z)) < 2.0 ** -15


@pytest.mark.parametrize("n,chunks", [(700, (1, 2, 3)), (2048, (8, 5))])
def test_seeded_step_small_matches_oracle_and_full_form(n, chunks):
    from paper_2006_10091_amd import he as H
    cfg = (13, 5, 1, 1, 30)
    P = O.Params(*cfg)
    ctx = H.Context(*cfg)
    X, y = synth.small_data(n=n)
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    steps = LR.rotation_steps(c, r)
    ok, gk = O.Keys(P, 2001, rot_steps=steps), ctx.keygen(2001, steps)
    coef = _coef()
    eta = 1.0 / n
    w0 = synth.initial_weights("small", 16, 4001)
    L = P.L
    Zs = ctx.seeded_block(len(blocks), L)
    oZ = []
    for i in range(len(blocks)):
        mz = O.encode(blocks[i], P.delta, P.N)
        ctx.encrypt_seeded(ctx.pt_load(mz, L, P.delta), gk, 17, 500 + i, out=Zs[i])
        oZ.append(O.encrypt_sk_seeded(P, ok, mz, L, P.delta, 17, 500 + i))
    mw = O.encode(LR.pack_weights(w0, P.S, c), P.delta, P.N)
    oW = O.encrypt_sk(P, ok, mw, L, P.delta, 17, 9)
    gW = ctx.encrypt(ctx.pt_load(mw, L, P.delta), gk, 17, 9)
    pl = LR.plan_lr_step(P.q, L, P.delta, P.delta, coef, eta)
    mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    mask = ctx.pt_load(mm, L - 1, pl["s_mask"])
    oWn, og = LR.lr_grad_step(P, ok, oZ, oW, mm, coef, eta, c, r, plan=pl)
    full = ctx.ct_block(len(blocks), L)
    ctx.expand(Zs, full)
    Wf, gf = ctx.lr_grad_step(full, gW, mask, coef, eta, c, r, gk, mode=1)
    assert np.array_equal(ctx.download(Wf), oWn.data) and np.array_equal(ctx.download(gf), og.data)
    for ch in chunks:
        Wn, g = ctx.lr_grad_step_seeded(Zs, gW, mask, coef, eta, c, r, gk, chunk=ch)
        assert np.array_equal(ctx.download(Wn), oWn.data), ch
        assert np.array_equal(ctx.download(g), og.data), ch


def test_seeded_step_large_parameters_matches_full_form():
    """At the large-shard parameters (c = 512 features, r = 64 rows per block):
    8 seeded blocks in chunks of 3 against the batched step on the expanded
    blocks, bit for bit, and the gradient within 2^-20 of FP64."""
    from paper_2006_10091_amd import he as H
    W = synth.WORKLOADS["large"]
    cfg = (W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"])
    ctx = H.Context(*cfg)
    S = ctx.S
    rows = S // 512
    Xs, ys = zip(*[synth.large_block(W["seed_data"], b, rows) for b in range(8)])
    X, y = np.concatenate(Xs), np.concatenate(ys)
    blocks, c, r = H.pack_blocks(X, y, S)
    gk = ctx.keygen(W["seed_keys"], H.rotation_steps(c, r))
    L = ctx.n_q - 1
    Zs = ctx.seeded_block(len(blocks), L)
    for i in range(len(blocks)):
        ctx.encrypt_seeded(ctx.pt_load(ctx.encode(blocks[i], ctx.delta), L, ctx.delta), gk, W["seed_enc"], i,
                           out=Zs[i])
    w0 = np.random.default_rng(3).uniform(-0.05, 0.05, 512)
    Wc = ctx.encrypt(ctx.pt_load(ctx.encode(H.pack_weights(w0, S, c), ctx.delta), L, ctx.delta), gk, 5, 1 << 20)
    coef, eta = _coef(), 1.0 / X.shape[0]
    pl = ctx.plan_lr_step(L, ctx.delta, ctx.delta, coef, eta)
    mask = ctx.pt_load(ctx.encode(H.column0_mask(S, c), pl["s_mask"]), L - 1, pl["s_mask"])
    full = ctx.ct_block(len(blocks), L)
    ctx.expand(Zs, full)
    Wf, gf = ctx.lr_grad_step(full, Wc, mask, coef, eta, c, r, gk, mode=1)
    Wn, g = ctx.lr_grad_step_seeded(Zs, Wc, mask, coef, eta, c, r, gk, chunk=3)
    assert np.array_equal(ctx.download(Wn), ctx.download(Wf))
    assert np.array_equal(ctx.download(g), ctx.download(gf))
    wd = H.unpack_weights(ctx.decrypt_decode(Wc, gk).real, c, 512)
    gref = LR.lr_gradient_fp64(X, y, wd, coef, eta)
    gd = H.unpack_weights(ctx.decrypt_decode(g, gk).real, c, 512)
    assert np.max(np.abs(gd - gref)) / np.max(np.abs(gref)) < 2.0 ** -20
