"""GPU tests of the boundary calls beyond the operations: the worker's
public-key encryption (Alg. 1), encrypted inference with the polynomial, the
caller-provided allocator, and the graph cache's invalidation when keys are
replaced.  Bit for bit against the oracle on identical integer inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ckks as O  # noqa: E402
from oracle import lr as LR  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402

SMALL40 = (13, 5, 2, 2, 40)


@pytest.fixture(scope="module")
def env():
    from paper_2006_10091_amd import he as H
    P = O.Params(*SMALL40)
    ctx = H.Context(*SMALL40)
    c, r = 16, P.S // 16
    steps = sorted(set(LR.rotation_steps(c, r)) | set(LR.rotation_steps(c, r, LR.FEATURES)))
    return dict(H=H, P=P, ctx=ctx, c=c, r=r, steps=steps, okeys=O.Keys(P, 61, rot_steps=steps, with_pk=True),
                gkeys=ctx.keygen(61, steps))


def test_public_key_bit_exact(env):
    ctx, P = env["ctx"], env["P"]
    pk = env["gkeys"].download(-5).reshape(2, P.nq, P.N)
    assert np.array_equal(pk, env["okeys"].pk)


@pytest.mark.parametrize("level", [4, 2, 0])
def test_public_key_encryption_bit_exact(env, level):
    ctx, P = env["ctx"], env["P"]
    z = np.random.default_rng(level).uniform(-1, 1, P.S)
    m = O.encode(z, P.delta, P.N)
    got = ctx.encrypt(ctx.pt_load(m, level, P.delta), env["gkeys"], 77, 5 + level, use_sk=False)
    want = O.encrypt_pk(P, env["okeys"], m, level, P.delta, 77, 5 + level)
    assert np.array_equal(ctx.download(got), want.data)
    assert np.max(np.abs(ctx.decrypt_decode(got, env["gkeys"]).real - z)) < 2.0 ** -20
    # the secret-key form of the same call differs (another sampler stream)
    sk = ctx.encrypt(ctx.pt_load(m, level, P.delta), env["gkeys"], 77, 5 + level)
    assert not np.array_equal(ctx.download(sk), want.data)


def _data(env, layout, n=300):
    P = env["P"]
    X, y = synth.small_data(n=n)
    pack = LR.pack_blocks_features if layout == LR.FEATURES else LR.pack_blocks
    pw = LR.pack_weights_features if layout == LR.FEATURES else LR.pack_weights
    blocks, c, r = pack(X, y, P.S)
    w = np.random.default_rng(4).uniform(-0.3, 0.3, 16)
    return X, y, blocks, pw(w, P.S, c), w


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("poly", ["ls", "hinge", None])
def test_inference_bit_exact_all_forms(env, layout, poly):
    ctx, P, H = env["ctx"], env["P"], env["H"]
    c, r = env["c"], env["r"]
    X, y, blocks, pwv, w = _data(env, layout)
    if poly == "hinge":
        coef = [0.5875, -0.1005, 0.0008, -0.00039]
    elif poly == "ls":
        coef = list(LR.grad_poly_binomial(8.0))
        coef[0], coef[2] = 0.5, 0.0
    else:
        coef = None
    oZ, gZ = [], ctx.ct_block(len(blocks), P.L)
    for i in range(len(blocks)):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, env["okeys"], m, P.L, P.delta, 3, i))
        ctx.encrypt(ctx.pt_load(m, P.L, P.delta), env["gkeys"], 3, i, out=gZ[i])
    mw = O.encode(pwv, P.delta, P.N)
    oW = O.encrypt_sk(P, env["okeys"], mw, P.L, P.delta, 3, 99)
    gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), env["gkeys"], 3, 99)
    want = LR.lr_infer(P, env["okeys"], oZ, oW, c, r, layout, coef)
    for mode in (0, 1, 2, 2):
        out = ctx.lr_infer(gZ, gW, c, r, env["gkeys"], coef=coef, mode=mode, layout=layout)
        for o, wd in zip(out, want):
            assert o.level == wd.level and o.scale == wd.scale
            assert np.array_equal(ctx.download(o), wd.data), mode
    if coef is not None:
        m = (y[:, None] * X) @ w
        p = coef[0] + coef[1] * m + coef[2] * m * m + coef[3] * m ** 3
        dec = ctx.decrypt_decode(out[0], env["gkeys"]).real
        grid = dec.reshape(c, r).T if layout else dec.reshape(r, c)
        assert np.max(np.abs(grid[:, 0] - p[:r])) < 2.0 ** -20


def test_inference_errors(env):
    ctx, P, H = env["ctx"], env["P"], env["H"]
    Z = ctx.ct_block(1, 2)
    W = ctx.ct_empty(2)
    W.level, W.scale = 2, P.delta
    for z in Z:
        z.level, z.scale = 2, P.delta
    with pytest.raises(H.HEError) as e:  # the polynomial needs W at level 3 or more
        ctx.lr_infer(Z, W, env["c"], env["r"], env["gkeys"], coef=[0.5, 0.1, 0.0, 0.01], out=ctx.ct_block(1, 0))
    assert e.value.status == 3


def test_tables_and_workspace_come_from_torch(env):
    """Every device byte the context holds is a torch allocation made through
    the allocator callback; trimming gives the workspace back."""
    import gc
    from paper_2006_10091_amd import he as H
    gc.collect()  # a cycle collected while the context is built would free earlier tests' tensors
    gc.disable()
    try:
        before = torch.cuda.memory_allocated()
        ctx = H.Context(*SMALL40)
        held = ctx.mem.bytes
        grew = torch.cuda.memory_allocated() - before
    finally:
        gc.enable()
    assert held > 0 and grew >= held
    keys = ctx.keygen(5, [1])
    a, _ = ctx.upload(np.zeros((2, 5, ctx.N), dtype=np.uint64), 4, 1.0), None
    ctx.rotate(a, 1, keys)
    torch.cuda.synchronize()
    assert ctx.mem.bytes > held  # the workspace
    ctx.trim()
    assert ctx.mem.bytes == held
    del keys, ctx


def test_graph_cache_after_keys_replaced(env):
    """A step replayed from a graph, then keys destroyed and regenerated with
    the same byte size but another rotation order (the torch allocator may hand
    back the same buffer and the same host handle): the next mode-2 step must
    read the new keys, bit-exact against the oracle."""
    ctx, P, H = env["ctx"], env["P"], env["H"]
    c, r = env["c"], env["r"]
    X, y, blocks, pwv, w = _data(env, LR.ROWS)
    coef = list(LR.grad_poly_binomial(8.0))
    coef[0], coef[2] = 0.5, 0.0
    eta = 1.0 / X.shape[0]
    steps = LR.rotation_steps(c, r)
    okeys = O.Keys(P, 71, rot_steps=steps)
    oZ, gZ = [], ctx.ct_block(len(blocks), P.L)
    for i in range(len(blocks)):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, okeys, m, P.L, P.delta, 4, i))
    mw = O.encode(pwv, P.delta, P.N)
    oW = O.encrypt_sk(P, okeys, mw, P.L, P.delta, 4, 99)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta)
    mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, okeys, oZ, oW, mm, coef, eta, c, r, plan=pl)
    mask = ctx.pt_load(mm, P.L - 1, pl["s_mask"])
    Wout, Gout = ctx.ct_empty(P.L - 4), ctx.ct_empty(P.L - 4)
    for order in (steps, steps[::-1], steps[1:] + steps[:1]):
        gk = ctx.keygen(71, order)
        for i in range(len(blocks)):
            ctx.encrypt(ctx.pt_load(O.encode(blocks[i], P.delta, P.N), P.L, P.delta), gk, 4, i, out=gZ[i])
        gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), gk, 4, 99)
        for _ in range(2):
            Wn, g = ctx.lr_grad_step(gZ, gW, mask, coef, eta, c, r, gk, mode=2, W_out=Wout, G_out=Gout)
            assert np.array_equal(ctx.download(Wn), oWn.data), order[:3]
            assert np.array_equal(ctx.download(g), og.data)
        del gk


def test_keys_released_after_their_context():
    """A context and its keys may be released in either order: with the
    context destroyed first (an order Python's cycle collector may take), the
    keys are still released cleanly, graphs captured with them included."""
    from paper_2006_10091_amd import he as H
    ctx = H.Context(*SMALL40)
    keys = ctx.keygen(5, [1])
    q = ctx.primes[:4]
    x = ctx.upload(np.stack([synth.uniform_residues(3, q, ctx.N), synth.uniform_residues(4, q, ctx.N)]), 3, 1.0)
    ctx.batch_submit([(H.OP_ROTATE, 1, x, None, None)], keys, mode=2)  # a graph that names these keys
    torch.cuda.synchronize()
    h, kh = ctx.h, keys.handle
    ctx.h, keys.handle = None, None  # the binding's destructors will not release them again
    assert H._lib.he_ctx_destroy(h) == 0
    assert H._lib.he_keys_destroy(kh) == 0
    # and the other order, for completeness
    ctx2 = H.Context(*SMALL40)
    k2 = ctx2.keygen(5, [1])
    h2, kh2 = ctx2.h, k2.handle
    ctx2.h, k2.handle = None, None
    assert H._lib.he_keys_destroy(kh2) == 0
    assert H._lib.he_ctx_destroy(h2) == 0
