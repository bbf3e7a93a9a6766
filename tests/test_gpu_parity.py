"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Ciphertexts, keys and every operation are compared BIT FOR BIT in coefficient
form on identical integer inputs (the oracle's encodings are fed to both
sides; no oracle input comes from the GPU).  Decrypted gradients are compared
with the FP64 plaintext gradient at the benchmark spec's tolerance 2^-20 (relative,
infinity norm).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ckks as O  # noqa: E402
from oracle import lr as LR  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402

TOL = 2.0 ** -20


def _H():
    from paper_2006_10091_amd import he as H
    return H


def _cfg(name):
    W = synth.WORKLOADS[name]
    return W, (W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"])


@pytest.fixture(scope="module")
def small():
    """Small workload: oracle params/keys and a GPU context/keys with the same seeds."""
    W, cfg = _cfg("small")
    P = O.Params(*cfg)
    H = _H()
    ctx = H.Context(*cfg)
    X, y = synth.small_data()
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    steps = set(LR.rotation_steps(c, r, LR.FEATURES))
    for nb in (1, 4, 8, 16):  # the row-major baby-step counts the tests take
        steps |= set(LR.rotation_steps(c, r, LR.ROWS, nb))
    steps = sorted(steps)
    okeys = O.Keys(P, W["seed_keys"], rot_steps=steps)
    gkeys = ctx.keygen(W["seed_keys"], steps)
    return dict(W=W, P=P, ctx=ctx, X=X, y=y, blocks=blocks, c=c, r=r, okeys=okeys, gkeys=gkeys, H=H)


def random_ct(ctx, P, level, seed, scale=1.0):
    data = np.stack([synth.uniform_residues(seed, P.q[: level + 1], P.N),
                     synth.uniform_residues(seed + 1, P.q[: level + 1], P.N)])
    return data, ctx.upload(data, level, scale)


# ------------------------------------------------------------------ chain, NTT, keys, encryption
def test_prime_chain_matches(small):
    assert small["ctx"].primes == small["P"].q


def test_upload_download_roundtrip_is_identity(small):
    ctx, P = small["ctx"], small["P"]
    for level in (0, 2, P.L):
        data, ct = random_ct(ctx, P, level, 10 + level)
        assert np.array_equal(ctx.download(ct), data)


def test_ntt_product_matches_oracle(small):
    """NTT -> pointwise -> iNTT through he_mul equals the oracle's negacyclic products."""
    ctx, P = small["ctx"], small["P"]
    xd, x = random_ct(ctx, P, P.L, 21)
    yd, y = random_ct(ctx, P, P.L, 23)
    d3 = ctx.mul(x, y)
    want, _ = O.tensor(P, O.CT(xd, P.L, 1.0), O.CT(yd, P.L, 1.0))
    H = small["H"]
    per = 2 * (P.L + 1) * P.N
    first = ctx.download(H.Ciphertext(d3.tensor, P.L, 1.0))
    last = ctx.download(H.Ciphertext(d3.tensor, P.L, 1.0, offset=per // 2))
    assert np.array_equal(first[0], want[0]) and np.array_equal(first[1], want[1])
    assert np.array_equal(last[1], want[2])


def test_keys_bit_exact(small):
    P, okeys, gkeys = small["P"], small["okeys"], small["gkeys"]
    nfull = P.nq + P.nk
    s = gkeys.download(-2).reshape(nfull, P.N)
    srns = np.array([[int(v) % q for v in okeys.s] for q in P.q], dtype=np.uint64)
    assert np.array_equal(s, srns)
    assert np.array_equal(gkeys.download(-1).reshape(okeys.rlk.shape), okeys.rlk)
    for j in (3, 4):  # keys for s^3 and s^4
        assert np.array_equal(gkeys.download(-j).reshape(okeys.rlk_pow[j].shape), okeys.rlk_pow[j])
    for t in (1, -1, small["c"]):
        g = O.galois(P, t)
        assert np.array_equal(gkeys.download(g).reshape(okeys.rot[g].shape), okeys.rot[g])


def test_encrypt_bit_exact(small):
    ctx, P = small["ctx"], small["P"]
    m = synth.small_poly(5, P.N, 1 << 40)
    for level, idx in ((P.L, 0), (1, 7)):
        pt = ctx.pt_load(m, level, P.delta)
        ct = ctx.encrypt(pt, small["gkeys"], 3001, idx)
        want = O.encrypt_sk(P, small["okeys"], m, level, P.delta, 3001, idx)
        assert np.array_equal(ctx.download(ct), want.data)
        res = ctx.decrypt(ct, small["gkeys"])
        assert np.array_equal(res, O.decrypt_residues(P, small["okeys"], want))


# ------------------------------------------------------------------ operations
def test_ops_bit_exact_small(small):
    ctx, P, ok, gk = small["ctx"], small["P"], small["okeys"], small["gkeys"]
    l = P.L
    xd, x = random_ct(ctx, P, l, 31)
    yd, y = random_ct(ctx, P, l, 33)
    ox, oy = O.CT(xd, l, 1.0), O.CT(yd, l, 1.0)
    # relinearised product
    got = ctx.relin(ctx.mul(x, y), gk)
    want = O.mul(P, ox, oy, ok)
    assert np.array_equal(ctx.download(got), want.data)
    # rescale (also in place)
    r = ctx.rescale(got)
    assert np.array_equal(ctx.download(r), O.rescale(P, want).data)
    # rotations, both directions
    for t in (1, -2, small["c"]):
        assert np.array_equal(ctx.download(ctx.rotate(x, t, gk)), O.rotate(P, ox, t, ok).data)
    # add, integer and plaintext products
    assert np.array_equal(ctx.download(ctx.add(x, y)), O.add(P, ox, oy).data)
    k = -(1 << 61) + 12345
    assert np.array_equal(ctx.download(ctx.mul_int(x, k, 1.0)), O.mul_int(P, ox, k).data)
    m = synth.small_poly(8, P.N, 1 << 30)
    pt = ctx.pt_load(m, l, 1.0)
    assert np.array_equal(ctx.download(ctx.mul_plain(x, pt)), O.mul_plain(P, ox, m, 1.0).data)
    # drop level
    assert np.array_equal(ctx.download(ctx.drop_level(x, 2)), O.drop(ox, 2).data)


@pytest.mark.parametrize("steps", [[512 * g for g in range(1, 8)], [1, 3, -100, 2048]])
@pytest.mark.parametrize("n_ct", [3, 9])
def test_rotate_sum_hoisted_bit_exact(small, steps, n_ct):
    """x + sum_s Rot(x, s) as one hoisted key switch, n_ct ciphertexts at a
    middle level, against the oracle bit for bit: the rotations by multiples
    of S/8 (a group: the gathers stay inside 16-coefficient runs) and an
    arbitrary set.  With 9 ciphertexts the 4 waves of a workgroup take two of
    them per pass on the wide primes, and one wave a last single one."""
    ctx, P, W = small["ctx"], small["P"], small["W"]
    okeys = O.Keys(P, W["seed_keys"] + 7, rot_steps=steps)
    gkeys = ctx.keygen(W["seed_keys"] + 7, steps)
    level = 3
    xs = ctx.ct_block(n_ct, level)
    want = []
    for i in range(n_ct):
        data = np.stack([synth.uniform_residues(61 + 2 * i, P.q[: level + 1], P.N),
                         synth.uniform_residues(62 + 2 * i, P.q[: level + 1], P.N)])
        ctx.upload(data, level, 1.0, out=xs[i])
        want.append(O.rotate_sum_hoisted(P, O.CT(data, level, 1.0), steps, okeys).data)
    got = ctx.rotate_sum(xs, steps, gkeys)
    for i in range(n_ct):
        assert np.array_equal(ctx.download(got[i]), want[i]), i
    with pytest.raises(small["H"].HEError):  # an output overlapping the input
        ctx.rotate_sum(xs, steps, gkeys, outs=xs)


def test_rotate_sum_and_data_terms_errors(small, small_step):
    """Errors before any launch: he_rotate_sum with more than 32 steps, a
    step without a key, and no steps; he_lr_data_terms with an unknown layout
    or weights too low to plan."""
    ctx, P, gk, H, s = small["ctx"], small["P"], small["gkeys"], small["H"], small_step
    xs = ctx.ct_block(2, 3)
    for i in range(2):
        d = np.stack([synth.uniform_residues(71 + 2 * i, P.q[:4], P.N), synth.uniform_residues(72 + 2 * i, P.q[:4], P.N)])
        ctx.upload(d, 3, 1.0, out=xs[i])
    with pytest.raises(H.HEError) as e:
        ctx.rotate_sum(xs, [1] * 33, gk)
    assert e.value.status == 1  # HE_EINVAL
    with pytest.raises(H.HEError) as e:
        ctx.rotate_sum(xs, [1, 17], gk)
    assert e.value.status == 5  # HE_EKEY
    with pytest.raises(H.HEError) as e:
        ctx.rotate_sum(xs, [], gk)
    assert e.value.status == 1
    with pytest.raises(H.HEError) as e:
        ctx.lr_data_terms(s["gZ"], s["gW"].level, s["gW"].scale, s["coef"], s["eta_n"], layout=7)
    assert e.value.status == 1
    with pytest.raises(H.HEError) as e:
        ctx.lr_data_terms(s["gZ"], 3, s["gW"].scale, s["coef"], s["eta_n"])
    assert e.value.status == 3  # HE_ELEVEL: fewer than 4 levels


def test_rescale_in_place(small):
    ctx, P = small["ctx"], small["P"]
    xd, x = random_ct(ctx, P, P.L, 41)
    want = O.rescale(P, O.CT(xd, P.L, 1.0))
    ctx.rescale(x, out=x)
    assert x.level == P.L - 1
    assert np.array_equal(ctx.download(x), want.data)


def test_error_paths(small):
    ctx, P, gk, H = small["ctx"], small["P"], small["gkeys"], small["H"]
    _, x = random_ct(ctx, P, 0, 51)
    with pytest.raises(H.HEError) as e:
        ctx.rescale(x)
    assert e.value.status == 3
    _, a = random_ct(ctx, P, 2, 52, scale=1.0)
    _, b = random_ct(ctx, P, 2, 53, scale=2.0)
    with pytest.raises(H.HEError) as e:
        ctx.add(a, b)
    assert e.value.status == 4
    with pytest.raises(H.HEError) as e:
        ctx.rotate(a, 17, gk)  # no key for step 17
    assert e.value.status == 5


# ------------------------------------------------------------------ the gradient step, small workload
def _encrypt_small(small, blocks, w0):
    """Same integer plaintexts and seeds on both sides."""
    P, ctx, W = small["P"], small["ctx"], small["W"]
    oZ, gZ = [], ctx.ct_block(blocks.shape[0], P.L)
    for i in range(blocks.shape[0]):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, small["okeys"], m, P.L, P.delta, W["seed_enc"], i))
        ctx.encrypt(ctx.pt_load(m, P.L, P.delta), small["gkeys"], W["seed_enc"], i, out=gZ[i])
    mw = O.encode(LR.pack_weights(w0, P.S, small["c"]), P.delta, P.N)
    oW = O.encrypt_sk(P, small["okeys"], mw, P.L, P.delta, W["seed_enc"], 100000)
    gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), small["gkeys"], W["seed_enc"], 100000)
    return oZ, gZ, oW, gW


COEF = None


def _coef():
    c = LR.grad_poly_binomial(8.0)
    c[0], c[2] = 0.5, 0.0
    return [float(v) for v in c]


@pytest.fixture(scope="module")
def small_step(small):
    P = small["P"]
    w0 = synth.initial_weights("small", 16, small["W"]["seed_w"])
    coef = _coef()
    eta_n = 1.0 / small["X"].shape[0]
    oZ, gZ, oW, gW = _encrypt_small(small, small["blocks"], w0)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n)
    mask_m = O.encode(LR.column_mask(P.S, small["c"]), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, small["okeys"], oZ, oW, mask_m, coef, eta_n, small["c"], small["r"], plan=pl)
    return dict(w0=w0, coef=coef, eta_n=eta_n, gZ=gZ, gW=gW, oW=oW, pl=pl, mask_m=mask_m, oWn=oWn, og=og)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_lr_step_bit_exact_small(small, small_step, mode):
    ctx, P, s = small["ctx"], small["P"], small_step
    mask = ctx.pt_load(s["mask_m"], P.L - 1, s["pl"]["s_mask"])
    for _ in range(2 if mode == 2 else 1):  # mode 2: capture, then replay
        Wn, g = ctx.lr_grad_step(s["gZ"], s["gW"], mask, s["coef"], s["eta_n"], small["c"], small["r"],
                                 small["gkeys"], mode=mode)
        assert Wn.level == P.L - 4 and Wn.scale == s["pl"]["s_g"]
        assert np.array_equal(ctx.download(Wn), s["oWn"].data)
        assert np.array_equal(ctx.download(g), s["og"].data)


def test_lr_step_gradient_within_tolerance_small(small, small_step):
    """End to end on the GPU (library encode): decrypted g vs the FP64 gradient
    at the decrypted input weights."""
    ctx, P, gk, s = small["ctx"], small["P"], small["gkeys"], small_step
    c, r = small["c"], small["r"]
    Z = ctx.ct_block(small["blocks"].shape[0], P.L)
    for i in range(len(Z)):
        ctx.encrypt(ctx.pt_load(ctx.encode(small["blocks"][i], P.delta), P.L, P.delta), gk, 77, i, out=Z[i])
    Wc = ctx.encrypt(ctx.pt_load(ctx.encode(LR.pack_weights(s["w0"], P.S, c), P.delta), P.L, P.delta), gk, 77,
                     9999)
    pl = ctx.plan_lr_step(P.L, P.delta, P.delta, s["coef"], s["eta_n"])
    mask = ctx.pt_load(ctx.encode(LR.column_mask(P.S, c), pl["s_mask"]), P.L - 1, pl["s_mask"])
    Wn, g = ctx.lr_grad_step(Z, Wc, mask, s["coef"], s["eta_n"], c, r, gk, mode=1)
    wdec = ctx.decrypt_decode(Wc, gk).real[:16]
    gref = LR.lr_gradient_fp64(small["X"], small["y"], wdec, s["coef"], s["eta_n"])
    gd = ctx.decrypt_decode(g, gk).real.reshape(r, c)[:, :16]
    for row in (0, r // 3, r - 1):
        assert np.max(np.abs(gd[row] - gref)) / np.max(np.abs(gref)) < TOL
    wn = ctx.decrypt_decode(Wn, gk).real.reshape(r, c)[0, :16]
    assert np.max(np.abs(wn - wdec - gref)) / np.max(np.abs(wdec + gref)) < TOL


def test_lr_step_ragged_single_block(small):
    """300 samples: one block, 44 zero rows; batched form vs oracle, bit for bit."""
    ctx, P = small["ctx"], small["P"]
    X, y = synth.small_data(n=300)
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    assert blocks.shape[0] == 2 and (300 % r) != 0
    w0 = synth.initial_weights("small", 16, 4321)
    coef = _coef()
    oZ, gZ, oW, gW = _encrypt_small(small, blocks, w0)
    for nb in (1, 2):
        pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, 1 / 300)
        mask_m = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
        oWn, og = LR.lr_grad_step(P, small["okeys"], oZ[:nb], oW, mask_m, coef, 1 / 300, c, r, plan=pl)
        mask = ctx.pt_load(mask_m, P.L - 1, pl["s_mask"])
        Wn, g = ctx.lr_grad_step(gZ[:nb], gW, mask, coef, 1 / 300, c, r, small["gkeys"], mode=1)
        assert np.array_equal(ctx.download(Wn), oWn.data)
        assert np.array_equal(ctx.download(g), og.data)


def test_lr_step_error_paths(small, small_step):
    ctx, P, gk, H, s = small["ctx"], small["P"], small["gkeys"], small["H"], small_step
    c, r = small["c"], small["r"]
    mask = ctx.pt_load(s["mask_m"], P.L - 1, s["pl"]["s_mask"])
    low = ctx.drop_level(s["gW"], 3)
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step(s["gZ"], low, mask, s["coef"], s["eta_n"], c, r, gk)
    assert e.value.status == 3  # HE_ELEVEL: fewer than 4 levels
    bad = ctx.pt_load(s["mask_m"], P.L - 1, s["pl"]["s_mask"] * 2)
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step(s["gZ"], s["gW"], bad, s["coef"], s["eta_n"], c, r, gk)
    assert e.value.status == 4  # HE_ESCALE: mask at the wrong scale
    few = ctx.keygen(2001, [1, -1])
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step(s["gZ"], s["gW"], mask, s["coef"], s["eta_n"], c, r, few)
    assert e.value.status == 5  # HE_EKEY: rotations missing
    # keys that only the grouped slot sums take (no power of two): column sum 3,
    # replication -12, row sum 3 c; each missing one is refused up front
    for gone in (3, -12, 3 * c):
        part = ctx.keygen(2001, [t for t in LR.rotation_steps(c, r, LR.ROWS, 1) if t != gone])
        with pytest.raises(H.HEError) as e:
            ctx.lr_grad_step(s["gZ"], s["gW"], mask, s["coef"], s["eta_n"], c, r, part)
        assert e.value.status == 5, gone
    # data terms of another plan (here another eta / n: another Z3 scale) are refused
    eta2 = s["eta_n"] * 64
    assert LR.plan_lr_step(P.q, P.L, P.delta, P.delta, s["coef"], eta2)["sZ3"] != s["pl"]["sZ3"]
    other = ctx.lr_data_terms(s["gZ"], s["gW"].level, s["gW"].scale, s["coef"], eta2)
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step(s["gZ"], s["gW"], mask, s["coef"], s["eta_n"], c, r, gk, Zk=other)
    assert e.value.status == 4  # HE_ESCALE
    good = ctx.lr_data_terms(s["gZ"], s["gW"].level, s["gW"].scale, s["coef"], s["eta_n"])
    n = len(s["gZ"])
    with pytest.raises(H.HEError) as e:  # the Z3 group where the Z1 group belongs
        ctx.lr_grad_step(s["gZ"], s["gW"], mask, s["coef"], s["eta_n"], c, r, gk, Zk=good[:n] + good[:n])
    assert e.value.status == 3  # HE_ELEVEL


def test_training_with_refresh_small(small):
    """Alg. 1 + Alg. 2 on the small workload: one step per refresh (4 levels);
    the trajectory follows FP64 plaintext training."""
    from paper_2006_10091_amd import train as T
    ctx, gk = small["ctx"], small["gkeys"]
    X, y = small["X"], small["y"]
    coef = _coef()
    w0 = synth.initial_weights("small", 16, small["W"]["seed_w"])
    rec = []
    w_final = T.train(ctx, gk, X, y, coef, 1.0, 3, 1, w0, 3003, mode=2, record=rec)
    w = w0.copy()
    for k in range(3):
        w = w + LR.lr_gradient_fp64(X, y, w, coef, 1.0 / X.shape[0])
        assert np.max(np.abs(rec[k] - w)) / np.max(np.abs(w)) < 2.0 ** -16, k
    assert np.max(np.abs(w_final - w)) / np.max(np.abs(w)) < 2.0 ** -16


@pytest.mark.parametrize("coef_name,w_decay", [("hinge", 0.0), ("binomial", 0.05)])
def test_lr_step_other_losses_bit_exact(small, coef_name, w_decay):
    """Table 2's hinge row (the x^2 product) and a regularised step, batched
    and graph forms, bit for bit against the oracle."""
    import os
    ctx, P = small["ctx"], small["P"]
    rows = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "table2_gradient_polynomials.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            rows[k] = [float(x) for x in v]
    coef = rows[coef_name]
    X, y = synth.small_data(n=600)
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    w0 = synth.initial_weights("small", 16, 77)
    oZ, gZ, oW, gW = _encrypt_small(small, blocks, w0)
    eta_n = 1.0 / 600
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n, w_decay)
    mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, small["okeys"], oZ, oW, mm, coef, eta_n, c, r, plan=pl)
    mask = ctx.pt_load(mm, P.L - 1, pl["s_mask"])
    zk = ctx.lr_data_terms(gZ, gW.level, gW.scale, coef, eta_n, w_decay)  # with Z2 for the hinge row
    assert len(zk) == (3 if coef[2] != 0 else 2) * len(gZ)
    for mode, terms in ((1, None), (2, None), (0, zk), (1, zk), (2, zk)):
        Wn, g = ctx.lr_grad_step(gZ, gW, mask, coef, eta_n, c, r, small["gkeys"], mode=mode, w_decay=w_decay,
                                 Zk=terms)
        assert np.array_equal(ctx.download(Wn), oWn.data), (mode, terms is not None)
        assert np.array_equal(ctx.download(g), og.data), (mode, terms is not None)


# ------------------------------------------------------------------ feature-major layout
def _table2(name):
    import os
    rows = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "table2_gradient_polynomials.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            rows[k] = [float(x) for x in v]
    return rows[name]


@pytest.fixture(scope="module")
def small40():
    """The small ring at scale 2^40 with keys for both layouts."""
    W = synth.WORKLOADS["small"]
    cfg = (13, 5, 2, 2, 40)
    P = O.Params(*cfg)
    ctx = _H().Context(*cfg)
    c, r = 16, P.S // 16
    steps = set(LR.rotation_steps(c, r))
    for nb in (2, 4, 16):  # the baby-step counts the tests take (2 and 4: hoisted giant sums)
        steps |= set(LR.rotation_steps(c, r, LR.FEATURES, nb))
    steps = sorted(steps)
    return dict(W=W, P=P, ctx=ctx, okeys=O.Keys(P, W["seed_keys"], rot_steps=steps),
                gkeys=ctx.keygen(W["seed_keys"], steps), H=_H())


@pytest.mark.parametrize("n_baby,n", [(4, 2048), (16, 700), (8, 256)])
def test_lr_step_row_major_baby_steps_bit_exact(small, n_baby, n):
    """Row-major column sums by baby steps over the rotated data (unit 1):
    the data copies and the step in its three forms, bit for bit against the
    oracle (16 = c: no giant step), and the decrypted g within 2^-20."""
    ctx, P, W, H = small["ctx"], small["P"], small["W"], small["H"]
    X, y = synth.small_data(n=n)
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    coef = _coef()
    w0 = synth.initial_weights("small", 16, 97)
    oZ, gZ = [], ctx.ct_block(blocks.shape[0], P.L)
    for i in range(blocks.shape[0]):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, small["okeys"], m, P.L, P.delta, W["seed_enc"], i))
        ctx.encrypt(ctx.pt_load(m, P.L, P.delta), small["gkeys"], W["seed_enc"], i, out=gZ[i])
    oZr = LR.rotate_data(P, small["okeys"], oZ, 1, n_baby)
    gZr = ctx.rotate_data(gZ, H.baby_unit(H.LAYOUT_ROWS, r), n_baby, small["gkeys"])
    for b in range(len(oZ)):
        for j in range(n_baby - 1):
            assert np.array_equal(ctx.download(gZr[b * (n_baby - 1) + j]), oZr[b][j].data), (b, j)
    mw = O.encode(LR.pack_weights(w0, P.S, c), P.delta, P.N)
    oW = O.encrypt_sk(P, small["okeys"], mw, P.L, P.delta, W["seed_enc"], 100005)
    gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), small["gkeys"], W["seed_enc"], 100005)
    eta_n = 1.0 / n
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n)
    mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, small["okeys"], oZ, oW, mm, coef, eta_n, c, r, plan=pl, Zrot=oZr, n_baby=n_baby)
    mask = ctx.pt_load(mm, P.L - 1, pl["s_mask"])
    for mode in (0, 1, 2, 2):
        Wn, g = ctx.lr_grad_step(gZ, gW, mask, coef, eta_n, c, r, small["gkeys"], mode=mode, Zrot=gZr,
                                 n_baby=n_baby)
        assert np.array_equal(ctx.download(Wn), oWn.data), mode
        assert np.array_equal(ctx.download(g), og.data), mode
    wdec = ctx.decrypt_decode(gW, small["gkeys"]).real[:16]
    gref = LR.lr_gradient_fp64(X, y, wdec, coef, eta_n)
    gd = ctx.decrypt_decode(g, small["gkeys"]).real.reshape(r, c)[:, :16]
    assert np.max(np.abs(gd - gref)) / np.max(np.abs(gref)) < TOL


@pytest.mark.parametrize("loss,w_decay,n", [("ls", 0.0, 2048), ("hinge", 0.0, 700), ("ls", 0.05, 300)])
def test_lr_step_feature_major_bit_exact(small40, loss, w_decay, n):
    """Feature-major step, plain, batched and graph-replayed forms, bit for bit
    against the oracle (full, ragged and single-block shards), and the
    decrypted g within 2^-20 of FP64."""
    small = small40
    ctx, P, W = small["ctx"], small["P"], small["W"]
    X, y = synth.small_data(n=n)
    blocks, c, r = LR.pack_blocks_features(X, y, P.S)
    coef = _coef() if loss == "ls" else _table2(loss)
    w0 = synth.initial_weights("small", 16, 91)
    oZ, gZ = [], ctx.ct_block(blocks.shape[0], P.L)
    for i in range(blocks.shape[0]):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, small["okeys"], m, P.L, P.delta, W["seed_enc"], i))
        ctx.encrypt(ctx.pt_load(m, P.L, P.delta), small["gkeys"], W["seed_enc"], i, out=gZ[i])
    mw = O.encode(LR.pack_weights_features(w0, P.S, c), P.delta, P.N)
    oW = O.encrypt_sk(P, small["okeys"], mw, P.L, P.delta, W["seed_enc"], 100001)
    gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), small["gkeys"], W["seed_enc"], 100001)
    eta_n = 1.0 / n
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n, w_decay, LR.FEATURES)
    mm = O.encode(LR.feature_mask(P.S, r), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, small["okeys"], oZ, oW, mm, coef, eta_n, c, r, plan=pl, layout=LR.FEATURES)
    H = small["H"]
    mask = ctx.pt_load(mm, H.mask_level(P.L, H.LAYOUT_FEATURES), pl["s_mask"])
    zk = ctx.lr_data_terms(gZ, gW.level, gW.scale, coef, eta_n, w_decay, H.LAYOUT_FEATURES)
    assert len(zk) == (3 if coef[2] != 0 else 2) * len(gZ)
    for mode, terms in ((0, None), (1, None), (2, None), (2, None), (0, zk), (1, zk), (2, zk)):
        Wn, g = ctx.lr_grad_step(gZ, gW, mask, coef, eta_n, c, r, small["gkeys"], mode=mode, w_decay=w_decay,
                                 layout=H.LAYOUT_FEATURES, Zk=terms)
        assert Wn.level == P.L - 4 and Wn.scale == pl["s_g"]
        assert np.array_equal(ctx.download(Wn), oWn.data), (mode, terms is not None)
        assert np.array_equal(ctx.download(g), og.data), (mode, terms is not None)
    wdec = ctx.decrypt_decode(gW, small["gkeys"]).real.reshape(c, r)[:16, 0]
    gref = LR.lr_gradient_fp64(X, y, wdec, coef, eta_n)
    gd = ctx.decrypt_decode(g, small["gkeys"]).real.reshape(c, r)[:16]
    assert np.max(np.abs(gd - gref[:, None])) / np.max(np.abs(gref)) < TOL


@pytest.mark.parametrize("n_baby,n", [(4, 700), (16, 700), (2, 256)])
def test_lr_step_feature_major_baby_steps_bit_exact(small40, n_baby, n):
    """Baby-step margins: he_rotate_many's copies of the data and the step in
    its three forms, bit for bit against the oracle (n_baby = 16 = c: no giant
    step), and the decrypted g within 2^-20 of FP64."""
    small = small40
    ctx, P, W, H = small["ctx"], small["P"], small["W"], small["H"]
    X, y = synth.small_data(n=n)
    blocks, c, r = LR.pack_blocks_features(X, y, P.S)
    coef = _coef()
    w0 = synth.initial_weights("small", 16, 93)
    oZ, gZ = [], ctx.ct_block(blocks.shape[0], P.L)
    for i in range(blocks.shape[0]):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, small["okeys"], m, P.L, P.delta, W["seed_enc"], i))
        ctx.encrypt(ctx.pt_load(m, P.L, P.delta), small["gkeys"], W["seed_enc"], i, out=gZ[i])
    oZr = LR.rotate_data(P, small["okeys"], oZ, r, n_baby)
    gZr = ctx.rotate_data(gZ, r, n_baby, small["gkeys"])
    assert len(gZr) == len(gZ) * (n_baby - 1)
    for b in range(len(oZ)):
        for j in range(n_baby - 1):
            assert np.array_equal(ctx.download(gZr[b * (n_baby - 1) + j]), oZr[b][j].data), (b, j)
    mw = O.encode(LR.pack_weights_features(w0, P.S, c), P.delta, P.N)
    oW = O.encrypt_sk(P, small["okeys"], mw, P.L, P.delta, W["seed_enc"], 100003)
    gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), small["gkeys"], W["seed_enc"], 100003)
    eta_n = 1.0 / n
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n, 0.0, LR.FEATURES)
    mm = O.encode(LR.feature_mask(P.S, r), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, small["okeys"], oZ, oW, mm, coef, eta_n, c, r, plan=pl, layout=LR.FEATURES,
                              Zrot=oZr, n_baby=n_baby)
    mask = ctx.pt_load(mm, H.mask_level(P.L, H.LAYOUT_FEATURES), pl["s_mask"])
    for mode in (0, 1, 2, 2):
        Wn, g = ctx.lr_grad_step(gZ, gW, mask, coef, eta_n, c, r, small["gkeys"], mode=mode,
                                 layout=H.LAYOUT_FEATURES, Zrot=gZr, n_baby=n_baby)
        assert np.array_equal(ctx.download(Wn), oWn.data), mode
        assert np.array_equal(ctx.download(g), og.data), mode
    wdec = ctx.decrypt_decode(gW, small["gkeys"]).real.reshape(c, r)[:16, 0]
    gref = LR.lr_gradient_fp64(X, y, wdec, coef, eta_n)
    gd = ctx.decrypt_decode(g, small["gkeys"]).real.reshape(c, r)[:16]
    assert np.max(np.abs(gd - gref[:, None])) / np.max(np.abs(gref)) < TOL


def test_lr_step_baby_step_errors(small40):
    """Baby-step arguments are checked before any launch: a count that is not a
    power of two or exceeds c, row-major, missing copies or keys."""
    small = small40
    ctx, P, H = small["ctx"], small["P"], small["H"]
    blocks, c, r = LR.pack_blocks_features(*synth.small_data(n=256), P.S)
    Z = ctx.ct_block(1, P.L)
    ctx.encrypt(ctx.pt_load(O.encode(blocks[0], P.delta, P.N), P.L, P.delta), small["gkeys"], 5, 0, out=Z[0])
    Wc = ctx.encrypt(ctx.pt_load(O.encode(np.zeros(P.S), P.delta, P.N), P.L, P.delta), small["gkeys"], 5, 1)
    coef = _coef()
    pl = ctx.plan_lr_step(P.L, P.delta, P.delta, coef, 1 / 256, layout=H.LAYOUT_FEATURES)
    mask = ctx.pt_load(O.encode(LR.feature_mask(P.S, r), pl["s_mask"], P.N), P.L - 3, pl["s_mask"])
    Zr4 = ctx.rotate_data(Z, r, 4, small["gkeys"])
    for kw in (dict(n_baby=3, Zrot=Zr4), dict(n_baby=32, Zrot=Zr4), dict(n_baby=4, Zrot=None)):
        with pytest.raises(H.HEError) as e:
            ctx.lr_grad_step(Z, Wc, mask, coef, 1 / 256, c, r, small["gkeys"], layout=H.LAYOUT_FEATURES, **kw)
        assert e.value.status == 1, kw
    with pytest.raises(H.HEError) as e:  # copies at a level below W's
        low = [ctx.drop_level(z, P.L - 1) for z in Zr4]
        ctx.lr_grad_step(Z, Wc, mask, coef, 1 / 256, c, r, small["gkeys"], layout=H.LAYOUT_FEATURES, Zrot=low,
                         n_baby=4)
    assert e.value.status in (1, 3)
    rk = ctx.keygen(3, [t for t in LR.rotation_steps(c, r, LR.FEATURES) if t != 3 * r])  # no baby step 3 r
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step(Z, Wc, mask, coef, 1 / 256, c, r, rk, layout=H.LAYOUT_FEATURES, Zrot=Zr4, n_baby=4)
    assert e.value.status == 5
    with pytest.raises(H.HEError) as e:
        ctx.rotate_many(Z, [3 * r], rk)
    assert e.value.status == 5


def test_lr_step_feature_major_errors(small, small40):
    """Wrong mask level, missing keys, an unknown layout and a data scale too
    small for the feature-major mask are refused before any launch."""
    ctx, P, H = small["ctx"], small["P"], small["H"]
    X, y = synth.small_data(n=256)
    blocks, c, r = LR.pack_blocks_features(X, y, P.S)
    Z = ctx.ct_block(1, P.L)
    ctx.encrypt(ctx.pt_load(O.encode(blocks[0], P.delta, P.N), P.L, P.delta), small["gkeys"], 5, 0, out=Z[0])
    Wc = ctx.encrypt(ctx.pt_load(O.encode(np.zeros(P.S), P.delta, P.N), P.L, P.delta), small["gkeys"], 5, 1)
    mask = ctx.pt_load(O.encode(LR.feature_mask(P.S, r), 2.0 ** 30, P.N), P.L - 3, 2.0 ** 30)
    with pytest.raises(H.HEError) as e:  # scale 2^30 data: the plan refuses the layout
        ctx.lr_grad_step(Z, Wc, mask, _coef(), 1 / 256, c, r, small["gkeys"], layout=H.LAYOUT_FEATURES)
    assert e.value.status == 4
    ctx, P = small40["ctx"], small40["P"]
    small = small40
    blocks, c, r = LR.pack_blocks_features(*synth.small_data(n=256), P.S)
    Z = ctx.ct_block(1, P.L)
    ctx.encrypt(ctx.pt_load(O.encode(blocks[0], P.delta, P.N), P.L, P.delta), small["gkeys"], 5, 0, out=Z[0])
    Wc = ctx.encrypt(ctx.pt_load(O.encode(np.zeros(P.S), P.delta, P.N), P.L, P.delta), small["gkeys"], 5, 1)
    coef = _coef()
    pl = ctx.plan_lr_step(P.L, P.delta, P.delta, coef, 1 / 256, layout=H.LAYOUT_FEATURES)
    mm = O.encode(LR.feature_mask(P.S, r), pl["s_mask"], P.N)
    bad_level = ctx.pt_load(mm, P.L - 1, pl["s_mask"])
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step(Z, Wc, bad_level, coef, 1 / 256, c, r, small["gkeys"], layout=H.LAYOUT_FEATURES)
    assert e.value.status == 3
    mask = ctx.pt_load(mm, P.L - 3, pl["s_mask"])
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step(Z, Wc, mask, coef, 1 / 256, c, r, small["gkeys"], layout=2)
    assert e.value.status == 1
    rk = ctx.keygen(3, LR.rotation_steps(c, r))  # row-major keys lack -16 .. -224
    with pytest.raises(H.HEError) as e:
        ctx.lr_grad_step(Z, Wc, mask, coef, 1 / 256, c, r, rk, layout=H.LAYOUT_FEATURES)
    assert e.value.status == 5
    for gone in (12, -12):  # taken only by the grouped sample sum and replication
        part = ctx.keygen(3, [t for t in LR.rotation_steps(c, r, LR.FEATURES) if t != gone])
        with pytest.raises(H.HEError) as e:
            ctx.lr_grad_step(Z, Wc, mask, coef, 1 / 256, c, r, part, layout=H.LAYOUT_FEATURES)
        assert e.value.status == 5, gone


# ------------------------------------------------------------------ rings below 2^12 (unfused kernels)
def test_small_ring_unfused_path_bit_exact():
    """N = 2^11 runs the stage-per-barrier NTT and the unfused key switch,
    rescale and rotate-and-add: products, rotations, the margins (grouped
    slot sum) and a whole row-major step (rescales of k Z read from the
    higher-level data) bit for bit against the oracle."""
    H = _H()
    cfg = (11, 5, 1, 1, 30)
    P = O.Params(*cfg)
    ctx = H.Context(*cfg)
    c, r = 16, P.S // 16
    steps = LR.rotation_steps(c, r)
    okeys, gkeys = O.Keys(P, 41, rot_steps=steps), ctx.keygen(41, steps)
    q = P.q
    def rct(level, seed):
        d = np.stack([synth.uniform_residues(seed, q[: level + 1], P.N), synth.uniform_residues(seed + 1, q[: level + 1],
                                                                                             P.N)])
        return d, ctx.upload(d, level, 1.0)
    xd, x = rct(P.L, 11)
    yd, y = rct(P.L, 13)
    want = O.rotate(P, O.rescale(P, O.mul(P, O.CT(xd, P.L, 1.0), O.CT(yd, P.L, 1.0), okeys)), 2, okeys)
    got = ctx.batch_mul_rotate([x], [y], [2], gkeys, mode=1)[0]
    assert np.array_equal(ctx.download(got), want.data)
    # the hoisted rotation sum and the multi-step rotations on the unfused key switch
    hs = [1, 2, 4]
    xs = ctx.ct_block(1, P.L)
    ctx.upload(xd, P.L, 1.0, out=xs[0])
    got = ctx.rotate_sum(xs, hs, gkeys)[0]
    assert np.array_equal(ctx.download(got), O.rotate_sum_hoisted(P, O.CT(xd, P.L, 1.0), hs, okeys).data)
    for s_, o in zip(hs, ctx.rotate_many(xs, hs, gkeys)):
        assert np.array_equal(ctx.download(o), O.rotate(P, O.CT(xd, P.L, 1.0), s_, okeys).data), s_
    X, yl = synth.small_data(n=r)
    blocks, c2, r2 = LR.pack_blocks(X, yl, P.S)
    assert (c2, r2) == (c, r)
    m = O.encode(blocks[0], P.delta, P.N)
    oZ = O.encrypt_sk(P, okeys, m, P.L, P.delta, 3, 0)
    gZ = ctx.ct_block(1, P.L)
    ctx.encrypt(ctx.pt_load(m, P.L, P.delta), gkeys, 3, 0, out=gZ[0])
    mw = O.encode(LR.pack_weights(synth.initial_weights("small", 16, 5), P.S, c), P.delta, P.N)
    oW = O.encrypt_sk(P, okeys, mw, P.L, P.delta, 3, 9)
    gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), gkeys, 3, 9)
    u = LR.lr_margins(P, okeys, [oZ], oW, c, r)[0]
    for mode in (0, 1):
        out = ctx.lr_margins(gZ, gW, c, r, gkeys, mode=mode)
        assert np.array_equal(ctx.download(out[0]), u.data), mode
    coef = _coef()
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, 1.0 / r, 0.0)
    mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, okeys, [oZ], oW, mm, coef, 1.0 / r, c, r, plan=pl)
    mask = ctx.pt_load(mm, P.L - 1, pl["s_mask"])
    for mode in (0, 1, 2):
        Wn, g = ctx.lr_grad_step(gZ, gW, mask, coef, 1.0 / r, c, r, gkeys, mode=mode)
        assert np.array_equal(ctx.download(Wn), oWn.data), mode
        assert np.array_equal(ctx.download(g), og.data), mode


# ------------------------------------------------------------------ encoding
@pytest.mark.parametrize("log_n,log_delta", [(13, 30), (16, 40)])
def test_encode_matches_oracle_encode(small, log_n, log_delta):
    """The library's host FP64 encode against the oracle's (a different FFT):
    every coefficient within 1, and a constant exactly (round(c Delta), 0, ...)."""
    H = small["H"]
    ctx = small["ctx"] if log_n == 13 else H.Context(16, 3, 1, 1, 40)
    N, S = 1 << log_n, 1 << (log_n - 1)
    delta = float(2 ** log_delta)
    g = np.random.default_rng(log_n)
    for z in (g.uniform(-1, 1, S), g.uniform(-1, 1, S) + 1j * g.uniform(-1, 1, S), g.uniform(0, 1, S // 3)):
        a = ctx.encode(z, delta)
        b = O.encode(z, delta, N)
        d = np.abs(a.astype(np.int64) - b.astype(np.int64))
        assert d.max() <= 1 and np.count_nonzero(d) < N // 100
    for cst in (0.75, -1.3125):
        want = np.zeros(N, dtype=np.int64)
        want[0] = int(round(cst * delta))
        assert np.array_equal(ctx.encode(np.full(S, cst), delta), want)
        assert np.array_equal(O.encode(np.full(S, cst), delta, N), want)


# ------------------------------------------------------------------ encrypted inference (margins)
@pytest.mark.parametrize("layout", [0, 1])
def test_margins_bit_exact_and_decrypt_to_inner_products(small, layout):
    """he_lr_margins in its three forms against the oracle's margins (product,
    rescale and grouped slot sum), bit for bit; the decrypted margins are w.z_i."""
    ctx, P, H = small["ctx"], small["P"], small["H"]
    X, y = synth.small_data(n=700)
    blocks, c, r = (LR.pack_blocks_features if layout else LR.pack_blocks)(X, y, P.S)
    w0 = synth.initial_weights("small", 16, 17)
    oZ, gZ = [], ctx.ct_block(blocks.shape[0], P.L)
    for i in range(blocks.shape[0]):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, small["okeys"], m, P.L, P.delta, 31, i))
        ctx.encrypt(ctx.pt_load(m, P.L, P.delta), small["gkeys"], 31, i, out=gZ[i])
    pw = LR.pack_weights_features(w0, P.S, c) if layout else LR.pack_weights(w0, P.S, c)
    mw = O.encode(pw, P.delta, P.N)
    level = P.L - 1
    oW = O.encrypt_sk(P, small["okeys"], mw, level, P.delta, 31, 500)
    gW = ctx.encrypt(ctx.pt_load(mw, level, P.delta), small["gkeys"], 31, 500)
    want = [u.data for u in LR.lr_margins(P, small["okeys"], oZ, oW, c, r, LR.FEATURES if layout else LR.ROWS)]
    for mode in (0, 1, 2, 2):
        out = ctx.lr_margins(gZ, gW, c, r, small["gkeys"], mode=mode, layout=layout)
        assert out[0].level == level - 1
        for o, wd in zip(out, want):
            assert np.array_equal(ctx.download(o), wd), mode
    z = y[:, None] * X
    m = z @ w0
    dec = ctx.decrypt_decode(out[1], small["gkeys"]).real
    grid = dec.reshape(c, r).T if layout else dec.reshape(r, c)
    assert np.max(np.abs(grid[:, 0] - m[r: 2 * r])) < 1e-5
