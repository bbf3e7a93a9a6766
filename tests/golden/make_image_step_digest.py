"""Writes image_step_digest.json: the oracle's result for one top-level
gradient step on the whole 47-block image shard (6000 x 196 stand-in for the
paper's MNIST 3-vs-8 workload at 14 x 14; N = 2^16, 20 + 4 primes, dnum 5,
scale 2^40), feature-major packing with 16 baby steps and the hoisted giant
sum -- the configuration the bench times.

Calls only the oracle (and the seeded input generator).  The digest holds
SHA-256 hashes of W' and g in canonical coefficient form, a sample of their
coefficients, and hashes of the plaintexts so that a consumer can tell a
different encoding from a different step.  Runs for about an hour on 8 cores.

    python tests/golden/make_image_step_digest.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ckks as O  # noqa: E402
from oracle import lr as LR  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "image_step_digest.json")
SPEC = dict(workload="image", layout="features", n_baby=16, seed_w=4002, w_range=0.05, enc_seed=3002,
            w_index=100000, eta_over_n="1/6000", coef="[0.5, ls8[1], 0, ls8[3]]")


def inputs(P):
    """The step's inputs (plaintext integer coefficients), shared by the oracle
    run and any consumer of the digest."""
    W = synth.WORKLOADS["image"]
    X, y = synth.image_data(W["seed_data"], W["n"])
    blocks, c, r = LR.pack_blocks_features(X, y, P.S)
    w0 = synth.rng(SPEC["seed_w"]).uniform(-SPEC["w_range"], SPEC["w_range"], X.shape[1])
    ls = LR.grad_poly_binomial(8.0)
    coef = [0.5, float(ls[1]), 0.0, float(ls[3])]
    eta_n = 1.0 / X.shape[0]
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n, 0.0, LR.FEATURES)
    mz = [O.encode(blocks[i], P.delta, P.N) for i in range(blocks.shape[0])]
    mw = O.encode(LR.pack_weights_features(w0, P.S, c), P.delta, P.N)
    mm = O.encode(LR.feature_mask(P.S, r), pl["s_mask"], P.N)
    return dict(X=X, y=y, c=c, r=r, w0=w0, coef=coef, eta_n=eta_n, plan=pl, mz=mz, mw=mw, mm=mm)


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()


def pt_hash(inp):
    h = hashlib.sha256()
    for m in inp["mz"] + [inp["mw"], inp["mm"]]:
        h.update(np.ascontiguousarray(m, dtype=np.int64).tobytes())
    return h.hexdigest()


def sample_positions(level, N, count=64, seed=77):
    g = np.random.default_rng(seed)
    return [(int(cc), int(li), int(k)) for cc, li, k in
            zip(g.integers(0, 2, count), g.integers(0, level + 1, count), g.integers(0, N, count))]


def main():
    W = synth.WORKLOADS["image"]
    P = O.Params(W["logN"], W["nq"], W["nk"], W["alpha"], W["log_delta"])
    t0 = time.time()
    inp = inputs(P)
    c, r, n_baby = inp["c"], inp["r"], SPEC["n_baby"]
    steps = LR.rotation_steps(c, r, LR.FEATURES, n_baby)
    keys = O.Keys(P, W["seed_keys"], rot_steps=steps)
    print("keys %.0f s" % (time.time() - t0), flush=True)
    Z = [O.encrypt_sk(P, keys, m, P.L, P.delta, SPEC["enc_seed"], i) for i, m in enumerate(inp["mz"])]
    Wc = O.encrypt_sk(P, keys, inp["mw"], P.L, P.delta, SPEC["enc_seed"], SPEC["w_index"])
    print("encrypted %d blocks %.0f s" % (len(Z), time.time() - t0), flush=True)
    Zrot = []
    for b, zb in enumerate(Z):
        Zrot.append([O.rotate(P, zb, j * r, keys) for j in range(1, n_baby)])
        print("baby copies of block %d %.0f s" % (b, time.time() - t0), flush=True)
    Wn, g = LR.lr_grad_step(P, keys, Z, Wc, inp["mm"], inp["coef"], inp["eta_n"], c, r, plan=inp["plan"],
                            layout=LR.FEATURES, Zrot=Zrot, n_baby=n_baby)
    print("step %.0f s" % (time.time() - t0), flush=True)
    wdec = O.decrypt(P, keys, Wc).real.reshape(c, r)[:196, 0]
    gref = LR.lr_gradient_fp64(inp["X"], inp["y"], wdec, inp["coef"], inp["eta_n"])
    gd = O.decrypt(P, keys, g).real.reshape(c, r)
    rel = max(float(np.max(np.abs(gd[:196, i] - gref)) / np.max(np.abs(gref))) for i in range(r))
    pos = sample_positions(Wn.level, P.N)
    out = dict(spec=SPEC, level_out=Wn.level, scale_out=Wn.scale, plaintext_sha256=pt_hash(inp),
               w_out_sha256=sha(Wn.data), g_sha256=sha(g.data), grad_rel_err_vs_fp64=rel,
               w_out_sample=[[cc, li, k, int(Wn.data[cc, li, k])] for cc, li, k in pos],
               g_sample=[[cc, li, k, int(g.data[cc, li, k])] for cc, li, k in pos],
               oracle_seconds=round(time.time() - t0))
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT, "rel err 2^%.1f" % np.log2(rel), flush=True)


if __name__ == "__main__":
    main()
