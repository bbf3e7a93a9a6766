"""The large shard at full size: 2^20 samples x 512 features (dense Gaussian,
labels from a random linear model with 10% flips) on one GPU, as one
worker's share of the paper's distributed training (Alg. 1).

N = 2^16, 24 ciphertext primes + 6 special primes (6 per digit), scale 2^40,
row-major blocks of 64 samples x 512 features: 16384 blocks.  The data are
encrypted by the server with sk as seeded ciphertexts (he_encrypt_seeded):
only the b components stay in HBM (192 GiB instead of 384 GiB), the uniform
parts are regenerated from their seeds chunk by chunk inside the step
(he_lr_grad_step_seeded).  5 gradient steps without refresh (levels 23, 19,
15, 11, 7), each checked against the FP64 gradient at the step's decrypted
input weights (2^-20, relative).

    python -m paper_2006_10091_amd.large_shard [--blocks 16384] [--steps 5] [--chunk 64]
"""
import argparse
import json
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import he as H
from . import synth


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def coef_binomial():
    # degree-3 least-squares fit of sigma(-m) on [-8, 8] (a0 = 1/2, a2 = 0 exactly)
    x, w = np.polynomial.legendre.leggauss(400)
    x, w = 8 * x, 8 * w
    G = np.array([[0.0 if (i + j) % 2 else 2 * 8.0 ** (i + j + 1) / (i + j + 1) for j in range(4)] for i in range(4)])
    rhs = np.array([np.sum(w / (1 + np.exp(x)) * x ** i) for i in range(4)])
    c = np.linalg.solve(G, rhs)
    return [0.5, float(c[1]), 0.0, float(c[3])]


def run(n_blocks=16384, steps=5, chunk=64, threads=8):
    import torch
    Wk = synth.WORKLOADS["large"]
    ctx = H.Context(Wk["logN"], Wk["nq"], Wk["nk"], Wk["alpha"], Wk["log_delta"])
    S, d = ctx.S, Wk["d"]
    c = d
    r = S // c
    n = n_blocks * r
    L = ctx.n_q - 1
    t0 = time.perf_counter()
    keys = ctx.keygen(Wk["seed_keys"], H.rotation_steps(c, r))
    torch.cuda.synchronize()
    log("keys: %d rotation keys (%.1f s)" % (len(H.rotation_steps(c, r)), time.perf_counter() - t0))
    Zs = ctx.seeded_block(n_blocks, L)
    seeded_gib = n_blocks * (L + 1) * ctx.N * 8 / 2 ** 30
    Zfp = np.empty((n, d), dtype=np.float64)  # y (.) X for the FP64 reference

    def make(b):
        X, y = synth.large_block(Wk["seed_data"], b, r, d)
        z = y[:, None] * X
        Zfp[b * r:(b + 1) * r] = z
        return ctx.encode(z.reshape(S), ctx.delta)  # row-major block: slot i*c + j

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        for b0 in range(0, n_blocks, 256):
            ms = list(ex.map(make, range(b0, min(n_blocks, b0 + 256))))
            for i, m in enumerate(ms):
                ctx.encrypt_seeded(ctx.pt_load(m, L, ctx.delta), keys, Wk["seed_enc"], b0 + i, out=Zs[b0 + i])
            if b0 % 4096 == 0:
                log("encrypted %d / %d blocks (%.0f s)" % (b0 + len(ms), n_blocks, time.perf_counter() - t0))
    torch.cuda.synchronize()
    t_enc = time.perf_counter() - t0
    log("data: %d x %d, %d seeded blocks, %.1f GiB in HBM (full ciphertexts: %.1f GiB); encoded and encrypted "
        "in %.1f s" % (n, d, n_blocks, seeded_gib, 2 * seeded_gib, t_enc))
    coef = coef_binomial()
    eta = 1.0 / n
    w = np.zeros(d)
    Wc = ctx.encrypt(ctx.pt_load(ctx.encode(H.pack_weights(w, S, c), ctx.delta), L, ctx.delta), keys,
                     Wk["seed_enc"], 1 << 30)
    za = (H.he_ct_seeded * n_blocks)(*[z.struct() for z in Zs])
    ws = ctx.step_seeded_bytes(L, L, chunk)
    log("workspace for chunks of %d blocks: %.1f GiB" % (chunk, ws / 2 ** 30))
    out = []
    t_steps = 0.0
    for k in range(steps):
        lv = Wc.level
        pl = ctx.plan_lr_step(lv, ctx.delta, Wc.scale, coef, eta)
        mask = ctx.pt_load(ctx.encode(H.column0_mask(S, c), pl["s_mask"]), lv - 1, pl["s_mask"])
        wdec = H.unpack_weights(ctx.decrypt_decode(Wc, keys).real, c, d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Wn, g = ctx.lr_grad_step_seeded(za, Wc, mask, coef, eta, c, r, keys, chunk)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_steps += dt
        m = Zfp @ wdec
        p = coef[0] + coef[1] * m + coef[2] * m * m + coef[3] * m ** 3
        gref = eta * (Zfp.T @ p)
        gd = H.unpack_weights(ctx.decrypt_decode(g, keys).real, c, d)
        rel = float(np.max(np.abs(gd - gref)) / np.max(np.abs(gref)))
        out.append(dict(step=k, level=lv, seconds=dt, grad_rel_err=rel))
        log("step %d at level %d: %.2f s (%.0f blocks/s), decrypted g rel err 2^%.1f" % (
            k, lv, dt, n_blocks / dt, np.log2(rel)))
        assert rel < 2.0 ** -20, rel
        Wc = Wn
    return dict(workload="large shard %d x %d, N=2^16, 24+6 primes, %d seeded blocks of %d samples, row-major, "
                         "chunks of %d blocks" % (n, d, n_blocks, r, chunk),
                steps_per_s=steps / t_steps, blocks_per_s=n_blocks * steps / t_steps, ms_per_step=t_steps / steps * 1e3,
                seeded_gib=seeded_gib, full_gib=2 * seeded_gib, encrypt_s=t_enc, workspace_gib=ws / 2 ** 30,
                steps=out, max_grad_rel_err=max(o["grad_rel_err"] for o in out))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks", type=int, default=16384)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--chunk", type=int, default=64)
    a = ap.parse_args(argv)
    res = run(a.blocks, a.steps, a.chunk)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
