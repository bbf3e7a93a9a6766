"""Benchmark: encrypted logistic-regression gradient steps/s on one MI355X.

Workload (the headline configuration): one server's shard of 6000 two-class
14x14 images (196 features; synthetic stand-in for the paper's MNIST 3-vs-8,
Sec. 5.1), packed row-major into 47 blocks of 128 rows x 256 columns,
RNS-CKKS at N = 2^16 with 20 ciphertext primes (scale 2^40) and 4 special
primes (3 digits of 4... dnum 5), one gradient step of eq. (appr) + eq. (update)
per timed step, taken at the top level (the most expensive step of a refresh
period).

value = batched form (every block in one launch per operation, replayed from
a captured HIP graph); plain form (one operation per block) and batched
without graph are reported beside it.  Inputs are resident in HBM before the
timed region.  The roofline entry measures the dominant kernel's average
launch time with HIP events on the stream it runs on; cpu_baseline times the
CPU oracle on a bounded sample (one instance of each distinct key-switching
operation of the step) and extrapolates by the operation counts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of one forward NTT over the 5640-limb digit batch, from
# FETCH_SIZE (x2, copy-calibrated) + WRITE_SIZE (x1) runs of the current
# kernels (profiles/ntt_forward_5640_limbs_pmc.md).  Set to None whenever the
# NTT kernels change until the counters are taken again.
NTT_TRAFFIC_BYTES = {5640: (2889540 + 4059300 + 2 * 2887680) * 1024}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--workload", default="image")
    return ap.parse_args()


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


class Events:
    """HIP event timing on a given stream (torch.cuda.Event on that stream)."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def time(self, fn, reps):
        t = self.torch
        s, e = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        with t.cuda.stream(self.stream):
            s.record(self.stream)
            for _ in range(reps):
                fn()
            e.record(self.stream)
        e.synchronize()
        return s.elapsed_time(e) / reps / 1e3  # seconds per call


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is designed, not built"}))
        sys.exit(2)
    import torch
    from paper_2006_10091_amd import he as H
    from paper_2006_10091_amd import synth

    torch.cuda.set_device(0)
    Wk = synth.WORKLOADS[args.workload]
    ctx = H.Context(Wk["logN"], Wk["nq"], Wk["nk"], Wk["alpha"], Wk["log_delta"])
    N, S, L = ctx.N, ctx.S, ctx.n_q - 1
    log("ctx: N=2^%d, %d+%d primes, dnum %d" % (Wk["logN"], Wk["nq"], Wk["nk"], ctx.dnum))
    t0 = time.time()
    if args.workload == "image":
        X, y = synth.image_data(Wk["seed_data"], Wk["n"])
    else:
        X, y = synth.small_data(Wk["seed_data"], Wk["n"], Wk["d"])
    blocks, c, r = H.pack_blocks(X, y, S)
    nb = blocks.shape[0]
    n = X.shape[0]
    log("data: %d x %d -> %d blocks of %d x %d (%.1fs)" % (n, X.shape[1], nb, r, c, time.time() - t0))
    steps = []
    t = 1
    while t < c:
        steps += [t, -t]
        t *= 2
    t = 1
    while t < r:
        steps.append(t * c)
        t *= 2
    t0 = time.time()
    keys = ctx.keygen(Wk["seed_keys"], steps)
    torch.cuda.synchronize()
    log("keygen: relin + %d rotation keys (%.1fs)" % (len(steps), time.time() - t0))
    t0 = time.time()
    Z = ctx.ct_block(nb, L)
    for i in range(nb):
        ctx.encrypt(ctx.pt_load(ctx.encode(blocks[i], ctx.delta), L, ctx.delta), keys, Wk["seed_enc"], i, out=Z[i])
    w0 = synth.initial_weights(args.workload, X.shape[1], Wk["seed_w"])
    Wc = ctx.encrypt(ctx.pt_load(ctx.encode(H.pack_weights(w0, S, c), ctx.delta), L, ctx.delta), keys,
                     Wk["seed_enc"], 1 << 20)
    coef = coef_binomial()
    eta_n = 1.0 / n
    pl = ctx.plan_lr_step(L, ctx.delta, Wc.scale, coef, eta_n)
    mask = ctx.pt_load(ctx.encode(H.column0_mask(S, c), pl["s_mask"]), L - 1, pl["s_mask"])
    Wout, Gout = ctx.ct_empty(L - 4), ctx.ct_empty(L - 4)
    torch.cuda.synchronize()
    log("encrypt %d blocks + weights (%.1fs)" % (nb, time.time() - t0))

    stream = torch.cuda.current_stream()
    ev = Events(torch, stream)

    def step(mode):
        ctx.lr_grad_step(Z, Wc, mask, coef, eta_n, c, r, keys, mode=mode, W_out=Wout, G_out=Gout)

    # correctness of the timed configuration: forms agree bit for bit, g within 2^-20
    step(0)
    ref_w, ref_g = ctx.download(Wout), ctx.download(Gout)
    step(2)
    assert np.array_equal(ctx.download(Wout), ref_w) and np.array_equal(ctx.download(Gout), ref_g)
    wdec = ctx.decrypt_decode(Wc, keys).real[: X.shape[1]]
    z = y[:, None] * X
    m = z @ wdec
    gref = eta_n * ((coef[0] + coef[1] * m + coef[3] * m ** 3)[:, None] * z).sum(0)
    gdec = ctx.decrypt_decode(Gout, keys).real[: X.shape[1]]
    rel = float(np.max(np.abs(gdec - gref)) / np.max(np.abs(gref)))
    log("parity: plain == batched (bit-exact); decrypted g rel err %.3g (2^%.1f)" % (rel, np.log2(rel)))

    for _ in range(args.warmup):
        step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    value = args.steps / dt
    log("batched+graph: %.2f ms/step, %.3f steps/s" % (ms, value))
    step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.plain_steps)):
        step(1)
    torch.cuda.synchronize()
    batched_nograph = max(1, args.plain_steps) / (time.perf_counter() - t0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.plain_steps)):
        step(0)
    torch.cuda.synchronize()
    plain = max(1, args.plain_steps) / (time.perf_counter() - t0)
    log("batched (no graph): %.3f steps/s; plain per-op: %.3f steps/s" % (batched_nograph, plain))

    # dominant kernel: the NTT over the step's key-switching digit batch
    # (nb blocks x dnum digits x (L+1+k) limbs, forward), timed with events
    nlimb = nb * ctx.dnum * (L + 1 + ctx.n_special) // 4 * 4
    period = L + 1
    nlimb = (nlimb // period) * period
    buf = torch.randint(0, 1 << 40, (nlimb * N,), dtype=torch.int64, device="cuda")
    ctx.ntt(buf, nlimb, 0, period, +1)
    ctx.ntt(buf, nlimb, 0, period, -1)
    t_fwd = ev.time(lambda: ctx.ntt(buf, nlimb, 0, period, +1), 5)
    t_inv = ev.time(lambda: ctx.ntt(buf, nlimb, 0, period, -1), 5)
    alg_bytes = 16.0 * N * nlimb  # read + write each limb once
    ntt_gbs = alg_bytes / t_fwd / 1e9
    log("NTT fwd %d limbs: %.3f ms (%.0f GB/s algorithmic); inv %.3f ms" % (nlimb, t_fwd * 1e3, ntt_gbs, t_inv * 1e3))
    del buf

    out = {
        "metric": "encrypted LR grad steps/s at N=2^16 (batched vs plain) + NTT HBM GB/s",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "image-shard 6000x196, N=2^16, 20+4 primes, dnum 5, scale 2^40, 47 blocks, "
                               "top-level step, batched form replayed from a HIP graph",
                   "n": n, "d": int(X.shape[1]), "blocks": nb, "log_n": Wk["logN"], "n_q": Wk["nq"],
                   "n_special": Wk["nk"]},
        "plain_steps_per_s": plain,
        "batched_nograph_steps_per_s": batched_nograph,
        "batched_over_plain": value / plain,
        "ntt_fwd_gbs_algorithmic": ntt_gbs,
        "ntt_inv_gbs_algorithmic": alg_bytes / t_inv / 1e9,
        "decrypted_grad_rel_err": rel,
        "roofline": {"bound": "hbm", "achieved": ntt_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ntt_gbs / HBM_PEAK_GBS, "traffic": NTT_TRAFFIC_BYTES.get(nlimb),
                     "kernel": "ntt (forward, two passes) over %d limbs of N=2^16" % nlimb},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(Wk, args.cpu_threads, nb, c, r)
    print(json.dumps(out), flush=True)


def cpu_baseline(Wk, threads, nb, c, r):
    """The oracle timed on one instance of each distinct key-switching
    operation of the step, extrapolated linearly by the counts in one step."""
    if threads:
        os.environ["OMP_NUM_THREADS"] = str(threads)
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    from oracle import ckks as O
    from paper_2006_10091_amd import synth
    P = O.Params(Wk["logN"], Wk["nq"], Wk["nk"], Wk["alpha"], Wk["log_delta"])
    L = P.L
    keys = O.Keys.__new__(O.Keys)
    keys.P, keys.seed = P, 7
    keys.s = np.zeros(P.N, dtype=np.int64)
    O.lib().orc_keygen_secret(P.cp, 7, O.HWT, O._i(keys.s))
    nfull = P.nq + P.nk
    sp = np.zeros((nfull, P.N), dtype=np.uint64)
    O.lib().orc_secret_square(P.cp, O._i(keys.s), O._u(sp))
    t0 = time.time()
    keys.rlk = keys._evk(sp, 0)
    keys.rot = {}
    keys.add_rotation(1)
    t_keys = time.time() - t0

    def ct(level, seed):
        return O.CT(np.stack([synth.uniform_residues(seed, P.q[: level + 1], P.N),
                              synth.uniform_residues(seed + 1, P.q[: level + 1], P.N)]), level, 1.0)

    def t_mul(level):
        x, y = ct(level, 1), ct(level, 3)
        t = time.time()
        O.rescale(P, O.mul(P, x, y, keys))
        return time.time() - t

    def t_rot(level):
        x = ct(level, 5)
        t = time.time()
        O.rotate(P, x, 1, keys)
        return time.time() - t

    lc, lr = int(np.log2(c)), int(np.log2(r))
    sample = {"mul19": t_mul(L), "rot18": t_rot(L - 1), "rot17": t_rot(L - 2), "mul17": t_mul(L - 2),
              "mul16": t_mul(L - 3), "rot15": t_rot(L - 4)}
    t_step = nb * (sample["mul19"] + lc * sample["rot18"] + lc * sample["rot17"] + 3 * sample["mul17"] +
                   sample["mul16"]) + lr * sample["rot15"]
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": nthreads, "kind": "oracle",
            "sample": "one oracle run of each distinct key-switching op of the step (mul+relin+rescale at "
                      "levels 19/17/16, rotation at 18/17/15; %.1fs total, keys %.1fs), extrapolated by the "
                      "per-step counts (%d blocks x (1+%d+%d+3+1) + %d)" % (sum(sample.values()), t_keys, nb, lc,
                                                                           lc, lr),
            "extrapolated": True, "sample_seconds": sample}


if __name__ == "__main__":
    main()
