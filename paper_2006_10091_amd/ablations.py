"""Training-loop ablations of Sec. 5.1 on one GPU, synthetic image-shaped shard.

Every variant trains logistic regression with the encrypted step (Alg. 1) and
the parameter server's refresh (Alg. 2) on this GPU, and is compared with the
same schedule run in plaintext FP64 (the paper's 'Plain' curve):

* ``refresh``  -- refresh period l in {1, 2, 3, 4} (the paper's Distributed-k,
  Fig. 'time'), each on the smallest prime chain that holds l steps of depth 4
  (4 l + 1 primes);
* ``modulus``  -- Distributed-var (Fig. 'modulus'): the l = 1 circuit on the
  full 20-prime chain instead of its 5-prime one, so every operation carries
  the larger modulus;
* ``lr``       -- learning rate in {0.25, 0.5, 1, 2, 4} at mini-batch 64;
* ``batch``    -- mini-batch size in {64, 128, 256, 512, full shard} at lr 1;
* ``loss``     -- the three rows of Table 2 (binomial, hinge, Huber).

A mini-batch of b samples is one packed group of ceil(b / r) blocks (rows past
b are zero) and takes eta / b; the shard is cut into floor(n / b) such groups,
visited in order.  Validation accuracy is the parameter server's: after each
refresh it evaluates its plaintext weights on a held-out set drawn from the
same generator.  Times are wall clock per iteration, refresh included.

Usage: python -m paper_2006_10091_amd.ablations [--what refresh,modulus,...]
       [--iterations K] [--n-train N] [--n-val M]
"""
import argparse
import json
import sys
import time

import numpy as np

from . import he as H
from . import synth
from .train import ParameterServer, Worker

# Table 2 rows as printed: a0 + a1 x + a2 x^2 + a3 x^3 approximating -L'(x)
TABLE2 = {
    "binomial": [0.5, -0.0843, 0.0, 0.0002],
    "hinge": [0.5875, -0.1005, 0.0008, -0.00039],
    "huber": [2.0, -0.1311, 0.0, 0.00005],
}


def ls_sigmoid(bound=8.0):
    """Degree-3 least-squares fit of sigma(-m) on [-bound, bound] (continuous
    L2; a0 = 1/2 and a2 = 0 by symmetry)."""
    x, w = np.polynomial.legendre.leggauss(400)
    x, w = bound * x, bound * w
    G = np.array([[0.0 if (i + j) % 2 else 2 * bound ** (i + j + 1) / (i + j + 1) for j in range(4)]
                  for i in range(4)])
    rhs = np.array([np.sum(w / (1 + np.exp(x)) * x ** i) for i in range(4)])
    c = np.linalg.solve(G, rhs)
    return [0.5, float(c[1]), 0.0, float(c[3])]


def plain_gradient(X, y, w, coef, eta_over_n):
    """(eta/n) sum_i p(y_i w.x_i) y_i x_i in FP64 -- the unencrypted step."""
    z = y[:, None] * X
    m = z @ w
    p = coef[0] + m * (coef[1] + m * (coef[2] + m * coef[3]))
    return eta_over_n * (p[:, None] * z).sum(0)


def accuracy(X, y, w):
    return float(np.mean(np.where(X @ w >= 0, 1.0, -1.0) == y))


def minibatches(n, batch):
    """Index ranges of the mini-batches, visited in order (remainder dropped
    unless the whole shard is one batch)."""
    if batch >= n:
        return [(0, n)]
    return [(k * batch, (k + 1) * batch) for k in range(n // batch)]


def schedule(iterations, refresh_every):
    """Iterations after which the worker asks for a refresh (Alg. 1)."""
    return [k for k in range(1, iterations + 1) if k % refresh_every == 0 or k == iterations]


class Run:
    """One variant: context, keys, encrypted mini-batches, worker per batch."""

    def __init__(self, n_q, Xtr, ytr, batch, seed_keys=2002, seed_enc=3002):
        W = synth.WORKLOADS["image"]
        self.ctx = ctx = H.Context(W["logN"], n_q, W["nk"], W["alpha"], W["log_delta"])
        self.Xtr, self.ytr, self.batch = Xtr, ytr, batch
        n, d = Xtr.shape
        self.ranges = minibatches(n, batch)
        blocks0, c, r = H.pack_blocks(Xtr[: min(batch, n)], ytr[: min(batch, n)], ctx.S)
        self.c, self.r = c, r
        self.keys = ctx.keygen(seed_keys, H.rotation_steps(c, r))  # the row-major step's rotations
        L = ctx.n_q - 1
        self.Z = []
        idx = 0
        for lo, hi in self.ranges:
            blocks, _, _ = H.pack_blocks(Xtr[lo:hi], ytr[lo:hi], ctx.S)
            Zb = ctx.ct_block(blocks.shape[0], L)
            for i in range(blocks.shape[0]):
                ctx.encrypt(ctx.pt_load(ctx.encode(blocks[i], ctx.delta), L, ctx.delta), self.keys, seed_enc, idx,
                            out=Zb[i])
                idx += 1
            self.Z.append(Zb)

    def train(self, coef, eta, iterations, refresh_every, Xval, yval, mode):
        """Runs the schedule twice and reports the second run (the first one
        captures the graphs and grows the workspace)."""
        self._train(coef, eta, min(iterations, refresh_every * len(self.ranges)), refresh_every, Xval, yval, mode)
        return self._train(coef, eta, iterations, refresh_every, Xval, yval, mode)

    def _train(self, coef, eta, iterations, refresh_every, Xval, yval, mode):
        """Encrypted training and the same schedule in FP64.  Returns per
        refresh: (iteration, seconds so far, validation accuracy, relative
        deviation of the server's weights from the FP64 trajectory, relative
        deviation from FP64 steps started at the previous refresh's weights)."""
        import torch
        ctx, keys = self.ctx, self.keys
        d = self.Xtr.shape[1]
        ps = ParameterServer(ctx, keys, d, self.c, 3002)
        workers = [Worker(ctx, keys, Zb, coef, eta / (hi - lo), self.c, self.r, mode=mode)
                   for Zb, (lo, hi) in zip(self.Z, self.ranges)]
        w_plain = np.zeros(d)
        W = ps.encrypt_weights(w_plain)
        w_period = ps.w.copy()
        refresh_at = set(schedule(iterations, refresh_every))
        trace = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(1, iterations + 1):
            j = (k - 1) % len(self.ranges)
            lo, hi = self.ranges[j]
            if W.level < 4:
                raise ValueError("refresh period %d needs more than %d primes" % (refresh_every, ctx.n_q))
            W, _ = workers[j].step(W)
            w_plain = w_plain + plain_gradient(self.Xtr[lo:hi], self.ytr[lo:hi], w_plain, coef, eta / (hi - lo))
            w_period = w_period + plain_gradient(self.Xtr[lo:hi], self.ytr[lo:hi], w_period, coef, eta / (hi - lo))
            if k in refresh_at:
                W = ps.refresh(W)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                dev = float(np.max(np.abs(ps.w - w_plain)) / max(np.max(np.abs(w_plain)), 1e-300))
                dev_p = float(np.max(np.abs(ps.w - w_period)) / max(np.max(np.abs(w_period)), 1e-300))
                trace.append((k, el, accuracy(Xval, yval, ps.w), dev, dev_p))
                w_period = ps.w.copy()
                t0 += time.perf_counter() - t0 - el  # the evaluation stays off the clock
        return trace, accuracy(Xval, yval, w_plain)


def summarise(name, trace, acc_plain, iterations):
    k, el, acc = trace[-1][:3]
    return {"variant": name, "iterations": iterations, "seconds": el, "ms_per_iteration": el / iterations * 1e3,
            "val_acc": acc, "val_acc_plain": acc_plain, "max_rel_dev_vs_plain": max(t[3] for t in trace),
            "max_rel_dev_per_period": max(t[4] for t in trace),
            "best_val_acc": max(t[2] for t in trace),
            "seconds_to_best": min(t[1] for t in trace if t[2] == max(u[2] for u in trace))}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--what", default="refresh,modulus,lr,batch,loss")
    ap.add_argument("--iterations", type=int, default=12)
    ap.add_argument("--n-train", type=int, default=6000)
    ap.add_argument("--n-val", type=int, default=1000)
    args = ap.parse_args(argv)
    what = args.what.split(",")
    X, y = synth.image_data(1002, args.n_train + args.n_val)
    Xtr, ytr, Xval, yval = X[: args.n_train], y[: args.n_train], X[args.n_train:], y[args.n_train:]
    K = args.iterations
    coef = ls_sigmoid(8.0)
    rows = []

    def emit(group, name, trace, acc_plain, iters=K):
        s = summarise(name, trace, acc_plain, iters)
        s["group"] = group
        s["trace"] = [[t[0], round(t[1], 4), t[2]] for t in trace]
        rows.append(s)
        print(json.dumps(s), flush=True)

    runs = {}

    def run(n_q, batch):
        key = (n_q, batch)
        if key not in runs:
            runs.clear()  # one variant's keys and shard resident at a time
            import torch
            torch.cuda.empty_cache()
            runs[key] = Run(n_q, Xtr, ytr, batch)
        return runs[key]

    full = args.n_train
    if "refresh" in what:
        for l in (1, 2, 3, 4):
            R = run(4 * l + 1, full)
            trace, ap_ = R.train(coef, 1.0, K, l, Xval, yval, mode=2)
            emit("refresh", "Distributed-%d (%d primes)" % (l, 4 * l + 1), trace, ap_)
    if "modulus" in what:
        R = run(20, full)
        trace, ap_ = R.train(coef, 1.0, K, 1, Xval, yval, mode=2)
        emit("modulus", "Distributed-var: l=1 on 20 primes", trace, ap_)
        R = run(5, full)
        trace, ap_ = R.train(coef, 1.0, K, 1, Xval, yval, mode=2)
        emit("modulus", "Distributed: l=1 on 5 primes", trace, ap_)
    if "lr" in what:
        for eta in (0.25, 0.5, 1.0, 2.0, 4.0):
            R = run(17, 64)
            trace, ap_ = R.train(coef, eta, 4 * K, 4, Xval, yval, mode=1)
            emit("lr", "lr %g, batch 64" % eta, trace, ap_, 4 * K)
    if "batch" in what:
        for b in (64, 128, 256, 512, full):
            R = run(17, b)
            trace, ap_ = R.train(coef, 1.0, 4 * K, 4, Xval, yval, mode=1 if b < full else 2)
            emit("batch", "batch %d, lr 1" % b, trace, ap_, 4 * K)
    if "loss" in what:
        for name, cf in TABLE2.items():
            R = run(17, full)
            trace, ap_ = R.train(cf, 1.0, K, 4, Xval, yval, mode=2)
            emit("loss", "Table 2 %s" % name, trace, ap_)
    print(markdown(rows), flush=True)
    return rows


def markdown(rows):
    out = ["| group | variant | iters | ms/iter | val acc | plain acc | best acc | s to best | dev (trajectory) "
           "| dev (per period) |",
           "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for s in rows:
        out.append("| %s | %s | %d | %.1f | %.4f | %.4f | %.4f | %.2f | %.2e | %.2e |" % (
            s["group"], s["variant"], s["iterations"], s["ms_per_iteration"], s["val_acc"], s["val_acc_plain"],
            s["best_val_acc"], s["seconds_to_best"], s["max_rel_dev_vs_plain"], s["max_rel_dev_per_period"]))
    return "\n".join(out)


if __name__ == "__main__":
    main(sys.argv[1:])
