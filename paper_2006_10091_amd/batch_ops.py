"""Batched ciphertext operations of mixed ring degree and level.

The workload: a batch of independent multiply -> relinearise -> rescale ->
rotate operations (the operations the gradient step is built from, Sec. 3)
whose ring degree N is drawn from {2^14, 2^15, 2^16}, level from [3, 20] and
rotation step from the powers of two below N/2, with uniform random residues
as inputs.  One context (and key set) per N, each with 21 ciphertext primes
and 4 special primes (scale 2^40, 4 primes per digit).  Each context's share
runs through he_batch_mul_rotate: entries of one level together, up to 32 per
launch, each with its own rotation key; in the graph form one captured graph
per context replays the whole share.  The same share also runs as a list of
operation descriptors through he_batch_submit (HE_OP_MUL_ROTATE entries):
its tensor products and result copies are one table-driven launch each over
all levels.

Usage: python -m paper_2006_10091_amd.batch_ops [--ops 256] [--reps 3]
"""
import argparse
import json
import sys
import time

import numpy as np

from . import he as H
from . import synth

LOG_NS = (14, 15, 16)
CHAIN = dict(n_q=21, n_special=4, alpha=4, log_delta=40)


def draw_ops(n_ops, seed=3003):
    """(log_n, level, step) per op, seeded."""
    g = synth.rng(seed)
    ops = []
    for _ in range(n_ops):
        log_n = int(g.choice(LOG_NS))
        level = int(g.integers(3, 21))
        u = int(g.integers(0, log_n - 1))
        ops.append((log_n, level, 1 << u))
    return ops


class Batch:
    """Contexts, keys and input/output ciphertexts of one mixed batch.

    streams: each ring degree's context works on a HIP stream of its own
    (default priority), so the three shares of the batch, which share no
    data, run concurrently; every allocation of a share is made on its
    stream.  Otherwise all contexts use the current stream, one after
    another."""

    def __init__(self, ops, seed=5003, streams=False):
        import torch
        self.torch = torch
        self.ops = ops
        self.ctx, self.keys, self.stream = {}, {}, {}
        self.x, self.y, self.out, self.idx = {}, {}, {}, {}
        for log_n in sorted({o[0] for o in ops}):
            st = torch.cuda.Stream() if streams else torch.cuda.current_stream()
            self.stream[log_n] = st
            with torch.cuda.stream(st):
                ctx = H.Context(log_n, CHAIN["n_q"], CHAIN["n_special"], CHAIN["alpha"], CHAIN["log_delta"])
                self.ctx[log_n] = ctx
                self.keys[log_n] = ctx.keygen(2003 + log_n, [1 << u for u in range(log_n - 1)])
            self.x[log_n], self.y[log_n], self.out[log_n], self.idx[log_n] = [], [], [], []
        for i, (log_n, level, _) in enumerate(ops):
            ctx = self.ctx[log_n]
            q = ctx.primes[: level + 1]
            with torch.cuda.stream(self.stream[log_n]):
                for dst, s in ((self.x, seed + 2 * i), (self.y, seed + 2 * i + 100003)):
                    d = np.stack([synth.uniform_residues(s, q, ctx.N), synth.uniform_residues(s + 1, q, ctx.N)])
                    dst[log_n].append(ctx.upload(d, level, 1.0))
                self.out[log_n].append(ctx.ct_empty(level - 1))
            self.idx[log_n].append(i)
        torch.cuda.synchronize()

    def run(self, mode):
        for log_n, ctx in self.ctx.items():
            steps = [self.ops[i][2] for i in self.idx[log_n]]
            with self.torch.cuda.stream(self.stream[log_n]):
                ctx.batch_mul_rotate(self.x[log_n], self.y[log_n], steps, self.keys[log_n], mode=mode,
                                     outs=self.out[log_n])

    def run_submit(self, mode):
        """The same operations as descriptors through he_batch_submit."""
        if not hasattr(self, "_desc"):
            self._desc = {log_n: [(H.OP_MUL_ROTATE, self.ops[i][2], x, y, o)
                                  for i, x, y, o in zip(self.idx[log_n], self.x[log_n], self.y[log_n], self.out[log_n])]
                          for log_n in self.ctx}
        for log_n, ctx in self.ctx.items():
            with self.torch.cuda.stream(self.stream[log_n]):
                ctx.batch_submit(self._desc[log_n], self.keys[log_n], mode=mode)

    def outputs(self):
        res = [None] * len(self.ops)
        for log_n, ctx in self.ctx.items():
            for i, o in zip(self.idx[log_n], self.out[log_n]):
                res[i] = ctx.download(o)
        return res


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--ops", type=int, default=256)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    ops = draw_ops(args.ops)
    ref = None
    result = {"ops": args.ops, "per_n": {str(1 << k): sum(1 for o in ops if o[0] == k) for k in LOG_NS}}
    for streams in (False, True):
        b = Batch(ops, streams=streams)
        forms = ((0, "plain", b.run), (1, "batched", b.run), (2, "graph", b.run), (1, "submit", b.run_submit),
                 (2, "submit_graph", b.run_submit))
        if streams:  # the concurrent shares: the batched forms only
            forms = tuple((m, n + "_streams", r) for m, n, r in forms[1:])
        for mode, name, run in forms:
            run(mode)  # first run: workspace growth, graph capture
            torch.cuda.synchronize()
            out = b.outputs()
            if ref is None:
                ref = out
            assert all(np.array_equal(a, r) for a, r in zip(out, ref)), name
            t0 = time.perf_counter()
            for _ in range(args.reps):
                run(mode)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.reps
            result[name + "_ms_per_batch"] = dt * 1e3
            result[name + "_ops_per_s"] = args.ops / dt
            print("%s: %.2f ms per batch of %d ops (%.0f ops/s)" % (name, dt * 1e3, args.ops, args.ops / dt),
                  file=sys.stderr, flush=True)
        del b
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    result["graph_over_plain"] = result["graph_ops_per_s"] / result["plain_ops_per_s"]
    print(json.dumps(result), flush=True)
    return result


if __name__ == "__main__":
    main(sys.argv[1:])
