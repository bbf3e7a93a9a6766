"""Serving encrypted gradient steps and encrypted inferences with continuous batching.

Requests arrive as a Poisson stream.  Each is either a gradient step (eq.
(appr) + eq. (update) on the request's blocks) or an inference (the margins
w.x_i, he_lr_margins).  A request has its own shard size n, feature count d
(padded to c = 2^ceil(log2 d)) and ring degree N.  Keys, the encrypted data
pools and the weights are resident in HBM; a request's blocks are the first
ceil(n / r) blocks of its (N, c) pool.

Continuous batching: each ring degree has `lanes` execution lanes.  A lane is
a library context of its own, bound to its own HIP stream, with its own
workspace and its own copy of the keys (same seed, so every lane computes
bit-identical results).  The loop runs on the host:
- move the requests whose arrival time has passed into the queue;
- admit: for each ring degree, the oldest queued request of that degree is
  launched on a free lane of that degree when its bytes fit the budget.  Its
  bytes are the workspace for its block count (he_lr_step_bytes /
  he_lr_margins_bytes) plus its outputs.  The budget is a fraction of the
  free HBM after keys and pools.  Ring degrees do not block each other; within
  one degree, admission is in arrival order;
- poll the lanes' completion events and release lanes and bytes.
So requests that arrive while others run are admitted as lanes and memory
free up, and their kernels overlap on the device.  Latency = completion -
arrival; the run reports p50 / p99 latency and throughput.

Usage: python -m paper_2006_10091_amd.serve [--requests 2000] [--rate 200]
       [--lanes 2] [--budget-frac 0.8]
"""
import argparse
import collections
import json
import math
import sys
import time

import numpy as np

from . import he as H
from . import synth

CHAIN = dict(n_q=8, n_special=2, alpha=2, log_delta=40)  # one step or one inference per request
LOG_NS = (15, 16)
N_RANGE = (512, 16384)
D_RANGE = (16, 512)

Request = collections.namedtuple("Request", "rid arrival kind log_n n d c r nb")


def make_requests(count, rate, seed=4004, log_ns=LOG_NS, n_range=N_RANGE, d_range=D_RANGE):
    """Poisson arrivals at `rate` per second; kind 50/50; n and d log-uniform;
    N uniform over log_ns."""
    g = synth.rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += g.exponential(1.0 / rate)
        kind = "grad" if g.uniform() < 0.5 else "infer"
        log_n = int(g.choice(log_ns))
        n = int(round(math.exp(g.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        d = int(round(math.exp(g.uniform(math.log(d_range[0]), math.log(d_range[1])))))
        c = 1 << max(0, math.ceil(math.log2(d)))
        r = (1 << (log_n - 1)) // c
        out.append(Request(i, t, kind, log_n, n, d, c, r, -(-n // r)))
    return out


def percentile(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if xs else float("nan")


def run_loop(requests, backend, lanes_per_n, budget, clock=time.perf_counter, idle=2e-4):
    """The continuous-batching loop over a backend with
    bytes(req) / launch(lane, req) -> handle / done(handle) -> bool /
    finish(handle, req).  Returns per-request (admit, complete) times
    relative to the run's start, and the peak bytes in flight."""
    pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
    queues = {k: collections.deque() for k in lanes_per_n}
    free = {k: list(range(v)) for k, v in lanes_per_n.items()}
    running = []  # (lane key, lane index, handle, request, bytes)
    in_flight = 0
    peak = 0
    times = {}
    t0 = clock()
    total = len(requests)
    while len(times) < total or running:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            q = pending.popleft()
            queues[q.log_n].append(q)
        progressed = False
        for k, qu in queues.items():
            while qu and free[k]:
                q = qu[0]
                b = backend.bytes(q)
                if b > budget:
                    raise ValueError("request %d needs %d bytes, over the whole budget %d" % (q.rid, b, budget))
                if in_flight + b > budget:
                    break  # waits for memory; the other ring degree is not blocked
                qu.popleft()
                lane = free[k].pop()
                h = backend.launch((k, lane), q)
                running.append((k, lane, h, q, b))
                in_flight += b
                peak = max(peak, in_flight)
                times[q.rid] = [clock() - t0, None]
                progressed = True
        still = []
        for item in running:
            k, lane, h, q, b = item
            if backend.done(h):
                times[q.rid][1] = clock() - t0
                backend.finish(h, q)
                free[k].append(lane)
                in_flight -= b
                progressed = True
            else:
                still.append(item)
        running = still
        if not progressed:
            if not running and pending and not any(queues.values()):
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            else:
                time.sleep(idle)
    return times, peak


def summarise(requests, times):
    lat = [times[q.rid][1] - q.arrival for q in requests]
    qwait = [times[q.rid][0] - q.arrival for q in requests]
    span = max(t[1] for t in times.values()) - min(q.arrival for q in requests)
    out = {"requests": len(requests), "p50_latency_ms": percentile(lat, 50) * 1e3,
           "p99_latency_ms": percentile(lat, 99) * 1e3, "mean_latency_ms": float(np.mean(lat)) * 1e3,
           "p50_queue_ms": percentile(qwait, 50) * 1e3, "p99_queue_ms": percentile(qwait, 99) * 1e3,
           "throughput_req_per_s": len(requests) / span, "span_s": span}
    for kind in ("grad", "infer"):
        lk = [times[q.rid][1] - q.arrival for q in requests if q.kind == kind]
        out[kind + "_p50_ms"] = percentile(lk, 50) * 1e3
        out[kind + "_p99_ms"] = percentile(lk, 99) * 1e3
    return out


class GpuBackend:
    """Lanes, pools and outputs on the GPU."""

    def __init__(self, requests, lanes, mode=1, keep_results=False, seed=6006, distinct=8):
        import torch
        self.torch = torch
        self.mode, self.keep = mode, keep_results
        self.results = {}
        self.lanes = {}
        need = collections.defaultdict(int)  # (log_n, c) -> max blocks
        maxnb = collections.defaultdict(int)  # log_n -> max blocks
        steps = collections.defaultdict(set)
        for q in requests:
            need[(q.log_n, q.c)] = max(need[(q.log_n, q.c)], q.nb)
            maxnb[q.log_n] = max(maxnb[q.log_n], q.nb)
            steps[q.log_n] |= set(H.rotation_steps(q.c, q.r))
        L = CHAIN["n_q"] - 1
        for log_n in sorted(maxnb):
            for j in range(lanes):
                stream = torch.cuda.Stream()
                ctx = H.Context(log_n, CHAIN["n_q"], CHAIN["n_special"], CHAIN["alpha"], CHAIN["log_delta"],
                                stream=stream.cuda_stream)
                keys = ctx.keygen(2004 + log_n, sorted(steps[log_n]))
                outs = dict(W=ctx.ct_empty(L - 4), G=ctx.ct_empty(L - 4), M=ctx.ct_block(maxnb[log_n], L - 1))
                self.lanes[(log_n, j)] = dict(ctx=ctx, stream=stream, keys=keys, outs=outs)
        # data pools: `distinct` encoded blocks per (N, c), encrypted into every pool slot
        self.pools = {}
        g = synth.rng(seed)
        for (log_n, c), nb in sorted(need.items()):
            ctx = self.lanes[(log_n, 0)]["ctx"]
            keys = self.lanes[(log_n, 0)]["keys"]
            S = ctx.S
            r = S // c
            pts = []
            for _ in range(min(distinct, nb)):
                X = g.uniform(0.0, 1.0, size=(r, c))
                y = np.where(g.uniform(size=r) < 0.5, 1.0, -1.0)
                pts.append(ctx.pt_load(ctx.encode((y[:, None] * X).reshape(S), ctx.delta), L, ctx.delta))
            Z = ctx.ct_block(nb, L)
            for i in range(nb):
                ctx.encrypt(pts[i % len(pts)], keys, seed, (c << 16) + i, out=Z[i])
            w = g.uniform(-0.05, 0.05, size=c)
            W = ctx.encrypt(ctx.pt_load(ctx.encode(H.pack_weights(w, S, c), ctx.delta), L, ctx.delta), keys, seed,
                            (c << 16) + 0xFFFF)
            pl = ctx.plan_lr_step(L, ctx.delta, ctx.delta, [0.5, -0.15, 0.0, 0.0016], 1.0 / 512)
            mask = ctx.pt_load(ctx.encode(H.column0_mask(S, c), pl["s_mask"]), L - 1, pl["s_mask"])
            self.pools[(log_n, c)] = dict(Z=Z, W=W, mask=mask)
        torch.cuda.synchronize()
        self.coef = [0.5, -0.1501204134, 0.0, 0.0015930174]

    def bytes(self, q):
        ctx = self.lanes[(q.log_n, 0)]["ctx"]
        L = CHAIN["n_q"] - 1
        if q.kind == "grad":
            return ctx.step_bytes(L, q.nb, H.LAYOUT_ROWS, self.mode) + 2 * (2 * (L - 3) * ctx.N * 8)
        return ctx.margins_bytes(L, q.nb, self.mode) + q.nb * 2 * L * ctx.N * 8

    def launch(self, lane_key, q):
        lane = self.lanes[lane_key]
        ctx, outs = lane["ctx"], lane["outs"]
        pool = self.pools[(q.log_n, q.c)]
        Z = pool["Z"][: q.nb]
        if q.kind == "grad":
            ctx.lr_grad_step(Z, pool["W"], pool["mask"], self.coef, 1.0 / q.n, q.c, q.r, lane["keys"],
                             mode=self.mode, W_out=outs["W"], G_out=outs["G"])
        else:
            ctx.lr_margins(Z, pool["W"], q.c, q.r, lane["keys"], mode=self.mode, out=outs["M"][: q.nb])
        ev = self.torch.cuda.Event()
        ev.record(lane["stream"])
        return (lane_key, ev)

    def done(self, h):
        return h[1].query()

    def finish(self, h, q):
        if not self.keep:
            return
        lane = self.lanes[h[0]]
        ctx, outs = lane["ctx"], lane["outs"]
        if q.kind == "grad":
            self.results[q.rid] = (ctx.download(outs["W"]), ctx.download(outs["G"]))
        else:
            self.results[q.rid] = tuple(ctx.download(m) for m in outs["M"][: q.nb])

    def free_bytes_after_setup(self):
        free, _ = self.torch.cuda.mem_get_info()
        return free


def serve(requests, lanes=2, mode=1, budget_frac=0.8, budget=None, keep_results=False, warm=True):
    """Set up the GPU backend for `requests`, warm each lane once on its
    largest request of each kind (workspace growth), run the loop."""
    be = GpuBackend(requests, lanes, mode=mode, keep_results=keep_results)
    if warm:
        for log_n in {q.log_n for q in requests}:
            for kind in ("grad", "infer"):
                qs = [q for q in requests if q.log_n == log_n and q.kind == kind]
                if qs:
                    big = max(qs, key=lambda q: q.nb)
                    for j in range(lanes):
                        be.launch((log_n, j), big)
        be.torch.cuda.synchronize()
    if budget is None:
        budget = int(budget_frac * be.free_bytes_after_setup())
    lanes_per_n = {k: lanes for k in sorted({q.log_n for q in requests})}
    times, peak = run_loop(requests, be, lanes_per_n, budget)
    stats = summarise(requests, times)
    stats.update(lanes_per_ring=lanes, mode=mode, budget_bytes=budget, peak_bytes_in_flight=peak)
    return stats, be, times


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--lanes", type=int, default=2)
    ap.add_argument("--mode", type=int, default=1)
    ap.add_argument("--budget-frac", type=float, default=0.8)
    args = ap.parse_args(argv)
    reqs = make_requests(args.requests, args.rate)
    stats, _, _ = serve(reqs, lanes=args.lanes, mode=args.mode, budget_frac=args.budget_frac)
    stats["rate_req_per_s"] = args.rate
    print(json.dumps(stats), flush=True)
    return stats


if __name__ == "__main__":
    main(sys.argv[1:])
