"""Serving encrypted gradient steps and encrypted inferences with continuous batching.

Requests arrive as a Poisson stream.  Each is either a gradient step (eq.
(appr) + eq. (update) on the request's blocks) or an inference (the margins
w.x_i, he_lr_margins, with the served model W).  A request has its own shard
size n, feature count d (padded to c = 2^ceil(log2 d)) and ring degree N.
Keys, the encrypted data pools and the models are resident in HBM; a
request's blocks are the first ceil(n / r) blocks of its (N, c) pool.

Lanes: each ring degree has `lanes` execution lanes.  A lane is a library
context of its own, bound to its own HIP stream; the lanes of a ring degree
share one key set (a key set is valid for every context of its parameter
set).  The loop runs on the host:
- move the requests whose arrival time has passed into their ring's queue;
- admit: for each ring degree, while a lane is free, the oldest queued request
  leads the next launch and takes along the later queued requests of its
  kind and (N, c) (gradient steps: also of its packing) in arrival order, up
  to `merge_blocks` blocks and 16 requests in all.  Merged inferences share
  the served model, so their blocks are staged side by side and their
  margins are one block-batched call.  Merged gradient steps keep their own
  blocks, weights, masks and eta/n; he_lr_grad_step_multi runs each one's
  per-block part and then their once-per-step tails together (the tail's
  key switches are latency-bound, so a batch of them costs about what one
  does).  The launch is admitted when its bytes fit the budget next to the
  launches in flight (a merged launch sheds its last members until it fits);
- poll the lanes' completion events; on completion the launch's staging,
  outputs and workspace go back to the allocator and its bytes to the budget.
A launch's bytes are what it really allocates: its library workspace
(he_lr_step_bytes / he_lr_margins_bytes, drawn through the context's
allocator at the call and given back by he_ctx_trim on completion), its
staged blocks and its outputs.  The budget is a fraction of the device memory
left after keys, pools and lanes.  Latency = completion - arrival; the run
reports p50 / p99 latency, throughput and the launches' sizes.

Gradient steps take the feature-major packing where the plan allows it (one
mask and replication per step instead of per block), else the row-major one.

Usage: python -m paper_2006_10091_amd.serve [--requests 2000] [--rate 200]
       [--lanes 4] [--merge-blocks 256] [--budget-frac 0.8]
"""
import argparse
import collections
import itertools
import json
import math
import sys
import time

import numpy as np

from . import he as H
from . import synth

CHAIN = dict(n_q=8, n_special=4, alpha=4, log_delta=40)  # one step or one inference per request
LOG_NS = (15, 16)
N_RANGE = (512, 16384)
D_RANGE = (16, 512)
COEF = [0.5, -0.1501204134, 0.0, 0.0015930174]  # the step's loss polynomial
MERGE_BLOCKS = 256
MAX_MERGE = 16  # requests per merged launch

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


def same_width(q):
    return (q.kind, q.c)


def take_batch(queue, merge_blocks, merge_key=same_width, max_requests=MAX_MERGE):
    """The launch the queue's oldest request leads: itself and the later
    queued requests with its merge key (kind and feature width; the backend
    adds the packing of gradient steps), in arrival order, while the blocks
    stay within merge_blocks and the requests within max_requests."""
    head = queue[0]
    batch = [head]
    if merge_blocks:
        key, total = merge_key(head), head.nb
        for q in itertools.islice(queue, 1, None):
            if len(batch) >= max_requests:
                break
            if merge_key(q) == key and total + q.nb <= merge_blocks:
                batch.append(q)
                total += q.nb
    return batch


class DeviceMemoryFull(Exception):
    """Raised by a backend's launch when the device could not hold the
    launch's allocations although the budget admitted it (the allocator's
    fragmentation across lanes' streams); nothing of the launch is left
    running and its requests stay queued."""


def run_loop(requests, backend, lanes_per_n, budget, merge_blocks=0, clock=time.perf_counter, idle=2e-4,
             merge_key=same_width, stats=None):
    """The continuous-batching loop over a backend with
    bytes(batch) / launch(lane, batch) -> handle / done(handle) -> bool /
    finish(handle, batch).  Returns per-request (admit, complete) times
    relative to the run's start, the peak bytes in flight and the launches
    (lists of request ids).  A launch refused with DeviceMemoryFull while
    others run leaves its requests at the head of their queue, and no ring
    admits anything until a running launch completes (stats, when given,
    counts these waits as memory_waits); refused with nothing running, it
    is an error."""
    pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
    queues = {k: collections.deque() for k in lanes_per_n}
    free = {k: list(range(v)) for k, v in lanes_per_n.items()}
    running = []  # (lane key, lane index, handle, batch, bytes)
    in_flight = 0
    peak = 0
    times = {}
    launches = []
    t0 = clock()
    total = len(requests)
    mem_wait = False  # a launch was refused for memory: wait for a completion
    waits = 0
    while len(times) < total or running:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            q = pending.popleft()
            queues[q.log_n].append(q)
        progressed = False
        for k, qu in queues.items():
            while qu and free[k] and not mem_wait:
                batch = take_batch(qu, merge_blocks, merge_key)
                b = backend.bytes(batch)
                while len(batch) > 1 and in_flight + b > budget:
                    batch.pop()
                    b = backend.bytes(batch)
                if b > budget:
                    raise ValueError("request %d needs %d bytes, over the whole budget %d" % (batch[0].rid, b, budget))
                if in_flight + b > budget:
                    break  # waits for memory; the other ring degree is not blocked
                lane = free[k].pop()
                try:
                    h = backend.launch((k, lane), batch)
                except DeviceMemoryFull:
                    free[k].append(lane)
                    if not running:
                        raise
                    mem_wait = True  # the batch stays queued, in order
                    waits += 1
                    break
                for q in batch:
                    qu.remove(q)
                running.append((k, lane, h, batch, b))
                launches.append([q.rid for q in batch])
                in_flight += b
                peak = max(peak, in_flight)
                t = clock() - t0
                for q in batch:
                    times[q.rid] = [t, None]
                progressed = True
        still = []
        for item in running:
            k, lane, h, batch, b = item
            if backend.done(h):
                t = clock() - t0
                for q in batch:
                    times[q.rid][1] = t
                backend.finish(h, batch)
                free[k].append(lane)
                in_flight -= b
                mem_wait = False
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
    if stats is not None:
        stats["memory_waits"] = waits
    return times, peak, launches


def summarise(requests, times, launches=None):
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
    if launches is not None:
        kind = {q.rid: q.kind for q in requests}
        out["launches"] = len(launches)
        out["requests_per_launch"] = len(requests) / max(1, len(launches))
        out["max_requests_per_launch"] = max((len(x) for x in launches), default=0)
        for k in ("grad", "infer"):
            out["merged_launches_" + k] = sum(1 for x in launches if len(x) > 1 and kind[x[0]] == k)
    return out


def step_layout(q, primes):
    """Feature-major where the plan accepts the request's 1/n, else row-major."""
    L = CHAIN["n_q"] - 1
    d = float(2 ** CHAIN["log_delta"])
    try:
        H.plan_lr_step(primes, CHAIN["n_q"], L, d, d, COEF, 1.0 / q.n, 0.0, H.LAYOUT_FEATURES)
        return H.LAYOUT_FEATURES
    except H.HEError:
        return H.LAYOUT_ROWS


class GpuBackend:
    """Lanes, key sets, pools and models on the GPU."""

    def __init__(self, requests, lanes, mode=1, keep_results=False, seed=6006, distinct=8):
        import torch
        self.torch = torch
        self.mode, self.keep = mode, keep_results
        self.results = {}
        self.lanes = {}
        self.keys = {}
        L = self.L = CHAIN["n_q"] - 1
        chain = (CHAIN["n_q"], CHAIN["n_special"], CHAIN["alpha"], CHAIN["log_delta"])
        primes = {log_n: H.params_primes(log_n, *chain) for log_n in {q.log_n for q in requests}}
        self.layout = {q.rid: step_layout(q, primes[q.log_n]) for q in requests if q.kind == "grad"}
        need = collections.defaultdict(int)  # (log_n, c, layout) -> most blocks of a request
        steps = collections.defaultdict(set)
        for q in requests:
            lay = self.layout.get(q.rid, H.LAYOUT_ROWS)
            need[(q.log_n, q.c, lay)] = max(need[(q.log_n, q.c, lay)], q.nb)
            steps[q.log_n] |= set(H.rotation_steps(q.c, q.r, lay))
        for log_n in sorted(primes):
            for j in range(lanes):
                stream = torch.cuda.Stream()
                ctx = H.Context(log_n, *chain, stream=stream.cuda_stream)
                self.lanes[(log_n, j)] = dict(ctx=ctx, stream=stream)
            # one key set per ring degree, shared by its lanes
            self.keys[log_n] = self.lanes[(log_n, 0)]["ctx"].keygen(2004 + log_n, sorted(steps[log_n]))
        # data pools: `distinct` plaintext blocks per (N, c, layout), encrypted into
        # every pool slot; one served model W per (N, c, layout)
        self.pools = {}
        g = synth.rng(seed)
        for (log_n, c, lay), nb in sorted(need.items()):
            ctx = self.lanes[(log_n, 0)]["ctx"]
            keys = self.keys[log_n]
            S = ctx.S
            r = S // c
            pts = []
            for _ in range(min(distinct, nb)):
                X = g.uniform(0.0, 1.0, size=(r, c))
                y = np.where(g.uniform(size=r) < 0.5, 1.0, -1.0)
                Zp = y[:, None] * X
                Zp = Zp.T if lay == H.LAYOUT_FEATURES else Zp  # slot j r + i, else i c + j
                pts.append(ctx.pt_load(ctx.encode(Zp.reshape(S), ctx.delta), L, ctx.delta))
            Z = ctx.ct_block(nb, L)
            for i in range(nb):
                ctx.encrypt(pts[i % len(pts)], keys, seed, (c << 17) + (lay << 16) + i, out=Z[i])
            w = g.uniform(-0.05, 0.05, size=c)
            W = ctx.encrypt(ctx.pt_load(ctx.encode(H.pack_weights(w, S, c, lay), ctx.delta), L, ctx.delta), keys,
                            seed, (c << 17) + (lay << 16) + 0xFFFF)
            self.pools[(log_n, c, lay)] = dict(Z=Z, W=W, masks={})
        # step masks: row-major, one per pool (its scale does not depend on n);
        # feature-major, one per shard size (its scale carries eta / n)
        for q in requests:
            if q.kind != "grad":
                continue
            lay = self.layout[q.rid]
            pool = self.pools[(q.log_n, q.c, lay)]
            key = q.n if lay == H.LAYOUT_FEATURES else 0
            if key not in pool["masks"]:
                ctx = self.lanes[(q.log_n, 0)]["ctx"]
                pl = ctx.plan_lr_step(L, ctx.delta, ctx.delta, COEF, 1.0 / q.n, layout=lay)
                ml = H.mask_level(L, lay)
                pool["masks"][key] = ctx.pt_load(ctx.encode(H.step_mask(ctx.S, q.c, lay), pl["s_mask"]), ml,
                                                 pl["s_mask"])
        torch.cuda.synchronize()

    def merge_key(self, q):
        """Requests that may share a launch: kind and width, and a step's packing."""
        return (q.kind, q.c, self.layout.get(q.rid))

    def ct_bytes(self, log_n, level):
        return 2 * (level + 1) * (1 << log_n) * 8

    def bytes(self, batch):
        """What the launch allocates: library workspace, staged blocks, outputs."""
        q = batch[0]
        ctx = self.lanes[(q.log_n, 0)]["ctx"]
        L = self.L
        if q.kind == "grad":
            lay = self.layout[q.rid]
            outs = 2 * len(batch) * self.ct_bytes(q.log_n, L - 4)
            if len(batch) == 1:
                return ctx.step_bytes(L, q.nb, lay, self.mode) + outs
            return ctx.step_multi_bytes(L, max(x.nb for x in batch), len(batch), lay, self.mode) + outs
        nb = sum(x.nb for x in batch)
        return ctx.margins_bytes(L, nb, self.mode) + nb * (self.ct_bytes(q.log_n, L) + self.ct_bytes(q.log_n, L - 1))

    def launch(self, lane_key, batch):
        try:
            return self._launch(lane_key, batch)
        except (H.HEError, self.torch.cuda.OutOfMemoryError) as e:
            if isinstance(e, H.HEError) and e.status != H.HE_ENOMEM:
                raise
            # nothing was launched after the failed allocation; what was
            # staged on the lane's stream finishes before its buffers go
            self.lanes[lane_key]["stream"].synchronize()
            raise DeviceMemoryFull(str(e)) from e

    def _launch(self, lane_key, batch):
        torch = self.torch
        lane = self.lanes[lane_key]
        ctx, stream = lane["ctx"], lane["stream"]
        keys = self.keys[lane_key[0]]
        q = batch[0]
        L = self.L
        held = {}
        if q.kind == "grad":
            lay = self.layout[q.rid]
            pool = self.pools[(q.log_n, q.c, lay)]
            reqs = []
            for x in batch:
                mask = pool["masks"][x.n if lay == H.LAYOUT_FEATURES else 0]
                held[("W", x.rid)], held[("G", x.rid)] = ctx.ct_empty(L - 4), ctx.ct_empty(L - 4)
                reqs.append(dict(Z=pool["Z"][: x.nb], W=pool["W"], mask=mask, coef=COEF, eta_over_n=1.0 / x.n,
                                 W_out=held[("W", x.rid)], G_out=held[("G", x.rid)]))
            if len(batch) == 1:
                r0 = reqs[0]
                ctx.lr_grad_step(r0["Z"], r0["W"], r0["mask"], COEF, r0["eta_over_n"], q.c, q.r, keys,
                                 mode=self.mode, W_out=r0["W_out"], G_out=r0["G_out"], layout=lay)
            else:
                ctx.lr_grad_step_multi(reqs, q.c, q.r, keys, mode=self.mode, layout=lay)
        else:
            pool = self.pools[(q.log_n, q.c, H.LAYOUT_ROWS)]
            nb = sum(x.nb for x in batch)
            # stage the requests' blocks side by side (a request's own upload
            # would land here), then one block-batched margins call
            Z = ctx.ct_block(nb, L)
            per = 2 * (L + 1) * ctx.N
            src = pool["Z"][0].tensor
            with torch.cuda.stream(stream):
                off = 0
                for x in batch:
                    Z[0].tensor[off * per:(off + x.nb) * per].copy_(src[: x.nb * per])
                    off += x.nb
            for z in Z:
                z.scale = pool["Z"][0].scale
            held["Z"], held["M"] = Z, ctx.ct_block(nb, L - 1)
            ctx.lr_margins(Z, pool["W"], q.c, q.r, keys, mode=self.mode, out=held["M"])
        ev = torch.cuda.Event()
        ev.record(stream)
        return (lane_key, ev, held)

    def done(self, h):
        return h[1].query()

    def finish(self, h, batch):
        lane = self.lanes[h[0]]
        ctx, held = lane["ctx"], h[2]
        if self.keep:
            if batch[0].kind == "grad":
                for x in batch:
                    self.results[x.rid] = (ctx.download(held[("W", x.rid)]), ctx.download(held[("G", x.rid)]))
            else:
                off = 0
                for x in batch:
                    self.results[x.rid] = tuple(ctx.download(m) for m in held["M"][off:off + x.nb])
                    off += x.nb
        held.clear()  # staging and outputs back to the allocator
        ctx.trim()  # and the workspace (the launch has completed)

    def free_bytes_after_setup(self):
        """Device memory free now, counting the allocator's cached blocks."""
        torch = self.torch
        free, _ = torch.cuda.mem_get_info()
        return free + torch.cuda.memory_reserved() - torch.cuda.memory_allocated()


def serve(requests, lanes=4, mode=1, budget_frac=0.8, budget=None, keep_results=False, warm=True,
          merge_blocks=MERGE_BLOCKS):
    """Set up the GPU backend for `requests`, warm up (first-call costs: the
    smallest request of every ring, kind, width and packing once, the largest
    of every ring and kind once, so that the allocator's cache holds blocks
    of the largest workspace, and one request on every lane), run the loop."""
    be = GpuBackend(requests, lanes, mode=mode, keep_results=keep_results)
    if warm:
        keep, be.keep = be.keep, False
        first = {}
        for q in sorted(requests, key=lambda q: q.nb):
            first.setdefault((q.log_n, q.kind, q.c, be.layout.get(q.rid)), q)
        runs = [((q.log_n, 0), q) for q in first.values()]
        for log_n in {q.log_n for q in requests}:
            for kind in ("grad", "infer"):
                qs = [q for q in requests if q.log_n == log_n and q.kind == kind]
                if qs:
                    runs.append(((log_n, 0), max(qs, key=lambda q: q.nb)))
        for log_n in {q.log_n for q in requests}:
            small = min((q for q in requests if q.log_n == log_n), key=lambda q: q.nb)
            runs += [((log_n, j), small) for j in range(1, lanes)]
        for lane, q in runs:
            h = be.launch(lane, [q])
            h[1].synchronize()
            be.finish(h, [q])
        be.keep = keep
        be.torch.cuda.synchronize()
    if budget is None:
        budget = int(budget_frac * be.free_bytes_after_setup())
    lanes_per_n = {k: lanes for k in sorted({q.log_n for q in requests})}
    base = be.torch.cuda.memory_allocated()
    be.torch.cuda.reset_peak_memory_stats()
    m0 = be.torch.cuda.memory_stats()
    loop_stats = {}
    times, peak, launches = run_loop(requests, be, lanes_per_n, budget, merge_blocks=merge_blocks,
                                     merge_key=be.merge_key, stats=loop_stats)
    m1 = be.torch.cuda.memory_stats()
    stats = summarise(requests, times, launches)
    stats.update(loop_stats)
    # the allocator's own work during the loop: device allocations and frees
    # (each free synchronises the device) and retries after running out
    for k in ("num_device_alloc", "num_device_free", "num_alloc_retries"):
        stats["allocator_" + k] = m1.get(k, 0) - m0.get(k, 0)
    stats.update(lanes_per_ring=lanes, mode=mode, budget_bytes=budget, peak_bytes_in_flight=peak,
                 peak_bytes_allocated=be.torch.cuda.max_memory_allocated() - base, merge_blocks=merge_blocks,
                 feature_major_steps=sum(1 for v in be.layout.values() if v == H.LAYOUT_FEATURES),
                 steps=len(be.layout))
    return stats, be, times


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--lanes", type=int, default=4)
    ap.add_argument("--mode", type=int, default=1)
    ap.add_argument("--merge-blocks", type=int, default=MERGE_BLOCKS)
    ap.add_argument("--budget-frac", type=float, default=0.8)
    args = ap.parse_args(argv)
    reqs = make_requests(args.requests, args.rate)
    stats, _, _ = serve(reqs, lanes=args.lanes, mode=args.mode, budget_frac=args.budget_frac,
                        merge_blocks=args.merge_blocks)
    stats["rate_req_per_s"] = args.rate
    print(json.dumps(stats), flush=True)
    return stats


if __name__ == "__main__":
    main(sys.argv[1:])
