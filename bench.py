"""Benchmark: encrypted logistic-regression gradient steps/s on one MI355X.

Workload (the headline configuration): one server's shard of 6000 two-class
14x14 images (196 features; synthetic stand-in for the paper's MNIST 3-vs-8,
Sec. 5.1) in 47 blocks of 128 samples x 256 feature slots, RNS-CKKS at
N = 2^16 with 20 ciphertext primes (scale 2^40) and 4 special primes (dnum 5),
trained with the paper's schedule: one gradient step of eq. (appr) +
eq. (update) per iteration (4 levels each: steps at levels 19, 15, 11, 7) and a
refresh by the parameter server every 4 steps (Alg. 1 / Alg. 2: decrypt,
re-encrypt at the top level).  A timed step is one iteration of that schedule,
its refresh included when due; the timed steps cover whole refresh periods.

value = the feature-major packing (slot j*r + i), batched form (every block
in one launch per operation) replayed from captured HIP graphs.  Beside it:
the row-major packing (slot i*c + j), and for both the batched form without
graphs and the plain form (one library operation per block), on the same
schedule and for the top-level step alone.  Inputs are resident in HBM before
the timed region.  The roofline entry measures the dominant kernel (the
forward NTT over the key-switching digit batch) with HIP events on the stream
it runs on; cpu_baseline times the CPU oracle on a bounded sample of the same
schedule's key-switching operations and extrapolates by their counts.

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
# FETCH_SIZE + WRITE_SIZE runs of this script under rocprofv3, each scaled by
# what the same counter reads for the 1 GiB calibration copy below
# (profiles/ntt_forward_5640_limbs_pmc.md).  None whenever the NTT kernels have
# changed since the counters were taken.
# counted HBM bytes per forward transform (FETCH_SIZE x2 calibration + WRITE_SIZE, KiB per dispatch, both
# passes) by limb count, from rocprofv3 --pmc over --ntt-counters in the tuned (XCD-grouped) block order
NTT_TRAFFIC_BYTES = {5640: (2 * 1444250 + 2 * 1449696 + 2887681 + 2887680) * 1024}
COPY_BYTES = 1 << 30
REFRESH_EVERY = 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12, help="timed schedule iterations (whole refresh periods "
                                                          "when a multiple of 4)")
    ap.add_argument("--warmup", type=int, default=4, help="untimed iterations (4 = one refresh period, which "
                                                          "captures every level's graph)")
    ap.add_argument("--plain-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--e2e-steps", type=int, default=10,
                    help="steps of the end-to-end figure (from the encrypted shard, everything included; 0 = skip)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--layout", choices=("both", "feature-major", "row-major"), default="both",
                    help="packings to run (value needs feature-major)")
    ap.add_argument("--baby", type=int, default=16,
                    help="baby steps of the margin sum, both packings (1 = rotations only)")
    ap.add_argument("--ntt-counters", action="store_true",
                    help="run only the calibration copy and the NTT batch (the target of rocprofv3 --pmc passes: "
                         "counters are taken over isolated kernels, never over the step, since a FETCH_SIZE pass "
                         "over the whole bench once ended in a host-thread SIGSEGV whose cause is not "
                         "established); prints no bench line")
    ap.add_argument("--giant-counters", action="store_true",
                    help="run only the calibration copy and the hoisted giant-step sum over the shard's blocks "
                         "(for rocprofv3 --pmc)")
    ap.add_argument("--schedule-only", action="store_true",
                    help="run only the headline schedule (feature-major, graph form): one warm-up refresh period, "
                         "then --steps timed steps between two marker fills (a target for rocprofv3 "
                         "--kernel-trace: the markers delimit the timed steps); prints no bench line")
    ap.add_argument("--configs", action="store_true",
                    help="CPU baseline of the other configurations (the oracle beside the GPU): the small workload's "
                         "full step, a 16-operation sample of the 256 mixed operations, per-request and per-block "
                         "samples of serving and of the large shard, each extrapolated and labelled; prints one "
                         "JSON line of them instead of the bench line")
    ap.add_argument("--ks-counters", action="store_true",
                    help="run only the calibration copy and 3 batched multiply-relinearise-rescale-rotate launches "
                         "over 32 ciphertexts at level 18 (key-switch kernels at the step's top-level shape, "
                         "without graphs); prints no bench line")
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


class Schedule:
    """Alg. 1 / Alg. 2 on one GPU: a gradient step per iteration, a refresh
    every REFRESH_EVERY iterations (or when fewer than 4 levels remain)."""

    def __init__(self, worker, ps, w0):
        self.worker, self.ps = worker, ps
        self.W = ps.encrypt_weights(w0)
        self.k = 0

    def iterate(self, n):
        for _ in range(n):
            self.W, _ = self.worker.step(self.W)
            self.k += 1
            if self.k % REFRESH_EVERY == 0 or self.W.level < 4:
                self.W = self.ps.refresh(self.W)


def trace_period(torch, ctx, wk, ps, d):
    """One refresh period of the schedule (REFRESH_EVERY steps and the
    refresh) in the batched form with every launch bracketed by HIP events on
    the context's stream (he_ctx_trace): per kernel kind, launches, time and
    the algorithmic bytes and modular products the library records for each
    launch.  Run after the timed region; the events add a few microseconds per
    launch, so the period's own time is that of the untraced runs."""
    sched = Schedule(wk, ps, np.zeros(d))
    sched.iterate(REFRESH_EVERY)
    torch.cuda.synchronize()
    ctx.trace(True)
    t0 = time.perf_counter()
    sched.iterate(REFRESH_EVERY)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.trace(False)
    return {"steps": REFRESH_EVERY, "wall_ms_traced": wall * 1e3, "stats": ctx.trace_read()}


def kernel_table(tr, peak_fp, peak_int):
    """Per kernel kind of a traced period: share of kernel time, algorithmic
    GB/s against the HBM peak, and the modular products' time at the measured
    butterfly rates (one product = one butterfly) over the kernel time."""
    tot = sum(st["ms"] for st in tr["stats"])
    rows = []
    for st in sorted(tr["stats"], key=lambda x: -x["ms"]):
        t = st["ms"] * 1e-3
        row = {"kernel": st["name"], "launches": st["launches"], "ms": st["ms"], "share": st["ms"] / tot,
               "avg_us": st["ms"] * 1e3 / st["launches"]}
        if st["bytes"] > 0 and t > 0:
            row["gbs"] = st["bytes"] / t / 1e9
            row["frac_hbm"] = row["gbs"] / HBM_PEAK_GBS
        if st["mm_fp64"] + st["mm_int"] > 0 and t > 0:
            row["frac_valu"] = (st["mm_fp64"] / peak_fp + st["mm_int"] / peak_int) / t
        rows.append(row)
    return {"steps": tr["steps"], "wall_ms_traced": tr["wall_ms_traced"], "kernel_ms": tot, "rows": rows}


def measure_copy_and_ntt(torch, ctx, ev, nb):
    """HBM copy rate, then the forward and inverse NTT over the step's
    key-switching digit batch (nb blocks x dnum digits x (L+1+k) limbs), each
    timed with HIP events on the stream it runs on."""
    N, L = ctx.N, ctx.n_q - 1
    # measured copy rate on a working set well above the Infinity Cache
    # (1 GiB read + 1 GiB written); also the calibration dispatch for the
    # FETCH_SIZE / WRITE_SIZE counters
    src = torch.ones(COPY_BYTES // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    t_copy = ev.time(lambda: dst.copy_(src), 5)
    copy_gbs = 2.0 * COPY_BYTES / t_copy / 1e9
    log("copy 1 GiB: %.3f ms (%.0f GB/s read+write)" % (t_copy * 1e3, copy_gbs))
    del src, dst

    nlimb = nb * ctx.dnum * (L + 1 + ctx.n_special) // 4 * 4
    period = L + 1
    nlimb = (nlimb // period) * period
    buf = torch.randint(0, 1 << 40, (nlimb * N,), dtype=torch.int64, device="cuda")
    ctx.ntt(buf, nlimb, 0, period, +1)
    ctx.ntt(buf, nlimb, 0, period, -1)
    t_fwd = ev.time(lambda: ctx.ntt(buf, nlimb, 0, period, +1), 5)
    t_inv = ev.time(lambda: ctx.ntt(buf, nlimb, 0, period, -1), 5)
    alg_bytes = 16.0 * N * nlimb  # read + write each limb once
    log("NTT fwd %d limbs: %.3f ms (%.0f GB/s algorithmic); inv %.3f ms" % (
        nlimb, t_fwd * 1e3, alg_bytes / t_fwd / 1e9, t_inv * 1e3))
    del buf
    return copy_gbs, dict(t_fwd=t_fwd, t_inv=t_inv, nlimb=nlimb, alg_bytes=alg_bytes)


def measure_copy_and_ks(torch, H, synth, ctx, ev, n_ct=32, level=18):
    """The calibration copy, then he_batch_mul_rotate (two key switches per
    entry: relinearisation at `level`, rotation by 1 at level - 1) over n_ct
    ciphertexts of uniform residues, batched form, 3 timed launches."""
    N = ctx.N
    src = torch.ones(COPY_BYTES // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    del src, dst
    keys = ctx.keygen(11, [1])
    q = ctx.primes[: level + 1]
    xs, ys = [], []
    for i in range(n_ct):
        for dst_, s_ in ((xs, 100 + 4 * i), (ys, 102 + 4 * i)):
            d = np.stack([synth.uniform_residues(s_, q, N), synth.uniform_residues(s_ + 1, q, N)])
            dst_.append(ctx.upload(d, level, 1.0))
    outs = [ctx.ct_empty(level - 1) for _ in range(n_ct)]
    ctx.batch_mul_rotate(xs, ys, [1] * n_ct, keys, mode=1, outs=outs)
    t = ev.time(lambda: ctx.batch_mul_rotate(xs, ys, [1] * n_ct, keys, mode=1, outs=outs), 3)
    log("batched mul+relin+rescale+rotate, %d entries at level %d: %.3f ms" % (n_ct, level, t * 1e3))


def measure_copy_and_giant(torch, H, synth, ctx, ev, n_ct, steps, level=18):
    """The calibration copy, then he_rotate_sum (the feature-major giant steps
    as one hoisted key switch) over n_ct ciphertexts of uniform residues at
    `level`, 3 timed launches."""
    N = ctx.N
    src = torch.ones(COPY_BYTES // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    del src, dst
    keys = ctx.keygen(11, steps)
    q = ctx.primes[: level + 1]
    xs = ctx.ct_block(n_ct, level)
    for i in range(n_ct):
        d = np.stack([synth.uniform_residues(300 + 2 * i, q, N), synth.uniform_residues(301 + 2 * i, q, N)])
        ctx.upload(d, level, 1.0, out=xs[i])
    outs = ctx.ct_block(n_ct, level)
    ctx.rotate_sum(xs, steps, keys, outs=outs)
    t = ev.time(lambda: ctx.rotate_sum(xs, steps, keys, outs=outs), 3)
    log("hoisted sum of %d rotations, %d entries at level %d: %.3f ms" % (len(steps), n_ct, level, t * 1e3))


def measure_ops(torch, H, synth, ctx, ev, nb, c, r, n_baby, level=18):
    """The step's two key-switching operations on their own, timed with HIP
    events on the stream they run on, against their algorithmic bytes (what
    a fully fused operation must move: inputs read once, outputs written once,
    each evaluation key read once per launch; every intermediate excluded):
      * mul+relin+rescale+rotate over 32 ciphertext pairs (he_batch_mul_rotate,
        one rotation key shared): 4(l+1) limbs in, 2l out per entry, plus the
        relinearisation and rotation keys, 2 beta (l+1+k) limbs each;
      * the hoisted giant-step sum over the shard's blocks (he_rotate_sum):
        2(l+1) limbs in and out per block, plus the c/n_baby - 1 giant-step
        keys."""
    N, k = ctx.N, ctx.n_special
    beta = -(-(level + 1) // ctx.alpha)
    limb = 8.0 * N
    key = 2 * beta * (level + 1 + k) * limb
    q = ctx.primes[: level + 1]
    out = []
    keys = ctx.keygen(11, [1])
    n_ct = 32
    xs, ys = [], []
    for i in range(n_ct):
        for dst_, s_ in ((xs, 100 + 4 * i), (ys, 102 + 4 * i)):
            d = np.stack([synth.uniform_residues(s_, q, N), synth.uniform_residues(s_ + 1, q, N)])
            dst_.append(ctx.upload(d, level, 1.0))
    outs = [ctx.ct_empty(level - 1) for _ in range(n_ct)]
    ctx.batch_mul_rotate(xs, ys, [1] * n_ct, keys, mode=1, outs=outs)
    t = ev.time(lambda: ctx.batch_mul_rotate(xs, ys, [1] * n_ct, keys, mode=1, outs=outs), 3)
    b = n_ct * (4 * (level + 1) + 2 * level) * limb + 2 * key
    out.append({"op": "mul+relin+rescale+rotate, %d entries at level %d" % (n_ct, level), "ms": t * 1e3,
                "algorithmic_bytes": b, "gbs": b / t / 1e9, "frac_hbm": b / t / 1e9 / HBM_PEAK_GBS})
    del xs, ys, outs, keys
    giant = [g * n_baby * r for g in range(1, c // n_baby)]
    keys = ctx.keygen(11, giant)
    xb = ctx.ct_block(nb, level)
    for i in range(nb):
        d = np.stack([synth.uniform_residues(300 + 2 * i, q, N), synth.uniform_residues(301 + 2 * i, q, N)])
        ctx.upload(d, level, 1.0, out=xb[i])
    ob = ctx.ct_block(nb, level)
    ctx.rotate_sum(xb, giant, keys, outs=ob)
    t = ev.time(lambda: ctx.rotate_sum(xb, giant, keys, outs=ob), 3)
    b = nb * 4 * (level + 1) * limb + len(giant) * key
    out.append({"op": "hoisted sum of %d rotations, %d blocks at level %d" % (len(giant), nb, level), "ms": t * 1e3,
                "algorithmic_bytes": b, "gbs": b / t / 1e9, "frac_hbm": b / t / 1e9 / HBM_PEAK_GBS})
    for o in out:
        log("%s: %.3f ms, %.0f GB/s algorithmic (%.3f of HBM peak)" % (o["op"], o["ms"], o["gbs"], o["frac_hbm"]))
    return out


def ntt_sweep(torch, H, ev):
    """Forward / inverse NTT over B limbs of a 20 + 4 prime chain (limb i on
    prime i mod 24), each N and B timed with HIP events; algorithmic GB/s =
    16 N B / time."""
    out = []
    for log_n in (13, 14, 15, 16):
        ctx = H.Context(log_n, 20, 4, 4, 40)
        N = ctx.N
        for B in (1, 24, 48, 768):
            per = 1 if B == 1 else 24  # limb i uses prime i mod 24 (all 20 + 4 primes)
            buf = torch.randint(0, 1 << 40, (B * N,), dtype=torch.int64, device="cuda")
            ctx.ntt(buf, B, 0, per, +1)
            ctx.ntt(buf, B, 0, per, -1)
            reps = 20 if B * N <= (1 << 22) else 5
            t_f = ev.time(lambda: ctx.ntt(buf, B, 0, per, +1), reps)
            t_i = ev.time(lambda: ctx.ntt(buf, B, 0, per, -1), reps)
            out.append({"log_n": log_n, "limbs": B, "fwd_us": t_f * 1e6, "inv_us": t_i * 1e6,
                        "fwd_gbs": 16.0 * N * B / t_f / 1e9, "inv_gbs": 16.0 * N * B / t_i / 1e9})
            del buf
        del ctx
    log("NTT sweep: " + ", ".join("2^%d x %d: %.0f GB/s" % (o["log_n"], o["limbs"], o["fwd_gbs"]) for o in out))
    return out


def bench_layout(torch, H, T, ctx, keys, X, y, coef, layout, args, Wk):
    """Parity of the top-level step (plain == batched == graph, bit for bit;
    decrypted g against FP64), then the top-level step time and the schedule
    rate in each form."""
    n, d = X.shape
    L = ctx.n_q - 1
    eta_n = 1.0 / n
    name = "feature-major" if layout == H.LAYOUT_FEATURES else "row-major"
    Z, c, r = T.encrypt_shard(ctx, keys, X, y, Wk["seed_enc"], layout)
    ps = T.ParameterServer(ctx, keys, d, c, Wk["seed_enc"], layout=layout)
    res = {"layout": name, "cols": c, "rows": r, "blocks": len(Z)}

    # the top-level step with nonzero weights: forms agree, gradient within tolerance
    wt = np.random.default_rng(Wk["seed_w"]).uniform(-0.05, 0.05, d)
    Wt = ctx.encrypt(ctx.pt_load(ctx.encode(H.pack_weights(wt, ctx.S, c, layout), ctx.delta), L, ctx.delta), keys,
                     Wk["seed_enc"], 1 << 22)
    n_baby = args.baby
    res["n_baby"] = n_baby
    Zrot = None
    if n_baby > 1:
        # the worker's baby-step copies of its data: computed once per shard
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Zrot = ctx.rotate_data(Z, H.baby_unit(layout, r), n_baby, keys)
        torch.cuda.synchronize()
        res["baby_step_data_s"] = time.perf_counter() - t0
        res["baby_step_data_gib"] = len(Zrot) * 2 * (L + 1) * ctx.N * 8 / 2 ** 30
        log("%s: baby-step data copies (%d per block, %.1f GiB) in %.2f s" % (
            name, n_baby - 1, res["baby_step_data_gib"], res["baby_step_data_s"]))
    workers = {mode: T.Worker(ctx, keys, Z, coef, eta_n, c, r, mode=mode, layout=layout, n_baby=n_baby, Zrot=Zrot)
               for mode in (0, 1, 2)}
    outs = {}
    for mode in (0, 1, 2):
        Wn, g = workers[mode].step(Wt, want_g=True)
        outs[mode] = (ctx.download(Wn), ctx.download(g))
    gd = H.unpack_weights(ctx.decrypt_decode(g, keys).real, c, d, layout)
    assert all(np.array_equal(outs[m][0], outs[0][0]) and np.array_equal(outs[m][1], outs[0][1]) for m in (1, 2))
    wdec = H.unpack_weights(ctx.decrypt_decode(Wt, keys).real, c, d, layout)
    z = y[:, None] * X
    m = z @ wdec
    gref = eta_n * ((coef[0] + coef[1] * m + coef[3] * m ** 3)[:, None] * z).sum(0)
    res["decrypted_grad_rel_err"] = float(np.max(np.abs(gd - gref)) / np.max(np.abs(gref)))
    log("%s: plain == batched == graph (bit-exact); decrypted g rel err 2^%.1f" % (
        name, np.log2(res["decrypted_grad_rel_err"])))

    # top-level step alone, then the training schedule, each form
    for mode, key, steps in ((2, "graph", args.steps), (1, "batched", args.plain_steps),
                             (0, "plain", args.plain_steps)):
        wk = workers[mode]
        reps = 3 if mode else 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            wk.step(Wt)
        torch.cuda.synchronize()
        res["top_level_step_ms_" + key] = (time.perf_counter() - t0) / reps * 1e3
        sched = Schedule(wk, ps, np.zeros(d))
        sched.iterate(args.warmup if mode == 2 else REFRESH_EVERY)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sched.iterate(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res["steps_per_s_" + key] = steps / dt
        if mode == 2:
            res["ms_per_step"] = dt / steps * 1e3
        log("%s, %s: schedule %.2f ms/step (%d steps); top-level step %.2f ms" % (
            name, key, dt / steps * 1e3, steps, res["top_level_step_ms_" + key]))
    if layout == H.LAYOUT_FEATURES:
        res["trace"] = trace_period(torch, ctx, workers[1], ps, d)
    res["batched_over_plain"] = res["steps_per_s_graph"] / res["steps_per_s_plain"]
    del workers, Zrot
    if args.e2e_steps > 0:
        # end to end from the encrypted shard: the worker's baby-step copies of
        # its data, the data terms and graph captures on first use of each
        # level, and the steps with their refreshes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wk = T.Worker(ctx, keys, Z, coef, eta_n, c, r, mode=2, layout=layout, n_baby=n_baby)
        sched = Schedule(wk, ps, np.zeros(d))
        sched.iterate(args.e2e_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res["end_to_end_s"] = dt
        res["end_to_end_steps"] = args.e2e_steps
        res["end_to_end_steps_per_s"] = args.e2e_steps / dt
        log("%s: end to end, %d steps from the encrypted shard (baby-step copies, data terms, graph captures, "
            "refreshes): %.3f s (%.2f steps/s)" % (name, args.e2e_steps, dt, args.e2e_steps / dt))
        del wk, sched
    del Z
    return res


def schedule_only(torch, H, T, ctx, keys, X, y, coef, args, Wk):
    """The headline schedule alone, its timed steps between two marker kernels."""
    layout = H.LAYOUT_FEATURES
    n, d = X.shape
    Z, c, r = T.encrypt_shard(ctx, keys, X, y, Wk["seed_enc"], layout)
    ps = T.ParameterServer(ctx, keys, d, c, Wk["seed_enc"], layout=layout)
    Zrot = ctx.rotate_data(Z, H.baby_unit(layout, r), args.baby, keys) if args.baby > 1 else None
    wk = T.Worker(ctx, keys, Z, coef, 1.0 / n, c, r, mode=2, layout=layout, n_baby=args.baby, Zrot=Zrot)
    sched = Schedule(wk, ps, np.zeros(d))
    sched.iterate(REFRESH_EVERY)
    marker = torch.zeros(1 << 20, device="cuda")
    torch.cuda.synchronize()
    marker.fill_(1.0)
    t0 = time.perf_counter()
    sched.iterate(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    marker.fill_(2.0)
    torch.cuda.synchronize()
    log("schedule only: %d steps, %.2f ms/step (between the two marker fills)" % (args.steps, dt / args.steps * 1e3))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; sharding over several GPUs is designed, not implemented"}))
        sys.exit(2)
    import torch
    from paper_2006_10091_amd import he as H
    from paper_2006_10091_amd import synth
    from paper_2006_10091_amd import train as T

    torch.cuda.set_device(0)
    if args.configs:
        print(json.dumps({"config_baselines": config_baselines(torch, H, args.cpu_threads)}), flush=True)
        return
    Wk = synth.WORKLOADS["image"]
    ctx = H.Context(Wk["logN"], Wk["nq"], Wk["nk"], Wk["alpha"], Wk["log_delta"])
    S = ctx.S
    log("ctx: N=2^%d, %d+%d primes, dnum %d" % (Wk["logN"], Wk["nq"], Wk["nk"], ctx.dnum))
    t0 = time.time()
    X, y = synth.image_data(Wk["seed_data"], Wk["n"])
    blocks, c, r = H.pack_blocks(X, y, S)
    nb = blocks.shape[0]
    n = X.shape[0]
    log("data: %d x %d -> %d blocks of %d samples x %d feature slots (%.1fs)" % (
        n, X.shape[1], nb, r, c, time.time() - t0))
    ev = Events(torch, torch.cuda.current_stream())
    if args.ntt_counters:
        measure_copy_and_ntt(torch, ctx, ev, nb)
        return
    if args.ks_counters:
        measure_copy_and_ks(torch, H, synth, ctx, ev)
        return
    if args.giant_counters:
        measure_copy_and_giant(torch, H, synth, ctx, ev, nb, [g * args.baby * r for g in range(1, c // args.baby)])
        return
    steps = sorted(set(H.rotation_steps(c, r, H.LAYOUT_ROWS, max(args.baby, 1))) |
                   set(H.rotation_steps(c, r, H.LAYOUT_FEATURES, max(args.baby, 1))))
    t0 = time.time()
    keys = ctx.keygen(Wk["seed_keys"], steps)
    torch.cuda.synchronize()
    log("keygen: 3 relinearisation + %d rotation keys (%.1fs)" % (len(steps), time.time() - t0))
    coef = coef_binomial()
    if args.schedule_only:
        schedule_only(torch, H, T, ctx, keys, X, y, coef, args, Wk)
        return

    layouts = {}
    for layout, name in ((H.LAYOUT_FEATURES, "feature-major"), (H.LAYOUT_ROWS, "row-major")):
        if args.layout in ("both", name):
            layouts[name] = bench_layout(torch, H, T, ctx, keys, X, y, coef, layout, args, Wk)
            torch.cuda.empty_cache()
    best = layouts.get("feature-major") or layouts["row-major"]

    copy_gbs, ntt = measure_copy_and_ntt(torch, ctx, ev, nb)
    t_fwd, t_inv, nlimb, alg_bytes = ntt["t_fwd"], ntt["t_inv"], ntt["nlimb"], ntt["alg_bytes"]
    ntt_gbs = alg_bytes / t_fwd / 1e9
    # VALU roofline of the transform: its butterflies at the measured peak of
    # each butterfly form (lazy FP64 for the 40-bit primes, 64-bit Shoup for q_0)
    L = ctx.n_q - 1
    peak_fp = ctx.valu_peak(1, True)
    peak_int = ctx.valu_peak(0, False)
    per_limb = (ctx.N // 2) * Wk["logN"]
    n_int = sum(1 for i in range(nlimb) if ctx.primes[i % (L + 1)] >= (1 << 46))
    t_valu = per_limb * ((nlimb - n_int) / peak_fp + n_int / peak_int)
    valu_frac = t_valu / t_fwd
    log("VALU peak: %.1f G butterflies/s (FP64 lazy), %.1f G/s (64-bit Shoup); forward NTT at %.2f of it" % (
        peak_fp / 1e9, peak_int / 1e9, valu_frac))
    kernels = None
    if "trace" in best:
        kernels = kernel_table(best.pop("trace"), peak_fp, peak_int)
        for row in kernels["rows"][:8]:
            log("  %-50s %4d launches %8.2f ms %5.1f%%  %s" % (
                row["kernel"], row["launches"], row["ms"], 100 * row["share"],
                " ".join("%s %.3f" % (k, row[k]) for k in ("frac_hbm", "frac_valu") if k in row)))
    ops = measure_ops(torch, H, synth, ctx, ev, nb, c, r, 16)  # the headline's giant sum, whatever --baby
    sweep = ntt_sweep(torch, H, ev)

    out = {
        "metric": "encrypted LR grad steps/s at N=2^16 (batched vs plain) + NTT HBM GB/s",
        "value": best["steps_per_s_graph"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "image-shard 6000x196, N=2^16, 20+4 primes, dnum 5, scale 2^40, 47 blocks; "
                               "training schedule: steps at levels 19/15/11/7, refresh every 4 steps; "
                               "%s packing%s; batched form replayed from HIP graphs" % (
                                   best["layout"], ", %d baby steps" % best["n_baby"] if best["n_baby"] > 1 else ""),
                   "n": n, "d": int(X.shape[1]), "blocks": nb, "log_n": Wk["logN"], "n_q": Wk["nq"],
                   "n_special": Wk["nk"], "refresh_every": REFRESH_EVERY, "layout": best["layout"],
                   "n_baby": best["n_baby"]},
        "plain_steps_per_s": best["steps_per_s_plain"],
        "batched_nograph_steps_per_s": best["steps_per_s_batched"],
        "batched_over_plain": best["batched_over_plain"],
        "decrypted_grad_rel_err": best["decrypted_grad_rel_err"],
        "end_to_end": {k: best[k] for k in ("end_to_end_s", "end_to_end_steps", "end_to_end_steps_per_s")
                       if k in best},
        "layouts": layouts,
        "ntt_fwd_gbs_algorithmic": ntt_gbs,
        "ntt_inv_gbs_algorithmic": alg_bytes / t_inv / 1e9,
        "ntt_sweep": sweep,
        "hbm_copy_gbs": copy_gbs,
        "ntt_fwd_frac_of_copy": ntt_gbs / copy_gbs,
        "roofline": {"bound": "hbm", "achieved": ntt_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ntt_gbs / HBM_PEAK_GBS, "traffic": NTT_TRAFFIC_BYTES.get(nlimb),
                     "kernel": "ntt (forward, two passes) over %d limbs of N=2^16" % nlimb,
                     "valu_frac": valu_frac, "valu_peak_bfly_per_s": {"fp64_lazy": peak_fp, "int64_shoup": peak_int}},
        "ops": ops,
        "kernels": kernels,
        "ntt_tuning": ctx.ntt_tuned,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(Wk, args.cpu_threads, nb, c, r, best["n_baby"])
    print(json.dumps(out), flush=True)


def config_baselines(torch, H, threads):
    """The oracle (all host threads; median of 3 where the run is short, one
    run for the larger samples) beside the GPU on the configurations other
    than the bench's own:
      * small workload (2048 x 16, N=2^13): one full gradient step, oracle
        and GPU (graph form, median of 20), and the oracle on one thread;
      * 256 mixed operations: the oracle on the first 16 of the seeded
        operations (mixed N and levels), extrapolated to 256; the GPU on all
        256 (he_batch_submit, median of 5);
      * serving: the oracle's row-major step and inference (the margins) for
        the median request (n = 2896 rows, d = 90 features) at N = 2^15 and
        2^16 on the 8 + 4 chain, from 1- and 2-block runs (per block, plus
        the fixed part) scaled to the request's blocks;
      * large shard (2^20 x 512, 24 + 6 primes): the oracle's step at level
        23 from 1- and 2-block runs, scaled to 16384 blocks; the GPU on 64
        seeded blocks (one chunk) at level 23, scaled the same way.
    Every extrapolated figure says so."""
    from oracle import ckks as O
    from oracle import lr as LR
    from paper_2006_10091_amd import batch_ops as BO
    from paper_2006_10091_amd import large_shard as LS
    from paper_2006_10091_amd import synth
    if threads:
        O.lib().orc_set_threads(threads)
    nth = int(O.lib().orc_max_threads())
    coef = coef_binomial()
    out = {"cores": nth, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "kind": "oracle"}

    def med(fn, k=3):
        ts = []
        for _ in range(k):
            t = time.time()
            fn()
            ts.append(time.time() - t)
        return float(np.median(ts))

    def oracle_step_time(P, ok, X, y, level, eta_n):
        """seconds of the oracle's row-major step on the blocks of X at level"""
        blocks, c, r = LR.pack_blocks(X, y, P.S)
        Z = [O.encrypt_sk(P, ok, O.encode(blocks[i], P.delta, P.N), level, P.delta, 5, i) for i in range(len(blocks))]
        W = O.encrypt_sk(P, ok, O.encode(LR.pack_weights(np.zeros(X.shape[1]), P.S, c), P.delta, P.N), level,
                         P.delta, 5, 1 << 20)
        pl = LR.plan_lr_step(P.q, level, P.delta, P.delta, coef, eta_n)
        mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
        t = time.time()
        LR.lr_grad_step(P, ok, Z, W, mm, coef, eta_n, c, r, plan=pl)
        return time.time() - t

    # small workload: one full step
    Wk = synth.WORKLOADS["small"]
    cfg = (Wk["logN"], Wk["nq"], Wk["nk"], Wk["alpha"], Wk["log_delta"])
    P = O.Params(*cfg)
    X, y = synth.small_data()
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    steps = LR.rotation_steps(c, r)
    ok = O.Keys(P, Wk["seed_keys"], rot_steps=steps)
    eta_n = 1.0 / X.shape[0]
    w0 = synth.initial_weights("small", X.shape[1], Wk["seed_w"])
    ms = [O.encode(blocks[i], P.delta, P.N) for i in range(blocks.shape[0])]
    mw = O.encode(LR.pack_weights(w0, P.S, c), P.delta, P.N)
    oZ = [O.encrypt_sk(P, ok, m, P.L, P.delta, 5, i) for i, m in enumerate(ms)]
    oW = O.encrypt_sk(P, ok, mw, P.L, P.delta, 5, 1000)
    pl = LR.plan_lr_step(P.q, P.L, P.delta, P.delta, coef, eta_n)
    mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    t_cpu = med(lambda: LR.lr_grad_step(P, ok, oZ, oW, mm, coef, eta_n, c, r, plan=pl))
    O.lib().orc_set_threads(1)
    t_cpu1 = med(lambda: LR.lr_grad_step(P, ok, oZ, oW, mm, coef, eta_n, c, r, plan=pl))
    O.lib().orc_set_threads(nth)
    ctx = H.Context(*cfg)
    gk = ctx.keygen(Wk["seed_keys"], steps)
    gZ = ctx.ct_block(len(ms), P.L)
    for i, m in enumerate(ms):
        ctx.encrypt(ctx.pt_load(m, P.L, P.delta), gk, 5, i, out=gZ[i])
    gW = ctx.encrypt(ctx.pt_load(mw, P.L, P.delta), gk, 5, 1000)
    gm = ctx.pt_load(mm, P.L - 1, pl["s_mask"])

    def gstep():
        ctx.lr_grad_step(gZ, gW, gm, coef, eta_n, c, r, gk, mode=2)
        torch.cuda.synchronize()
    gstep()
    t_gpu = med(gstep, 20)
    out["small_step"] = {"blocks": len(ms), "cpu_s": t_cpu, "cpu_s_one_thread": t_cpu1, "gpu_ms": t_gpu * 1e3,
                         "gpu_over_cpu": t_cpu / t_gpu, "runs": "median of 3 (CPU), 20 (GPU)"}
    log("small workload, one step: oracle %.3f s (%.3f s one thread), GPU %.3f ms" % (t_cpu, t_cpu1, t_gpu * 1e3))
    del ctx, gk, gZ, gW, gm

    # 256 mixed operations: the oracle on the first 16
    log("configurations: 256 mixed operations ..." )
    ops = BO.draw_ops(256)
    b = BO.Batch(ops)
    b.run_submit(1)
    torch.cuda.synchronize()

    def gbatch():
        b.run_submit(1)
        torch.cuda.synchronize()
    t_gpu = med(gbatch, 5)
    cache = {}
    t_cpu = 0.0
    for i in range(16):
        log_n, level, step = ops[i]
        key = ("P", log_n)
        if key not in cache:
            cache[key] = O.Params(log_n, BO.CHAIN["n_q"], BO.CHAIN["n_special"], BO.CHAIN["alpha"],
                                  BO.CHAIN["log_delta"])
        Pn = cache[key]
        okn = O.Keys(Pn, 2003 + log_n, rot_steps=[step])
        j = b.idx[log_n].index(i)
        x = O.CT(b.ctx[log_n].download(b.x[log_n][j]), level, 1.0)
        z = O.CT(b.ctx[log_n].download(b.y[log_n][j]), level, 1.0)
        t = time.time()
        O.rotate(Pn, O.rescale(Pn, O.mul(Pn, x, z, okn)), step, okn)
        t_cpu += time.time() - t
    out["mixed_ops"] = {"ops": 256, "cpu_ops_timed": 16, "cpu_s_per_op": t_cpu / 16,
                        "cpu_ops_per_s": 16 / t_cpu, "gpu_ms_per_256": t_gpu * 1e3, "gpu_ops_per_s": 256 / t_gpu,
                        "extrapolated": True, "runs": "one run per sampled op (CPU), median of 5 (GPU)"}
    log("256 mixed operations: oracle %.3f s per op (16 timed, extrapolated: %.1f ops/s), GPU %.2f ms (%.0f ops/s)"
        % (t_cpu / 16, 16 / t_cpu, t_gpu * 1e3, 256 / t_gpu))
    del b

    # serving: the median request, step and inference, at both ring degrees
    log("configurations: serving requests ..." )
    n_med, d_med = 2896, 90
    g = synth.rng(7007)
    Xr = g.uniform(-1, 1, (n_med, d_med))
    yr = np.where(Xr @ g.standard_normal(d_med) >= 0, 1.0, -1.0)
    reqs = {}
    for log_n in (15, 16):
        cfg = (log_n, 8, 4, 4, 40)
        Pn = O.Params(*cfg)
        c = 1 << int(np.ceil(np.log2(d_med)))
        r = Pn.S // c
        nblk = -(-n_med // r)
        okn = O.Keys(Pn, 2100 + log_n, rot_steps=LR.rotation_steps(c, r))
        t1 = oracle_step_time(Pn, okn, Xr[:r], yr[:r], Pn.L, 1.0 / n_med)
        t2 = oracle_step_time(Pn, okn, Xr[:2 * r], yr[:2 * r], Pn.L, 1.0 / n_med)
        reqs["step_2^%d" % log_n] = {"blocks": nblk, "cpu_s": t1 + (nblk - 1) * max(t2 - t1, 0.0)}
        bl, _, _ = LR.pack_blocks(Xr[:2 * r], yr[:2 * r], Pn.S)
        Zi = [O.encrypt_sk(Pn, okn, O.encode(bl[k], Pn.delta, Pn.N), Pn.L, Pn.delta, 5, k) for k in range(2)]
        Wi = O.encrypt_sk(Pn, okn, O.encode(LR.pack_weights(np.zeros(d_med), Pn.S, c), Pn.delta, Pn.N), Pn.L,
                          Pn.delta, 5, 99)
        t = time.time()
        LR.lr_margins(Pn, okn, Zi[:1], Wi, c, r)
        ti1 = time.time() - t
        t = time.time()
        LR.lr_margins(Pn, okn, Zi, Wi, c, r)
        ti2 = time.time() - t
        reqs["inference_2^%d" % log_n] = {"blocks": nblk, "cpu_s": ti1 + (nblk - 1) * max(ti2 - ti1, 0.0)}
    mean = float(np.mean([v["cpu_s"] for v in reqs.values()]))
    out["serving"] = {"request": "median shape n=%d, d=%d; 8+4 primes" % (n_med, d_med), "per_request": reqs,
                      "cpu_requests_per_s": 1.0 / mean, "extrapolated": True,
                      "runs": "1- and 2-block runs scaled to the request's blocks (one run each)"}
    log("serving, median request: oracle %.2f s mean over step/inference x N (%.3f req/s, extrapolated)" % (
        mean, 1.0 / mean))

    # large shard: per-block cost at level 23
    log("configurations: large shard ..." )
    Wl = synth.WORKLOADS["large"]
    cfg = (Wl["logN"], Wl["nq"], Wl["nk"], Wl["alpha"], Wl["log_delta"])
    Pl = O.Params(*cfg)
    c = Wl["d"]
    r = Pl.S // c
    Xs, ys = synth.large_block(Wl["seed_data"], 0, 2 * r, c)
    eta_n = 1.0 / Wl["n"]
    okl = O.Keys(Pl, Wl["seed_keys"], rot_steps=LR.rotation_steps(c, r))
    t1 = oracle_step_time(Pl, okl, Xs[:r], ys[:r], Pl.L, eta_n)
    t2 = oracle_step_time(Pl, okl, Xs, ys, Pl.L, eta_n)
    nb = Wl["n"] // r
    cpu_step = t1 + (nb - 1) * max(t2 - t1, 0.0)
    res = LS.run(n_blocks=64, steps=1, chunk=64)
    gpu_step = res["ms_per_step"] * 1e-3 * nb / 64
    out["large_shard"] = {"blocks": nb, "level": Pl.L, "cpu_s_per_step": cpu_step, "cpu_steps_per_s": 1.0 / cpu_step,
                          "gpu_s_per_step_64_blocks": res["ms_per_step"] * 1e-3,
                          "gpu_s_per_step_scaled": gpu_step, "gpu_over_cpu": cpu_step / gpu_step,
                          "extrapolated": True,
                          "runs": "oracle: 1- and 2-block steps at level %d scaled to %d blocks; GPU: one 64-block "
                                  "chunk scaled the same way" % (Pl.L, nb)}
    log("large shard step at level %d: oracle %.0f s (extrapolated from 1- and 2-block runs), GPU %.1f s (64 blocks "
        "scaled)" % (Pl.L, cpu_step, gpu_step))
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(Wk, threads, nb, c, r, n_baby=1):
    """The oracle on a bounded sample of the feature-major schedule: one
    mul+relin+rescale and one rotation at every level the schedule's key
    switches run at, and one hoisted giant-step sum at the top step level
    (scaled to the other levels by the rotation times), each the median of 3
    runs on all host threads, extrapolated by the schedule's counts: per block
    the margin relinearisation and the giant steps (one hoisted sum, or
    log2(c / n_baby) rotations); per step W's n_baby - 1 baby-step rotations,
    the one relinearisation of the summed degree-4 terms (three key switches,
    each timed as a mul+relin+rescale) and the sample sum and replication,
    counted as log2 r rotations each (the oracle takes them, and the giant
    sum when not hoisted, as grouped sums of more key-switch products, so
    this undercounts its time).  The degree-2 products A and B3 (tensor and rescale),
    plaintext products, additions, the data's baby-step copies (built once per
    shard) and the refresh are left out, so the CPU rate is an upper bound.
    The one-thread figure scales it by the measured all-threads / one-thread
    time ratio of a mul+relin+rescale and a rotation at the lowest step level
    (median of 3 each)."""
    from oracle import ckks as O
    from paper_2006_10091_amd import synth
    if threads:
        O.lib().orc_set_threads(threads)
    nthreads = int(O.lib().orc_max_threads())
    P = O.Params(Wk["logN"], Wk["nq"], Wk["nk"], Wk["alpha"], Wk["log_delta"])
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
    from oracle import lr as LR
    hoisted = LR.giant_hoisted(c, LR.FEATURES, n_baby)
    giant = [g * n_baby * r for g in range(1, c // n_baby)]
    if hoisted:  # the giant-step keys g n_baby r
        for t in giant:
            keys.add_rotation(t)
    t_keys = time.time() - t0

    def ct(level, seed):
        return O.CT(np.stack([synth.uniform_residues(seed, P.q[: level + 1], P.N),
                              synth.uniform_residues(seed + 1, P.q[: level + 1], P.N)]), level, 1.0)

    def timed(fn):
        ts = []
        for _ in range(3):
            t = time.time()
            fn()
            ts.append(time.time() - t)
        return float(np.median(ts))

    lc, lr = int(np.log2(c // n_baby)), int(np.log2(r))
    levels = [P.L - 4 * k for k in range(REFRESH_EVERY)]
    need_mul = sorted({l - k for l in levels for k in (0, 2)})
    need_rot = sorted({l - k for l in levels for k in ((0, 1, 3, 4) if n_baby > 1 else (1, 3, 4))})
    sample = {}
    for lv in need_mul:
        x, z = ct(lv, 1), ct(lv, 3)
        sample["mul%d" % lv] = timed(lambda: O.rescale(P, O.mul(P, x, z, keys)))
    for lv in need_rot:
        x = ct(lv, 5)
        sample["rot%d" % lv] = timed(lambda: O.rotate(P, x, 1, keys))
    if hoisted:  # timed at the top step level, scaled to the others by the rotation times
        lt = levels[0] - 1
        x = ct(lt, 7)
        sample["giant%d" % lt] = timed(lambda: O.rotate_sum_hoisted(P, x, giant, keys))
    t_sched = 0.0
    for l in levels:  # the feature-major step at level l
        if hoisted:
            t_giant = sample["giant%d" % lt] * sample["rot%d" % (l - 1)] / sample["rot%d" % lt]
        else:
            t_giant = lc * sample["rot%d" % (l - 1)]
        t_sched += nb * (sample["mul%d" % l] + t_giant)
        t_sched += 3 * sample["mul%d" % (l - 2)] + lr * sample["rot%d" % (l - 3)] + lr * sample["rot%d" % (l - 4)]
        if n_baby > 1:
            t_sched += (n_baby - 1) * sample["rot%d" % l]
    t_step = t_sched / len(levels)
    # one thread: the same operations at the lowest step level, timed again
    lo = levels[-1]
    x, z, xr = ct(lo, 1), ct(lo, 3), ct(lo - 1, 5)
    O.lib().orc_set_threads(1)
    t1 = timed(lambda: O.rescale(P, O.mul(P, x, z, keys))) + timed(lambda: O.rotate(P, xr, 1, keys))
    O.lib().orc_set_threads(nthreads)
    ta = sample["mul%d" % lo] + sample["rot%d" % (lo - 1)]
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": nthreads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "one_thread_value": 1.0 / (t_step * t1 / ta), "one_thread_over_all": t1 / ta,
            "sample": "one oracle mul+relin+rescale and one rotation at each level the feature-major schedule "
                      "key-switches at, and one hoisted sum of the %d giant steps at the top step level, scaled to "
                      "the others by the rotation times (median of 3 runs each on %d threads; %.1fs of sampled work, "
                      "keys %.1fs), extrapolated by the schedule's counts (steps at levels %s, "
                      "%d baby steps: %d blocks x (1 mul + %s) + %d+3+2x%d rotations per step; tensor products and "
                      "rescales of A and B3, which need no key switch, are left out); one thread: scaled by the "
                      "1-thread / %d-thread time of a mul+relin+rescale and a rotation at level %d (%.1fx)" % (
                          len(giant) if hoisted else 0, nthreads, 3 * sum(sample.values()), t_keys,
                          "/".join(map(str, levels)), n_baby, nb, "1 hoisted sum" if hoisted else "%d rotations" % lc,
                          n_baby - 1, lr, nthreads, lo, t1 / ta),
            "extrapolated": True, "sample_seconds": sample}


if __name__ == "__main__":
    main()
