"""Autotuner of the NTT launch shape (he_ctx_set_ntt), by measurement.

For each ring degree and batch size (limbs per transform) it times the
forward and inverse transforms of uniform residues with HIP events:
  * the two-launch form (one launch per pass, the intermediate through HBM);
  * the persistent form (both passes in one launch, the intermediate kept in
    each XCD's L2) for every workgroups-per-XCD and lag in the grid below;
  * the workgroup-per-limb forms (mode 2: 512 threads, mode 3: 1024 threads
    per limb, intermediate in a scratch limb per workgroup) for every
    workgroups-per-XCD in LIMB_GRID;
  * the two-launch form with XCD-grouped block order (mode 4: column passes,
    mode 5: both passes).
The table maps (log N, batch) to the fastest shape; per ring degree it also
derives the context setting he_ctx_set_ntt takes: the shape that wins at the
largest batch, and min_limbs = the smallest measured batch from
which that shape's mode wins at every larger measured batch.  Every shape
gives bit-identical results (checked here on every measurement).

    python -m paper_2006_10091_amd.autotune [--out ntt_tuning.json] [--quick]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

WG_GRID = (32, 64, 96, 128)
LAG_GRID = (1, 2, 3)
LIMB_GRID = (32, 64)
BATCHES = {14: (24, 192, 1536, 6144), 15: (24, 192, 768, 3072), 16: (24, 120, 768, 5640)}
DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ntt_tuning.json")


def _time(torch, fn, reps):
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps * 1e-3


def tune(log_ns=(14, 15, 16), quick=False, log=print):
    import torch
    from . import he as H
    from . import synth
    wgs, lags = ((64,), (2,)) if quick else (WG_GRID, LAG_GRID)
    table = {}
    settings = {}
    for log_n in log_ns:
        ctx = H.Context(log_n, 20, 4, 4, 40)
        N = ctx.N
        rows = []
        for nl in BATCHES[log_n]:
            per = 24 if nl % 24 == 0 else 20
            host = np.concatenate([synth.uniform_residues(nl + b, ctx.primes[:per], N).ravel()
                                   for b in range(nl // per)])
            src = torch.from_numpy(host.view(np.int64)).cuda()
            x = src.clone()
            reps = max(3, min(50, int(2e8 // (nl * N))))
            res = []
            ref = None
            shapes = [(0, 64, 2)] + [(1, w, g) for w in wgs for g in lags]
            shapes += [(m, w, 2) for m in (2, 3) for w in ((32,) if quick else LIMB_GRID)]
            shapes += [(4, 64, 2), (5, 64, 2)]  # two launches, XCD-grouped block order
            for shape in shapes:
                ctx.set_ntt(shape[0], shape[1], shape[2])
                x.copy_(src)
                ctx.ntt(x, nl, 0, per, 1)
                if ref is None:
                    ref = x.clone()
                elif not torch.equal(x, ref):
                    raise RuntimeError("NTT shape %s changed the result" % (shape,))
                tf = _time(torch, lambda: ctx.ntt(x, nl, 0, per, 1), reps)
                ti = _time(torch, lambda: ctx.ntt(x, nl, 0, per, -1), reps)
                res.append(dict(persistent=shape[0], wg_per_xcd=shape[1], lag=shape[2], fwd_us=tf * 1e6,
                                inv_us=ti * 1e6, gbs=16.0 * N * nl / ((tf + ti) / 2) / 1e9))
            best = min(res, key=lambda r: r["fwd_us"] + r["inv_us"])
            two = res[0]
            rows.append(dict(limbs=nl, best=best, two_launch=two, all=res))
            log("2^%d x %d limbs: two-launch %.0f/%.0f us, best %s %.0f/%.0f us (%.0f GB/s algorithmic)" % (
                log_n, nl, two["fwd_us"], two["inv_us"],
                "mode %d wg %d lag %d" % (best["persistent"], best["wg_per_xcd"], best["lag"])
                if best["persistent"] else "two-launch",
                best["fwd_us"], best["inv_us"], best["gbs"]))
            del src, x, ref
        table[str(log_n)] = rows
        big = rows[-1]["best"]
        if big["persistent"]:
            mins = rows[-1]["limbs"]
            for r in reversed(rows):
                if r["best"]["persistent"] == big["persistent"]:
                    mins = r["limbs"]
                else:
                    break
            settings[str(log_n)] = dict(persistent=big["persistent"], wg_per_xcd=big["wg_per_xcd"], lag=big["lag"],
                                        min_limbs=mins)
        else:
            settings[str(log_n)] = dict(persistent=0, wg_per_xcd=64, lag=2, min_limbs=1)
        del ctx
    return dict(measured=table, settings=settings, when=time.strftime("%Y-%m-%d %H:%M:%S"))


def apply(ctx, path=DEFAULT_OUT):
    """Set a context's NTT launch shape from a tuning table, if one exists for its ring degree."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        s = json.load(f).get("settings", {}).get(str(ctx.log_n))
    if not s:
        return False
    ctx.set_ntt(s["persistent"], s["wg_per_xcd"], s["lag"], s["min_limbs"])
    return True


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--log-n", type=int, nargs="*", default=[14, 15, 16])
    a = ap.parse_args(argv)
    res = tune(tuple(a.log_n), a.quick, log=lambda *x: print(*x, file=sys.stderr, flush=True))
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["settings"]))


if __name__ == "__main__":
    main(sys.argv[1:])
