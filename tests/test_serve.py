"""Serving loop: admission logic on the CPU with a simulated backend, and on
the GPU: every request's result is bit-identical alone and in the mix."""
import numpy as np
import pytest

from paper_2006_10091_amd import serve as SV


class FakeBackend:
    """Each launch completes `dur` seconds after it starts (wall clock)."""

    def __init__(self, dur, nbytes):
        self.dur, self.nbytes = dur, nbytes
        self.log = []
        self.live = 0
        self.max_live = {}

    def bytes(self, q):
        return self.nbytes(q)

    def launch(self, lane, q):
        import time
        self.live += 1
        self.max_live[lane[0]] = max(self.max_live.get(lane[0], 0), sum(1 for e in self.log if e[2] is None
                                                                        and e[1][0] == lane[0]) + 1)
        self.log.append([q.rid, lane, None])
        return (time.perf_counter() + self.dur(q), len(self.log) - 1)

    def done(self, h):
        import time
        return time.perf_counter() >= h[0]

    def finish(self, h, q):
        self.log[h[1]][2] = True
        self.live -= 1


def test_request_generator_shapes():
    reqs = SV.make_requests(400, 200.0, seed=1)
    gaps = np.diff([0.0] + [q.arrival for q in reqs])
    assert abs(np.mean(gaps) - 1 / 200) < 0.25 / 200
    for q in reqs:
        assert 512 <= q.n <= 16384 and 16 <= q.d <= 512 and q.c >= q.d and q.c < 2 * q.d
        assert q.c * q.r == 1 << (q.log_n - 1) and q.nb == -(-q.n // q.r)
    kinds = [q.kind for q in reqs]
    assert 0.4 < kinds.count("grad") / len(kinds) < 0.6
    assert {q.log_n for q in reqs} == {15, 16}


def test_loop_respects_lanes_and_budget_and_order():
    reqs = SV.make_requests(60, 2000.0, seed=2)
    be = FakeBackend(lambda q: 0.002, lambda q: 10)
    times, peak = SV.run_loop(reqs, be, {15: 2, 16: 1}, budget=25)
    assert len(times) == 60 and peak <= 25
    assert all(t[0] >= q.arrival - 1e-9 and t[1] >= t[0] for q, t in ((q, times[q.rid]) for q in reqs))
    assert be.max_live.get(16, 0) <= 1 and be.max_live.get(15, 0) <= 2
    # within one ring degree, admission follows arrival order
    for k in (15, 16):
        adm = [times[q.rid][0] for q in reqs if q.log_n == k]
        assert adm == sorted(adm)


def test_loop_memory_admission_waits_but_other_ring_proceeds():
    """A request too big to share the budget waits; the other ring keeps running."""
    reqs = [SV.Request(0, 0.0, "grad", 16, 512, 16, 16, 1024, 1), SV.Request(1, 0.0, "grad", 16, 512, 16, 16, 1024, 1),
            SV.Request(2, 0.0, "infer", 15, 512, 16, 16, 512, 1)]
    be = FakeBackend(lambda q: 0.02, lambda q: 60 if q.log_n == 16 else 30)
    times, peak = SV.run_loop(reqs, be, {15: 1, 16: 2}, budget=100)
    assert peak <= 100
    # request 1 (ring 2^16, second lane free) waits for memory, request 2 (2^15) does not
    assert times[1][0] >= times[0][1] - 1e-3
    assert times[2][0] < times[0][1]
    with pytest.raises(ValueError):
        SV.run_loop(reqs[:1], FakeBackend(lambda q: 0.0, lambda q: 1000), {16: 1}, budget=100)


@pytest.mark.gpu
def test_serving_results_identical_alone_and_in_the_mix():
    pytest.importorskip("torch")
    reqs = SV.make_requests(40, 400.0, seed=5, n_range=(512, 4096), d_range=(16, 128))
    stats, be, times = SV.serve(reqs, lanes=2, mode=1, keep_results=True)
    mix = dict(be.results)
    assert len(mix) == 40 and stats["p99_latency_ms"] >= stats["p50_latency_ms"] > 0
    # overlap: some request was admitted before an earlier one had completed
    ordered = sorted(reqs, key=lambda q: times[q.rid][0])
    assert any(times[b.rid][0] < times[a.rid][1] for a, b in zip(ordered, ordered[1:]))
    # alone: one request at a time on lane 0 of its ring
    be.results.clear()
    for q in reqs:
        h = be.launch((q.log_n, 0), q)
        be.torch.cuda.synchronize()
        be.finish(h, q)
        alone = be.results[q.rid]
        assert len(alone) == len(mix[q.rid])
        for a, b in zip(alone, mix[q.rid]):
            assert np.array_equal(a, b), q


@pytest.mark.gpu
def test_serving_chain_step_and_margins_bit_exact():
    """The serving parameters (8 + 2 primes, two-prime digits, N = 2^15): one
    gradient step and one margins call, as a serving lane runs them, bit for
    bit against the oracle."""
    import numpy as np
    from oracle import ckks as O
    from oracle import lr as LR
    from paper_2006_10091_amd import he as H
    from paper_2006_10091_amd import serve as SV
    from paper_2006_10091_amd import synth
    cfg = (15, SV.CHAIN["n_q"], SV.CHAIN["n_special"], SV.CHAIN["alpha"], SV.CHAIN["log_delta"])
    P = O.Params(*cfg)
    ctx = H.Context(*cfg)
    n, d = 1500, 24
    g = synth.rng(12)
    X = g.uniform(0.0, 1.0, size=(n, d))
    y = np.where(g.uniform(size=n) < 0.5, 1.0, -1.0)
    blocks, c, r = LR.pack_blocks(X, y, P.S)
    steps = LR.rotation_steps(c, r)
    okeys, gk = O.Keys(P, 2019, rot_steps=steps), ctx.keygen(2019, steps)
    L = P.L
    oZ, gZ = [], ctx.ct_block(len(blocks), L)
    for i in range(len(blocks)):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, okeys, m, L, P.delta, 8, i))
        ctx.encrypt(ctx.pt_load(m, L, P.delta), gk, 8, i, out=gZ[i])
    w = g.uniform(-0.05, 0.05, size=d)
    mw = O.encode(LR.pack_weights(w, P.S, c), P.delta, P.N)
    oW = O.encrypt_sk(P, okeys, mw, L, P.delta, 8, 999)
    gW = ctx.encrypt(ctx.pt_load(mw, L, P.delta), gk, 8, 999)
    coef = [0.5, -0.1501204134, 0.0, 0.0015930174]
    pl = LR.plan_lr_step(P.q, L, P.delta, P.delta, coef, 1.0 / n)
    mm = O.encode(LR.column_mask(P.S, c), pl["s_mask"], P.N)
    oWn, og = LR.lr_grad_step(P, okeys, oZ, oW, mm, coef, 1.0 / n, c, r, plan=pl)
    Wn, gg = ctx.lr_grad_step(gZ, gW, ctx.pt_load(mm, L - 1, pl["s_mask"]), coef, 1.0 / n, c, r, gk, mode=1)
    assert np.array_equal(ctx.download(Wn), oWn.data) and np.array_equal(ctx.download(gg), og.data)
    want = LR.lr_margins(P, okeys, oZ, oW, c, r)
    got = ctx.lr_margins(gZ, gW, c, r, gk, mode=1)
    for a, b in zip(got, want):
        assert np.array_equal(ctx.download(a), b.data)
