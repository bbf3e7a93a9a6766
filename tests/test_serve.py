"""Serving loop: admission and merging logic on the CPU with a simulated
backend, and on the GPU: every request's result is bit-identical alone and in
the mix (merged launches included), the lanes share one key set, and what the
loop really allocates stays within its budget."""
import numpy as np
import pytest

from paper_2006_10091_amd import serve as SV


class FakeBackend:
    """Each launch completes `dur` seconds after it starts (wall clock)."""

    def __init__(self, dur, nbytes):
        self.dur, self.nbytes = dur, nbytes
        self.log = []
        self.max_live = {}

    def bytes(self, batch):
        return sum(self.nbytes(q) for q in batch)

    def launch(self, lane, batch):
        import time
        live = sum(1 for e in self.log if e[2] is None and e[1][0] == lane[0]) + 1
        self.max_live[lane[0]] = max(self.max_live.get(lane[0], 0), live)
        self.log.append([[q.rid for q in batch], lane, None])
        return (time.perf_counter() + max(self.dur(q) for q in batch), len(self.log) - 1)

    def done(self, h):
        import time
        return time.perf_counter() >= h[0]

    def finish(self, h, batch):
        self.log[h[1]][2] = True


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
    times, peak, launches = SV.run_loop(reqs, be, {15: 2, 16: 1}, budget=25)
    assert len(times) == 60 and peak <= 25 and all(len(x) == 1 for x in launches)
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
    times, peak, _ = SV.run_loop(reqs, be, {15: 1, 16: 2}, budget=100)
    assert peak <= 100
    # request 1 (ring 2^16, second lane free) waits for memory, request 2 (2^15) does not
    assert times[1][0] >= times[0][1] - 1e-3
    assert times[2][0] < times[0][1]
    with pytest.raises(ValueError):
        SV.run_loop(reqs[:1], FakeBackend(lambda q: 0.0, lambda q: 1000), {16: 1}, budget=100)


def _req(rid, kind, c, nb, log_n=16, t=0.0):
    return SV.Request(rid, t, kind, log_n, nb * ((1 << (log_n - 1)) // c), c, c, (1 << (log_n - 1)) // c, nb)


def test_take_batch_merges_same_kind_and_width_only():
    from collections import deque
    qu = deque([_req(0, "infer", 64, 10), _req(1, "grad", 64, 5), _req(2, "infer", 128, 5), _req(3, "infer", 64, 20),
                _req(4, "infer", 64, 30), _req(5, "infer", 64, 1), _req(6, "grad", 64, 7), _req(7, "grad", 32, 2)])
    assert [q.rid for q in SV.take_batch(qu, 40)] == [0, 3, 5]  # 10 + 20 + 1; 30 more would pass 40
    assert [q.rid for q in SV.take_batch(qu, 0)] == [0]
    assert [q.rid for q in SV.take_batch(qu, 1000, max_requests=2)] == [0, 3]
    qu.popleft()
    assert [q.rid for q in SV.take_batch(qu, 1000)] == [1, 6]  # gradient steps of one width merge too
    # a merge key that also tells packings apart (the backend's) keeps them apart
    assert [q.rid for q in SV.take_batch(qu, 1000, merge_key=lambda q: (q.kind, q.c, q.rid % 2))] == [1]


def test_loop_merges_queued_inferences_and_keeps_leaders_in_order():
    reqs = [_req(i, "infer" if i % 3 else "grad", (64, 128)[i % 2], 1 + i % 7, t=i * 1e-4) for i in range(80)]
    be = FakeBackend(lambda q: 0.004, lambda q: q.nb)
    times, peak, launches = SV.run_loop(reqs, be, {16: 2}, budget=10 ** 6, merge_blocks=24)
    by = {q.rid: q for q in reqs}
    assert sorted(r for x in launches for r in x) == list(range(80))
    assert any(len(x) > 1 for x in launches)
    for x in launches:
        qs = [by[r] for r in x]
        if len(qs) > 1:
            assert all(q.kind == qs[0].kind and q.c == qs[0].c for q in qs) and sum(q.nb for q in qs) <= 24
            assert [q.rid for q in qs] == sorted(q.rid for q in qs)
        assert len({times[q.rid][0] for q in qs}) == 1 and len({times[q.rid][1] for q in qs}) == 1
    # leaders (the oldest queued request when admitted) go in arrival order, and
    # nobody is admitted after a leader that arrived later than it
    leaders = [by[x[0]] for x in launches]
    assert [q.rid for q in leaders] == sorted(q.rid for q in leaders)
    for q in reqs:
        later = [times[p.rid][0] for p in leaders if p.rid > q.rid]
        assert all(times[q.rid][0] <= t + 1e-9 for t in later)


def test_merged_launch_sheds_members_to_fit_the_budget():
    reqs = [_req(i, "infer", 64, 10) for i in range(4)]
    be = FakeBackend(lambda q: 0.003, lambda q: q.nb)
    times, peak, launches = SV.run_loop(reqs, be, {16: 1}, budget=25, merge_blocks=1000)
    assert peak <= 25 and [len(x) for x in launches] == [2, 2]


class TightBackend(FakeBackend):
    """The device holds `cap` bytes whatever the budget says: a launch that
    does not fit next to the running ones is refused with DeviceMemoryFull."""

    def __init__(self, dur, nbytes, cap):
        super().__init__(dur, nbytes)
        self.cap, self.live, self.refused = cap, 0, []

    def launch(self, lane, batch):
        b = self.bytes(batch)
        if self.live + b > self.cap:
            self.refused.append([q.rid for q in batch])
            raise SV.DeviceMemoryFull("over the device")
        self.live += b
        return super().launch(lane, batch)

    def finish(self, h, batch):
        self.live -= self.bytes(batch)
        super().finish(h, batch)


def test_launch_refused_for_memory_waits_for_a_completion_and_keeps_order():
    # the budget admits two 10-byte launches at once, the device holds one
    reqs = [_req(i, "infer", 64, 10) for i in range(4)]
    be = TightBackend(lambda q: 0.003, lambda q: q.nb, cap=15)
    st = {}
    times, peak, launches = SV.run_loop(reqs, be, {16: 2}, budget=25, stats=st)
    assert sorted(times) == [0, 1, 2, 3] and all(t[1] is not None for t in times.values())
    assert launches == [[0], [1], [2], [3]]  # in queue order, one at a time
    assert be.refused and st["memory_waits"] == len(be.refused)
    for a, b in zip(launches, launches[1:]):  # each launch waited for the previous one's completion
        assert times[b[0]][0] >= times[a[0]][1] - 1e-9
    # refused with nothing running: an error, not a wait
    with pytest.raises(SV.DeviceMemoryFull):
        SV.run_loop(reqs[:1], TightBackend(lambda q: 0.0, lambda q: q.nb, cap=5), {16: 1}, budget=100)


@pytest.mark.gpu
def test_serving_results_identical_alone_and_in_the_mix():
    pytest.importorskip("torch")
    from paper_2006_10091_amd import he as H
    reqs = SV.make_requests(48, 400.0, seed=5, n_range=(512, 4096), d_range=(16, 128))
    stats, be, times = SV.serve(reqs, lanes=3, mode=1, keep_results=True, merge_blocks=64)
    print(stats, flush=True)
    mix = dict(be.results)
    assert len(mix) == 48 and stats["p99_latency_ms"] >= stats["p50_latency_ms"] > 0
    # overlap: some launch was admitted before an earlier one had completed
    ordered = sorted(reqs, key=lambda q: times[q.rid][0])
    assert any(times[b.rid][0] < times[a.rid][1] for a, b in zip(ordered, ordered[1:]))
    assert stats["merged_launches_grad"] > 0 and stats["merged_launches_infer"] > 0  # both kinds merged
    assert stats["feature_major_steps"] > 0
    # what the loop allocated stayed within its budget (allocator rounding aside)
    assert stats["peak_bytes_allocated"] <= stats["budget_bytes"] + (64 << 20)
    assert stats["peak_bytes_in_flight"] <= stats["budget_bytes"]
    # one key set per ring degree, and no lane holds keys of its own
    assert set(be.keys) == {q.log_n for q in reqs}
    # alone: one request at a time on lane 0 of its ring
    be.results.clear()
    for q in reqs:
        h = be.launch((q.log_n, 0), [q])
        be.torch.cuda.synchronize()
        be.finish(h, [q])
        alone = be.results[q.rid]
        assert len(alone) == len(mix[q.rid])
        for a, b in zip(alone, mix[q.rid]):
            assert np.array_equal(a, b), q
    # a key set of another parameter set is refused
    other = H.Context(15, 6, 2, 2, 40)
    with pytest.raises(H.HEError):
        ctx = be.lanes[(15, 0)]["ctx"]
        ctx.rotate(be.pools[next(k for k in be.pools if k[0] == 15)]["W"], 1, other.keygen(1, [1]))


@pytest.mark.gpu
@pytest.mark.parametrize("layout", ["rows", "features"])
def test_serving_chain_step_and_margins_bit_exact(layout):
    """The serving parameters (8 + 4 primes, four-prime digits, N = 2^15): one
    gradient step in the packing a serving lane picks for it (row-major, or
    feature-major where the plan allows it) and one margins call, bit for bit
    against the oracle."""
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
    fm = layout == "features"
    lay, olay = (H.LAYOUT_FEATURES, LR.FEATURES) if fm else (H.LAYOUT_ROWS, LR.ROWS)
    q = SV.Request(0, 0.0, "grad", 15, n, d, 32, P.S // 32, 0)
    if fm:
        assert SV.step_layout(q, ctx.primes) == H.LAYOUT_FEATURES
    g = synth.rng(12)
    X = g.uniform(0.0, 1.0, size=(n, d))
    y = np.where(g.uniform(size=n) < 0.5, 1.0, -1.0)
    blocks, c, r = (LR.pack_blocks_features if fm else LR.pack_blocks)(X, y, P.S)
    steps = LR.rotation_steps(c, r, olay)
    okeys, gk = O.Keys(P, 2019, rot_steps=steps), ctx.keygen(2019, steps)
    L = P.L
    oZ, gZ = [], ctx.ct_block(len(blocks), L)
    for i in range(len(blocks)):
        m = O.encode(blocks[i], P.delta, P.N)
        oZ.append(O.encrypt_sk(P, okeys, m, L, P.delta, 8, i))
        ctx.encrypt(ctx.pt_load(m, L, P.delta), gk, 8, i, out=gZ[i])
    w = g.uniform(-0.05, 0.05, size=d)
    mw = O.encode((LR.pack_weights_features if fm else LR.pack_weights)(w, P.S, c), P.delta, P.N)
    oW = O.encrypt_sk(P, okeys, mw, L, P.delta, 8, 999)
    gW = ctx.encrypt(ctx.pt_load(mw, L, P.delta), gk, 8, 999)
    coef = SV.COEF
    pl = LR.plan_lr_step(P.q, L, P.delta, P.delta, coef, 1.0 / n, 0.0, olay)
    msk = LR.feature_mask(P.S, r) if fm else LR.column_mask(P.S, c)
    mm = O.encode(msk, pl["s_mask"], P.N)
    print("serving chain, %s step: %d blocks" % (layout, len(blocks)), flush=True)
    oWn, og = LR.lr_grad_step(P, okeys, oZ, oW, mm, coef, 1.0 / n, c, r, plan=pl, layout=olay)
    Wn, gg = ctx.lr_grad_step(gZ, gW, ctx.pt_load(mm, H.mask_level(L, lay), pl["s_mask"]), coef, 1.0 / n, c, r, gk,
                              mode=1, layout=lay)
    assert np.array_equal(ctx.download(Wn), oWn.data) and np.array_equal(ctx.download(gg), og.data)
    want = LR.lr_margins(P, okeys, oZ, oW, c, r, layout=olay)
    got = ctx.lr_margins(gZ, gW, c, r, gk, mode=1, layout=lay)
    for a, b in zip(got, want):
        assert np.array_equal(ctx.download(a), b.data)
