"""The kernel trace (he_ctx_trace): one record per launch with the kind and
the algorithmic work its launch site states, results unchanged by tracing,
and nothing recorded for launches under graph capture."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2006_10091_amd import synth  # noqa: E402


def test_trace_of_plain_ntts_counts_both_passes():
    from paper_2006_10091_amd import he as H
    ctx = H.Context(16, 20, 4, 4, 40)
    N, per, nl = ctx.N, 24, 48
    ctx.set_ntt(0)
    host = np.concatenate([synth.uniform_residues(7 + b, ctx.primes[:per], N).ravel() for b in range(nl // per)])
    src = torch.from_numpy(host.view(np.int64)).cuda()
    ref = src.clone()
    ctx.ntt(ref, nl, 0, per, 1)
    x = src.clone()
    ctx.trace(True)
    ctx.ntt(x, nl, 0, per, 1)
    assert torch.equal(x, ref)
    ctx.ntt(x, nl, 0, per, -1)
    ctx.trace(False)
    ctx.ntt(x, nl, 0, per, 1)  # not recorded
    st = {s["kind"]: s for s in ctx.trace_read()}
    assert sorted(st) == [0, 1, 2, 3]  # forward columns, rows; inverse rows, columns
    n_fp = sum(1 for i in range(nl) if ctx.primes[i % per] < 2 ** 46)
    for k in range(4):
        assert st[k]["launches"] == 1 and st[k]["ms"] > 0
        assert st[k]["bytes"] == 8 * N * nl  # each pass: the input or the output (not the intermediate)
        assert st[k]["mm_fp64"] == n_fp * (N // 2) * 8  # 8 butterfly stages per pass at 2^16
        assert st[k]["mm_int"] == (nl - n_fp) * (N // 2) * 8
    assert ctx.trace_read() == []  # read clears


def test_trace_leaves_key_switches_unchanged_and_names_their_kernels():
    from paper_2006_10091_amd import he as H
    ctx = H.Context(15, 8, 4, 4, 40)
    N, level = ctx.N, 7
    keys = ctx.keygen(5, [1, 3])
    q = ctx.primes[:level + 1]
    a = ctx.upload(np.stack([synth.uniform_residues(11, q, N), synth.uniform_residues(12, q, N)]), level, 1.0)
    b = ctx.upload(np.stack([synth.uniform_residues(13, q, N), synth.uniform_residues(14, q, N)]), level, 1.0)

    def run():
        r = ctx.rescale(ctx.relin(ctx.mul(a, b), keys))
        return ctx.download(r), ctx.download(ctx.rotate(r, 3, keys))

    ref = run()
    ctx.trace(True)
    got = run()
    ctx.trace(False)
    assert all(np.array_equal(u, v) for u, v in zip(got, ref))
    st = {s["name"]: s for s in ctx.trace_read()}
    for kind in (H.K_MODUP, H.K_KS_COLS, H.K_KS_ROWS, H.K_MD_CONV, H.K_MD_FINISH):
        name = H._lib.he_kernel_kind_name(kind).decode()
        assert name in st and st[name]["launches"] >= 1 and st[name]["bytes"] > 0, name
    assert all(s["ms"] > 0 for s in st.values())


def test_graph_replays_record_nothing():
    from paper_2006_10091_amd import he as H
    ctx = H.Context(14, 8, 2, 2, 40)
    N, level, n = ctx.N, 6, 4
    keys = ctx.keygen(9, [1])
    q = ctx.primes[:level + 1]
    xs, ys = [], []
    for i in range(n):
        xs.append(ctx.upload(np.stack([synth.uniform_residues(40 + 4 * i, q, N),
                                       synth.uniform_residues(41 + 4 * i, q, N)]), level, 1.0))
        ys.append(ctx.upload(np.stack([synth.uniform_residues(42 + 4 * i, q, N),
                                       synth.uniform_residues(43 + 4 * i, q, N)]), level, 1.0))
    out1 = [ctx.ct_empty(level - 1) for _ in range(n)]
    out2 = [ctx.ct_empty(level - 1) for _ in range(n)]
    ctx.trace(True)
    ctx.batch_mul_rotate(xs, ys, [1] * n, keys, mode=1, outs=out1)
    eager = ctx.trace_read()
    assert sum(s["launches"] for s in eager) > 0
    ctx.trace(True)
    for _ in range(2):  # capture, then replay
        ctx.batch_mul_rotate(xs, ys, [1] * n, keys, mode=2, outs=out2)
    assert ctx.trace_read() == []
    ctx.trace(False)
    assert all(np.array_equal(ctx.download(u), ctx.download(v)) for u, v in zip(out1, out2))
