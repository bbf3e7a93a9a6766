"""he_batch_submit: a list of operation descriptors of mixed kinds and levels.

* every kind (multiply-relinearise-rescale, the same then a rotation, a
  rotation, a rescale, an addition; a rotation by a multiple of the slot
  count; several entries per level, levels 1..20) equals the single-operation
  calls bit for bit, in the plain, grouped and graph-replayed forms;
* a graph replay over new input values (same buffers) gives the new results;
* sampled entries of each kind equal the oracle's operations bit for bit;
* errors are reported before any launch.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ckks as O  # noqa: E402
from paper_2006_10091_amd import he as H  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402

CFG = (14, 21, 4, 4, 40)
EINVAL, ELEVEL, ESCALE, EKEY = 1, 3, 4, 5  # he_status codes


def _ct(ctx, seed, level, scale=1.0):
    q = ctx.primes[: level + 1]
    d = np.stack([synth.uniform_residues(seed, q, ctx.N), synth.uniform_residues(seed + 1, q, ctx.N)])
    return ctx.upload(d, level, scale)


def _draw(ctx, seed):
    g = synth.rng(seed)
    kinds = [H.OP_MUL, H.OP_MUL_ROTATE, H.OP_ROTATE, H.OP_RESCALE, H.OP_ADD]
    ops = []
    for i in range(60):
        op = kinds[i % 5]
        level = int(g.integers(1, 21)) if i < 45 else 9  # many entries at one level
        step = 1 << int(g.integers(0, ctx.log_n - 1))
        if i in (2, 7):
            step = ctx.S  # a whole turn: the identity rotation
        x = _ct(ctx, 1000 + 7 * i, level)
        y = _ct(ctx, 5000 + 7 * i, level) if op in (H.OP_MUL, H.OP_MUL_ROTATE, H.OP_ADD) else None
        ops.append((op, step, x, y, None))
    return ops


def _single(ctx, keys, op, step, x, y):
    if op in (H.OP_MUL, H.OP_MUL_ROTATE):
        r = ctx.rescale(ctx.relin(ctx.mul(x, y), keys))
        return ctx.rotate(r, step, keys) if op == H.OP_MUL_ROTATE else r
    if op == H.OP_ROTATE:
        return ctx.rotate(x, step, keys)
    if op == H.OP_RESCALE:
        return ctx.rescale(x)
    return ctx.add(x, y)


def test_submit_matches_single_operations_in_every_form():
    ctx = H.Context(*CFG)
    keys = ctx.keygen(31, [1 << u for u in range(ctx.log_n - 1)] + [ctx.S])
    ops = _draw(ctx, 17)
    want = [ctx.download(_single(ctx, keys, op, st, x, y)) for op, st, x, y, _ in ops]
    assert ctx.batch_submit_bytes(ops, 1) > 0
    for mode in (0, 1, 2, 2):
        outs = ctx.batch_submit(ops, keys, mode=mode)
        for i, (o, w) in enumerate(zip(outs, want)):
            assert o.level == H.Context.op_out_level(ops[i][0], ops[i][2]), (mode, i)
            assert np.array_equal(ctx.download(o), w), (mode, i, ops[i][0], ops[i][2].level)
        ops = [(op, st, x, y, o) for (op, st, x, y, _), o in zip(ops, outs)]  # same buffers from now on
    # new input values in the same buffers: the replayed graph computes the new results
    for i, (op, st, x, y, o) in enumerate(ops):
        x.tensor.copy_(_ct(ctx, 9000 + 3 * i, x.level).tensor)
    want = [ctx.download(_single(ctx, keys, op, st, x, y)) for op, st, x, y, _ in ops]
    outs = ctx.batch_submit(ops, keys, mode=2)
    for i, (o, w) in enumerate(zip(outs, want)):
        assert np.array_equal(ctx.download(o), w), ("replay", i)


def test_submit_sampled_entries_against_oracle():
    ctx = H.Context(*CFG)
    P = O.Params(*CFG)
    steps = [1, 8, 256]
    keys = ctx.keygen(41, steps)
    okeys = O.Keys(P, 41, rot_steps=steps)
    specs = [(H.OP_MUL, 0, 5), (H.OP_MUL_ROTATE, 8, 12), (H.OP_ROTATE, 256, 20), (H.OP_RESCALE, 0, 3),
             (H.OP_ADD, 0, 7), (H.OP_MUL_ROTATE, 1, 12)]
    ops = []
    for i, (op, st, level) in enumerate(specs):
        x = _ct(ctx, 300 + 11 * i, level)
        y = _ct(ctx, 700 + 11 * i, level) if op in (H.OP_MUL, H.OP_MUL_ROTATE, H.OP_ADD) else None
        ops.append((op, st, x, y, None))
    outs = ctx.batch_submit(ops, keys, mode=1)
    for (op, st, x, y, _), o in zip(ops, outs):
        print("oracle: op %d at level %d" % (op, x.level), flush=True)
        ox = O.CT(ctx.download(x), x.level, 1.0)
        oy = O.CT(ctx.download(y), y.level, 1.0) if y is not None else None
        if op in (H.OP_MUL, H.OP_MUL_ROTATE):
            r = O.rescale(P, O.mul(P, ox, oy, okeys))
            r = O.rotate(P, r, st, okeys) if op == H.OP_MUL_ROTATE else r
        elif op == H.OP_ROTATE:
            r = O.rotate(P, ox, st, okeys)
        elif op == H.OP_RESCALE:
            r = O.rescale(P, ox)
        else:
            r = O.add(P, ox, oy)
        assert np.array_equal(ctx.download(o), r.data), (op, x.level)


def test_submit_errors():
    ctx = H.Context(*CFG)
    keys = ctx.keygen(51, [1])
    x, y = _ct(ctx, 1, 5), _ct(ctx, 3, 5)
    out = ctx.ct_empty(4)

    def code(ops, k=keys):
        try:
            ctx.batch_submit(ops, k)
        except H.HEError as e:
            return e.status
        return 0

    assert code([(9, 0, x, y, out)]) == EINVAL  # op code
    assert code([(H.OP_MUL, 0, x, _ct(ctx, 5, 4), out)]) == ELEVEL
    assert code([(H.OP_ROTATE, 2, x, None, None)]) == EKEY  # no key for 2 steps
    assert code([(H.OP_RESCALE, 0, _ct(ctx, 7, 0), None, ctx.ct_empty(0))]) == ELEVEL
    y2 = _ct(ctx, 9, 5, scale=2.0)
    assert code([(H.OP_ADD, 0, x, y2, None)]) == ESCALE
    # an output overlapping an input or another output
    assert code([(H.OP_ADD, 0, x, y, None), (H.OP_RESCALE, 0, y, None, x)]) == EINVAL
    assert code([(H.OP_RESCALE, 0, x, None, out), (H.OP_RESCALE, 0, y, None, out)]) == EINVAL
    other = H.Context(14, 6, 2, 2, 40)
    assert code([(H.OP_RESCALE, 0, x, None, out)], other.keygen(1, [1])) == EKEY
    # nothing was launched by the refused calls: a valid one still works
    assert ctx.batch_submit([(H.OP_RESCALE, 0, x, None, out)], keys)[0].level == 4
