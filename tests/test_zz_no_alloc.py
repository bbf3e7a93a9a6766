"""he_rotate_noalloc (the rotation for callers that cannot allocate) against
he_rotate through the C ABI: bit-identical outputs on two calls in a row, the
second with a smaller input, no device allocation inside the call, and the
size limit refused with HE_ENOMEM."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ckks as O  # noqa: E402
from paper_2006_10091_amd import synth  # noqa: E402


def _ct(ctx, P, level, seed):
    d = np.stack([synth.uniform_residues(seed, P.q[: level + 1], P.N),
                  synth.uniform_residues(seed + 1, P.q[: level + 1], P.N)])
    return d, ctx.upload(d, level, 3.0)


@pytest.mark.parametrize("cfg,levels,step", [((13, 5, 2, 2, 40), (4, 1), 3), ((16, 20, 4, 4, 40), (9, 5), -64)])
def test_rotate_noalloc_matches_rotate(cfg, levels, step):
    from paper_2006_10091_amd import he as H
    P = O.Params(*cfg)
    ctx = H.Context(*cfg)
    gk = ctx.keygen(31, [step])
    ok = O.Keys(P, 31, rot_steps=[step])
    for level in levels:  # the second call has the smaller input
        d, x = _ct(ctx, P, level, 100 + level)
        out = ctx.ct_empty(level)
        torch.cuda.synchronize()
        held, alloc = ctx.mem.bytes, torch.cuda.memory_allocated()
        ctx.rotate_noalloc(x, step, gk, out)
        torch.cuda.synchronize()
        assert ctx.mem.bytes == held and torch.cuda.memory_allocated() == alloc  # nothing allocated
        assert (out.level, out.scale) == (level, 3.0)
        ref = ctx.rotate(x, step, gk)
        got = ctx.download(out)
        assert np.array_equal(got, ctx.download(ref))
        assert np.array_equal(got, O.rotate(P, O.CT(d, level, 3.0), step, ok).data)
    assert ctx._noalloc_bytes(levels[0]) <= H.NOALLOC_SCRATCH_BYTES


def test_rotate_noalloc_refuses_beyond_its_scratch():
    from paper_2006_10091_amd import he as H
    cfg = (16, 20, 4, 4, 40)
    ctx = H.Context(*cfg)
    gk = ctx.keygen(31, [1])
    assert ctx._noalloc_bytes(19) > H.NOALLOC_SCRATCH_BYTES >= ctx._noalloc_bytes(9)
    _, x = _ct(ctx, O.Params(*cfg), 19, 7)
    with pytest.raises(H.HEError) as e:
        ctx.rotate_noalloc(x, 1, gk, ctx.ct_empty(19))
    assert e.value.status == 2
