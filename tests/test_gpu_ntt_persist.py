"""The single-launch NTT forms against the two-launch form, bit for bit, over
ring degrees, batch sizes (fewer limbs than XCDs included), launch shapes and
both directions; and forward then inverse is the identity:
  * the persistent form (both passes in one launch, the intermediate kept in
    each XCD's L2, workgroups handing limbs over through per-XCD tickets);
  * the workgroup-per-limb forms (512 or 1024 threads transform a whole limb
    through a scratch limb of their own, no inter-workgroup waits);
  * the two-launch form with XCD-grouped block order (modes 4 and 5), which
    also reorders the fused passes: a key switch and a rescale are compared
    with the default order too."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2006_10091_amd import synth  # noqa: E402

SHAPES = [(64, 2), (1, 1), (13, 3), (128, 2), (96, 1)]


@pytest.mark.parametrize("log_n", [13, 14, 15, 16])
def test_persistent_ntt_matches_two_launch(log_n):
    from paper_2006_10091_amd import he as H
    ctx = H.Context(log_n, 20, 4, 4, 40)
    N = ctx.N
    for nl, per in ((1, 1), (3, 1), (7, 7), (24, 24), (200, 20), (774, 18)):
        host = np.concatenate([synth.uniform_residues(nl * 10 + b, ctx.primes[:per], N).ravel()
                               for b in range(nl // per)])
        src = torch.from_numpy(host.view(np.int64)).cuda()
        print("2^%d: %d limbs, period %d" % (log_n, nl, per), flush=True)
        for d in (1, -1):
            ref = src.clone()
            ctx.set_ntt(0)
            ctx.ntt(ref, nl, 0, per, d)
            for wg, lag in SHAPES:
                x = src.clone()
                ctx.set_ntt(1, wg, lag)
                ctx.ntt(x, nl, 0, per, d)
                assert torch.equal(x, ref), (nl, per, d, wg, lag)
        x = src.clone()
        ctx.set_ntt(1, 64, 2)
        ctx.ntt(x, nl, 0, per, 1)
        ctx.ntt(x, nl, 0, per, -1)
        assert torch.equal(x, src)
    # the threshold: small transforms take the two-launch form, same values
    ctx.set_ntt(1, 64, 2, min_limbs=100)
    x = src.clone()
    ctx.ntt(x, nl, 0, per, 1)
    ctx.set_ntt(0)
    y = src.clone()
    ctx.ntt(y, nl, 0, per, 1)
    assert torch.equal(x, y)
    with pytest.raises(H.HEError):
        ctx.set_ntt(1, 64, 4)  # lag below the slot count only


@pytest.mark.parametrize("log_n", [12, 13, 14, 15, 16])
def test_workgroup_per_limb_ntt_matches_two_launch(log_n):
    from paper_2006_10091_amd import he as H
    ctx = H.Context(log_n, 20, 4, 4, 40)
    N = ctx.N
    for nl, per in ((1, 1), (5, 5), (24, 24), (300, 20), (774, 18)):
        host = np.concatenate([synth.uniform_residues(nl * 10 + b, ctx.primes[:per], N).ravel()
                               for b in range(nl // per)])
        src = torch.from_numpy(host.view(np.int64)).cuda()
        print("2^%d: %d limbs, period %d" % (log_n, nl, per), flush=True)
        for d in (1, -1):
            ref = src.clone()
            ctx.set_ntt(0)
            ctx.ntt(ref, nl, 0, per, d)
            for mode, wg in ((2, 32), (2, 64), (2, 1), (3, 32), (3, 7)):
                x = src.clone()
                ctx.set_ntt(mode, wg)
                ctx.ntt(x, nl, 0, per, d)
                assert torch.equal(x, ref), (nl, per, d, mode, wg)
        for mode in (2, 3):
            x = src.clone()
            ctx.set_ntt(mode, 32)
            ctx.ntt(x, nl, 0, per, 1)
            ctx.ntt(x, nl, 0, per, -1)
            assert torch.equal(x, src)
    ctx.set_ntt(0)


@pytest.mark.parametrize("log_n", [13, 14, 16])
def test_xcd_grouped_order_matches_default(log_n):
    from paper_2006_10091_amd import he as H
    ctx = H.Context(log_n, 20, 4, 4, 40)
    N = ctx.N
    for nl, per in ((1, 1), (7, 7), (300, 20), (774, 18)):
        host = np.concatenate([synth.uniform_residues(nl * 10 + b, ctx.primes[:per], N).ravel()
                               for b in range(nl // per)])
        src = torch.from_numpy(host.view(np.int64)).cuda()
        print("2^%d: %d limbs, period %d" % (log_n, nl, per), flush=True)
        for d in (1, -1):
            ref = src.clone()
            ctx.set_ntt(0)
            ctx.ntt(ref, nl, 0, per, d)
            for mode in (4, 5):
                x = src.clone()
                ctx.set_ntt(mode)
                ctx.ntt(x, nl, 0, per, d)
                assert torch.equal(x, ref), (nl, per, d, mode)
    # the fused passes: a relinearised, rescaled product and a rotation
    keys = ctx.keygen(3, [1, 5])
    q = ctx.primes[:13]
    a = ctx.upload(np.stack([synth.uniform_residues(1, q, N), synth.uniform_residues(2, q, N)]), 12, 1.0)
    b = ctx.upload(np.stack([synth.uniform_residues(3, q, N), synth.uniform_residues(4, q, N)]), 12, 1.0)
    outs = {}
    for mode in (0, 4, 5):
        ctx.set_ntt(mode)
        r = ctx.rescale(ctx.relin(ctx.mul(a, b), keys))
        outs[mode] = (ctx.download(r), ctx.download(ctx.rotate(r, 5, keys)))
    for mode in (4, 5):
        assert all(np.array_equal(u, v) for u, v in zip(outs[mode], outs[0])), mode
    ctx.set_ntt(0)
