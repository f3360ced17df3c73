"""Volumes streamed from pinned host memory in slabs along t, against the resident path.

A slab computed with the exact halo of the method gives the same raw maps as the whole
volume on the device, so the streamed raw maps must equal the resident ones bit for bit
when the per-voxel arithmetic does not depend on where a slab starts (every kernel that
contracts each window on its own), and the final map must match the oracle like the
resident one does.  At cube 16 in FP32 the windows slide along t and restart their running
spectra at fixed rows of the volume they are given, other rows in a slab: there the streamed
maps equal the resident ones to rounding.  Slab sizes below the halo, ragged last slabs and
a single slab are covered.
"""
import numpy as np
import pytest
import torch

from paper_1901_11095_amd import sal, stream, surrogate, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,shape,slab", [
    (8, (40, 24, 28), 8),      # slab below the halo (8): four slabs, one ragged
    (8, (37, 20, 33), 16),     # ragged last slab
    (16, (50, 40, 36), 24),    # cube 16 with the direct t contraction
    (8, (12, 16, 16), 64),     # one slab
])
def test_plain_streamed_equals_resident(L, shape, slab):
    V = synth.make_volume(shape, seed=5, n_faults=1, throw=3, n_chaotic=1, chaotic_size=8)
    ctx = sal.Saliency(L=L, t_direct=True)
    Vd = torch.from_numpy(V).cuda()
    S, E, Sr, st = ctx.saliency_maps(Vd)
    S2, Sr2, st2 = stream.plain_streamed(ctx, stream.pinned(V), slab=slab)
    torch.cuda.synchronize()
    assert torch.equal(Sr2, Sr)
    assert torch.equal(st2[:7], st[:7])   # max|V| reduced slab by slab by sal_absmax
    assert torch.equal(S2, S)


def test_plain_streamed_sliding_to_rounding():
    """Cube 16, FP32, windows sliding along t: slabs of 24 output rows (56 rows with the
    halo, so the slabs slide too) against the resident volume of 90 rows."""
    V = synth.make_volume((90, 40, 36), seed=5, n_faults=1, throw=3, n_chaotic=1, chaotic_size=8)
    ctx = sal.Saliency(L=16)
    Vd = torch.from_numpy(V).cuda()
    S, E, Sr, st = ctx.saliency_maps(Vd)
    S2, Sr2, st2 = stream.plain_streamed(ctx, stream.pinned(V), slab=24)
    torch.cuda.synchronize()
    for m in range(3):
        assert float((Sr2[m] - Sr[m]).abs().max()) <= 1e-6 * float(Sr[m].abs().max()), m
    assert st2[6].item() == st[6].item()   # max|V|, exact
    assert float((S2 - S).abs().max()) <= 1e-5


def test_plain_streamed_matches_oracle(oracle_mod):
    shape = (30, 20, 22)
    V = synth.make_volume(shape, seed=11, n_faults=1, throw=2, n_chaotic=0)
    ctx = sal.Saliency(L=8)
    S, _, _ = stream.plain_streamed(ctx, stream.pinned(V), slab=7)
    ref = oracle_mod.saliency(V, oracle_mod.Params(L=8))
    err = np.abs(S.cpu().numpy().astype(np.float64) - ref["S"]).max()
    assert err <= 1e-5, err


def test_plain_streamed_constant_volume():
    """Zero contrast everywhere: the slab-wise max|V| feeds the zero-range rule."""
    V = np.full((20, 16, 16), 3.0, dtype=np.float32)
    ctx = sal.Saliency(L=8)
    S, Sr, st = stream.plain_streamed(ctx, stream.pinned(V), slab=6)
    S_ref = ctx.saliency(torch.from_numpy(V).cuda())
    torch.cuda.synchronize()
    assert torch.equal(S, S_ref)


@pytest.fixture(scope="module")
def net():
    return surrogate.load()


def test_surrogate_streamed_equals_resident(net):
    n = 72
    V = synth.make_volume(**surrogate.volume_kwargs(99, (n, 56, 64)))
    Vd = torch.from_numpy(V).cuda()
    P = net.infer(Vd)
    Sr, vmax = stream.raw_maps_streamed(stream.pinned(V), net.infer, 5, slab=20)
    torch.cuda.synchronize()
    assert torch.equal(Sr, P)
    assert vmax == float(Vd.abs().max())


def test_surrogate_streamed_tiles_within_bound(net):
    shape = (80, 64, 64)
    V = synth.make_volume(**surrogate.volume_kwargs(99, shape))
    ctx = sal.Saliency(L=16)
    res = stream.surrogate_streamed(net, ctx, stream.pinned(V), slab=24, tile=32, frac=0.3,
                                    bound=0.02, seed=1)
    Vd = torch.from_numpy(V).cuda()
    ref = surrogate.infer_with_fallback(net, ctx, Vd, tile=32, frac=0.3, bound=0.02, seed=1)
    torch.cuda.synchronize()
    assert [t for t, _ in res["tiles"]] == [t for t, _ in ref["tiles"]]
    assert torch.equal(res["S_raw"], ref["S_raw"])
    assert torch.equal(res["S"], ref["S"])
    assert bool(torch.isfinite(res["S"]).all())
