"""Batched tile checks (sal_check_tiles) against the one-tile path (sal_raw_box plus
sal_tile_merge), which the box tests tie to the whole-volume maps.

For every tile of a batch the exact maps must equal sal_raw_box bit for bit, the error must
equal the one-tile check's, and the tiles over the bound must be replaced exactly as one by
one: tiles at the volume faces (grown boxes clipped), ragged last tiles, tiles in a stack
of crops (vol_stride) and in one volume, the FP32, split-BF16 and vector-ALU kernels, all
26 rays.
"""
import numpy as np
import pytest
import torch

from paper_1901_11095_amd import sal, stream, surrogate, synth

pytestmark = pytest.mark.gpu


def _perturbed(Sr, seed):
    """Predicted maps: the exact ones plus noise of up to 4 % of each map's range on the rows
    t < 24, and up to 1 % elsewhere, so tiles there fail a 2 % bound and the others pass."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    rng = (Sr.amax(dim=(1, 2, 3)) - Sr.amin(dim=(1, 2, 3))).view(3, 1, 1, 1).cpu()
    amp = torch.full((1, Sr.shape[1], 1, 1), 0.02)
    amp[:, :24] = 0.08
    noise = (torch.rand(Sr.shape, generator=g) - 0.5) * amp * rng
    return (Sr + noise.cuda()).contiguous()


def _one_by_one(ctx, V, P, stats, tiles, tile, bound):
    P = P.clone()
    errs = torch.zeros(len(tiles), dtype=torch.float32, device="cuda")
    exact = []
    for j, lo in enumerate(tiles):
        td = tuple(min(tile, n - a) for a, n in zip(lo, V.shape))
        X = ctx.raw_box(V, lo, td)
        sal.tile_merge(ctx, P, X, lo, lo, td, stats, bound, errs[j:j + 1])
        exact.append(X)
    return P, errs, exact


@pytest.mark.parametrize("L,prec,rays", [(8, sal.FP32, None), (16, sal.FP32, None), (16, sal.BF16_SPLIT, None),
                                         (5, sal.FP32, None), (8, sal.FP32, (sal.RAY_ALL,) * 3),
                                         (12, sal.FP32, None)])
def test_batch_equals_one_by_one(L, prec, rays):
    shape = (52, 44, 60)
    tile = 16
    V = torch.from_numpy(synth.make_volume(shape, seed=8, n_faults=2, throw=3, n_chaotic=1,
                                           chaotic_size=12)).cuda()
    ctx = sal.Saliency(L=L, precision=prec, **({"rays": rays} if rays else {}))
    _, _, Sr, st = ctx.saliency_maps(V)
    P = _perturbed(Sr, L)
    stats = st.clone()
    # face, corner, interior and ragged tiles (52 = 3*16 + 4, 44 = 2*16 + 12, 60 = 3*16 + 12)
    tiles = [(0, 0, 0), (16, 16, 16), (32, 0, 48), (48, 32, 0), (48, 32, 48), (16, 32, 32), (0, 16, 48)]
    bound = 0.02
    P1, e1, X1 = _one_by_one(ctx, V, P, stats, tiles, tile, bound)
    P2 = P.clone()
    e2 = torch.zeros(len(tiles), dtype=torch.float32, device="cuda")
    by = {}
    for j, lo in enumerate(tiles):
        by.setdefault(tuple(min(tile, n - a) for a, n in zip(lo, shape)), []).append(j)
    for td, js in by.items():
        X = torch.empty((len(js), 3) + td, dtype=torch.float32, device="cuda")
        err = torch.zeros(len(js), dtype=torch.float32, device="cuda")
        los = [tiles[j] for j in js]
        sal.check_tiles(ctx, V, los, P2, los, td, stats, bound, err, exact_out=X)
        torch.cuda.synchronize()
        for k, j in enumerate(js):
            assert torch.equal(X[k], X1[j]), (tiles[j], td)
            e2[j] = err[k]
    torch.cuda.synchronize()
    assert torch.equal(e1, e2)
    assert bool((e1 > bound).any()) and bool((e1 <= bound).any())
    assert torch.equal(P1, P2)


def test_stacked_crops_equal_resident():
    """Tiles in a stack of equal crops (vol_stride), each crop's inner faces L voxels from
    its tile, give the maps of the tiles in the whole volume."""
    L, tile = 16, 16
    shape = (64, 60, 56)
    V = torch.from_numpy(synth.make_volume(shape, seed=3, n_faults=1, n_chaotic=1, chaotic_size=10)).cuda()
    ctx = sal.Saliency(L=L, precision=sal.BF16_SPLIT)
    _, _, Sr, st = ctx.saliency_maps(V)
    P = _perturbed(Sr, 5)
    tiles = [(0, 0, 0), (16, 16, 16), (48, 44, 40), (32, 0, 32)]
    cd = tuple(min(n, tile + 2 * L) for n in shape)
    clo = [tuple(min(max(0, a - L), n - c) for a, n, c in zip(lo, shape, cd)) for lo in tiles]
    stack = torch.stack([V[c[0]:c[0] + cd[0], c[1]:c[1] + cd[1], c[2]:c[2] + cd[2]] for c in clo]).contiguous()
    box = [tuple(a - c for a, c in zip(lo, co)) for lo, co in zip(tiles, clo)]
    bound = 0.02
    Pa, Pb = P.clone(), P.clone()
    ea = torch.zeros(len(tiles), dtype=torch.float32, device="cuda")
    eb = torch.zeros_like(ea)
    Xa = torch.empty((len(tiles), 3, tile, tile, tile), dtype=torch.float32, device="cuda")
    Xb = torch.empty_like(Xa)
    sal.check_tiles(ctx, V, tiles, Pa, tiles, (tile,) * 3, st, bound, ea, exact_out=Xa)
    sal.check_tiles(ctx, stack, box, Pb, tiles, (tile,) * 3, st, bound, eb, exact_out=Xb)
    torch.cuda.synchronize()
    assert torch.equal(Xa, Xb)
    assert torch.equal(ea, eb)
    assert torch.equal(Pa, Pb)
    for k, lo in enumerate(tiles):
        assert torch.equal(Xa[k], Sr[:, lo[0]:lo[0] + tile, lo[1]:lo[1] + tile, lo[2]:lo[2] + tile])


def test_check_tiles_rejects():
    ctx = sal.Saliency(L=8)
    V = torch.zeros((40, 40, 40), device="cuda")
    P = torch.zeros((3, 40, 40, 40), device="cuda")
    st = torch.zeros(8, dtype=torch.float64, device="cuda")
    err = torch.zeros(4, device="cuda")
    with pytest.raises(sal.SalError):   # tile leaves its volume
        sal.check_tiles(ctx, V, [(30, 0, 0)], P, [(0, 0, 0)], (16, 16, 16), st, 0.02, err)
    with pytest.raises(sal.SalError):   # tile leaves the map
        sal.check_tiles(ctx, V, [(0, 0, 0)], P, [(0, 30, 0)], (16, 16, 16), st, 0.02, err)
    with pytest.raises(sal.SalError):   # no tiles
        sal.check_tiles(ctx, V, np.zeros((0, 3)), P, np.zeros((0, 3)), (16, 16, 16), st, 0.02, err)


@pytest.fixture(scope="module")
def net():
    return surrogate.load()


def test_check_many_equals_one_by_one(net):
    """The fallback with batched checks equals the same checks one tile at a time."""
    shape = (64, 64, 96)
    V = torch.from_numpy(synth.make_volume(**surrogate.volume_kwargs(99, shape))).cuda()
    ctx = sal.Saliency(L=16, precision=sal.BF16_SPLIT)
    res = surrogate.infer_with_fallback(net, ctx, V, tile=32, frac=0.2, bound=0.02, seed=2)
    P = net.infer(V)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    sal.normalize_combine(ctx, P, V, stats_out=stats)
    chk = surrogate.TileCheck(ctx, P, stats, lambda lo, hi: (V, (0, 0, 0)), 32, 0.02, len(res["tiles"]))
    order = [chk.tile_of_voxel(int(np.ravel_multi_index(lo, shape))) for lo, _ in res["tiles"]]
    for ti in order:
        chk.check(ti)
    torch.cuda.synchronize()
    assert torch.equal(chk.errors(), res["tile_err"])
    assert torch.equal(P, res["S_raw"])


def test_streamed_restream_equals_kept(net):
    """Checks on slabs streamed again equal checks on the volume kept while streaming."""
    shape = (96, 64, 64)
    V = synth.make_volume(**surrogate.volume_kwargs(7, shape))
    ctx = sal.Saliency(L=16, precision=sal.BF16_SPLIT)
    Vh = stream.pinned(V)
    a = stream.surrogate_streamed(net, ctx, Vh, slab=32, tile=32, frac=0.25, seed=3)
    b = stream.surrogate_streamed(net, ctx, Vh, slab=32, tile=32, frac=0.25, seed=3, keep_volume=False)
    torch.cuda.synchronize()
    assert sorted(t for t, _ in a["tiles"]) == sorted(t for t, _ in b["tiles"])
    assert torch.equal(a["S_raw"], b["S_raw"])
    assert torch.equal(a["S"], b["S"])


@pytest.mark.parametrize("L,rays", [(5, None), (8, None), (16, None), (8, "all26"), (16, "all26"), (11, None)])
def test_check_tiles_vs_oracle(L, rays):
    """The batched check's exact maps (energy launch over the box table, k_dcs_boxes) against
    the oracle's raw maps of each tile, FP32, within 1e-5 of each map's maximum; the error of
    each tile against max |pred - exact| / range computed on the host from the oracle's maps;
    and the replacement of exactly the tiles over the bound."""
    import oracle as O
    print("check_tiles vs oracle L=%d rays=%s" % (L, rays), flush=True)
    shape = (44, 40, 52)
    Vn = synth.make_volume(shape, seed=21, n_faults=2, throw=3, n_chaotic=1, chaotic_size=10)
    V = torch.from_numpy(Vn).cuda()
    ray_masks = (sal.RAY_ALL,) * 3 if rays == "all26" else sal.RAYS_AXIS
    ctx = sal.Saliency(L=L, rays=ray_masks)
    _, _, Sr, st = ctx.saliency_maps(V)
    P = _perturbed(Sr, 7 + L)
    Pn = P.cpu().numpy().astype(np.float64)
    stats = st.cpu().numpy()
    rng = np.array([stats[2 * m + 1] - stats[2 * m] for m in range(3)])
    td = (8, 9, 7)
    # corner, far corner (ragged against the sides), faces, interior
    tiles = [(0, 0, 0), (36, 31, 45), (0, 15, 45), (20, 0, 22), (14, 12, 20), (36, 31, 0)]
    bound = 0.02
    X = torch.empty((len(tiles), 3) + td, dtype=torch.float32, device="cuda")
    err = torch.zeros(len(tiles), dtype=torch.float32, device="cuda")
    P2 = P.clone()
    sal.check_tiles(ctx, V, tiles, P2, tiles, td, st, bound, err, exact_out=X)
    torch.cuda.synchronize()
    Xn, errn, P2n = X.cpu().numpy(), err.cpu().numpy(), P2.cpu().numpy()
    p = O.Params(L=L, rays=ray_masks)
    replaced = 0
    for k, lo in enumerate(tiles):
        _, ref = O.raw_box(Vn, p, lo, td)
        sl = tuple(slice(a, a + d) for a, d in zip(lo, td))
        for m in range(3):
            e = np.abs(Xn[k, m] - ref[m]).max() / np.abs(ref[m]).max()
            assert e <= 1e-5, (lo, m, e)
        host_err = max(float(np.abs(Pn[(m,) + sl] - ref[m]).max() / rng[m]) for m in range(3))
        # the exact maps differ from the oracle's by at most 1e-5 of each map's maximum
        tol = max(1e-5 * float(np.abs(ref[m]).max()) / rng[m] for m in range(3)) + 1e-6 * host_err
        assert abs(float(errn[k]) - host_err) <= tol, (lo, errn[k], host_err, tol)
        if errn[k] > bound:
            replaced += 1
            assert np.array_equal(P2n[(slice(None),) + sl], Xn[k])
        else:
            assert np.array_equal(P2n[(slice(None),) + sl], P.cpu().numpy()[(slice(None),) + sl])
    assert 0 < replaced < len(tiles)
