"""Raw maps of one box of the volume (sal_raw_box) against the whole-volume path.

Energies are computed on the box grown by r and windows reflect at the volume faces only,
so the box values equal the same positions of the whole-volume raw maps, for boxes at the
volume faces and inside, on the whole volume or on a crop holding the box plus floor(L/2) + r.
"""
import pytest
import torch

from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,prec", [(8, sal.FP32), (16, sal.FP32), (16, sal.BF16_SPLIT)])
@pytest.mark.parametrize("lo,dims", [((0, 0, 0), (16, 16, 16)), ((5, 9, 13), (20, 7, 11)),
                                     ((30, 40, 20), (18, 8, 28)), ((1, 0, 47), (3, 48, 1))])
def test_raw_box_equals_whole_volume(L, prec, lo, dims):
    shape = (48, 48, 48)
    V = torch.from_numpy(synth.make_volume(shape, seed=4, n_faults=2, throw=3, n_chaotic=1,
                                           chaotic_size=12)).cuda()
    ctx = sal.Saliency(L=L, precision=prec)
    _, _, Sr, _ = ctx.saliency_maps(V)
    box = ctx.raw_box(V, lo, dims)
    ref = Sr[:, lo[0]:lo[0] + dims[0], lo[1]:lo[1] + dims[1], lo[2]:lo[2] + dims[2]]
    torch.cuda.synchronize()
    assert torch.equal(box, ref)
    # through a crop of the box plus floor(L/2) + r
    h = L // 2 + L // 2
    clo = [max(0, a - h) for a in lo]
    chi = [min(n, a + d + h) for a, d, n in zip(lo, dims, shape)]
    crop = V[clo[0]:chi[0], clo[1]:chi[1], clo[2]:chi[2]].contiguous()
    if min(crop.shape) > L // 2:
        box2 = ctx.raw_box(crop, [a - c for a, c in zip(lo, clo)], dims)
        torch.cuda.synchronize()
        if L in (8, 16) and prec == sal.FP32:
            # windows sliding along t restart their running spectra at fixed rows of the
            # volume they are given, other rows in the crop (or, under 2L rows, each window
            # is contracted on its own): the maps agree to rounding
            assert float((box2 - ref).abs().max()) <= 1e-5 * float(ref.abs().max())
        else:
            assert torch.equal(box2, ref)


@pytest.mark.parametrize("L,stride,lo", [(16, 1, (8, 4, 10)), (8, 1, (4, 4, 10)), (16, 2, (8, 4, 10)),
                                         (16, 5, (8, 4, 10)), (8, 3, (4, 4, 10))])
def test_raw_box_stays_in_its_workspace(L, stride, lo):
    """A box one row deep along t and long along x, whose grown box crosses the restart of the
    sliding sums at t0 = L/2: the energy kernel's per-workgroup partials (one x position per
    sliding workgroup) fit the workspace sal_raw_box_workspace_size gives, and no byte past
    it changes."""
    shape, dims = (40, 120, 40), (1, 100, 16)
    V = torch.from_numpy(synth.make_volume(shape, seed=7, n_faults=1, throw=3, n_chaotic=1,
                                           chaotic_size=8)).cuda()
    ctx = sal.Saliency(L=L, stride=stride)
    _, _, Sr, _ = ctx.saliency_maps(V)
    need = ctx.raw_box_workspace_size(dims)
    buf = torch.full((need + 65536,), 0xA5, dtype=torch.uint8, device="cuda")
    box = ctx.raw_box(V, lo, dims, workspace=buf[:need])
    torch.cuda.synchronize()
    assert bool(torch.all(buf[need:] == 0xA5))
    assert torch.equal(box, Sr[:, lo[0]:lo[0] + dims[0], lo[1]:lo[1] + dims[1], lo[2]:lo[2] + dims[2]])


def test_raw_box_rejects():
    ctx = sal.Saliency(L=8)
    V = torch.zeros((20, 20, 20), device="cuda")
    with pytest.raises(sal.SalError):
        ctx.raw_box(V, (10, 0, 0), (11, 4, 4))
    with pytest.raises(sal.SalError):
        ctx.raw_box(V, (-1, 0, 0), (4, 4, 4))


ORACLE_BOX_CASES = [
    # (L, rays, box origin, box dims): corner, far corner, faces, ragged sides, interior
    (5, None, (0, 0, 0), (6, 7, 9)),
    (5, "all26", (30, 41, 0), (6, 7, 9)),
    (8, None, (0, 20, 44), (9, 12, 4)),
    (8, None, (17, 3, 19), (8, 8, 16)),
    (8, "all26", (0, 0, 0), (5, 6, 7)),
    (8, "all26", (39, 40, 41), (9, 8, 7)),
    (16, None, (40, 0, 17), (8, 13, 6)),
    (16, None, (20, 21, 22), (7, 6, 9)),
    (16, "all26", (0, 43, 0), (5, 5, 7)),
]


@pytest.mark.parametrize("L,rays,lo,dims", ORACLE_BOX_CASES)
def test_raw_box_vs_oracle(L, rays, lo, dims):
    """sal_raw_box (energies of the grown box by the fused kernels, then k_dcs_box) against the
    oracle's raw maps of the same box, FP32, within 1e-5 of the map maximum."""
    import numpy as np

    import oracle as O
    print("raw_box vs oracle L=%d rays=%s lo=%s dims=%s" % (L, rays, lo, dims), flush=True)
    shape = (48, 48, 48)
    Vn = synth.make_volume(shape, seed=11, n_faults=2, throw=3, n_chaotic=1, chaotic_size=12)
    ray_masks = (sal.RAY_ALL,) * 3 if rays == "all26" else sal.RAYS_AXIS
    ctx = sal.Saliency(L=L, rays=ray_masks)
    box = ctx.raw_box(torch.from_numpy(Vn).cuda(), lo, dims).cpu().numpy()
    _, ref = O.raw_box(Vn, O.Params(L=L, rays=ray_masks), lo, dims)
    for m in range(3):
        err = np.abs(box[m] - ref[m]).max() / np.abs(ref[m]).max()
        assert err <= 1e-5, (m, err)
