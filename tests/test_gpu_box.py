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
        assert torch.equal(box2, ref)


def test_raw_box_rejects():
    ctx = sal.Saliency(L=8)
    V = torch.zeros((20, 20, 20), device="cuda")
    with pytest.raises(sal.SalError):
        ctx.raw_box(V, (10, 0, 0), (11, 4, 4))
    with pytest.raises(sal.SalError):
        ctx.raw_box(V, (-1, 0, 0), (4, 4, 4))
