"""Strided windows on the GPU against the FP64 oracle: energies of the windows on the
stride-s lattice, trilinear interpolation to every voxel, Eq. (5) and Eq. (6) on the full
grid.  At cube 8 and 16 in FP32 every stride below L/2 runs on the kernel whose windows slide
along t (on volumes of at least 2L rows); otherwise stride 2 runs on the fused kernels, and
strides 3 .. ceil(L/2) - 1 (overlap above one half) and the non-overlapping s = L on the
window-by-window kernel.  Ragged volumes put
lattice points and held values at every face."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu


def relmax(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def check(L, shape, prec=sal.FP32, tol=1e-5, seed=3, stride=2):
    print("strided L=%d s=%d shape %s precision %d" % (L, stride, shape, prec), flush=True)
    V = synth.make_volume(shape, seed=seed + L, n_faults=1, throw=2, n_chaotic=1, chaotic_size=8)
    ctx = sal.Saliency(L=L, stride=stride, precision=prec)
    ref = O.saliency(V, O.Params(L=L, stride=stride))
    S, E, Sr, st = ctx.saliency_maps(torch.from_numpy(V).cuda())
    E, Sr, S = E.cpu().numpy(), Sr.cpu().numpy(), S.cpu().numpy()
    for m in range(3):
        assert relmax(E[m], ref["E"][m]) <= tol, ("E", m, relmax(E[m], ref["E"][m]))
        assert relmax(Sr[m], ref["S_raw"][m]) <= tol, ("S_raw", m, relmax(Sr[m], ref["S_raw"][m]))
    assert relmax(S, ref["S"]) <= tol, ("S", relmax(S, ref["S"]))


@pytest.mark.parametrize("L", [5, 6, 7, 8])
@pytest.mark.parametrize("shape", [(21, 19, 35), (34, 40, 17)])
def test_strided_fp32(L, shape):
    check(L, shape)


@pytest.mark.parametrize("shape", [(20, 18, 33), (33, 40, 24)])
def test_strided_fp32_L16(shape):
    check(16, shape)


@pytest.mark.parametrize("L", [8, 16])
def test_strided_bf16_split(L):
    check(L, (24, 36, 40), prec=sal.BF16_SPLIT, tol=1e-3)


def test_strided_vol64_paper_cube():
    V = synth.workload("vol64")
    ctx = sal.Saliency(L=5, stride=2)
    ref = O.saliency(V, O.Params(L=5, stride=2))
    S = ctx.saliency(torch.from_numpy(V).cuda()).cpu().numpy()
    assert relmax(S, ref["S"]) <= 1e-5


STRIDES = [(8, 3), (8, 8), (16, 3), (16, 5), (16, 7), (16, 16), (5, 5), (7, 3), (7, 7), (12, 2), (12, 5),
           (12, 12), (2, 2), (3, 3), (6, 6)]


@pytest.mark.parametrize("L,s", STRIDES)
def test_strides_vs_oracle(L, s):
    check(L, (21, 19, 35), stride=s)


def test_stride_4_L16_larger_volume():
    """Stride 4 at cube 16 on a volume of several workgroups' windows per axis."""
    check(16, (45, 38, 51), stride=4)


def test_strided_rejects():
    with pytest.raises(sal.SalError) as ei:
        sal.Saliency(L=8, stride=5)        # neither above half overlap nor non-overlapping
    assert ei.value.status == sal.SAL_E_INVAL
    with pytest.raises(sal.SalError) as ei:
        sal.Saliency(L=8, stride=4)
    assert ei.value.status == sal.SAL_E_INVAL
    with pytest.raises(sal.SalError) as ei:
        sal.Saliency(L=4, stride=2)
    assert ei.value.status == sal.SAL_E_INVAL
    with pytest.raises(sal.SalError) as ei:
        sal.Saliency(L=16, stride=3, precision=sal.BF16_SPLIT)
    assert ei.value.status == sal.SAL_E_UNSUPPORTED


@pytest.mark.parametrize("L,s,prec", [(8, 2, sal.FP32), (16, 2, sal.FP32), (16, 2, sal.BF16_SPLIT), (8, 3, sal.FP32),
                                      (16, 5, sal.FP32), (12, 12, sal.FP32), (5, 2, sal.FP32)])
def test_strided_box_tiles_stream_equal_resident(L, s, prec):
    """With windows on the lattice, the box maps (lattice windows around the grown box,
    interpolated onto it), the batched tile checks and the host-streamed slabs (each starting
    on a lattice row) equal the whole-volume maps bit for bit.  Where the windows slide along
    t (cube 8 and 16, FP32, strides below L/2) a slab restarts the running sums at its own first row:
    there the slabs equal the whole volume to rounding, and bit for bit with every window's
    t contraction computed on its own."""
    from paper_1901_11095_amd import stream
    print("strided box/tiles/stream L=%d s=%d" % (L, s), flush=True)
    shape = (45, 38, 51)
    V = synth.make_volume(shape, seed=31, n_faults=2, throw=3, n_chaotic=1, chaotic_size=10)
    ctx = sal.Saliency(L=L, stride=s, precision=prec)
    Vd = torch.from_numpy(V).cuda()
    S, _, Sr, st = ctx.saliency_maps(Vd)
    for lo, dims in [((0, 0, 0), (9, 10, 11)), ((7, 13, 21), (16, 9, 12)), ((36, 29, 40), (9, 9, 11))]:
        box = ctx.raw_box(Vd, lo, dims)
        torch.cuda.synchronize()
        assert torch.equal(box, Sr[:, lo[0]:lo[0] + dims[0], lo[1]:lo[1] + dims[1], lo[2]:lo[2] + dims[2]]), lo
    td = (8, 8, 8)
    tiles = [(0, 0, 0), (16, 8, 24), (37, 30, 43)]
    X = torch.empty((len(tiles), 3) + td, dtype=torch.float32, device="cuda")
    err = torch.zeros(len(tiles), dtype=torch.float32, device="cuda")
    P = Sr.clone()
    sal.check_tiles(ctx, Vd, tiles, P, tiles, td, st, 0.02, err, exact_out=X)
    torch.cuda.synchronize()
    for k, lo in enumerate(tiles):
        assert torch.equal(X[k], Sr[:, lo[0]:lo[0] + 8, lo[1]:lo[1] + 8, lo[2]:lo[2] + 8]), lo
    assert float(err.max()) == 0.0
    S2, Sr2, _ = stream.plain_streamed(ctx, stream.pinned(V), slab=10)
    torch.cuda.synchronize()
    if L in (8, 16) and prec == sal.FP32 and 2 * s < L:
        for m in range(3):
            assert float((Sr2[m] - Sr[m]).abs().max()) <= 1e-6 * float(Sr[m].abs().max()), m
        assert float((S2 - S).abs().max()) <= 1e-5
        cd = sal.Saliency(L=L, stride=s, t_direct=True)
        Sd, _, Srd, _ = cd.saliency_maps(Vd)
        S3, Sr3, _ = stream.plain_streamed(cd, stream.pinned(V), slab=10)
        torch.cuda.synchronize()
        assert torch.equal(Sr3, Srd) and torch.equal(S3, Sd)
    else:
        assert torch.equal(Sr2, Sr) and torch.equal(S2, S)
