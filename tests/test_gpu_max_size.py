"""The largest volume the library accepts (2^31 - 1 voxels at most): 2047 x 1024 x 1024 =
2,146,435,072 voxels, 8 GiB.  Every index of the fused kernels, the directional comparison and
the statistics then spans nearly the whole 32-bit range.  The volume is the 256 x 512 x 512
survey volume tiled 8 x 2 x 2 (then cut to 2047 rows); the raw maps of seeded 16^3 blocks at the
far faces and inside are compared with the FP64 oracle, computed on a crop that reaches the
block's whole dependence (or the true volume face), and the volume-wide statistics with a
reduction of the GPU's own raw maps."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu

SHAPE = (2047, 1024, 1024)
BLOCK = 16


def relmax(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def volume():
    assert SHAPE[0] * SHAPE[1] * SHAPE[2] <= 2 ** 31 - 1
    base = torch.from_numpy(synth.workload("survey256x512x512")).cuda()
    V = base.repeat(8, 2, 2)[:SHAPE[0]].contiguous()
    del base
    torch.cuda.empty_cache()
    return V


def crop_for(V, lo, h, s=1):
    """Host copy of V around the block [lo, lo + BLOCK) extended by h on every side (clipped at
    the volume faces, where the oracle then reflects exactly as on the whole volume); with
    windows on a stride-s lattice the crop starts on a lattice row."""
    c_lo = [max(0, a - h) // s * s for a in lo]
    c_hi = [min(n, a + BLOCK + h) for a, n in zip(lo, V.shape)]
    crop = V[c_lo[0]:c_hi[0], c_lo[1]:c_hi[1], c_lo[2]:c_hi[2]].cpu().numpy()
    return crop, [a - c for a, c in zip(lo, c_lo)]


@pytest.mark.parametrize("L,prec,tol,stride", [(8, sal.FP32, 1e-5, 1), (16, sal.FP32, 1e-5, 1),
                                               (16, sal.BF16_SPLIT, 1e-3, 1), (8, sal.FP32, 1e-5, 2)])
def test_max_size_volume(volume, L, prec, tol, stride):
    V = volume
    print("max-size volume %s L=%d precision %d stride %d" % (tuple(V.shape), L, prec, stride), flush=True)
    ctx = sal.Saliency(L=L, precision=prec, stride=stride)
    shp = (3,) + tuple(V.shape)
    E = torch.empty(shp, dtype=torch.float32, device=V.device)
    Sr = torch.empty(shp, dtype=torch.float32, device=V.device)
    st = torch.empty(sal.STATS_LEN, dtype=torch.float64, device=V.device)
    S = ctx.saliency(V, E_out=E, S_raw_out=Sr, stats_out=st)
    torch.cuda.synchronize()
    stats = st.cpu().numpy()
    # volume-wide statistics: min and max of the GPU's own raw maps, and max |V|, exactly
    for m in range(3):
        assert stats[2 * m] == float(Sr[m].amin()) and stats[2 * m + 1] == float(Sr[m].amax()), m
    assert stats[6] == float(V.abs().amax())
    assert torch.isfinite(S).all()
    # a block's raw maps depend on V up to r + L/2 = L voxels away (d = L, r = L/2), plus one
    # lattice step with strided windows
    h = L + (stride if stride > 1 else 0)
    rng = np.random.default_rng(2047 + L)
    far = [n - BLOCK for n in V.shape]
    blocks = [far, [far[0], int(rng.integers(0, V.shape[1] - BLOCK)), int(rng.integers(0, V.shape[2] - BLOCK))],
              [int(rng.integers(0, n - BLOCK)) for n in V.shape]]
    for lo in blocks:
        crop, lo_c = crop_for(V, lo, h, stride)
        if stride == 1:
            Eo, So = O.raw_box(crop, O.Params(L=L), lo_c, (BLOCK,) * 3)
        else:
            ref = O.saliency(crop, O.Params(L=L, stride=stride))
            bsl = (slice(None),) + tuple(slice(a, a + BLOCK) for a in lo_c)
            Eo, So = ref["E"][bsl], ref["S_raw"][bsl]
        sl = (slice(None),) + tuple(slice(a, a + BLOCK) for a in lo)
        eg, sg = E[sl].cpu().numpy(), Sr[sl].cpu().numpy()
        for m in range(3):
            assert relmax(eg[m], Eo[m]) <= tol, ("E", lo, m, relmax(eg[m], Eo[m]))
            assert relmax(sg[m], So[m]) <= tol, ("S_raw", lo, m, relmax(sg[m], So[m]))
        Sref = O.combine_with_stats(So, stats[:6], vmax=stats[6])
        sb = S[tuple(slice(a, a + BLOCK) for a in lo)].cpu().numpy()
        assert np.abs(sb - Sref).max() <= 10 * tol, ("S", lo, float(np.abs(sb - Sref).max()))
        print("  block %s: E %.2e S_raw %.2e" % (lo, max(relmax(eg[m], Eo[m]) for m in range(3)),
                                                 max(relmax(sg[m], So[m]) for m in range(3))), flush=True)
    del E, Sr, S
    torch.cuda.empty_cache()
