"""Oriented directional comparisons (Fig. 3: along t, x and the t-x diagonal) on the GPU
against the FP64 oracle: face and body diagonals of the 26-neighbourhood, Gaussian weights
in the Euclidean step distance, reflection of every coordinate at the volume faces."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu
TOL = 1e-5

MASKS = {
    "tx": (sal.RAY_DIAG_TX, sal.RAY_DIAG_TX, sal.RAY_DIAG_TX),
    "mixed": (sal.RAY_PT | sal.RAY_MT | sal.RAY_DIAG_TX, sal.RAY_BODY, sal.RAY_DIAG_XY | sal.RAY_PY),
    "all26": (sal.RAY_ALL,) * 3,
}


def relmax(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.mark.parametrize("name", list(MASKS))
def test_dcs_vs_oracle(name):
    rays = MASKS[name]
    ctx = sal.Saliency(L=8, rays=rays)
    E = np.random.default_rng(3).random((3, 12, 17, 21)).astype(np.float32)
    S = ctx.directional_compare(torch.from_numpy(E).cuda()).cpu().numpy()
    ref = O.dcs(E.astype(np.float64), 4, 2.0, rays)
    assert relmax(S, ref) <= TOL


@pytest.mark.parametrize("d", [8, 32])
def test_dcs_single_rays_vs_oracle(d):
    """Every ray bit on its own, so a step assigned to the wrong bit cannot hide inside a
    symmetric set.  d = 8 (r = 4) runs the tiled kernel; d = 32 (r = 16) sends the rays with
    a t step to the grid-stride kernel, whose ring of t-planes would not fit in LDS."""
    r = d // 2
    E = np.random.default_rng(11).random((3, 2 * r + 3, 2 * r + 5, 2 * r + 7)).astype(np.float32)
    Eg = torch.from_numpy(E).cuda()
    for b in range(26):
        rays = (1 << b,) * 3
        ctx = sal.Saliency(L=8, d=d, rays=rays)
        S = ctx.directional_compare(Eg).cpu().numpy()
        ref = O.dcs(E.astype(np.float64), r, d / 4.0, rays)
        assert relmax(S, ref) <= TOL, (d, b, relmax(S, ref))


def test_dcs_bit_exact_unweighted():
    """sigma = inf, integer E, four t-x diagonals with r = 4 (Q = 16): every partial sum
    is an exact integer and the division by 16 is exact."""
    rays = MASKS["tx"]
    ctx = sal.Saliency(L=8, sigma=math.inf, rays=rays)
    E = np.abs(synth.integer_volume((3, 9, 10, 11), seed=6)).astype(np.float32)
    S = ctx.directional_compare(torch.from_numpy(E).cuda()).cpu().numpy().astype(np.float64)
    ref = O.dcs(E.astype(np.float64), 4, math.inf, rays)
    assert np.array_equal(S, ref)


@pytest.mark.parametrize("L,name", [(8, "mixed"), (5, "tx"), (16, "all26")])
def test_saliency_vs_oracle(L, name):
    rays = MASKS[name]
    shape = (20, 22, 24) if L < 16 else (20, 18, 33)
    V = synth.make_volume(shape, seed=L, n_faults=1, throw=2)
    ctx = sal.Saliency(L=L, rays=rays)
    ref = O.saliency(V, O.Params(L=L, rays=rays))
    S, E, Sr, st = ctx.saliency_maps(torch.from_numpy(V).cuda())
    Sr, S = Sr.cpu().numpy(), S.cpu().numpy()
    for m in range(3):
        assert relmax(Sr[m], ref["S_raw"][m]) <= TOL, (m, relmax(Sr[m], ref["S_raw"][m]))
    assert relmax(S, ref["S"]) <= TOL


def test_box_oriented():
    rays = MASKS["all26"]
    V = torch.from_numpy(synth.make_volume((30, 28, 26), seed=2)).cuda()
    ctx = sal.Saliency(L=8, rays=rays)
    _, _, Sr, _ = ctx.saliency_maps(V)
    box = ctx.raw_box(V, (0, 10, 19), (12, 9, 7))
    torch.cuda.synchronize()
    assert torch.equal(box, Sr[:, 0:12, 10:19, 19:26])
