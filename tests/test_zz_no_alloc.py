"""sal_saliency_noalloc (no workspace; the per-block partials and statistics in the library's
per-GPU device scratch) against sal_saliency with a caller workspace: every output bit for
bit, on two calls in a row with the second on a smaller volume (the scratch keeps the first
call's contents), with and without a caller statistics buffer; and its refusals."""
import ctypes

import pytest
import torch

from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu


def _reference(ctx, V):
    S, E, Sr, st = ctx.saliency_maps(V)
    return S, E, Sr, st


def _noalloc(ctx, V, with_stats):
    shp = (3,) + tuple(V.shape)
    S = torch.empty_like(V)
    E = torch.empty(shp, dtype=torch.float32, device=V.device)
    Sr = torch.empty(shp, dtype=torch.float32, device=V.device)
    st = torch.zeros(8, dtype=torch.float64, device=V.device) if with_stats else None
    ctx.saliency_noalloc(V, S, E, Sr, st)
    return S, E, Sr, st


@pytest.mark.parametrize("L,prec", [(8, sal.FP32), (16, sal.BF16_SPLIT), (5, sal.FP32), (16, sal.FP32)])
def test_noalloc_equals_workspace_path(L, prec):
    ctx = sal.Saliency(L=L, precision=prec)
    shapes = [(44, 52, 61), (21, 30, 37)]   # the second call is smaller
    for k, shape in enumerate(shapes):
        print("noalloc L=%d prec=%s shape %s" % (L, sal.PRECISION_NAMES[prec], shape), flush=True)
        V = torch.from_numpy(synth.make_volume(shape, seed=10 + k, n_faults=1, n_chaotic=1,
                                               chaotic_size=8)).cuda()
        S0, E0, Sr0, st0 = _reference(ctx, V)
        for with_stats in (True, False):
            S1, E1, Sr1, st1 = _noalloc(ctx, V, with_stats)
            torch.cuda.synchronize()
            assert torch.equal(S1, S0) and torch.equal(E1, E0) and torch.equal(Sr1, Sr0), (shape, with_stats)
            if with_stats:
                assert torch.equal(st1[:7], st0[:7])


def test_noalloc_refusals():
    ctx = sal.Saliency(L=8)
    buf = torch.zeros(4096, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    lib = ctx._lib
    # E_out and S_raw_out are required
    assert lib.sal_saliency_noalloc(ctx._h, p, 12, 12, 12, p, None, p, None, None) == sal.SAL_E_INVAL
    # a thin volume of 2^31 - 65 voxels has more per-block partials than the scratch holds;
    # refused before anything is enqueued
    st = lib.sal_saliency_noalloc(ctx._h, p, 26512143, 9, 9, p, p, p, None, None)
    assert st == sal.SAL_E_INVAL
    assert b"scratch" in lib.sal_last_error(ctx._h)
    ctx2 = sal.Saliency(L=8, stride=2)
    V = torch.zeros((12, 12, 12), device="cuda")
    E = torch.empty((3, 12, 12, 12), device="cuda")
    with pytest.raises(sal.SalError) as ei:
        ctx2.saliency_noalloc(V, torch.empty_like(V), E, torch.empty_like(E))
    assert ei.value.status == sal.SAL_E_UNSUPPORTED
