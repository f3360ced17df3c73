"""The trained surrogate with its tile check and exact fallback, against the plain method.

The plain method (FP32 path, itself parity-tested against the FP64 oracle) is the judge:
every checked tile ends within the bound of the plain method's raw maps (kept when within,
replaced by the exact values otherwise), a zero bound reproduces the plain values on every
checked tile, and the surrogate pipeline is measured against the plain pipeline on the
same volume (speed and mean error of the final map).
"""
import time

import numpy as np
import pytest
import torch

from paper_1901_11095_amd import sal, surrogate, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def net():
    return surrogate.load()


@pytest.fixture(scope="module")
def ctx():
    return sal.Saliency(L=16)


def held_out(n):
    return torch.from_numpy(synth.make_volume(**surrogate.volume_kwargs(99, (n, n, n)))).cuda()


def test_inference_finite(net):
    V = held_out(40)
    P = net.infer(V)
    assert P.shape == (3, 40, 40, 40) and bool(torch.isfinite(P).all())


@pytest.mark.parametrize("bound", [0.02, 0.0])
def test_checked_tiles_within_bound(net, ctx, bound):
    V = held_out(96)
    res = surrogate.infer_with_fallback(net, ctx, V, tile=32, frac=0.25, bound=bound, seed=3)
    S_raw, stats = res["S_raw"], res["stats"]
    rng = (stats[1:6:2] - stats[0:6:2]).float()
    for lo, td in res["tiles"]:
        clo = tuple(max(0, a - 16) for a in lo)
        chi = tuple(min(n, a + d + 16) for a, d, n in zip(lo, td, V.shape))
        exact = surrogate.exact_raw_maps(ctx, V[clo[0]:chi[0], clo[1]:chi[1], clo[2]:chi[2]].contiguous())
        sl = tuple(slice(a - c, a - c + d) for a, c, d in zip(lo, clo, td))
        ex = exact[(slice(None),) + sl]
        got = S_raw[(slice(None), slice(lo[0], lo[0] + td[0]), slice(lo[1], lo[1] + td[1]),
                     slice(lo[2], lo[2] + td[2]))]
        err = float(((got - ex).abs() / rng.reshape(3, 1, 1, 1)).max())
        if bound == 0.0:
            assert torch.equal(got, ex)
        else:
            assert err <= bound + 1e-6, (lo, err)
    assert len(res["tiles"]) >= round(0.25 * res["n_tiles"])


def test_surrogate_gain_over_plain_method(net, ctx):
    """What the trained network buys: the surrogate pipeline (inference, 2% seeded tile
    check with split-BF16 fallback, exact normalisation) against the plain FP32 method on a
    256^3 volume: faster, with the mean error of the final map stated."""
    V = held_out(256)
    ctx_fb = sal.Saliency(L=16, precision=sal.BF16_SPLIT)
    S_ref = ctx.saliency(V)
    for _ in range(2):
        surrogate.infer_with_fallback(net, ctx_fb, V)
        ctx.saliency(V)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = surrogate.infer_with_fallback(net, ctx_fb, V)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    t0 = time.perf_counter()
    S_ref = ctx.saliency(V, S=S_ref)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    err = (res["S"] - S_ref).abs()
    print("surrogate %.1f ms, plain %.1f ms, speedup %.1fx, mean |dS| %.4f, max %.3f"
          % (1e3 * t_sur, 1e3 * t_plain, t_plain / t_sur, float(err.mean()), float(err.max())))
    assert t_plain / t_sur > 1.5
    assert float(err.mean()) <= 0.03
