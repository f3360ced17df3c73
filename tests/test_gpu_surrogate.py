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
    # the exact raw maps of the whole volume (the checks run on it, so a replaced tile equals
    # them bit for bit whatever kernel computes the energies)
    exact = surrogate.exact_raw_maps(ctx, V)
    for lo, td in res["tiles"]:
        ex = exact[(slice(None),) + tuple(slice(a, a + d) for a, d in zip(lo, td))]
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


def test_survey_like_volume(net):
    """A volume with the survey's structure and noise (six faults, two chaotic bodies,
    5 dB, 256 x 512 x 512): most 32^3 tiles are within the 2% bound before any fallback,
    and after the check (with the extremes' tiles verified) the final map is close to the
    plain one.  The error is relative to each map's range, which the chaotic bodies set,
    so the same network is further off on smaller volumes of this kind."""
    V = torch.from_numpy(synth.make_volume(shape=(256, 512, 512), seed=7, n_faults=6, n_chaotic=2,
                                           chaotic_size=64, snr_db=5.0)).cuda()
    ctx = sal.Saliency(L=16)
    st = torch.zeros(8, dtype=torch.float64, device="cuda")
    Sr = torch.empty((3,) + tuple(V.shape), dtype=torch.float32, device="cuda")
    S_ref = ctx.saliency(V, S_raw_out=Sr, stats_out=st)
    P = net.infer(V)
    rng = (st[1:6:2] - st[0:6:2]).float().reshape(3, 1, 1, 1)
    err = ((P - Sr).abs() / rng).amax(0)
    tmax = err.reshape(8, 32, 16, 32, 16, 32).amax(dim=(1, 3, 5))
    within = float((tmax <= 0.02).float().mean())
    res = surrogate.infer_with_fallback(net, ctx, V)
    dS = (res["S"] - S_ref).abs()
    print("tiles within bound %.3f, mean |dS| %.4f, extreme rounds %d"
          % (within, float(dS.mean()), res["extreme_rounds"]))
    assert within >= 0.85
    assert float(dS.mean()) <= 0.01
    # no unchecked tile passes the extremes of the checked ones by more than the bound
    chk = {tuple(lo) for lo, _ in res["tiles"]}
    for m in range(3):
        inside = torch.zeros_like(res["S_raw"][m], dtype=torch.bool)
        for lo in chk:
            inside[lo[0]:lo[0] + 32, lo[1]:lo[1] + 32, lo[2]:lo[2] + 32] = True
        a, b = res["S_raw"][m][inside], res["S_raw"][m][~inside]
        tol = 0.02 * float(a.max() - a.min())
        assert float(b.max()) <= float(a.max()) + tol and float(b.min()) >= float(a.min()) - tol


def test_top_saliency_tiles_checked(net, ctx):
    """The default pipeline also checks the 5% of tiles with the highest predicted Eq. (6)
    upper bound (where the network's largest errors sit on survey-sized volumes)."""
    V = held_out(128)
    S_ref = ctx.saliency(V)
    P = net.infer(V)
    st = torch.zeros(8, dtype=torch.float64, device="cuda")
    sal.normalize_combine(ctx, P, V, stats_out=st)
    mm = sal.tile_minmax(ctx, P, 32).cpu().numpy().astype(np.float64)
    s = st.cpu().numpy()
    score = sum((mm[:, 2 * m + 1] - s[2 * m]) / (s[2 * m + 1] - s[2 * m]) / 3 for m in range(3))
    k = int(np.ceil(0.05 * len(score)))
    top = set(np.argsort(-score, kind="stable")[:k].tolist())
    res = surrogate.infer_with_fallback(net, ctx, V)
    checked = {(lo[0] // 32 * 16 + lo[1] // 32 * 4 + lo[2] // 32) for lo, _ in res["tiles"]}
    assert top <= checked
    assert float((res["S"] - S_ref).abs().mean()) <= 0.01


def test_train_real_network_short():
    """The real network (five 3^3 layers, 24 channels) trained by the library's forward,
    backward and Adam kernels on pairs that the plain method labels on two seeded 64^3
    volumes: the loss falls, and on a held-out volume the trained network predicts the raw
    maps better than the untrained one does."""
    cfg = surrogate.TrainConfig(n_volumes=2, shape=(64, 64, 64), seeds=(10, 11), pairs_per_epoch=32 * 216 * 16,
                                epochs=4, batch=32, lr=2e-3, mix=True)
    net, cfg = surrogate.train(cfg, net=sal.Net(seed=0), log=print)
    print("loss history", cfg.history)
    assert cfg.history[-1] < 0.9 * cfg.history[0]
    net0 = sal.Net(seed=0)
    net0.set_output_scale(net.out_scale)
    V = held_out(48)
    Sr = surrogate.exact_raw_maps(sal.Saliency(L=16), V)
    inner = (slice(None), slice(8, 40), slice(8, 40), slice(8, 40))
    e1 = float(((net.infer(V) - Sr)[inner] ** 2).mean())
    e0 = float(((net0.infer(V) - Sr)[inner] ** 2).mean())
    print("held-out MSE trained %.3e untrained %.3e" % (e1, e0))
    assert e1 < 0.8 * e0
