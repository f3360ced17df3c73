"""Surrogate network kernels (BF16 MFMA convolutions, FP32 accumulation) against the FP64
oracle, and the exact normalisation / tile-merge entry points.

Tolerance of the network checks: weights and activations are rounded to BF16 (unit
roundoff 2^-8) at every layer, so the output carries a relative error of a few 2^-9 per
layer; over five layers the relative L2 error stays below 2e-2 (forward) and the gradients,
which pass through the same roundings twice plus BF16 output gradients, below 5e-2.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def net():
    return sal.Net(seed=5)


def test_forward_vs_oracle(net):
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 10, 10, 10)).astype(np.float32)
    p = net.get_params().astype(np.float64)
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = O.net_forward(X[..., None], p)
    err = rel_l2(Y, ref)
    print("forward rel L2 %.3e" % err)
    assert err <= 2e-2


@pytest.mark.parametrize("S", [5, 9, 17])
def test_forward_ragged_cubes(net, S):
    """Cube sides that are not multiples of the 4 x 4 x 16 output tile."""
    rng = np.random.default_rng(S)
    X = rng.standard_normal((3, S, S, S)).astype(np.float32)
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = O.net_forward(X[..., None], net.get_params().astype(np.float64))
    assert rel_l2(Y, ref) <= 2e-2


def test_gradient_vs_oracle(net):
    """dY nonzero only >= 5 voxels from every face: the zero-padded input gradient is then
    the exact adjoint, so the GPU gradient matches the oracle's true gradient."""
    rng = np.random.default_rng(2)
    S = 13
    X = rng.standard_normal((2, S, S, S)).astype(np.float32)
    dY = np.zeros((2, S, S, S, 3), np.float32)
    dY[:, 5:S - 5, 5:S - 5, 5:S - 5, :] = rng.standard_normal((2, S - 10, S - 10, S - 10, 3))
    p = net.get_params().astype(np.float64)
    Xg = torch.from_numpy(X).cuda()
    net.grads(zero=True)
    net.forward(Xg)
    net.backward(Xg, torch.from_numpy(dY).cuda())
    g = net.grads(zero=True).astype(np.float64)
    ref = O.net_backward(X[..., None], p, dY)
    off = 0
    for l in range(5):
        ci, co = O.SURROGATE_CHANNELS[l], O.SURROGATE_CHANNELS[l + 1]
        nw = co * 27 * ci
        ew = rel_l2(g[off:off + nw], ref[off:off + nw])
        eb = rel_l2(g[off + nw:off + nw + co], ref[off + nw:off + nw + co])
        print("layer %d dW rel L2 %.3e db %.3e" % (l, ew, eb))
        assert ew <= 5e-2 and eb <= 5e-2
        off += nw + co


def test_train_step_reduces_loss():
    net = sal.Net(seed=11)
    rng = np.random.default_rng(3)
    S = 16
    X = torch.from_numpy(rng.standard_normal((4, S, S, S)).astype(np.float32)).cuda()
    # a learnable target: a smoothed copy of the input in each channel
    Xn = X.cpu().numpy()
    T = np.stack([Xn, 0.5 * Xn, np.roll(Xn, 1, axis=3)], -1).astype(np.float32)
    Tg = torch.from_numpy(T).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for it in range(60):
        net.train_step(X, Tg, 5, 3e-3, loss_out=loss)
        hist.append(float(loss.item()))
    print("loss", hist[0], hist[-1])
    assert hist[-1] < 0.3 * hist[0]


def test_infer_matches_forward(net):
    rng = np.random.default_rng(4)
    V = torch.from_numpy(rng.standard_normal((12, 20, 35)).astype(np.float32)).cuda()
    Y = net.forward(V[None].contiguous())[0]          # [n0, n1, n2, 3]
    Z = net.infer(V)                                  # [3, n0, n1, n2]
    assert torch.equal(Y.permute(3, 0, 1, 2), Z)


def test_normalize_combine_vs_oracle():
    ctx = sal.Saliency(L=16)
    rng = np.random.default_rng(5)
    S_raw = np.abs(rng.standard_normal((3, 18, 17, 20))).astype(np.float32)
    V = rng.standard_normal((18, 17, 20)).astype(np.float32)
    st = torch.zeros(8, dtype=torch.float64, device="cuda")
    S = sal.normalize_combine(ctx, torch.from_numpy(S_raw).cuda(), torch.from_numpy(V).cuda(),
                              stats_out=st).cpu().numpy()
    ref, stats = O.combine(S_raw.astype(np.float64), vmax=float(np.abs(V).max()))
    assert np.array_equal(st.cpu().numpy()[:6], stats)
    assert st.cpu().numpy()[6] == np.abs(V).max()
    assert np.abs(S - ref).max() <= 1e-6


def test_tile_merge():
    ctx = sal.Saliency(L=16)
    n = (20, 24, 28)
    S_raw = torch.zeros((3,) + n, dtype=torch.float32, device="cuda")
    S_raw[:, 0, 0, 0] = 1.0                              # range [0, 1] for every map
    stats = torch.tensor([0, 1, 0, 1, 0, 1, 1, 0], dtype=torch.float64, device="cuda")
    crop_lo, tile_lo, tile_d = (2, 3, 4), (5, 6, 7), (4, 5, 6)
    exact = torch.zeros((3, 10, 12, 14), dtype=torch.float32, device="cuda")
    exact[1, 4, 4, 4] = 0.01                             # inside the tile: 1% error
    err = torch.zeros(1, dtype=torch.float32, device="cuda")
    sal.tile_merge(ctx, S_raw, exact, crop_lo, tile_lo, tile_d, stats, 0.02, err)
    assert abs(err.item() - 0.01) <= 1e-7
    assert S_raw[1, 6, 7, 8].item() == 0.0               # under the bound: kept
    exact[1, 4, 4, 4] = 0.05
    sal.tile_merge(ctx, S_raw, exact, crop_lo, tile_lo, tile_d, stats, 0.02, err)
    assert abs(err.item() - 0.05) <= 1e-7
    assert abs(S_raw[1, 6, 7, 8].item() - 0.05) <= 1e-7  # over the bound: replaced
    assert S_raw[1, 5, 6, 7].item() == 0.0 and S_raw[0, 0, 0, 0].item() == 1.0


@pytest.mark.parametrize("shape,tile", [((37, 20, 45), 16), ((32, 32, 32), 32), ((5, 7, 3), 4)])
def test_tile_minmax(shape, tile):
    """Per-tile extremes equal a direct reduction over every (ragged) tile, bit for bit."""
    ctx = sal.Saliency(L=8)
    g = torch.Generator().manual_seed(3)
    S_raw = torch.randn((3,) + shape, generator=g).cuda()
    out = sal.tile_minmax(ctx, S_raw, tile).cpu()
    ref = []
    for t in range(0, shape[0], tile):
        for x in range(0, shape[1], tile):
            for y in range(0, shape[2], tile):
                blk = S_raw[:, t:t + tile, x:x + tile, y:y + tile].reshape(3, -1).cpu()
                ref.append(torch.stack([blk.amin(1), blk.amax(1)], 1).reshape(6))
    assert torch.equal(out, torch.stack(ref))


def test_params_roundtrip_and_output_scale(net):
    """sal_net_params writes and reads back the FP32 masters unchanged; the inference output
    is the network output times sal_net_set_output_scale per channel (powers of two here, so
    the products are exact)."""
    p = net.get_params()
    net.set_params(p)
    assert np.array_equal(net.get_params(), p)
    V = torch.from_numpy(np.random.default_rng(9).standard_normal((10, 12, 18)).astype(np.float32)).cuda()
    old = getattr(net, "out_scale", (1.0, 1.0, 1.0))
    try:
        net.set_output_scale((1.0, 1.0, 1.0))
        Y1 = net.infer(V).clone()
        net.set_output_scale((2.0, 0.5, 0.25))
        Y2 = net.infer(V)
        torch.cuda.synchronize()
        for c, s in enumerate((2.0, 0.5, 0.25)):
            assert torch.equal(Y2[c], Y1[c] * s), c
    finally:
        net.set_output_scale(old)
