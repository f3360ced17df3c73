"""Surrogate network kernels (BF16 MFMA convolutions, FP32 accumulation) against the FP64
oracle, and the exact normalisation / tile-merge entry points.

Three bars:
* FP32-operand mode (sal_net_set_precision(SAL_FP32): the same kernels, tiles, K order and
  epilogues with FP32 operands): forward outputs and every weight and bias gradient element by
  element within 1e-5 of the largest reference magnitude of the tensor.  FP32 accumulation of
  at most 648 products per output and five layers keep the error near 1e-6.
* BF16 forward against the oracle of the BF16 network (input, weights, pre-activations and
  activations rounded to BF16 where they are formed, everything else FP64), element by
  element.  Both sides round the same values; they differ by the FP32 accumulation order and
  the FP32 erf of the kernels (together about 1e-6 of a value), and where such a difference
  moves a value across a BF16 rounding boundary (a chance of about 1e-6 / 2^-9 = 5e-4 per
  rounded value) one value changes by one BF16 unit (2^-8 relative).  An output depends on
  about 3e4 rounded activations (11^3 voxels, 24 channels), so on about ten such changes, each
  moving it by up to |w| |a| 2^-8: the bound is 5e-3 of the largest output (measured: up to
  2.1e-3 on random weights).
* BF16 gradients against the FP64 gradient: relative L2 error at most 1e-2 per tensor (the
  roundings of activations, gradients and weights enter twice).  The FP64 forward bounds the
  BF16 forward at 2e-2 relative L2.
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


def relmax(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


BF16_ELEM = 5e-3


@pytest.mark.parametrize("S", [5, 10, 17])
def test_forward_vs_bf16_oracle_elementwise(net, S):
    rng = np.random.default_rng(10 + S)
    X = rng.standard_normal((2, S, S, S)).astype(np.float32)
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = O.net_forward_bf16(X[..., None], net.get_params().astype(np.float64))
    err = relmax(Y, ref)
    print("BF16 forward vs BF16 oracle S=%d: max rel %.3e" % (S, err))
    assert err <= BF16_ELEM


@pytest.fixture(scope="module")
def net32():
    n = sal.Net(seed=5)
    n.set_precision(sal.FP32)
    return n


@pytest.mark.parametrize("S", [5, 10, 17])
def test_f32_forward_vs_oracle(net32, S):
    """FP32-operand mode, element by element: cube sides below, at and above one output tile
    (4 x 8 x 16), two blocks."""
    rng = np.random.default_rng(20 + S)
    X = rng.standard_normal((2, S, S, S)).astype(np.float32)
    Y = net32.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = O.net_forward(X[..., None], net32.get_params().astype(np.float64))
    err = relmax(Y, ref)
    print("FP32 forward S=%d: max rel %.3e" % (S, err))
    assert err <= 1e-5


def _grad_case(S, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((2, S, S, S)).astype(np.float32)
    dY = np.zeros((2, S, S, S, 3), np.float32)
    dY[:, 5:S - 5, 5:S - 5, 5:S - 5, :] = rng.standard_normal((2, S - 10, S - 10, S - 10, 3))
    return X, dY


def _layers(g):
    off = 0
    for l in range(5):
        ci, co = O.SURROGATE_CHANNELS[l], O.SURROGATE_CHANNELS[l + 1]
        nw = co * 27 * ci
        yield l, slice(off, off + nw), slice(off + nw, off + nw + co)
        off += nw + co


@pytest.mark.parametrize("S", [13, 21])
def test_f32_gradient_vs_oracle(net32, S):
    """FP32-operand mode: the weight and bias gradients of every layer (which carry the input
    gradient of every later layer) element by element against the oracle's exact gradient;
    dY vanishes within 5 voxels of the faces, where the zero-padded input gradient is exact."""
    X, dY = _grad_case(S, 30 + S)
    Xg = torch.from_numpy(X).cuda()
    net32.grads(zero=True)
    net32.forward(Xg)
    net32.backward(Xg, torch.from_numpy(dY).cuda())
    g = net32.grads(zero=True).astype(np.float64)
    ref = O.net_backward(X[..., None], net32.get_params().astype(np.float64), dY)
    for l, sw, sb in _layers(g):
        ew, eb = relmax(g[sw], ref[sw]), relmax(g[sb], ref[sb])
        print("FP32 layer %d dW max rel %.3e db %.3e" % (l, ew, eb))
        assert ew <= 1e-5 and eb <= 1e-5, (l, ew, eb)


def _crop_checks(shape, c):
    """Crops of side c at three corners and inside, with the region of each whose outputs
    depend only on samples of the crop (5 voxels from a face inside the volume)."""
    n0, n1, n2 = shape
    out = []
    for lo in [(0, 0, 0), (n0 - c, n1 - c, n2 - c), (n0 // 2 - c // 2, n1 // 3, n2 // 2 - c // 2),
               (0, n1 - c, n2 // 2)]:
        valid = []
        for a, n in zip(lo, shape):
            v0 = 0 if a == 0 else 5
            v1 = c if a + c == n else c - 5
            valid.append(slice(v0, v1))
        out.append((lo, tuple(valid)))
    return out


@pytest.mark.parametrize("prec", [sal.FP32, sal.BF16])
def test_infer_full_size_vs_oracle_crops(prec):
    """sal_net_infer on a 128^3 volume with the trained weights, on the persistent grid of the
    benchmark (more tiles than workgroups, so every workgroup walks several tiles and both LDS
    buffers), against the oracle on 20^3 crops: corners (their volume faces reflect as the
    crop's do) and inside, element by element on the voxels 5 or more from every crop face
    inside the volume.  FP32-operand mode against the FP64 network at 1e-5, BF16 against the
    BF16 network."""
    from paper_1901_11095_amd import surrogate
    net = surrogate.load()
    if prec == sal.FP32:
        net.set_precision(sal.FP32)
    shape = (128, 128, 128)
    V = synth.make_volume(**surrogate.volume_kwargs(99, shape))
    Sr = net.infer(torch.from_numpy(V).cuda()).cpu().numpy()
    p = net.get_params().astype(np.float64)
    scale = np.asarray(net.out_scale, np.float64)
    c = 20
    for lo, valid in _crop_checks(shape, c):
        crop = V[lo[0]:lo[0] + c, lo[1]:lo[1] + c, lo[2]:lo[2] + c]
        if prec == sal.FP32:
            ref = O.net_forward(crop[None, ..., None], p)[0]
        else:
            ref = O.net_forward_bf16(crop[None, ..., None], p)[0]
        ref = ref * scale
        got = Sr[:, lo[0]:lo[0] + c, lo[1]:lo[1] + c, lo[2]:lo[2] + c].transpose(1, 2, 3, 0)
        err = relmax(got[valid], ref[valid])
        print("infer %s crop %s: max rel %.3e" % (sal.PRECISION_NAMES[prec], lo, err), flush=True)
        assert err <= (1e-5 if prec == sal.FP32 else BF16_ELEM), (lo, err)


def test_adam_steps_closed_form():
    """sal_net_adam on the gradient of sal_net_backward.  From zero moments the bias-corrected
    moments of the first step are g and g^2, so every parameter moves by -lr g / (|g| + eps);
    after a second gradient g2 they are (0.09 g + 0.1 g2) / 0.19 and
    (0.000999 g^2 + 0.001 g2^2) / (1 - 0.999^2).  Each step clears the gradient."""
    n = sal.Net(seed=7)
    X, dY = _grad_case(13, 40)
    Xg, dYg = torch.from_numpy(X).cuda(), torch.from_numpy(dY).cuda()
    lr = 1e-3
    ps, gs = [n.get_params().astype(np.float64)], []
    n.grads(zero=True)
    for step in range(2):
        n.forward(Xg)
        n.backward(Xg, dYg)
        gs.append(n.grads(zero=False).astype(np.float64))
        n.adam(lr)
        torch.cuda.synchronize()
        ps.append(n.get_params().astype(np.float64))
        assert not n.grads(zero=False).any()
    g1, g2 = gs
    assert np.abs(g1).max() > 0
    tol = 1e-7  # FP32 parameters below 0.5: half a unit in the last place is 1.5e-8
    want1 = ps[0] - lr * g1 / (np.abs(g1) + 1e-8)
    assert np.abs(ps[1] - want1).max() <= tol
    m = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.9 ** 2)
    v = (0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    want2 = ps[1] - lr * m / (np.sqrt(v) + 1e-8)
    assert np.abs(ps[2] - want2).max() <= tol


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
        assert ew <= 1e-2 and eb <= 1e-2
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
