"""Pins of the FP64 surrogate-network oracle (CPU only): GELU against the normal CDF of
scipy, convolution taps against numpy reflect padding, gradients against central finite
differences."""
import math

import numpy as np
import pytest
from scipy.stats import norm


def test_gelu_matches_normal_cdf(oracle_mod):
    for z in (-3.0, -1.0, -0.25, 0.0, 0.5, 1.0, 2.5):
        assert abs(oracle_mod.gelu(z) - z * norm.cdf(z)) <= 1e-15
        assert abs(oracle_mod.gelu(z) - oracle_mod.gelu(-z) - z) <= 1e-15


def test_gelu_grad_finite_difference(oracle_mod):
    h = 1e-6
    for z in (-2.0, -0.3, 0.0, 0.7, 1.9):
        fd = (oracle_mod.gelu(z + h) - oracle_mod.gelu(z - h)) / (2 * h)
        assert abs(oracle_mod.gelu_grad(z) - fd) <= 1e-9


@pytest.mark.parametrize("k", [0, 4, 13, 17, 26])
def test_conv_shift_kernel(oracle_mod, k):
    """A kernel that copies channel c from tap k shifts the crop by (dt-1, du-1, dw-1) with
    reflection at the crop faces."""
    rng = np.random.default_rng(k)
    S, C = 6, 2
    x = rng.standard_normal((2, S, S, S, C))
    W = np.zeros((C, 27, C))
    for c in range(C):
        W[c, k, c] = 1.0
    y = oracle_mod.conv3d(x, W, np.array([0.5, -1.0]))
    dt, du, dw = k // 9, (k // 3) % 3, k % 3
    P = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)), mode="reflect")
    ref = P[:, dt:dt + S, du:du + S, dw:dw + S, :] + np.array([0.5, -1.0])
    assert np.abs(y - ref).max() <= 1e-15


def test_conv_backward_finite_difference(oracle_mod):
    rng = np.random.default_rng(1)
    S, ci, co = 4, 3, 2
    x = rng.standard_normal((1, S, S, S, ci))
    W = rng.standard_normal((co, 27, ci))
    b = rng.standard_normal(co)
    dy = rng.standard_normal((1, S, S, S, co))
    dx, dW, db = oracle_mod.conv3d_backward(x, W, dy)
    f = lambda xx, WW, bb: float(np.sum(dy * oracle_mod.conv3d(xx, WW, bb)))
    h = 1e-4
    for _ in range(12):
        i = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        assert abs((f(xp, W, b) - f(xm, W, b)) / (2 * h) - dx[i]) <= 1e-8
        j = tuple(rng.integers(0, s) for s in W.shape)
        Wp, Wm = W.copy(), W.copy()
        Wp[j] += h
        Wm[j] -= h
        assert abs((f(x, Wp, b) - f(x, Wm, b)) / (2 * h) - dW[j]) <= 1e-8
    bp = b.copy()
    bp[1] += 1.0
    assert abs(f(x, W, bp) - f(x, W, b) - db[1]) <= 1e-9


def _small_net(rng, ch):
    n = sum(ch[l + 1] * 27 * ch[l] + ch[l + 1] for l in range(len(ch) - 1))
    return rng.standard_normal(n) * 0.3


def test_net_single_layer_is_conv(oracle_mod):
    rng = np.random.default_rng(2)
    ch = (2, 3)
    p = _small_net(rng, ch)
    x = rng.standard_normal((2, 5, 5, 5, 2))
    W = p[:3 * 27 * 2].reshape(3, 27, 2)
    b = p[3 * 27 * 2:]
    assert np.abs(oracle_mod.net_forward(x, p, ch) - oracle_mod.conv3d(x, W, b)).max() <= 1e-14


def test_net_gradient_finite_difference(oracle_mod):
    """Backpropagation through conv + GELU layers against central differences."""
    rng = np.random.default_rng(3)
    ch = (1, 3, 2, 3)
    p = _small_net(rng, ch)
    x = rng.standard_normal((2, 5, 5, 5, 1))
    dy = rng.standard_normal((2, 5, 5, 5, 3))
    g = oracle_mod.net_backward(x, p, dy, ch)
    f = lambda pp: float(np.sum(dy * oracle_mod.net_forward(x, pp, ch)))
    h = 1e-5
    for i in rng.choice(len(p), 25, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (f(pp) - f(pm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_round_bf16_matches_library(oracle_mod):
    """BF16 rounding of the oracle against torch's float32 -> bfloat16 conversion (round to
    nearest, ties to even) over magnitudes from 1e-9 to 1e9, plus exact ties."""
    import torch
    rng = np.random.default_rng(4)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    # exact ties: halfway between two BF16 neighbours with an even and an odd lower neighbour
    ties = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(2.0 + 2.0 ** -7), 3.0 + 2.0 ** -7],
                    np.float32)
    x = np.concatenate([x, ties, np.array([0.0, -0.0], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle_mod.round_bf16(float(v)) for v in x])
    assert np.array_equal(got, ref)
    assert oracle_mod.round_bf16(1.0 + 2.0 ** -8) == 1.0          # tie to the even neighbour
    assert oracle_mod.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_net_bf16_exact_on_representable_single_layer(oracle_mod):
    """One layer (no activation) whose input and weights are BF16 values: the BF16 network
    rounds nothing, so it equals the FP64 network exactly."""
    rng = np.random.default_rng(5)
    ch = (2, 3)
    r = np.vectorize(oracle_mod.round_bf16)
    p = _small_net(rng, ch)
    p[:3 * 27 * 2] = r(p[:3 * 27 * 2])
    x = r(rng.standard_normal((1, 5, 5, 5, 2)))
    assert np.array_equal(oracle_mod.net_forward_bf16(x, p, ch), oracle_mod.net_forward(x, p, ch))


def test_net_bf16_within_rounding_bound(oracle_mod):
    """The BF16 network differs from the FP64 one by the BF16 roundings only: relative to the
    output scale, a few units of 2^-9 per layer (here at most 4 layers of rounded values), and
    it is not the FP64 network (the roundings are really applied)."""
    rng = np.random.default_rng(6)
    ch = (1, 4, 4, 3)
    p = _small_net(rng, ch)
    x = rng.standard_normal((2, 6, 6, 6, 1))
    y = oracle_mod.net_forward(x, p, ch)
    yb = oracle_mod.net_forward_bf16(x, p, ch)
    rel = np.abs(yb - y).max() / np.abs(y).max()
    assert 0 < rel <= 4 * 3 * 2.0 ** -9, rel
