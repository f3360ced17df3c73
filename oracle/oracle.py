"""ctypes front end of the FP64 C oracle (``sal_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU path.

Every function takes and returns NumPy arrays; volumes are float32 ``[n0][n1][n2]`` (axis 0
is t), results are float64.  Each wrapper names the passage of the paper its C function
follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "sal_oracle.c"), os.path.join(_HERE, "net_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_lp = ctypes.POINTER(ctypes.c_long)
_up = ctypes.POINTER(ctypes.c_uint32)
_L = ctypes.c_long

# rays: bit 2a enables the ray along +axis a, bit 2a+1 the ray along -axis a
RAY_PT, RAY_MT, RAY_PX, RAY_MX, RAY_PY, RAY_MY = 1, 2, 4, 8, 16, 32
RAYS_AXIS = (RAY_PT | RAY_MT, RAY_PX | RAY_MX, RAY_PY | RAY_MY)  # S_t: +-t, S_x: +-x, S_y: +-y
RAYS_ALL = (63, 63, 63)
# oriented rays (Fig. 3): bits 6-9 the t-x diagonals (+t+x, -t-x, +t-x, -t+x), 10-13 the
# t-y diagonals, 14-17 the x-y diagonals, 18-25 the body diagonals
RAY_DIAG_TX, RAY_DIAG_TY, RAY_DIAG_XY, RAY_BODY = 0xF << 6, 0xF << 10, 0xF << 14, 0xFF << 18
RAYS_26 = ((1 << 26) - 1,) * 3


def build(force: bool = False) -> str:
    """Compile the C oracle (FP64, OpenMP) with gcc into ``liboracle.so``."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s)
                                            for s in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build()
        l = ctypes.CDLL(_LIB)
        l.oracle_window_spectrum.argtypes = [_fp, _L, _L, _L, _L, _L, _L, _L, _dp]
        l.oracle_project.argtypes = [_dp, _L, _dp]
        l.oracle_local_spectra.argtypes = [_fp, _L, _L, _L, _L, _lp, _lp, _dp]
        l.oracle_energy_box.argtypes = [_fp, _L, _L, _L, _L, _lp, _lp, _dp]
        l.oracle_energy.argtypes = [_fp, _L, _L, _L, _L, _dp]
        l.oracle_dcs.argtypes = [_dp, _L, _L, _L, _L, ctypes.c_double, _up, _dp]
        l.oracle_dcs.restype = ctypes.c_int
        l.oracle_combine.argtypes = [_dp, _L, _dp, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, _dp, _dp]
        l.oracle_combine_with_stats.argtypes = [_dp, _L, _dp, ctypes.c_int, ctypes.c_double,
                                                ctypes.c_double, _dp, _dp]
        l.oracle_absmax.argtypes = [_fp, _L]
        l.oracle_absmax.restype = ctypes.c_double
        l.oracle_saliency.argtypes = [_fp, _L, _L, _L, _L, _L, ctypes.c_double, _up, _dp,
                                      ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
        l.oracle_raw_box.argtypes = [_fp, _L, _L, _L, _L, _L, ctypes.c_double, _up, _lp, _lp,
                                     _dp, _dp]
        l.oracle_raw_box.restype = ctypes.c_int
        l.oracle_energy_lattice.argtypes = [_fp, _L, _L, _L, _L, _L, _dp]
        l.oracle_upsample.argtypes = [_dp, _L, _L, _L, _L, _dp]
        l.oracle_saliency_strided.argtypes = [_fp, _L, _L, _L, _L, _L, _L, ctypes.c_double, _up, _dp,
                                              ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
        l.oracle_gelu.argtypes = [ctypes.c_double]
        l.oracle_gelu.restype = ctypes.c_double
        l.oracle_gelu_grad.argtypes = [ctypes.c_double]
        l.oracle_gelu_grad.restype = ctypes.c_double
        l.oracle_conv3d.argtypes = [_dp, _L, _L, _L, _dp, _dp, _L, _dp]
        l.oracle_conv3d_backward.argtypes = [_dp, _L, _L, _L, _dp, _L, _dp, _dp, _dp, _dp]
        l.oracle_net_forward.argtypes = [_dp, _L, _L, _L, _lp, _dp, _dp, _dp]
        l.oracle_net_backward.argtypes = [_dp, _L, _L, _L, _lp, _dp, _dp, _dp]
        l.oracle_net_forward_bf16.argtypes = [_dp, _L, _L, _L, _lp, _dp, _dp]
        l.oracle_round_bf16.argtypes = [ctypes.c_double]
        l.oracle_round_bf16.restype = ctypes.c_double
        _lib = l
    return _lib


@dataclass
class Params:
    """Method parameters (Sec. 2 and Eq. (5)-(6)); defaults are the declared readings."""
    L: int = 8                      # cube side (first step of Sec. 2; the paper uses 5)
    d: int | None = None            # DCS line length, defaults to L (after Fig. 3)
    sigma: float | None = None      # Gaussian width of the DCS weights, defaults to d/4
    rays: tuple = RAYS_AXIS         # rays used by S_t, S_x, S_y
    abc: tuple = (1.0 / 3, 1.0 / 3, 1.0 / 3)  # Eq. (6) weights, equal (Sec. 2, last para.)
    normalize: int = 1
    zero_range: float = 1e-6
    stride: int = 1                 # window lattice stride (Sec. 2 first step: overlap > 50%)

    @property
    def r(self) -> int:
        return (self.d if self.d is not None else self.L) // 2

    @property
    def sig(self) -> float:
        return self.sigma if self.sigma is not None else (self.d if self.d is not None else self.L) / 4.0


def _f32(V):
    V = np.ascontiguousarray(V, dtype=np.float32)
    return V, V.ctypes.data_as(_fp)


def _d(a):
    return a.ctypes.data_as(_dp)


def _longs(x):
    return (ctypes.c_long * 3)(*[int(v) for v in x])


def _rays(r):
    return (ctypes.c_uint32 * 3)(*[int(v) for v in r])


def window_spectrum(V, t, x, y, L) -> np.ndarray:
    """Local spectrum F[mu,nu,om] (complex128) of voxel (t,x,y): DFT definition after Eq. (2)."""
    V, pV = _f32(V)
    F = np.zeros((L, L, L, 2), np.float64)
    lib().oracle_window_spectrum(pV, *V.shape, t, x, y, L, _d(F))
    return F[..., 0] + 1j * F[..., 1]


def project(F) -> np.ndarray:
    """(E_t, E_x, E_y) of one spectrum: Eqs. (1)-(4), DC excluded, absolute mean (Sec. 2)."""
    F = np.asarray(F, np.complex128)
    L = F.shape[0]
    buf = np.ascontiguousarray(np.stack([F.real, F.imag], -1))
    E = np.zeros(3, np.float64)
    lib().oracle_project(_d(buf), L, _d(E))
    return E


def local_spectra(V, L, lo, bn) -> np.ndarray:
    """Spectra of every voxel of box [lo, lo+bn): complex128 [bn0][bn1][bn2][L][L][L]."""
    V, pV = _f32(V)
    out = np.zeros(tuple(bn) + (L, L, L, 2), np.float64)
    lib().oracle_local_spectra(pV, *V.shape, L, _longs(lo), _longs(bn), _d(out))
    return out[..., 0] + 1j * out[..., 1]


def energy(V, L) -> np.ndarray:
    """E[3][n0][n1][n2]: Sec. 2 steps one to three over the whole volume."""
    V, pV = _f32(V)
    E = np.zeros((3,) + V.shape, np.float64)
    lib().oracle_energy(pV, *V.shape, L, _d(E))
    return E


def energy_box(V, L, lo, bn) -> np.ndarray:
    V, pV = _f32(V)
    E = np.zeros((3,) + tuple(bn), np.float64)
    lib().oracle_energy_box(pV, *V.shape, L, _longs(lo), _longs(bn), _d(E))
    return E


def dcs(E, r, sigma, rays=RAYS_AXIS) -> np.ndarray:
    """Raw S_m[3][...] from E[3][...]: Eq. (5), reflect at the volume edges."""
    E = np.ascontiguousarray(E, np.float64)
    S = np.zeros_like(E)
    bad = lib().oracle_dcs(_d(E), *E.shape[1:], r, float(sigma), _rays(rays), _d(S))
    assert bad == 0
    return S


def combine(S_raw, abc=(1 / 3, 1 / 3, 1 / 3), normalize=1, zero_range=1e-6, vmax=1.0):
    """Eq. (6) after per-component volume-wide min-max normalisation.  Returns (S, stats)."""
    S_raw = np.ascontiguousarray(S_raw, np.float64)
    n = S_raw[0].size
    S = np.zeros(S_raw.shape[1:], np.float64)
    stats = np.zeros(6, np.float64)
    w = np.asarray(abc, np.float64)
    lib().oracle_combine(_d(S_raw), n, _d(w), int(normalize), float(zero_range), float(vmax),
                         _d(S), _d(stats))
    return S, stats


def combine_with_stats(S_raw, stats, abc=(1 / 3, 1 / 3, 1 / 3), normalize=1, zero_range=1e-6,
                       vmax=1.0):
    S_raw = np.ascontiguousarray(S_raw, np.float64)
    stats = np.ascontiguousarray(stats, np.float64)
    S = np.zeros(S_raw.shape[1:], np.float64)
    w = np.asarray(abc, np.float64)
    lib().oracle_combine_with_stats(_d(S_raw), S_raw[0].size, _d(w), int(normalize),
                                    float(zero_range), float(vmax), _d(stats), _d(S))
    return S


def absmax(V) -> float:
    V, pV = _f32(V)
    return lib().oracle_absmax(pV, V.size)


def saliency(V, p: Params = Params()):
    """Whole method (Sec. 2 steps one to five).  Returns dict with S, E, S_raw, stats."""
    V, pV = _f32(V)
    S = np.zeros(V.shape, np.float64)
    E = np.zeros((3,) + V.shape, np.float64)
    Sr = np.zeros((3,) + V.shape, np.float64)
    stats = np.zeros(6, np.float64)
    w = np.asarray(p.abc, np.float64)
    if p.stride == 1:
        lib().oracle_saliency(pV, *V.shape, p.L, p.r, float(p.sig), _rays(p.rays), _d(w),
                              int(p.normalize), float(p.zero_range), _d(S), _d(E), _d(Sr), _d(stats))
    else:
        lib().oracle_saliency_strided(pV, *V.shape, p.L, p.stride, p.r, float(p.sig), _rays(p.rays),
                                      _d(w), int(p.normalize), float(p.zero_range), _d(S), _d(E),
                                      _d(Sr), _d(stats))
    return {"S": S, "E": E, "S_raw": Sr, "stats": stats}


def lattice_shape(shape, s: int):
    return tuple((n + s - 1) // s for n in shape)


def energy_lattice(V, L: int, s: int) -> np.ndarray:
    """Energies E_t, E_x, E_y of the windows at the lattice positions k s (Sec. 2, first and
    third steps, strided windows): double [3][K0][K1][K2]."""
    V, pV = _f32(V)
    E = np.zeros((3,) + lattice_shape(V.shape, s), np.float64)
    lib().oracle_energy_lattice(pV, *V.shape, L, s, _d(E))
    return E


def upsample(E_lat, s: int, shape) -> np.ndarray:
    """Trilinear interpolation of lattice values [3][K...] onto the full grid [3][shape]."""
    E_lat = np.ascontiguousarray(E_lat, np.float64)
    assert E_lat.shape[1:] == lattice_shape(shape, s)
    E = np.zeros((3,) + tuple(shape), np.float64)
    lib().oracle_upsample(_d(E_lat), s, *shape, _d(E))
    return E


def raw_box(V, p: Params, lo, bn):
    """E and raw S_m on the box [lo, lo+bn) of a large volume (energies on box + r halo)."""
    V, pV = _f32(V)
    E = np.zeros((3,) + tuple(bn), np.float64)
    S = np.zeros((3,) + tuple(bn), np.float64)
    bad = lib().oracle_raw_box(pV, *V.shape, p.L, p.r, float(p.sig), _rays(p.rays),
                               _longs(lo), _longs(bn), _d(E), _d(S))
    assert bad == 0
    return E, S


# ------------------------------------------------------------------ learned surrogate ----
# Channel-last activations x[b][t][u][w][c] over crops of S^3; weights W[co][27][ci] with tap
# k = (dt*3 + du)*3 + dw reading (t+dt-1, u+du-1, w+dw-1), reflected inside the crop.

SURROGATE_CHANNELS = (1, 24, 24, 24, 24, 3)


def gelu(z: float) -> float:
    return lib().oracle_gelu(float(z))


def gelu_grad(z: float) -> float:
    return lib().oracle_gelu_grad(float(z))


def conv3d(x, W, b=None):
    """y = conv3d(x) + b with reflect padding inside each crop (FP64)."""
    x = np.ascontiguousarray(x, np.float64)
    W = np.ascontiguousarray(W, np.float64)
    nb, S = x.shape[0], x.shape[1]
    ci, co = x.shape[-1], W.shape[0]
    y = np.zeros((nb, S, S, S, co), np.float64)
    bb = None if b is None else np.ascontiguousarray(b, np.float64)
    lib().oracle_conv3d(_d(x), nb, S, ci, _d(W), None if bb is None else _d(bb), co, _d(y))
    return y


def conv3d_backward(x, W, dy):
    """(dx, dW, db) of sum(dy * conv3d(x)) -- the exact adjoint, reflect taps included."""
    x = np.ascontiguousarray(x, np.float64)
    W = np.ascontiguousarray(W, np.float64)
    dy = np.ascontiguousarray(dy, np.float64)
    nb, S, ci, co = x.shape[0], x.shape[1], x.shape[-1], W.shape[0]
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    db = np.zeros(co, np.float64)
    lib().oracle_conv3d_backward(_d(x), nb, S, ci, _d(W), co, _d(dy), _d(dx), _d(dW), _d(db))
    return dx, dW, db


def net_num_params(ch=SURROGATE_CHANNELS) -> int:
    return sum(ch[l + 1] * 27 * ch[l] + ch[l + 1] for l in range(len(ch) - 1))


def net_forward(x, params, ch=SURROGATE_CHANNELS):
    """Output of the conv/GELU stack for x[b][S][S][S][ch0]; params flat FP64 (per layer W
    then bias)."""
    x = np.ascontiguousarray(x, np.float64)
    p = np.ascontiguousarray(params, np.float64)
    nb, S = x.shape[0], x.shape[1]
    y = np.zeros((nb, S, S, S, ch[-1]), np.float64)
    cha = (ctypes.c_long * len(ch))(*ch)
    lib().oracle_net_forward(_d(x), nb, S, len(ch) - 1, cha, _d(p), _d(y), None)
    return y


def round_bf16(v: float) -> float:
    """v rounded to 8 significant bits, to nearest, ties to even (the BF16 values)."""
    return lib().oracle_round_bf16(float(v))


def net_forward_bf16(x, params, ch=SURROGATE_CHANNELS):
    """net_forward in the network's specified arithmetic: input, weights, pre-activations and
    activations rounded to BF16 where they are formed, sums and biases in FP64."""
    x = np.ascontiguousarray(x, np.float64)
    p = np.ascontiguousarray(params, np.float64)
    nb, S = x.shape[0], x.shape[1]
    y = np.zeros((nb, S, S, S, ch[-1]), np.float64)
    cha = (ctypes.c_long * len(ch))(*ch)
    lib().oracle_net_forward_bf16(_d(x), nb, S, len(ch) - 1, cha, _d(p), _d(y))
    return y


def net_backward(x, params, dy, ch=SURROGATE_CHANNELS):
    """Gradient of sum(dy * net(x)) with respect to the flat parameter vector."""
    x = np.ascontiguousarray(x, np.float64)
    p = np.ascontiguousarray(params, np.float64)
    dy = np.ascontiguousarray(dy, np.float64)
    nb, S = x.shape[0], x.shape[1]
    g = np.zeros_like(p)
    cha = (ctypes.c_long * len(ch))(*ch)
    lib().oracle_net_backward(_d(x), nb, S, len(ch) - 1, cha, _d(p), _d(dy), _d(g))
    return g
