"""Python binding of libsal (ctypes): argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch supplies device memory
and the current HIP stream.  If ``libsal.so`` has not been built this module raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

from .build import LIB as _LIB_PATH

SAL_OK, SAL_E_INVAL, SAL_E_UNSUPPORTED, SAL_E_DEVICE, SAL_E_WORKSPACE = range(5)
FP32, BF16, BF16_SPLIT, FP16, FP16_SPLIT, BF16_SPLITW, FP16_SPLITW = range(7)
PRECISION_NAMES = {FP32: "fp32", BF16: "bf16", BF16_SPLIT: "bf16_split", FP16: "fp16",
                   FP16_SPLIT: "fp16_split", BF16_SPLITW: "bf16_splitw",
                   FP16_SPLITW: "fp16_splitw"}
RAY_PT, RAY_MT, RAY_PX, RAY_MX, RAY_PY, RAY_MY = 1, 2, 4, 8, 16, 32
# oriented rays (bit layout of SAL_RAY_* in sal.h): t-x, t-y, x-y diagonals, body diagonals
RAY_DIAG_TX, RAY_DIAG_TY, RAY_DIAG_XY, RAY_BODY = 0xF << 6, 0xF << 10, 0xF << 14, 0xFF << 18
RAY_ALL = (1 << 26) - 1
RAYS_AXIS = (RAY_PT | RAY_MT, RAY_PX | RAY_MX, RAY_PY | RAY_MY)
RAYS_ALL = (63, 63, 63)
STATS_LEN = 7

EXPORTS = ("sal_default_params", "sal_create", "sal_destroy", "sal_last_error",
           "sal_workspace_size", "sal_local_spectra", "sal_project", "sal_directional_compare",
           "sal_saliency", "sal_profile_enable", "sal_profile_read", "sal_normalize_combine",
           "sal_tile_merge", "sal_tile_minmax", "sal_raw_box_workspace_size", "sal_raw_box",
           "sal_check_tiles_workspace_size", "sal_check_tiles", "sal_absmax", "sal_saliency_noalloc",
           "sal_net_num_params", "sal_net_last_error", "sal_net_create",
           "sal_net_destroy", "sal_net_params", "sal_net_grads", "sal_net_set_output_scale",
           "sal_net_workspace_size", "sal_net_forward", "sal_net_backward", "sal_net_train_step",
           "sal_net_infer", "sal_net_set_precision", "sal_net_adam")
KERNELS = ("energy", "dcs", "stats", "combine")


class SalError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("sal status %d: %s" % (status, msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("d", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("rays", ctypes.c_uint32 * 3), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("c", ctypes.c_double), ("normalize", ctypes.c_int32),
                ("zero_range", ctypes.c_double), ("precision", ctypes.c_int32),
                ("stride", ctypes.c_int32), ("t_direct", ctypes.c_int32)]


_i64p = ctypes.POINTER(ctypes.c_int64)
_lib = None


def load(path: str = _LIB_PATH) -> ctypes.CDLL:
    """Load libsal.so; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsal.so is not built (%s); run python -m paper_1901_11095_amd.build"
                           % path)
    l = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    l.sal_default_params.argtypes = [ctypes.POINTER(Params), ctypes.c_int32]
    l.sal_default_params.restype = None
    l.sal_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(vp)]
    l.sal_destroy.argtypes = [vp]
    l.sal_destroy.restype = None
    l.sal_last_error.argtypes = [vp]
    l.sal_last_error.restype = ctypes.c_char_p
    l.sal_workspace_size.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_size_t)]
    l.sal_local_spectra.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                    _i64p, _i64p, vp, vp]
    l.sal_project.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    l.sal_directional_compare.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, vp, vp]
    l.sal_saliency.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, vp, vp,
                               vp, vp, vp, ctypes.c_size_t, vp]
    l.sal_profile_enable.argtypes = [vp, ctypes.c_int]
    l.sal_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    i64, sz, fp = ctypes.c_int64, ctypes.c_size_t, ctypes.POINTER(ctypes.c_float)
    l.sal_normalize_combine.argtypes = [vp, vp, ctypes.c_double, vp, i64, i64, i64, vp, vp, vp, sz,
                                        vp]
    l.sal_tile_merge.argtypes = [vp, vp, i64, i64, i64, vp, _i64p, _i64p, _i64p, _i64p, vp,
                                 ctypes.c_double, vp, vp]
    l.sal_tile_minmax.argtypes = [vp, vp, i64, i64, i64, ctypes.c_int32, vp, vp]
    l.sal_raw_box_workspace_size.argtypes = [vp, _i64p, ctypes.POINTER(sz)]
    l.sal_raw_box.argtypes = [vp, vp, i64, i64, i64, _i64p, _i64p, vp, vp, sz, vp]
    l.sal_check_tiles_workspace_size.argtypes = [vp, i64, i64, i64, i64, _i64p, ctypes.POINTER(sz)]
    l.sal_check_tiles.argtypes = [vp, vp, i64, i64, i64, i64, _i64p, vp, i64, i64, i64, _i64p, i64,
                                  _i64p, vp, ctypes.c_double, vp, vp, vp, sz, vp]
    l.sal_absmax.argtypes = [vp, vp, i64, vp, ctypes.c_int, vp]
    l.sal_saliency_noalloc.argtypes = [vp, vp, i64, i64, i64, vp, vp, vp, vp, vp]
    l.sal_net_set_precision.argtypes = [vp, ctypes.c_int32]
    l.sal_net_adam.argtypes = [vp, ctypes.c_float, vp]
    l.sal_net_num_params.argtypes = []
    l.sal_net_num_params.restype = i64
    l.sal_net_last_error.argtypes = [vp]
    l.sal_net_last_error.restype = ctypes.c_char_p
    l.sal_net_create.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(vp)]
    l.sal_net_destroy.argtypes = [vp]
    l.sal_net_destroy.restype = None
    l.sal_net_params.argtypes = [vp, fp, i64, ctypes.c_int]
    l.sal_net_grads.argtypes = [vp, fp, i64, ctypes.c_int]
    l.sal_net_set_output_scale.argtypes = [vp, fp]
    l.sal_net_workspace_size.argtypes = [vp, i64, i64, i64, i64, ctypes.c_int,
                                         ctypes.POINTER(sz)]
    l.sal_net_forward.argtypes = [vp, vp, i64, i64, i64, i64, vp, vp, sz, vp]
    l.sal_net_backward.argtypes = [vp, vp, vp, i64, i64, i64, i64, vp, sz, vp]
    l.sal_net_train_step.argtypes = [vp, vp, vp, i64, i64, ctypes.c_int32, ctypes.c_float, vp,
                                     vp, sz, vp]
    l.sal_net_infer.argtypes = [vp, vp, i64, i64, i64, vp, vp, sz, vp]
    for f in ("sal_create", "sal_workspace_size", "sal_local_spectra", "sal_project",
              "sal_directional_compare", "sal_saliency", "sal_profile_enable",
              "sal_profile_read", "sal_normalize_combine", "sal_tile_merge", "sal_tile_minmax",
              "sal_raw_box_workspace_size", "sal_raw_box", "sal_check_tiles_workspace_size",
              "sal_check_tiles", "sal_absmax", "sal_saliency_noalloc", "sal_net_create", "sal_net_set_precision", "sal_net_adam",
              "sal_net_params", "sal_net_grads", "sal_net_set_output_scale",
              "sal_net_workspace_size", "sal_net_forward", "sal_net_backward",
              "sal_net_train_step", "sal_net_infer"):
        getattr(l, f).restype = ctypes.c_int
    _lib = l
    return l


def default_params(L: int = 8) -> Params:
    p = Params()
    load().sal_default_params(ctypes.byref(p), L)
    return p


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_vol(V: torch.Tensor, name: str = "V"):
    if not (V.is_cuda and V.dtype == torch.float32 and V.is_contiguous()):
        raise ValueError("%s must be a contiguous float32 CUDA tensor" % name)


class Saliency:
    """A library context: method parameters plus the device tables built from them."""

    def __init__(self, L: int = 8, d: Optional[int] = None, sigma: Optional[float] = None,
                 rays: Sequence[int] = RAYS_AXIS, abc=(1 / 3, 1 / 3, 1 / 3),
                 normalize: bool = True, zero_range: float = 1e-6, precision: int = FP32,
                 stride: int = 1, device: int = 0, t_direct: bool = False):
        self._lib = load()
        p = default_params(L)
        if d is not None:
            p.d = d
            p.sigma = d / 4.0
        if sigma is not None:
            p.sigma = sigma
        for m in range(3):
            p.rays[m] = int(rays[m])
        p.a, p.b, p.c = (float(x) for x in abc)
        p.normalize = int(bool(normalize))
        p.zero_range = float(zero_range)
        p.precision = int(precision)
        p.stride = int(stride)
        p.t_direct = int(bool(t_direct))
        self.params = p
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        st = self._lib.sal_create(ctypes.byref(p), device, ctypes.byref(h))
        if st != SAL_OK:
            raise SalError(st, self._lib.sal_last_error(None).decode())
        self._h = h
        self._ws = None

    @property
    def L(self) -> int:
        return self.params.L

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st: int):
        if st != SAL_OK:
            raise SalError(st, self._lib.sal_last_error(self._h).decode())

    def workspace_size(self, shape) -> int:
        n = ctypes.c_size_t()
        self._raise(self._lib.sal_workspace_size(self._h, *[int(s) for s in shape],
                                                 ctypes.byref(n)))
        return n.value

    def workspace(self, shape) -> torch.Tensor:
        need = self.workspace_size(shape)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def local_spectra(self, V: torch.Tensor, lo, bn) -> torch.Tensor:
        """complex64 [bn0, bn1, bn2, L, L, L] spectra of the voxels of box [lo, lo+bn)."""
        _check_vol(V)
        L = self.L
        out = torch.empty(tuple(int(b) for b in bn) + (L, L, L, 2), dtype=torch.float32,
                          device=V.device)
        lo_a = (ctypes.c_int64 * 3)(*[int(x) for x in lo])
        bn_a = (ctypes.c_int64 * 3)(*[int(x) for x in bn])
        self._raise(self._lib.sal_local_spectra(self._h, _ptr(V), *V.shape, lo_a, bn_a,
                                                _ptr(out), _stream(V.device)))
        return torch.view_as_complex(out)

    def project(self, spectra: torch.Tensor) -> torch.Tensor:
        """E [3, nvox] from complex64 spectra [..., L, L, L]."""
        if spectra.dtype == torch.complex64:
            spectra = torch.view_as_real(spectra)
        spectra = spectra.contiguous()
        L = self.L
        nvox = spectra.numel() // (2 * L ** 3)
        E = torch.empty((3, nvox), dtype=torch.float32, device=spectra.device)
        self._raise(self._lib.sal_project(self._h, _ptr(spectra), nvox, _ptr(E),
                                          _stream(spectra.device)))
        return E

    def directional_compare(self, E: torch.Tensor) -> torch.Tensor:
        """raw S [3, n0, n1, n2] from E [3, n0, n1, n2] (Eq. (5))."""
        _check_vol(E, "E")
        S = torch.empty_like(E)
        self._raise(self._lib.sal_directional_compare(self._h, _ptr(E), *E.shape[1:], _ptr(S),
                                                      _stream(E.device)))
        return S

    def saliency(self, V: torch.Tensor, S: Optional[torch.Tensor] = None, E_out=None,
                 S_raw_out=None, stats_out=None, workspace: Optional[torch.Tensor] = None):
        """Saliency map of V (float32 [n0, n1, n2], CUDA).  Optional outputs are written
        when given (E_out/S_raw_out float32 [3, n0, n1, n2], stats_out float64 [7])."""
        _check_vol(V)
        if S is None:
            S = torch.empty_like(V)
        ws = workspace if workspace is not None else self.workspace(V.shape)
        self._raise(self._lib.sal_saliency(self._h, _ptr(V), *V.shape, _ptr(S), _ptr(E_out),
                                           _ptr(S_raw_out), _ptr(stats_out), _ptr(ws),
                                           ws.numel() * ws.element_size(), _stream(V.device)))
        return S

    def saliency_noalloc(self, V: torch.Tensor, S: torch.Tensor, E_out: torch.Tensor,
                         S_raw_out: torch.Tensor, stats_out: Optional[torch.Tensor] = None):
        """sal_saliency_noalloc: the library allocates nothing; S [n0, n1, n2] and E_out,
        S_raw_out [3, n0, n1, n2] are caller buffers, the partials use the library's scratch."""
        _check_vol(V)
        for t, shp in ((S, V.shape), (E_out, (3,) + tuple(V.shape)), (S_raw_out, (3,) + tuple(V.shape))):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == tuple(shp)):
                raise ValueError("output buffers must be contiguous float32 CUDA tensors of the volume's shape")
        self._raise(self._lib.sal_saliency_noalloc(self._h, _ptr(V), *V.shape, _ptr(S), _ptr(E_out),
                                                   _ptr(S_raw_out), _ptr(stats_out), _stream(V.device)))
        return S

    def raw_box_workspace_size(self, box_dims) -> int:
        """Bytes of device workspace raw_box needs for a box of box_dims."""
        n = ctypes.c_size_t()
        self._raise(self._lib.sal_raw_box_workspace_size(self._h, _i64x3(tuple(int(d) for d in box_dims)),
                                                         ctypes.byref(n)))
        return n.value

    def raw_box(self, V: torch.Tensor, box_lo, box_dims, out: Optional[torch.Tensor] = None,
                workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Raw maps [3, *box_dims] of the positions box_lo + [0, box_dims) of V."""
        _check_vol(V)
        dims = tuple(int(d) for d in box_dims)
        if out is None:
            out = torch.empty((3,) + dims, dtype=torch.float32, device=V.device)
        if workspace is None:
            n = self.raw_box_workspace_size(dims)
            wsb = getattr(self, "_wsb", None)
            if wsb is None or wsb.numel() < n:
                wsb = self._wsb = torch.empty(max(1, n), dtype=torch.uint8, device=V.device)
            workspace = wsb
        self._raise(self._lib.sal_raw_box(self._h, _ptr(V), *V.shape, _i64x3(box_lo), _i64x3(dims),
                                          _ptr(out), _ptr(workspace), workspace.numel(),
                                          _stream(V.device)))
        return out

    def profile(self, on: bool = True):
        """Enable/disable per-kernel HIP-event timing of saliency()."""
        self._raise(self._lib.sal_profile_enable(self._h, int(bool(on))))

    def profile_read(self, reset: bool = True):
        """(dict kernel -> summed ms, number of timed calls)."""
        ms = (ctypes.c_double * 4)()
        n = ctypes.c_int64()
        self._raise(self._lib.sal_profile_read(self._h, ms, ctypes.byref(n), int(bool(reset))))
        return dict(zip(KERNELS, list(ms))), n.value

    def saliency_maps(self, V: torch.Tensor):
        """(S, E, S_raw, stats) with every intermediate map returned."""
        shp = (3,) + tuple(V.shape)
        E = torch.empty(shp, dtype=torch.float32, device=V.device)
        Sr = torch.empty(shp, dtype=torch.float32, device=V.device)
        st = torch.empty(STATS_LEN + 1, dtype=torch.float64, device=V.device)
        S = self.saliency(V, E_out=E, S_raw_out=Sr, stats_out=st)
        return S, E, Sr, st[:STATS_LEN]


def _i64x3(v):
    return (ctypes.c_int64 * 3)(*[int(x) for x in v])


def normalize_combine(ctx: "Saliency", S_raw: torch.Tensor, V: Optional[torch.Tensor] = None,
                      S: Optional[torch.Tensor] = None, stats_out: Optional[torch.Tensor] = None,
                      vmax: float = 1.0):
    """Exact FP64 statistics and Eq. (6) on given raw maps [3, n0, n1, n2] (CUDA float32);
    max|V| from V when given, else `vmax`."""
    if not (S_raw.is_cuda and S_raw.dtype == torch.float32 and S_raw.is_contiguous()):
        raise ValueError("S_raw must be a contiguous float32 CUDA tensor")
    shape = tuple(S_raw.shape[1:])
    if S is None:
        S = torch.empty(shape, dtype=torch.float32, device=S_raw.device)
    ws = ctx.workspace(shape)
    ctx._raise(ctx._lib.sal_normalize_combine(ctx._h, _ptr(V), float(vmax), _ptr(S_raw), *shape, _ptr(S),
                                              _ptr(stats_out), _ptr(ws), ws.numel(),
                                              _stream(S_raw.device)))
    return S


def tile_merge(ctx: "Saliency", S_raw: torch.Tensor, exact: torch.Tensor, crop_lo, tile_lo,
               tile_dims, stats: torch.Tensor, bound: float, err_out: torch.Tensor):
    """Check the tile of S_raw against `exact` (raw maps of the crop at crop_lo) and replace
    it when max |pred - exact| / range > bound.  err_out: CUDA float32 [>=1]."""
    shape = tuple(S_raw.shape[1:])
    ctx._raise(ctx._lib.sal_tile_merge(ctx._h, _ptr(S_raw), *shape, _ptr(exact), _i64x3(crop_lo),
                                       _i64x3(exact.shape[1:]), _i64x3(tile_lo), _i64x3(tile_dims),
                                       _ptr(stats), float(bound), _ptr(err_out),
                                       _stream(S_raw.device)))


def check_tiles_workspace_size(ctx: "Saliency", vshape, nbox: int, tile_dims) -> int:
    """Workspace bytes of check_tiles for volumes of shape vshape and nbox tiles."""
    n = ctypes.c_size_t()
    ctx._raise(ctx._lib.sal_check_tiles_workspace_size(ctx._h, *[int(v) for v in vshape], int(nbox),
                                                       _i64x3(tile_dims), ctypes.byref(n)))
    return n.value


def check_tiles(ctx: "Saliency", V: torch.Tensor, box_lo, S_raw: torch.Tensor, tile_lo, tile_dims,
                stats: torch.Tensor, bound: float, err_out: torch.Tensor,
                exact_out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None):
    """Batched tile check: V is one volume [n0, n1, n2] holding every tile, or a stack
    [nbox, n0, n1, n2] with tile b in volume b; box_lo / tile_lo: nbox origins (in V, in
    S_raw); tiles over `bound` are replaced in S_raw.  err_out: CUDA float32 [nbox]."""
    if not (V.is_cuda and V.dtype == torch.float32 and V.is_contiguous() and V.dim() in (3, 4)):
        raise ValueError("V must be a contiguous float32 CUDA tensor [n0, n1, n2] or [nbox, n0, n1, n2]")
    box = np.ascontiguousarray(np.asarray(box_lo, dtype=np.int64).reshape(-1, 3))
    til = np.ascontiguousarray(np.asarray(tile_lo, dtype=np.int64).reshape(-1, 3))
    nbox = len(box)
    if len(til) != nbox:
        raise ValueError("box_lo and tile_lo must hold the same number of origins")
    vshape = tuple(V.shape[-3:])
    vstride = 0
    if V.dim() == 4:
        if V.shape[0] != nbox:
            raise ValueError("a stacked V must hold one volume per tile")
        vstride = vshape[0] * vshape[1] * vshape[2]
    dims = _i64x3(tile_dims)
    if workspace is None:
        workspace = torch.empty(max(1, check_tiles_workspace_size(ctx, vshape, nbox, tile_dims)),
                                dtype=torch.uint8, device=V.device)
    ctx._raise(ctx._lib.sal_check_tiles(
        ctx._h, _ptr(V), *vshape, vstride, box.ctypes.data_as(_i64p), _ptr(S_raw), *S_raw.shape[1:],
        til.ctypes.data_as(_i64p), nbox, dims, _ptr(stats), float(bound), _ptr(err_out), _ptr(exact_out),
        _ptr(workspace), workspace.numel(), _stream(V.device)))


def absmax(ctx: "Saliency", V: torch.Tensor, out: torch.Tensor, accumulate: bool = False) -> torch.Tensor:
    """out[0] = max |V| (accumulate: max(out[0], max |V|)); V any contiguous float32 CUDA
    tensor, out a CUDA float32 tensor of at least one element."""
    if not (V.is_cuda and V.dtype == torch.float32 and V.is_contiguous()):
        raise ValueError("V must be a contiguous float32 CUDA tensor")
    if not (out.is_cuda and out.dtype == torch.float32 and out.numel() >= 1):
        raise ValueError("out must be a float32 CUDA tensor")
    ctx._raise(ctx._lib.sal_absmax(ctx._h, _ptr(V), V.numel(), _ptr(out), int(bool(accumulate)),
                                   _stream(V.device)))
    return out


def tile_minmax(ctx: "Saliency", S_raw: torch.Tensor, tile: int,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per-tile {min, max} of each raw map: float32 [ntiles, 6] on the device."""
    if not (S_raw.is_cuda and S_raw.dtype == torch.float32 and S_raw.is_contiguous()):
        raise ValueError("S_raw must be a contiguous float32 CUDA tensor")
    shape = tuple(S_raw.shape[1:])
    nt = 1
    for n in shape:
        nt *= (n + tile - 1) // tile
    if out is None:
        out = torch.empty((nt, 6), dtype=torch.float32, device=S_raw.device)
    ctx._raise(ctx._lib.sal_tile_minmax(ctx._h, _ptr(S_raw), *shape, int(tile), _ptr(out),
                                        _stream(S_raw.device)))
    return out


class Net:
    """The learned surrogate (five 3x3x3 conv layers, 24 channels, GELU) in HIP kernels."""

    def __init__(self, seed: int = 0, device: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        st = self._lib.sal_net_create(device, int(seed), ctypes.byref(h))
        if st != SAL_OK:
            raise SalError(st, self._lib.sal_net_last_error(None).decode())
        self._h = h
        self.device = torch.device("cuda", device)
        self.num_params = int(self._lib.sal_net_num_params())
        self._ws = None
        self.out_scale = (1.0, 1.0, 1.0)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sal_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        if st != SAL_OK:
            raise SalError(st, self._lib.sal_net_last_error(self._h).decode())

    def set_precision(self, precision: int):
        """FP32 (the FP32-operand mode of the same kernels) or BF16 (default)."""
        self._raise(self._lib.sal_net_set_precision(self._h, int(precision)))
        self._ws = None

    def adam(self, lr: float):
        """One Adam step on the accumulated gradient (cleared afterwards)."""
        self._raise(self._lib.sal_net_adam(self._h, float(lr), _stream(self.device)))

    def get_params(self):
        import numpy as np
        a = np.zeros(self.num_params, np.float32)
        self._raise(self._lib.sal_net_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                             self.num_params, 0))
        return a

    def set_params(self, a):
        import numpy as np
        a = np.ascontiguousarray(a, np.float32)
        self._raise(self._lib.sal_net_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                             self.num_params, 1))

    def grads(self, zero: bool = True):
        import numpy as np
        a = np.zeros(self.num_params, np.float32)
        self._raise(self._lib.sal_net_grads(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            self.num_params, int(zero)))
        return a

    def set_output_scale(self, scale):
        self.out_scale = tuple(float(s) for s in scale)
        arr = (ctypes.c_float * 3)(*self.out_scale)
        self._raise(self._lib.sal_net_set_output_scale(self._h, arr))

    def workspace(self, nb, shape, train: bool):
        n = ctypes.c_size_t()
        self._raise(self._lib.sal_net_workspace_size(self._h, int(nb), *[int(s) for s in shape],
                                                     int(train), ctypes.byref(n)))
        if self._ws is None or self._ws.numel() < n.value:
            self._ws = None
            self._ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        return self._ws

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        """X [nb, n0, n1, n2] float32 -> Y [nb, n0, n1, n2, 3] (activations kept)."""
        nb, shape = X.shape[0], tuple(X.shape[1:])
        Y = torch.empty(X.shape + (3,), dtype=torch.float32, device=X.device)
        ws = self.workspace(nb, shape, True)
        self._raise(self._lib.sal_net_forward(self._h, _ptr(X), nb, *shape, _ptr(Y), _ptr(ws),
                                              ws.numel(), _stream(X.device)))
        return Y

    def backward(self, X: torch.Tensor, dY: torch.Tensor):
        nb, shape = X.shape[0], tuple(X.shape[1:])
        ws = self.workspace(nb, shape, True)
        self._raise(self._lib.sal_net_backward(self._h, _ptr(X), _ptr(dY.contiguous()), nb, *shape,
                                               _ptr(ws), ws.numel(), _stream(X.device)))

    def train_step(self, X: torch.Tensor, T: torch.Tensor, margin: int, lr: float,
                   loss_out: Optional[torch.Tensor] = None):
        nb, S = X.shape[0], X.shape[1]
        ws = self.workspace(nb, (S, S, S), True)
        self._raise(self._lib.sal_net_train_step(self._h, _ptr(X), _ptr(T), nb, S, int(margin),
                                                 float(lr), _ptr(loss_out), _ptr(ws), ws.numel(),
                                                 _stream(X.device)))

    def infer(self, V: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Predicted raw maps [3, n0, n1, n2] of a whole volume."""
        _check_vol(V)
        shape = tuple(V.shape)
        if out is None:
            out = torch.empty((3,) + shape, dtype=torch.float32, device=V.device)
        ws = self.workspace(1, shape, False)
        self._raise(self._lib.sal_net_infer(self._h, _ptr(V), *shape, _ptr(out), _ptr(ws),
                                            ws.numel(), _stream(V.device)))
        return out
