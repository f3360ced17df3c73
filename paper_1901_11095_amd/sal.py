"""Python binding of libsal (ctypes): argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch supplies device memory
and the current HIP stream.  If ``libsal.so`` has not been built this module raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

from .build import LIB as _LIB_PATH

SAL_OK, SAL_E_INVAL, SAL_E_UNSUPPORTED, SAL_E_DEVICE, SAL_E_WORKSPACE = range(5)
FP32, BF16, BF16_SPLIT, FP16, FP16_SPLIT, BF16_SPLITW, FP16_SPLITW = range(7)
PRECISION_NAMES = {FP32: "fp32", BF16: "bf16", BF16_SPLIT: "bf16_split", FP16: "fp16",
                   FP16_SPLIT: "fp16_split", BF16_SPLITW: "bf16_splitw",
                   FP16_SPLITW: "fp16_splitw"}
RAY_PT, RAY_MT, RAY_PX, RAY_MX, RAY_PY, RAY_MY = 1, 2, 4, 8, 16, 32
RAYS_AXIS = (RAY_PT | RAY_MT, RAY_PX | RAY_MX, RAY_PY | RAY_MY)
RAYS_ALL = (63, 63, 63)
STATS_LEN = 7

EXPORTS = ("sal_default_params", "sal_create", "sal_destroy", "sal_last_error",
           "sal_workspace_size", "sal_local_spectra", "sal_project", "sal_directional_compare",
           "sal_saliency", "sal_profile_enable", "sal_profile_read")
KERNELS = ("energy", "dcs", "stats", "combine")


class SalError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("sal status %d: %s" % (status, msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("d", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("rays", ctypes.c_uint32 * 3), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("c", ctypes.c_double), ("normalize", ctypes.c_int32),
                ("zero_range", ctypes.c_double), ("precision", ctypes.c_int32)]


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
    for f in ("sal_create", "sal_workspace_size", "sal_local_spectra", "sal_project",
              "sal_directional_compare", "sal_saliency", "sal_profile_enable",
              "sal_profile_read"):
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
                 device: int = 0):
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
