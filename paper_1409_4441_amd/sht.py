"""Harmonic half of the kernel split and the hybrid apply: ctypes binding of include/convsht.h
(argument marshalling only; every transform runs in libconvreal's kernels).

    from paper_1409_4441_amd import sht
    t = sht.Sht(nside, lmax)                     # plan on the current device
    alm = t.analysis(x)                          # complex128 cuda tensor, m-major (l, m >= 0)
    y = t.synthesis(alm, dtype=torch.float64)    # map
    y = t.convolve(x, k_ell)                     # synthesis(k_l * analysis(x))
    cl = t.power_spectrum(alm)
    y = sht.hybrid_apply(real_plan, t, k_hat, x, stream_sht=torch.cuda.Stream())   # Eq. 1, Fig. 1
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import ConvRealError, _check, _stream_handle, lib

F64, F32 = 0, 1

# Every entry point that include/convsht.h declares.
EXPORTS = ("conv_sht_init", "conv_sht_alm_size", "conv_sht_analysis", "conv_sht_synthesis", "conv_sht_almxfl",
           "conv_sht_convolve", "conv_sht_power_spectrum", "conv_hybrid_apply", "conv_sht_destroy")

_c_int, _c_void_p = ctypes.c_int, ctypes.c_void_p


def _bind():
    lib.conv_sht_init.argtypes = [ctypes.POINTER(_c_void_p), _c_int, _c_int]
    lib.conv_sht_alm_size.argtypes = [_c_int, ctypes.POINTER(ctypes.c_longlong)]
    lib.conv_sht_analysis.argtypes = [_c_void_p, _c_void_p, _c_int, _c_void_p, _c_void_p]
    lib.conv_sht_synthesis.argtypes = [_c_void_p, _c_void_p, _c_void_p, _c_int, _c_int, _c_void_p]
    lib.conv_sht_almxfl.argtypes = [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]
    lib.conv_sht_convolve.argtypes = [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_int, _c_int, _c_void_p]
    lib.conv_sht_power_spectrum.argtypes = [_c_void_p, _c_void_p, _c_void_p, _c_void_p]
    lib.conv_hybrid_apply.argtypes = [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_int, _c_void_p,
                                      _c_void_p]
    lib.conv_sht_destroy.argtypes = [_c_void_p]
    for f in EXPORTS:
        getattr(lib, f).restype = _c_int


_bind()


def alm_size(lmax: int) -> int:
    n = ctypes.c_longlong()
    _check(lib.conv_sht_alm_size(int(lmax), ctypes.byref(n)), "conv_sht_alm_size")
    return int(n.value)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("maps must be float64 or float32")


class Sht:
    """Spherical-harmonic transforms of one (nside, lmax) on the current device."""

    def __init__(self, nside: int, lmax: int):
        h = _c_void_p()
        _check(lib.conv_sht_init(ctypes.byref(h), int(nside), int(lmax)), "conv_sht_init")
        self._h = h
        self.nside = int(nside)
        self.lmax = int(lmax)
        self.npix = 12 * self.nside ** 2
        self.nalm = alm_size(lmax)

    def _map(self, x, name="x"):
        import torch
        if not isinstance(x, torch.Tensor) or not x.is_cuda or not x.is_contiguous() or x.numel() != self.npix:
            raise ValueError(f"{name} must be a contiguous cuda tensor of {self.npix} values")
        return _dtype_code(x)

    def _alm(self, a, name="alm"):
        import torch
        if (not isinstance(a, torch.Tensor) or not a.is_cuda or a.dtype != torch.complex128
                or not a.is_contiguous() or a.numel() != self.nalm):
            raise ValueError(f"{name} must be a contiguous complex128 cuda tensor of {self.nalm} values")

    def _fl(self, fl):
        import torch
        if not isinstance(fl, torch.Tensor):
            fl = torch.as_tensor(np.ascontiguousarray(fl, dtype=np.float64), device="cuda")
        if not fl.is_cuda or fl.dtype != torch.float64 or fl.numel() != self.lmax + 1 or not fl.is_contiguous():
            raise ValueError(f"the kernel must hold lmax + 1 = {self.lmax + 1} float64 values on the device")
        return fl

    def analysis(self, x, out=None, stream=None):
        import torch
        dt = self._map(x)
        if out is None:
            out = torch.empty(self.nalm, dtype=torch.complex128, device=x.device)
        self._alm(out, "out")
        _check(lib.conv_sht_analysis(self._h, _ptr(x), dt, _ptr(out), _stream_handle(stream)), "conv_sht_analysis")
        return out

    def synthesis(self, alm, out=None, dtype=None, accumulate: bool = False, stream=None):
        import torch
        self._alm(alm)
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs out")
            out = torch.empty(self.npix, dtype=dtype or torch.float64, device=alm.device)
        dt = self._map(out, "out")
        _check(lib.conv_sht_synthesis(self._h, _ptr(alm), _ptr(out), dt, int(bool(accumulate)), _stream_handle(stream)),
               "conv_sht_synthesis")
        return out

    def almxfl(self, alm, fl, out=None, stream=None):
        import torch
        self._alm(alm)
        fl = self._fl(fl)
        if out is None:
            out = torch.empty_like(alm)
        self._alm(out, "out")
        _check(lib.conv_sht_almxfl(self._h, _ptr(alm), _ptr(fl), _ptr(out), _stream_handle(stream)), "conv_sht_almxfl")
        return out

    def convolve(self, x, k_ell, out=None, accumulate: bool = False, stream=None):
        import torch
        dt = self._map(x)
        k = self._fl(k_ell)
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs out")
            out = torch.empty_like(x)
        if self._map(out, "out") != dt:
            raise TypeError("x and out must have the same dtype")
        _check(lib.conv_sht_convolve(self._h, _ptr(x), _ptr(k), _ptr(out), dt, int(bool(accumulate)),
                                     _stream_handle(stream)), "conv_sht_convolve")
        return out

    def power_spectrum(self, alm, stream=None):
        import torch
        self._alm(alm)
        cl = torch.empty(self.lmax + 1, dtype=torch.float64, device=alm.device)
        _check(lib.conv_sht_power_spectrum(self._h, _ptr(alm), _ptr(cl), _stream_handle(stream)),
               "conv_sht_power_spectrum")
        return cl

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and lib is not None:
            lib.conv_sht_destroy(self._h)
            self._h = _c_void_p()

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def hybrid_apply(real_plan, sht: Sht, k_hat, x, out=None, stream=None, stream_sht=None):
    """maps_out = real-space part (real_plan) + synthesis(k_hat * analysis(x)) (conv_hybrid_apply):
    x [npix] or [nmaps, npix] (float64 for an "f64" real-space plan, float32 otherwise); the harmonic
    half runs on stream_sht at the same time as the real-space half (None: one after the other)."""
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or not x.is_contiguous() or x.shape[-1] != sht.npix:
        raise ValueError("x must be a contiguous cuda tensor of maps on the plans' grid")
    k = sht._fl(k_hat)
    if out is None:
        out = torch.empty_like(x)
    if out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must match x")
    nmaps = 1 if x.dim() == 1 else x.shape[0]
    s2 = None if stream_sht is None else _stream_handle(stream_sht)
    _check(lib.conv_hybrid_apply(real_plan._h, sht._h, _ptr(k), _ptr(x), _ptr(out), int(nmaps),
                                 _stream_handle(stream), s2), "conv_hybrid_apply")
    return out


__all__ = ["Sht", "hybrid_apply", "alm_size", "ConvRealError"]
