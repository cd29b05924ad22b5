"""paper_1409_4441_amd - real-space half of a split spherical convolution on MI355X.

Thin ctypes binding of libconvreal.so (declared in include/convreal.h): argument
marshalling only. Every step of the convolution runs in the library's HIP
kernels; PyTorch supplies device memory and streams. There is no CPU fallback:
if the library is missing, importing this package raises.

    import paper_1409_4441_amd as cr
    table = cr.tabulate(k_ell, theta_cut, n_tab)           # K on chord nodes (device FP64)
    plan = cr.Plan(nside, table, theta_cut, "f32")          # ring windows, pair count, tables
    y = plan.apply(x)                                       # x: cuda tensor [nmaps, 12 nside^2]
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CONVREAL_LIB selects another build of the same library (e.g. one with host sanitizers)
LIB_PATH = os.environ.get("CONVREAL_LIB") or os.path.join(_HERE, "libconvreal.so")

F64 = 0
F32 = 1
MIXED = 2
_PRECISIONS = {"f64": F64, "f32": F32, "mixed": MIXED}

_STORE_MODES = {"off": 0, "on": 1, "auto": 2}
_METHODS = {"direct": 0, "ring_fft": 1}

OK = 0
EINVAL = -1
ENOMEM = -2
EHIP = -3
EALIAS = -4
ENODEV = -5

# Every entry point that include/convreal.h declares.
EXPORTS = ("conv_real_tabulate", "conv_real_init", "conv_real_apply", "conv_real_pairs",
           "conv_real_profile", "conv_real_set_tuning", "conv_real_get_tuning", "conv_real_autotune",
           "conv_real_batch_create", "conv_real_batch_apply", "conv_real_batch_set_tuning",
           "conv_real_batch_autotune", "conv_real_batch_pairs", "conv_real_batch_destroy",
           "conv_real_destroy", "conv_real_strerror", "conv_real_last_error",
           "conv_real_set_weight_store", "conv_real_get_weight_store", "conv_real_set_method",
           "conv_real_get_method", "conv_real_apply_noalloc")


class Tuning(ctypes.Structure):
    """conv_real_tuning: seg (256|512), wg_per_cu (1..4), order (0..4)."""
    _fields_ = [("seg", ctypes.c_int), ("wg_per_cu", ctypes.c_int), ("order", ctypes.c_int)]

    def as_dict(self):
        return {"seg": self.seg, "wg_per_cu": self.wg_per_cu, "order": self.order}


class ConvRealError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        text = msg if msg.startswith(where) else f"{where}: {msg}"
        super().__init__(f"{text} (code {code})")
        self.code = code


def _load():
    # PyTorch bundles HIP and HSA runtime libraries with the same sonames as the system ROCm ones
    # this library links (libamdhip64.so.7, libhsa-runtime64.so.1). Whichever loads first serves the
    # whole process; PyTorch does not find the device on the system runtime, while this library runs
    # on PyTorch's. So PyTorch is imported before the library is loaded: one runtime, shared.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_1409_4441_amd/build.py` "
                          "(the convolution has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    dptr = ctypes.POINTER(ctypes.c_double)
    lib.conv_real_tabulate.argtypes = [dptr, c_int, c_double, c_int, dptr]
    lib.conv_real_tabulate.restype = c_int
    lib.conv_real_init.argtypes = [ctypes.POINTER(c_void_p), c_int, dptr, c_int, c_double, c_int]
    lib.conv_real_init.restype = c_int
    lib.conv_real_apply.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_void_p]
    lib.conv_real_apply.restype = c_int
    lib.conv_real_apply_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_void_p]
    lib.conv_real_apply_noalloc.restype = c_int
    lib.conv_real_pairs.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_longlong)]
    lib.conv_real_pairs.restype = c_int
    lib.conv_real_profile.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_void_p,
                                      ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(c_int)]
    lib.conv_real_profile.restype = c_int
    tp = ctypes.POINTER(Tuning)
    fpp = ctypes.POINTER(c_void_p)
    lib.conv_real_set_tuning.argtypes = [c_void_p, tp]
    lib.conv_real_get_tuning.argtypes = [c_void_p, tp]
    lib.conv_real_autotune.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_void_p, tp]
    lib.conv_real_batch_create.argtypes = [ctypes.POINTER(c_void_p), fpp, c_int]
    lib.conv_real_batch_apply.argtypes = [c_void_p, fpp, fpp, c_void_p]
    lib.conv_real_batch_set_tuning.argtypes = [c_void_p, tp]
    lib.conv_real_batch_autotune.argtypes = [c_void_p, fpp, fpp, c_void_p, tp]
    lib.conv_real_batch_pairs.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_longlong)]
    lib.conv_real_batch_destroy.argtypes = [c_void_p]
    for name in ("conv_real_set_tuning", "conv_real_get_tuning", "conv_real_autotune", "conv_real_batch_create",
                 "conv_real_batch_apply", "conv_real_batch_set_tuning", "conv_real_batch_autotune",
                 "conv_real_batch_pairs", "conv_real_batch_destroy"):
        getattr(lib, name).restype = c_int
    lib.conv_real_set_weight_store.argtypes = [c_void_p, c_int]
    lib.conv_real_set_weight_store.restype = c_int
    lib.conv_real_get_weight_store.argtypes = [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(ctypes.c_longlong)]
    lib.conv_real_get_weight_store.restype = c_int
    lib.conv_real_set_method.argtypes = [c_void_p, c_int]
    lib.conv_real_set_method.restype = c_int
    lib.conv_real_get_method.argtypes = [c_void_p, ctypes.POINTER(c_int)]
    lib.conv_real_get_method.restype = c_int
    lib.conv_real_destroy.argtypes = [c_void_p]
    lib.conv_real_destroy.restype = c_int
    lib.conv_real_strerror.argtypes = [c_int]
    lib.conv_real_strerror.restype = ctypes.c_char_p
    lib.conv_real_last_error.argtypes = []
    lib.conv_real_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(code: int, where: str):
    if code != OK:
        msg = lib.conv_real_last_error().decode() or lib.conv_real_strerror(code).decode()
        raise ConvRealError(code, where, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tabulate(k_ell, theta_cut: float, n_tab: int) -> np.ndarray:
    """K(d_k) = sum_l (2l+1)/(4 pi) k_l P_l(cos theta_k) on the plan's chord nodes (device FP64)."""
    k = np.ascontiguousarray(k_ell, dtype=np.float64)
    out = np.empty(int(n_tab), dtype=np.float64)
    _check(lib.conv_real_tabulate(_dptr(k), len(k) - 1, float(theta_cut), int(n_tab), _dptr(out)),
           "conv_real_tabulate")
    return out


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Plan:
    """One (nside, kernel table, theta_cut, precision) on the current device."""

    def __init__(self, nside: int, table, theta_cut: float, precision: str = "f64"):
        if precision not in _PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(_PRECISIONS)}")
        t = np.ascontiguousarray(table, dtype=np.float64)
        handle = ctypes.c_void_p()
        _check(lib.conv_real_init(ctypes.byref(handle), int(nside), _dptr(t), len(t),
                                  float(theta_cut), _PRECISIONS[precision]), "conv_real_init")
        self._h = handle
        self.nside = int(nside)
        self.npix = 12 * self.nside * self.nside
        self.theta_cut = float(theta_cut)
        self.precision = precision
        self.n_tab = len(t)

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == "f64" else torch.float32

    def pairs(self) -> int:
        n = ctypes.c_longlong()
        _check(lib.conv_real_pairs(self._h, ctypes.byref(n)), "conv_real_pairs")
        return int(n.value)

    def set_weight_store(self, mode: str):
        """"off", "on" or "auto": cap weights evaluated per apply, or computed once and streamed."""
        _check(lib.conv_real_set_weight_store(self._h, _STORE_MODES.get(mode, -1)), "conv_real_set_weight_store")

    def weight_store(self):
        """(active, bytes) of the cap weight store."""
        a, b = ctypes.c_int(), ctypes.c_longlong()
        _check(lib.conv_real_get_weight_store(self._h, ctypes.byref(a), ctypes.byref(b)),
               "conv_real_get_weight_store")
        return bool(a.value), int(b.value)

    def set_method(self, method: str):
        """"direct" or "ring_fft" (FP64 and mixed plans): pair sums, or belt ring pairs through ring
        FFTs (the cap-touching pairs stay on the plan's own cap path)."""
        _check(lib.conv_real_set_method(self._h, _METHODS.get(method, -1)), "conv_real_set_method")

    def method(self) -> str:
        m = ctypes.c_int()
        _check(lib.conv_real_get_method(self._h, ctypes.byref(m)), "conv_real_get_method")
        return {v: k for k, v in _METHODS.items()}[m.value]

    def apply(self, x, out=None, stream=None):
        """y = A x. x: CUDA tensor [npix] or [nmaps, npix], contiguous, plan dtype."""
        import torch
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError("x must be a CUDA tensor")
        if x.dtype != self.dtype:
            raise TypeError(f"x must be {self.dtype}")
        if x.shape[-1] != self.npix or x.dim() not in (1, 2):
            raise ValueError(f"x must have shape [nmaps, {self.npix}]")
        if not x.is_contiguous():
            raise ValueError("x must be contiguous")
        if out is None:
            out = torch.empty_like(x)
        elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or not out.is_cuda:
            raise ValueError("out must match x")
        nmaps = 1 if x.dim() == 1 else x.shape[0]
        _check(lib.conv_real_apply(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   int(nmaps), _stream_handle(stream)), "conv_real_apply")
        return out

    def apply_noalloc(self, x, out, stream=None):
        """y = A x through conv_real_apply_noalloc: the library allocates nothing (its per-launch
        scratch is a fixed device array shared by all such calls on the device, so calls that may
        overlap in time race). out must be given (a preallocated tensor like x)."""
        if out is None:
            raise ValueError("apply_noalloc needs a preallocated out tensor")
        out, nmaps = self._check_maps(x, out)
        _check(lib.conv_real_apply_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           int(nmaps), _stream_handle(stream)), "conv_real_apply_noalloc")
        return out

    def _check_maps(self, x, out):
        import torch
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError("x must be a CUDA tensor")
        if x.dtype != self.dtype:
            raise TypeError(f"x must be {self.dtype}")
        if x.shape[-1] != self.npix or x.dim() not in (1, 2) or not x.is_contiguous():
            raise ValueError(f"x must be contiguous with shape [nmaps, {self.npix}]")
        if out is None:
            out = torch.empty_like(x)
        elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or not out.is_cuda:
            raise ValueError("out must match x")
        return out, (1 if x.dim() == 1 else x.shape[0])

    def profile(self, x, out=None, stream=None):
        """Run one apply with events between the library's kernels (synchronous).
        Returns (out, [(kernel_name, milliseconds, pixel_pairs), ...])."""
        out, nmaps = self._check_maps(x, out)
        cap = 32
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_float * cap)()
        work = (ctypes.c_longlong * cap)()
        n = ctypes.c_int(cap)
        _check(lib.conv_real_profile(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     int(nmaps), _stream_handle(stream), names, ms, work, ctypes.byref(n)),
               "conv_real_profile")
        return out, [(names[k].decode(), float(ms[k]), int(work[k])) for k in range(n.value)]

    def set_tuning(self, seg: int = 256, wg_per_cu: int = 2, order: int = 0):
        t = Tuning(seg, wg_per_cu, order)
        _check(lib.conv_real_set_tuning(self._h, ctypes.byref(t)), "conv_real_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib.conv_real_get_tuning(self._h, ctypes.byref(t)), "conv_real_get_tuning")
        return t.as_dict()

    def autotune(self, x, out=None, stream=None, cache: str | None = None) -> dict:
        """Fastest launch configuration for maps like x (timed by the library), kept on the plan.
        With `cache`, a JSON file keyed by (nside, theta_cut, precision, nmaps bucket) is read
        first and updated after a search."""
        out, nmaps = self._check_maps(x, out)
        key = f"{self.nside}|{self.theta_cut:.6g}|{self.precision}|{1 if nmaps == 1 else 2 ** (nmaps - 1).bit_length()}"
        if cache is not None:
            found = _cache_get(cache, key)
            if found is not None:
                self.set_tuning(**found)
                return found
        t = Tuning()
        _check(lib.conv_real_autotune(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      int(nmaps), _stream_handle(stream), ctypes.byref(t)), "conv_real_autotune")
        if cache is not None:
            _cache_put(cache, key, t.as_dict())
        return t.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.conv_real_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _cache_get(path, key):
    import json
    try:
        with open(path) as f:
            data = json.load(f)
        t = data.get(key)
        if isinstance(t, dict) and set(t) == {"seg", "wg_per_cu", "order"}:
            return {k: int(v) for k, v in t.items()}
    except (OSError, ValueError):
        pass                                     # missing or corrupt cache: search again
    return None


def _cache_put(path, key, value):
    import json
    import os
    data = {}
    try:
        with open(path) as f:
            data = json.load(f)
        if not isinstance(data, dict):
            data = {}
    except (OSError, ValueError):
        data = {}
    data[key] = value
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class Batch:
    """Maps of different grids and kernels (one mixed plan each) in one persistent launch."""

    def __init__(self, plans):
        if not plans or len(plans) > 64:
            raise ValueError("need 1..64 plans")
        self.plans = list(plans)                 # keeps the plans alive
        arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
        h = ctypes.c_void_p()
        _check(lib.conv_real_batch_create(ctypes.byref(h), arr, len(plans)), "conv_real_batch_create")
        self._h = h

    def _ptrs(self, xs, outs):
        import torch
        if len(xs) != len(self.plans):
            raise ValueError("one map per plan")
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        for p, x, o in zip(self.plans, xs, outs):
            if not (x.is_cuda and o.is_cuda and x.dtype == torch.float32 and o.dtype == torch.float32):
                raise TypeError("maps must be float32 CUDA tensors")
            if x.numel() != p.npix or o.numel() != p.npix or not x.is_contiguous() or not o.is_contiguous():
                raise ValueError("map k must hold 12 nside_k^2 contiguous values")
        pin = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        pout = (ctypes.c_void_p * len(xs))(*[o.data_ptr() for o in outs])
        return outs, pin, pout

    def apply(self, xs, outs=None, stream=None):
        outs, pin, pout = self._ptrs(xs, outs)
        _check(lib.conv_real_batch_apply(self._h, pin, pout, _stream_handle(stream)), "conv_real_batch_apply")
        return outs

    def pairs(self) -> int:
        n = ctypes.c_longlong()
        _check(lib.conv_real_batch_pairs(self._h, ctypes.byref(n)), "conv_real_batch_pairs")
        return int(n.value)

    def set_tuning(self, seg: int = 256, wg_per_cu: int = 2, order: int = 0):
        t = Tuning(seg, wg_per_cu, order)
        _check(lib.conv_real_batch_set_tuning(self._h, ctypes.byref(t)), "conv_real_batch_set_tuning")

    def autotune(self, xs, outs=None, stream=None) -> dict:
        outs, pin, pout = self._ptrs(xs, outs)
        t = Tuning()
        _check(lib.conv_real_batch_autotune(self._h, pin, pout, _stream_handle(stream), ctypes.byref(t)),
               "conv_real_batch_autotune")
        return t.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.conv_real_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
