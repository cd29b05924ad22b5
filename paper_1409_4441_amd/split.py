"""Kernel-split model: ctypes binding of include/convsplit.h (argument marshalling only).

    from paper_1409_4441_amd import split
    ctx = split.Context(lmax, theta_max)                  # Gauss-Legendre samples, Legendre operator
    k_hat, k_theta, k_real, k_tilde = ctx.lsq(k_ell, ell_cut, theta_cut)   # Eqs. 3-5
    sigma_rms, sigma = ctx.error(k_ell, ell_cut, theta_cut, alpha=5.0)      # Eqs. 2 and 6
    model = split.CostModel.fit(pairs, t_real, npix_sht, work_sht, t_sht)
    best = ctx.search(k_ell, nside, bound, theta_grid, model)             # the split scan

Everything runs in libconvreal's host code (FP64); no GPU is needed.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import ConvRealError, _check, lib

INFEASIBLE = 1

# Every entry point that include/convsplit.h declares.
EXPORTS = ("conv_split_create", "conv_split_destroy", "conv_split_nodes", "conv_split_lsq", "conv_split_error",
           "conv_cost_pairs", "conv_cost_fit", "conv_cost_eval", "conv_split_search", "conv_split_search_many",
           "conv_split_compensation", "conv_split_set_max_compensation", "conv_split_set_max_ell_fraction")

_c_int, _c_double, _c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
_dptr_t = ctypes.POINTER(ctypes.c_double)
_iptr_t = ctypes.POINTER(ctypes.c_int)


class _Cost(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double), ("c0", ctypes.c_double),
                ("c1", ctypes.c_double)]


def _bind():
    lib.conv_split_create.argtypes = [ctypes.POINTER(_c_void_p), _c_int, _dptr_t, _c_double, _c_double]
    lib.conv_split_destroy.argtypes = [_c_void_p]
    lib.conv_split_nodes.argtypes = [_c_void_p, _c_double, _iptr_t]
    lib.conv_split_lsq.argtypes = [_c_void_p, _dptr_t, _c_int, _c_double, _dptr_t, _dptr_t, _dptr_t, _dptr_t]
    lib.conv_split_error.argtypes = [_c_void_p, _dptr_t, _c_int, _c_double, _c_double, _dptr_t, _dptr_t]
    lib.conv_split_compensation.argtypes = [_c_void_p, _dptr_t, _c_int, _c_double, _dptr_t]
    lib.conv_split_set_max_compensation.argtypes = [_c_void_p, _c_double]
    lib.conv_split_set_max_ell_fraction.argtypes = [_c_void_p, _c_double]
    lib.conv_cost_pairs.argtypes = [_c_int, _c_double]
    lib.conv_cost_pairs.restype = _c_double
    lib.conv_cost_fit.argtypes = [_dptr_t, _dptr_t, _c_int, _dptr_t, _dptr_t, _dptr_t, _c_int, ctypes.POINTER(_Cost)]
    lib.conv_cost_eval.argtypes = [ctypes.POINTER(_Cost), _c_int, _c_int, _c_double, _c_int, _dptr_t, _dptr_t,
                                   _dptr_t]
    lib.conv_split_search.argtypes = [_c_void_p, _dptr_t, _c_int, _c_double, _c_double, _dptr_t, _c_int, _c_int,
                                      ctypes.POINTER(_Cost), _dptr_t, _iptr_t, _dptr_t, _dptr_t]
    lib.conv_split_search_many.argtypes = [_c_void_p, _dptr_t, _c_int, _c_int, _dptr_t, _c_double, _dptr_t, _c_int,
                                           _c_int, ctypes.POINTER(_Cost), _c_int, _dptr_t, _iptr_t, _dptr_t,
                                           _dptr_t]
    for f in ("conv_split_create", "conv_split_destroy", "conv_split_nodes", "conv_split_lsq", "conv_split_error",
              "conv_cost_fit", "conv_cost_eval", "conv_split_search", "conv_split_search_many",
              "conv_split_compensation", "conv_split_set_max_compensation", "conv_split_set_max_ell_fraction"):
        getattr(lib, f).restype = _c_int


_bind()


def _d(a):
    return a.ctypes.data_as(_dptr_t)


def _f64(a, n=None, name="array"):
    out = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and out.shape != (n,):
        raise ConvRealError(-1, name, f"expected {n} values, got shape {out.shape}")
    return out


class CostModel:
    """t_real = a + b pairs, t_sht = c0 + c1 npix + c ell_cut^2 lmax, wall = max of the two."""

    def __init__(self, a: float, b: float, c: float, c0: float = 0.0, c1: float = 0.0):
        self._s = _Cost(float(a), float(b), float(c), float(c0), float(c1))

    @property
    def a(self):
        return self._s.a

    @property
    def b(self):
        return self._s.b

    @property
    def c(self):
        return self._s.c

    @property
    def c0(self):
        return self._s.c0

    @property
    def c1(self):
        return self._s.c1

    def as_dict(self):
        return {"a": self.a, "b": self.b, "c": self.c, "c0": self.c0, "c1": self.c1}

    @classmethod
    def from_dict(cls, d) -> "CostModel":
        """From a dict with a, b, c and optionally c0, c1 (cost_model.json)."""
        return cls(d["a"], d["b"], d["c"], d.get("c0", 0.0), d.get("c1", 0.0))

    @classmethod
    def fit(cls, pairs, t_real, npix_sht, work_sht, t_sht) -> "CostModel":
        p, tr = _f64(pairs), _f64(t_real)
        npx, w, ts = _f64(npix_sht), _f64(work_sht), _f64(t_sht)
        m = _Cost()
        _check(lib.conv_cost_fit(_d(p), _d(tr), len(p), _d(npx), _d(w), _d(ts), len(w), ctypes.byref(m)),
               "conv_cost_fit")
        return cls(m.a, m.b, m.c, m.c0, m.c1)

    def eval(self, nside: int, lmax: int, theta_cut: float, ell_cut: int):
        """(t_real, t_sht, wall) in seconds."""
        tr, ts, wl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib.conv_cost_eval(ctypes.byref(self._s), int(nside), int(lmax), float(theta_cut), int(ell_cut),
                                  ctypes.byref(tr), ctypes.byref(ts), ctypes.byref(wl)), "conv_cost_eval")
        return tr.value, ts.value, wl.value


def wiener_weights(signal_cl, noise_cl) -> np.ndarray:
    """Input weights of Eqs. 2 and 6 for a Wiener-filter convolution (text after Eq. 2):
    C^in_l = S_l^2 / (S_l + N_l) for signal power S_l and noise power N_l (scalar or per l); 0 where
    both vanish."""
    S = np.asarray(signal_cl, dtype=np.float64)
    N = np.asarray(noise_cl, dtype=np.float64) * np.ones_like(S)
    den = S + N
    return np.where(den > 0, S * S / np.where(den > 0, den, 1.0), 0.0)


def pairs_estimate(nside: int, theta_cut: float) -> float:
    """Npix^2 (1 - cos theta_cut) / 2."""
    return float(lib.conv_cost_pairs(int(nside), float(theta_cut)))


class Context:
    """Split model for one lmax and input weighting C_in (None: flat), theta_cut <= theta_max; the
    search accepts splits of compensation <= max_comp (0: any) and l_cut <= max_ell_frac lmax (or
    l_cut = lmax)."""

    def __init__(self, lmax: int, theta_max: float, c_in=None, sv_cut: float = 1e-6, max_comp: float = 0.0,
                 max_ell_frac: float = 1.0):
        self.lmax = int(lmax)
        self.theta_max = float(theta_max)
        c = None if c_in is None else _f64(c_in, self.lmax + 1, "c_in")
        h = _c_void_p()
        _check(lib.conv_split_create(ctypes.byref(h), self.lmax, None if c is None else _d(c), self.theta_max,
                                     float(sv_cut)), "conv_split_create")
        self._h = h
        if max_comp:
            _check(lib.conv_split_set_max_compensation(h, float(max_comp)), "conv_split_set_max_compensation")
        if max_ell_frac < 1.0:
            _check(lib.conv_split_set_max_ell_fraction(h, float(max_ell_frac)), "conv_split_set_max_ell_fraction")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and lib is not None:
            lib.conv_split_destroy(self._h)
            self._h = _c_void_p()

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def nodes(self, theta_cut: float) -> int:
        n = ctypes.c_int()
        _check(lib.conv_split_nodes(self._h, float(theta_cut), ctypes.byref(n)), "conv_split_nodes")
        return n.value

    def lsq(self, k_ell, ell_cut: int, theta_cut: float):
        """(k_hat[ell_cut+1], k_theta[z_cut], k_real[lmax+1], k_tilde[lmax+1])."""
        k = _f64(k_ell, self.lmax + 1, "k_ell")
        n = self.nodes(theta_cut)
        kh = np.empty(int(ell_cut) + 1 if 0 <= int(ell_cut) <= self.lmax else 1)
        kt = np.empty(max(n, 1))
        kr = np.empty(self.lmax + 1)
        ktl = np.empty(self.lmax + 1)
        _check(lib.conv_split_lsq(self._h, _d(k), int(ell_cut), float(theta_cut), _d(kh), _d(kt), _d(kr), _d(ktl)),
               "conv_split_lsq")
        return kh, kt[:n], kr, ktl

    def compensation(self, k_ell, ell_cut: int, theta_cut: float) -> float:
        """max_{l <= l_cut} |(P x)_l| / max_l |K_l| of the split."""
        k = _f64(k_ell, self.lmax + 1, "k_ell")
        c = ctypes.c_double()
        _check(lib.conv_split_compensation(self._h, _d(k), int(ell_cut), float(theta_cut), ctypes.byref(c)),
               "conv_split_compensation")
        return c.value

    def error(self, k_ell, ell_cut: int, theta_cut: float, alpha: float = 5.0):
        """(sigma_rms of Eq. 2, sigma of Eq. 6)."""
        k = _f64(k_ell, self.lmax + 1, "k_ell")
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib.conv_split_error(self._h, _d(k), int(ell_cut), float(theta_cut), float(alpha), ctypes.byref(a),
                                    ctypes.byref(b)), "conv_split_error")
        return a.value, b.value

    def search(self, k_ell, nside: int, bound: float, theta_grid, model: CostModel, alpha: float = 5.0,
               ell_step: int = 1):
        """Cheapest feasible (theta_cut, ell_cut, wall, sigma), or None."""
        k = _f64(k_ell, self.lmax + 1, "k_ell")
        g = _f64(theta_grid)
        th, lc, wl, sg = ctypes.c_double(), ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        code = lib.conv_split_search(self._h, _d(k), int(nside), float(bound), float(alpha), _d(g), len(g),
                                     int(ell_step), ctypes.byref(model._s), ctypes.byref(th), ctypes.byref(lc),
                                     ctypes.byref(wl), ctypes.byref(sg))
        if code == INFEASIBLE:
            return None
        _check(code, "conv_split_search")
        return th.value, lc.value, wl.value, sg.value

    def search_many(self, k_ells, nside: int, bounds, theta_grid, model: CostModel, alpha: float = 5.0,
                    ell_step: int = 1, nthreads: int = 0):
        """Arrays (theta_cut, ell_cut, wall, sigma) per kernel; theta_cut < 0 marks infeasible.
        theta_grid is one grid for all kernels or one row per kernel."""
        K = np.ascontiguousarray(k_ells, dtype=np.float64)
        if K.ndim != 2 or K.shape[1] != self.lmax + 1:
            raise ConvRealError(-1, "search_many", f"k_ells must be [n, {self.lmax + 1}]")
        n = K.shape[0]
        b = _f64(bounds, n, "bounds")
        g = np.asarray(theta_grid, dtype=np.float64)
        g = np.ascontiguousarray(np.broadcast_to(g, (n, g.shape[-1])) if g.ndim == 1 else g)
        if g.shape[0] != n:
            raise ConvRealError(-1, "search_many", "theta_grid must be [n_theta] or [n, n_theta]")
        th, wl, sg = np.empty(n), np.empty(n), np.empty(n)
        lc = np.empty(n, dtype=np.int32)
        _check(lib.conv_split_search_many(self._h, _d(K), n, int(nside), _d(b), float(alpha), _d(g), g.shape[1],
                                          int(ell_step), ctypes.byref(model._s), int(nthreads), _d(th),
                                          lc.ctypes.data_as(_iptr_t), _d(wl), _d(sg)), "conv_split_search_many")
        return th, lc, wl, sg
