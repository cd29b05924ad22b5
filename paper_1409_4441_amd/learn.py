"""Learned split: ctypes binding of include/convlearn.h, and the predict / judge / fall back flow.

The network maps normalised (log2 Nside, ln FWHM, log10 target error) to normalised
(ln(theta_cut / sigma), l_cut / lmax), sigma = FWHM / sqrt(8 ln 2), for the kernels
K_l = sqrt(C_l) B_l (Gaussian beam B_l, C_l = 1/(l(l+1))) with lmax = 2 Nside, C^in = 1 and the
Eq. 6 error with alpha = 5. Labels are the split search's answers
(conv_split_search_many) under the measured cost model; training runs on the device with the
library's forward, back-propagation and Adam kernels. A prediction is judged by the error model
(conv_split_error); if it misses the bound, the split search decides instead.

    from paper_1409_4441_amd import learn
    net = learn.Network()                       # device buffers
    net.set_params(learn.init_params(seed))
    net.train(x, t, steps=3000)                 # x [n, 3], t [n, 2] cuda tensors
    pred = learn.Predictor.load()               # trained parameters + measured cost model
    theta_cut, ell_cut, source = pred.predict(nside, fwhm_arcmin, eps)
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np

from . import ConvRealError, _check, _stream_handle, lib
from . import split as _split

N_PARAMS = 4546
IN, HIDDEN, OUT = 3, 64, 2
# Eq. 6's alpha: the paper's 5, an upper bound for this library (the measured ratio of the split's
# power-spectrum error to Eq. 6 with alpha = 1 is 1.0-4.6 over the splits the search chooses)
ALPHA = 5.0
# largest compensation (max_{l <= l_cut} |(P x)_l| / max |K_l|) a split may need: the paper's fits
# adjust the harmonic kernel at the percent level; splits needing more are not trusted
MAX_COMP = 1e-2
# largest l_cut / lmax of a split with a real-space part: above it the measured errors exceed the
# error model's (the real-space part then carries only multipoles near the grid's resolution)
MAX_ELL_FRAC = 0.45
# network answers l_cut / lmax at or above this are taken as the all-harmonic split; answers in
# [UNCERTAIN_FRAC, ALL_HARMONIC_FRAC) are left to the search
ALL_HARMONIC_FRAC = 0.95
UNCERTAIN_FRAC = 0.45
ARCMIN = math.pi / (180.0 * 60.0)

# Ranges of the learned map: Nside 256..2048, FWHM 5'..30', target error 1e-6..1e-4.
NSIDES = (256, 512, 1024, 2048)
FWHM_RANGE = (5.0, 30.0)
EPS_RANGE = (1e-6, 1e-4)
# scan grid of theta_cut in units of the beam's sigma, and the l_cut resolution of the labels
THETA_SIGMAS = tuple(np.round(np.arange(2.0, 12.01, 0.5), 2))
ELL_STEP = 8

EXPORTS = ("conv_mlp_create", "conv_mlp_destroy", "conv_mlp_set_params", "conv_mlp_get_params",
           "conv_mlp_forward", "conv_mlp_gradient", "conv_mlp_train")

_c_int, _c_void_p = ctypes.c_int, ctypes.c_void_p
_fptr_t = ctypes.POINTER(ctypes.c_float)


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


def _bind():
    lib.conv_mlp_create.argtypes = [ctypes.POINTER(_c_void_p), _c_int]
    lib.conv_mlp_destroy.argtypes = [_c_void_p]
    lib.conv_mlp_set_params.argtypes = [_c_void_p, _fptr_t]
    lib.conv_mlp_get_params.argtypes = [_c_void_p, _fptr_t]
    lib.conv_mlp_forward.argtypes = [_c_void_p, _c_void_p, _c_int, _c_void_p, _c_void_p]
    lib.conv_mlp_gradient.argtypes = [_c_void_p, _c_void_p, _c_void_p, _c_int, _c_void_p, _c_void_p, _c_void_p]
    lib.conv_mlp_train.argtypes = [_c_void_p, _c_void_p, _c_void_p, _c_int, _c_int, ctypes.POINTER(Adam), _c_void_p,
                                   _c_void_p]
    for f in EXPORTS:
        getattr(lib, f).restype = _c_int


_bind()


def _tensor(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ConvRealError(-1, name, "expected a contiguous float32 cuda tensor")
    if tuple(t.shape) != tuple(shape):
        raise ConvRealError(-1, name, f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Network:
    """The 3-64-64-2 network on the current device; batches of up to max_batch samples."""

    def __init__(self, max_batch: int = 4096):
        h = _c_void_p()
        _check(lib.conv_mlp_create(ctypes.byref(h), int(max_batch)), "conv_mlp_create")
        self._h = h
        self.max_batch = int(max_batch)
        self.norm = None   # feature/target normalisation of a trained network

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and lib is not None:
            lib.conv_mlp_destroy(self._h)
            self._h = _c_void_p()

    def __del__(self):
        self.close()

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        if a.shape != (N_PARAMS,):
            raise ConvRealError(-1, "set_params", f"expected {N_PARAMS} parameters")
        _check(lib.conv_mlp_set_params(self._h, a.ctypes.data_as(_fptr_t)), "conv_mlp_set_params")

    def get_params(self) -> np.ndarray:
        a = np.empty(N_PARAMS, dtype=np.float32)
        _check(lib.conv_mlp_get_params(self._h, a.ctypes.data_as(_fptr_t)), "conv_mlp_get_params")
        return a

    def forward(self, x, out=None, stream=None):
        import torch
        n = x.shape[0]
        y = out if out is not None else torch.empty((n, OUT), dtype=torch.float32, device=x.device)
        _check(lib.conv_mlp_forward(self._h, _tensor(x, (n, IN), "x"), n, _tensor(y, (n, OUT), "y"),
                                    _stream_handle(stream)), "conv_mlp_forward")
        return y

    def gradient(self, x, t, stream=None):
        """(loss [1], grad [4546]) as cuda tensors."""
        import torch
        n = x.shape[0]
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib.conv_mlp_gradient(self._h, _tensor(x, (n, IN), "x"), _tensor(t, (n, OUT), "t"), n,
                                     ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
                                     _stream_handle(stream)), "conv_mlp_gradient")
        return loss, g

    def train(self, x, t, steps: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8, stream=None):
        """Full-batch Adam; returns the loss before each step (cuda tensor)."""
        import torch
        n = x.shape[0]
        hist = torch.empty(max(int(steps), 1), dtype=torch.float32, device=x.device)
        opt = Adam(float(lr), float(beta1), float(beta2), float(eps))
        _check(lib.conv_mlp_train(self._h, _tensor(x, (n, IN), "x"), _tensor(t, (n, OUT), "t"), n, int(steps),
                                  ctypes.byref(opt), ctypes.c_void_p(hist.data_ptr()), _stream_handle(stream)),
               "conv_mlp_train")
        return hist[:int(steps)]


# ---------------------------------------------------------------------------- data
def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases."""
    g = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((HIDDEN, IN), (HIDDEN, HIDDEN), (OUT, HIDDEN)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(g.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def sigma_of(fwhm_arcmin: float) -> float:
    return fwhm_arcmin * ARCMIN / math.sqrt(8.0 * math.log(2.0))


def beam(lmax: int, fwhm_arcmin: float) -> np.ndarray:
    """Gaussian beam b_l = exp(-l (l + 1) sigma^2 / 2)."""
    s = sigma_of(fwhm_arcmin)
    ell = np.arange(lmax + 1)
    return np.exp(-0.5 * ell * (ell + 1.0) * s * s)


def kernel_ell(lmax: int, fwhm_arcmin: float) -> np.ndarray:
    """The kernels of the paper's Results section, K_l = sqrt(C_l) B_l (simulating a map with
    spectrum C_l seen through a Gaussian beam, input C^in = 1), with C_l = 1/(l(l+1)) for l >= 2
    (0 below) standing in for the WMAP spectrum."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    c = np.zeros(lmax + 1)
    c[2:] = 1.0 / (ell[2:] * (ell[2:] + 1.0))
    return np.sqrt(c) * beam(lmax, fwhm_arcmin)


def features(nside, fwhm_arcmin, eps) -> np.ndarray:
    """Inputs scaled to [-1, 1] over the learned ranges."""
    nside, fwhm, eps = (np.asarray(v, dtype=np.float64) for v in (nside, fwhm_arcmin, eps))
    f0 = (np.log2(nside) - 9.5) / 1.5
    lo, hi = math.log(FWHM_RANGE[0]), math.log(FWHM_RANGE[1])
    f1 = 2.0 * (np.log(fwhm) - lo) / (hi - lo) - 1.0
    f2 = (np.log10(eps) + 5.0)
    return np.stack([f0, f1, f2], axis=-1)


def draw_triples(n: int, seed: int):
    """n seeded (Nside, FWHM arcmin, target error): Nside uniform over NSIDES, FWHM and error
    log-uniform over their ranges."""
    g = np.random.default_rng(seed)
    nside = g.choice(NSIDES, n)
    fwhm = np.exp(g.uniform(math.log(FWHM_RANGE[0]), math.log(FWHM_RANGE[1]), n))
    eps = 10.0 ** g.uniform(math.log10(EPS_RANGE[0]), math.log10(EPS_RANGE[1]), n)
    return nside, fwhm, eps


def eval_grid():
    """The evaluation grid of the learned split: Nside 2048, FWHM 5', 6', ..., 10', target errors
    1e-6, 1e-5, 1e-4 (18 triples)."""
    fw = np.repeat(np.arange(5.0, 10.01, 1.0), 3)
    ep = np.tile([1e-6, 1e-5, 1e-4], 6)
    return np.full(len(fw), 2048), fw, ep


def _contexts():
    """One split context per Nside (lmax = 2 Nside), wide enough for the largest scan angle."""
    theta_max = max(THETA_SIGMAS) * sigma_of(FWHM_RANGE[1]) * 1.0001
    return {ns: _split.Context(2 * ns, theta_max, max_comp=MAX_COMP, max_ell_frac=MAX_ELL_FRAC) for ns in NSIDES}


def scan(nside, fwhm, eps, model, ctxs=None, nthreads: int = 0):
    """The split search for each triple (scan grid THETA_SIGMAS x sigma, l_cut in steps of
    ELL_STEP): arrays (theta_cut, ell_cut, wall, sigma)."""
    nside, fwhm, eps = np.asarray(nside), np.asarray(fwhm, float), np.asarray(eps, float)
    own = ctxs is None
    ctxs = _contexts() if own else ctxs
    n = len(nside)
    th, lc, wl, sg = np.empty(n), np.empty(n, dtype=np.int64), np.empty(n), np.empty(n)
    try:
        for ns in np.unique(nside):
            idx = np.nonzero(nside == ns)[0]
            K = np.stack([kernel_ell(2 * int(ns), fwhm[k]) for k in idx])
            grids = np.stack([np.array(THETA_SIGMAS) * sigma_of(fwhm[k]) for k in idx])
            r = ctxs[int(ns)].search_many(K, int(ns), eps[idx], grids, model, alpha=ALPHA, ell_step=ELL_STEP,
                                          nthreads=nthreads)
            th[idx], lc[idx], wl[idx], sg[idx] = r
    finally:
        if own:
            for c in ctxs.values():
                c.close()
    return th, lc, wl, sg


def raw_targets(theta_cut, ell_cut, nside, fwhm) -> np.ndarray:
    """Split in the network's coordinates before standardisation: ln(theta_cut / sigma), l_cut / lmax."""
    sig = np.array([sigma_of(f) for f in np.atleast_1d(fwhm)])
    return np.stack([np.log(np.asarray(theta_cut, float) / sig),
                     np.asarray(ell_cut, float) / (2.0 * np.asarray(nside, float))], axis=-1)


def fit_norm(raw: np.ndarray) -> dict:
    """Per-output mean and spread of the training targets."""
    return {"mu": [float(v) for v in raw.mean(axis=0)], "sd": [float(max(v, 1e-6)) for v in raw.std(axis=0)]}


def encode(raw: np.ndarray, norm: dict) -> np.ndarray:
    return (raw - np.asarray(norm["mu"])) / np.asarray(norm["sd"])


def decode(y, nside, fwhm, norm: dict):
    """Split (theta_cut, ell_cut) from network outputs; l_cut rounded and clamped to [0, lmax]."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64)) * np.asarray(norm["sd"]) + np.asarray(norm["mu"])
    lmax = 2 * np.asarray(nside)
    # theta_cut within the scan's range (the labels' range): the network does not extrapolate beyond it
    lt = np.clip(y[:, 0], math.log(min(THETA_SIGMAS)), math.log(max(THETA_SIGMAS)))
    theta = np.exp(lt) * np.array([sigma_of(f) for f in np.atleast_1d(fwhm)])
    # the labels are binary in character: mostly a split with l_cut well below lmax, or all harmonic
    # (l_cut = lmax). An answer near lmax is read as the latter; one in between (UNCERTAIN_FRAC) lies
    # where the network interpolates across the feasibility edge and is marked -1 (the search decides)
    f = y[:, 1]
    frac = np.where(f >= ALL_HARMONIC_FRAC, 1.0, f)
    ell = np.clip(np.rint(frac * lmax), 0, lmax).astype(np.int64)
    ell = np.where((f >= UNCERTAIN_FRAC) & (f < ALL_HARMONIC_FRAC), -1, ell)
    return theta, ell


class Predictor:
    """A trained network with its normalisation, the cost model and one split context per Nside:
    predict() returns the network's split when the error model accepts it, else the search's."""

    def __init__(self, params, norm: dict, model):
        self.net = Network(max_batch=4096)
        self.net.set_params(params)
        self.norm = norm
        self.model = model
        self.ctxs = _contexts()

    @classmethod
    def load(cls, path: str = None, cost_path: str = None) -> "Predictor":
        params, meta = load(path or DEFAULT_MODEL)
        with open(cost_path or DEFAULT_COST) as f:
            c = json.load(f)
        return cls(params, meta["norm"], _split.CostModel.from_dict(c))

    def close(self):
        self.net.close()
        for c in self.ctxs.values():
            c.close()

    def network_split(self, nside, fwhm, eps):
        """The network's raw answer for arrays of triples: (theta_cut, ell_cut)."""
        import torch
        x = torch.tensor(features(nside, fwhm, eps), dtype=torch.float32, device="cuda")
        y = self.net.forward(x.contiguous()).cpu().numpy()
        return decode(y, nside, fwhm, self.norm)

    def judge(self, nside: int, fwhm: float, eps: float, theta_cut: float, ell_cut: int):
        """Eq. 6 error of a split and whether it is accepted: it meets eps, and it is all harmonic or
        has l_cut <= MAX_ELL_FRAC lmax and a compensation of at most MAX_COMP (the search's own
        conditions)."""
        if int(ell_cut) < 0:           # the network left this triple to the search
            return float("nan"), False
        ctx = self.ctxs[int(nside)]
        th = min(max(float(theta_cut), 1e-9), ctx.theta_max)
        K = kernel_ell(2 * int(nside), fwhm)
        _, sig = ctx.error(K, int(ell_cut), th, alpha=ALPHA)
        lmax = 2 * int(nside)
        ok = sig <= eps and (int(ell_cut) >= lmax or (int(ell_cut) <= MAX_ELL_FRAC * lmax and
                                                        ctx.compensation(K, int(ell_cut), th) <= MAX_COMP))
        return sig, ok

    def predict(self, nside: int, fwhm: float, eps: float):
        """(theta_cut, ell_cut, source), source "mlp" or "fallback"."""
        theta, ell = self.network_split([nside], [fwhm], [eps])
        th = min(max(float(theta[0]), 1e-9), self.ctxs[int(nside)].theta_max)
        _, ok = self.judge(nside, fwhm, eps, th, int(ell[0]))
        if ok:
            return th, int(ell[0]), "mlp"
        r = scan([nside], [fwhm], [eps], self.model, ctxs=self.ctxs, nthreads=1)
        return float(r[0][0]), int(r[1][0]), "fallback"


def save(path: str, params: np.ndarray, meta: dict):
    with open(path, "w") as f:
        json.dump({"params": [float(v) for v in params], **meta}, f)


def load(path: str):
    with open(path) as f:
        d = json.load(f)
    return np.asarray(d.pop("params"), dtype=np.float32), d


DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_split.json")
DEFAULT_COST = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_model.json")
