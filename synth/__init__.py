"""Seeded synthetic workloads for the real-space spherical convolution.

This module is shared by the tests, the benchmark and the CPU oracle's
checks. It holds random draws and workload definitions only: maps of
i.i.d. noise, Gaussian-random-field maps, and the harmonic coefficients of
the radial kernels the workloads use. It performs none of the convolution's
own arithmetic (pixel-pair geometry, kernel tabulation, interpolation,
summation); those live separately in the library and in the oracle.

Workloads follow the paper's setting (Results section): an equal-area
iso-latitude ring-ordered sphere pixelization (HEALPix), Gaussian beams
given by FWHM, kernels K_l = sqrt(C_l) B_l (Eq. 9) with a flat input
spectrum for noise maps. The WMAP 7-year spectrum the paper uses is not
available; a red spectrum C_l = 1/(l(l+1)) stands in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 14094441
ARCMIN = math.pi / (180.0 * 60.0)
DEG = math.pi / 180.0
FWHM_TO_SIGMA = 1.0 / math.sqrt(8.0 * math.log(2.0))


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for one named draw."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def npix_of(nside: int) -> int:
    return 12 * int(nside) * int(nside)


def white_noise(nside: int, nmaps: int = 1, seed: int = BASE_SEED,
                dtype=np.float64) -> np.ndarray:
    """i.i.d. N(0,1) pixel values, shape [nmaps, 12*nside^2]."""
    g = rng(seed)
    return g.standard_normal((int(nmaps), npix_of(nside))).astype(dtype)


def gaussian_beam(lmax: int, fwhm_rad: float) -> np.ndarray:
    """Gaussian beam transfer function B_l = exp(-l(l+1) sigma^2 / 2), l = 0..lmax."""
    sigma = fwhm_rad * FWHM_TO_SIGMA
    ell = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * ell * (ell + 1.0) * sigma * sigma)


def gaussian_beam_sigma(lmax: int, sigma_rad: float) -> np.ndarray:
    ell = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * ell * (ell + 1.0) * sigma_rad * sigma_rad)


def cosine_taper(lmax: int, ell_cut: float, width: float) -> np.ndarray:
    """Low-l window g_l: 1 below ell_cut - w/2, 0 above ell_cut + w/2, raised cosine between."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    lo = ell_cut - 0.5 * width
    hi = ell_cut + 0.5 * width
    g = np.where(ell <= lo, 1.0, 0.0)
    mid = (ell > lo) & (ell < hi)
    g[mid] = 0.5 * (1.0 + np.cos(math.pi * (ell[mid] - lo) / width))
    return g


def residual_beam(lmax: int, fwhm_rad: float, ell_cut: float, width: float) -> np.ndarray:
    """Harmonic coefficients of the part of a Gaussian beam left to real space once a
    cosine-tapered low-l part (up to ell_cut) is handed to harmonic space: B_l (1 - g_l)."""
    return gaussian_beam(lmax, fwhm_rad) * (1.0 - cosine_taper(lmax, ell_cut, width))


def red_spectrum(lmax: int, lmin: int = 2) -> np.ndarray:
    """C_l = 1/(l(l+1)) for lmin <= l <= lmax, zero below lmin."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    sel = ell >= max(lmin, 1)
    cl[sel] = 1.0 / (ell[sel] * (ell[sel] + 1.0))
    return cl


def draw_alm(cl: np.ndarray, seed: int) -> np.ndarray:
    """Random harmonic coefficients with power spectrum cl, packed m-major.

    Returns a complex array of length (lmax+1)(lmax+2)/2 holding a_lm for
    m = 0..lmax, l = m..lmax in that order. a_l0 ~ N(0, C_l) is real;
    for m > 0 the real and imaginary parts are each N(0, C_l / 2).
    """
    lmax = len(cl) - 1
    g = rng(seed)
    out = np.empty((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    pos = 0
    for m in range(lmax + 1):
        ells = np.arange(m, lmax + 1)
        sd = np.sqrt(cl[m:])
        if m == 0:
            out[pos:pos + len(ells)] = g.standard_normal(len(ells)) * sd
        else:
            re = g.standard_normal(len(ells))
            im = g.standard_normal(len(ells))
            out[pos:pos + len(ells)] = (re + 1j * im) * sd * math.sqrt(0.5)
        pos += len(ells)
    return out


@dataclass
class Workload:
    """One named workload: a map recipe and a radial kernel given by k_l."""
    name: str
    nside: int
    theta_cut: float            # radians
    lmax: int                   # band limit of the kernel series
    kernel: str                 # "gauss" or "residual"
    fwhm: float = 0.0           # radians (beam FWHM)
    sigma: float = 0.0          # radians (Gaussian sigma, cfg "gauss")
    ell_cut: float = 0.0
    taper_width: float = 0.0
    map_kind: str = "white"     # "white" | "red" | "red+noise"
    map_lmax: int = 0
    noise_frac: float = 0.0
    dtype: str = "f64"
    nmaps: int = 1
    n_tab: int = 2048
    seed: int = BASE_SEED
    extra: dict = field(default_factory=dict)

    def k_ell(self) -> np.ndarray:
        if self.kernel == "gauss":
            return gaussian_beam_sigma(self.lmax, self.sigma)
        if self.kernel == "residual":
            return residual_beam(self.lmax, self.fwhm, self.ell_cut, self.taper_width)
        raise ValueError(self.kernel)


def workload(name: str) -> Workload:
    """The named workloads: small parity case, medium and full-size single maps."""
    if name == "gauss32":
        sigma = 1.5 * DEG
        return Workload(name, nside=32, theta_cut=5.0 * sigma, lmax=512, kernel="gauss",
                        sigma=sigma, map_kind="white", dtype="f64", seed=BASE_SEED + 0)
    if name == "resid512":
        return Workload(name, nside=512, theta_cut=60.0 * ARCMIN, lmax=1536, kernel="residual",
                        fwhm=30.0 * ARCMIN, ell_cut=600.0, taper_width=100.0,
                        map_kind="red", map_lmax=1536, dtype="f32", seed=BASE_SEED + 1)
    if name == "resid2048":
        return Workload(name, nside=2048, theta_cut=30.0 * ARCMIN, lmax=4096, kernel="residual",
                        fwhm=5.0 * ARCMIN, ell_cut=1500.0, taper_width=100.0,
                        map_kind="red+noise", map_lmax=4096, noise_frac=0.01, dtype="f32",
                        seed=BASE_SEED + 2)
    raise KeyError(name)
