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


_SHT_LIB = None
_HERE = __import__("os").path.dirname(__import__("os").path.abspath(__file__))
SHT_SO = __import__("os").path.join(_HERE, "_sht_synth.so")


def build_sht(verbose: bool = False) -> str:
    """Compile the ring synthesis helper (plain C, OpenMP) next to this file."""
    import subprocess
    src = __import__("os").path.join(_HERE, "sht_synth.c")
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-o", SHT_SO + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    __import__("os").replace(SHT_SO + ".tmp", SHT_SO)
    return SHT_SO


def _sht():
    global _SHT_LIB
    if _SHT_LIB is None:
        import ctypes
        import os
        if not os.path.exists(SHT_SO):
            build_sht()
        lib = ctypes.CDLL(SHT_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.synth_ring_pairs.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, dp, dp]
        lib.synth_ring_pairs.restype = None
        _SHT_LIB = lib
    return _SHT_LIB


def _ring_layout(nside: int):
    """Where the pixels of the ring-ordered equal-area grid sit (needed to place a field on them):
    per ring z, sin(theta), azimuth of its first pixel, pixel count, first pixel index."""
    N = int(nside)
    rings = []
    z = np.empty(4 * N - 1)
    st = np.empty(4 * N - 1)
    start = 0
    for i in range(1, 4 * N):
        k = min(i, 4 * N - i)                    # rings counted from the nearer pole
        if k < N:                                # polar cap: 4k pixels, half-step offset
            n = 4 * k
            om = k * k / (3.0 * N * N)           # 1 - |z|
            zabs = 1.0 - om
            s = math.sqrt(om * (2.0 - om))
            phi0 = math.pi / (4.0 * k)
        else:                                    # belt: 4N pixels, offset alternating by ring
            n = 4 * N
            zabs = abs(2.0 * N - i) * 2.0 / (3.0 * N)
            s = math.sqrt((1.0 - zabs) * (1.0 + zabs))
            phi0 = math.pi * ((i - N + 1) % 2) / (4.0 * N)
        z[i - 1] = zabs if i <= 2 * N else -zabs
        st[i - 1] = s
        rings.append((n, start, phi0))
        start += n
    return z, st, rings


def synthesize(nside: int, alm: np.ndarray, lmax: int) -> np.ndarray:
    """Real map sum_lm a_lm Y_lm on the ring grid from m-major packed a_lm (m >= 0)."""
    import ctypes
    N = int(nside)
    z, st, rings = _ring_layout(N)
    nr = 4 * N - 1
    npix = 12 * N * N
    out = np.empty(npix)
    re = np.ascontiguousarray(alm.real)
    im = np.ascontiguousarray(alm.imag)
    dp = ctypes.POINTER(ctypes.c_double)
    lib = _sht()
    north = list(range(0, 2 * N))              # rings 1..2N (equator last)
    m = np.arange(lmax + 1)
    cm = np.where(m == 0, 1.0, 2.0)
    block = 256
    for b0 in range(0, len(north), block):
        idx = north[b0:b0 + block]
        zn = np.ascontiguousarray(z[idx])
        sn = np.ascontiguousarray(st[idx])
        fn = np.zeros((len(idx), lmax + 1, 2))
        fs = np.zeros((len(idx), lmax + 1, 2))
        lib.synth_ring_pairs(lmax, re.ctypes.data_as(dp), im.ctypes.data_as(dp), len(idx),
                             zn.ctypes.data_as(dp), sn.ctypes.data_as(dp),
                             fn.ctypes.data_as(dp), fs.ctypes.data_as(dp))
        for t, r in enumerate(idx):
            todo = [(r, fn[t])]
            if nr - 1 - r != r:                  # the equator ring is its own mirror
                todo.append((nr - 1 - r, fs[t]))
            for rr, F in todo:
                n, s0, phi0 = rings[rr]
                c = (F[:, 0] + 1j * F[:, 1]) * cm * np.exp(1j * m * phi0)
                G = np.bincount(m % n, weights=c.real, minlength=n) + \
                    1j * np.bincount(m % n, weights=c.imag, minlength=n)
                out[s0:s0 + n] = np.real(np.fft.ifft(G)) * n
    return out


def grf_map(nside: int, cl: np.ndarray, seed: int) -> np.ndarray:
    """Gaussian random field with power spectrum cl on the ring grid (FP64)."""
    lmax = len(cl) - 1
    return synthesize(nside, draw_alm(cl, seed), lmax)


def workload_maps(w, nmaps: int = 1) -> np.ndarray:
    """The maps of a named workload, [nmaps, Npix], in the workload's map dtype."""
    dt = np.float64 if w.dtype == "f64" else np.float32
    if w.map_kind == "white":
        return white_noise(w.nside, nmaps, seed=w.seed, dtype=dt)
    maps = []
    for k in range(nmaps):
        f = grf_map(w.nside, red_spectrum(w.map_lmax), w.seed + 1000 * k)
        if w.map_kind == "red+noise":
            g = rng(w.seed + 1000 * k + 1)
            f = f + w.noise_frac * float(np.std(f)) * g.standard_normal(f.size)
        maps.append(f)
    return np.stack(maps).astype(dt)


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


def batch_workload(nmaps: int = 32, seed: int = BASE_SEED + 3):
    """The batched workload: nmaps maps of uneven size and beam, drawn from one PCG64 stream.

    Per map k: Nside uniform over {256, 512, 1024, 2048}, FWHM uniform in [5', 30'],
    sigma = FWHM / sqrt(8 ln 2), theta_cut = 6 sigma, l_cut = 0.3 / sigma (radians), taper width
    round(l_cut / 6), kernel band limit 2 Nside; even k white N(0, 1) maps, odd k red fields
    C_l = 1/(l(l+1)) to l = 2 Nside. Returns a list of Workload records (FP32 maps)."""
    g = rng(seed)
    nsides = g.choice([256, 512, 1024, 2048], nmaps)
    fwhms = g.uniform(5.0, 30.0, nmaps) * ARCMIN
    out = []
    for k in range(nmaps):
        ns, fwhm = int(nsides[k]), float(fwhms[k])
        sigma = fwhm / np.sqrt(8.0 * np.log(2.0))
        lc = 0.3 / sigma
        out.append(Workload(f"batch{k}", nside=ns, theta_cut=6.0 * sigma, lmax=2 * ns, kernel="residual",
                            fwhm=fwhm, ell_cut=lc, taper_width=float(round(lc / 6.0)),
                            map_kind="white" if k % 2 == 0 else "red", map_lmax=2 * ns, dtype="f32",
                            seed=seed + 1 + k))
    return out


def batch_maps(ws, shared_red: bool = True):
    """Maps of a batched workload. With shared_red, the red maps of one Nside share a single field
    (the seed of the first such map), which keeps the host synthesis to one field per Nside; the
    convolution's cost does not depend on the values."""
    red = {}
    maps = []
    for w in ws:
        if w.map_kind == "white":
            maps.append(white_noise(w.nside, 1, seed=w.seed, dtype=np.float32)[0])
            continue
        if not shared_red or w.nside not in red:
            red[w.nside] = grf_map(w.nside, red_spectrum(w.map_lmax), w.seed).astype(np.float32)
        maps.append(red[w.nside])
    return maps
