"""Spherical-harmonic analysis, synthesis and harmonic convolution on the ring grid (oracle).

Test infrastructure (see the package docstring). The paper's split (Estimating Errors section,
Eq. 1; Fig. 1) applies the band-limited part of the kernel, K^_l for l <= l_cut, in harmonic space
by spherical-harmonic transforms, beside the real-space part. For a real map x on the pixel grid:

    analysis     a_lm = Omega * sum_p x_p conj(Y_lm(v_p))           (equal pixel weights Omega)
    synthesis    y_p  = sum_{l <= L} sum_{|m| <= l} b_lm Y_lm(v_p)
    convolution  y    = synthesis(k_l * analysis(x))                 (radial kernel k_l, l <= L)

with Y_lm(theta, phi) = lambda_lm(cos theta) exp(i m phi), the orthonormal spherical harmonics with
the Condon-Shortley phase. Real maps have a_{l,-m} = (-1)^m conj(a_lm), so only m >= 0 is kept, in
m-major order: index(l, m) = m (2L + 3 - m) / 2 + (l - m).

lambda_lm follows the textbook recurrence in l at fixed m:
    lambda_mm     = (-1)^m sqrt((2m + 1) / (4 pi) * prod_{k=1}^{m} (2k - 1) / (2k)) * sin^m theta
    lambda_m+1,m  = z sqrt(2m + 3) lambda_mm
    lambda_lm     = a_lm (z lambda_l-1,m - b_lm lambda_l-2,m),
                    a_lm = sqrt((4l^2 - 1) / (l^2 - m^2)),
                    b_lm = sqrt(((l - 1)^2 - m^2) / (4 (l - 1)^2 - 1)),
started from log(lambda_mm) with a power-of-two exponent carried beside the value, so that starting
values below the FP64 range (sin^m theta at large m) do not vanish before the recurrence grows them
back into range; values still below 2^-900 are taken as zero.

Ring sums are plain loops over the pixels of a ring (no FFT), FP64 throughout.
"""
from __future__ import annotations

import math

import numpy as np

from . import geometry

_SCALE = 2.0 ** 600
_LOG_SCALE = 600.0 * math.log(2.0)


def alm_size(L: int) -> int:
    return (L + 1) * (L + 2) // 2


def alm_index(L: int, ell: int, m: int) -> int:
    return m * (2 * L + 3 - m) // 2 + (ell - m)


def _log_lambda_mm(m: int, sin_theta: np.ndarray) -> np.ndarray:
    s = 0.5 * math.log((2 * m + 1) / (4.0 * math.pi))
    for k in range(1, m + 1):
        s += 0.5 * math.log((2 * k - 1) / (2.0 * k))
    with np.errstate(divide="ignore"):
        return s + m * np.log(sin_theta)


def lambda_lm(L: int, m: int, z: np.ndarray, sin_theta: np.ndarray = None) -> np.ndarray:
    """lambda_lm(z) for l = m..L (rows) at the points z (columns); sin_theta may be given exactly
    (else sqrt((1 - z)(1 + z)))."""
    z = np.asarray(z, dtype=np.float64)
    st = np.sqrt((1.0 - z) * (1.0 + z)) if sin_theta is None else np.asarray(sin_theta, dtype=np.float64)
    out = np.zeros((L - m + 1, z.size))
    lg = _log_lambda_mm(m, st)
    # value * SCALE^(-e): e >= 0 counts the factors 2^600 still to be taken out
    e = np.maximum(0, np.ceil((-650.0 - lg) / _LOG_SCALE)).astype(np.int64)
    sign = -1.0 if m % 2 else 1.0
    p0 = np.where(np.isfinite(lg), sign * np.exp(np.where(np.isfinite(lg), lg, 0.0) + e * _LOG_SCALE), 0.0)
    out[0] = np.where(e == 0, p0, 0.0)
    if L == m:
        return out
    p1 = z * math.sqrt(2 * m + 3) * p0
    out[1] = np.where(e == 0, p1, 0.0)
    for ell in range(m + 2, L + 1):
        a = math.sqrt((4.0 * ell * ell - 1.0) / (ell * ell - m * m))
        b = math.sqrt(((ell - 1.0) ** 2 - m * m) / (4.0 * (ell - 1.0) ** 2 - 1.0))
        p2 = a * (z * p1 - b * p0)
        big = (e > 0) & (np.abs(p2) > 2.0 ** 400)
        if np.any(big):
            p2 = np.where(big, p2 / _SCALE, p2)
            p1 = np.where(big, p1 / _SCALE, p1)
            e = e - big
        out[ell - m] = np.where(e == 0, p2, 0.0)
        p0, p1 = p1, p2
    return out


def _rings(nside: int):
    rt = geometry.ring_table(nside)
    return rt["z"], rt["sin"], rt["n"], rt["start"], rt["phi0"], rt["dphi"]


def analysis(nside: int, x, L: int) -> np.ndarray:
    """a_lm (complex, m-major, m >= 0) of a real map x [Npix] up to band limit L."""
    x = np.asarray(x, dtype=np.float64)
    z, st, n, start, phi0, dphi = _rings(nside)
    omega = geometry.pixel_area(nside)
    nr = len(z)
    G = np.zeros((L + 1, nr), dtype=np.complex128)       # G[m, ring] = sum_a x_a exp(-i m phi_a)
    ms = np.arange(L + 1)
    for r in range(nr):
        a = np.arange(n[r])
        phi = phi0[r] + a * dphi[r]
        xr = x[start[r]: start[r] + n[r]]
        G[:, r] = np.exp(-1j * np.outer(ms, phi)) @ xr
    alm = np.zeros(alm_size(L), dtype=np.complex128)
    for m in range(L + 1):
        lam = lambda_lm(L, m, z, st)                      # [L - m + 1, rings]
        i0 = alm_index(L, m, m)
        alm[i0: i0 + L - m + 1] = omega * (lam @ G[m])
    return alm


def synthesis(nside: int, alm: np.ndarray, L: int) -> np.ndarray:
    """Real map y [Npix] = sum_lm b_lm Y_lm (m < 0 from the reality condition)."""
    alm = np.asarray(alm, dtype=np.complex128)
    z, st, n, start, phi0, dphi = _rings(nside)
    nr = len(z)
    F = np.zeros((L + 1, nr), dtype=np.complex128)        # F[m, ring] = sum_l b_lm lambda_lm(z)
    for m in range(L + 1):
        lam = lambda_lm(L, m, z, st)
        i0 = alm_index(L, m, m)
        F[m] = alm[i0: i0 + L - m + 1] @ lam
    y = np.zeros(int(start[-1] + n[-1]))
    ms = np.arange(L + 1)
    for r in range(nr):
        a = np.arange(n[r])
        phi = phi0[r] + a * dphi[r]
        e = np.exp(1j * np.outer(phi, ms))                # [pixels, m]
        # y = F_0 + 2 Re sum_{m > 0} F_m exp(i m phi)  (F_0 is real for a real map)
        y[start[r]: start[r] + n[r]] = F[0, r].real + 2.0 * (e[:, 1:] @ F[1:, r]).real
    return y


def analysis_orders(nside: int, x, L: int, orders) -> dict:
    """a_lm for l = m..L of the listed orders m only ({m: array}): the sums of analysis() restricted
    to those orders, for checks on grids where the whole transform takes too long here."""
    x = np.asarray(x, dtype=np.float64)
    z, st, n, start, phi0, dphi = _rings(nside)
    omega = geometry.pixel_area(nside)
    ms = np.asarray(list(orders), dtype=np.int64)
    G = np.zeros((len(ms), len(z)), dtype=np.complex128)
    for r in range(len(z)):
        a = np.arange(n[r])
        phi = phi0[r] + a * dphi[r]
        G[:, r] = np.exp(-1j * np.outer(ms, phi)) @ x[start[r]: start[r] + n[r]]
    return {int(m): omega * (lambda_lm(L, int(m), z, st) @ G[i]) for i, m in enumerate(ms)}


def synthesis_rings(nside: int, alm: np.ndarray, L: int, rings) -> dict:
    """The pixels of the listed rings only ({ring: array}, 0-based ring index): the sums of
    synthesis() restricted to those rings."""
    alm = np.asarray(alm, dtype=np.complex128)
    z, st, n, start, phi0, dphi = _rings(nside)
    rs = np.asarray(list(rings), dtype=np.int64)
    F = np.zeros((L + 1, len(rs)), dtype=np.complex128)
    for m in range(L + 1):
        i0 = alm_index(L, m, m)
        F[m] = alm[i0: i0 + L - m + 1] @ lambda_lm(L, m, z[rs], st[rs])
    ms = np.arange(L + 1)
    out = {}
    for i, r in enumerate(rs):
        a = np.arange(n[r])
        phi = phi0[r] + a * dphi[r]
        e = np.exp(1j * np.outer(phi, ms))
        out[int(r)] = F[0, i].real + 2.0 * (e[:, 1:] @ F[1:, i]).real
    return out


def multiply(alm: np.ndarray, k_ell: np.ndarray, L: int) -> np.ndarray:
    """b_lm = k_l a_lm."""
    out = np.array(alm, dtype=np.complex128)
    for m in range(L + 1):
        i0 = alm_index(L, m, m)
        out[i0: i0 + L - m + 1] *= k_ell[m: L + 1]
    return out


def convolve(nside: int, x, k_ell: np.ndarray) -> np.ndarray:
    """Harmonic-space convolution of a real map with the radial kernel k_l, l <= L = len(k_ell) - 1."""
    L = len(k_ell) - 1
    return synthesis(nside, multiply(analysis(nside, x, L), np.asarray(k_ell, dtype=np.float64), L), L)


def power_spectrum(alm: np.ndarray, L: int) -> np.ndarray:
    """C_l = (|a_l0|^2 + 2 sum_{m > 0} |a_lm|^2) / (2l + 1)."""
    cl = np.zeros(L + 1)
    for m in range(L + 1):
        i0 = alm_index(L, m, m)
        p = np.abs(alm[i0: i0 + L - m + 1]) ** 2
        cl[m:] += p if m == 0 else 2.0 * p
    return cl / (2.0 * np.arange(L + 1) + 1.0)
