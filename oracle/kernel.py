"""Radial kernel: Legendre-series tabulation on chord nodes and interpolation (oracle).

A radially symmetric kernel with harmonic coefficients k_l has the real-space
profile (Estimating Errors section: the Legendre transformation operator of
Eq. 1 links the l-space and real-space representations)

    K(theta) = sum_{l=0}^{lmax} (2l+1)/(4 pi) k_l P_l(cos theta).

The real-space convolver evaluates K from an interpolation table (Results
section, discussion of Fig. 4). Here the table is uniform in chord
d = 2 sin(theta/2): node k sits at d_k = k h with h = d_cut / (n_tab - 3), so
the two last nodes lie beyond d_cut and every d <= d_cut is interpolated from
a centred 4-node stencil. Since 1 - cos(theta) = d^2 / 2, the series is summed
with the Bonnet recurrence rewritten in u = 1 - x (x = cos theta) so that no
1 - x cancellation occurs near theta = 0:

    D_{l+1} = (l D_l - (2l+1) u P_l) / (l+1),  P_{l+1} = P_l + D_{l+1},

where D_l = P_l - P_{l-1}. (This is the textbook three-term recurrence
(l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1} with x = 1 - u substituted.)
"""
from __future__ import annotations

import math

import numpy as np


def chord_cut(theta_cut: float) -> float:
    return 2.0 * math.sin(0.5 * theta_cut)


def node_spacing(theta_cut: float, n_tab: int) -> float:
    if n_tab < 4:
        raise ValueError("n_tab must be >= 4")
    return chord_cut(theta_cut) / (n_tab - 3)


def legendre_series_u(k_ell: np.ndarray, u: np.ndarray) -> np.ndarray:
    """K at 1 - cos(theta) = u: sum_l (2l+1)/(4 pi) k_l P_l(1 - u), FP64."""
    u = np.asarray(u, dtype=np.float64)
    k_ell = np.asarray(k_ell, dtype=np.float64)
    p = np.ones_like(u)          # P_0
    dd = np.zeros_like(u)        # D_0 (unused: multiplied by l = 0)
    acc = (1.0 / (4.0 * math.pi)) * k_ell[0] * p
    for ell in range(0, len(k_ell) - 1):
        dd = (ell * dd - (2 * ell + 1) * u * p) / (ell + 1)
        p = p + dd
        acc = acc + ((2 * ell + 3) / (4.0 * math.pi)) * k_ell[ell + 1] * p
    return acc


def tabulate(k_ell: np.ndarray, theta_cut: float, n_tab: int) -> np.ndarray:
    """Table T[k] = K(d_k), d_k = k h, k = 0..n_tab-1 (chord nodes past 2 map to theta = pi)."""
    h = node_spacing(theta_cut, n_tab)
    d = np.arange(n_tab, dtype=np.float64) * h
    u = np.minimum(0.5 * d * d, 2.0)
    return legendre_series_u(k_ell, u)


def tabulate_function(fn_theta, theta_cut: float, n_tab: int) -> np.ndarray:
    """Table of an explicit profile K(theta) on the same chord nodes."""
    h = node_spacing(theta_cut, n_tab)
    d = np.minimum(np.arange(n_tab, dtype=np.float64) * h, 2.0)
    theta = 2.0 * np.arcsin(0.5 * d)
    return fn_theta(theta)


def interpolate(table: np.ndarray, h: float, d: np.ndarray) -> np.ndarray:
    """4-point Lagrange interpolation on the uniform chord grid.

    Segment k = floor(d / h), clamped to [0, n_tab - 3], uses nodes
    k-1, k, k+1, k+2 with local coordinate f = d/h - k. The node at k = -1
    is the ghost T[-1] := T[1], because K is an even function of d.
    """
    table = np.asarray(table, dtype=np.float64)
    n = len(table)
    t = np.asarray(d, dtype=np.float64) / h
    k = np.clip(np.floor(t).astype(np.int64), 0, n - 3)
    f = t - k
    km1 = np.where(k - 1 < 0, 1, k - 1)
    t_m1 = table[km1]
    t_0 = table[k]
    t_1 = table[k + 1]
    t_2 = table[k + 2]
    w_m1 = -f * (f - 1.0) * (f - 2.0) / 6.0
    w_0 = (f + 1.0) * (f - 1.0) * (f - 2.0) / 2.0
    w_1 = -(f + 1.0) * f * (f - 2.0) / 2.0
    w_2 = (f + 1.0) * f * (f - 1.0) / 6.0
    return w_m1 * t_m1 + w_0 * t_0 + w_1 * t_1 + w_2 * t_2


def legendre_p(ell_max: int, x: np.ndarray) -> np.ndarray:
    """P_0..P_ellmax at x (rows), plain three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((ell_max + 1,) + x.shape)
    out[0] = 1.0
    if ell_max >= 1:
        out[1] = x
    for ell in range(1, ell_max):
        out[ell + 1] = ((2 * ell + 1) * x * out[ell] - ell * out[ell - 1]) / (ell + 1)
    return out


def truncated_transfer(table: np.ndarray, theta_cut: float, ell_max: int,
                       points_per_segment: int = 8) -> np.ndarray:
    """k_l^trunc = 2 pi * int_{cos theta_cut}^{1} Ktilde(d(x)) P_l(x) dx, l = 0..ell_max.

    The harmonic response of the truncated, interpolated kernel: with the
    pixel area factor inside the operator, a spherical-harmonic input of
    degree l comes out multiplied by this number (up to the pixel-centre
    quadrature error). Integrated in d (x = 1 - d^2/2, dx = -d dd), segment by
    segment of the table so that the piecewise-cubic Ktilde is integrated by a
    Gauss-Legendre rule of ample order on each piece.
    """
    n = len(table)
    h = node_spacing(theta_cut, n)
    dcut = chord_cut(theta_cut)
    g, w = np.polynomial.legendre.leggauss(points_per_segment)
    nseg = int(math.ceil(dcut / h - 1e-12))
    lo = np.arange(nseg) * h
    hi = np.minimum(lo + h, dcut)
    mid = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    d = (mid[:, None] + half[:, None] * g[None, :]).ravel()
    wd = (half[:, None] * w[None, :]).ravel()
    kt = interpolate(table, h, d)
    x = 1.0 - 0.5 * d * d
    pl = legendre_p(ell_max, x)
    return 2.0 * math.pi * (pl * (kt * d * wd)[None, :]).sum(axis=1)
