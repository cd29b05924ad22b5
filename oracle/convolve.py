"""Plain-definition sums of the truncated real-space convolution (oracle).

    y_p = Omega * sum_{q : d_pq <= d_cut} Ktilde(d_pq) * x_q

(the real-space half of the split kernel of Eq. 1, applied to a pixelized map;
Omega = 4 pi / Npix). Pairs with d exactly equal to d_cut are included; a cut of
theta_cut = pi keeps every pair (no chord exceeds 2, so ties at d = 2 are inside).
The chord is |v_p - v_q| from the pixel-centre unit vectors, component by
component (no 1 - v.v form).

Two ways of visiting pairs, neither using any window logic:
  * brute force: every (p, q) pair of the map, in row chunks (small Nside);
  * ring-exhaustive: for one output pixel p, every pixel of every ring whose
    z differs from z_p by at most d_cut (a necessary condition, since
    |z_p - z_q| <= |v_p - v_q|), then the exact chord test.
"""
from __future__ import annotations

import numpy as np

from . import geometry, kernel


def _pair_limit(theta_cut: float) -> float:
    """Largest chord kept: d_cut, or no limit for a cut of pi."""
    return np.inf if theta_cut >= np.pi else kernel.chord_cut(theta_cut)


def _as_maps(x):
    x = np.asarray(x)
    single = x.ndim == 1
    x2 = x.reshape(1, -1) if single else x
    return x2.astype(np.float64), single


def convolve_bruteforce(nside: int, table: np.ndarray, theta_cut: float, x,
                        chunk: int = 0) -> np.ndarray:
    """All pixels of all maps by visiting every pixel pair. x: [Npix] or [nmaps, Npix]."""
    xm, single = _as_maps(x)
    v = geometry.pixel_vectors(nside)
    npix = v.shape[0]
    assert xm.shape[1] == npix
    omega = geometry.pixel_area(nside)
    dcut = _pair_limit(theta_cut)
    h = kernel.node_spacing(theta_cut, len(table))
    if chunk <= 0:
        chunk = max(1, int(2.0e6 // npix))
    y = np.zeros_like(xm)
    for p0 in range(0, npix, chunk):
        p1 = min(npix, p0 + chunk)
        diff = v[p0:p1, None, :] - v[None, :, :]
        d = np.sqrt((diff * diff).sum(axis=2))
        rows, cols = np.nonzero(d <= dcut)
        kt = kernel.interpolate(table, h, d[rows, cols])
        for m in range(xm.shape[0]):
            contrib = kt * xm[m, cols]
            y[m, p0:p1] += np.bincount(rows, weights=contrib, minlength=p1 - p0)
    y *= omega
    return y[0] if single else y


def _candidate_range(rt, dcut, z_p):
    """Pixel index range [lo, hi) covering all rings with |z_j - z_p| <= d_cut."""
    sel = np.nonzero(np.abs(rt["z"] - z_p) <= dcut)[0]
    r0, r1 = sel[0], sel[-1]
    return int(rt["start"][r0]), int(rt["start"][r1] + rt["n"][r1])


def convolve_sampled(nside: int, table: np.ndarray, theta_cut: float, x,
                     pix: np.ndarray) -> np.ndarray:
    """y at the listed output pixels only (ring-exhaustive candidates). Returns [nmaps, len(pix)]
    (or [len(pix)] for a single map)."""
    xm, single = _as_maps(x)
    pix = np.asarray(pix, dtype=np.int64)
    rt = geometry.ring_table(nside)
    z, st, phi, _ = geometry.pixel_angles(nside)
    omega = geometry.pixel_area(nside)
    dcut = _pair_limit(theta_cut)
    h = kernel.node_spacing(theta_cut, len(table))
    out = np.zeros((xm.shape[0], len(pix)))
    cache = {}
    for idx, p in enumerate(pix):
        lo, hi = cache.get(z[p], (None, None))
        if lo is None:
            lo, hi = _candidate_range(rt, dcut, z[p])
            cache[z[p]] = (lo, hi)
        vx = st[lo:hi] * np.cos(phi[lo:hi]) - st[p] * np.cos(phi[p])
        vy = st[lo:hi] * np.sin(phi[lo:hi]) - st[p] * np.sin(phi[p])
        vz = z[lo:hi] - z[p]
        d = np.sqrt(vx * vx + vy * vy + vz * vz)
        sel = np.nonzero(d <= dcut)[0]
        kt = kernel.interpolate(table, h, d[sel])
        out[:, idx] = omega * (xm[:, lo + sel] @ kt)
    return out[0] if single else out


def pair_counts_sampled(nside: int, theta_cut: float, pix: np.ndarray):
    """Per-pixel neighbour counts |{q : d_pq <= d_cut}| and the smallest relative
    distance of any candidate chord from d_cut, at the listed pixels."""
    pix = np.asarray(pix, dtype=np.int64)
    rt = geometry.ring_table(nside)
    z, st, phi, _ = geometry.pixel_angles(nside)
    dcut = _pair_limit(theta_cut)
    dref = kernel.chord_cut(theta_cut)
    counts = np.zeros(len(pix), dtype=np.int64)
    margin = np.inf
    for idx, p in enumerate(pix):
        lo, hi = _candidate_range(rt, dcut, z[p])
        vx = st[lo:hi] * np.cos(phi[lo:hi]) - st[p] * np.cos(phi[p])
        vy = st[lo:hi] * np.sin(phi[lo:hi]) - st[p] * np.sin(phi[p])
        vz = z[lo:hi] - z[p]
        d = np.sqrt(vx * vx + vy * vy + vz * vz)
        counts[idx] = int(np.count_nonzero(d <= dcut))
        if np.isfinite(dcut):
            margin = min(margin, float(np.min(np.abs(d - dcut))) / dref)
    return counts, margin


def pair_count_total(nside: int, theta_cut: float) -> int:
    """Exact number of ordered pixel pairs with d <= d_cut over the whole map."""
    npix = 12 * int(nside) ** 2
    counts, _ = pair_counts_sampled(nside, theta_cut, np.arange(npix))
    return int(counts.sum())


def rel_rms(y, y_ref) -> float:
    """sqrt(sum (y - y_ref)^2 / sum y_ref^2)."""
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    return float(np.sqrt(np.sum((y - y_ref) ** 2) / np.sum(y_ref ** 2)))
