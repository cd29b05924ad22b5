"""Pixel centres of the ring-ordered equal-area iso-latitude pixelization (oracle).

The paper assumes HEALPix at Nside 2048 (Estimating Errors section, cost
models paragraph). Pixel centres follow the HEALPix ring scheme
(Gorski et al. 2005) in the ordering of the HEALPix library:

* north polar cap, rings i = 1..N-1: 4i pixels, z = 1 - i^2/(3N^2),
  phi_a = (pi / 2i)(a + 1/2), a = 0..4i-1;
* equatorial belt, rings i = N..3N: 4N pixels, z = 4/3 - 2i/(3N),
  phi_a = (pi / 2N)(a + s/2), s = (i - N + 1) mod 2;
* south polar cap, rings i = 3N+1..4N-1: mirror of ring k = 4N - i
  (z -> -z, same azimuths).

Pixels are numbered ring by ring from the north pole, increasing phi within
a ring. Everything is FP64.
"""
from __future__ import annotations

import math

import numpy as np


def ring_table(nside: int):
    """Per-ring arrays for rings i = 1..4N-1 (index i-1).

    Returns dict with:
      z        cos(theta) of the ring
      sin      sin(theta) of the ring, from (1-z)(1+z) formed without cancellation
      n        pixel count
      start    index of the ring's first pixel
      phi0     azimuth of pixel a = 0
      dphi     azimuth step 2 pi / n
    """
    N = int(nside)
    nr = 4 * N - 1
    z = np.empty(nr)
    sin = np.empty(nr)
    n = np.empty(nr, dtype=np.int64)
    start = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    pos = 0
    for i in range(1, 4 * N):
        if i < N or i > 3 * N:
            k = i if i < N else 4 * N - i          # ring counted from the nearer pole
            one_minus = k * k / (3.0 * N * N)       # 1 - |z|
            zz = 1.0 - one_minus
            s_theta = math.sqrt(one_minus * (2.0 - one_minus))
            cnt = 4 * k
            p0 = math.pi / (2.0 * k) * 0.5
            if i > 3 * N:
                zz = -zz
        else:
            zz = (2.0 * N - i) * 2.0 / (3.0 * N)       # = 4/3 - 2i/(3N), sign-symmetric
            one_minus = (2.0 * i - N) / (3.0 * N)   # 1 - z
            one_plus = (7.0 * N - 2.0 * i) / (3.0 * N)  # 1 + z
            s_theta = math.sqrt(one_minus * one_plus)
            cnt = 4 * N
            s = (i - N + 1) % 2
            p0 = math.pi / (2.0 * N) * (0.5 * s)
        z[i - 1] = zz
        sin[i - 1] = s_theta
        n[i - 1] = cnt
        start[i - 1] = pos
        phi0[i - 1] = p0
        pos += cnt
    assert pos == 12 * N * N
    return {"z": z, "sin": sin, "n": n, "start": start, "phi0": phi0,
            "dphi": 2.0 * math.pi / n.astype(np.float64)}


def pixel_angles(nside: int):
    """(z, sin_theta, phi, ring_index0) for every pixel in ring order."""
    rt = ring_table(nside)
    npix = 12 * int(nside) ** 2
    ring_of = np.repeat(np.arange(len(rt["n"])), rt["n"])
    a = np.arange(npix) - rt["start"][ring_of]
    phi = rt["phi0"][ring_of] + a * rt["dphi"][ring_of]
    return rt["z"][ring_of], rt["sin"][ring_of], phi, ring_of


def pixel_vectors(nside: int) -> np.ndarray:
    """Unit vectors of all pixel centres, shape [Npix, 3], ring order."""
    z, st, phi, _ = pixel_angles(nside)
    return np.stack([st * np.cos(phi), st * np.sin(phi), z], axis=1)


def pixel_area(nside: int) -> float:
    """Omega = 4 pi / Npix (all pixels have equal area)."""
    return 4.0 * math.pi / (12.0 * int(nside) ** 2)
