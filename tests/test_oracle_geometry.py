"""Pins of the oracle's pixel geometry against properties the pixelization fixes.

The pixelization is HEALPix in ring order (the paper's Nside-2048 setting,
Estimating Errors section). Checks: pixel counts, the equal-area property
(area above each ring centre equals the pixel count above it plus half the
ring), known base-pixel centres, mirror symmetry, centroid at the origin,
and the chord computed in extended precision.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import geometry


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 32, 64])
def test_pixel_counts(nside):
    rt = geometry.ring_table(nside)
    assert len(rt["n"]) == 4 * nside - 1
    assert int(rt["n"].sum()) == 12 * nside * nside
    assert np.all(np.diff(rt["start"]) == rt["n"][:-1])
    # polar caps: 4i pixels on ring i counted from the nearer pole; belt: 4N
    for i in range(1, 4 * nside):
        k = min(i, 4 * nside - i)
        assert rt["n"][i - 1] == 4 * min(k, nside)


@pytest.mark.parametrize("nside", [1, 2, 5, 16, 64])
def test_equal_area(nside):
    """Equal-area pixels: the cap above ring i's centre, of area 2 pi (1 - z_i), holds
    exactly the pixels of rings 1..i-1 plus half of ring i (in units of 4 pi / Npix)."""
    rt = geometry.ring_table(nside)
    npix = 12 * nside * nside
    above = 0
    for i in range(1, 4 * nside):
        n = int(rt["n"][i - 1])
        expect = above + n / 2.0
        got = npix * (1.0 - rt["z"][i - 1]) / 2.0
        assert abs(got - expect) <= 1e-9 * npix
        above += n


def test_base_pixels_nside1():
    """Nside 1: twelve base pixels; the library ordering puts pixel 4 at (z=0, phi=0)."""
    z, st, phi, _ = geometry.pixel_angles(1)
    for p in range(4):
        assert z[p] == pytest.approx(2.0 / 3.0, abs=1e-15)
        assert phi[p] == pytest.approx(math.pi / 4 + p * math.pi / 2, abs=1e-15)
        assert z[p + 8] == pytest.approx(-2.0 / 3.0, abs=1e-15)
        assert phi[p + 8] == pytest.approx(math.pi / 4 + p * math.pi / 2, abs=1e-15)
    for p in range(4, 8):
        assert z[p] == pytest.approx(0.0, abs=1e-15)
        assert phi[p] == pytest.approx((p - 4) * math.pi / 2, abs=1e-15)


def test_nside2_rings():
    """Nside 2: ring 1 has 4 pixels at z = 11/12; ring 2 (first belt ring) 8 pixels at z = 2/3 with
    half-step offset; ring 3 starts at phi = 0, z = 1/3."""
    z, st, phi, ring = geometry.pixel_angles(2)
    assert np.allclose(z[0:4], 11.0 / 12.0, atol=1e-15)
    assert np.allclose(phi[0:4], (np.arange(4) + 0.5) * math.pi / 2, atol=1e-15)
    assert np.allclose(z[4:12], 2.0 / 3.0, atol=1e-15)
    assert np.allclose(phi[4:12], (np.arange(8) + 0.5) * math.pi / 4, atol=1e-15)
    assert np.allclose(z[12:20], 1.0 / 3.0, atol=1e-15)
    assert np.allclose(phi[12:20], np.arange(8) * math.pi / 4, atol=1e-15)


@pytest.mark.parametrize("nside", [4, 7, 32])
def test_mirror_and_centroid(nside):
    rt = geometry.ring_table(nside)
    nr = len(rt["z"])
    for i in range(nr):
        assert rt["z"][nr - 1 - i] == -rt["z"][i]
        assert rt["phi0"][nr - 1 - i] == rt["phi0"][i]
        assert rt["n"][nr - 1 - i] == rt["n"][i]
    v = geometry.pixel_vectors(nside)
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
    assert np.allclose(v.sum(axis=0), 0.0, atol=1e-10)


def test_sin_theta_accurate():
    """sin(theta) near the poles from (1-z)(1+z) without cancellation (vs extended precision)."""
    nside = 2048
    rt = geometry.ring_table(nside)
    mpmath.mp.dps = 40
    for i in [1, 2, 3, 100, 2047, 2048, 2049, 4095]:
        if i < nside:
            zz = 1 - mpmath.mpf(i * i) / (3 * nside * nside)
        else:
            zz = mpmath.mpf(4) / 3 - mpmath.mpf(2 * i) / (3 * nside)
        ref = mpmath.sqrt(1 - zz * zz)
        assert abs(rt["sin"][i - 1] - float(ref)) <= 2e-16 * float(ref)


def test_chord_extended_precision():
    """The oracle's chord |v_p - v_q| for close pixels at Nside 2048 is accurate to ~1e-12 relative."""
    nside = 2048
    rt = geometry.ring_table(nside)
    mpmath.mp.dps = 40
    g = np.random.default_rng(7)
    for _ in range(200):
        i = int(g.integers(1, 4 * nside - 2))
        j = i + int(g.integers(-3, 4))
        j = min(max(j, 1), 4 * nside - 1)
        a = int(g.integers(0, rt["n"][i - 1]))
        b = (int(round(a * rt["n"][j - 1] / rt["n"][i - 1])) + int(g.integers(-3, 4))) % int(rt["n"][j - 1])
        pa = rt["phi0"][i - 1] + a * rt["dphi"][i - 1]
        pb = rt["phi0"][j - 1] + b * rt["dphi"][j - 1]
        va = np.array([rt["sin"][i - 1] * math.cos(pa), rt["sin"][i - 1] * math.sin(pa), rt["z"][i - 1]])
        vb = np.array([rt["sin"][j - 1] * math.cos(pb), rt["sin"][j - 1] * math.sin(pb), rt["z"][j - 1]])
        d = float(np.linalg.norm(va - vb))

        def mpv(ring, pix):
            n = int(rt["n"][ring - 1])
            nn = nside
            if ring < nn or ring > 3 * nn:
                k = ring if ring < nn else 4 * nn - ring
                zz = 1 - mpmath.mpf(k * k) / (3 * nn * nn)
                if ring > 3 * nn:
                    zz = -zz
                ph = mpmath.pi / (2 * k) * (pix + mpmath.mpf(1) / 2)
            else:
                zz = mpmath.mpf(4) / 3 - mpmath.mpf(2 * ring) / (3 * nn)
                s = (ring - nn + 1) % 2
                ph = mpmath.pi / (2 * nn) * (pix + mpmath.mpf(s) / 2)
            assert n > 0
            st = mpmath.sqrt(1 - zz * zz)
            return [st * mpmath.cos(ph), st * mpmath.sin(ph), zz]

        A = mpv(i, a)
        B = mpv(j, b)
        ref = mpmath.sqrt(sum((A[k] - B[k]) ** 2 for k in range(3)))
        if ref > 0:
            assert abs(d - float(ref)) <= 1e-12 * float(ref) + 1e-16
