"""Pins of the oracle's spherical-harmonic transforms (oracle/sht.py): the harmonic half of the
kernel split (Eq. 1; Fig. 1: the band-limited part applied by spherical-harmonic transforms).

* lambda_lm(cos theta) equals SciPy's Y_lm(theta, 0) (same normalisation and Condon-Shortley phase),
  also where lambda_mm is far below the FP64 range and the recurrence grows it back;
* synthesis equals the direct sum of SciPy's Y_lm at the pixel centres;
* analysis equals Omega * sum_p x_p conj(Y_lm) with SciPy's Y_lm;
* the harmonic convolution of a delta map equals Omega K(gamma), K the kernel's Legendre series at the
  true angle (addition theorem: sum_m Y_lm(p) conj(Y_lm(q)) = (2l+1)/(4 pi) P_l(cos gamma_pq)), i.e. the
  harmonic path applies the same operator as the real-space definition before truncation;
* the power spectrum of a_lm."""
import math

import numpy as np
import pytest
from scipy import special

import synth
from oracle import geometry, kernel, sht


def _Y(L, theta, phi):
    """[alm_size(L), points] of Y_lm (m >= 0) from SciPy."""
    out = np.zeros((sht.alm_size(L), len(theta)), dtype=np.complex128)
    for m in range(L + 1):
        for ell in range(m, L + 1):
            out[sht.alm_index(L, ell, m)] = special.sph_harm_y(ell, m, theta, phi)
    return out


def test_lambda_matches_scipy():
    g = np.random.default_rng(1)
    theta = g.uniform(0.01, math.pi - 0.01, 40)
    L = 60
    for m in (0, 1, 7, 30, 60):
        lam = sht.lambda_lm(L, m, np.cos(theta), np.sin(theta))
        for ell in range(m, L + 1):
            ref = special.sph_harm_y(ell, m, theta, 0.0).real
            assert np.allclose(lam[ell - m], ref, rtol=1e-11, atol=1e-13)


def test_lambda_from_below_the_fp64_range():
    # sin^m theta with m = 700 at theta = 0.35 rad is about 1e-325: lambda_mm underflows, yet lambda_lm
    # reaches order one by l = 2100; 50-digit mpmath (Ferrers function, Condon-Shortley phase, times
    # the orthonormalisation) gives the values
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    L, m, theta = 2200, 700, 0.35
    lam = sht.lambda_lm(L, m, np.array([math.cos(theta)]), np.array([math.sin(theta)]))
    th = mp.mpf(theta)
    for ell in (1900, 2000, 2100, 2200):
        p = mp.legenp(ell, m, mp.cos(th), type=2)
        ref = float(p * mp.sqrt((2 * ell + 1) / (4 * mp.pi) * mp.factorial(ell - m) / mp.factorial(ell + m)))
        assert lam[ell - m][0] == pytest.approx(ref, rel=1e-11, abs=1e-300), ell
    assert abs(lam[2100 - m][0]) > 0.5


@pytest.mark.parametrize("nside,L", [(2, 6), (4, 10), (8, 20)])
def test_synthesis_and_analysis_match_direct_sums(nside, L):
    z, st, phi, _ = geometry.pixel_angles(nside)
    theta = np.arctan2(st, z)
    Y = _Y(L, theta, phi)
    alm = synth.draw_alm(np.ones(L + 1), 100 + nside)
    # direct synthesis: sum over m >= 0 with the m < 0 terms from the reality condition
    w = np.ones(sht.alm_size(L))
    for ell in range(L + 1):
        w[sht.alm_index(L, ell, 0)] = 0.5
    direct = 2.0 * np.real((w * alm) @ Y)
    y = sht.synthesis(nside, alm, L)
    assert np.allclose(y, direct, rtol=1e-12, atol=1e-12 * np.max(np.abs(direct)))
    x = synth.white_noise(nside, 1, seed=nside)[0]
    a = sht.analysis(nside, x, L)
    ref = geometry.pixel_area(nside) * (np.conj(Y) @ x)
    assert np.allclose(a, ref, rtol=1e-11, atol=1e-12 * np.max(np.abs(ref)))


@pytest.mark.parametrize("nside,L", [(4, 10), (8, 20)])
def test_restricted_transforms_match_direct_sums(nside, L):
    # analysis_orders / synthesis_rings (the transforms restricted to a few orders or rings, for
    # checks on large grids) against the same direct sums over Y_lm
    z, st, phi, _ = geometry.pixel_angles(nside)
    Y = _Y(L, np.arctan2(st, z), phi)
    x = synth.white_noise(nside, 1, seed=3 * nside)[0]
    ref = geometry.pixel_area(nside) * (np.conj(Y) @ x)
    orders = [0, 1, L // 2, L]
    got = sht.analysis_orders(nside, x, L, orders)
    for m in orders:
        i0 = sht.alm_index(L, m, m)
        r = ref[i0: i0 + L - m + 1]
        assert np.allclose(got[m], r, rtol=1e-11, atol=1e-12 * np.max(np.abs(ref))), m
    alm = synth.draw_alm(np.ones(L + 1), 200 + nside)
    w = np.ones(sht.alm_size(L))
    for ell in range(L + 1):
        w[sht.alm_index(L, ell, 0)] = 0.5
    direct = 2.0 * np.real((w * alm) @ Y)
    rt = geometry.ring_table(nside)
    rings = [0, nside - 1, 2 * nside - 1, 4 * nside - 2]
    got_y = sht.synthesis_rings(nside, alm, L, rings)
    for r in rings:
        d = direct[rt["start"][r]: rt["start"][r] + rt["n"][r]]
        assert np.allclose(got_y[r], d, rtol=1e-12, atol=1e-12 * np.max(np.abs(direct))), r


@pytest.mark.parametrize("nside,L,q", [(4, 16, 5), (8, 24, 100), (16, 40, 1500)])
def test_convolution_of_a_delta_is_the_kernel_profile(nside, L, q):
    k_ell = synth.gaussian_beam_sigma(L, 0.3)
    x = np.zeros(12 * nside * nside)
    x[q] = 1.0
    y = sht.convolve(nside, x, k_ell)
    v = geometry.pixel_vectors(nside)
    d2 = np.sum((v - v[q]) ** 2, axis=1)                  # chord^2 = 2 (1 - cos gamma)
    ref = geometry.pixel_area(nside) * kernel.legendre_series_u(k_ell, 0.5 * d2)
    assert np.allclose(y, ref, rtol=1e-10, atol=1e-12 * np.max(np.abs(ref)))


def test_power_spectrum():
    L = 30
    c = 1.0 + np.arange(L + 1)
    alm = synth.draw_alm(c, 3)
    cl = sht.power_spectrum(alm, L)
    ell = 10
    ref = sum((abs(alm[sht.alm_index(L, ell, m)]) ** 2) * (1 if m == 0 else 2) for m in range(ell + 1)) / (2 * ell + 1)
    assert cl[ell] == pytest.approx(ref, rel=1e-14)
    big = synth.draw_alm(np.full(401, 2.0), 4)
    assert np.mean(sht.power_spectrum(big, 400)[200:]) == pytest.approx(2.0, rel=0.02)
