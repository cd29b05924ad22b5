"""Pins of the oracle's truncated real-space sum against what the mathematics fixes.

* Two independent ways of visiting pairs (all pairs; ring-exhaustive per pixel) agree.
* Point spread: a delta input returns Omega * Ktilde(d_pq).
* The operator is symmetric (d_pq = d_qp) and commutes with the pixelization's
  quarter-turn and north/south mirror.
* Harmonic response: a constant map and P_l(n . n0) inputs come out multiplied by
  k_l^trunc, the truncated kernel's transfer function (eigenfunctions of a radial
  convolution), up to the pixel-centre quadrature error; tolerances from the
  measured floor at these resolutions.
* Special cases: a cut below the smallest pixel separation keeps only q = p;
  a cut of pi keeps every pair.
"""
import math

import numpy as np
import pytest

import synth
from oracle import convolve, geometry, kernel


def _gauss_table(nside, sigma_deg=1.5, cut_sigma=5.0, n_tab=2048):
    sigma = sigma_deg * math.pi / 180
    tc = cut_sigma * sigma
    k_ell = synth.gaussian_beam_sigma(512, sigma)
    return kernel.tabulate(k_ell, tc, n_tab), tc


@pytest.mark.parametrize("nside", [4, 8, 16])
def test_bruteforce_equals_ring_exhaustive(nside):
    T, tc = _gauss_table(nside, sigma_deg=6.0, cut_sigma=4.0)
    x = synth.white_noise(nside, 2, seed=11)
    yb = convolve.convolve_bruteforce(nside, T, tc, x)
    ys = convolve.convolve_sampled(nside, T, tc, x, np.arange(12 * nside * nside))
    assert np.max(np.abs(yb - ys)) <= 1e-14 * np.max(np.abs(yb))


def test_point_spread():
    nside = 8
    T, tc = _gauss_table(nside, sigma_deg=7.0, cut_sigma=4.0)
    npix = 12 * nside * nside
    q = 123
    x = np.zeros(npix)
    x[q] = 1.0
    y = convolve.convolve_bruteforce(nside, T, tc, x)
    v = geometry.pixel_vectors(nside)
    d = np.linalg.norm(v - v[q], axis=1)
    h = kernel.node_spacing(tc, len(T))
    ref = np.where(d <= kernel.chord_cut(tc), geometry.pixel_area(nside) * kernel.interpolate(T, h, d), 0.0)
    assert np.max(np.abs(y - ref)) <= 1e-14 * np.max(np.abs(ref))
    assert y[q] == pytest.approx(geometry.pixel_area(nside) * T[0], rel=1e-14)


def test_symmetry_and_equivariance():
    nside = 16
    T, tc = _gauss_table(nside, sigma_deg=3.0, cut_sigma=5.0)
    g = np.random.default_rng(2)
    npix = 12 * nside * nside
    u = g.standard_normal(npix)
    x = g.standard_normal(npix)
    Au, Ax = convolve.convolve_sampled(nside, T, tc, np.stack([u, x]), np.arange(npix))
    assert abs(u @ Ax - Au @ x) <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(Ax)
    rt = geometry.ring_table(nside)
    # quarter turn: pixel a of every ring -> a + n/4
    rot = np.empty(npix, dtype=np.int64)
    mir = np.empty(npix, dtype=np.int64)
    nr = len(rt["n"])
    for r in range(nr):
        s, n = int(rt["start"][r]), int(rt["n"][r])
        rot[s:s + n] = s + (np.arange(n) + n // 4) % n
        sm = int(rt["start"][nr - 1 - r])
        mir[s:s + n] = sm + np.arange(n)
    Axr = convolve.convolve_sampled(nside, T, tc, x[rot], np.arange(npix))
    assert np.max(np.abs(Axr - Ax[rot])) <= 1e-14 * np.max(np.abs(Ax))
    Axm = convolve.convolve_sampled(nside, T, tc, x[mir], np.arange(npix))
    assert np.max(np.abs(Axm - Ax[mir])) <= 1e-14 * np.max(np.abs(Ax))


@pytest.mark.parametrize("nside,ells,tol", [(32, [0, 10, 30], 5e-3), (64, [0, 10, 30], 1.5e-3)])
def test_harmonic_response(nside, ells, tol):
    """x = P_l(n . n0) for an oblique axis n0 is an eigenfunction: y = k_l^trunc x."""
    T, tc = _gauss_table(nside)
    kt = kernel.truncated_transfer(T, tc, max(ells))
    v = geometry.pixel_vectors(nside)
    n0 = np.array([0.3, -0.5, 0.81])
    n0 /= np.linalg.norm(n0)
    npix = v.shape[0]
    pix = np.arange(npix) if nside <= 32 else np.random.default_rng(1).choice(npix, 4000, replace=False)
    for ell in ells:
        x = kernel.legendre_p(ell, v @ n0)[ell]
        y = convolve.convolve_sampled(nside, T, tc, x, pix)
        err = convolve.rel_rms(y, kt[ell] * x[pix])
        assert err <= tol, (ell, err)


def test_harmonic_response_sectoral():
    """Re (x + i y)^l is a degree-l harmonic (proportional to Re Y_ll)."""
    nside = 32
    T, tc = _gauss_table(nside)
    ell = 12
    kt = kernel.truncated_transfer(T, tc, ell)
    v = geometry.pixel_vectors(nside)
    x = np.real((v[:, 0] + 1j * v[:, 1]) ** ell)
    y = convolve.convolve_sampled(nside, T, tc, x, np.arange(v.shape[0]))
    assert convolve.rel_rms(y, kt[ell] * x) <= 5e-3


def test_cut_below_pixel_spacing_keeps_self():
    nside = 16
    tc = 1e-3                       # far below the ~3.7 deg pixel spacing
    T = np.linspace(2.0, 1.0, 16)
    counts, margin = convolve.pair_counts_sampled(nside, tc, np.arange(12 * nside * nside))
    assert np.all(counts == 1)
    x = synth.white_noise(nside, 1, seed=4)[0]
    y = convolve.convolve_sampled(nside, T, tc, x, np.arange(len(x)))
    assert np.allclose(y, geometry.pixel_area(nside) * T[0] * x, rtol=1e-15, atol=0)


def test_cut_pi_keeps_all_pairs():
    nside = 4
    npix = 12 * nside * nside
    counts, _ = convolve.pair_counts_sampled(nside, math.pi, np.arange(npix))
    assert np.all(counts == npix)
    assert convolve.pair_count_total(nside, math.pi) == npix * npix


def test_pair_count_symmetric_total():
    """Counting from the other side of each pair gives the same total: sum_p n_p = sum_q n_q, and
    the ring-exhaustive counts equal the brute-force neighbour sets."""
    nside = 8
    tc = 0.31
    v = geometry.pixel_vectors(nside)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    adj = d <= kernel.chord_cut(tc)
    counts, margin = convolve.pair_counts_sampled(nside, tc, np.arange(v.shape[0]))
    assert np.array_equal(counts, adj.sum(axis=1))
    assert np.array_equal(adj, adj.T)
    assert margin > 1e-10
