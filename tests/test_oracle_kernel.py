"""Pins of the oracle's kernel tabulation and interpolation.

* Legendre series (Legendre transformation operator of Eq. 1): against
  scipy's independent P_l at exactly representable x; against the
  Christoffel-Darboux closed form for k_l = 1; round trip through
  Gauss-Legendre quadrature returns k_l (orthogonality of P_l).
* Interpolation: exact on cubics away from the origin, exact on even
  quadratics at the origin (ghost node T[-1] = T[1]), O(h^4) convergence.
* Truncated transfer function: closed forms for a constant kernel.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import kernel


def test_series_vs_scipy_legendre():
    g = np.random.default_rng(3)
    lmax = 300
    k_ell = g.standard_normal(lmax + 1)
    u = np.array([0.0, 2.0 ** -30, 2.0 ** -20, 3 * 2.0 ** -12, 0.25, 1.0, 1.5, 2.0])
    x = 1.0 - u                                   # exact in FP64 for these u
    ells = np.arange(lmax + 1)
    ref = np.array([np.sum((2 * ells + 1) / (4 * math.pi) * k_ell * sp.eval_legendre(ells, xx)) for xx in x])
    got = kernel.legendre_series_u(k_ell, u)
    scale = np.sum((2 * ells + 1) / (4 * math.pi) * np.abs(k_ell))
    assert np.max(np.abs(got - ref)) <= 1e-13 * scale


@pytest.mark.parametrize("L", [10, 512, 4096])
def test_christoffel_darboux(L):
    """sum_{l<=L} (2l+1) P_l(x) = (L+1)(P_L(x) - P_{L+1}(x)) / (1 - x); value (L+1)^2 at x = 1."""
    k_ell = np.ones(L + 1)
    u = np.array([2.0 ** -24, 2.0 ** -16, 2.0 ** -10, 0.125, 0.75, 1.25])
    x = 1.0 - u
    ref = (L + 1) * (sp.eval_legendre(L, x) - sp.eval_legendre(L + 1, x)) / u / (4 * math.pi)
    got = kernel.legendre_series_u(k_ell, u)
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-12 * (L + 1) ** 2 / (4 * math.pi))
    assert kernel.legendre_series_u(k_ell, np.array([0.0]))[0] == pytest.approx((L + 1) ** 2 / (4 * math.pi), rel=1e-14)


def test_round_trip_gauss_legendre():
    """2 pi * int_{-1}^{1} K(x) P_l(x) dx = k_l for l <= lmax."""
    lmax = 200
    g = np.random.default_rng(5)
    k_ell = g.standard_normal(lmax + 1)
    xg, wg = sp.roots_legendre(lmax + 2)
    K = kernel.legendre_series_u(k_ell, 1.0 - xg)
    scale = np.sum((2 * np.arange(lmax + 1) + 1) * np.abs(k_ell))
    for ell in [0, 1, 2, 17, 99, 200]:
        got = 2 * math.pi * np.sum(wg * K * sp.eval_legendre(ell, xg))
        assert got == pytest.approx(k_ell[ell], abs=1e-13 * scale)


def test_tabulate_nodes():
    k_ell = np.exp(-np.arange(100) * 0.05)
    theta_cut = 0.1
    n_tab = 64
    T = kernel.tabulate(k_ell, theta_cut, n_tab)
    h = kernel.node_spacing(theta_cut, n_tab)
    assert h == pytest.approx(2 * math.sin(0.05) / 61)
    d = np.arange(n_tab) * h
    assert np.allclose(T, kernel.legendre_series_u(k_ell, 0.5 * d * d), rtol=0, atol=0)
    # the node at index n_tab-3 is exactly the chord of theta_cut
    assert (n_tab - 3) * h == pytest.approx(2 * math.sin(theta_cut / 2), rel=1e-15)


def test_interp_exact_on_cubics():
    n = 40
    h = 0.01
    c = np.array([0.3, -1.7, 2.9, 4.1])
    f = lambda d: c[0] + c[1] * d + c[2] * d ** 2 + c[3] * d ** 3
    T = f(np.arange(n) * h)
    d = np.linspace(h, (n - 1) * h, 1001)          # segments k >= 1: no ghost node involved
    assert np.max(np.abs(kernel.interpolate(T, h, d) - f(d))) <= 1e-13
    # nodes are reproduced
    assert np.max(np.abs(kernel.interpolate(T, h, np.arange(n - 2) * h) - T[:n - 2])) <= 1e-14


def test_interp_even_at_origin():
    """Segment 0 uses the ghost T[-1] = T[1]; exact for even quadratics in d."""
    n = 20
    h = 0.05
    f = lambda d: 1.5 - 2.5 * d * d
    T = f(np.arange(n) * h)
    d = np.linspace(0.0, h, 101)
    assert np.max(np.abs(kernel.interpolate(T, h, d) - f(d))) <= 1e-14
    # an odd term breaks the ghost-node assumption: not exact there (control)
    g = lambda d: 1.5 + 0.7 * d
    Tg = g(np.arange(n) * h)
    assert np.max(np.abs(kernel.interpolate(Tg, h, d) - g(d))) > 1e-4


def test_interp_convergence_h4():
    f = lambda d: np.cos(7.0 * d) * np.exp(-d * d)
    errs = []
    for n in [34, 66, 130]:
        h = 1.0 / (n - 3)
        T = f(np.arange(n) * h)
        d = np.linspace(0.0, 1.0, 5001)
        errs.append(np.max(np.abs(kernel.interpolate(T, h, d) - f(d))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0


def test_truncated_transfer_constant_kernel():
    """For K = c: k_0 = 2 pi c (1 - cos tc); k_1 = pi c sin^2 tc; k_2 = pi c cos tc sin^2 tc."""
    c = 0.37
    tc = 0.3
    T = np.full(50, c)
    kt = kernel.truncated_transfer(T, tc, 3)
    assert kt[0] == pytest.approx(2 * math.pi * c * (1 - math.cos(tc)), rel=1e-13)
    assert kt[1] == pytest.approx(math.pi * c * math.sin(tc) ** 2, rel=1e-13)
    assert kt[2] == pytest.approx(math.pi * c * math.cos(tc) * math.sin(tc) ** 2, rel=1e-12)


def test_truncated_transfer_tends_to_k_ell():
    """A Gaussian beam truncated far in its tail keeps its harmonic coefficients."""
    sigma = 0.02
    lmax = 800
    ell = np.arange(lmax + 1)
    k_ell = np.exp(-0.5 * ell * (ell + 1) * sigma ** 2)
    tc = 10 * sigma
    T = kernel.tabulate(k_ell, tc, 2048)
    kt = kernel.truncated_transfer(T, tc, 60)
    assert np.allclose(kt, k_ell[:61], atol=1e-9)
