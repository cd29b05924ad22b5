"""The seeded input generators: reproducible draws, and the random-field synthesis places
exactly sum a_lm Y_lm on the ring grid (checked against scipy's spherical harmonics at the
oracle's pixel centres)."""
import math

import numpy as np
import pytest
import scipy.special as sp

import synth
from oracle import geometry


def test_white_noise_reproducible():
    a = synth.white_noise(8, 2, seed=5)
    b = synth.white_noise(8, 2, seed=5)
    assert a.shape == (2, 768) and np.array_equal(a, b)
    assert not np.array_equal(a, synth.white_noise(8, 2, seed=6))


@pytest.mark.parametrize("l,m,val", [(0, 0, 1.0), (5, 0, 0.7), (7, 3, 1.0 + 0.5j), (40, 40, 0.3 - 1j), (33, 17, -2j)])
def test_synthesis_single_harmonic(l, m, val):
    nside, lmax = 16, 40
    z, st, phi, _ = geometry.pixel_angles(nside)
    alm = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=complex)
    alm[sum(lmax + 1 - mm for mm in range(m)) + (l - m)] = val
    f = synth.synthesize(nside, alm, lmax)
    ref = (val * sp.sph_harm_y(l, m, np.arccos(z), phi)).real * (1 if m == 0 else 2)
    assert np.max(np.abs(f - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_synthesis_polar_underflow_orders():
    """High orders at Nside 256 near the poles (lambda_mm underflows): values stay finite and
    match scipy where it is representable."""
    nside, lmax = 256, 700
    z, st, phi, _ = geometry.pixel_angles(nside)
    for l, m in [(700, 650), (300, 280)]:
        alm = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=complex)
        alm[sum(lmax + 1 - mm for mm in range(m)) + (l - m)] = 1.0
        f = synth.synthesize(nside, alm, lmax)
        assert np.all(np.isfinite(f))
        pix = np.random.default_rng(0).choice(f.size, 2000, replace=False)
        with np.errstate(all="ignore"):
            ref = 2 * sp.sph_harm_y(l, m, np.arccos(z[pix]), phi[pix]).real
        ok = np.isfinite(ref)                   # scipy itself overflows at high orders
        if ok.sum() > 1000:
            assert np.max(np.abs(f[pix][ok] - ref[ok])) <= 1e-10 * np.max(np.abs(ref[ok]))
        # Y_lm with m close to l vanishes towards the poles
        polar = np.abs(z) > 0.99
        assert np.max(np.abs(f[polar])) < 1e-6 * np.max(np.abs(f))


def test_grf_variance():
    """Pixel variance of a red-spectrum field equals sum (2l+1) C_l / (4 pi) within sampling error."""
    cl = synth.red_spectrum(256)
    f = synth.grf_map(128, cl, seed=3)
    expect = np.sum((2 * np.arange(257) + 1) * cl) / (4 * math.pi)
    assert abs(np.var(f) / expect - 1.0) < 0.1


def test_workloads():
    w = synth.workload("gauss32")
    assert w.nside == 32 and w.k_ell()[0] == 1.0
    w3 = synth.workload("resid2048")
    k = w3.k_ell()
    assert len(k) == 4097 and k[1000] == 0.0 and k[1600] > 0
    g = synth.cosine_taper(2000, 600, 100)
    assert g[550] == 1.0 and g[650] == 0.0 and g[600] == pytest.approx(0.5)


def test_batch_workload_recipe():
    ws = synth.batch_workload()
    assert len(ws) == 32
    assert {w.nside for w in ws} <= {256, 512, 1024, 2048}
    for k, w in enumerate(ws):
        fwhm = w.fwhm / synth.ARCMIN
        sigma = w.fwhm / math.sqrt(8 * math.log(2))
        assert 5.0 <= fwhm <= 30.0
        assert w.theta_cut == pytest.approx(6 * sigma)
        assert w.ell_cut == pytest.approx(0.3 / sigma) and w.taper_width == round(w.ell_cut / 6)
        assert w.lmax == 2 * w.nside and w.map_kind == ("white" if k % 2 == 0 else "red")
    again = synth.batch_workload()
    assert [(w.nside, w.fwhm) for w in again] == [(w.nside, w.fwhm) for w in ws]
    small = [w for w in ws if w.nside == 256][:2]
    maps = synth.batch_maps(small)
    assert all(m.dtype == np.float32 and m.shape == (12 * 256 ** 2,) for m in maps)
