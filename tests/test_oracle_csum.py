"""The C oracle sums (oracle/csum.c) against the NumPy oracle's plain definitions.

The C code narrows each ring's candidates by the exact azimuth bound (plus two pixels) before the
exact chord test, so it must find the same pair set as the ring-exhaustive NumPy search and the
brute-force sum, and the same sums up to summation order: pair counts equal, values within 1e-13
relative rms. Cuts include rings that cross the poles, a cut below the pixel spacing, a cut of pi,
and the Nside 1 and 2 grids."""
import math

import numpy as np
import pytest

import synth
from oracle import convolve as oc
from oracle import csum
from oracle import kernel as ok

DEG = math.pi / 180


@pytest.mark.parametrize("nside,tc", [(1, 1.2), (2, 0.7), (8, 20 * DEG), (16, 12 * DEG), (16, math.pi),
                                      (32, 7.5 * DEG), (32, 0.5 * DEG), (64, 3 * DEG)])
def test_c_sums_equal_numpy_sums(nside, tc):
    table = ok.tabulate(synth.gaussian_beam_sigma(256, tc / 5), tc, 512)
    x = synth.white_noise(nside, 3, seed=nside + 11)
    npix = 12 * nside * nside
    pix = np.arange(npix) if npix <= 3072 else np.random.default_rng(nside).choice(npix, 1500, replace=False)
    want = oc.convolve_sampled(nside, table, tc, x, pix)
    cnt_want, margin = oc.pair_counts_sampled(nside, tc, pix)
    assert margin > 1e-12            # no chord within rounding of the cut
    got, cnt = csum.convolve_sampled(nside, table, tc, x, pix, nthreads=4)
    assert np.array_equal(cnt, cnt_want)
    for m in range(3):
        assert oc.rel_rms(got[m], want[m]) <= 1e-13


def test_c_sums_equal_brute_force_and_chunk_maps():
    nside, tc = 16, 10 * DEG
    table = ok.tabulate(synth.gaussian_beam_sigma(256, 2 * DEG), tc, 256)
    x = synth.white_noise(nside, 70, seed=5)          # more than one 64-map block
    want = oc.convolve_bruteforce(nside, table, tc, x[[0, 65]])
    got, _ = csum.convolve_sampled(nside, table, tc, x, np.arange(12 * nside * nside))
    assert oc.rel_rms(got[0], want[0]) <= 1e-13 and oc.rel_rms(got[65], want[1]) <= 1e-13
    with pytest.raises(ValueError):
        csum.convolve_sampled(nside, table, tc, x, np.array([12 * nside * nside]))
