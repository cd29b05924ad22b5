"""The library's split model (include/convsplit.h) against the oracle: Gauss-Legendre samples,
least-squares split (reduced form of Eqs. 3-5), Eqs. 2 and 6, the cost model and the split scan.
Host code only: these run without a GPU."""
import math

import numpy as np
import pytest

from oracle import split as osplit

cr = pytest.importorskip("paper_1409_4441_amd")
from paper_1409_4441_amd import split  # noqa: E402

ARCMIN = math.pi / (180 * 60)


def _beam(lmax, fwhm_arcmin):
    s = fwhm_arcmin * ARCMIN / math.sqrt(8 * math.log(2))
    ell = np.arange(lmax + 1)
    return np.exp(-0.5 * ell * (ell + 1) * s * s)


CASES = [  # (lmax, fwhm arcmin, ell_cut, theta_cut)
    (96, 150.0, 20, 0.12),
    (128, 120.0, 40, 0.15),      # eigenvalue cutoff active
    (256, 60.0, 90, 0.06),
    (512, 30.0, 200, 0.04),
    (512, 30.0, 511, 0.04),
    (300, 45.0, 0, 0.08),
]


@pytest.mark.parametrize("lmax,fwhm,ell_cut,tc", CASES)
def test_lsq_matches_oracle(lmax, fwhm, ell_cut, tc):
    K = _beam(lmax, fwhm)
    C = np.ones(lmax + 1)
    with split.Context(lmax, 0.2) as ctx:
        kh, kt, kr, ktl = ctx.lsq(K, ell_cut, tc)
    okh, ox, oz, oktl = osplit.lsq_split_reduced(K, C, ell_cut, tc)
    assert len(kt) == len(oz)
    P = osplit.legendre_operator(lmax, *osplit.real_space_nodes(lmax, tc))
    # The oracle's quadrature weights (NumPy's leggauss) carry relative errors up to ~1e-9 at these
    # sizes (measured against 40-digit Newton nodes), and a nearly singular reduced problem turns
    # them into large, mutually cancelling samples; tolerances scale with the summed terms.
    terms = np.max(np.abs(P) @ np.abs(ox)) if len(ox) else 0.0
    tol = 1e-11 * np.max(np.abs(K)) + 2e-9 * terms
    assert np.allclose(ktl, oktl, rtol=1e-9, atol=tol)
    assert np.allclose(kh, okh, rtol=1e-9, atol=tol)
    assert np.allclose(kr, P @ ox, rtol=1e-9, atol=tol)
    # samples in decreasing z on the library side, increasing in the oracle
    assert np.allclose(kt, ox[::-1], rtol=1e-7, atol=1e-7 * max(1.0, np.max(np.abs(ox), initial=0.0)))


@pytest.mark.parametrize("lmax,fwhm,ell_cut,tc", CASES)
def test_errors_match_oracle(lmax, fwhm, ell_cut, tc):
    K = _beam(lmax, fwhm)
    g = np.random.default_rng(lmax)
    C = np.exp(g.uniform(-1, 1, lmax + 1))
    with split.Context(lmax, 0.2, c_in=C) as ctx:
        srms, sig = ctx.error(K, ell_cut, tc, alpha=5.0)
    _, _, _, oktl = osplit.lsq_split_reduced(K, C, ell_cut, tc)
    assert srms == pytest.approx(osplit.rms_error(K, oktl, C), rel=1e-8, abs=1e-14)
    assert sig == pytest.approx(osplit.fractional_error(K, oktl, C, 5.0), rel=1e-8, abs=1e-14)


def test_node_counts_match_the_rule():
    with split.Context(1024, 0.5) as ctx:
        for tc in (0.01, 0.05, 0.2, 0.5):
            assert ctx.nodes(tc) == len(osplit.real_space_nodes(1024, tc)[0])


def test_cost_model_matches_oracle():
    pairs = np.array([2e9, 9e9, 4.8e10])
    t_real = np.array([0.9e-3, 1.7e-3, 4.1e-3])
    npix = np.array([3.1e6, 1.26e7, 5.03e7, 5.03e7])
    work = np.array([512.0 ** 2 * 1024, 1024.0 ** 2 * 2048, 512.0 ** 2 * 4096, 1500.0 ** 2 * 4096])
    t_sht = np.array([0.3e-3, 1.2e-3, 1.8e-3, 4.2e-3])
    m = split.CostModel.fit(pairs, t_real, npix, work, t_sht)
    a, b, c, c0, c1 = osplit.cost_fit(pairs, t_real, npix, work, t_sht)
    assert (m.a, m.b) == (pytest.approx(a, rel=1e-9, abs=1e-15), pytest.approx(b, rel=1e-9))
    assert (m.c, m.c0, m.c1) == (pytest.approx(c, rel=1e-8, abs=1e-25), pytest.approx(c0, rel=1e-8, abs=1e-15),
                                 pytest.approx(c1, rel=1e-8, abs=1e-22))
    assert m.c > 0 and (m.c0 > 0 or m.c1 > 0)   # this data needs more than Eq. 8's term
    for nside, tc in [(2048, 30 * ARCMIN), (256, 2.0 * math.pi / 180), (64, math.pi)]:
        assert split.pairs_estimate(nside, tc) == pytest.approx(osplit.pairs_estimate(nside, tc), rel=1e-12)
    tr, ts, wall = m.eval(2048, 4096, 30 * ARCMIN, 1500)
    assert tr == pytest.approx(a + b * osplit.pairs_estimate(2048, 30 * ARCMIN), rel=1e-12)
    assert ts == pytest.approx(c0 + c1 * 12 * 2048 ** 2 + c * 1500 ** 2 * 4096, rel=1e-8)
    assert wall == max(tr, ts)
    # Eq. 8's form alone (c0 = c1 = 0) when the times follow it
    m2 = split.CostModel.fit(pairs, t_real, npix, work, 1e-12 * work)
    assert (m2.c, m2.c0, m2.c1) == (pytest.approx(1e-12, rel=1e-12), 0.0, 0.0)


def test_search_matches_oracle_scan():
    lmax, nside = 128, 64
    K = _beam(lmax, 100.0)
    C = np.ones(lmax + 1)
    m = split.CostModel(1e-4, 1e-12, 1e-9)
    grid = [0.03, 0.05, 0.08, 0.12]
    bound = 1e-3
    with split.Context(lmax, max(grid)) as ctx:
        got = ctx.search(K, nside, bound, grid, m)
    want = osplit.split_search(
        K, C, bound, grid,
        t_gpu=lambda tc: m.a + m.b * osplit.pairs_estimate(nside, tc),
        t_cpu=lambda lc: m.c * lc * lc * lmax, solver=osplit.lsq_split_reduced)
    assert got is not None and want is not None
    assert got[0] == want[0] and got[1] == want[1]
    assert got[2] == pytest.approx(want[2], rel=1e-12)
    assert got[3] == pytest.approx(want[3], rel=1e-8)


def test_search_step_and_many():
    lmax, nside = 200, 128
    m = split.CostModel(1e-4, 5e-13, 2e-10)
    grid = np.array([0.02, 0.04, 0.06, 0.09])
    kernels = np.stack([_beam(lmax, f) for f in (60.0, 80.0, 100.0)])
    bounds = np.array([1e-3, 1e-4, 1e-2])
    with split.Context(lmax, grid.max()) as ctx:
        single = [ctx.search(k, nside, b, grid, m, ell_step=8) for k, b in zip(kernels, bounds)]
        th, lc, wl, sg = ctx.search_many(kernels, nside, bounds, grid, m, ell_step=8, nthreads=3)
    for k, s in enumerate(single):
        assert s is not None
        assert (th[k], lc[k]) == (s[0], s[1]) and wl[k] == s[2] and sg[k] == s[3]
        assert lc[k] % 8 == 0 or lc[k] == lmax
        assert sg[k] <= bounds[k]


def test_search_infeasible_and_bad_arguments():
    lmax = 64
    K = _beam(lmax, 200.0)
    m = split.CostModel(0.0, 1e-12, 1e-9)
    with split.Context(lmax, 0.3) as ctx:
        with pytest.raises(cr.ConvRealError):
            ctx.lsq(K, lmax + 1, 0.1)
        with pytest.raises(cr.ConvRealError):
            ctx.error(K, 10, 0.31)
        with pytest.raises(cr.ConvRealError):
            ctx.search(K, 32, 1e-3, [0.0], m)
        # ell_cut = lmax is always exact, so a bound is always met; with no real-space sample inside
        # the cut nothing can replace the dropped coefficients, so that is the only feasible split
        assert ctx.nodes(1e-3) == 0
        assert ctx.search(K, 32, 1e-12, [1e-3], m)[1] == lmax
        best = ctx.search(K, 32, 1e-12, [0.1], m)
        assert best is not None and best[3] <= 1e-12
    with pytest.raises(cr.ConvRealError):
        split.Context(0, 0.1)
    with pytest.raises(cr.ConvRealError):
        split.Context(64, 4.0)


def _paper_kernel(lmax, fwhm_arcmin):
    ell = np.arange(lmax + 1, dtype=np.float64)
    c = np.zeros(lmax + 1)
    c[2:] = 1.0 / (ell[2:] * (ell[2:] + 1.0))
    return np.sqrt(c) * _beam(lmax, fwhm_arcmin)


@pytest.mark.slow
def test_table1_errors_match_oracle():
    # the reduced solve at the paper's own operating point (lmax 4096, Table 1's cuts, where the
    # singular-value cutoff removes about a quarter of the samples' directions): the library's
    # Eq. 6 errors equal the oracle's SVD solve
    lmax = 4096
    C = np.ones(lmax + 1)
    with split.Context(lmax, 390 * ARCMIN) as ctx:
        for fwhm, lc, tc in [(7, 1158, 390), (10, 979, 360), (15, 961, 270)]:
            K = _paper_kernel(lmax, fwhm)
            _, sig = ctx.error(K, lc, tc * ARCMIN, alpha=5.0)
            _, _, _, oktl = osplit.lsq_split_reduced(K, C, lc, tc * ARCMIN)
            assert sig == pytest.approx(osplit.fractional_error(K, oktl, C, 5.0), rel=1e-6)


@pytest.mark.parametrize("fwhm,bound", [(90.0, 1e-4), (60.0, 1e-5)])
def test_search_equals_exhaustive_scan(fwhm, bound):
    # the library's bisection finds the cheapest feasible (theta_cut, l_cut) that enumerating every
    # pair of the grid finds
    lmax, nside = 64, 32
    K = _paper_kernel(lmax, fwhm)
    m = split.CostModel(2e-4, 3e-11, 4e-9)
    grid = [0.05, 0.08, 0.12, 0.18, 0.26]
    best = None
    with split.Context(lmax, max(grid)) as ctx:
        for tc in grid:
            for lc in range(lmax + 1):
                if ctx.error(K, lc, tc, alpha=5.0)[1] <= bound:
                    wall = m.eval(nside, lmax, tc, lc)[2]
                    if best is None or wall < best[2]:
                        best = (tc, lc, wall)
        got = ctx.search(K, nside, bound, grid, m)
    assert best is not None and got is not None
    assert (got[0], got[1]) == best[:2] and got[2] == pytest.approx(best[2], rel=1e-15)


def test_compensation_matches_oracle():
    lmax = 256
    K = _paper_kernel(lmax, 40.0)
    C = np.ones(lmax + 1)
    sig = 40.0 * ARCMIN / math.sqrt(8 * math.log(2))
    with split.Context(lmax, 0.3) as ctx:
        for lc, tc in [(255, 2 * sig), (60, 0.2), (120, 0.1), (200, 0.05)]:
            kh, _, _, kt = osplit.lsq_split_reduced(K, C, lc, tc)
            assert ctx.compensation(K, lc, tc) == pytest.approx(osplit.compensation(K, kh, kt), rel=1e-7, abs=1e-14)


def test_search_with_compensation_limit_matches_oracle():
    # with a cheap harmonic part the unconstrained scan takes l_cut just below lmax at a cut holding
    # two real-space samples, whose harmonic part must cancel far more than the kernel's own scale;
    # with the limit that cut keeps only the all-harmonic split, in the library as in the oracle
    lmax, nside, fwhm, bound = 512, 256, 25.0, 1e-4
    K = _paper_kernel(lmax, fwhm)
    C = np.ones(lmax + 1)
    sig = fwhm * ARCMIN / math.sqrt(8 * math.log(2))
    grid = [k * sig for k in (2.0, 3.0, 3.5, 5.0, 8.0)]
    m = split.CostModel(1e-4, 1e-13, 3e-12)
    t_gpu = lambda tc: m.a + m.b * osplit.pairs_estimate(nside, tc)   # noqa: E731
    t_cpu = lambda lc: m.c * lc * lc * lmax                             # noqa: E731
    with split.Context(lmax, max(grid)) as free, split.Context(lmax, max(grid), max_comp=1e-2) as guarded:
        r_free = free.search(K, nside, bound, grid, m)
        r_guard = guarded.search(K, nside, bound, grid, m)
        assert r_free[1] < lmax and free.compensation(K, r_free[1], r_free[0]) > 1e-2
    want_free = osplit.split_search(K, C, bound, grid, t_gpu, t_cpu, solver=osplit.lsq_split_reduced)
    want_guard = osplit.split_search(K, C, bound, grid, t_gpu, t_cpu, solver=osplit.lsq_split_reduced,
                                     max_comp=1e-2)
    assert r_free[:2] == want_free[:2]
    assert r_guard[:2] == want_guard[:2]
    assert r_guard[:2] != r_free[:2]


def test_wiener_weights_match_oracle_and_relax_the_split():
    # the library's errors under Wiener weights equal the oracle's; noise dominating above l_n lowers
    # the error of a split, so the smallest feasible l_cut at a cut does not grow
    lmax, fwhm, ell_n = 512, 25.0, 300
    K = _paper_kernel(lmax, fwhm)
    ell = np.arange(lmax + 1, dtype=np.float64)
    c = np.zeros(lmax + 1)
    c[2:] = 1.0 / (ell[2:] * (ell[2:] + 1.0))
    S = c * _beam(lmax, fwhm) ** 2
    W = split.wiener_weights(S, S[ell_n])
    assert np.allclose(W, osplit.wiener_weights(S, S[ell_n]), rtol=1e-15)
    tc = 20 * fwhm * ARCMIN
    with split.Context(lmax, tc, c_in=W) as cw, split.Context(lmax, tc) as cf:
        for lc in (120, 200, 260):
            kh, _, _, kt = osplit.lsq_split_reduced(K, W, lc, tc)
            assert cw.error(K, lc, tc, alpha=5.0)[1] == pytest.approx(
                osplit.fractional_error(K, kt, W, 5.0), rel=1e-7)
            assert cw.error(K, lc, tc)[1] < cf.error(K, lc, tc)[1]
        m = split.CostModel(1e-4, 1e-13, 3e-12)
        rw = cw.search(K, 256, 1e-5, [tc], m)
        rf = cf.search(K, 256, 1e-5, [tc], m)
        assert rw is not None and rf is not None and rw[1] <= rf[1]


def test_search_with_ell_cut_limit_matches_oracle():
    # a 100' beam at lmax 256 splits best at 5 sigma with l_cut 243 (0.95 lmax); with the limit that
    # cut keeps only the all-harmonic split, while a 120' beam's split at l_cut 57 is untouched; the
    # library's scan equals the oracle's in every case
    lmax, nside = 256, 128
    C = np.ones(lmax + 1)
    m = split.CostModel(1e-4, 1e-14, 1e-9)
    t_gpu = lambda tc: m.a + m.b * osplit.pairs_estimate(nside, tc)   # noqa: E731
    t_cpu = lambda lc: m.c * lc * lc * lmax                             # noqa: E731
    answers = {}
    for fwhm in (100.0, 120.0):
        K = _paper_kernel(lmax, fwhm)
        sig = fwhm * ARCMIN / math.sqrt(8 * math.log(2))
        grid = [k * sig for k in (1.0, 1.5, 2.0, 3.0, 5.0, 8.0)]
        for frac in (1.0, 0.45):
            with split.Context(lmax, max(grid), max_ell_frac=frac) as ctx:
                got = ctx.search(K, nside, 1e-3, grid, m)
            want = osplit.split_search(K, C, 1e-3, grid, t_gpu, t_cpu, solver=osplit.lsq_split_reduced,
                                       max_ell_frac=frac)
            assert got[:2] == want[:2], (fwhm, frac, got, want)
            assert got[1] == lmax or got[1] <= frac * lmax
            answers[fwhm, frac] = got[1]
    assert answers[100.0, 1.0] > 0.45 * lmax and answers[100.0, 0.45] == lmax
    assert answers[120.0, 1.0] == answers[120.0, 0.45] <= 0.45 * lmax
