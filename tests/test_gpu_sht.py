"""GPU parity of the harmonic half of the split (analysis, synthesis, harmonic convolution, power
spectrum) and of the hybrid apply, against the FP64 oracle (oracle/sht.py, oracle/convolve.py).

Tolerances (FP64 arithmetic on both sides, different summation orders and ring-sum forms):
transforms of FP64 maps agree to 1e-11 of the largest coefficient or pixel value (the GPU takes ring
DFTs by FFT, chirp-z convolution or Horner's rule, the oracle by explicit exponentials); FP32 maps are
promoted exactly, so the same bound holds. The hybrid apply adds the real-space part, at that part's own tolerance (1e-12 for
FP64 plans, 1e-6 relative rms for the mixed path).
"""
import math

import numpy as np
import pytest

import synth
from oracle import convolve as oc
from oracle import kernel as ok
from oracle import sht as osht

torch = pytest.importorskip("torch")
cr = pytest.importorskip("paper_1409_4441_amd")
from paper_1409_4441_amd import sht  # noqa: E402

pytestmark = pytest.mark.gpu

DEG = math.pi / 180


def _rand_alm(L, seed):
    g = np.random.default_rng(seed)
    a = g.standard_normal(osht.alm_size(L)) + 1j * g.standard_normal(osht.alm_size(L))
    a[: L + 1] = a[: L + 1].real          # m = 0 coefficients of a real map are real
    return a


def _close(got, ref, rtol):
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    assert err <= rtol * scale, (err, scale)


# (nside, L): L above 4 nside folds frequencies of the small polar rings (m >= n); L = 3 nside - 1
# is the usual band limit; power-of-two grids from Nside 4 take the belt rings through FFTs, Nside 12
# and the smallest grids through the folded sums; rings of 16 pixels or more per quarter take the
# chirp-z sums (polar rings from Nside 32, every ring but the smallest at Nside 24 and 48; at Nside 64 /
# L 300 every such ring also folds frequencies, at Nside 48 / L 60 the band limit cuts each class short;
# L 2 and 0 leave residue classes without a frequency)
CASES = [(1, 6), (2, 17), (4, 11), (8, 23), (12, 40), (16, 40), (32, 95), (24, 71), (48, 60), (64, 300),
         (32, 2), (48, 0)]


@pytest.mark.parametrize("nside,L", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_analysis_matches_oracle(cuda_device, nside, L, dtype):
    npix = 12 * nside * nside
    x = np.random.default_rng(nside + L).standard_normal(npix)
    if dtype == "f32":
        x = x.astype(np.float32)
    ref = osht.analysis(nside, x.astype(np.float64), L)
    with sht.Sht(nside, L) as t:
        got = t.analysis(torch.from_numpy(x).to(cuda_device)).cpu().numpy()
    _close(got, ref, 1e-11)


@pytest.mark.parametrize("nside,L", CASES)
def test_synthesis_matches_oracle(cuda_device, nside, L):
    a = _rand_alm(L, 7 * nside + L)
    ref = osht.synthesis(nside, a, L)
    with sht.Sht(nside, L) as t:
        at = torch.from_numpy(a).to(cuda_device)
        got = t.synthesis(at).cpu().numpy()
        got32 = t.synthesis(at, dtype=torch.float32).cpu().numpy()
        # accumulate adds onto what the map holds
        base = torch.full((12 * nside * nside,), 0.5, dtype=torch.float64, device=cuda_device)
        acc = t.synthesis(at, out=base, accumulate=True).cpu().numpy()
    _close(got, ref, 1e-11)
    assert np.max(np.abs(got32 - ref)) <= 1e-6 * np.max(np.abs(ref))
    _close(acc - 0.5, ref, 1e-11)


def test_polar_orders_below_fp64_range(cuda_device):
    # at Nside 128, l and m up to 600, lambda_mm of the polar rings is far below 1e-308; the
    # recurrence must start scaled and still give the oracle's coefficients
    nside, L = 128, 600
    x = np.random.default_rng(3).standard_normal(12 * nside * nside)
    ref = osht.analysis(nside, x, L)
    a = _rand_alm(L, 4)
    ref_y = osht.synthesis(nside, a, L)
    with sht.Sht(nside, L) as t:
        got = t.analysis(torch.from_numpy(x).to(cuda_device)).cpu().numpy()
        got_y = t.synthesis(torch.from_numpy(a).to(cuda_device)).cpu().numpy()
    _close(got, ref, 1e-11)
    _close(got_y, ref_y, 1e-11)


def test_transforms_at_nside_2048_sampled(cuda_device):
    # the workload's grid: chirp-z convolutions up to 4096 points (polar rings up to 2047 pixels per
    # quarter), belt rings of 8192 pixels two per FFT; the oracle restricted to a few orders (analysis)
    # or rings (synthesis: first polar rings, the first chirp-z ring, the last polar ring, the first belt
    # rings, the equator, the south pole's ring)
    from oracle import geometry
    nside, L = 2048, 1500
    x = np.random.default_rng(21).standard_normal(12 * nside * nside)
    orders = [0, 1, 1024, 1500]
    ref = osht.analysis_orders(nside, x, L, orders)
    with sht.Sht(nside, L) as t:
        got = t.analysis(torch.from_numpy(x).to(cuda_device)).cpu().numpy()
    scale = max(float(np.max(np.abs(v))) for v in ref.values())
    for m in orders:
        i0 = osht.alm_index(L, m, m)
        err = float(np.max(np.abs(got[i0: i0 + L - m + 1] - ref[m])))
        assert err <= 1e-11 * scale, (m, err, scale)
    Ls = 600
    a = _rand_alm(Ls, 5)
    rings = [0, 1, 15, 16, 1500, 2046, 2047, 2048, 4095, 8190]
    ref_y = osht.synthesis_rings(nside, a, Ls, rings)
    with sht.Sht(nside, Ls) as t:
        got_y = t.synthesis(torch.from_numpy(a).to(cuda_device)).cpu().numpy()
    rt = geometry.ring_table(nside)
    scale_y = max(float(np.max(np.abs(v))) for v in ref_y.values())
    for r in rings:
        g = got_y[rt["start"][r]: rt["start"][r] + rt["n"][r]]
        err = float(np.max(np.abs(g - ref_y[r])))
        assert err <= 1e-11 * scale_y, (r, err, scale_y)


def test_synthesis_after_analysis_on_one_plan(cuda_device):
    # polar rings that an order leaves out of the Legendre sums (their scaled values never come back
    # into the FP64 range before L; chunks of 256 rings from the pole) get F_m = 0 from the synthesis,
    # also where the plan's ring-sum buffer still holds an analysis's values: rings on both sides of
    # the chunk edges, in both hemispheres, against the oracle
    from oracle import geometry
    nside, L = 2048, 1500
    x = np.random.default_rng(31).standard_normal(12 * nside * nside)
    a = _rand_alm(L, 6)
    rings = [0, 255, 256, 511, 512, 767, 768, 1023, 1024, 1279, 1280, 1535, 1536, 1800, 8190 - 1279, 8190]
    ref_y = osht.synthesis_rings(nside, a, L, rings)
    with sht.Sht(nside, L) as t:
        t.analysis(torch.from_numpy(x).to(cuda_device))
        got_y = t.synthesis(torch.from_numpy(a).to(cuda_device)).cpu().numpy()
    rt = geometry.ring_table(nside)
    scale_y = max(float(np.max(np.abs(v))) for v in ref_y.values())
    for r in rings:
        g = got_y[rt["start"][r]: rt["start"][r] + rt["n"][r]]
        err = float(np.max(np.abs(g - ref_y[r])))
        assert err <= 1e-11 * scale_y, (r, err, scale_y)


@pytest.mark.parametrize("nside,L", [(8, 20), (32, 64)])
def test_convolve_and_power_spectrum(cuda_device, nside, L):
    x = np.random.default_rng(11).standard_normal(12 * nside * nside)
    k = synth.gaussian_beam_sigma(L, 3.0 * DEG)
    ref = osht.convolve(nside, x, k)
    ref_cl = osht.power_spectrum(osht.analysis(nside, x, L), L)
    with sht.Sht(nside, L) as t:
        xt = torch.from_numpy(x).to(cuda_device)
        got = t.convolve(xt, k).cpu().numpy()
        cl = t.power_spectrum(t.analysis(xt)).cpu().numpy()
        b = t.almxfl(t.analysis(xt), k)
        got2 = t.synthesis(b).cpu().numpy()
    _close(got, ref, 1e-11)
    _close(got2, ref, 1e-11)
    _close(cl, ref_cl, 1e-11)


def _split_case(nside):
    """A Gaussian kernel split at l_cut with a raised-cosine taper: harmonic part g_l k_l, real-space
    part the Legendre series of (1 - g_l) k_l truncated at theta_cut (any split of this form tests
    the sum of the two halves)."""
    L = 3 * nside - 1
    sigma = 1.5 * math.sqrt(math.pi / 3) / nside       # 1.5 pixel sizes
    k = synth.gaussian_beam_sigma(L, sigma)
    lc, w = L // 3, max(2, L // 8)
    ell = np.arange(L + 1)
    g = np.where(ell <= lc - w / 2, 1.0, np.where(ell >= lc + w / 2, 0.0,
                 0.5 * (1 + np.cos(np.pi * (ell - lc + w / 2) / w))))
    tc = 5.0 * sigma
    table = ok.tabulate(k * (1 - g), tc, 2048)
    return L, k * g, table, tc


@pytest.mark.parametrize("precision,tol", [("f64", 1e-11), ("mixed", 1e-6)])
def test_hybrid_apply_matches_oracle(cuda_device, precision, tol):
    nside = 16
    L, k_hat, table, tc = _split_case(nside)
    x = np.random.default_rng(5).standard_normal((2, 12 * nside * nside))
    if precision != "f64":
        x = x.astype(np.float32)
    xd = x.astype(np.float64)
    pix = np.arange(x.shape[1])
    ref = oc.convolve_sampled(nside, table, tc, xd, pix) + np.stack([osht.convolve(nside, xd[m], k_hat)
                                                                      for m in range(2)])
    with cr.Plan(nside, table, tc, precision) as plan, sht.Sht(nside, L) as t:
        xt = torch.from_numpy(x).to(cuda_device)
        side = torch.cuda.Stream()
        y2 = sht.hybrid_apply(plan, t, k_hat, xt, stream_sht=side)
        torch.cuda.synchronize()
        y1 = sht.hybrid_apply(plan, t, k_hat, xt)
        torch.cuda.synchronize()
    y1, y2 = y1.cpu().numpy().astype(np.float64), y2.cpu().numpy().astype(np.float64)
    assert np.array_equal(y1, y2)      # two streams or one: the same kernels and the same sums
    for m in range(2):
        assert oc.rel_rms(y1[m], ref[m]) <= tol, (m, oc.rel_rms(y1[m], ref[m]))


def test_hybrid_rejects_mismatched_plans(cuda_device):
    L, k_hat, table, tc = _split_case(8)
    with cr.Plan(16, table, tc, "f64") as plan, sht.Sht(8, L) as t:
        x = torch.zeros(12 * 8 * 8, dtype=torch.float64, device=cuda_device)
        with pytest.raises(cr.ConvRealError) as err:
            sht.hybrid_apply(plan, t, k_hat, x)
        assert err.value.code == cr.EINVAL
