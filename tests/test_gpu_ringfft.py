"""Ring-FFT method of FP64 plans (conv_real_set_method): belt ring pairs as products of ring
spectra, cap-touching pairs per pair. Same pairs and kernel values as the per-pair sum, so the
result meets the oracle at the FP64 bound (rel rms <= 1e-12, max error <= 1e-12 max |y|) on grids
where every ring is a belt ring (Nside 1), where windows cover whole rings and every pair is kept
(theta_cut = pi), and at cuts below the pixel spacing; it equals the direct method to rounding at a
larger grid; switching methods keeps results; only FP64 and mixed plans of power-of-two Nside <= 2048
take it (mixed plans: tests/test_gpu_ringfft_mixed.py)."""
import math

import numpy as np
import pytest

import synth
from oracle import convolve as oc
from oracle import kernel as ok

torch = pytest.importorskip("torch")
cr = pytest.importorskip("paper_1409_4441_amd")

pytestmark = pytest.mark.gpu

DEG = math.pi / 180


def _table(sigma, tc, n_tab=256, lmax=96):
    return ok.tabulate(synth.gaussian_beam_sigma(lmax, sigma), tc, n_tab)


def _run(plan, x_np):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to("cuda:0")
    y = plan.apply(x)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _check(y, ref):
    for m in range(ref.shape[0]):
        assert oc.rel_rms(y[m], ref[m]) <= 1e-12, (m, oc.rel_rms(y[m], ref[m]))
        assert np.max(np.abs(y[m] - ref[m])) <= 1e-12 * np.max(np.abs(ref[m]))


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("tc_deg", [0.5, 9.0, 40.0, 180.0])
def test_ring_fft_matches_oracle(cuda_device, nside, tc_deg):
    tc = tc_deg * DEG
    T = _table(max(tc / 3, 0.05), tc, n_tab=64, lmax=64)
    x = synth.white_noise(nside, 2, seed=300 + nside)
    with cr.Plan(nside, T, tc, "f64") as plan:
        assert plan.method() == "direct"
        plan.set_method("ring_fft")
        assert plan.method() == "ring_fft"
        y = _run(plan, x)
    ref = oc.convolve_sampled(nside, T, tc, x, np.arange(x.shape[1]))
    _check(y, ref)


@pytest.mark.parametrize("n_tab", [2050, 3000])
def test_ring_fft_table_forms(cuda_device, n_tab):
    """The cap-touching pairs' kernel stages the table as cubic coefficients up to 2048 segments and
    as nodes beyond; the spectra always interpolate from the nodes."""
    nside, sigma = 8, 5.0 * DEG
    tc = 4 * sigma
    T = _table(sigma, tc, n_tab=n_tab, lmax=64)
    x = synth.white_noise(nside, 2, seed=n_tab)
    with cr.Plan(nside, T, tc, "f64") as plan:
        plan.set_method("ring_fft")
        y = _run(plan, x)
    _check(y, oc.convolve_sampled(nside, T, tc, x, np.arange(x.shape[1])))


def test_ring_fft_equals_direct_and_oracle_nside128(cuda_device):
    nside, sigma = 128, 2.0 * DEG
    tc = 5 * sigma
    T = _table(sigma, tc, n_tab=2048, lmax=384)
    x = synth.white_noise(nside, 3, seed=31)
    with cr.Plan(nside, T, tc, "f64") as plan:
        y_direct = _run(plan, x)
        plan.set_method("ring_fft")
        y_fft = _run(plan, x)
        y_fft1 = _run(plan, x[1:2])                 # one map alone equals the same map in a batch
        plan.set_method("direct")
        assert np.array_equal(_run(plan, x), y_direct)
    _check(y_fft, y_direct)
    assert np.array_equal(y_fft1[0], y_fft[1])
    pix = np.random.default_rng(5).choice(x.shape[1], 1500, replace=False)
    ref = oc.convolve_sampled(nside, T, tc, x, pix)
    _check(y_fft[:, pix], ref)


@pytest.mark.parametrize("nside", [512, 1024])
def test_ring_fft_ring_groups(cuda_device, nside):
    """The belt sums run on groups of output rings per workgroup, as many as still fill the chip: two
    at Nside 512, eight at Nside 1024 (one on the smaller grids above). Equal to the direct method to
    rounding, and to the oracle on sampled pixels."""
    tc = 30.0 / 60.0 * DEG
    T = _table(tc / 4, tc, n_tab=1024, lmax=1024)
    x = synth.white_noise(nside, 1, seed=77)
    with cr.Plan(nside, T, tc, "f64") as plan:
        y_direct = _run(plan, x)
        plan.set_method("ring_fft")
        y_fft = _run(plan, x)
    _check(y_fft, y_direct)
    pix = np.random.default_rng(8).choice(x.shape[1], 400, replace=False)
    _check(y_fft[:, pix], oc.convolve_sampled(nside, T, tc, x, pix))


def test_ring_fft_only_where_defined(cuda_device):
    T = _table(3 * DEG, 9 * DEG)
    with cr.Plan(8, T, 9 * DEG, "f32") as plan:
        with pytest.raises(cr.ConvRealError):
            plan.set_method("ring_fft")
    with cr.Plan(6, T, 9 * DEG, "f64") as plan:       # 24-pixel belt rings: not a power of two
        with pytest.raises(cr.ConvRealError):
            plan.set_method("ring_fft")
        assert plan.method() == "direct"
    with cr.Plan(8, T, 9 * DEG, "f64") as plan:
        with pytest.raises(cr.ConvRealError):
            plan.set_method("sideways")


def test_ring_fft_nside2048(cuda_device):
    """Nside 2048 (8192-pixel belt rings: the largest transform, 128 KB of LDS, several strided passes
    per thread in the butterfly, spectrum and inverse loops): equal to the direct method over the full
    map and to the C FP64 oracle at 2000 sampled pixels (polar and belt-edge rings included), both at
    the FP64 bound."""
    from oracle import csum, geometry
    nside = 2048
    tc = 30.0 / 60.0 * DEG
    T = _table(tc / 4, tc, n_tab=2048, lmax=4096)
    x = synth.white_noise(nside, 1, seed=2048)
    print("ring-fft nside 2048: direct, then ring_fft", flush=True)
    with cr.Plan(nside, T, tc, "f64") as plan:
        y_direct = _run(plan, x)
        plan.set_method("ring_fft")
        y_fft = _run(plan, x)
    _check(y_fft, y_direct)
    rt = geometry.ring_table(nside)
    edge = [int(rt["start"][i - 1]) + o for i in (1, 2, nside - 1, nside, nside + 1, 3 * nside, 3 * nside + 1,
                                                  4 * nside - 1) for o in (0, 1)]
    pix = np.unique(np.concatenate([np.random.default_rng(9).choice(x.shape[1], 2000, replace=False), edge]))
    ref, _ = csum.convolve_sampled(nside, T, tc, x, pix, nthreads=8)
    _check(y_fft[:, pix], ref)
