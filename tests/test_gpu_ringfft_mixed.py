"""Ring-FFT method of mixed plans (conv_real_set_method on CONV_REAL_MIXED): FP32 maps, belt ring
pairs through the FP64 ring FFTs, cap-touching pairs on the split-FP16 cap tiles (weights from the
store or evaluated on the fly), the FFTs writing the belt rings and the cap tiles adding to them.
Checked against the oracle at the mixed path's bound (rel rms <= 1e-6) on full maps of small grids
and on sampled pixels (polar, cap-edge and belt-edge rings included) at Nside 512 and 2048, against
the direct method, with and without the weight store; switching back to the direct method restores
its result bit for bit; batches and the no-allocation entry point refuse such plans; applies of
both FP64 and mixed plans on the method replay from a HIP graph bit for bit."""
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
ARCMIN = DEG / 60
TOL = 1e-6


def _apply(plan, x):
    y = plan.apply(x)
    torch.cuda.synchronize()
    return y.clone()


def _check(y, ref):
    for m in range(ref.shape[0]):
        e = oc.rel_rms(y[m].astype(np.float64), ref[m])
        assert e <= TOL, (m, e)
        assert np.max(np.abs(y[m] - ref[m])) <= 1e-5 * np.max(np.abs(ref[m]))


def _edge_pixels(nside):
    from oracle import geometry
    rt = geometry.ring_table(nside)
    out = []
    for i in (1, 2, nside - 1, nside, nside + 1, 2 * nside, 3 * nside - 1, 3 * nside, 3 * nside + 1, 4 * nside - 1):
        s0, n = int(rt["start"][i - 1]), int(rt["n"][i - 1])
        out += [s0, s0 + n // 2, s0 + n - 1]
    return np.asarray(out, dtype=np.int64)


@pytest.mark.parametrize("nside,sigma_deg,cut_sigma", [(8, 6.0, 4.0), (16, 3.0, 5.0), (32, 1.5, 5.0), (64, 1.0, 6.0)])
@pytest.mark.parametrize("store", ["on", "off"])
def test_mixed_ring_fft_full_maps(cuda_device, nside, sigma_deg, cut_sigma, store):
    sigma = sigma_deg * DEG
    tc = cut_sigma * sigma
    T = ok.tabulate(synth.gaussian_beam_sigma(3 * nside, sigma), tc, 1024)
    xn = synth.white_noise(nside, 2, seed=nside + 91, dtype=np.float32)
    x = torch.from_numpy(xn).to("cuda:0")
    ref = oc.convolve_sampled(nside, T, tc, xn.astype(np.float64), np.arange(xn.shape[1]))
    with cr.Plan(nside, T, tc, "mixed") as plan:
        plan.set_weight_store(store)
        y_direct = _apply(plan, x)
        plan.set_method("ring_fft")
        assert plan.method() == "ring_fft"
        y_fft = _apply(plan, x)
        assert torch.equal(_apply(plan, x), y_fft)        # deterministic
        plan.set_method("direct")
        assert torch.equal(_apply(plan, x), y_direct)     # the direct queue is back
    _check(y_fft.cpu().numpy(), ref)
    _check(y_direct.cpu().numpy(), ref)


def test_mixed_ring_fft_residual_512(cuda_device):
    """The oscillating residual kernel at Nside 512 (wide windows relative to the grid), sampled pixels."""
    w = synth.workload("resid512")
    T = ok.tabulate(w.k_ell(), w.theta_cut, w.n_tab)
    xn = synth.white_noise(w.nside, 1, seed=17, dtype=np.float32)
    x = torch.from_numpy(xn).to("cuda:0")
    pix = np.unique(np.concatenate([np.random.default_rng(3).choice(xn.shape[1], 2000, replace=False),
                                    _edge_pixels(w.nside)]))
    ref = oc.convolve_sampled(w.nside, T, w.theta_cut, xn.astype(np.float64), pix)
    with cr.Plan(w.nside, T, w.theta_cut, "mixed") as plan:
        plan.set_method("ring_fft")
        y = _apply(plan, x).cpu().numpy()
    _check(y[:, pix], ref)


def test_mixed_ring_fft_nside2048_wide(cuda_device):
    """Nside 2048 at 120' (Table 1's range of cuts): sampled pixels against the C FP64 oracle."""
    from oracle import csum
    nside = 2048
    tc = 120.0 * ARCMIN
    k = synth.residual_beam(4096, 10.0 * ARCMIN, 1000.0, 150.0)
    T = ok.tabulate(k, tc, 4096)
    xn = synth.white_noise(nside, 1, seed=120, dtype=np.float32)
    x = torch.from_numpy(xn).to("cuda:0")
    pix = np.unique(np.concatenate([np.random.default_rng(5).choice(xn.shape[1], 300, replace=False),
                                    _edge_pixels(nside)]))
    print("mixed ring-fft nside 2048 120': plan", flush=True)
    with cr.Plan(nside, T, tc, "mixed") as plan:
        plan.set_method("ring_fft")
        print("apply", flush=True)
        y = _apply(plan, x).cpu().numpy()
    ref, _ = csum.convolve_sampled(nside, T, tc, xn.astype(np.float64), pix, nthreads=8)
    _check(y[:, pix], ref)


def test_mixed_ring_fft_refusals(cuda_device):
    nside, sigma = 16, 3.0 * DEG
    T = ok.tabulate(synth.gaussian_beam_sigma(48, sigma), 5 * sigma, 1024)
    with cr.Plan(nside, T, 5 * sigma, "mixed") as plan:
        plan.set_method("ring_fft")
        with pytest.raises(cr.ConvRealError):
            cr.Batch([plan])
        x = torch.zeros(12 * nside * nside, device="cuda:0")
        out = torch.empty_like(x)
        with pytest.raises(cr.ConvRealError):
            plan.apply_noalloc(x, out)
    with cr.Plan(12, T, 5 * sigma, "mixed") as plan:    # 48-pixel belt rings: not a power of two
        with pytest.raises(cr.ConvRealError):
            plan.set_method("ring_fft")
        assert plan.method() == "direct"


@pytest.mark.parametrize("precision", ["mixed", "f64"])
def test_ring_fft_graph_capture(cuda_device, precision):
    """An apply on the ring-FFT method recorded in a HIP graph (the transforms' LDS limits are set at
    plan set-up, so applies make no attribute calls): every replay, with eager work between them,
    equals the eager result bit for bit."""
    nside, sigma = 32, 1.5 * DEG
    tc = 5 * sigma
    T = ok.tabulate(synth.gaussian_beam_sigma(96, sigma), tc, 1024)
    dtype = np.float32 if precision == "mixed" else np.float64
    x = torch.from_numpy(synth.white_noise(nside, 2, seed=77, dtype=dtype)).to("cuda:0")
    with cr.Plan(nside, T, tc, precision) as plan:
        plan.set_method("ring_fft")
        ref = plan.apply(x).clone()
        y = torch.empty_like(x)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.apply(x, out=y)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            plan.apply(x, out=y)
        for rep in range(4):
            y.fill_(float("nan"))
            junk = torch.randn(1 << 20, device="cuda:0").sum()     # eager work between replays
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(y, ref), rep
            del junk
