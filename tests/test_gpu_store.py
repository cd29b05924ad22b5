"""The mixed path's cap weight store (conv_real_set_weight_store): weights evaluated on the fly and
weights computed once and streamed both meet the oracle at the mixed path's tolerance, on grids
that exercise the short and long weight forms, whole-ring windows near the poles, the smallest
rings and inputs that wrap around a ring; switching modes frees and rebuilds the store and resets
the default launch configuration (never one the caller set); results are deterministic in each
mode."""
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
TOL = 1e-6


def _apply(plan, x):
    y = plan.apply(x)
    torch.cuda.synchronize()
    return y


def _check(y, ref):
    for m in range(ref.shape[0]):
        assert oc.rel_rms(y[m], ref[m]) <= TOL, (m, oc.rel_rms(y[m], ref[m]))
        assert np.max(np.abs(y[m] - ref[m])) <= 1e-5 * np.max(np.abs(ref[m]))


CASES = [  # nside, sigma (deg), cut in sigma, n_tab
    (8, 6.0, 5.0, 256),      # windows covering whole polar rings
    (16, 4.0, 4.0, 1024),
    (32, 1.5, 5.0, 2048),
    (64, 1.0, 5.0, 2048),
    (128, 0.3, 6.0, 2048),   # short form on almost every cap tile
]


@pytest.mark.parametrize("nside,sigma_deg,cut_sigma,n_tab", CASES)
def test_store_modes_match_oracle(cuda_device, nside, sigma_deg, cut_sigma, n_tab):
    sigma = sigma_deg * DEG
    tc = cut_sigma * sigma
    T = ok.tabulate(synth.gaussian_beam_sigma(3 * nside, sigma), tc, n_tab)
    xn = synth.white_noise(nside, 2, seed=nside + 7, dtype=np.float32)
    x = torch.from_numpy(xn).to("cuda:0")
    npix = xn.shape[1]
    pix = np.arange(npix) if nside <= 32 else np.random.default_rng(nside).choice(npix, 2500, replace=False)
    ref = oc.convolve_sampled(nside, T, tc, xn.astype(np.float64), pix)
    with cr.Plan(nside, T, tc, "mixed") as plan:
        active, nbytes = plan.weight_store()
        assert active and nbytes > 0                  # new plans take the automatic mode; small ones fit
        assert plan.get_tuning() == {"seg": 256, "wg_per_cu": 3, "order": 3}   # the default with a store
        y_on = _apply(plan, x).clone()
        assert torch.equal(_apply(plan, x), y_on)     # deterministic
        plan.set_weight_store("off")
        assert plan.weight_store() == (False, 0)
        assert plan.get_tuning() == {"seg": 256, "wg_per_cu": 3, "order": 3}   # the table shares the belt stage
        y_off = _apply(plan, x).clone()
        assert torch.equal(_apply(plan, x), y_off)
        plan.set_weight_store("on")
        assert plan.weight_store() == (True, nbytes)
        assert torch.equal(_apply(plan, x), y_on)     # rebuilt store, same weights
    _check(y_on.cpu().numpy()[:, pix], ref)
    _check(y_off.cpu().numpy()[:, pix], ref)


def test_store_residual_kernel_512(cuda_device):
    """The oscillating residual kernel at Nside 512, both modes, sampled pixels."""
    w = synth.workload("resid512")
    T = ok.tabulate(w.k_ell(), w.theta_cut, w.n_tab)
    xn = synth.white_noise(w.nside, 1, seed=5, dtype=np.float32)
    x = torch.from_numpy(xn).to("cuda:0")
    pix = np.random.default_rng(2).choice(xn.shape[1], 2000, replace=False)
    ref = oc.convolve_sampled(w.nside, T, w.theta_cut, xn.astype(np.float64), pix).reshape(1, -1)
    with cr.Plan(w.nside, T, w.theta_cut, "mixed") as plan:
        for mode in ("on", "off"):
            plan.set_weight_store(mode)
            _check(_apply(plan, x).cpu().numpy()[:, pix], ref)


def test_store_size_and_bad_mode(cuda_device):
    nside, sigma = 64, 1.0 * DEG
    tc = 5 * sigma
    T = ok.tabulate(synth.gaussian_beam_sigma(192, sigma), tc, 2048)
    with cr.Plan(nside, T, tc, "mixed") as plan:
        plan.set_weight_store("on")
        active, nbytes = plan.weight_store()
        # 16-byte groups of 4 weights per (fundamental-domain pixel, input group meeting its window)
        # of the cap-touching ring pairs: about 4 bytes per pixel pair / 16, plus the groups' padding
        assert active
        assert nbytes % 16 == 0
        assert plan.pairs() / 200 < nbytes <= 4 * 1.6 * plan.pairs() / 16 + 32
        with pytest.raises(cr.ConvRealError):
            plan.set_weight_store("sometimes")
    with cr.Plan(nside, T, tc, "f32") as plain:
        with pytest.raises(cr.ConvRealError):
            plain.set_weight_store("on")


def test_store_keeps_caller_tuning(cuda_device):
    nside, sigma = 32, 1.5 * DEG
    tc = 5 * sigma
    T = ok.tabulate(synth.gaussian_beam_sigma(96, sigma), tc, 1024)
    with cr.Plan(nside, T, tc, "mixed") as plan:
        plan.set_tuning(256, 3, 1)
        plan.set_weight_store("off")
        plan.set_weight_store("on")
        assert plan.get_tuning() == {"seg": 256, "wg_per_cu": 3, "order": 1}
