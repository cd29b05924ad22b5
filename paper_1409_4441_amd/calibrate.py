"""Measure the constants of the split cost model on this machine and write them as JSON.

    python -m paper_1409_4441_amd.calibrate [--out cost_model.json] [--quick]

Real-space part: conv_real_apply of the mixed-precision path on one white-noise map, for Gaussian
beams over Nside 256..2048, FWHM 5'..30' and theta_cut 2..12 sigma (the range the split scan
visits); times from HIP events around the applies, pair counts exact (conv_real_pairs). Fitted:
t_real = a + b pairs.
Harmonic part: the library's harmonic convolution on the GPU (conv_sht_convolve: analysis, product,
synthesis) with band limit l_cut, at several (Nside, l_cut); fitted: t_sht = c0 + c1 Npix + c l_cut^2
lmax with lmax = 2 Nside (Eq. 8's form, c l_cut^2 lmax, for the Legendre sums, plus the launches and
the ring sums, which grow with the pixel count; coefficients >= 0). The two halves of a hybrid apply run at the same time on two
streams (Fig. 1), so the model's wall time is the slower of the two; a few hybrid applies are timed
beside the model to show how far that holds on one device.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ARCMIN = math.pi / (180.0 * 60.0)


def real_space_points(quick: bool):
    import torch

    import paper_1409_4441_amd as cr
    from paper_1409_4441_amd import learn
    nsides = (256, 512, 1024) if quick else (256, 512, 1024, 2048)
    pts = []
    for nside in nsides:
        for fwhm in (5.0, 15.0, 30.0):
            for ns in (2.0, 4.0, 8.0, 12.0):
                s = learn.sigma_of(fwhm)
                tc = ns * s
                lmax = 2 * nside
                table = cr.tabulate(learn.beam(lmax, fwhm), tc, 1024)
                with cr.Plan(nside, table, tc, "mixed") as plan:
                    g = torch.Generator(device="cuda").manual_seed(nside * 1000 + int(fwhm * 10) + int(ns))
                    x = torch.randn((1, 12 * nside * nside), device="cuda", generator=g)
                    y = torch.empty_like(x)
                    for _ in range(2):
                        plan.apply(x, out=y)
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    reps = 5
                    e0.record()
                    for _ in range(reps):
                        plan.apply(x, out=y)
                    e1.record()
                    torch.cuda.synchronize()
                    t = e0.elapsed_time(e1) / reps * 1e-3
                    pts.append({"nside": nside, "fwhm_arcmin": fwhm, "theta_cut": tc, "pairs": plan.pairs(),
                                "seconds": t})
                print(f"real-space nside {nside} fwhm {fwhm}' theta {ns} sigma: {pts[-1]['pairs']:.3e} pairs "
                      f"{t * 1e3:.3f} ms", flush=True)
    return pts


def harmonic_points(quick: bool):
    import torch

    from paper_1409_4441_amd import sht
    cases = [(256, 64), (256, 256), (512, 256), (512, 1024), (1024, 512), (1024, 2048)] if quick else \
        [(256, 64), (256, 256), (256, 512), (512, 128), (512, 512), (512, 1024), (1024, 256), (1024, 1024),
         (1024, 2048), (2048, 512), (2048, 1500), (2048, 4096)]
    pts = []
    for nside, lc in cases:
        with sht.Sht(nside, lc) as t:
            g = torch.Generator(device="cuda").manual_seed(nside + lc)
            x = torch.randn(12 * nside * nside, device="cuda", generator=g)
            k = torch.ones(lc + 1, dtype=torch.float64, device="cuda")
            y = torch.empty_like(x)
            t.convolve(x, k, out=y)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 3
            e0.record()
            for _ in range(reps):
                t.convolve(x, k, out=y)
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / reps * 1e-3
        pts.append({"nside": nside, "ell_cut": lc, "lmax": 2 * nside, "npix": 12 * nside * nside, "seconds": sec})
        print(f"harmonic nside {nside} l_cut {lc}: {sec * 1e3:.2f} ms", flush=True)
    return pts


def hybrid_points(model):
    """Hybrid applies (mixed real-space plan + harmonic half at band limit l_cut, two streams) timed
    against the model's max(t_real, t_sht) and the sum of the two."""
    import torch

    import paper_1409_4441_amd as cr
    from paper_1409_4441_amd import learn, sht
    pts = []
    for nside, fwhm, ns, lc in [(1024, 10.0, 8.0, 512), (2048, 5.0, 6.0, 1500), (2048, 10.0, 12.0, 800)]:
        s = learn.sigma_of(fwhm)
        tc = ns * s
        table = cr.tabulate(learn.beam(2 * nside, fwhm), tc, 1024)
        with cr.Plan(nside, table, tc, "mixed") as plan, sht.Sht(nside, lc) as t:
            x = torch.randn((1, 12 * nside * nside), device="cuda")
            k = torch.ones(lc + 1, dtype=torch.float64, device="cuda")
            side = torch.cuda.Stream()
            y = sht.hybrid_apply(plan, t, k, x, stream_sht=side)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 3
            e0.record()
            for _ in range(reps):
                sht.hybrid_apply(plan, t, k, x, out=y, stream_sht=side)
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / reps * 1e-3
            pairs = plan.pairs()
        tr, ts, wl = model.eval(nside, 2 * nside, tc, lc)
        pts.append({"nside": nside, "fwhm_arcmin": fwhm, "theta_cut": tc, "ell_cut": lc, "pairs": pairs,
                    "seconds": sec, "model_t_real": tr, "model_t_sht": ts, "model_wall": wl})
        print(f"hybrid nside {nside} fwhm {fwhm}' theta {ns} sigma l_cut {lc}: {sec * 1e3:.2f} ms "
              f"(model max {wl * 1e3:.2f}, sum {(tr + ts) * 1e3:.2f})", flush=True)
    return pts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_model.json"))
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    from paper_1409_4441_amd import split
    real = real_space_points(args.quick)
    harm = harmonic_points(args.quick)
    m = split.CostModel.fit([p["pairs"] for p in real], [p["seconds"] for p in real], [p["npix"] for p in harm],
                            [p["ell_cut"] ** 2 * p["lmax"] for p in harm], [p["seconds"] for p in harm])
    hyb = hybrid_points(m)
    for p in harm:
        p["model_seconds"] = m.eval(p["nside"], p["lmax"], 1e-3, p["ell_cut"])[1]
    out = dict(m.as_dict(), real_space=real, harmonic=harm, hybrid=hyb,
               note="t_real = a + b pairs (mixed-precision path, one map); "
                    "t_sht = c0 + c1 npix + c l_cut^2 lmax (GPU harmonic convolution at band limit l_cut); "
                    "hybrid: measured two-stream applies beside the model")
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(m.as_dict()), flush=True)


if __name__ == "__main__":
    main()
