"""Measure the constants of the split cost model on this machine and write them as JSON.

    python -m paper_1409_4441_amd.calibrate [--out cost_model.json] [--quick]

Real-space part: conv_real_apply of the mixed-precision path on one white-noise map, for Gaussian
beams over Nside 256..2048, FWHM 5'..30' and theta_cut 4..8 sigma; times from HIP events around the
applies, pair counts exact (conv_real_pairs). Fitted: t_real = a + b pairs.
Harmonic part: the seeded-input package's host spherical-harmonic synthesis (OpenMP) at several
(Nside, l_cut); a harmonic convolution is an analysis and a synthesis of the same size, so its time
is taken as twice the synthesis. Fitted: t_sht = c l_cut^2 lmax with lmax = 2 Nside.
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
            for ns in (4.0, 8.0):
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
    import synth
    cases = [(256, 128), (256, 512), (512, 512), (512, 1024)] if quick else \
        [(256, 256), (256, 512), (512, 512), (512, 1024), (1024, 1024), (1024, 2048)]
    pts = []
    for nside, lc in cases:
        alm = synth.draw_alm(synth.red_spectrum(lc), seed=nside + lc)
        synth.synthesize(nside, alm, lc)             # warm-up
        t0 = time.perf_counter()
        synth.synthesize(nside, alm, lc)
        t = 2.0 * (time.perf_counter() - t0)
        pts.append({"nside": nside, "ell_cut": lc, "lmax": 2 * nside, "seconds": t})
        print(f"harmonic nside {nside} l_cut {lc}: {t:.3f} s", flush=True)
    return pts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_model.json"))
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    from paper_1409_4441_amd import split
    real = real_space_points(args.quick)
    harm = harmonic_points(args.quick)
    m = split.CostModel.fit([p["pairs"] for p in real], [p["seconds"] for p in real],
                            [p["ell_cut"] ** 2 * p["lmax"] for p in harm], [p["seconds"] for p in harm])
    out = {"a": m.a, "b": m.b, "c": m.c, "threads": os.cpu_count(),
           "real_space": real, "harmonic": harm,
           "note": "t_real = a + b pairs (mixed-precision path, one map); "
                   "t_sht = c l_cut^2 lmax (twice the host synthesis time)"}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"a": m.a, "b": m.b, "c": m.c}), flush=True)


if __name__ == "__main__":
    main()
