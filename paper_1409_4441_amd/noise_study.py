"""Splits under Wiener-filter input weights: how far noise at high l relaxes the split (the paper's
Conclusions: with noise dominating the high-l regime the splits reach speedups of order 20, against
12-15 for the flat, noise-free weights of the Results section).

    python -m paper_1409_4441_amd.noise_study [--out noise_study.json]

Kernels K_l = sqrt(C_l) B_l (Eq. 9; C_l = 1/(l(l+1)) standing in for WMAP, Gaussian beam B_l), lmax 4096
(Nside 2048). The input weights of Eqs. 2 and 6 are C^in = 1 (Results section) or the Wiener weights
C^in = S^2 / (S + N) (text after Eq. 2) for the beam-smoothed signal S_l = C_l B_l^2 and white noise N
equal to S at a crossover multipole l_n (noise dominates above it). For each case the split scan
(theta_cut 30'..390' in steps of 30', the range of Table 1; the smallest l_cut meeting the bound by
bisection; compensation limit 1e-2 and l_cut <= 0.45 lmax for a split with a real-space part;
alpha = 5; bound 1e-5) picks the cheapest split under

* the paper's cost models (Eqs. 7-8: GTX 480 real-space convolver, one CPU core for the harmonic part):
  speedup = 160 s / max(t_gpu, t_cpu), the ratio the paper quotes;
* this library's measured model (cost_model.json: mixed-precision real-space path and the GPU harmonic
  convolution on one MI355X): speedup = t_sht(lmax) / wall.
The error of every split is the library's (conv_split_error with the case's weights).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ARCMIN = math.pi / (180.0 * 60.0)
LMAX = 4096
NSIDE = 2048
THETAS = tuple(30.0 * k for k in range(1, 14))   # arcmin
MAX_COMP = 1e-2
MAX_ELL_FRAC = 0.45


def paper_cost(theta_arcmin: float, ell_cut: int):
    """Eqs. 7-8 (seconds): GPU real-space part, one-core harmonic part, wall = the slower."""
    t_gpu = 0.0232 * theta_arcmin + 2.428
    t_cpu = 160.0 * ell_cut ** 2 * LMAX / 4096.0 ** 3
    return t_gpu, t_cpu, max(t_gpu, t_cpu)


def wiener_weights(fwhm_arcmin: float, ell_n: int | None):
    """C^in for the case: 1 (no noise) or S^2 / (S + N) with N = S_{ell_n}, S = C_l B_l^2."""
    from paper_1409_4441_amd import learn, split
    if ell_n is None:
        return None
    ell = np.arange(LMAX + 1, dtype=np.float64)
    c = np.zeros(LMAX + 1)
    c[2:] = 1.0 / (ell[2:] * (ell[2:] + 1.0))
    S = c * learn.beam(LMAX, fwhm_arcmin) ** 2
    return split.wiener_weights(S, S[ell_n])


def scan(ctx, K, bound, cost, alpha=5.0, step=8):
    """For each theta, the smallest l_cut (multiple of step, or lmax) whose Eq. 6 error meets the
    bound, bisected; above MAX_ELL_FRAC lmax or with a compensation above MAX_COMP, only the
    all-harmonic split; the cheapest
    pair by cost(theta_arcmin, l_cut)[2]. Returns (theta_arcmin, l_cut, wall, sigma)."""
    cands = list(range(0, LMAX, step)) + [LMAX]
    best = None
    for th in THETAS:
        tc = th * ARCMIN

        def sig(i):
            return ctx.error(K, cands[i], tc, alpha=alpha)[1]
        lo, hi = -1, len(cands) - 1
        if sig(0) <= bound:
            hi = 0
        else:
            lo = 0
            while hi - lo > 1:
                mid = (lo + hi) // 2
                if sig(mid) <= bound:
                    hi = mid
                else:
                    lo = mid
        lc = cands[hi]
        if lc < LMAX and (lc > MAX_ELL_FRAC * LMAX or ctx.compensation(K, lc, tc) > MAX_COMP):
            lc = LMAX
        s = 0.0 if lc == LMAX else ctx.error(K, lc, tc, alpha=alpha)[1]
        wall = cost(th, lc)[2]
        if best is None or wall < best[2]:
            best = (th, lc, wall, s)
    return best


def study(cost_json: str, fwhms=(7.0, 8.0, 9.0, 10.0), ell_ns=(None, 3000, 2000, 1500, 1000), bound=1e-5):
    from paper_1409_4441_amd import learn, split
    with open(cost_json) as f:
        c = json.load(f)
    model = split.CostModel.from_dict(c)
    t_full_here = model.eval(NSIDE, LMAX, 1e-3, LMAX)[1]
    rows = []
    for ell_n in ell_ns:
        for fwhm in fwhms:
            K = learn.kernel_ell(LMAX, fwhm)
            c_in = wiener_weights(fwhm, ell_n)
            with split.Context(LMAX, max(THETAS) * ARCMIN * 1.0001, c_in=c_in) as ctx:
                th, lc, wall, s = scan(ctx, K, bound, paper_cost)
                th2, lc2, wall2, s2 = scan(ctx, K, bound,
                                           lambda t, l: model.eval(NSIDE, LMAX, t * ARCMIN, l))
            rows.append({"fwhm_arcmin": fwhm, "noise_crossover_ell": ell_n,
                         "paper_model": {"theta_cut_arcmin": th, "ell_cut": lc, "wall_s": wall, "sigma": s,
                                         "speedup": 160.0 / wall},
                         "measured_model": {"theta_cut_arcmin": th2, "ell_cut": lc2, "wall_s": wall2, "sigma": s2,
                                            "speedup": t_full_here / wall2}})
            r = rows[-1]
            print(f"FWHM {fwhm:4.1f}' noise l_n {str(ell_n):>5s}: paper model ({th:5.0f}', {lc:4d}) "
                  f"speedup {r['paper_model']['speedup']:6.2f} | MI355X model ({th2:5.0f}', {lc2:4d}) "
                  f"speedup {r['measured_model']['speedup']:6.2f}", flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--cost", default=os.path.join(here, "cost_model.json"))
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    rows = study(args.cost)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
