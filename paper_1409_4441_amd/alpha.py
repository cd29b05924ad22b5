"""Measure alpha of Eq. 6 for this library: the actual error of the split convolution against the
full-kernel convolution, divided by the error model's estimate (Eq. 6 with alpha = 1).

    python -m paper_1409_4441_amd.alpha [--nside 512] [--paths f64,mixed] [--out alpha_512.json]

The paper fixes alpha = 5 from its own implementation (single-precision real-space convolver,
kernel interpolation; Results section, Figs. 8 and 11) and asks for it to be determined
empirically. Here, for each split (FWHM, theta_cut, l_cut) of the paper's kernels K_l = sqrt(C_l) B_l
(Eq. 9; C_l = 1/(l(l+1)) standing in for the WMAP spectrum, lmax = 2 Nside, C_in = 1):

* the split: the least-squares model (conv_split_lsq, Eqs. 3-5) gives the harmonic part K^_l (l <= l_cut)
  and the real-space part's spectrum k_real_l; the real-space table is k_real's Legendre series on the
  chord nodes (conv_real_tabulate), applied up to theta_cut by the real-space plan of the chosen path;
* the input: band-limited white noise, a_lm ~ N(0, 1) for l <= lmax, x = synthesis(a) (FP64 maps, FP32
  for the mixed path);
* full-kernel output y_full = synthesis(K a); split output y = R x + synthesis(K^ a) (harmonic half from
  the known a_lm, so that only the split and the real-space convolution contribute), and, as the
  pipeline runs it, y_hyb = conv_hybrid_apply (harmonic half from the GPU analysis of x);
* errors: map sigma_map = rms(y - y_full) / rms(y_full); spectrum sigma_P = the fractional rms of Eq. 6
  applied to the measured amplitude spectra, sqrt(sum (2l+1) K_l^2 (1 - sqrt(C_y / C_full))^2 /
  sum (2l+1) K_l^2), with C_full = |K a|^2 per l and C_y that of K a + analysis(y - y_full);
* alpha = sigma_P / sigma(Eq. 6, alpha = 1), and the same ratio for the map error.
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
SEED = 14094441 + 60


def paper_kernel(lmax: int, fwhm_arcmin: float) -> np.ndarray:
    from paper_1409_4441_amd import learn
    return learn.kernel_ell(lmax, fwhm_arcmin)


def random_alm(lmax: int, seed: int) -> np.ndarray:
    """C_in = 1: a_l0 ~ N(0, 1), Re and Im of a_lm (m > 0) ~ N(0, 1/2); m-major order."""
    g = np.random.default_rng(seed)
    n = (lmax + 1) * (lmax + 2) // 2
    a = (g.standard_normal(n) + 1j * g.standard_normal(n)) * math.sqrt(0.5)
    a[: lmax + 1] = g.standard_normal(lmax + 1)
    return a


def spectrum_error(cl_y, cl_full, K) -> float:
    ell = np.arange(len(K))
    w = (2 * ell + 1) * K * K
    ok = cl_full > 0
    r = np.zeros_like(cl_full)
    r[ok] = 1.0 - np.sqrt(np.maximum(cl_y[ok], 0.0) / cl_full[ok])
    return float(math.sqrt(np.sum(w * r * r) / np.sum(w)))


def measure(nside: int, cases, paths, n_tab: int = 4096, seed: int = SEED, log=print):
    import torch

    import paper_1409_4441_amd as cr
    from paper_1409_4441_amd import sht, split
    lmax = 2 * nside
    dev = torch.device("cuda:0")
    out = []
    a_np = random_alm(lmax, seed)
    theta_max = max(tc for _, tc, _ in cases) * 1.0001
    with sht.Sht(nside, lmax) as T, split.Context(lmax, theta_max) as ctx:
        a = torch.from_numpy(a_np).to(dev)
        x64 = T.synthesis(a)
        x32 = x64.float()
        for fwhm, tc, lc in cases:
            K = paper_kernel(lmax, fwhm)
            kh, _, kr, _ = ctx.lsq(K, lc, tc)
            _, est1 = ctx.error(K, lc, tc, alpha=1.0)
            k_hat = np.zeros(lmax + 1)
            k_hat[: lc + 1] = kh
            Kt = torch.from_numpy(K).to(dev)
            kht = torch.from_numpy(k_hat).to(dev)
            a_full = T.almxfl(a, Kt)
            y_full = T.synthesis(a_full)
            y_harm = T.synthesis(T.almxfl(a, kht))
            cl_full = T.power_spectrum(a_full).cpu().numpy()
            rms_full = float(torch.sqrt(torch.mean(y_full * y_full)))
            table = cr.tabulate(kr, tc, n_tab)
            for path in paths:
                prec = "f64" if path in ("f64", "ring_fft") else path
                x = x64 if prec == "f64" else x32
                t0 = time.perf_counter()
                with cr.Plan(nside, table, tc, prec) as plan:
                    if path == "ring_fft":
                        plan.set_method("ring_fft")
                    if prec == "mixed":
                        # wide cuts: weights on the fly (a store would take tens of GB for one apply)
                        plan.set_weight_store("off")
                    t_init = time.perf_counter() - t0
                    y_real = plan.apply(x)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    y_real = plan.apply(x, out=y_real)
                    torch.cuda.synchronize()
                    t_real = time.perf_counter() - t1
                    y_hyb = sht.hybrid_apply(plan, T, kht, x, stream_sht=torch.cuda.Stream())
                    torch.cuda.synchronize()
                    pairs = plan.pairs()
                res = {"nside": nside, "lmax": lmax, "fwhm_arcmin": fwhm, "theta_cut_arcmin": tc / ARCMIN,
                       "ell_cut": lc, "path": path, "pairs": pairs, "real_space_s": t_real, "plan_s": t_init,
                       "estimate_alpha1": est1}
                for name, y in (("known_alm", y_real.double() + y_harm), ("pipeline", y_hyb.double())):
                    e = y - y_full
                    s_map = float(torch.sqrt(torch.mean(e * e))) / rms_full
                    cl_y = T.power_spectrum(a_full + T.analysis(e)).cpu().numpy()
                    s_p = spectrum_error(cl_y, cl_full, K)
                    res[name] = {"sigma_map": s_map, "sigma_spectrum": s_p,
                                 "alpha_map": s_map / est1 if est1 > 0 else None,
                                 "alpha_spectrum": s_p / est1 if est1 > 0 else None}
                log(json.dumps(res))
                out.append(res)
                del y_real, y_hyb
    return out


def default_cases(nside: int):
    """Fig. 11's study scaled to the grid: the 7' beam at lmax 4096 with theta_cut 240', l_cut from
    1500 up; at lmax = 2 nside the beam and angles scale by 2048 / nside, l_cut by nside / 2048."""
    s = 2048.0 / nside
    fwhm = 7.0 * s
    cases = []
    for tc_am in (240.0, 120.0):
        for lc in (1500, 1750, 2000, 2250, 2500, 3000):
            cases.append((fwhm, tc_am * s * ARCMIN, int(round(lc / s))))
    return cases


TABLE1 = ((9, 1055, 360), (10, 979, 360), (12, 960, 330), (15, 961, 270))


def feasible_cases(cost_path: str):
    """Splits the method would run at Nside 2048 (lmax 4096): the split search's answers on the
    learned split's evaluation grid (FWHM 5'..10', target errors 1e-6, 1e-5, 1e-4; the measured cost
    model, alpha = 5), and Table 1's cuts for the beams whose rows meet the bound with the stand-in
    spectrum (Results section). Returns [(fwhm, theta_cut, l_cut, bound)]."""
    from paper_1409_4441_amd import learn, split
    with open(cost_path) as f:
        c = json.load(f)
    model = split.CostModel.from_dict(c)
    ns, fw, ep = learn.eval_grid()
    th, lc, _, _ = learn.scan(ns, fw, ep, model)
    cases = []
    for k in range(len(ns)):
        if th[k] > 0 and lc[k] < 2 * ns[k]:
            cases.append((float(fw[k]), float(th[k]), int(lc[k]), float(ep[k])))
    for fwhm, l_cut, tc_am in TABLE1:
        cases.append((float(fwhm), tc_am * ARCMIN, l_cut, 1e-5))
    return cases


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--paths", default="f64,mixed")
    ap.add_argument("--set", default="fig11", choices=["fig11", "feasible"])
    ap.add_argument("--cost", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_model.json"))
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.set == "feasible":
        full = feasible_cases(args.cost)
        args.nside = 2048
        cases = [c[:3] for c in full]
        bounds = {c[:3]: c[3] for c in full}
    else:
        cases = default_cases(args.nside)
        bounds = {}
    res = measure(args.nside, cases, args.paths.split(","))
    for r in res:
        key = next((c for c in cases if abs(c[0] - r["fwhm_arcmin"]) < 1e-9 and c[2] == r["ell_cut"]
                    and abs(c[1] / ARCMIN - r["theta_cut_arcmin"]) < 1e-6), None)
        if key in bounds:
            r["bound"] = bounds[key]
            r["meets_bound"] = r["pipeline"]["sigma_spectrum"] <= bounds[key]
    summary = {}
    for path in args.paths.split(","):
        for kind in ("known_alm", "pipeline"):
            vals = [r[kind]["alpha_spectrum"] for r in res if r["path"] == path and r[kind]["alpha_spectrum"]]
            vm = [r[kind]["alpha_map"] for r in res if r["path"] == path and r[kind]["alpha_map"]]
            if vals:
                summary[f"{path}/{kind}"] = {"alpha_spectrum_median": float(np.median(vals)),
                                             "alpha_spectrum_max": float(np.max(vals)),
                                             "alpha_map_median": float(np.median(vm)), "n": len(vals)}
    print(json.dumps({"summary": summary}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"cases": res, "summary": summary}, f, indent=1)


if __name__ == "__main__":
    main()
