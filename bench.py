"""Throughput of the real-space convolution on one MI355X: pixel-pairs/s and maps/s.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload resid2048] [--precision f32]

One step = one conv_real_apply over the workload's maps, inputs already in HBM.
Prints ONE JSON line. The roofline object is for the kernel that does the
pair sums; its average launch duration comes from HIP events recorded on the
stream it runs on. The cpu_baseline object times the CPU oracle on a bounded
sample of output pixels of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pixel-pairs/s & maps/s, Nside 2048: batched MFMA vs plain FP64 @≤1e-6 rel rms"

# MI355X published peaks.
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP16_MFMA_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="resid2048")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--cpu-sample", type=int, default=400, help="output pixels the oracle sums")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def make_map(w, nmaps):
    import synth
    dt = np.float64 if w.dtype == "f64" else np.float32
    return synth.white_noise(w.nside, nmaps, seed=w.seed, dtype=dt), "white N(0,1)"


def cpu_baseline(w, table, x, y_gpu, nsamp):
    """The oracle, as it stands, on nsamp sampled output pixels of the same map; single thread."""
    from threadpoolctl import threadpool_limits

    from oracle import convolve as oc
    g = np.random.default_rng(w.seed + 99)
    pix = np.sort(g.choice(x.shape[1], nsamp, replace=False))
    counts, _ = oc.pair_counts_sampled(w.nside, w.theta_cut, pix)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ref = oc.convolve_sampled(w.nside, table, w.theta_cut, x.astype(np.float64), pix)
        dt = time.perf_counter() - t0
    pairs = float(counts.sum()) * x.shape[0]
    err = oc.rel_rms(y_gpu[:, pix], ref.reshape(x.shape[0], -1))
    return {"value": pairs / dt, "unit": "pixel-pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{nsamp} seeded output pixels x {x.shape[0]} map(s) of {w.name} "
                      f"({int(counts.sum())} pairs/map), ring-exhaustive NumPy FP64, {dt:.2f} s"}, err


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); the real-space convolution of one map runs on one device, "
              "and sharding by latitude band is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1409_4441_amd as cr
    import synth

    w = synth.workload(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    table = cr.tabulate(w.k_ell(), w.theta_cut, w.n_tab)
    x_np, map_desc = make_map(w, w.nmaps)
    if args.precision == "f64":
        x_np = x_np.astype(np.float64)
    t0 = time.perf_counter()
    plan = cr.Plan(w.nside, table, w.theta_cut, args.precision)
    init_s = time.perf_counter() - t0
    pairs_per_map = plan.pairs()
    x = torch.from_numpy(x_np).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.apply(x, out=y, stream=stream)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.apply(x, out=y, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = 1e3 * wall / args.steps

    nmaps = x.shape[0]
    total_pairs = pairs_per_map * nmaps
    value = total_pairs * args.steps / wall
    maps_per_s = nmaps * args.steps / wall

    # Dominant kernel: the per-pair FP64 sum. Algorithmic work: one multiply-add (2 flops) per
    # pixel pair per map, against the FP64 vector peak (the path is FP64 ALU-bound).
    achieved_tflops = 2.0 * total_pairs / (kern_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP64_TFLOPS, "traffic": None,
                "kernel": "pair_accumulate_kernel", "kernel_ms": kern_ms,
                "algorithmic": "2 flop per pixel pair per map"}
    elem = x.element_size()
    hbm_gbs = 2.0 * elem * w.nside * w.nside * 12 * nmaps / (kern_ms * 1e-3) / 1e9

    y_np = y.cpu().numpy()
    cpu = None
    err = None
    if not args.no_cpu:
        cpu, err = cpu_baseline(w, table, x_np, y_np, args.cpu_sample)

    out = {
        "metric": METRIC, "value": value, "unit": "pixel-pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "nside": w.nside, "npix": 12 * w.nside ** 2, "nmaps": nmaps,
                   "theta_cut_arcmin": w.theta_cut / synth.ARCMIN, "fwhm_arcmin": w.fwhm / synth.ARCMIN,
                   "ell_cut": w.ell_cut, "lmax": w.lmax, "n_tab": w.n_tab, "map": map_desc,
                   "maps_dtype": args.precision if args.precision == "f64" else "f32",
                   "path": "plain FP64 per-pair (CONV_REAL_%s)" % args.precision.upper()},
        "maps_per_s": maps_per_s, "pairs_per_map": pairs_per_map, "init_s": init_s,
        "achieved_hbm_gbs": hbm_gbs,
        "rel_rms_vs_oracle_sample": err,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
