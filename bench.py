"""Throughput of the real-space convolution on one MI355X: pixel-pairs/s and maps/s.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload resid2048] [--precision mixed]

One step = one conv_real_apply over the workload's maps (the whole real-space convolution),
inputs already in HBM. Prints ONE JSON line:
  value          pixel pairs per second of the timed path (exact pair count x maps / wall time)
  maps_per_s     maps per second
  plain_fp64     the plain FP64 per-pair kernel on the same map, timed beside it
  ring_fft_fp64  the FP64 ring-FFT method (belt ring pairs in Fourier space, cap-touching pairs per
                 pair) on the same map promoted to FP64, timed beside it
  roofline       the kernel that takes most of the step, timed with HIP events recorded between
                 the library's kernels on the stream they run on (conv_real_profile)
  cpu_baseline   the C FP64 oracle on the host cores over a bounded sample of output pixels of the
                 same workload (the NumPy oracle on one core beside it); the same sums check the
                 timed path's accuracy, and the batched workload's maps are checked at their own
                 sampled pixels
  split_convolution  the whole split convolution (real-space half + harmonic half on two streams)
                 against the full-kernel harmonic convolution, both with this library's kernels
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
    ap.add_argument("--precision", default="mixed", choices=["mixed", "f32", "f64"])
    ap.add_argument("--plain-steps", type=int, default=3, help="timed applies of the plain kernel")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=5000000,
                    help="output pixels the C oracle sums (timed baseline and accuracy check)")
    ap.add_argument("--cpu-sample-numpy", type=int, default=400, help="of those, pixels the NumPy oracle sums")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-ringfft", action="store_true", help="skip the FP64 ring-FFT measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-map batched measurement")
    ap.add_argument("--no-split", action="store_true", help="skip the whole split convolution (hybrid) leg")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--weight-store", default="auto", choices=["auto", "on", "off"],
                    help="cap weight store of the mixed plan (auto: the library's default)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain device copy of the map (reference for HBM counters)")
    return ap.parse_args()


def make_map(w, nmaps):
    import synth
    desc = {"white": "white N(0,1)",
            "red": f"Gaussian random field C_l = 1/(l(l+1)), 2 <= l <= {w.map_lmax}",
            "red+noise": f"Gaussian random field C_l = 1/(l(l+1)), 2 <= l <= {w.map_lmax}, "
                         f"plus white noise of {w.noise_frac:g} x the field's rms"}[w.map_kind]
    return synth.workload_maps(w, nmaps), desc


def time_applies(plan, x, y, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        plan.apply(x, out=y, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        plan.apply(x, out=y, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / steps


def kernel_table(plan, x, y, reps, stream):
    """Average per-kernel milliseconds and pixel pairs over reps profiled applies."""
    acc = {}
    for _ in range(reps):
        _, stages = plan.profile(x, out=y, stream=stream)
        for name, ms, work in stages:
            a = acc.setdefault(name, [0.0, 0])
            a[0] += ms
            a[1] = work
    return {k: {"ms": v[0] / reps, "pairs": v[1]} for k, v in acc.items()}


TRAFFIC_NOTE = os.path.join(ROOT, "profiles", "traffic_mixed_persistent_resid2048.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1409_4441_amd", "csrc", f) for f in ("mixed.hip", "internal.h", "common.h")]


def kernel_source_hash() -> str:
    """SHA-256 over the persistent kernel's sources with comments removed and whitespace runs folded
    to one space, so that only a change of the code itself voids the committed traffic figure."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the persistent kernel from the committed FETCH_SIZE / WRITE_SIZE
    summary, or None if that summary was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_NOTE):
        return None
    vals = {}
    for line in open(TRAFFIC_NOTE):
        if ":" in line and line.split(":", 1)[0].strip() in ("source_sha256", "hbm_bytes_per_launch"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash() or "hbm_bytes_per_launch" not in vals:
        return None
    return float(vals["hbm_bytes_per_launch"])


def roofline_for(name, ms, pairs, map_bytes, traffic_applies=False):
    """Roofline of the dominant kernel per launch. Algorithmic bytes: one read of every input map and
    one write of every output map (map_bytes in total); algorithmic flops: 2 per pixel pair per map.
    The binding roofline is the one with the larger floor time (bytes / 8 TB/s against flops / the
    peak of the unit used); at Nside 2048, 30' that is HBM (50.3 us against 38.6 us of FP16 matrix
    work). The other one is reported beside it."""
    flops = 2.0 * pairs
    sec = ms * 1e-3
    if "mfma" in name or "persistent" in name:
        peak_flops, funit = PEAK_FP16_MFMA_TFLOPS, "FP16 matrix"
    else:
        peak_flops, funit = PEAK_FP64_TFLOPS, "FP64 vector"
    t_hbm = map_bytes / (PEAK_HBM_GBS * 1e9)
    t_flop = flops / (peak_flops * 1e12)
    hbm = {"bound": "hbm", "achieved": map_bytes / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": map_bytes / sec / 1e9 / PEAK_HBM_GBS, "floor_us": t_hbm * 1e6,
           "algorithmic": f"{map_bytes} bytes per launch (FP32 maps read once and written once)"}
    fl = {"bound": "mfma" if "FP16" in funit else "alu", "achieved": flops / sec / 1e12, "peak": peak_flops,
          "unit": "TFLOP/s", "frac": flops / sec / 1e12 / peak_flops, "floor_us": t_flop * 1e6,
          "algorithmic": f"{flops:.6g} flop per launch (2 per pixel pair, {funit} peak)"}
    bind, other = (hbm, fl) if t_hbm >= t_flop else (fl, hbm)
    out = dict(bind)
    # the committed traffic figure is for the persistent kernel on one resid2048 map in its default
    # configuration (the plan holding its weight store)
    out.update({"traffic": measured_traffic() if traffic_applies and "persistent" in name else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-kernel scaled)",
                "kernel": name, "kernel_ms": ms, "other_roofline": other})
    return out


def batched(steps, stream):
    """The batched workload: 32 maps of uneven Nside and beam in one persistent launch per step,
    tiles autotuned by the library, the apply captured in a HIP graph and replayed."""
    import torch

    import paper_1409_4441_amd as cr
    import synth
    ws = synth.batch_workload()
    t0 = time.perf_counter()
    maps = synth.batch_maps(ws)
    t_maps = time.perf_counter() - t0
    plans = []
    t0 = time.perf_counter()
    for w in ws:
        table = cr.tabulate(w.k_ell(), w.theta_cut, w.n_tab)
        plans.append(cr.Plan(w.nside, table, w.theta_cut, "mixed"))
    init_s = time.perf_counter() - t0
    xs = [torch.from_numpy(m).to("cuda:0") for m in maps]
    outs = [torch.empty_like(x) for x in xs]
    batch = cr.Batch(plans)
    pairs = batch.pairs()
    t0 = time.perf_counter()
    best = batch.autotune(xs)
    tune_s = time.perf_counter() - t0
    for _ in range(2):
        batch.apply(xs, outs=outs, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        batch.apply(xs, outs=outs, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / steps
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.apply(xs, outs=outs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        batch.apply(xs, outs=outs)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) / steps
    host = [(w, m, o.cpu().numpy()) for w, m, o in zip(ws, maps, outs)]
    counts = {}
    for w in ws:
        counts[w.nside] = counts.get(w.nside, 0) + 1
    out = {"workload": "batch32", "nmaps": len(ws), "nsides": {str(k): v for k, v in sorted(counts.items())},
           "pairs_per_batch": pairs, "tuning": best, "autotune_s": tune_s, "init_s": init_s, "maps_s": t_maps,
           "eager_ms_per_batch": eager_ms, "graph_ms_per_batch": graph_s * 1e3,
           "pixel_pairs_per_s": pairs / graph_s, "maps_per_s": len(ws) / graph_s,
           "maps": "even white N(0,1), odd red C_l = 1/(l(l+1)) (one field per Nside)"}
    batch.close()
    for p in plans:
        p.close()
    return out, host


def split_convolution(w, plan, x, stream, reps: int = 3):
    """The whole split convolution of the workload (Eq. 1, Fig. 1): the real-space half (the timed
    plan, the beam's residual B_l (1 - g_l) truncated at theta_cut) plus the harmonic half (B_l g_l,
    band limit l_cut + w/2) on a second stream, against the full-kernel harmonic convolution with B_l
    at lmax. Times from HIP events; the accuracy is the whole-map relative rms difference of the two
    (what the split and its truncation at theta_cut cost)."""
    import torch

    import synth
    from paper_1409_4441_amd import sht
    beam = synth.gaussian_beam(w.lmax, w.fwhm)
    L_h = int(math.ceil(w.ell_cut + 0.5 * w.taper_width))
    k_hat = (beam - w.k_ell())[: L_h + 1].copy()
    side = torch.cuda.Stream()
    out = {"harmonic_band_limit": L_h, "lmax": w.lmax}
    with sht.Sht(w.nside, L_h) as T, sht.Sht(w.nside, w.lmax) as F:
        kh = torch.from_numpy(k_hat).to(x.device)
        kb = torch.from_numpy(beam).to(x.device)
        y = sht.hybrid_apply(plan, T, kh, x, stream=stream, stream_sht=side)
        yf = F.convolve(x[0], kb, stream=stream)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        e[0].record(stream)
        for _ in range(reps):
            sht.hybrid_apply(plan, T, kh, x, out=y, stream=stream, stream_sht=side)
        e[1].record(stream)
        for _ in range(reps):
            plan.apply(x, out=y, stream=stream)
        e[2].record(stream)
        for _ in range(reps):
            T.convolve(x[0], kh, out=yf, stream=stream)
        e[3].record(stream)
        for _ in range(reps):
            F.convolve(x[0], kb, out=yf, stream=stream)
        e[4].record(stream)
        torch.cuda.synchronize()
        sht.hybrid_apply(plan, T, kh, x, out=y, stream=stream, stream_sht=side)
        torch.cuda.synchronize()
        diff = torch.sqrt(torch.sum((y[0].double() - yf.double()) ** 2) / torch.sum(yf.double() ** 2)).item()
        t = [e[k].elapsed_time(e[k + 1]) / reps for k in range(4)]
    out.update({"hybrid_two_streams_ms": t[0], "real_space_ms": t[1], "harmonic_half_ms": t[2],
                "full_harmonic_ms": t[3], "speedup_vs_full_harmonic": t[3] / t[0],
                "rel_rms_vs_full_harmonic": diff,
                "note": "harmonic half and full convolution: this library's FP64 GPU transforms"})
    return out


def paper_context(theta_cut, pairs_per_map, maps_per_s):
    """The paper's cost model for its GPU real-space convolution (Eq. 7, fitted on a GeForce GTX 480
    in single precision, Nside 2048, l_max 4096): t = 0.0232 s per arcminute of theta_cut + 2.428 s.
    Context for the figures measured here, not a target (it is a model of another design on other
    hardware)."""
    t = 0.0232 * math.degrees(theta_cut) * 60.0 + 2.428
    return {"source": "Eq. 7 cost model, GeForce GTX 480, single precision, Nside 2048",
            "seconds_per_map": t, "maps_per_s": 1.0 / t, "pixel_pairs_per_s_implied": pairs_per_map / t,
            "ratio_maps_per_s_here": maps_per_s * t}


def check_pixels(nside: int, n: int, seed: int) -> np.ndarray:
    """n seeded uniform output pixels plus the first, middle and last pixel of the two rings at
    each pole and of the rings on both sides of each belt edge (sorted, unique)."""
    N = int(nside)
    npix = 12 * N * N

    def ring_start_len(i):
        if i < N:
            return 2 * i * (i - 1), 4 * i
        if i <= 3 * N:
            return 2 * N * (N - 1) + 4 * N * (i - N), 4 * N
        k = 4 * N - i
        return npix - 2 * k * (k + 1), 4 * k

    rings = {1, 2, N - 1, N, N + 1, 2 * N, 3 * N - 1, 3 * N, 3 * N + 1, 4 * N - 2, 4 * N - 1}
    extra = []
    for i in sorted(r for r in rings if 1 <= r <= 4 * N - 1):
        s0, n_i = ring_start_len(i)
        extra += [s0, s0 + n_i // 2, s0 + n_i - 1]
    rnd = np.random.default_rng(seed).choice(npix, min(n, npix), replace=False)
    return np.unique(np.concatenate([rnd, np.asarray(extra, dtype=np.int64)]))


def _cpu_threads() -> int:
    """Host threads for the C oracle: every core this process may use, at most 16 (a GPU machine's
    CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, x, y_gpu, nsamp, nsamp_numpy, batch_outputs=None):
    """The oracle, as it stands, on the host: the C FP64 oracle on all host cores over nsamp seeded
    output pixels of the same map (the timed baseline, and the accuracy check of the timed path on
    those pixels), the NumPy oracle on one core over nsamp_numpy of them (timed beside it), and,
    for the batched workload, each map's output against the C oracle at its check pixels. The
    oracle tabulates its own kernel tables."""
    from threadpoolctl import threadpool_limits

    from oracle import convolve as oc
    from oracle import csum
    from oracle import kernel as ok
    table = ok.tabulate(w.k_ell(), w.theta_cut, w.n_tab)
    g = np.random.default_rng(w.seed + 99)
    npix = x.shape[1]
    pix = np.sort(g.choice(npix, min(nsamp, npix), replace=False))
    nt = _cpu_threads()
    xd = x.astype(np.float64)
    t0 = time.perf_counter()
    ref, counts = csum.convolve_sampled(w.nside, table, w.theta_cut, xd, pix, nthreads=nt)
    dt = time.perf_counter() - t0
    pairs = float(counts.sum()) * x.shape[0]
    yg = y_gpu[:, pix].astype(np.float64)
    err = max(oc.rel_rms(yg[m], ref[m]) for m in range(x.shape[0]))
    err_max = max(float(np.max(np.abs(yg[m] - ref[m])) / np.sqrt(np.mean(ref[m] ** 2))) for m in range(x.shape[0]))
    sub = pix[np.random.default_rng(w.seed + 98).choice(len(pix), min(nsamp_numpy, len(pix)), replace=False)]
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        ref_np = oc.convolve_sampled(w.nside, table, w.theta_cut, xd, sub).reshape(x.shape[0], -1)
        dt_np = time.perf_counter() - t1
    counts_np, _ = oc.pair_counts_sampled(w.nside, w.theta_cut, sub)
    cpu = {"value": pairs / dt, "unit": "pixel-pairs/s", "cores": nt, "kind": "oracle",
           "sample": f"{len(pix)} seeded output pixels x {x.shape[0]} map(s) of {w.name} "
                     f"({int(counts.sum())} pairs), C FP64 oracle (oracle/csum.c) on {nt} threads, {dt:.2f} s; "
                     f"host os.cpu_count() = {os.cpu_count()}",
           "numpy_oracle": {"value": float(counts_np.sum()) * x.shape[0] / dt_np, "unit": "pixel-pairs/s",
                            "cores": 1, "sample": f"{len(sub)} of those pixels, ring-exhaustive NumPy FP64, "
                                                  f"{dt_np:.2f} s"}}
    acc = {"pixels": int(len(pix)), "rel_rms": err, "max_abs_over_rms": err_max,
           "numpy_vs_c_oracle_rel_rms": max(oc.rel_rms(ref_np[m], ref[m][np.searchsorted(pix, sub)])
                                             for m in range(x.shape[0]))}
    if batch_outputs is not None:
        worst, npx = 0.0, 0
        for k, (wb, xb, yb) in enumerate(batch_outputs):
            tb = ok.tabulate(wb.k_ell(), wb.theta_cut, wb.n_tab)
            pb = check_pixels(wb.nside, 300, wb.seed + 7 * k)
            rb, _ = csum.convolve_sampled(wb.nside, tb, wb.theta_cut, xb.astype(np.float64), pb, nthreads=nt)
            e = oc.rel_rms(yb[pb].astype(np.float64), rb[0])
            worst, npx = max(worst, e), npx + len(pb)
        acc["batched"] = {"maps": len(batch_outputs), "pixels": npx, "worst_map_rel_rms": worst,
                          "pixels_per_map": "300 seeded + first/middle/last of the polar and belt-edge rings"}
    return cpu, acc


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}, "
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
    if args.precision == "mixed" and args.weight_store != "auto":
        plan.set_weight_store(args.weight_store)
    init_s = time.perf_counter() - t0
    pairs_per_map = plan.pairs()
    x = torch.from_numpy(x_np).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    nmaps = x.shape[0]

    wall, apply_ms = time_applies(plan, x, y, args.steps, args.warmup, stream)
    value = pairs_per_map * nmaps * args.steps / wall
    maps_per_s = nmaps * args.steps / wall

    store = None
    if args.precision == "mixed":
        active, nbytes = plan.weight_store()
        store = {"active": active, "bytes": nbytes}
        # the other mode, timed beside the chosen one (a few applies), then restored
        other = "off" if active else "on"
        try:
            plan.set_weight_store(other)
            _, ms_other = time_applies(plan, x, y, 5, 1, stream)
            store["ms_" + ("store_off" if active else "store_on")] = ms_other
        except Exception as exc:  # the device may not hold a store of this size
            store["other_mode_error"] = str(exc)
        plan.set_weight_store("on" if active else "off")
        store["ms_" + ("store_on" if active else "store_off")] = apply_ms

    kernels = kernel_table(plan, x, y, args.profile_steps, stream)
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    default_run = (args.workload == "resid2048" and nmaps == 1 and args.precision == "mixed"
                   and store is not None and store["active"])
    roofline = roofline_for(dom, kernels[dom]["ms"], kernels[dom]["pairs"], 2 * x.element_size() * x.numel(),
                            traffic_applies=default_run)
    hbm_gbs = 2.0 * x.element_size() * x.numel() / (apply_ms * 1e-3) / 1e9

    plan.apply(x, out=y, stream=stream)
    torch.cuda.synchronize()
    y_np = y.cpu().numpy()

    plain = None
    if not args.no_plain and args.precision != "f64":
        with cr.Plan(w.nside, table, w.theta_cut, "f32") as pf:
            yf = torch.empty_like(x)
            wall_f, ms_f = time_applies(pf, x, yf, args.plain_steps, 1, stream)
            diff = torch.sqrt(torch.sum((y.double() - yf.double()) ** 2) / torch.sum(yf.double() ** 2)).item()
        plain = {"ms_per_map": 1e3 * wall_f / (args.plain_steps * nmaps),
                 "pixel_pairs_per_s": pairs_per_map * nmaps * args.plain_steps / wall_f,
                 "maps_per_s": nmaps * args.plain_steps / wall_f,
                 "speedup_of_timed_path": (wall_f / args.plain_steps) / (wall / args.steps),
                 "rel_rms_timed_path_vs_plain": diff,
                 "kernel": "pair_accumulate_kernel<float> (FP64 per pair)"}

    ring_fft = None
    if not args.no_ringfft and args.precision != "f64" and (w.nside & (w.nside - 1)) == 0 and w.nside <= 2048:
        xd = x.double()
        yd = torch.empty_like(xd)
        with cr.Plan(w.nside, table, w.theta_cut, "f64") as pd:
            t1 = time.perf_counter()
            pd.set_method("ring_fft")
            setup_s = time.perf_counter() - t1
            wall_d, ms_d = time_applies(pd, xd, yd, args.plain_steps, 1, stream)
            kern_d = kernel_table(pd, xd, yd, 1, stream)
        diff_d = torch.sqrt(torch.sum((y.double() - yd) ** 2) / torch.sum(yd ** 2)).item()
        ring_fft = {"ms_per_map": 1e3 * wall_d / (args.plain_steps * nmaps),
                    "pixel_pairs_per_s": pairs_per_map * nmaps * args.plain_steps / wall_d,
                    "maps_per_s": nmaps * args.plain_steps / wall_d, "setup_s": setup_s, "kernels": kern_d,
                    "rel_rms_timed_path_vs_ring_fft": diff_d,
                    "method": "FP64 maps: belt ring pairs as per-frequency products of ring spectra, "
                              "cap-touching ring pairs on the FP64 matrix cores, each weight once for its 16 "
                              "symmetric images"}
        del xd, yd

    if args.copy_probe:
        # one plain device-to-device copy of the map: a kernel of known traffic (read + write of
        # x.nbytes) whose HBM counters scale the counters of the library's kernels
        yc = torch.empty_like(x)
        yc.copy_(x)
        torch.cuda.synchronize()
        del yc

    split_conv = None
    if not args.no_split and w.ell_cut > 0 and args.precision != "f64" and nmaps == 1:
        split_conv = split_convolution(w, plan, x, stream)

    bat, bat_host = None, None
    if not args.no_batched and args.precision == "mixed":
        bat, bat_host = batched(args.batched_steps, stream)

    cpu = None
    acc = None
    if not args.no_cpu:
        cpu, acc = cpu_baseline(w, x_np, y_np, args.cpu_sample, args.cpu_sample_numpy, bat_host)
        if bat is not None and "batched" in acc:
            bat["oracle_check"] = acc.pop("batched")

    path = {"mixed": "split-FP16 matrix cores: precomputed Toeplitz weights for belt ring pairs, cap-touching "
                     "ring pairs with weights shared by 16 symmetric images (stored or evaluated on the fly), "
                     "one persistent launch",
            "f32": "plain FP64 per-pair (FP32 maps)", "f64": "plain FP64 per-pair (FP64 maps)"}[args.precision]
    out = {
        "metric": METRIC, "value": value, "unit": "pixel-pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"mixed": "f16", "f32": "f64", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "nside": w.nside, "npix": 12 * w.nside ** 2, "nmaps": nmaps,
                   "theta_cut_arcmin": w.theta_cut / synth.ARCMIN, "fwhm_arcmin": w.fwhm / synth.ARCMIN,
                   "ell_cut": w.ell_cut, "lmax": w.lmax, "n_tab": w.n_tab, "map": map_desc,
                   "maps_dtype": "f64" if args.precision == "f64" else "f32", "path": path},
        "maps_per_s": maps_per_s, "pairs_per_map": pairs_per_map, "init_s": init_s,
        "apply_ms_events": apply_ms, "achieved_hbm_gbs": hbm_gbs,
        "kernels": kernels,
        "accuracy_vs_oracle": acc,
        "plain_fp64": plain,
        "ring_fft_fp64": ring_fft,
        "weight_store": store,
        "batched": bat,
        "split_convolution": split_conv,
        "roofline": roofline, "cpu_baseline": cpu,
        "paper_context": paper_context(w.theta_cut, pairs_per_map, maps_per_s) if w.nside == 2048 else None,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
