"""Train the learned split on the device and write its parameters and held-out evaluation as JSON.

    python -m paper_1409_4441_amd.train_split [--cost cost_model.json] [--out learned_split.json]

Data: 2000 training and 200 held-out (Nside, FWHM, target error) triples (Nside uniform over
256..2048, FWHM log-uniform 5'..30', error log-uniform 1e-6..1e-4), seeded; labels are the split
search's answers under the measured cost model (conv_split_search_many on host threads). Training:
full-batch Adam on the library's kernels, learning rate stepped down 3e-3 -> 1e-3 -> 3e-4.
Evaluation on the held-out triples and on the evaluation grid (Nside 2048, FWHM 5'..10', target
errors 1e-6..1e-4): how often the network's split meets the bound (judged by the error model), its
modelled wall time against the search's, and the time each takes to decide.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAIN_SEED = 14094441 + 50
TEST_SEED = 14094441 + 51
INIT_SEED = 14094441 + 52
SCHEDULE = ((3000, 3e-3), (3000, 1e-3), (2000, 3e-4))


def labels(triples, model):
    from paper_1409_4441_amd import learn
    ns, fw, ep = triples
    t0 = time.perf_counter()
    th, lc, wl, sg = learn.scan(ns, fw, ep, model)
    return th, lc, wl, sg, time.perf_counter() - t0


def evaluate(pred, triples, scan_result, model):
    """Held-out metrics of a Predictor against the search's splits."""
    import torch
    from paper_1409_4441_amd import learn
    ns, fw, ep = triples
    th_s, lc_s, wl_s, _ = scan_result
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th_n, lc_n = pred.network_split(ns, fw, ep)
    t_net = time.perf_counter() - t0
    accepted, ratio, t_judge = [], [], 0.0
    for k in range(len(ns)):
        t1 = time.perf_counter()
        _, ok = pred.judge(int(ns[k]), float(fw[k]), float(ep[k]), float(th_n[k]), int(lc_n[k]))
        t_judge += time.perf_counter() - t1
        accepted.append(bool(ok))
        if ok:
            _, _, w = model.eval(int(ns[k]), 2 * int(ns[k]), min(float(th_n[k]), pred.ctxs[int(ns[k])].theta_max),
                                 int(lc_n[k]))
            ratio.append(w / wl_s[k])
    # a fixed rule for comparison: theta_cut = 6 sigma, l_cut = 0.3 / sigma
    fixed_ok, fixed_ratio = 0, []
    for k in range(len(ns)):
        s = learn.sigma_of(float(fw[k]))
        th, lc = 6.0 * s, int(min(2 * int(ns[k]), round(0.3 / s)))
        _, ok = pred.judge(int(ns[k]), float(fw[k]), float(ep[k]), th, lc)
        if ok:
            fixed_ok += 1
            fixed_ratio.append(model.eval(int(ns[k]), 2 * int(ns[k]), th, lc)[2] / wl_s[k])
    t0 = time.perf_counter()
    learn.scan(ns, fw, ep, model, ctxs=pred.ctxs, nthreads=1)
    t_scan = time.perf_counter() - t0
    n = len(ns)
    return {
        "n": n,
        "accepted": int(sum(accepted)),
        "acceptance_rate": float(np.mean(accepted)),
        "wall_ratio_accepted_mean": float(np.mean(ratio)) if ratio else None,
        "wall_ratio_accepted_median": float(np.median(ratio)) if ratio else None,
        "wall_ratio_accepted_p90": float(np.percentile(ratio, 90)) if ratio else None,
        "seconds_per_decision_network": t_net / n,
        "seconds_per_decision_judge": t_judge / n,
        "seconds_per_decision_search": t_scan / n,
        "fixed_rule_acceptance_rate": fixed_ok / n,
        "fixed_rule_wall_ratio_mean": float(np.mean(fixed_ratio)) if fixed_ratio else None,
        "label_ell_cut_fraction_zero": float(np.mean(lc_s == 0)),
        "label_ell_cut_fraction_lmax": float(np.mean(lc_s == 2 * ns)),
    }


def main():
    ap = argparse.ArgumentParser()
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--cost", default=os.path.join(here, "cost_model.json"))
    ap.add_argument("--out", default=os.path.join(here, "learned_split.json"))
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-test", type=int, default=200)
    args = ap.parse_args()

    import torch

    from paper_1409_4441_amd import learn, split
    with open(args.cost) as f:
        c = json.load(f)
    model = split.CostModel.from_dict(c)

    train = learn.draw_triples(args.n_train, TRAIN_SEED)
    test = learn.draw_triples(args.n_test, TEST_SEED)
    th, lc, wl, sg, t_lab = labels(train, model)
    print(f"labels: {args.n_train} training triples in {t_lab:.1f} s", flush=True)
    test_scan = labels(test, model)[:4]

    raw = learn.raw_targets(th, lc, train[0], train[1])
    norm = learn.fit_norm(raw)
    x = torch.tensor(learn.features(*train), dtype=torch.float32, device="cuda").contiguous()
    t = torch.tensor(learn.encode(raw, norm), dtype=torch.float32, device="cuda").contiguous()
    net = learn.Network(max_batch=args.n_train)
    net.set_params(learn.init_params(INIT_SEED))
    hist = []
    t0 = time.perf_counter()
    for steps, lr in SCHEDULE:
        hist.append(net.train(x, t, steps=steps, lr=lr).cpu().numpy())
        print(f"  {steps} steps at lr {lr:g}: loss {float(hist[-1][-1]):.4g}", flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    hist = np.concatenate(hist)
    params = net.get_params()
    net.close()

    pred = learn.Predictor(params, norm, model)
    metrics = evaluate(pred, test, test_scan, model)
    grid = learn.eval_grid()
    grid_metrics = evaluate(pred, grid, labels(grid, model)[:4], model)
    pred.close()
    meta = {"norm": norm, "cost_model": model.as_dict(),
            "train": {"n": args.n_train, "seed": TRAIN_SEED, "init_seed": INIT_SEED,
                      "schedule": [list(s) for s in SCHEDULE], "seconds": t_train,
                      "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
                      "loss_every_500": [float(v) for v in hist[::500]]},
            "test": {"seed": TEST_SEED, **metrics},
            "eval_grid": {"triples": "Nside 2048 x FWHM 5'..10' (1' steps) x target error 1e-6, 1e-5, 1e-4",
                          **grid_metrics},
            "labels": {"alpha": learn.ALPHA, "max_compensation": learn.MAX_COMP,
                       "ell_cut_fraction_lmax": float(np.mean(lc == 2 * train[0])),
                       "ell_cut_fraction_zero": float(np.mean(lc == 0))}}
    learn.save(args.out, params, meta)
    print(json.dumps({"test": meta["test"], "eval_grid": meta["eval_grid"], "labels": meta["labels"]}), flush=True)


if __name__ == "__main__":
    main()
