"""Learned single-pair angles at scale: train on optimizer labels, infer on new
instances, and compare with the optimizers and the clustering-only baseline.

Workload (defaults): training instances from SeedSequence(5), n ~ U{12..20},
d ~ U{3.0, 4.2, 5.0}, satisfiable; labels are the batched optimizer's
P_sol-maximizing pairs over the fundamental domain (the paper's pi/180 grid,
then two zoom levels) at p in {1, 4, 16, 64}. Inference instances from SeedSequence(6),
n ~ U{12..24}. Reported, per p and overall:

* mean P_sol of the learned pair, of the learned pair plus four shrinking
  16 x 16 local window scans, of the fixed cluster-median pair (clustering alone), of the
  batched optimizer (all inference instances) and of the plain per-instance
  optimizer (a seeded subsample);
* instances per second of each form on the GPU, the fallback count (instances
  whose learned pair plus windows stays below 0.99 of the cluster-median pair
  go to the plain optimizer, inside the learned form's timed region).

Usage: python -m paper_2402_02585_amd.learned_eval [--train N] [--test N] [--out file]
       [--save ckpt.npz] [--load ckpt.npz]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import gqaoa as g
from . import instances as inst
from . import learned, optim

P_LIST = [1, 4, 16, 64]


def log(msg):
    print(f"[learned] {msg}", file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--test", type=int, default=65536)
    ap.add_argument("--plain", type=int, default=16, help="instances for the plain optimizer")
    ap.add_argument("--plain-grid", type=int, nargs=2, default=[360, 181],
                    help="beta x gamma grid of the plain optimizer (default: the paper's pi/180 spacing)")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save", default=None, help="write the trained network and its optimizer state (.npz)")
    ap.add_argument("--load", default=None, help="start from a saved network; --steps more training steps (0: none)")
    a = ap.parse_args(argv)

    t0 = time.perf_counter()
    train = inst.batched_scan_instances(5, a.train, 12, 20, workers=a.workers)
    test = inst.batched_scan_instances(6, a.test, 12, 24, workers=a.workers)
    log(f"generated {a.train} + {a.test} instances in {time.perf_counter() - t0:.1f} s")

    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, Y, lab = learned.training_set(train, P_LIST)
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    log(f"labels for {a.train} x {len(P_LIST)} in {t_label:.2f} s")
    model = learned.AngleMLP.load(a.load) if a.load else learned.AngleMLP(seed=0)
    t0 = time.perf_counter()
    losses = model.train(X, Y, steps=a.steps, batch=a.batch, lr=1e-3, log_every=max(1, a.steps // 8))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if losses:
        log(f"trained {a.steps} steps in {t_train:.2f} s; loss {losses[0][1]:.4f} -> {losses[-1][1]:.4f}")
    else:
        losses = [(0, float("nan"))]
    if a.save:
        model.save(a.save)
    med = learned.cluster_median(lab, P_LIST)

    ns = [it.n for it in test]
    ms = [it.m for it in test]
    I = len(test)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hd = g.gqaoa_hist_batched(ns, ms, [it.lits for it in test], hist_stride=max(ms) + 1)
    H = hd.cpu().numpy()
    t_hist = time.perf_counter() - t0

    res = {"workload": {"train": a.train, "test": a.test, "train_n": "12..20", "test_n": "12..24",
                        "densities": [3.0, 4.2, 5.0], "p_list": P_LIST},
           "label_seconds": t_label, "train_seconds": t_train, "train_steps": a.steps,
           "loss_first_last": [losses[0][1], losses[-1][1]], "hist_seconds": t_hist, "per_p": {}}

    # batched optimizer on every inference instance
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ob, og, op, _ = optim.batched_single_pair(ns, ms, H, P_LIST)
    torch.cuda.synchronize()
    t_opt = time.perf_counter() - t0

    # learned: features -> MLP -> pair; the learned form adds the local windows
    # and the plain-optimizer fallback (learned.solve)
    t_learn = t_win = 0.0
    rng = np.random.Generator(np.random.PCG64(7))
    sub = rng.choice(I, min(a.plain, I), replace=False)
    total = {"learned": 0.0, "window": 0.0, "median": 0.0, "optimizer": 0.0}
    fallbacks = 0
    for q, p in enumerate(P_LIST):
        # warm the scan autotuner's cache for this p's shapes (one-pair scans
        # and window plans) on a few instances, outside the timed region
        learned.solve(model, hd[:64], ns[:64], ms[:64], H[:64], p, med[p])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = learned.features_for(hd, ns, ms, p)
        bl, gl = model.angles(x)
        p_learn = learned.evaluate_pairs(ns, ms, H, bl, gl, p)
        torch.cuda.synchronize()
        t_learn += time.perf_counter() - t0
        t0 = time.perf_counter()
        sol = learned.solve(model, hd, ns, ms, H, p, med[p], plain_grid=tuple(a.plain_grid))
        torch.cuda.synchronize()
        t_win += time.perf_counter() - t0
        p_win, p_med, fb = sol["psol"], sol["psol_median"], sol["fallback"]
        fallbacks += int(fb.sum())
        # plain optimizer on the subsample (one device call per evaluation)
        plain_p, plain_t = [], 0.0
        gb, gg = optim.fundamental_grid(*a.plain_grid)
        for i in sub:
            hdev = hd[i, :ms[i] + 1].contiguous()
            t0 = time.perf_counter()
            r = optim.plain_single_pair(ns[i], ms[i], hdev, p, gb, gg)
            plain_t += time.perf_counter() - t0
            plain_p.append(r["psol"])
        plain_p = np.asarray(plain_p)
        res["per_p"][str(p)] = {
            "mean_psol_learned": float(p_learn.mean()), "mean_psol_learned_window": float(p_win.mean()),
            "fallbacks": int(fb.sum()),
            "mean_psol_cluster_median": float(p_med.mean()), "mean_psol_batched_optimizer": float(op[:, q].mean()),
            "ratio_learned_window_to_optimizer": float(p_win.mean() / op[:, q].mean()),
            "ratio_learned_to_median": float(p_learn.mean() / p_med.mean()),
            "plain_subsample": {"instances": int(len(sub)), "mean_psol_plain": float(plain_p.mean()),
                                "mean_psol_learned_window_same": float(p_win[sub].mean()),
                                "mean_psol_batched_optimizer_same": float(op[sub, q].mean()),
                                "ratio_learned_window_to_plain": float(p_win[sub].mean() / plain_p.mean()),
                                "seconds_per_instance": plain_t / len(sub)},
            "cluster_median_pair": list(med[p]),
        }
        total["learned"] += p_learn.mean()
        total["window"] += p_win.mean()
        total["median"] += p_med.mean()
        total["optimizer"] += op[:, q].mean()
        log(f"p={p}: learned {p_learn.mean():.4f} window {p_win.mean():.4f} median {p_med.mean():.4f} "
            f"optimizer {op[:, q].mean():.4f} | subsample: plain {plain_p.mean():.4f} "
            f"learned+window {p_win[sub].mean():.4f} optimizer {op[sub, q].mean():.4f}")
    plain_sec = np.mean([res["per_p"][str(p)]["plain_subsample"]["seconds_per_instance"] for p in P_LIST])
    res["throughput_instances_per_s"] = {
        "learned": I * len(P_LIST) / t_learn, "learned_window": I * len(P_LIST) / t_win,
        "batched_optimizer": I * len(P_LIST) / t_opt, "plain_optimizer": 1.0 / plain_sec}
    res["speedup_learned_window_vs_plain"] = res["throughput_instances_per_s"]["learned_window"] / (1.0 / plain_sec)
    res["speedup_learned_window_vs_batched_optimizer"] = t_opt / t_win
    res["fallbacks"] = fallbacks
    res["mean_over_p"] = {k: v / len(P_LIST) for k, v in total.items()}
    res["ratio_window_to_optimizer_mean_over_p"] = total["window"] / total["optimizer"]
    out = json.dumps(res, default=float)
    print(out, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(out + "\n")


if __name__ == "__main__":
    main()
