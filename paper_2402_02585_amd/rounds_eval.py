"""Rounds-to-target experiment (Sec. III.A, Fig. 2 (a), (b), (d); the
convergence study of the angle-optimization appendix) on synthetic instances.

Workload (defaults, the paper's sizes): for every n in [10, 26], ``per_n``
(100; 50 for n >= 23) satisfiable instances with d ~ U(2, 4.5) and as many
unsatisfiable ones with d ~ U(4.6, 8) (seeded, duplicate clauses dropped as
in the paper, m = round(n d)). Angle grid: pi/180 spacing over the
fundamental domain for every n (the paper samples 4000 pairs beyond n = 20
for its energy optimization; for the first-crossing search a 90 x 45 grid
there leaves a third of the instances unreached, all of them at n > 20). Targets: level 0 for the satisfiable set (probability P = N_0 /
2^n), the Max-SAT level k_min for the unsatisfiable set (D = N_kmin / 2^n).

Reported:
  * single-angle-pair rounds to S = 50% for every instance (grid pi/180 over
    the fundamental domain, two zoom refinements), with a round cap of
    ceil(cap_c / sqrt(P)); the fit log p = a + b log(1/P) (b = 1/2 is the
    quadratic speed-up) and the median of p sqrt(P);
  * S = 25% and 75% for the n = ``conv_n`` instances (the convergence study),
    with ``--full-conv`` also full G-QAOA there;
  * full G-QAOA rounds (all 2p angles optimized by L-BFGS-B with the
    level-space adjoint gradient, bisection below the single-pair count) for
    every instance with ``full_n_min`` <= n <= ``full_n_max`` (default n <= 20:
    Sec. V compares the single-pair results at 26 qubits with full G-QAOA
    results at 20);
  * rounds against density (slope of a linear fit) for both sets;
  * the spread of the single-pair angles (median and interquartile range),
    which is the parameter clustering of Sec. III.B and its Max-SAT appendix.

Usage: python -m paper_2402_02585_amd.rounds_eval [--per-n 100] [--out file]
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
from . import rounds


def log(msg):
    print(f"[rounds] {msg}", file=sys.stderr, flush=True)


def _set(kind, n_lo, n_hi, per_n, per_n_large, workers):
    out = []
    for n in range(n_lo, n_hi + 1):
        cnt = per_n if n < 23 else per_n_large
        if kind == "sat":
            out += inst.batched_scan_instances(1000 + n, cnt, n, n, density_range=(2.0, 4.5), dup="drop",
                                               workers=workers)
        else:
            out += inst.batched_scan_instances(2000 + n, cnt, n, n, want="unsat", density_range=(4.6, 8.0),
                                               dup="drop", workers=workers)
    return out


def _quartiles(x):
    q1, q2, q3 = np.percentile(x, [25, 50, 75])
    return {"median": float(q2), "iqr": float(q3 - q1)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-lo", type=int, default=10)
    ap.add_argument("--n-hi", type=int, default=26)
    ap.add_argument("--per-n", type=int, default=100)
    ap.add_argument("--per-n-large", type=int, default=50, help="instances per n for n >= 23")
    ap.add_argument("--cap-c", type=float, default=3.0)
    ap.add_argument("--conv-n", type=int, default=16)
    ap.add_argument("--full", type=int, default=0,
                    help="full G-QAOA on a seeded subsample of this many instances per set (0: all with n <= full-n-max)")
    ap.add_argument("--full-n-min", type=int, default=0)
    ap.add_argument("--full-n-max", type=int, default=20)
    ap.add_argument("--kinds", default="sat,unsat", help="instance sets to run (sat, unsat or both)")
    ap.add_argument("--full-conv", action="store_true",
                    help="also full G-QAOA at S = 25%% and 75%% on the conv-n instances")
    ap.add_argument("--full-slice", type=int, nargs=2, default=[0, 1], metavar=("OFFSET", "STRIDE"),
                    help="full G-QAOA on every STRIDE-th eligible instance from OFFSET (to split a long run)")
    ap.add_argument("--full-grid", type=int, nargs=2, default=[120, 61],
                    help="grid of the single-pair seed at each candidate p of the full G-QAOA search")
    ap.add_argument("--grid", type=int, nargs=2, default=[360, 181], help="grid for n <= 20")
    ap.add_argument("--grid-large", type=int, nargs=2, default=[360, 181],
                    help="grid for n > 20 (the paper samples 4000 pairs there; a coarse grid misses the narrow "
                         "region of angles that reach S at large n)")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    import torch

    res = {"workload": {"n": [a.n_lo, a.n_hi], "per_n": a.per_n, "per_n_large": a.per_n_large,
                        "sat_density": [2.0, 4.5], "unsat_density": [4.6, 8.0], "grid": a.grid,
                        "grid_large": a.grid_large, "cap": f"ceil({a.cap_c}/sqrt(P))"}}
    for kind in [k for k in ("sat", "unsat") if k in a.kinds.split(",")]:
        t0 = time.perf_counter()
        its = _set(kind, a.n_lo, a.n_hi, a.per_n, a.per_n_large, a.workers)
        t_gen = time.perf_counter() - t0
        ns = np.array([it.n for it in its])
        ms = np.array([it.m for it in its])
        ds = np.array([it.d for it in its])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = g.gqaoa_hist_batched(ns, ms, [it.lits for it in its], hist_stride=int(ms.max()) + 1).cpu().numpy()
        t_hist = time.perf_counter() - t0
        if kind == "sat":
            targets = np.zeros(len(its), dtype=np.int32)
            P = H[:, 0].astype(np.float64) / np.exp2(ns)
        else:
            targets, P = rounds.maxsat_targets(ns, H)
        caps = np.clip(np.ceil(a.cap_c / np.sqrt(P)), 8, 100000).astype(np.int32)
        log(f"{kind}: {len(its)} instances generated in {t_gen:.1f} s, histograms {t_hist:.2f} s, "
            f"caps {caps.min()}..{caps.max()}")
        entry = {"instances": len(its), "hist_seconds": t_hist, "per_S": {}}
        for S in (0.5, 0.25, 0.75):
            sel = np.arange(len(its)) if S == 0.5 else np.nonzero(ns == a.conv_n)[0]
            if sel.size == 0:
                continue
            cap_s = caps[sel] * (3 if S == 0.75 else 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p_star = np.zeros(sel.size, dtype=np.int64)
            beta = np.zeros(sel.size)
            gamma = np.zeros(sel.size)
            work = 0.0
            for small in (True, False):
                part = np.nonzero((ns[sel] <= 20) == small)[0]
                if part.size == 0:
                    continue
                grid = tuple(a.grid if small else a.grid_large)
                ix = sel[part]
                p_star[part], beta[part], gamma[part] = rounds.single_pair_rounds(
                    ns[ix], ms[ix], H[ix], S, cap_s[part], targets=targets[ix], grid=grid)
                work += grid[0] * grid[1] * cap_s[part].astype(np.float64).sum()
            torch.cuda.synchronize()
            t_s = time.perf_counter() - t0
            ok = p_star > 0
            rec = {"instances": int(sel.size), "reached": int(ok.sum()), "seconds": t_s,
                   "grid_pair_round_caps_per_s": float(work / t_s)}
            if ok.sum() >= 3:
                b, icpt, c = rounds.sqrt_fit(P[sel][ok], p_star[ok])
                rec.update({"fit_slope_log_p_vs_log_inv_P": b, "fit_intercept": icpt, "median_p_sqrtP": c,
                            "p_range": [int(p_star[ok].min()), int(p_star[ok].max())],
                            "inv_P_range": [float(1 / P[sel][ok].max()), float(1 / P[sel][ok].min())]})
                if S == 0.5:
                    slope_d, icpt_d = np.polyfit(ds[sel][ok], p_star[ok], 1)
                    rec["rounds_vs_density_slope"] = float(slope_d)
                    rec["angles"] = {"beta": _quartiles(beta[ok]), "gamma": _quartiles(gamma[ok])}
                    per_n = {}
                    for n in range(a.n_lo, a.n_hi + 1):
                        mk = ok & (ns[sel] == n)
                        if mk.any():
                            per_n[str(n)] = {"median_p": float(np.median(p_star[mk])),
                                             "median_inv_sqrtP": float(np.median(1 / np.sqrt(P[sel][mk])))}
                    rec["per_n"] = per_n
            if S == 0.5:
                # per instance: n, m, d, P (or D), rounds (0: not reached within the cap), cap
                rec["records"] = [[int(ns[i]), int(ms[i]), round(float(ds[i]), 4), float(P[i]), int(p_star[k]),
                                   int(cap_s[k])] for k, i in enumerate(sel)]
            if S != 0.5 and a.full_conv and ok.sum() >= 3:
                # full G-QAOA at this target on the same n = conv_n instances
                ix = sel[ok]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pf, _, _, _, okf = rounds.full_rounds_batched(
                    ns[ix], ms[ix], H[ix], S, p_star[ok], targets=targets[ix], grid=tuple(a.full_grid))
                rec["full_gqaoa"] = {"instances": int(ix.size), "seconds": time.perf_counter() - t0,
                                     "mean_ratio_full_to_single": float(np.mean(pf / p_star[ok])),
                                     "instances_below_single": int(okf.sum()),
                                     "median_p_full": float(np.median(pf)), "median_p_single": float(np.median(p_star[ok])),
                                     "median_p_sqrtP": float(np.median(pf * np.sqrt(P[ix])))}
                log(f"{kind} S={S} full G-QAOA: mean p_full/p_single {rec['full_gqaoa']['mean_ratio_full_to_single']:.3f}")
            entry["per_S"][str(S)] = rec
            log(f"{kind} S={S}: {rec.get('reached')}/{rec['instances']} reached, slope "
                f"{rec.get('fit_slope_log_p_vs_log_inv_P', float('nan')):.3f}, c {rec.get('median_p_sqrtP', float('nan')):.3f}, "
                f"{t_s:.1f} s")
            if S == 0.5:
                p_half, b_half, g_half = p_star, beta, gamma
        # full G-QAOA (all 2p angles, level-space adjoint) on every instance with
        # n <= full_n_max that the single pair reached in more than one round
        # (or a seeded subsample of --full of them)
        pool = np.nonzero((ns >= a.full_n_min) & (ns <= a.full_n_max) & (p_half > 1))[0]
        if a.full and pool.size > a.full:
            rng = np.random.Generator(np.random.PCG64(77 if kind == "sat" else 78))
            pool = np.sort(rng.choice(pool, a.full, replace=False))
        pool = pool[a.full_slice[0]::a.full_slice[1]]
        if pool.size:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pf, _, _, Pf, okf = rounds.full_rounds_batched(
                ns[pool], ms[pool], H[pool], 0.5, p_half[pool], targets=targets[pool], grid=tuple(a.full_grid),
                progress=lambda st, c, r: log(f"{kind} full G-QAOA bisection step {st}: {c} candidates, {r} reach S"),
                on_batch=lambda k, w: k % 200 == 0 and log(f"{kind} full G-QAOA: {k} batched gradients, {w} in the last"))
            t_full = time.perf_counter() - t0
            full = [{"n": int(ns[i]), "m": int(ms[i]), "P": float(P[i]), "p_single": int(p_half[i]),
                     "p_full": int(pf[k])} for k, i in enumerate(pool)]
            rec = {"instances": len(full), "seconds": t_full, "grid": a.full_grid,
                   "mean_ratio_full_to_single": float(np.mean(pf / p_half[pool])),
                   "instances_below_single": int(okf.sum()), "records": full}
            if len(full) >= 3:
                b, icpt, c = rounds.sqrt_fit(P[pool], pf)
                rec.update({"fit_slope": b, "median_p_sqrtP": c})
                per_n = {}
                for n in np.unique(ns[pool]):
                    mk = ns[pool] == n
                    per_n[str(int(n))] = {"median_p_full": float(np.median(pf[mk])),
                                          "median_p_single": float(np.median(p_half[pool][mk]))}
                rec["per_n"] = per_n
            entry["full_gqaoa"] = rec
            log(f"{kind} full G-QAOA: {len(full)} instances, slope {rec.get('fit_slope', float('nan')):.3f}, "
                f"mean p_full/p_single {rec['mean_ratio_full_to_single']:.3f}, {t_full:.1f} s")
        res[kind] = entry
        if a.out:   # keep what is done so far
            with open(a.out, "w") as f:
                f.write(json.dumps(res, default=float) + "\n")
    out = json.dumps(res, default=float)
    print(out, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(out + "\n")


if __name__ == "__main__":
    main()
