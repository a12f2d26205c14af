"""Table I, noiseless: solution probability and the two fair-sampling
metrics for X-QAOA and G-QAOA at p = 1, 2 on the paper's 4- and 5-variable
instances (the footnote of Sec. IV).

Angles minimize the energy of Eq. (4) (the paper's objective): G-QAOA p = 1
by the batched single-pair scan over the pi/180 grid with two zoom levels,
X-QAOA p = 1 over a 61 x 61 grid of [0, pi]^2, each refined by L-BFGS-B; at
p = 2 all four angles are refined by L-BFGS-B from the p = 1 pair repeated
and from 12 seeded random starts. States come from the complex128
statevector kernels; the metrics from the Monte Carlo kernels (100,000 runs
for shots-to-all-solutions, 10,000 trials for shots-to-reject-fairness,
chi-squared at the 5% level from 5 K draws on, at most 10^5 draws).

The paper's shots columns were measured on IonQ Aria; its noiseless
distributions give other numbers (G-QAOA samples its solutions exactly
uniformly), so only the noiseless solution % is compared with the paper.

Usage: python -m paper_2402_02585_amd.fairness_eval [--out file]
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np
from scipy.optimize import minimize

from . import fairness
from . import gqaoa as g
from . import instances as inst
from . import optim

# The two worked instances of Sec. IV.
PAPER_INSTANCES = {"4var": (4, inst.PAPER_4VAR), "5var": (5, inst.PAPER_5VAR)}


def log(msg):
    print(f"[fairness] {msg}", file=sys.stderr, flush=True)


def _energy_x(n, m, cost):
    def f(x):
        p = x.size // 2
        return g.gqaoa_evolve_x(n, m, cost, x[:p], x[p:], dtype=g.C128)[2][-1]
    return f


def _energy_g(n, m, hist):
    def f(x):
        p = x.size // 2
        return g.gqaoa_hist_evolve(n, m, hist, x[:p], x[p:])[1][-1]
    return f


def _best(f, starts):
    best = None
    for x0 in starts:
        r = minimize(f, x0, method="L-BFGS-B", options={"ftol": 1e-10})
        if best is None or r.fun < best.fun:
            best = r
    return best.x


def angles(kind, n, m, cost, hist):
    rng = np.random.Generator(np.random.PCG64(1))
    if kind == "G":
        f = _energy_g(n, m, hist)
        b, gm, _, _ = optim.batched_single_pair([n], [m], hist.cpu().numpy().reshape(1, -1), [1], objective="energy")
        x1 = _best(f, [np.array([b[0, 0], gm[0, 0]])])
    else:
        f = _energy_x(n, m, cost)
        grid = np.linspace(0, math.pi, 61)
        e = np.array([[f(np.array([bb, gg])) for bb in grid] for gg in grid])
        i, j = np.unravel_index(np.argmin(e), e.shape)
        x1 = _best(f, [np.array([grid[j], grid[i]])])
    starts = [np.array([x1[0], x1[0], x1[1], x1[1]])] + [rng.uniform(0, math.pi, 4) for _ in range(12)]
    x2 = _best(f, starts)
    return {1: x1, 2: x2}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=100000)
    ap.add_argument("--trials", type=int, default=10000)
    ap.add_argument("--max-draws", type=int, default=100000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    rows = []
    for key, (n, text) in PAPER_INSTANCES.items():
        lits = inst.parse_paper_clauses(text)
        m = lits.shape[0]
        cost, hist = g.gqaoa_cost_table(n, lits)
        for kind in ("X", "G"):
            ang = angles(kind, n, m, cost, hist)
            for p in (1, 2):
                x = ang[p]
                evolve = g.gqaoa_evolve_x if kind == "X" else g.gqaoa_evolve
                psi, psol, energy, _ = evolve(n, m, cost, x[:p], x[p:], dtype=g.C128)
                _, pr = fairness.solution_probs(cost, psi)
                shots = fairness.shots_to_all_solutions(pr, runs=a.runs, seed=100 + p)
                rej = fairness.shots_to_reject_fairness(pr, trials=a.trials, seed=200 + p, max_draws=a.max_draws)
                row = {"instance": key, "protocol": kind, "p": p, "betas": list(x[:p]), "gammas": list(x[p:]),
                       "energy": float(energy[-1]), "solution_percent": 100 * float(psol[-1]),
                       "solutions": int(pr.size), "max_over_min_solution_prob": float(pr.max() / pr.min()),
                       "shots_to_all_solutions": shots, "shots_to_reject_fairness": rej}
                rows.append(row)
                log(f"{key} p={p} {kind}: solution {row['solution_percent']:.1f}% | shots-to-all "
                    f"{shots['mean']:.2f}({shots['ci95']:.2f}) | reject median {rej['median']} "
                    f"(never {rej['never_rejected']}/{rej['trials']})")
    out = json.dumps({"rows": rows}, default=float)
    print(out, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(out + "\n")


if __name__ == "__main__":
    main()
