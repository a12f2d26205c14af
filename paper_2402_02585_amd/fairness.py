"""Fair-sampling metrics of output distributions (Sec. IV, Table I).

The paper rates how uniformly a protocol samples the solutions of an
instance with two numbers: the shots needed to see every solution, and the
draws from the solution distribution needed before a chi-squared test rejects
uniform sampling (median over trials). Here both are taken from noiseless
output probabilities with the library's Monte Carlo kernels
(``gqaoa_shots_to_all``, ``gqaoa_draws_to_reject``); this module selects the
solution probabilities from a device state and summarizes the runs.

G-QAOA gives every solution the same amplitude (all of them sit on level 0
of the cost), so its noiseless solution distribution is exactly uniform;
X-QAOA's is not.
"""
from __future__ import annotations

import math

import numpy as np

from . import gqaoa as g


def solution_probs(cost, psi, level: int = 0):
    """(z values, |psi_z|^2) of the assignments with C(z) = level, z ascending
    (selected on the device by ``gqaoa_level_probs``)."""
    import torch
    n = int(psi.numel()).bit_length() - 1
    dt = g.C64 if psi.dtype == torch.complex64 else g.C128
    return g.gqaoa_level_probs(n, cost, psi, dt, level)


def shots_to_all_solutions(p_sol, runs: int = 100000, seed: int = 0, max_shots: int = 1 << 30):
    """Mean shots until every solution is seen, with its 95% confidence
    half-width, over ``runs`` independent runs."""
    s = g.gqaoa_shots_to_all(p_sol, runs, seed, max_shots).cpu().numpy().astype(np.float64)
    done = s[s > 0]
    return {"mean": float(done.mean()), "ci95": float(1.96 * done.std(ddof=1) / math.sqrt(done.size)),
            "runs": int(runs), "unfinished": int(runs - done.size)}


def chi2_critical(num_solutions: int, alpha: float = 0.05) -> float:
    from scipy import stats
    return float(stats.chi2.isf(alpha, num_solutions - 1))


def shots_to_reject_fairness(p_sol, trials: int = 10000, seed: int = 1, alpha: float = 0.05, n_min: int | None = None,
                             max_draws: int = 100000):
    """Median draws until uniform sampling is rejected at level ``alpha``
    (``inf`` when at least half of the trials never reject)."""
    K = len(p_sol)
    n_min = n_min if n_min is not None else 5 * K
    d = g.gqaoa_draws_to_reject(p_sol, trials, seed, chi2_critical(K, alpha), n_min, max_draws).cpu().numpy()
    v = np.where(d > 0, d.astype(np.float64), np.inf)
    return {"median": float(np.median(v)), "trials": int(trials), "never_rejected": int((d == 0).sum()),
            "n_min": int(n_min), "max_draws": int(max_draws), "alpha": alpha}
