"""Angle optimization: grid search, then L-BFGS-B (oracle, test only).

Follows App. C, "Optimization": evaluate the objective on a uniform
(beta, gamma) grid (spacing pi/180 for n <= 20) or on uniformly sampled angle
pairs (n > 20), then start scipy's L-BFGS-B from the best point with a 1e-6
relative-change stopping rule. Full G-QAOA starts every round's pair from the
single-pair optimum ("the same initial seeds") and relaxes all 2p angles.

The objective is a parameter: ``"energy"`` (Eq. (4), the paper's) or
``"psol"`` (maximize the solution probability).

Pinned by a closed form: on a two-level cost the single-pair optimum is
Grover's sin^2((2p+1) theta) (tests/test_instances_and_optimizer.py). Beyond
that, the refined value is never worse than the best grid
point, and the objective is invariant under (beta, gamma) -> (-beta, -gamma)
and 2 pi shifts. Local optima of L-BFGS-B are not unique.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize

from .evolve import evolve_hist
from .grad import grad_hist


def _objective(hist, betas, gammas, objective, target):
    _, psol, energy, _ = evolve_hist(hist, betas, gammas, target)
    return float(energy[-1]) if objective == "energy" else -float(psol[-1])


def single_pair_grid(hist, p: int, betas_grid, gammas_grid, objective="psol", target=0):
    """Objective on the grid betas_grid x gammas_grid (beta-major)."""
    out = np.empty((len(betas_grid), len(gammas_grid)))
    for i, b in enumerate(betas_grid):
        for j, g in enumerate(gammas_grid):
            out[i, j] = _objective(hist, np.full(p, b), np.full(p, g), objective, target)
    return out


def optimize_single_pair(hist, p: int, betas_grid, gammas_grid, objective="psol", target=0):
    """Grid argmin (ties to the lowest (beta, gamma) index), then L-BFGS-B.

    Returns (beta, gamma, value_at_grid_best, value_refined) where value is
    the minimized objective (energy, or -P_sol).
    """
    vals = single_pair_grid(hist, p, betas_grid, gammas_grid, objective, target)
    i, j = np.unravel_index(int(np.argmin(vals)), vals.shape)
    x0 = np.array([betas_grid[i], gammas_grid[j]])

    def f(x):
        return _objective(hist, np.full(p, x[0]), np.full(p, x[1]), objective, target)

    res = minimize(f, x0, method="L-BFGS-B", options={"ftol": 1e-6})
    best = res.x if res.fun <= vals[i, j] else x0
    return float(best[0]), float(best[1]), float(vals[i, j]), float(min(res.fun, vals[i, j]))


def optimize_full(hist, beta0: float, gamma0: float, p: int, objective="psol", target=0):
    """All 2p angles by L-BFGS-B from the single-pair seed (App. C).

    For objective "psol" the exact gradient comes from ``grad_hist``.
    Returns (betas, gammas, value).
    """
    x0 = np.concatenate([np.full(p, beta0), np.full(p, gamma0)])

    if objective == "psol":
        def f(x):
            P, db, dg = grad_hist(hist, x[:p], x[p:], target)
            return -P, -np.concatenate([db, dg])
        res = minimize(f, x0, jac=True, method="L-BFGS-B", options={"ftol": 1e-6})
    else:
        def f(x):
            return _objective(hist, x[:p], x[p:], objective, target)
        res = minimize(f, x0, method="L-BFGS-B", options={"ftol": 1e-6})
    return res.x[:p].copy(), res.x[p:].copy(), float(res.fun)
