"""Rounds-to-target and the Max-SAT level (oracle, test infrastructure only).

Sec. III.A measures how many rounds p the protocol needs before the state
holds at least a fraction S of its probability on the target level (S = 50%,
and 25% / 75% in the appendix on angle optimization):
  * satisfiable instances, d in (2, 4.5): the target is level 0 and random
    guessing succeeds with P = N_0 / 2^n;
  * unsatisfiable instances, d in (4.6, 8): the target is the Max-SAT level
    k_min, the lowest occupied level, with D = N_{k_min} / 2^n (App. B).
The claim is p ~ 1/sqrt(P) (or 1/sqrt(D)), against 1/P for random guessing.

Reading used here: for the single-angle-pair protocol, the rounds required is
the least p for which some pair (beta, gamma) reaches P_target >= S. Over a
grid of pairs that is the minimum, over the grid, of the first round at
which each pair crosses S. The evolution is the level-space one of
``oracle.evolve.evolve_hist`` (complex128).
"""
from __future__ import annotations

import numpy as np

from .evolve import evolve_hist


def maxsat_level(hist, n: int):
    """(k_min, D): the lowest occupied level and its probability under |s>."""
    hist = np.asarray(hist)
    k = int(np.nonzero(hist)[0][0])
    return k, float(hist[k]) / float(1 << n)


def first_crossing(hist, beta: float, gamma: float, S: float, p_max: int, target: int = 0) -> int:
    """First round j in [1, p_max] after which P_target >= S under the single
    pair (beta, gamma), or 0 if it never does (Eq. (5), level space)."""
    _, psol, _, _ = evolve_hist(hist, np.full(p_max, beta), np.full(p_max, gamma), target)
    hit = np.nonzero(psol[1:] >= S)[0]
    return int(hit[0]) + 1 if hit.size else 0


def crossing_trace(hist, beta: float, gamma: float, p_max: int, target: int = 0) -> np.ndarray:
    """P_target after rounds 0..p_max (for judging how close a crossing is)."""
    return evolve_hist(hist, np.full(p_max, beta), np.full(p_max, gamma), target)[1]


def grid_rounds_to_target(hist, betas, gammas, S: float, p_max: int, target: int = 0):
    """(p_star, first[ng, nb]): first crossing of every grid pair and their
    minimum over the pairs that cross (0 if none does)."""
    first = np.array([[first_crossing(hist, b, g, S, p_max, target) for b in betas] for g in gammas],
                     dtype=np.int64)
    hits = first[first > 0]
    return (int(hits.min()) if hits.size else 0), first


def sqrt_fit(P, p):
    """Least-squares line log p = a + b log(1/P) and the median of p sqrt(P):
    returns (b, a, c) with c the constant of p ~ c / sqrt(P)."""
    P = np.asarray(P, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    x, y = np.log(1.0 / P), np.log(p)
    b, a = np.polyfit(x, y, 1)
    return float(b), float(a), float(np.median(p * np.sqrt(P)))
