"""Fair-sampling metrics of a solution distribution (oracle, test
infrastructure only).

Sec. IV judges how uniformly G-QAOA samples the solutions with two numbers
(the two right-hand columns of Table I):
  * shots-to-all-solutions: shots from the output distribution until every
    solution has been seen at least once (a coupon collector with unequal
    probabilities and a "not a solution" outcome), averaged over runs;
  * shots-to-reject-fairness: draws from the distribution conditioned on
    solutions until a chi-squared test rejects uniform sampling, the median
    over trials.

Readings (the paper names the metrics, not their mechanics):
  * random numbers come from SplitMix64 (Steele, Lea and Flood, 2014), used
    counter-based: draw d of run r is output number r * 2^32 + d of the
    generator seeded with ``seed``; u = (x >> 11) * 2^-53;
  * a draw picks the first category k with u < cdf[k] (cdf: running sums in
    index order); for shots, an u beyond every solution's cdf is a
    non-solution; for the conditional draws the last solution takes the rest;
  * the chi-squared test is re-run after every draw once N >= n_min draws
    were taken, rejecting when sum_k (O_k - N/K)^2 / (N/K) > crit, i.e. when
    K sum_k O_k^2 - N^2 > crit * N (the left side is an exact integer);
  * a run or trial that does not finish within its draw limit reports 0.
"""
from __future__ import annotations

import itertools

import numpy as np

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_at(seed: int, k: int) -> int:
    """Output k (k >= 0) of SplitMix64 started from state ``seed``."""
    z = (seed + (k + 1) * _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniform_at(seed: int, k: int) -> float:
    return (splitmix64_at(seed, k) >> 11) * 2.0 ** -53


def shots_to_all(p_sol, runs: int, seed: int, max_shots: int):
    """Shots until every solution is seen, per run (0: not within max_shots).
    p_sol: probability of each solution in the full output distribution."""
    p = np.asarray(p_sol, dtype=np.float64)
    K = p.size
    cdf = np.cumsum(p)
    out = []
    for r in range(runs):
        seen = set()
        res = 0
        for d in range(max_shots):
            u = uniform_at(seed, (r << 32) + d)
            k = next((i for i in range(K) if u < cdf[i]), K)
            if k < K:
                seen.add(k)
                if len(seen) == K:
                    res = d + 1
                    break
        out.append(res)
    return np.asarray(out, dtype=np.int64)


def expected_shots_to_all(p_sol) -> float:
    """Exact mean of the above by inclusion-exclusion over solution subsets:
    E[T] = sum_{S nonempty} (-1)^(|S|+1) / P(S), P(S) = sum_{i in S} p_i."""
    p = list(np.asarray(p_sol, dtype=np.float64))
    total = 0.0
    for r in range(1, len(p) + 1):
        for S in itertools.combinations(p, r):
            total += (-1) ** (r + 1) / sum(S)
    return total


def chi2_statistic(counts) -> float:
    """Pearson's statistic against the uniform distribution."""
    c = np.asarray(counts, dtype=np.float64)
    e = c.sum() / c.size
    return float(((c - e) ** 2 / e).sum())


def draws_to_reject(q_sol, trials: int, seed: int, crit: float, n_min: int, max_draws: int):
    """Draws (conditioned on solutions) until the chi-squared test rejects
    uniformity, per trial (0: not within max_draws)."""
    q = np.asarray(q_sol, dtype=np.float64)
    K = q.size
    cdf = np.cumsum(q) / q.sum()
    out = []
    for r in range(trials):
        counts = [0] * K
        res = 0
        for N in range(1, max_draws + 1):
            u = uniform_at(seed, (r << 32) + N - 1)
            k = next((i for i in range(K - 1) if u < cdf[i]), K - 1)
            counts[k] += 1
            if N >= n_min and float(K * sum(c * c for c in counts) - N * N) > crit * float(N):
                res = N
                break
        out.append(res)
    return np.asarray(out, dtype=np.int64)
