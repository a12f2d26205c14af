"""Pins for the fair-sampling oracle (CPU only): SplitMix64's published
outputs, the coupon-collector closed forms, Monte Carlo against the exact
mean, and the chi-squared statistic against scipy."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle.fairness import (chi2_statistic, draws_to_reject, expected_shots_to_all, shots_to_all,
                             splitmix64_at, uniform_at)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.json")) as f:
        g = json.load(f)
    for k, h in enumerate(g["outputs_hex"]):
        assert splitmix64_at(g["seed"], k) == int(h, 16)


def test_uniforms_in_unit_interval_and_spread():
    u = np.array([uniform_at(7, k) for k in range(20000)])
    assert (u >= 0).all() and (u < 1).all()
    assert abs(u.mean() - 0.5) < 0.01
    counts = np.histogram(u, bins=20, range=(0, 1))[0]
    assert stats.chisquare(counts).pvalue > 1e-4


def test_exact_mean_closed_forms():
    # one solution: geometric, mean 1/p
    assert expected_shots_to_all([0.2]) == pytest.approx(5.0, rel=1e-12)
    # K equally likely solutions of total mass P: (K / P) * H_K
    for K, P in [(2, 1.0), (5, 0.8), (8, 0.3)]:
        H = sum(1.0 / i for i in range(1, K + 1))
        assert expected_shots_to_all([P / K] * K) == pytest.approx(K / P * H, rel=1e-10)
    # two unequal solutions: 1/p1 + 1/p2 - 1/(p1 + p2)
    assert expected_shots_to_all([0.1, 0.3]) == pytest.approx(10 + 1 / 0.3 - 2.5, rel=1e-12)


def test_monte_carlo_mean_matches_exact():
    p = np.array([0.3, 0.15, 0.2, 0.05])
    runs = 3000
    s = shots_to_all(p, runs, seed=11, max_shots=10000)
    assert (s > 0).all()
    exact = expected_shots_to_all(p)
    assert abs(s.mean() - exact) < 5 * s.std() / math.sqrt(runs)


def test_chi2_statistic_matches_scipy():
    counts = [12, 7, 30, 1, 9]
    assert chi2_statistic(counts) == pytest.approx(stats.chisquare(counts).statistic, rel=1e-12)
    # the integer form used for the decision equals the statistic times N
    N, K = sum(counts), len(counts)
    assert (K * sum(c * c for c in counts) - N * N) / N == pytest.approx(chi2_statistic(counts), rel=1e-12)


def test_rejection_fast_for_skewed_and_slow_for_uniform():
    crit = stats.chi2.isf(0.05, 3)
    skew = draws_to_reject([0.97, 0.01, 0.01, 0.01], 50, seed=3, crit=crit, n_min=20, max_draws=2000)
    assert (skew > 0).all() and np.median(skew) <= 25
    flat = draws_to_reject([0.25] * 4, 50, seed=3, crit=crit, n_min=20, max_draws=60)
    # under uniform sampling each test rejects with probability about 5%
    assert (flat == 0).mean() > 0.3
