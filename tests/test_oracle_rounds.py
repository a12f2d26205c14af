"""Pins for the rounds-to-target and Max-SAT oracle (CPU only): the Grover
closed form on two-level instances (for level 0 and for a Max-SAT level),
agreement with the statevector definition, the no-crossing case, and the
fit on exact 1/sqrt(P) data."""
import math

import numpy as np
import pytest

from oracle.cost import cost_table, level_histogram
from oracle.evolve import evolve_sv
from oracle.rounds import first_crossing, grid_rounds_to_target, maxsat_level, sqrt_fit
from paper_2402_02585_amd import instances as inst


def _grover_rounds(P, S):
    """Least j >= 1 with sin^2((2j+1) theta) >= S, sin^2 theta = P (before the
    first maximum, which these cases reach first)."""
    theta = math.asin(math.sqrt(P))
    j = max(1, math.ceil((math.asin(math.sqrt(S)) / theta - 1) / 2))
    assert math.sin((2 * j + 1) * theta) ** 2 >= S
    return j


@pytest.mark.parametrize("S", [0.25, 0.5, 0.75])
@pytest.mark.parametrize("levels,target", [((0, 1), 0), ((3, 4), 3), ((5, 6), 5)])
def test_two_level_grover_closed_form(S, levels, target):
    # two adjacent occupied levels: gamma = pi is a -1 phase on one of them,
    # beta = pi makes the mixer the reflection 1 - 2|s><s|: Grover's iteration
    n = 16
    hist = np.zeros(8, dtype=np.int64)
    hist[levels[0]] = 37
    hist[levels[1]] = (1 << n) - 37
    P = 37 / (1 << n)
    assert first_crossing(hist, math.pi, math.pi, S, 400, target) == _grover_rounds(P, S)


def test_maxsat_level():
    hist = np.array([0, 0, 12, 30, 22], dtype=np.int64)
    assert maxsat_level(hist, 6) == (2, 12 / 64)


def test_unsat_instance_has_positive_kmin():
    # an unsatisfiable draw above the threshold: N_0 = 0 and k_min >= 1
    its = inst.batched_scan_instances(11, 3, 8, 10, want="unsat", density_range=(4.6, 8.0), dup="drop")
    for it in its:
        h = level_histogram(cost_table(it.n, it.lits), it.m)
        assert h[0] == 0
        k, D = maxsat_level(h, it.n)
        assert k >= 1 and 0 < D < 1
        assert 4.6 <= it.d <= 8.0 and it.m <= inst.m_from_density(it.n, it.d)


@pytest.mark.parametrize("seed", [1, 2])
def test_crossing_matches_statevector_definition(seed):
    n, m = 9, 38
    lits = inst.first_satisfiable(seed, n, m).lits
    cost = cost_table(n, lits)
    hist = level_histogram(cost, m)
    for beta, gamma in [(2.9, 0.6), (1.3, 2.2), (math.pi, math.pi)]:
        for target in (0, 1):
            j = first_crossing(hist, beta, gamma, 0.3, 60, target)
            _, ps, _, _ = evolve_sv(n, cost, np.full(60, beta), np.full(60, gamma), target=target)
            hit = np.nonzero(ps[1:] >= 0.3)[0]
            assert j == (hit[0] + 1 if hit.size else 0)


def test_no_crossing_returns_zero():
    hist = np.array([3, 100, 200, 40], dtype=np.int64)
    # beta = 0: the mixer is the identity and P_0 never moves from 3/343
    assert first_crossing(hist, 0.0, 1.0, 0.5, 50) == 0
    p_star, first = grid_rounds_to_target(hist, [0.0], [0.5, 1.0], 0.5, 20)
    assert p_star == 0 and (first == 0).all()


def test_sqrt_fit_recovers_exact_scaling():
    P = np.logspace(-6, -2, 9)
    p = 0.33 / np.sqrt(P)
    b, a, c = sqrt_fit(P, p)
    assert b == pytest.approx(0.5, abs=1e-12)
    assert c == pytest.approx(0.33, rel=1e-12)
    assert math.exp(a) == pytest.approx(0.33, rel=1e-9)
