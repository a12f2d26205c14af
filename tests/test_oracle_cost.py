"""Pins for the oracle's cost table and level histogram (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle import brute
from oracle.cost import (cost_eq1_pauli, cost_table, count_solutions_enum, level_histogram,
                         min_level, satisfying_probability)
from paper_2402_02585_amd import instances as inst

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(n, m, seed):
    return inst.random_3sat(np.random.Generator(np.random.PCG64(seed)), n, m)


def test_hand_computed_single_clauses():
    # (x0 v x1 v x2): false only when bits 0,1,2 are all 0 (App. B)
    c = cost_table(4, [[0, 2, 4]])
    assert [int(z) for z in np.nonzero(c)[0]] == [0, 8]
    # (~x0 v x1 v x2): false only when x0=1, x1=0, x2=0 -> z & 7 == 1
    c = cost_table(4, [[1, 2, 4]])
    assert [int(z) for z in np.nonzero(c)[0]] == [1, 9]
    # (~x1 v ~x2 v x3) on n=4: false iff x1=1, x2=1, x3=0 -> z in {6, 7}
    c = cost_table(4, [[3, 5, 6]])
    assert [int(z) for z in np.nonzero(c)[0]] == [6, 7]


@pytest.mark.parametrize("n,m,seed", [(3, 5, 1), (6, 20, 2), (9, 38, 3), (11, 46, 4), (12, 60, 5)])
def test_sat_count_matches_enumeration(n, m, seed):
    lits = _rand(n, m, seed)
    hist = level_histogram(cost_table(n, lits), m)
    assert hist[0] == count_solutions_enum(n, lits)


@pytest.mark.parametrize("n,m,seed", [(5, 10, 7), (10, 42, 8), (14, 59, 9), (16, 67, 10)])
def test_histogram_invariants(n, m, seed):
    lits = _rand(n, m, seed)
    hist = level_histogram(cost_table(n, lits), m)
    assert hist.sum() == 2 ** n
    # each clause on 3 distinct variables is unsatisfied on exactly 2^(n-3) z
    assert int((np.arange(m + 1) * hist).sum()) == m * 2 ** (n - 3)


@pytest.mark.parametrize("n,m,seed", [(4, 8, 11), (6, 17, 12), (8, 30, 13)])
def test_eq1_pauli_form_is_bit_complement(n, m, seed):
    lits = _rand(n, m, seed)
    text = cost_table(n, lits)
    eq1 = cost_eq1_pauli(n, lits)
    z = np.arange(2 ** n)
    comp = (~z) & (2 ** n - 1)
    np.testing.assert_array_equal(eq1, text[comp].astype(np.float64))


def test_paper_worked_instances():
    with open(os.path.join(GOLDEN, "paper_instances.json")) as f:
        gold = json.load(f)
    for key in ("4var", "5var"):
        g = gold[key]
        lits = inst.parse_paper_clauses(g["clauses"])
        n = g["n"]
        assert lits.shape == (8, 3)
        hist = level_histogram(cost_table(n, lits), lits.shape[0])
        nsat = count_solutions_enum(n, lits)
        assert hist[0] == nsat
        assert hist.sum() == 2 ** n
        assert satisfying_probability(hist, n) == nsat / 2 ** n
        assert int((np.arange(9) * hist).sum()) == 8 * 2 ** (n - 3)


@pytest.mark.parametrize("n,m,seed", [(10, 42, 21), (14, 59, 22), (16, 70, 23)])
def test_brute_c_matches_numpy(n, m, seed):
    lits = _rand(n, m, seed)
    np.testing.assert_array_equal(brute.level_histogram_brute(n, lits),
                                  level_histogram(cost_table(n, lits), m))
    c = cost_table(n, lits)
    np.testing.assert_array_equal(brute.cost_range_brute(n, lits, 3, 2 ** n - 5), c[3:-2])


def test_brute_c_invariants_large():
    n, m = 24, 101
    lits = _rand(n, m, 24)
    hist = brute.level_histogram_brute(n, lits)
    assert hist.sum() == 2 ** n
    assert int((np.arange(m + 1) * hist).sum()) == m * 2 ** (n - 3)


def test_two_level_instance():
    for n in (3, 5, 8):
        lits = inst.two_level_instance(n, keep_pattern=5)
        c = cost_table(n, lits)
        assert set(np.unique(c)) == {0, 1}
        assert (c == 0).sum() == 2 ** (n - 3)
        assert all((z & 7) == 5 for z in np.nonzero(c == 0)[0])


def test_min_level():
    assert min_level(np.array([0, 0, 3, 4])) == 2
