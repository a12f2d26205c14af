"""Seeded input generator checks and the optimizer oracle's properties (CPU)."""
import numpy as np
import pytest

from oracle.cost import cost_table, count_solutions_enum, level_histogram
from oracle.evolve import psol_single_pair_hist
from oracle.optimize import optimize_single_pair, single_pair_grid
from paper_2402_02585_amd import instances as inst


def test_generator_shape_and_rules():
    rng = np.random.Generator(np.random.PCG64(0))
    lits = inst.random_3sat(rng, 10, 42)
    assert lits.shape == (42, 3) and lits.dtype == np.int32
    var = lits >> 1
    assert (var >= 0).all() and (var < 10).all()
    assert all(len(set(v)) == 3 for v in var.tolist())
    keys = {tuple(sorted(c)) for c in lits.tolist()}
    assert len(keys) == 42


def test_generator_is_deterministic():
    a = inst.first_satisfiable(1, 10, 42)
    b = inst.first_satisfiable(1, 10, 42)
    np.testing.assert_array_equal(a.lits, b.lits)
    assert a.draw == b.draw
    c = inst.draw_at(1, 10, 42, a.draw)
    np.testing.assert_array_equal(a.lits, c.lits)


def test_impossible_clause_count_raises():
    rng = np.random.Generator(np.random.PCG64(3))
    with pytest.raises(ValueError):
        inst.random_3sat(rng, 3, 9)                      # only 8 distinct clauses on 3 variables
    assert inst.random_3sat(rng, 3, 8).shape == (8, 3)


def test_drop_mode_can_shrink():
    rng = np.random.Generator(np.random.PCG64(3))
    lits = inst.random_3sat(rng, 3, 8, dup="drop")     # only 8 distinct clauses exist
    assert lits.shape[0] <= 8


def test_m_from_density():
    assert inst.m_from_density(10, 4.2) == 42
    assert inst.m_from_density(28, 4.2) == 118
    assert inst.m_from_density(20, 4.25) == 85
    assert inst.m_from_density(13, 4.5) == 59          # 58.5 rounds up


@pytest.mark.parametrize("seed", range(12))
def test_dpll_agrees_with_enumeration(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(5, 12))
    m = int(n * rng.choice([3.0, 4.2, 5.5, 7.0]))
    lits = inst.random_3sat(rng, n, m)
    assert inst.dpll_satisfiable(n, lits) == (count_solutions_enum(n, lits) > 0)


def test_parse_paper_notation():
    lits = inst.parse_paper_clauses("[-0, +2, +3], [+0, -2, 4]")
    np.testing.assert_array_equal(lits, [[1, 4, 6], [0, 5, 8]])


def test_batched_instances():
    insts = inst.batched_scan_instances(3, 12, 8, 12)
    assert len(insts) == 12
    for it in insts:
        assert 8 <= it.n <= 12 and it.d in (3.0, 4.2, 5.0)
        assert it.m == inst.m_from_density(it.n, it.d)
        assert level_histogram(cost_table(it.n, it.lits), it.m)[0] > 0


def test_optimizer_refines_and_is_symmetric():
    n, m, p = 10, 42, 4
    it = inst.first_satisfiable(5, n, m)
    hist = level_histogram(cost_table(n, it.lits), m)
    gb = np.linspace(0, 2 * np.pi, 24, endpoint=False)
    gg = np.linspace(0, np.pi, 12)
    b, g, v_grid, v_ref = optimize_single_pair(hist, p, gb, gg, objective="psol")
    assert v_ref <= v_grid + 1e-15
    assert psol_single_pair_hist(hist, b, g, p) == pytest.approx(-v_ref, abs=1e-12)
    grid = single_pair_grid(hist, p, gb, gg)
    mirror = single_pair_grid(hist, p, -gb, -gg)
    np.testing.assert_allclose(grid, mirror, atol=1e-13)


@pytest.mark.parametrize("N0,n,p", [(4, 10, 1), (4, 10, 3), (16, 12, 5), (1, 8, 2)])
def test_optimizer_reaches_grover_bound_on_two_levels(N0, n, p):
    """A two-level cost (solutions at level 0, every other assignment at
    level 1) makes the single-pair protocol a p-query search with a phase
    oracle: no angle pair can beat Grover's sin^2((2p+1) theta), sin^2 theta =
    N0 / 2^n (optimality of Grover search for symmetric algorithms, Zalka
    1999), and (beta, gamma) = (pi, pi) is Grover's iteration, which reaches
    it. So the optimizer's maximum must be that closed form, not less, and
    no grid point may exceed it."""
    hist = np.array([N0, 2 ** n - N0], dtype=np.int64)
    theta = np.arcsin(np.sqrt(N0 / 2 ** n))
    bound = np.sin((2 * p + 1) * theta) ** 2
    assert (2 * p + 1) * theta <= np.pi / 2          # below the first Grover peak
    gb = np.linspace(0, 2 * np.pi, 48, endpoint=False)
    gg = np.linspace(0, np.pi, 25)
    b, g, v_grid, v_ref = optimize_single_pair(hist, p, gb, gg, objective="psol")
    assert -v_ref == pytest.approx(bound, abs=1e-6)
    assert -single_pair_grid(hist, p, gb, gg).min() <= bound + 1e-12
    assert psol_single_pair_hist(hist, np.pi, np.pi, p) == pytest.approx(bound, abs=1e-12)
    # a grid that misses (pi, pi): the L-BFGS-B refinement has to climb to the bound
    gb2 = np.linspace(0.05, 2 * np.pi + 0.05, 47, endpoint=False)
    gg2 = np.linspace(0.03, np.pi - 0.03, 23)
    b2, g2, v_grid2, v_ref2 = optimize_single_pair(hist, p, gb2, gg2, objective="psol")
    assert -v_grid2 < bound - 1e-9
    assert -v_ref2 == pytest.approx(bound, abs=1e-5)
    assert -v_ref2 <= bound + 1e-12
