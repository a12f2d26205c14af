"""Property tests of the oracle on random small instances (hypothesis,
derandomized so every run draws the same cases): the identities of the cost
histogram, the symmetry of the evolution from |s> (the amplitude of z depends
on C(z) only, so amplitudes within a level stay exactly equal), norm
conservation, the level-space form (App. C) against the statevector form
(Eq. (3)), and the p = 0 readout #SAT / 2^n."""
import numpy as np
from hypothesis import given, settings, strategies as st

from oracle.cost import cost_table, level_histogram
from oracle.evolve import evolve_hist, evolve_sv
from paper_2402_02585_amd import instances as inst


@st.composite
def instances(draw, n_max=9):
    n = draw(st.integers(3, n_max))
    m = draw(st.integers(1, min(40, 4 * (n * (n - 1) * (n - 2) // 6))))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    return n, inst.random_3sat(np.random.Generator(np.random.PCG64(seed)), n, m)


angles = st.lists(st.tuples(st.floats(0.0, 2 * np.pi), st.floats(0.0, np.pi)), min_size=0, max_size=6)


@settings(max_examples=60, deadline=None, derandomize=True)
@given(instances())
def test_histogram_identities(ins):
    n, lits = ins
    m = lits.shape[0]
    c = cost_table(n, lits)
    h = level_histogram(c, m)
    assert int(h.sum()) == 2 ** n
    # each clause is false on exactly 2^(n-3) assignments
    assert int((np.arange(m + 1) * h.astype(np.int64)).sum()) == m * 2 ** (n - 3)
    assert c.min() >= 0 and c.max() <= m


@settings(max_examples=60, deadline=None, derandomize=True)
@given(instances(), angles)
def test_evolution_from_s_properties(ins, ang):
    n, lits = ins
    m = lits.shape[0]
    c = cost_table(n, lits)
    h = level_histogram(c, m)
    b = np.array([a[0] for a in ang])
    g = np.array([a[1] for a in ang])
    psi, ps, en, nm = evolve_sv(n, c, b, g)
    # the same operations act on every z of one level, so their amplitudes are equal bit for bit
    for k in np.nonzero(h)[0]:
        amp = psi[c == k]
        assert (amp == amp[0]).all()
    assert np.abs(nm - 1.0).max() < 1e-12
    assert abs(ps[0] - h[0] / 2 ** n) < 1e-15
    _, hp, he, hn = evolve_hist(h, b, g)
    assert np.abs(hp - ps).max() < 1e-12
    assert np.abs(he - en).max() < 1e-12 * max(1, m)
    assert np.abs(hn - nm).max() < 1e-12
