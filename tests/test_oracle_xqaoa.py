"""Pins for the X-QAOA oracle (CPU only): dense expm of sum_i X_i, the single
qubit rotation closed form, invariants, and the noiseless X rows of Table I."""
import json
import os

import numpy as np
import pytest
import scipy.linalg
from scipy.optimize import minimize

from oracle.cost import cost_table, level_histogram
from oracle.xqaoa import apply_x_mixer, evolve_x
from paper_2402_02585_amd import instances as inst

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
_X = np.array([[0.0, 1.0], [1.0, 0.0]])


def _hx(n):
    H = np.zeros((2 ** n, 2 ** n))
    for q in range(n):
        op = np.array([[1.0]])
        for k in range(n - 1, -1, -1):
            op = np.kron(op, _X if k == q else np.eye(2))
        H += op
    return H


@pytest.mark.parametrize("n", [1, 3, 5])
def test_mixer_matches_dense_expm(n):
    rng = np.random.Generator(np.random.PCG64(n))
    psi = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    for beta in (0.3, 1.7, -2.2):
        ref = scipy.linalg.expm(-1j * beta * _hx(n)) @ psi
        np.testing.assert_allclose(apply_x_mixer(psi, n, beta), ref, atol=1e-12)


def test_single_qubit_rotation():
    # on one qubit, exp(-i b X)|0> = cos b |0> - i sin b |1>
    out = apply_x_mixer(np.array([1.0 + 0j, 0.0]), 1, 0.4)
    np.testing.assert_allclose(out, [np.cos(0.4), -1j * np.sin(0.4)], atol=1e-15)


def test_invariants():
    n, m = 8, 34
    lits = inst.random_3sat(np.random.Generator(np.random.PCG64(4)), n, m)
    cost = cost_table(n, lits)
    P0 = level_histogram(cost, m)[0] / 2 ** n
    beta, gamma = inst.uniform_angles(4, 6)
    # |+> is an eigenvector of H_X: gamma = 0 leaves every probability unchanged
    _, psol, _, norm = evolve_x(n, cost, beta, np.zeros(6))
    np.testing.assert_allclose(psol, P0, atol=1e-13)
    # beta = 0: only phases
    _, psol, _, _ = evolve_x(n, cost, np.zeros(6), gamma)
    np.testing.assert_allclose(psol, P0, atol=1e-13)
    _, _, _, norm = evolve_x(n, cost, beta, gamma)
    np.testing.assert_allclose(norm, 1.0, atol=1e-13)
    # beta = pi: exp(-i pi X) = -I on every qubit
    psi_a = evolve_x(n, cost, np.full(3, np.pi), gamma[:3])[0]
    psi_b = evolve_x(n, cost, np.zeros(3), gamma[:3])[0]
    np.testing.assert_allclose(np.abs(psi_a), np.abs(psi_b), atol=1e-13)


def _min_energy(n, cost, p, starts):
    best = None
    for x0 in starts:
        f = lambda x: evolve_x(n, cost, x[:p], x[p:])[2][-1]
        r = minimize(f, x0, method="L-BFGS-B", options={"ftol": 1e-10})
        if best is None or r.fun < best.fun:
            best = r
    return best.x


@pytest.mark.parametrize("key", ["4var", "5var"])
def test_table1_noiseless_xqaoa(key):
    """Table I, noiseless X rows, at energy-minimizing angles (Eq. (4)),
    +-0.3 percentage points (the printed angles are not given)."""
    with open(os.path.join(GOLDEN, "paper_instances.json")) as f:
        g = json.load(f)[key]
    n = g["n"]
    cost = cost_table(n, inst.parse_paper_clauses(g["clauses"]))
    bb, gg = np.meshgrid(np.linspace(0, np.pi, 61), np.linspace(0, np.pi, 61), indexing="ij")
    e1 = np.array([[evolve_x(n, cost, [b], [gm])[2][-1] for b, gm in zip(rb, rg)] for rb, rg in zip(bb, gg)])
    i, j = np.unravel_index(np.argmin(e1), e1.shape)
    x1 = _min_energy(n, cost, 1, [np.array([bb[i, j], gg[i, j]])])
    p1 = evolve_x(n, cost, x1[:1], x1[1:])[1][-1]
    assert 100 * p1 == pytest.approx(g["table1_noiseless_percent"]["p1_X"], abs=0.3)
    rng = np.random.Generator(np.random.PCG64(1))
    starts = [np.array([x1[0], x1[0], x1[1], x1[1]])] + [rng.uniform(0, np.pi, 4) for _ in range(12)]
    x2 = _min_energy(n, cost, 2, starts)
    p2 = evolve_x(n, cost, x2[:2], x2[2:])[1][-1]
    assert 100 * p2 == pytest.approx(g["table1_noiseless_percent"]["p2_X"], abs=0.3)
