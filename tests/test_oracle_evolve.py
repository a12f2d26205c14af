"""Pins for the oracle's G-QAOA evolution (CPU only).

Each test checks the oracle against something other than itself: a dense
matrix exponential of the Pauli-form Hamiltonians, closed forms derived from
Eq. (3), Grover's rotation formula, symmetries, and Table I of the paper.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle.cost import cost_table, level_histogram
from oracle.evolve import evolve_hist, evolve_sv, psol_single_pair_hist
from oracle.optimize import optimize_full, optimize_single_pair
from paper_2402_02585_amd import instances as inst

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(n, m, seed):
    return inst.random_3sat(np.random.Generator(np.random.PCG64(seed)), n, m)


def _rand_state(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    return v / np.linalg.norm(v)


# ---- dense reference: Pauli matrices, Kronecker products, expm -------------

_I2 = np.eye(2)
_X = np.array([[0.0, 1.0], [1.0, 0.0]])
_Z = np.array([[1.0, 0.0], [0.0, -1.0]])


def _on_qubit(op, q, n):
    """op acting on qubit q (bit q of the index; qubit 0 is the last factor)."""
    out = np.array([[1.0]])
    for k in range(n - 1, -1, -1):
        out = np.kron(out, op if k == q else _I2)
    return out


def _dense_hamiltonians(n, lits):
    dim = 2 ** n
    HP = np.zeros((dim, dim))
    for clause in lits:
        term = np.eye(dim) / 8.0
        for lit in clause:
            s = -1.0 if lit & 1 else 1.0
            term = term @ (np.eye(dim) - s * _on_qubit(_Z, lit >> 1, n))
        HP += term
    HM = np.eye(dim)
    for q in range(n):
        HM = HM @ ((np.eye(dim) + _on_qubit(_X, q, n)) / 2.0)
    return HP, HM


@pytest.mark.parametrize("n,m,p,seed", [(3, 4, 3, 1), (4, 9, 4, 2), (5, 14, 3, 3), (6, 20, 5, 4)])
def test_statevector_matches_dense_expm(n, m, p, seed):
    """Eq. (3) evaluated with dense expm of Eq. (1) and Eq. (2) Hamiltonians.

    Eq. (1)'s Pauli form labels the text's assignment z by its complement ~z;
    the Grover mixer is invariant under that relabeling.
    """
    lits = _rand(n, m, seed)
    beta, gamma = inst.uniform_angles(seed + 100, p)
    HP, HM = _dense_hamiltonians(n, lits)
    comp = (~np.arange(2 ** n)) & (2 ** n - 1)
    psi0 = _rand_state(n, seed + 7)
    dense = psi0[comp].astype(np.complex128)
    for b, g in zip(beta, gamma):
        dense = scipy.linalg.expm(-1j * b * HM) @ (scipy.linalg.expm(-1j * g * HP) @ dense)
    cost = cost_table(n, lits)
    psi, psol, energy, norm = evolve_sv(n, cost, beta, gamma, psi0=psi0)
    np.testing.assert_allclose(psi, dense[comp], atol=1e-12)
    # the default initial state is |+>
    plus = np.ones(2 ** n) / 2 ** (n / 2)
    assert np.allclose(HM @ plus, plus)


@pytest.mark.parametrize("n,m,seed", [(8, 34, 5), (10, 42, 6), (12, 50, 7)])
def test_p0_and_trivial_angles(n, m, seed):
    lits = _rand(n, m, seed)
    cost = cost_table(n, lits)
    hist = level_histogram(cost, m)
    P0 = hist[0] / 2 ** n
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.uniform(0, np.pi, 6)
    b = rng.uniform(0, np.pi, 6)
    for beta, gamma in [(np.zeros(6), g), (2 * np.pi * np.ones(6), g), (b, np.zeros(6)),
                        (b, 2 * np.pi * np.ones(6))]:
        _, psol, _, norm = evolve_sv(n, cost, beta, gamma)
        np.testing.assert_allclose(psol, P0, atol=1e-13)
        np.testing.assert_allclose(norm, 1.0, atol=1e-13)
    _, psol, energy, _ = evolve_sv(n, cost, b, g)
    assert psol[0] == pytest.approx(P0, abs=1e-15)
    # E at p=0 is m/8 (each clause is unsatisfied on 1/8 of the assignments)
    assert energy[0] == pytest.approx(m / 8.0, abs=1e-12)


@pytest.mark.parametrize("n,m,p,seed", [(8, 34, 7, 8), (11, 46, 12, 9), (13, 55, 20, 10)])
def test_level_space_equals_statevector(n, m, p, seed):
    lits = _rand(n, m, seed)
    cost = cost_table(n, lits)
    hist = level_histogram(cost, m)
    beta, gamma = inst.uniform_angles(seed, p)
    psi, psol, energy, norm = evolve_sv(n, cost, beta, gamma)
    b, psol_h, energy_h, norm_h = evolve_hist(hist, beta, gamma)
    np.testing.assert_allclose(psi, b[cost] / 2 ** (n / 2), atol=1e-14)
    np.testing.assert_allclose(psol, psol_h, atol=1e-13)
    np.testing.assert_allclose(energy, energy_h, atol=1e-11)
    np.testing.assert_allclose(norm, 1.0, atol=1e-13)
    # equal amplitudes within a level
    for k in np.nonzero(hist)[0]:
        vals = psi[cost == k]
        assert np.abs(vals - vals[0]).max() < 1e-14


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_p1_closed_form(seed):
    """From Eq. (3) with p = 1: psi_z = 2^(-n/2)[e^{-i g C(z)} + (e^{-i b}-1) f(g)],
    f(g) = sum_k w_k e^{-i g k}, so P_sol = w_0 |1 + (e^{-i b} - 1) f(g)|^2."""
    n, m = 10, 42
    lits = _rand(n, m, seed)
    cost = cost_table(n, lits)
    hist = level_histogram(cost, m)
    w = hist / 2 ** n
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(5):
        b, g = rng.uniform(-7, 7, 2)
        f = (w * np.exp(-1j * g * np.arange(m + 1))).sum()
        expect = w[0] * abs(1 + (np.exp(-1j * b) - 1) * f) ** 2
        _, psol, _, _ = evolve_sv(n, cost, [b], [g])
        assert psol[1] == pytest.approx(expect, abs=1e-14)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_two_level_grover_rotation(n):
    """A two-valued cost with w_0 = 1/8 at beta = gamma = pi is Grover search:
    P_sol(p) = sin^2((2p+1) theta), sin^2 theta = 1/8."""
    lits = inst.two_level_instance(n, keep_pattern=3)
    cost = cost_table(n, lits)
    p = 12
    _, psol, _, _ = evolve_sv(n, cost, np.full(p, np.pi), np.full(p, np.pi))
    theta = math.asin(math.sqrt(1.0 / 8.0))
    expect = [math.sin((2 * j + 1) * theta) ** 2 for j in range(p + 1)]
    np.testing.assert_allclose(psol, expect, atol=1e-13)


def test_two_level_general_angles_matrix_power():
    """General (beta, gamma) on a two-level cost: P_sol is |<e_0|U^p v>|^2 for
    the 2x2 unitary U = M D in the orthonormal level basis sqrt(w_k) b_k."""
    n = 7
    lits = inst.two_level_instance(n, keep_pattern=6)
    cost = cost_table(n, lits)
    w0 = 1.0 / 8.0
    v = np.array([math.sqrt(w0), math.sqrt(1 - w0)])
    rng = np.random.Generator(np.random.PCG64(77))
    for _ in range(4):
        b, g = rng.uniform(0, 2 * np.pi, 2)
        p = int(rng.integers(1, 30))
        D = np.diag([1.0, np.exp(-1j * g)])
        M = np.eye(2) + (np.exp(-1j * b) - 1) * np.outer(v, v)
        a = np.linalg.matrix_power(M @ D, p) @ v
        _, psol, _, _ = evolve_sv(n, cost, np.full(p, b), np.full(p, g))
        assert psol[-1] == pytest.approx(abs(a[0]) ** 2, abs=1e-13)


def test_symmetries():
    n, m = 9, 38
    hist = level_histogram(cost_table(n, _rand(n, m, 31)), m)
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(5):
        b, g = rng.uniform(0, np.pi, 2)
        p = 9
        P = psol_single_pair_hist(hist, b, g, p)
        assert psol_single_pair_hist(hist, -b, -g, p) == pytest.approx(P, abs=1e-13)
        assert psol_single_pair_hist(hist, b + 2 * np.pi, g, p) == pytest.approx(P, abs=1e-13)
        assert psol_single_pair_hist(hist, b, g + 2 * np.pi, p) == pytest.approx(P, abs=1e-13)


def test_norm_conserved_random_state():
    n, m, p = 10, 42, 15
    cost = cost_table(n, _rand(n, m, 41))
    beta, gamma = inst.uniform_angles(41, p)
    _, _, _, norm = evolve_sv(n, cost, beta, gamma, psi0=_rand_state(n, 3))
    np.testing.assert_allclose(norm, 1.0, atol=1e-13)


@pytest.mark.parametrize("key", ["4var", "5var"])
def test_table1_noiseless_gqaoa(key):
    """Table I, noiseless G-QAOA column, at energy-minimizing angles (Eq. (4)):
    p = 1 with one pair; p = 2 with per-round angles. The paper does not print
    its angles, so this is a sanity pin at +-0.3 percentage points."""
    with open(os.path.join(GOLDEN, "paper_instances.json")) as f:
        g = json.load(f)[key]
    n = g["n"]
    lits = inst.parse_paper_clauses(g["clauses"])
    hist = level_histogram(cost_table(n, lits), lits.shape[0])
    grid_b = np.arange(0, 360) * np.pi / 180.0
    grid_g = np.arange(0, 181) * np.pi / 180.0
    b1, g1, _, _ = optimize_single_pair(hist, 1, grid_b, grid_g, objective="energy")
    p1 = psol_single_pair_hist(hist, b1, g1, 1)
    assert 100 * p1 == pytest.approx(g["table1_noiseless_percent"]["p1_G"], abs=0.3)
    best = None
    for bs, gs in [(b1, g1)] + [(bb, gg) for bb in (1.0, 2.5, 4.0, 5.5) for gg in (0.5, 1.5, 2.5)]:
        betas, gammas, e = optimize_full(hist, bs, gs, 2, objective="energy")
        if best is None or e < best[2]:
            best = (betas, gammas, e)
    _, psol, _, _ = evolve_hist(hist, best[0], best[1])
    assert 100 * psol[-1] == pytest.approx(g["table1_noiseless_percent"]["p2_G"], abs=0.3)
