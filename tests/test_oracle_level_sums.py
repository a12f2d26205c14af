"""The oracle's statevector evolution (oracle.evolve.evolve_sv) from a random,
level-asymmetric initial state, pinned by an exact reformulation that shares
none of its steps.

The phase of a round depends on z only through C(z), and the Grover mixer
adds one constant to every amplitude. So after j rounds
    psi_j(z) = exp(-i G_j C(z)) psi_0(z) + L_j(C(z)),   G_j = gamma_1 + ... + gamma_j,
with a table L_j over the levels: L_0 = 0 and
    L_j(k) = exp(-i gamma_j k) L_{j-1}(k) + c_j,
    c_j = (exp(-i beta_j) - 1) / 2^n * sum_k [exp(-i G_j k) A_k + N_k exp(-i gamma_j k) L_{j-1}(k)],
where N_k counts the assignments on level k, A_k = sum_{C(z)=k} psi_0(z) and
Q_k = sum_{C(z)=k} |psi_0(z)|^2. Every readout follows from N, A and Q:
    sum_{C(z)=k} |psi_j(z)|^2 = Q_k + 2 Re(conj(L_j(k)) exp(-i G_j k) A_k) + N_k |L_j(k)|^2.
The recursion below runs on the level tables only (no 2^n-length state
until the final state is formed from it), so a mistake in the oracle's
phase, mixer or readouts (a sign, a dropped term, the wrong normalization)
shows up as a mismatch."""
import numpy as np
import pytest

from oracle.cost import cost_table
from oracle.evolve import evolve_sv
from paper_2402_02585_amd import instances as inst


def _level_sum_evolution(n, cost, betas, gammas, psi0, target):
    m = int(cost.max())
    N = np.bincount(cost, minlength=m + 1).astype(np.float64)
    A = np.bincount(cost, weights=psi0.real, minlength=m + 1) + 1j * np.bincount(cost, weights=psi0.imag, minlength=m + 1)
    Q = np.bincount(cost, weights=np.abs(psi0) ** 2, minlength=m + 1)
    k = np.arange(m + 1, dtype=np.float64)
    L = np.zeros(m + 1, dtype=np.complex128)
    G = 0.0

    def levels(L, G):
        return Q + 2.0 * np.real(np.conj(L) * np.exp(-1j * G * k) * A) + N * np.abs(L) ** 2

    p = len(betas)
    psol, energy, norm = np.empty(p + 1), np.empty(p + 1), np.empty(p + 1)
    lv = levels(L, G)
    psol[0], energy[0], norm[0] = lv[target], (k * lv).sum(), lv.sum()
    for j in range(p):
        G += gammas[j]
        Lp = np.exp(-1j * gammas[j] * k) * L
        total = (np.exp(-1j * G * k) * A).sum() + (N * Lp).sum()
        c = (np.exp(-1j * betas[j]) - 1.0) * total / 2.0 ** n
        L = Lp + c
        lv = levels(L, G)
        psol[j + 1], energy[j + 1], norm[j + 1] = lv[target], (k * lv).sum(), lv.sum()
    psi = np.exp(-1j * G * cost) * psi0 + L[cost]
    return psi, psol, energy, norm


@pytest.mark.parametrize("n, seed", [(5, 1), (8, 2), (11, 3)])
def test_statevector_oracle_matches_level_sum_recursion(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    m = int(round(4.2 * n))
    lits = inst.random_3sat(rng, n, m)
    cost = cost_table(n, lits).astype(np.int64)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    p = 6
    betas = rng.uniform(0, 2 * np.pi, p)
    gammas = rng.uniform(0, np.pi, p)
    target = int(np.sort(np.unique(cost))[1])      # a Max-SAT-like target: the second occupied level
    for t in (0, target):
        got = evolve_sv(n, cost, betas, gammas, psi0=psi0, target=t)
        ref = _level_sum_evolution(n, cost, betas, gammas, psi0, t)
        np.testing.assert_allclose(got[0], ref[0], rtol=0, atol=1e-12)
        for a, b in zip(got[1:], ref[1:]):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * max(1.0, m))


def test_level_sum_recursion_catches_a_planted_sign_error():
    """The pin has teeth: flipping the sign of the mixer's phase in the
    recursion (a plausible slip) moves the readouts far beyond the bar."""
    n, seed = 8, 4
    rng = np.random.Generator(np.random.PCG64(seed))
    lits = inst.random_3sat(rng, n, 34)
    cost = cost_table(n, lits).astype(np.int64)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    betas, gammas = np.array([0.7, 1.9, 2.6]), np.array([0.4, 1.1, 0.8])
    got = evolve_sv(n, cost, betas, gammas, psi0=psi0)
    wrong = _level_sum_evolution(n, cost, -betas, gammas, psi0, 0)
    assert np.abs(got[1] - wrong[1]).max() > 1e-6
