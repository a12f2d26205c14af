"""The largest sizes the library accepts, n = 34 (a 16 GiB cost table and a
128 GiB complex64 state), checked against the oracle where it can follow and
against properties that hold at any size:
  * cost table of a random instance: sum_k N_k = 2^n, sum_k k N_k = m 2^(n-3)
    (each clause is false on 2^(n-3) assignments), and C(z) at 4096 sampled z;
  * G-QAOA on the two-level instance (7 clauses on variables 0..2, so
    N_0 = 2^(n-3) and N_1 = 7 * 2^(n-3) in closed form): readouts and sampled
    amplitudes against the oracle's level-space evolution of that histogram;
    on the random instance, E(0) = m/8 and the norm;
  * X-QAOA: the beta = pi/2 bit-flip closed form at sampled z."""
import math

import numpy as np
import pytest

from oracle.cost import cost_of
from oracle.evolve import evolve_hist
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

from gpu_common import log, need_gpu, rand_lits

pytestmark = pytest.mark.gpu
N_MAX = 34


def _samples(n, seed, count=4096):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 2 ** n, size=count, dtype=np.int64)


def test_cost_table_and_evolve_at_n34():
    torch = need_gpu()
    n = N_MAX
    m = inst.m_from_density(n, 4.2)
    lits = rand_lits(n, m, 34)
    log(f"cost table n={n} m={m}")
    cost, hist = g.gqaoa_cost_table(n, lits)
    h = hist.cpu().numpy().astype(np.int64)
    assert h.sum() == 2 ** n
    assert (np.arange(m + 1) * h).sum() == m * 2 ** (n - 3)
    z = _samples(n, 1)
    got = cost[torch.tensor(z, device="cuda")].cpu().numpy().astype(np.int64)
    assert (got == cost_of(z, lits)).all()
    log(f"evolve n={n} complex64 p=2 (random instance)")
    beta, gamma = inst.uniform_angles(34, 2)
    psi, psol, energy, norm = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=g.C64)
    assert abs(energy[0] - m / 8) < 1e-6 * m
    assert abs(psol[0] - h[0] / 2 ** n) < 1e-9
    assert np.abs(norm - 1).max() < 1e-5
    del psi, cost, hist
    torch.cuda.empty_cache()


def test_two_level_gqaoa_at_n34():
    torch = need_gpu()
    n = N_MAX
    lits = inst.two_level_instance(n)
    m = lits.shape[0]
    cost, hist = g.gqaoa_cost_table(n, lits)
    ref_hist = np.zeros(m + 1, dtype=np.int64)
    ref_hist[0], ref_hist[1] = 2 ** (n - 3), 7 * 2 ** (n - 3)
    assert (hist.cpu().numpy().astype(np.int64) == ref_hist).all()
    beta, gamma = inst.uniform_angles(35, 3)
    log(f"evolve n={n} complex64 p=3 (two-level instance)")
    psi, psol, energy, norm = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=g.C64)
    b, rp, re, rn = evolve_hist(ref_hist, beta, gamma)
    assert np.abs(psol - rp).max() < 1e-5
    assert np.abs(energy - re).max() / m < 1e-5
    assert np.abs(norm - rn).max() < 1e-5
    z = _samples(n, 2)
    amp = psi[torch.tensor(z, device="cuda")].cpu().numpy().astype(np.complex128) * 2 ** (n / 2)
    assert np.abs(amp - b[cost_of(z, lits)]).max() < 1e-4
    del psi, cost, hist
    torch.cuda.empty_cache()


def test_xqaoa_bit_flip_at_n34():
    torch = need_gpu()
    n = N_MAX
    m = inst.m_from_density(n, 4.2)
    lits = rand_lits(n, m, 34)
    cost, _ = g.gqaoa_cost_table(n, lits, with_hist=False)
    gamma = np.array([0.61, 2.03])
    log(f"x-qaoa n={n} complex64 p=2")
    psi, psol, _, norm = g.gqaoa_evolve_x(n, m, cost, [math.pi / 2] * 2, gamma, dtype=g.C64)
    z = _samples(n, 3)
    zbar = (2 ** n - 1) ^ z
    ref = (-1) ** n * np.exp(-1j * (gamma[0] * cost_of(z, lits) + gamma[1] * cost_of(zbar, lits)))
    got = psi[torch.tensor(z, device="cuda")].cpu().numpy().astype(np.complex128) * 2 ** (n / 2)
    assert np.abs(got - ref).max() < 1e-4
    assert np.abs(norm - 1).max() < 1e-5
    del psi, cost
    torch.cuda.empty_cache()
