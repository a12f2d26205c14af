"""X-QAOA rounds on the GPU against the oracle (oracle/xqaoa.py): whole
states at small n (every tiling case: one tile, low pass plus one or two high
passes, a ragged last high pass), and at n = 28 a sampled closed form and the
norm."""
import numpy as np
import pytest

from oracle.cost import cost_of, cost_table, level_histogram
from oracle.xqaoa import evolve_x
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

from gpu_common import c2_instance, log, need_gpu, rand_lits, rand_state

pytestmark = pytest.mark.gpu

TOL = {g.C64: 1e-5, g.C128: 1e-12}


def _torch_dtype(torch, dt):
    return torch.complex64 if dt == g.C64 else torch.complex128


# n = 3..11: a single low tile; 12: complex64 one low tile, complex128 low
# + a 1-qubit high group; 13: complex64 low + 1 qubit (its high tile is the
# whole state); 17: one ragged high group; 20: complex64 one full high group
# (compile-time plan), complex128 a full and a 1-qubit one; 22: two high
# groups, the last ragged
@pytest.mark.parametrize("n", [3, 7, 11, 12, 13, 17, 20, 22])
@pytest.mark.parametrize("dt", [g.C64, g.C128])
def test_states_match_oracle(n, dt):
    torch = need_gpu()
    m = min(int(round(4.2 * n)), 4 * (n * (n - 1) * (n - 2) // 6))  # n = 3: 4 of the 8 possible clauses
    lits = rand_lits(n, m, 100 + n)
    cost, hist = g.gqaoa_cost_table(n, lits)
    ref_cost = cost_table(n, lits)
    p = 3
    beta, gamma = inst.uniform_angles(300 + n, p)
    psi0 = rand_state(n, 200 + n)
    log(f"x-qaoa n={n} dtype={dt}")
    psi_d = torch.tensor(psi0, dtype=_torch_dtype(torch, dt), device="cuda")
    psi, psol, energy, norm = g.gqaoa_evolve_x(n, m, cost, beta, gamma, dtype=dt, psi=psi_d, init_uniform=False)
    rpsi, rpsol, renergy, rnorm = evolve_x(n, ref_cost, beta, gamma, psi0=psi0)
    # complex64: relative to the largest amplitude; complex128: absolute
    err = np.abs(psi.cpu().numpy().astype(np.complex128) - rpsi).max()
    scale = np.abs(rpsi).max() if dt == g.C64 else 1.0
    assert err < TOL[dt] * scale, err
    assert np.abs(psol - rpsol).max() < TOL[dt]
    assert np.abs(energy - renergy).max() / m < TOL[dt]
    assert np.abs(norm - rnorm).max() < TOL[dt]


@pytest.mark.parametrize("dt", [g.C64, g.C128])
def test_uniform_start_and_target_level(dt):
    torch = need_gpu()
    n, m = 14, 60
    lits = rand_lits(n, m, 7)
    cost, _ = g.gqaoa_cost_table(n, lits)
    ref_cost = cost_table(n, lits)
    t = int(np.nonzero(level_histogram(ref_cost, m))[0][0]) + 1
    beta, gamma = inst.uniform_angles(8, 5)
    psi, psol, energy, norm = g.gqaoa_evolve_x(n, m, cost, beta, gamma, dtype=dt, target_level=t)
    rpsi, rpsol, renergy, rnorm = evolve_x(n, ref_cost, beta, gamma, target=t)
    assert np.abs(psi.cpu().numpy() - rpsi).max() < TOL[dt]
    assert np.abs(psol - rpsol).max() < TOL[dt]
    assert np.abs(energy - renergy).max() / m < TOL[dt]
    torch.cuda.synchronize()


def test_zero_rounds_writes_uniform_state():
    torch = need_gpu()
    n, m = 12, 50
    lits = rand_lits(n, m, 9)
    cost, hist = g.gqaoa_cost_table(n, lits)
    psi, psol, energy, norm = g.gqaoa_evolve_x(n, m, cost, [], [], dtype=g.C128)
    np.testing.assert_allclose(psi.cpu().numpy(), np.full(2 ** n, 2 ** (-n / 2)), atol=1e-15)
    h = level_histogram(cost_table(n, lits), m)
    assert abs(psol[0] - h[0] / 2 ** n) < 1e-14
    assert abs(norm[0] - 1.0) < 1e-13
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,dt", [(12, g.C64), (20, g.C64), (22, g.C128)])
def test_zero_rounds_reads_out_given_state(n, dt):
    """p = 0 from a given state: the state is left as it is and the readout is
    the oracle's readout of it (the readout-only pass on the streaming tiles)."""
    torch = need_gpu()
    m = int(round(4.2 * n))
    lits = rand_lits(n, m, 500 + n)
    cost, _ = g.gqaoa_cost_table(n, lits)
    ref_cost = cost_table(n, lits)
    psi0 = rand_state(n, 600 + n)
    psi_d = torch.tensor(psi0, dtype=_torch_dtype(torch, dt), device="cuda")
    t = int(np.nonzero(level_histogram(ref_cost, m))[0][0])
    psi, psol, energy, norm = g.gqaoa_evolve_x(n, m, cost, [], [], dtype=dt, psi=psi_d, init_uniform=False,
                                               target_level=t)
    _, rpsol, renergy, rnorm = evolve_x(n, ref_cost, [], [], psi0=psi0, target=t)
    got = psi.cpu().numpy().astype(np.complex128)
    ref0 = psi0.astype(np.complex64).astype(np.complex128) if dt == g.C64 else psi0
    assert np.array_equal(got, ref0)
    assert abs(psol[0] - rpsol[0]) < TOL[dt]
    assert abs(energy[0] - renergy[0]) / m < TOL[dt]
    assert abs(norm[0] - rnorm[0]) < TOL[dt]
    torch.cuda.synchronize()


def test_full_size_n28_bit_flip_closed_form():
    """n = 28, m = 118, complex64, at the X-QAOA launch shape. With beta = pi/2
    every factor exp(-i pi/2 X_q) = -i X_q, so a round maps psi_z to
    (-i)^n e^{-i gamma C(zbar)} psi_zbar (zbar the complement of z). Two
    such rounds from |+> give psi_z = (-1)^n e^{-i (gamma_1 C(z) + gamma_2 C(zbar))} / 2^{n/2},
    checked at 4096 sampled z against the oracle's C; then a run with random
    angles keeps the norm within 1e-5 and matches complex128 P_sol."""
    torch = need_gpu()
    n, m = 28, 118
    it = c2_instance()
    cost, _ = g.gqaoa_cost_table(n, it.lits)
    gamma = np.array([0.37, 1.21])
    log("x-qaoa n=28 closed form")
    psi, psol, _, norm = g.gqaoa_evolve_x(n, m, cost, [np.pi / 2] * 2, gamma, dtype=g.C64)
    rng = np.random.Generator(np.random.PCG64(28))
    z = rng.integers(0, 2 ** n, size=4096, dtype=np.int64)
    zbar = (2 ** n - 1) ^ z
    ref = (-1) ** n * np.exp(-1j * (gamma[0] * cost_of(z, it.lits) + gamma[1] * cost_of(zbar, it.lits))) / 2 ** (n / 2)
    got = psi[torch.tensor(z, device="cuda")].cpu().numpy().astype(np.complex128)
    assert np.abs(got - ref).max() * 2 ** (n / 2) < 1e-5
    assert np.abs(norm - 1).max() < 1e-5
    del psi
    torch.cuda.empty_cache()
    beta, gamma = inst.uniform_angles(2, 8)
    log("x-qaoa n=28 complex64 vs complex128")
    _, p64, e64, n64 = g.gqaoa_evolve_x(n, m, cost, beta, gamma, dtype=g.C64)
    torch.cuda.empty_cache()
    _, p128, e128, n128 = g.gqaoa_evolve_x(n, m, cost, beta, gamma, dtype=g.C128)
    assert np.abs(n64 - 1).max() < 1e-5 and np.abs(n128 - 1).max() < 1e-12
    assert np.abs(p64 - p128).max() < 1e-5
    assert np.abs(e64 - e128).max() / m < 1e-5
    torch.cuda.empty_cache()


def test_bit_flip_closed_form_complex128_n30():
    """complex128 at n = 30: the high groups' 64 KiB tiles outnumber the
    passes' largest grid (2^18 tiles, 65,536 blocks), so every block loops
    over four tiles with the next one in flight. The beta = pi/2 closed form
    (see the n = 28 test) at 4096 sampled z, to 1e-12 after scaling by
    2^(n/2), and the norm to 1e-12."""
    torch = need_gpu()
    n = 30
    m = inst.m_from_density(n, 4.2)
    lits = rand_lits(n, m, 30)
    cost, _ = g.gqaoa_cost_table(n, lits, with_hist=False)
    gamma = np.array([0.83, 1.57])
    log(f"x-qaoa n={n} complex128 closed form")
    psi, _, _, norm = g.gqaoa_evolve_x(n, m, cost, [np.pi / 2] * 2, gamma, dtype=g.C128)
    rng = np.random.Generator(np.random.PCG64(30))
    z = rng.integers(0, 2 ** n, size=4096, dtype=np.int64)
    zbar = (2 ** n - 1) ^ z
    ref = (-1) ** n * np.exp(-1j * (gamma[0] * cost_of(z, lits) + gamma[1] * cost_of(zbar, lits)))
    got = psi[torch.tensor(z, device="cuda")].cpu().numpy() * 2 ** (n / 2)
    assert np.abs(got - ref).max() < 1e-12
    assert np.abs(norm - 1).max() < 1e-12
    del psi, cost
    torch.cuda.empty_cache()
