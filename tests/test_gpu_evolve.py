"""GPU parity: statevector evolution (Eq. (3)) against the complex128 oracle.

Tolerances: P_sol, E/m and norm within 1e-12 (complex128) and 1e-5
(complex64), absolute.
"""
import numpy as np
import pytest

from gpu_common import c2_instance, log, need_gpu, rand_lits, rand_state
from oracle import brute
from oracle.cost import cost_table, level_histogram, min_level
from oracle.evolve import evolve_hist, evolve_sv
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

pytestmark = pytest.mark.gpu
TOL = {g.C128: 1e-12, g.C64: 1e-5}


def _check(res, ref, dt, m):
    _, psol, energy, norm = res
    _, rp, re, rn = ref
    assert np.abs(psol - rp).max() < TOL[dt], np.abs(psol - rp).max()
    assert np.abs(energy - re).max() / m < TOL[dt], np.abs(energy - re).max()
    assert np.abs(norm - rn).max() < TOL[dt]


@pytest.mark.parametrize("dt", [g.C128, g.C64])
def test_small_config_n10_p20(dt):
    """n = 10, m = 42, seed 1, p = 20 independent angles on [0, pi]."""
    need_gpu()
    it = inst.first_satisfiable(1, 10, 42)
    beta, gamma = inst.uniform_angles(1, 20)
    cost, _ = g.gqaoa_cost_table(10, it.lits)
    ref_cost = cost_table(10, it.lits)
    res = g.gqaoa_evolve(10, 42, cost, beta, gamma, dtype=dt)
    ref = evolve_sv(10, ref_cost, beta, gamma)
    _check(res, ref, dt, 42)
    psi = res[0].cpu().numpy()
    assert np.abs(psi - ref[0]).max() < (1e-13 if dt == g.C128 else 2e-6)


@pytest.mark.parametrize("n,m,p,seed", [(3, 5, 4, 1), (4, 9, 6, 2), (5, 18, 5, 3), (7, 30, 9, 4), (9, 38, 7, 5),
                                        (13, 55, 12, 6), (15, 64, 10, 7)])
@pytest.mark.parametrize("dt", [g.C128, g.C64])
def test_random_initial_state(n, m, p, seed, dt):
    """A random (not level-symmetric) initial state exercises every amplitude."""
    torch = need_gpu()
    log(f"evolve random psi0 n={n} m={m} p={p} dt={dt}")
    lits = rand_lits(n, m, seed)
    beta, gamma = inst.uniform_angles(seed + 50, p)
    psi0 = rand_state(n, seed)
    cost, _ = g.gqaoa_cost_table(n, lits)
    tdt = torch.complex128 if dt == g.C128 else torch.complex64
    psi = torch.tensor(psi0, dtype=tdt, device="cuda")
    res = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=dt, psi=psi, init_uniform=False)
    psi0_used = psi0 if dt == g.C128 else psi0.astype(np.complex64).astype(np.complex128)
    ref = evolve_sv(n, cost_table(n, lits), beta, gamma, psi0=psi0_used)
    _check(res, ref, dt, m)
    assert np.abs(res[0].cpu().numpy() - ref[0]).max() < (1e-13 if dt == g.C128 else 2e-6)


@pytest.mark.parametrize("n,dt", [(22, g.C64), (21, g.C128), (22, g.C128)])
def test_random_initial_state_folded_grid(n, dt):
    """The launch shape the headline uses: one tile per block, with the
    per-round partial rows folded before the finalize (complex64 from n = 22,
    complex128 from n = 21), from a random state that no level symmetry masks;
    the whole final state and every round's readouts against the oracle."""
    torch = need_gpu()
    m, p, seed = inst.m_from_density(n, 4.2), 6, 300 + n
    log(f"evolve random psi0 folded grid n={n} m={m} p={p} dt={dt}")
    lits = rand_lits(n, m, seed)
    beta, gamma = inst.uniform_angles(seed, p)
    psi0 = rand_state(n, seed)
    cost, _ = g.gqaoa_cost_table(n, lits)
    tdt = torch.complex128 if dt == g.C128 else torch.complex64
    psi = torch.tensor(psi0, dtype=tdt, device="cuda")
    res = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=dt, psi=psi, init_uniform=False)
    psi0_used = psi0 if dt == g.C128 else psi0.astype(np.complex64).astype(np.complex128)
    ref = evolve_sv(n, cost_table(n, lits), beta, gamma, psi0=psi0_used)
    _check(res, ref, dt, m)
    assert np.abs(res[0].cpu().numpy() - ref[0]).max() < (1e-13 if dt == g.C128 else 2e-6)


@pytest.mark.parametrize("dt", [g.C128, g.C64])
def test_max_sat_target_and_solution_prob(dt):
    need_gpu()
    n, m = 12, 90
    lits = rand_lits(n, m, 77)
    ref_cost = cost_table(n, lits)
    t = min_level(level_histogram(ref_cost, m))
    beta, gamma = inst.uniform_angles(77, 8)
    cost, _ = g.gqaoa_cost_table(n, lits)
    res = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=dt, target_level=t)
    ref = evolve_sv(n, ref_cost, beta, gamma, target=t)
    _check(res, ref, dt, m)
    P = g.gqaoa_solution_prob(n, cost, res[0], dtype=dt, target_level=t)
    assert abs(P - ref[1][-1]) < TOL[dt]


def test_p0_writes_uniform_state():
    torch = need_gpu()
    n, m = 9, 38
    lits = rand_lits(n, m, 5)
    cost, hist = g.gqaoa_cost_table(n, lits)
    psi, psol, energy, norm = g.gqaoa_evolve(n, m, cost, [], [], dtype=g.C128)
    assert np.allclose(psi.cpu().numpy(), 2 ** (-n / 2), atol=1e-15)
    assert psol[0] == pytest.approx(hist.cpu().numpy()[0] / 2 ** n, abs=1e-15)
    assert energy[0] == pytest.approx(m / 8, abs=1e-12)


@pytest.mark.parametrize("dt", [g.C64, g.C128])
def test_n20_seed2_p64(dt):
    """A seed-2 n = 20, m = 84 instance, p = 64: GPU against the oracle statevector."""
    need_gpu()
    it = inst.first_satisfiable(2, 20, 84)
    beta, gamma = inst.uniform_angles(2, 64)
    cost, _ = g.gqaoa_cost_table(20, it.lits)
    res = g.gqaoa_evolve(20, 84, cost, beta, gamma, dtype=dt)
    ref = evolve_sv(20, cost_table(20, it.lits), beta, gamma)
    _check(res, ref, dt, 84)


def test_deterministic_reruns():
    need_gpu()
    n, m = 16, 67
    cost, _ = g.gqaoa_cost_table(n, rand_lits(n, m, 3))
    beta, gamma = inst.uniform_angles(3, 10)
    a = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=g.C64)
    b = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=g.C64)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert bool((a[0] == b[0]).all())


def test_full_size_n28_p64_complex64():
    """n = 28, m = 118, p = 64 at the benchmarked launch shape: P_sol per round
    of the complex64 state against (i) the oracle's level-space evolution of
    the brute-force histogram and (ii) a complex128 GPU run, within 1e-5."""
    torch = need_gpu()
    it = c2_instance()
    beta, gamma = inst.uniform_angles(2, 64)
    cost, hist = g.gqaoa_cost_table(28, it.lits)
    log("n=28 complex64 run")
    _, psol64, e64, n64 = g.gqaoa_evolve(28, 118, cost, beta, gamma, dtype=g.C64)
    ref_hist = brute.level_histogram_brute(28, it.lits)
    _, rp, re, rn = evolve_hist(ref_hist, beta, gamma)
    assert np.abs(psol64 - rp).max() < 1e-5, np.abs(psol64 - rp).max()
    assert np.abs(e64 - re).max() / 118 < 1e-5
    assert np.abs(n64 - 1).max() < 1e-5
    torch.cuda.empty_cache()
    log("n=28 complex128 run")
    _, psol128, _, _ = g.gqaoa_evolve(28, 118, cost, beta, gamma, dtype=g.C128)
    assert np.abs(psol64 - psol128).max() < 1e-5
    assert np.abs(psol128 - rp).max() < 1e-10
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dt", [g.C64, g.C128])
def test_fused_and_separate_finalize_agree(dt, monkeypatch):
    """The round pass either launches its finalize separately (default, one
    tile per block) or folds it into its last block (GQAOA_SV_FUSE=1, on the
    persistent grid). The two grids round their float32 tile sums differently,
    so the results agree to the state's precision: 1e-6 on P_sol and the norm,
    1e-6 m on E (E is of order m/8) for complex64; 1e-14 (times m for E) for
    complex128."""
    need_gpu()
    n, m = 18, 76
    lits = rand_lits(n, m, 44)
    beta, gamma = inst.uniform_angles(44, 12)
    cost, _ = g.gqaoa_cost_table(n, lits)
    sep = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=dt)
    monkeypatch.setenv("GQAOA_SV_FUSE", "1")
    fused = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=dt)
    monkeypatch.delenv("GQAOA_SV_FUSE")
    for a, b, scale in zip(fused[1:], sep[1:], (1, m, 1)):
        assert np.abs(a - b).max() < (1e-14 if dt == g.C128 else 1e-6) * scale
    ref = evolve_sv(n, cost_table(n, lits), beta, gamma)
    _check(fused, ref, dt, m)


def test_sampled_profiling_counts():
    """gqaoa_profile_enable(k) times one round pass in k (n = 16 streams its
    rounds); a small state's single resident launch is timed under its own
    name; the evolution itself is unchanged by profiling."""
    need_gpu()
    n, m = 16, 67
    cost, _ = g.gqaoa_cost_table(n, rand_lits(n, m, 5))
    beta, gamma = inst.uniform_angles(6, 10)
    ref = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=g.C64)[1]
    g.gqaoa_profile_reset()
    g.gqaoa_profile_enable(True, every=4)
    got = g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=g.C64)[1]
    g.gqaoa_profile_enable(False)
    ms, cnt = g.gqaoa_profile_read("sv_round_c64")
    g.gqaoa_profile_reset()
    assert cnt == 3 and ms > 0          # passes 0, 4, 8 of the 10
    assert (got == ref).all()
    n, m = 12, 50
    cost, _ = g.gqaoa_cost_table(n, rand_lits(n, m, 7))
    g.gqaoa_profile_enable(True)
    g.gqaoa_evolve(n, m, cost, beta, gamma, dtype=g.C128)
    g.gqaoa_profile_enable(False)
    ms, cnt = g.gqaoa_profile_read("sv_resident_c128")
    assert g.gqaoa_profile_read("sv_round_c128")[1] == 0
    g.gqaoa_profile_reset()
    assert cnt == 1 and ms > 0
