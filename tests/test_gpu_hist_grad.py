"""GPU parity: level-space evolution and the adjoint gradient."""
import numpy as np
import pytest

from gpu_common import log, need_gpu, rand_lits
from oracle.cost import cost_table, level_histogram, min_level
from oracle.evolve import evolve_hist, evolve_sv
from oracle.grad import grad_hist, grad_sv
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m,p,seed,same", [(10, 42, 20, 1, False), (14, 59, 64, 2, True), (18, 255, 30, 3, False),
                                             (20, 84, 64, 4, True), (6, 26, 1, 5, False), (8, 34, 0, 6, False)])
def test_hist_evolve_float64(n, m, p, seed, same):
    need_gpu()
    lits = rand_lits(n, m, seed)
    cost, hist = g.gqaoa_cost_table(n, lits)
    if same:
        b, gm = inst.uniform_angles(seed, 1)
        beta, gamma = np.full(p, b[0]), np.full(p, gm[0])
    else:
        beta, gamma = inst.uniform_angles(seed, p)
    ref_hist = level_histogram(cost_table(n, lits), m)
    psol, energy, norm = g.gqaoa_hist_evolve(n, m, hist, beta, gamma)
    _, rp, re, rn = evolve_hist(ref_hist, beta, gamma)
    assert np.abs(psol - rp).max() < 1e-12
    assert np.abs(energy - re).max() / m < 1e-12
    assert np.abs(norm - rn).max() < 1e-12


@pytest.mark.parametrize("dt,ckpt", [(g.C128, 0), (g.C128, 1), (g.C128, 3), (g.C128, 7), (g.C128, 50), (g.C64, 2)])
def test_grad_single_vs_oracle(dt, ckpt):
    need_gpu()
    n, m, p = 11, 47, 7
    lits = rand_lits(n, m, 9)
    ref_cost = cost_table(n, lits)
    beta, gamma = inst.uniform_angles(19, p)
    cost, _ = g.gqaoa_cost_table(n, lits)
    P, db, dg = g.gqaoa_grad(n, m, cost, beta, gamma, dtype=dt, ckpt_every=ckpt)
    rP, rdb, rdg = grad_sv(n, ref_cost, beta, gamma)
    tol = 1e-12 if dt == g.C128 else 2e-5
    assert abs(P - rP) < tol
    assert np.abs(db - rdb).max() < tol, np.abs(db - rdb).max()
    assert np.abs(dg - rdg).max() < tol * m, np.abs(dg - rdg).max()


def test_grad_max_sat_target_and_central_fd():
    need_gpu()
    n, m, p = 10, 70, 6
    lits = rand_lits(n, m, 21)
    ref_cost = cost_table(n, lits)
    t = min_level(level_histogram(ref_cost, m))
    beta, gamma = inst.uniform_angles(21, p)
    cost, _ = g.gqaoa_cost_table(n, lits)
    P, db, dg = g.gqaoa_grad(n, m, cost, beta, gamma, dtype=g.C128, target_level=t, ckpt_every=2)
    h = 1e-4
    for k in range(p):
        for arr, d in ((beta, db), (gamma, dg)):
            ap, am = arr.copy(), arr.copy()
            ap[k] += h
            am[k] -= h
            if arr is beta:
                fd = (evolve_sv(n, ref_cost, ap, gamma, target=t)[1][-1] - evolve_sv(n, ref_cost, am, gamma, target=t)[1][-1]) / (2 * h)
            else:
                fd = (evolve_sv(n, ref_cost, beta, ap, target=t)[1][-1] - evolve_sv(n, ref_cost, beta, am, target=t)[1][-1]) / (2 * h)
            assert d[k] == pytest.approx(fd, abs=1e-6)


def test_grad_batched_adjoint_config_sample():
    """Adjoint workload shape: n = 20, m = 85, p = 32, checkpoints every 8 rounds
    (a batch of 6 of the seeded instances); every instance against the
    oracle's level-space sweep, one against the statevector sweep."""
    torch = need_gpu()
    n, m, p, I = 20, 85, 32, 6
    insts = []
    rng_seed = 4
    for k, lits in inst.sat_stream(rng_seed, n, m):
        if inst.dpll_satisfiable(n, lits):
            insts.append(lits)
        if len(insts) == I:
            break
    costs = torch.empty((I, 2 ** n), dtype=torch.uint8, device="cuda")
    for i, lits in enumerate(insts):
        g.gqaoa_cost_table(n, lits, with_hist=False, cost=costs[i])
    betas = np.stack([inst.uniform_angles(100 + i, p)[0] for i in range(I)])
    gammas = np.stack([inst.uniform_angles(100 + i, p)[1] for i in range(I)])
    log("grad batched n=20 p=32")
    P, db, dg = g.gqaoa_grad_batched(n, [m] * I, costs, betas, gammas, dtype=g.C128, ckpt_every=8)
    for i, lits in enumerate(insts):
        ref_cost = cost_table(n, lits)
        rP, rdb, rdg = grad_hist(level_histogram(ref_cost, m), betas[i], gammas[i])
        assert abs(P[i] - rP) < 1e-12
        assert np.abs(db[i] - rdb).max() < 1e-11
        assert np.abs(dg[i] - rdg).max() < 1e-10
        if i == 0:
            sP, sdb, sdg = grad_sv(n, ref_cost, betas[i], gammas[i])
            assert np.abs(db[i] - sdb).max() < 1e-11 and np.abs(dg[i] - sdg).max() < 1e-10


def test_grad_auto_checkpointing_matches_explicit():
    """ckpt_every=None keeps every state when that fits (bit-identical to
    ckpt_every=0); given a workspace one byte short of that, it checkpoints at
    the largest interval that fits, and the recomputed states (the same
    launches on the same inputs) give bit-identical results."""
    torch = need_gpu()
    n, m, p, I = 14, 59, 12, 3
    costs = torch.empty((I, 2 ** n), dtype=torch.uint8, device="cuda")
    for i in range(I):
        g.gqaoa_cost_table(n, rand_lits(n, m, 400 + i), with_hist=False, cost=costs[i])
    rng = np.random.Generator(np.random.PCG64(401))
    betas, gammas = rng.uniform(0, np.pi, (I, p)), rng.uniform(0, np.pi, (I, p))
    ref = g.gqaoa_grad_batched(n, [m] * I, costs, betas, gammas, ckpt_every=0)
    auto = g.gqaoa_grad_batched(n, [m] * I, costs, betas, gammas)
    for a, b in zip(ref, auto):
        assert np.array_equal(a, b)
    budget = g.gqaoa_grad_workspace_bytes(I, n, p, g.C128, 0) - 1
    c = g.choose_ckpt_every(I, n, p, g.C128, budget_bytes=budget)
    assert 1 <= c < p
    ws = torch.empty(budget, dtype=torch.uint8, device="cuda")
    small = g.gqaoa_grad_batched(n, [m] * I, costs, betas, gammas, workspace=ws)
    for a, b in zip(ref, small):
        assert np.array_equal(a, b)


def _hist_batch(specs, seed0):
    """Histograms (host, int64 [I, stride]) of random instances (n, m) and, for
    m >= 128 entries given as ("synthetic", K, m, n), synthetic ones with K
    occupied levels."""
    from gpu_common import synthetic_hist
    rows, ns, ms = [], [], []
    for j, sp in enumerate(specs):
        if sp[0] == "synthetic":
            _, K, m, n = sp
            h = synthetic_hist(K, m, n, seed0 + j).astype(np.int64)
        else:
            n, m = sp
            h = level_histogram(cost_table(n, rand_lits(n, m, seed0 + j)), m)
        rows.append(h)
        ns.append(n)
        ms.append(m)
    stride = max(ms) + 1
    H = np.zeros((len(rows), stride), dtype=np.int64)
    for i, h in enumerate(rows):
        H[i, :len(h)] = h
    return H, ns, ms


def test_hist_grad_batched_vs_oracle_sweep():
    """Level-space adjoint (float64) for a batch of instances with different
    n, m, targets and round counts, including 65..256 occupied levels (all
    three register layouts), against the oracle's level-space sweep: 1e-12 on
    P and dP/dbeta, 1e-12 * m on dP/dgamma; entries past an instance's p are 0."""
    need_gpu()
    specs = [(8, 34), (10, 42), (12, 50), (14, 59), (16, 67), (11, 90), (9, 60), (20, 84),
             ("synthetic", 100, 200, 30), ("synthetic", 129, 180, 26), ("synthetic", 256, 255, 40),
             ("synthetic", 64, 64, 20), ("synthetic", 65, 70, 22)]
    H, ns, ms = _hist_batch(specs, 700)
    I, pmax = len(specs), 24
    rng = np.random.Generator(np.random.PCG64(701))
    p = rng.integers(1, pmax + 1, I)
    p[0], p[1] = pmax, 1
    targets = np.zeros(I, dtype=np.int32)
    for i in (2, 5, 6, 9):
        targets[i] = int(np.nonzero(H[i])[0][0]) if H[i, 0] == 0 else int(np.nonzero(H[i])[0][1])
    targets[7] = ms[7]                       # an unoccupied level: P = 0, gradient 0
    B = rng.uniform(0, np.pi, (I, pmax))
    G = rng.uniform(0, np.pi, (I, pmax))
    log(f"hist grad batched I={I} pmax={pmax}")
    P, db, dg = g.gqaoa_hist_grad_batched(ns, ms, H, B, G, targets=targets, p=p)
    for i in range(I):
        rP, rdb, rdg = grad_hist(H[i, :ms[i] + 1], B[i, :p[i]], G[i, :p[i]], int(targets[i]))
        assert abs(P[i] - rP) < 1e-12, (i, P[i], rP)
        assert np.abs(db[i, :p[i]] - rdb).max() < 1e-12, (i, np.abs(db[i, :p[i]] - rdb).max())
        assert np.abs(dg[i, :p[i]] - rdg).max() < 1e-12 * ms[i], (i, np.abs(dg[i, :p[i]] - rdg).max())
        assert not db[i, p[i]:].any() and not dg[i, p[i]:].any()
    assert P[7] == 0.0 and not db[7].any() and not dg[7].any()


def test_hist_grad_batched_central_fd_and_statevector():
    """The same gradient against central differences (h = 1e-4, float64) of the
    oracle's level-space P (bar 1e-6, the truncation error h^2 P'''/6 being
    far smaller), and against the device statevector adjoint (complex128) on
    the same instance (1e-12)."""
    need_gpu()
    n, m, p = 10, 44, 9
    lits = rand_lits(n, m, 731)
    ref_cost = cost_table(n, lits)
    h = level_histogram(ref_cost, m)
    beta, gamma = inst.uniform_angles(732, p)
    P, db, dg = g.gqaoa_hist_grad_batched([n], [m], h[None, :], beta[None, :], gamma[None, :])
    eps = 1e-4
    for k in range(p):
        for arr, d in ((beta, db[0, k]), (gamma, dg[0, k])):
            xp, xm = arr.copy(), arr.copy()
            xp[k] += eps
            xm[k] -= eps
            bp, gp = (xp, gamma) if arr is beta else (beta, xp)
            bm, gm_ = (xm, gamma) if arr is beta else (beta, xm)
            fd = (evolve_hist(h, bp, gp)[1][-1] - evolve_hist(h, bm, gm_)[1][-1]) / (2 * eps)
            assert abs(d - fd) < 1e-6, (k, d, fd)
    cost, _ = g.gqaoa_cost_table(n, lits)
    Ps, dbs, dgs = g.gqaoa_grad(n, m, cost, beta, gamma, dtype=g.C128, ckpt_every=0)
    assert abs(P[0] - Ps) < 1e-12
    assert np.abs(db[0] - dbs).max() < 1e-12
    assert np.abs(dg[0] - dgs).max() < 1e-12 * m


def test_hist_grad_batched_many_rounds():
    """p = 400 rounds: the reverse sweep runs every round backwards instead of
    storing the forward states; its rounding stays within 1e-11 of the
    oracle's stored-state sweep."""
    need_gpu()
    H, ns, ms = _hist_batch([(16, 67), (20, 84), ("synthetic", 120, 150, 28)], 740)
    rng = np.random.Generator(np.random.PCG64(741))
    pmax = 400
    B = rng.uniform(0, 2 * np.pi, (3, pmax))
    G = rng.uniform(0, np.pi, (3, pmax))
    P, db, dg = g.gqaoa_hist_grad_batched(ns, ms, H, B, G)
    for i in range(3):
        rP, rdb, rdg = grad_hist(H[i, :ms[i] + 1], B[i], G[i])
        assert abs(P[i] - rP) < 1e-11
        assert np.abs(db[i] - rdb).max() < 1e-11, np.abs(db[i] - rdb).max()
        assert np.abs(dg[i] - rdg).max() < 1e-11 * ms[i], np.abs(dg[i] - rdg).max()
