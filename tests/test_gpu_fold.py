"""GPU: streaming passes with more blocks per instance than one finalize block
takes, whose partial rows are folded first, in launches of several
instances.

- Three statevector items at n = 26 (complex64) stream as one batch of three
  instances on a grid of 256 blocks per CU (GQAOA_SV_SHAPE): the 65,536
  partial rows of a pass are shared out as 21,845 per instance, so every
  instance folds 21 full runs of 1024 rows and a ragged run of 341. P_sol and
  E against the oracle's float64 level-space evolution of the brute-force
  histogram (1e-5, 1e-5 m).
- A two-instance adjoint batch at n = 22 (complex128): 4096 blocks per
  instance, 4 folded rows each, in the forward and the reverse passes; P_sol
  and the gradient against the oracle's level-space sweep (1e-12, 1e-10).
"""
import numpy as np
import pytest

from gpu_common import log, need_gpu, rand_lits
from oracle import brute
from oracle.cost import cost_table, level_histogram
from oracle.evolve import evolve_hist
from oracle.grad import grad_hist
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

pytestmark = pytest.mark.gpu
P_LIST = [1, 5, 12]


def test_three_streamed_items_ragged_fold(monkeypatch):
    torch = need_gpu()
    monkeypatch.setenv("GQAOA_SV_SHAPE", "2,4,256,1")
    n = 26
    m = inst.m_from_density(n, 4.2)
    lits = [rand_lits(n, m, 300 + k) for k in range(3)]
    log(f"streamed items: 3 instances n={n} m={m}")
    costs, _, _ = g.gqaoa_cost_batched([n] * 3, [m] * 3, lits, with_hist=False)
    beta = np.array([0.7, 2.9, 4.4])
    gamma = np.array([0.35, 0.2, 1.1])
    ps, en = g.gqaoa_sv_items([n] * 3, [m] * 3, costs, [0, 1, 2], beta, gamma, P_LIST, with_energy=True)
    monkeypatch.delenv("GQAOA_SV_SHAPE")
    ps, en = ps.cpu().numpy(), en.cpu().numpy()
    del costs
    torch.cuda.empty_cache()
    for k in range(3):
        hist = brute.level_histogram_brute(n, lits[k])
        _, rp, re, _ = evolve_hist(hist, np.full(P_LIST[-1], beta[k]), np.full(P_LIST[-1], gamma[k]))
        assert np.abs(ps[k] - rp[P_LIST]).max() < 1e-5, (k, ps[k], rp[P_LIST])
        assert np.abs(en[k] - re[P_LIST]).max() < 1e-5 * m, k


def test_two_instance_adjoint_fold():
    torch = need_gpu()
    n, p = 22, 4
    m = inst.m_from_density(n, 4.2)
    lits = [rand_lits(n, m, 310 + k) for k in range(2)]
    costs = torch.empty((2, 2 ** n), dtype=torch.uint8, device="cuda")
    for k in range(2):
        g.gqaoa_cost_table(n, lits[k], with_hist=False, cost=costs[k])
    rng = np.random.Generator(np.random.PCG64(311))
    betas = rng.uniform(0, np.pi, (2, p))
    gammas = rng.uniform(0, np.pi, (2, p))
    log(f"adjoint: 2 instances n={n} p={p} complex128")
    P, db, dg = g.gqaoa_grad_batched(n, [m, m], costs, betas, gammas, dtype=g.C128, ckpt_every=0)
    for k in range(2):
        rP, rdb, rdg = grad_hist(level_histogram(cost_table(n, lits[k]), m), betas[k], gammas[k])
        assert abs(P[k] - rP) < 1e-12, k
        assert np.abs(db[k] - rdb).max() < 1e-10, k
        assert np.abs(dg[k] - rdg).max() < 1e-10, k
