"""GPU: the streaming passes under every compiled launch shape (the
GQAOA_SV_SHAPE tuning hook: amplitudes per lane, groups per loop trip,
blocks per CU, nontemporal or plain stores), including shapes outside the
compiled set, which fall back to a default kernel on the same grid. Each
shape's P_sol, E and norm (complex64, complex128) and adjoint gradient
(complex128) must match the oracle at the dtype's bar; a shape only changes
which lanes and blocks take which amplitudes."""
import numpy as np
import pytest

from gpu_common import log, need_gpu, rand_lits
from oracle.cost import cost_table, level_histogram
from oracle.evolve import evolve_sv
from oracle.grad import grad_hist
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

pytestmark = pytest.mark.gpu

C64_SHAPES = ["2,4,256,1", "2,8,16,1", "2,16,32,1", "2,8,8,0", "2,16,8,0", "4,4,64,1", "4,4,64,0", "2,1,4,1",
              "3,5,7,1"]
C128_SHAPES = ["1,4,256,1", "1,8,16,1", "1,16,64,1", "1,8,8,0", "2,4,256,1", "1,1,4,1", "5,3,9,1"]


@pytest.mark.parametrize("dt,shapes", [(g.C64, C64_SHAPES), (g.C128, C128_SHAPES)])
def test_evolve_under_every_shape(dt, shapes, monkeypatch):
    need_gpu()
    n, p = 18, 6
    m = inst.m_from_density(n, 4.2)
    lits = rand_lits(n, m, 500)
    cost, _ = g.gqaoa_cost_table(n, lits)
    ref_cost = cost_table(n, lits)
    rng = np.random.Generator(np.random.PCG64(501))
    b, gm = rng.uniform(0, 2 * np.pi, p), rng.uniform(0, np.pi, p)
    _, rp, re, rn = evolve_sv(n, ref_cost, b, gm)
    tol = 1e-5 if dt == g.C64 else 1e-12
    for shape in shapes:
        monkeypatch.setenv("GQAOA_SV_SHAPE", shape)
        log(f"shape {shape} dtype {dt}")
        _, ps, en, nm = g.gqaoa_evolve(n, m, cost, b, gm, dtype=dt)
        assert np.abs(ps - rp).max() < tol, shape
        assert np.abs(en - re).max() < tol * m, shape
        assert np.abs(nm - rn).max() < tol, shape


def test_adjoint_under_shapes(monkeypatch):
    torch = need_gpu()
    n, p, I = 16, 5, 2
    m = inst.m_from_density(n, 4.2)
    lits = [rand_lits(n, m, 510 + k) for k in range(I)]
    costs = torch.empty((I, 2 ** n), dtype=torch.uint8, device="cuda")
    for k in range(I):
        g.gqaoa_cost_table(n, lits[k], with_hist=False, cost=costs[k])
    rng = np.random.Generator(np.random.PCG64(511))
    betas, gammas = rng.uniform(0, np.pi, (I, p)), rng.uniform(0, np.pi, (I, p))
    refs = [grad_hist(level_histogram(cost_table(n, lits[k]), m), betas[k], gammas[k]) for k in range(I)]
    for shape in ["1,4,256,1", "1,8,16,1", "1,1,4,1", "1,16,64,1"]:
        monkeypatch.setenv("GQAOA_SV_SHAPE", shape)
        log(f"adjoint shape {shape}")
        P, db, dg = g.gqaoa_grad_batched(n, [m] * I, costs, betas, gammas, dtype=g.C128, ckpt_every=2)
        for k in range(I):
            assert abs(P[k] - refs[k][0]) < 1e-12, shape
            assert np.abs(db[k] - refs[k][1]).max() < 1e-11, shape
            assert np.abs(dg[k] - refs[k][2]).max() < 1e-10, shape
