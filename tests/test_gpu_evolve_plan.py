"""GPU: the graph-captured evolution (gqaoa_evolve_plan_*) and the resident
one-launch evolution of small states against the eager streaming rounds and
the oracle.

The plan computes its phase tables on the device (float64 sin/cos, then the
state's precision), the eager call on the host, so the two can differ in the
last bit of a table entry: the bar between them is 1e-12 (complex128) and
1e-6 (complex64) on every readout and amplitude. Against the oracle the bars
of the statevector tests hold (1e-12 and 1e-5). Replays are interleaved with
eager calls and synchronizations, with new angles each time, and the readout
arrays are refilled before each run so a stale value cannot pass.
"""
import os

import numpy as np
import pytest

from gpu_common import log, need_gpu, rand_lits
from oracle.cost import cost_table
from oracle.evolve import evolve_sv
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m,p,dtype,tol,otol", [(10, 42, 20, g.C128, 1e-12, 1e-12), (16, 67, 64, g.C64, 1e-6, 1e-5),
                                                  (6, 20, 7, g.C128, 1e-12, 1e-12),
                                                  (15, 63, 12, g.C128, 1e-12, 1e-12),
                                                  (22, 92, 6, g.C64, 1e-6, 1e-5)])
def test_plan_matches_eager_and_oracle(n, m, p, dtype, tol, otol):
    """n = 6, 10: both resident; n = 15 (complex128) and 16 (complex64): the
    captured streaming rounds with their finalize launches against the eager
    calls; n = 22: more than 1024 blocks per pass, so the captured graph also
    folds the partial rows before each finalize."""
    torch = need_gpu()
    lits = rand_lits(n, m, 70 + n)
    cost, _ = g.gqaoa_cost_table(n, lits)
    ref_cost = cost_table(n, lits)
    target = int(np.min(ref_cost))                    # the lowest occupied level (0 when satisfiable)
    plan = g.EvolvePlan(n, m, cost, p, dtype=dtype, target_level=target)
    try:
        for rep in range(3):
            b, gm = inst.uniform_angles(80 + rep, p)
            psi_e, pe, ee, ne = g.gqaoa_evolve(n, m, cost, b, gm, dtype=dtype, target_level=target)
            torch.cuda.synchronize()
            plan.psi.fill_(0)
            ps, en, no = plan.run(b, gm)
            log(f"evolve plan n={n} p={p} dtype={dtype} replay {rep}")
            for x, y in ((ps, pe), (en, ee), (no, ne)):
                assert np.abs(x - y).max() <= tol * max(1.0, np.abs(y).max())
            assert float((plan.psi - psi_e).abs().max()) <= tol
            _, rp, re, rn = evolve_sv(n, ref_cost, b, gm, target=target)
            assert np.abs(ps - rp).max() < otol and np.abs(no - rn).max() < otol
            assert np.abs(en - re).max() < otol * m
    finally:
        plan.close()


def test_plan_from_given_state():
    """init_uniform = 0: each run starts from psi's contents; two runs of p
    rounds from |s> equal one eager call of 2p rounds."""
    torch = need_gpu()
    n, m, p = 12, 50, 9
    lits = rand_lits(n, m, 77)
    cost, _ = g.gqaoa_cost_table(n, lits)
    b, gm = inst.uniform_angles(78, 2 * p)
    psi0 = torch.full((1 << n,), 2.0 ** (-n / 2), dtype=torch.complex128, device="cuda")
    plan = g.EvolvePlan(n, m, cost, p, dtype=g.C128, init_uniform=False, psi=psi0.clone())
    try:
        plan.run(b[:p], gm[:p])
        ps2, _, _ = plan.run(b[p:], gm[p:])
        psi_e, pe, _, _ = g.gqaoa_evolve(n, m, cost, b, gm, dtype=g.C128)
        torch.cuda.synchronize()
        assert float((plan.psi - psi_e).abs().max()) < 1e-12
        assert abs(ps2[-1] - pe[-1]) < 1e-12
        with pytest.raises(ValueError):
            plan.run(b[:p - 1], gm[:p - 1])
        with pytest.raises(g.GQAOAError):
            bad = b[:p].copy()
            bad[0] = np.nan
            plan.run(bad, gm[:p])
    finally:
        plan.close()


@pytest.mark.parametrize("dtype,n_max,tol,otol", [(g.C64, 14, 5e-6, 1e-5), (g.C128, 13, 1e-12, 1e-12)])
def test_resident_matches_streaming_every_size(dtype, n_max, tol, otol):
    """Every n from 3 to the largest resident size (each block shape and
    amplitudes-per-thread count): the one-launch resident evolution against
    the streaming round passes (forced by GQAOA_SV_RESIDENT=0) and the
    oracle, from |s> and from a given state, with a Max-SAT-style target."""
    torch = need_gpu()
    for n in range(3, n_max + 1):
        m = min(inst.m_from_density(n, 4.2), 4 * (n * (n - 1) * (n - 2) // 6))
        lits = rand_lits(n, m, 90 + n)
        cost, _ = g.gqaoa_cost_table(n, lits)
        ref_cost = cost_table(n, lits)
        target = int(np.min(ref_cost))
        p = 12
        b, gm = inst.uniform_angles(91 + n, p)
        rng = np.random.Generator(np.random.PCG64(92 + n))
        v = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
        v /= np.linalg.norm(v)
        cdt = torch.complex64 if dtype == g.C64 else torch.complex128
        for init_uniform in (True, False):
            psi0 = torch.tensor(v, dtype=cdt, device="cuda")
            psi_r, pr, er, nr = g.gqaoa_evolve(n, m, cost, b, gm, dtype=dtype, psi=psi0.clone(),
                                               init_uniform=init_uniform, target_level=target)
            os.environ["GQAOA_SV_RESIDENT"] = "0"
            try:
                psi_s, ps, es, ns = g.gqaoa_evolve(n, m, cost, b, gm, dtype=dtype, psi=psi0.clone(),
                                                   init_uniform=init_uniform, target_level=target)
            finally:
                del os.environ["GQAOA_SV_RESIDENT"]
            torch.cuda.synchronize()
            assert float((psi_r - psi_s).abs().max()) <= tol, (n, init_uniform)
            for x, y in ((pr, ps), (nr, ns)):
                assert np.abs(x - y).max() <= tol, (n, init_uniform)
            assert np.abs(er - es).max() <= tol * m
            _, rp, re, rn = evolve_sv(n, ref_cost, b, gm, psi0=None if init_uniform else v, target=target)
            assert np.abs(pr - rp).max() < otol and np.abs(nr - rn).max() < otol, (n, init_uniform)
            assert np.abs(er - re).max() < otol * m
        log(f"resident n={n} dtype={dtype} ok")
