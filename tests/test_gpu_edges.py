"""GPU: degenerate sizes of the newer paths, against the oracle or the eager
calls: one round (p = 1), one grid cell, one instance, one readout, the
smallest n, for the resident and streaming evolutions, both plans and the
statevector items."""
import numpy as np
import pytest

from gpu_common import log, need_gpu, rand_lits
from oracle.cost import cost_table, level_histogram
from oracle.evolve import evolve_hist, evolve_sv
from paper_2402_02585_amd import gqaoa as g

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,dtype", [(3, g.C128), (3, g.C64), (13, g.C128), (14, g.C64), (15, g.C64)])
def test_one_round(n, dtype):
    """p = 1: resident (n <= 13/14) or streaming (n = 15), eager and plan."""
    torch = need_gpu()
    m = min(4 * (n * (n - 1) * (n - 2) // 6), 60)
    lits = rand_lits(n, m, 300 + n)
    cost, _ = g.gqaoa_cost_table(n, lits)
    ref = evolve_sv(n, cost_table(n, lits), [1.1], [0.7])
    tol = 1e-12 if dtype == g.C128 else 1e-5
    _, ps, en, no = g.gqaoa_evolve(n, m, cost, [1.1], [0.7], dtype=dtype)
    assert np.abs(ps - ref[1]).max() < tol and np.abs(no - ref[3]).max() < tol
    assert np.abs(en - ref[2]).max() < tol * m
    plan = g.EvolvePlan(n, m, cost, 1, dtype=dtype)
    try:
        ps2, _, _ = plan.run([1.1], [0.7])
    finally:
        plan.close()
    torch.cuda.synchronize()
    assert np.abs(ps2 - ps).max() < tol


def test_scan_plan_one_cell_one_instance_one_readout():
    torch = need_gpu()
    n, m = 9, 38
    lits = rand_lits(n, m, 310)
    h = level_histogram(cost_table(n, lits), m)
    H = np.zeros((1, m + 1), dtype=np.uint64)
    H[0] = h
    costs, off, _ = g.gqaoa_cost_batched([n], [m], [lits], with_hist=False)
    plan = g.ScanPlan([n], [m], H, [0.9], [0.4], [1], items=[[0, 0, 0]], costs=costs, cost_off=off[:-1])
    try:
        ps, _ = plan.run()
        ps2, _ = plan.run([2.0], [0.3])
        torch.cuda.synchronize()
        ref = evolve_hist(h, [2.0], [0.3])[1][1]
        assert abs(float(ps2.reshape(-1)[0]) - ref) < 1e-5
        assert abs(float(plan.item_psol.reshape(-1)[0]) - ref) < 1e-5
    finally:
        plan.close()


def test_items_one_readout_and_streamed_single_item():
    """One item of an n = 16 instance (a batch of one streamed state) and one of
    n = 5, num_p = 1, p = 1."""
    need_gpu()
    its = [(16, rand_lits(16, 67, 311)), (5, rand_lits(5, 21, 312))]
    ns = [n for n, _ in its]
    ms = [l.shape[0] for _, l in its]
    costs, _, _ = g.gqaoa_cost_batched(ns, ms, [l for _, l in its], with_hist=False)
    ps, en = g.gqaoa_sv_items(ns, ms, costs, [0, 1], [0.8, 2.2], [0.5, 1.3], [1], with_energy=True)
    ps, en = ps.cpu().numpy(), en.cpu().numpy()
    for k, (n, l) in enumerate(its):
        ref = evolve_sv(n, cost_table(n, l), [[0.8], [2.2]][k], [[0.5], [1.3]][k])
        assert abs(ps[k, 0] - ref[1][1]) < 1e-5 and abs(en[k, 0] - ref[2][1]) / ms[k] < 1e-5
    log("edge items ok")
