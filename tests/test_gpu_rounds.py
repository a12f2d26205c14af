"""Rounds-to-target (crossing scan) and Max-SAT targets on the GPU against
the oracle (oracle/rounds.py): every grid pair's first crossing on
satisfiable (target 0) and unsatisfiable (target k_min) instances, the
Grover closed form on two-level histograms, the grid minimum with and
without refinement, and the full-angle search."""
import math

import numpy as np
import pytest

from oracle.cost import cost_table, level_histogram
from oracle.evolve import evolve_hist
from oracle.rounds import crossing_trace, first_crossing, grid_rounds_to_target, maxsat_level
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst
from paper_2402_02585_amd import optim, rounds

from gpu_common import log, need_gpu

pytestmark = pytest.mark.gpu

# The kernel decides P >= S on its float32 P_sol; a first-crossing round that
# differs from the oracle's is accepted only if the oracle's own P trace is
# within this margin of S at every round between the two answers.
MARGIN = 1e-4


def _consistent(trace, S, j_gpu):
    """j_gpu agrees with the oracle P trace (rounds 0..p_max) up to MARGIN."""
    before = trace[1:j_gpu] if j_gpu else trace[1:]
    if (before >= S + MARGIN).any():
        return False
    return j_gpu == 0 or trace[j_gpu] >= S - MARGIN


def _instances(kind):
    if kind == "sat":
        its = inst.batched_scan_instances(21, 5, 8, 12, density_range=(2.0, 4.5), dup="drop")
    else:
        its = inst.batched_scan_instances(22, 5, 8, 12, want="unsat", density_range=(4.6, 8.0), dup="drop")
    ns = [it.n for it in its]
    ms = [it.m for it in its]
    hd = g.gqaoa_hist_batched(ns, ms, [it.lits for it in its], hist_stride=max(ms) + 1).cpu().numpy()
    for k, it in enumerate(its):
        ref = level_histogram(cost_table(it.n, it.lits), it.m)
        assert (hd[k, :it.m + 1].astype(np.int64) == ref).all()
    return its, ns, ms, hd


@pytest.mark.parametrize("kind", ["sat", "unsat"])
@pytest.mark.parametrize("S", [0.25, 0.5])
def test_crossing_grid_matches_oracle(kind, S):
    need_gpu()
    its, ns, ms, hd = _instances(kind)
    if kind == "sat":
        targets = np.zeros(len(its), dtype=np.int32)
    else:
        targets, D = rounds.maxsat_targets(ns, hd)
        assert (targets >= 1).all()
    gb, gg = optim.fundamental_grid(20, 12)
    p_max = 120
    log(f"crossing {kind} S={S}")
    first = g.gqaoa_scan_crossing(ns, ms, hd, gb, gg, p_max, S, targets=targets).cpu().numpy()
    exact = total = 0
    for k, it in enumerate(its):
        ref_h = level_histogram(cost_table(it.n, it.lits), it.m)
        if kind == "unsat":
            assert maxsat_level(ref_h, it.n)[0] == targets[k]
        for gi, gm in enumerate(gg):
            for bi, b in enumerate(gb):
                j_ref = first_crossing(ref_h, b, gm, S, p_max, int(targets[k]))
                j_gpu = int(first[k, gi, bi])
                total += 1
                if j_gpu == j_ref:
                    exact += 1
                    continue
                tr = crossing_trace(ref_h, b, gm, p_max, int(targets[k]))
                assert _consistent(tr, S, j_gpu), (k, gi, bi, j_gpu, j_ref)
    assert exact >= 0.99 * total, (exact, total)


@pytest.mark.parametrize("levels,target", [((0, 1), 0), ((3, 4), 3)])
@pytest.mark.parametrize("S", [0.25, 0.5, 0.75])
def test_two_level_grover_closed_form(levels, target, S):
    # synthetic two-level histogram (n = 16, 37 states on the lower level):
    # beta = gamma = pi is Grover's iteration, P_j = sin^2((2j+1) theta)
    need_gpu()
    n = 16
    h = np.zeros((1, 6), dtype=np.uint64)
    h[0, levels[0]] = 37
    h[0, levels[1]] = (1 << n) - 37
    theta = math.asin(math.sqrt(37 / 2 ** n))
    j = max(1, math.ceil((math.asin(math.sqrt(S)) / theta - 1) / 2))
    first = g.gqaoa_scan_crossing([n], [5], h, [math.pi], [math.pi], 400, S, targets=[target])
    assert int(first.item()) == j


def test_no_crossing_and_early_exit():
    need_gpu()
    h = np.array([[2, 100, 110, 44]], dtype=np.uint64)   # sums to 256 = 2^8
    # beta = 0: the mixer is the identity, P_0 stays at 2/256 for every gamma
    first = g.gqaoa_scan_crossing([8], [3], h, [0.0, 0.0], np.linspace(0, math.pi, 5), 1000, 0.5)
    assert int(first.abs().sum().item()) == 0


def test_single_pair_rounds_against_oracle_grid():
    need_gpu()
    its, ns, ms, hd = _instances("sat")
    grid = (24, 12)
    p_max = 150
    p0, b0, g0 = rounds.single_pair_rounds(ns, ms, hd, 0.5, p_max, grid=grid, zoom_levels=0)
    gb, gg = optim.fundamental_grid(*grid)
    for k, it in enumerate(its):
        ref_h = level_histogram(cost_table(it.n, it.lits), it.m)
        p_ref, first_ref = grid_rounds_to_target(ref_h, gb, gg, 0.5, p_max)
        if p0[k] != p_ref:
            # only a near-threshold pair may move the minimum
            tr = crossing_trace(ref_h, b0[k], g0[k], p_max)
            assert abs(int(p0[k]) - p_ref) <= 1 and _consistent(tr, 0.5, int(p0[k]))
        if p0[k]:
            # the returned pair reaches S at p0 in the oracle's evolution
            ps = evolve_hist(ref_h, np.full(p0[k], b0[k]), np.full(p0[k], g0[k]))[1][-1]
            assert ps >= 0.5 - MARGIN
    p1, b1, g1 = rounds.single_pair_rounds(ns, ms, hd, 0.5, p_max, grid=grid, zoom_levels=2)
    assert ((p1 <= p0) | (p0 == 0)).all()
    for k, it in enumerate(its):
        if p1[k]:
            ref_h = level_histogram(cost_table(it.n, it.lits), it.m)
            ps = evolve_hist(ref_h, np.full(p1[k], b1[k]), np.full(p1[k], g1[k]))[1][-1]
            assert ps >= 0.5 - MARGIN


def test_full_rounds_reach_target_in_oracle():
    torch = need_gpu()
    it = inst.batched_scan_instances(23, 1, 10, 10, density_range=(3.5, 4.5), dup="drop")[0]
    cost, hist = g.gqaoa_cost_table(it.n, it.lits)
    h = hist.cpu().numpy().reshape(1, -1)
    p1, b1, g1 = rounds.single_pair_rounds([it.n], [it.m], h, 0.5, 200, grid=(60, 31), zoom_levels=1)
    assert p1[0] > 1
    pf, bs, gs, P = rounds.full_rounds(it.n, it.m, h[0], 0.5, int(p1[0]), grid=(60, 31))
    assert pf <= p1[0]
    ref_h = level_histogram(cost_table(it.n, it.lits), it.m)
    if bs is not None:
        ps = evolve_hist(ref_h, bs, gs)[1][-1]
        assert ps >= 0.5 - 1e-9 and abs(ps - P) < 1e-9
    # the same optimum through the statevector adjoint at p_full
    if bs is not None:
        j = pf
        b0 = optim.fundamental_grid(60, 31)
        ps_grid, _ = g.gqaoa_scan_batched([it.n], [it.m], h, b0[0], b0[1], [j], with_energy=False)
        k = int(ps_grid.reshape(-1).argmax().item())
        sb, sg = b0[0][k % 60], b0[1][k // 60]
        _, _, Psv = optim.full_gqaoa_statevector(it.n, it.m, cost, j, sb, sg)
        assert abs(Psv - P) < 1e-5, (Psv, P)
    torch.cuda.synchronize()


def test_full_rounds_batched_matches_single_and_oracle():
    """Full G-QAOA rounds for a batch (satisfiable, target 0, and unsatisfiable,
    target k_min) equal the one-instance calls (the lockstep runs take the
    same steps), and the returned angles reach S in the oracle's evolution."""
    need_gpu()
    its = (inst.batched_scan_instances(24, 4, 9, 12, density_range=(3.0, 4.5), dup="drop") +
           inst.batched_scan_instances(25, 3, 9, 11, want="unsat", density_range=(4.6, 8.0), dup="drop"))
    ns = [it.n for it in its]
    ms = [it.m for it in its]
    H = g.gqaoa_hist_batched(ns, ms, [it.lits for it in its], hist_stride=max(ms) + 1).cpu().numpy()
    tg, _ = rounds.maxsat_targets(ns, H)
    tg[:4] = 0
    p1, _, _ = rounds.single_pair_rounds(ns, ms, H, 0.5, 300, targets=tg, grid=(60, 31), zoom_levels=1)
    log(f"full rounds batched: p_single {p1.tolist()}")
    pf, B, G, P, ok = rounds.full_rounds_batched(ns, ms, H, 0.5, p1, targets=tg, grid=(60, 31))
    assert ((pf <= p1) & ((pf > 0) == (p1 > 0))).all()
    assert ok.any()
    for i, it in enumerate(its):
        if p1[i] == 0:
            continue
        pf1, b1, g1, P1 = rounds.full_rounds(it.n, it.m, H[i, :it.m + 1], 0.5, int(p1[i]), target=int(tg[i]),
                                             grid=(60, 31))
        assert pf1 == pf[i]
        if ok[i]:
            np.testing.assert_array_equal(b1, B[i, :pf[i]])
            assert P1 == P[i]
            ref_h = level_histogram(cost_table(it.n, it.lits), it.m)
            ps = evolve_hist(ref_h, B[i, :pf[i]], G[i, :pf[i]], int(tg[i]))[1][-1]
            assert ps >= 0.5 - 1e-9 and abs(ps - P[i]) < 1e-9


def test_per_instance_caps():
    # a per-instance cap only truncates: same rounds where they fit, 0 beyond
    need_gpu()
    its, ns, ms, hd = _instances("sat")
    gb, gg = optim.fundamental_grid(12, 6)
    full = g.gqaoa_scan_crossing(ns, ms, hd, gb, gg, 120, 0.5).cpu().numpy()
    caps = np.array([120, 10, 40, 5, 77])[:len(ns)]
    capped = g.gqaoa_scan_crossing(ns, ms, hd, gb, gg, caps, 0.5).cpu().numpy()
    for k in range(len(ns)):
        assert (capped[k] == np.where(full[k] <= caps[k], full[k], 0)).all()
