"""Batched cost tables and the statevector work items of the batched scan,
against the oracle: tables bit-exact (every size class, n < 5 included);
item P_sol and E against the oracle's complex128 statevector evolution
(float32 state, 1e-5), including Max-SAT targets, every block shape (n = 3
to 14) and the n = 14 limit; and the level-space scan of the same items
within 1e-5."""
import numpy as np
import pytest

from oracle.cost import cost_table, level_histogram, min_level
from oracle.evolve import evolve_sv
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

from gpu_common import log, need_gpu, rand_lits

pytestmark = pytest.mark.gpu
P_LIST = [1, 4, 16, 64]


def _set(seed, sizes, d=4.2):
    its = []
    for k, n in enumerate(sizes):
        m = max(1, min(inst.m_from_density(n, d), 4 * (n * (n - 1) * (n - 2) // 6)))
        its.append((n, rand_lits(n, m, seed + k)))
    return its


def test_cost_batched_bit_exact():
    need_gpu()
    its = _set(40, [3, 4, 5, 7, 9, 11, 12, 14, 16, 13])
    ns = [n for n, _ in its]
    ms = [l.shape[0] for _, l in its]
    costs, off, hists = g.gqaoa_cost_batched(ns, ms, [l for _, l in its])
    c = costs.cpu().numpy()
    h = hists.cpu().numpy()
    assert (off[1:] - off[:-1] >= 2 ** np.array(ns)).all() and (off % 64 == 0).all()
    for i, (n, l) in enumerate(its):
        ref = cost_table(n, l)
        np.testing.assert_array_equal(c[off[i]:off[i] + 2 ** n], ref.astype(np.uint8))
        np.testing.assert_array_equal(h[i, :ms[i] + 1], level_histogram(ref, ms[i]))
    np.testing.assert_array_equal(h, g.gqaoa_hist_batched(ns, ms, [l for _, l in its], hist_stride=h.shape[1]).cpu().numpy())


@pytest.mark.parametrize("unsat", [False, True])
def test_items_match_oracle_statevector(unsat):
    need_gpu()
    if unsat:
        pool = inst.batched_scan_instances(44, 6, 6, 12, want="unsat", density_range=(4.6, 8.0), dup="drop")
    else:
        pool = inst.batched_scan_instances(43, 6, 5, 14)
    ns = [it.n for it in pool]
    ms = [it.m for it in pool]
    refc = [cost_table(it.n, it.lits) for it in pool]
    targets = [min_level(level_histogram(c, it.m)) for c, it in zip(refc, pool)] if unsat else None
    costs, _, _ = g.gqaoa_cost_batched(ns, ms, [it.lits for it in pool], with_hist=False)
    rng = np.random.Generator(np.random.PCG64(45 + unsat))
    item_inst = np.repeat(np.arange(len(pool)), 4)
    beta = rng.uniform(0, 2 * np.pi, item_inst.size)
    gamma = rng.uniform(0, np.pi, item_inst.size)
    log(f"sv items unsat={unsat}: {item_inst.size} items")
    ps, en = g.gqaoa_sv_items(ns, ms, costs, item_inst, beta, gamma, P_LIST, targets=targets, with_energy=True)
    ps, en = ps.cpu().numpy(), en.cpu().numpy()
    for k, i in enumerate(item_inst):
        t = 0 if targets is None else targets[i]
        _, rp, re, _ = evolve_sv(ns[i], refc[i], np.full(64, beta[k]), np.full(64, gamma[k]), target=t)
        assert np.abs(ps[k] - rp[P_LIST]).max() < 1e-5, (k, ps[k], rp[P_LIST])
        assert np.abs(en[k] - re[P_LIST]).max() / ms[i] < 1e-5
    # the level-space scan of the same items (per-instance one-pair grids)
    H = np.zeros((len(pool), max(ms) + 1), dtype=np.int64)
    for i, c in enumerate(refc):
        H[i, :ms[i] + 1] = level_histogram(c, ms[i])
    for k in range(4):
        sel = np.arange(len(pool)) * 4 + k
        sp, _ = g.gqaoa_scan_batched(ns, ms, H, beta[sel].reshape(-1, 1), gamma[sel].reshape(-1, 1), P_LIST,
                                     targets=targets, with_energy=False)
        assert np.abs(sp.cpu().numpy().reshape(len(pool), -1) - ps[sel]).max() < 1e-5


def test_items_every_block_shape():
    """One instance for every n from 3 to 14: one-wave blocks with 1 to 16
    amplitudes per lane (n <= 6 leaves lanes without amplitudes) and blocks
    of 128 to 1024 threads, against the oracle's statevector."""
    need_gpu()
    its = _set(50, list(range(3, 15)))
    ns = [n for n, _ in its]
    ms = [l.shape[0] for _, l in its]
    costs, _, _ = g.gqaoa_cost_batched(ns, ms, [l for _, l in its], with_hist=False)
    rng = np.random.Generator(np.random.PCG64(51))
    item_inst = np.repeat(np.arange(len(its)), 3)
    beta = rng.uniform(0, 2 * np.pi, item_inst.size)
    gamma = rng.uniform(0, np.pi, item_inst.size)
    refc = [cost_table(n, l) for n, l in its]
    targets = [min_level(level_histogram(c, m)) for c, m in zip(refc, ms)]
    log(f"sv items n=3..14: {item_inst.size} items")
    ps, en = g.gqaoa_sv_items(ns, ms, costs, item_inst, beta, gamma, P_LIST, targets=targets, with_energy=True)
    ps, en = ps.cpu().numpy(), en.cpu().numpy()
    for k, i in enumerate(item_inst):
        _, rp, re, _ = evolve_sv(ns[i], refc[i], np.full(64, beta[k]), np.full(64, gamma[k]), target=targets[i])
        assert np.abs(ps[k] - rp[P_LIST]).max() < 1e-5, (ns[i], ps[k], rp[P_LIST])
        assert np.abs(en[k] - re[P_LIST]).max() / ms[i] < 1e-5, ns[i]


def test_streamed_items_beyond_registers():
    """Instances with n = 15..17 take the streaming round passes (all items of
    one n in one batch) in the same call as register-held ones (n = 12..14),
    with Max-SAT targets: against the oracle's statevector (1e-5) and the
    level-space scan of the same cells (1e-5)."""
    need_gpu()
    its = _set(60, [12, 15, 13, 16, 14, 17], d=5.5)
    ns = [n for n, _ in its]
    ms = [l.shape[0] for _, l in its]
    costs, _, _ = g.gqaoa_cost_batched(ns, ms, [l for _, l in its], with_hist=False)
    refc = [cost_table(n, l) for n, l in its]
    hists = [level_histogram(c, m) for c, m in zip(refc, ms)]
    targets = [min_level(h) for h in hists]
    rng = np.random.Generator(np.random.PCG64(61))
    item_inst = np.array([0, 1, 1, 2, 3, 3, 3, 4, 5, 5], dtype=np.int32)
    beta = rng.uniform(0, 2 * np.pi, item_inst.size)
    gamma = rng.uniform(0, np.pi, item_inst.size)
    log(f"streamed + register items: {item_inst.size} items, n = {ns}")
    ps, en = g.gqaoa_sv_items(ns, ms, costs, item_inst, beta, gamma, P_LIST, targets=targets, with_energy=True)
    ps, en = ps.cpu().numpy(), en.cpu().numpy()
    H = np.zeros((len(its), max(ms) + 1), dtype=np.int64)
    for i, h in enumerate(hists):
        H[i, :ms[i] + 1] = h
    for k, i in enumerate(item_inst):
        _, rp, re, _ = evolve_sv(ns[i], refc[i], np.full(64, beta[k]), np.full(64, gamma[k]), target=targets[i])
        assert np.abs(ps[k] - rp[P_LIST]).max() < 1e-5, (ns[i], ps[k], rp[P_LIST])
        assert np.abs(en[k] - re[P_LIST]).max() / ms[i] < 1e-5, ns[i]
        sp, _ = g.gqaoa_scan_batched([ns[i]], [ms[i]], H[i:i + 1], [beta[k]], [gamma[k]], P_LIST,
                                     targets=[targets[i]], with_energy=False)
        assert np.abs(sp.cpu().numpy().reshape(-1) - ps[k]).max() < 1e-5, ns[i]


def test_items_at_the_size_limit():
    """n = 14, the largest item: 1024 threads of 16 register-held amplitudes."""
    need_gpu()
    n, m = 14, 59
    lits = rand_lits(n, m, 46)
    costs, _, _ = g.gqaoa_cost_batched([n], [m], [lits], with_hist=False)
    ref = cost_table(n, lits)
    beta, gamma = np.array([2.4, 4.1]), np.array([0.3, 1.9])
    ps, _ = g.gqaoa_sv_items([n], [m], costs, [0, 0], beta, gamma, [2, 7, 30])
    for k in range(2):
        _, rp, _, _ = evolve_sv(n, ref, np.full(30, beta[k]), np.full(30, gamma[k]))
        assert np.abs(ps.cpu().numpy()[k] - rp[[2, 7, 30]]).max() < 1e-5
