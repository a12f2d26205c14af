"""GPU parity: cost table and level histograms are bit-exact with the oracle."""
import numpy as np
import pytest

from gpu_common import c2_instance, log, need_gpu, rand_lits
from oracle import brute
from oracle.cost import cost_table, level_histogram
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

pytestmark = pytest.mark.gpu

CASES = [(3, 1, 1), (3, 8, 2), (4, 9, 3), (5, 20, 4), (6, 25, 5), (8, 34, 6), (10, 42, 7), (11, 46, 8),
         (12, 80, 9), (13, 55, 10), (14, 59, 11), (16, 255, 12), (17, 71, 13), (18, 76, 14), (20, 84, 15),
         (20, 200, 16)]


@pytest.mark.parametrize("n,m,seed", CASES)
def test_cost_table_bit_exact(n, m, seed):
    need_gpu()
    log(f"cost table n={n} m={m} seed={seed}")
    lits = rand_lits(n, m, seed)
    cost, hist = g.gqaoa_cost_table(n, lits)
    ref = cost_table(n, lits)
    np.testing.assert_array_equal(cost.cpu().numpy(), ref.astype(np.uint8))
    np.testing.assert_array_equal(hist.cpu().numpy(), level_histogram(ref, m))


def test_cost_table_deterministic_and_two_level():
    need_gpu()
    lits = inst.two_level_instance(15, keep_pattern=6)
    c1, h1 = g.gqaoa_cost_table(15, lits)
    c2, h2 = g.gqaoa_cost_table(15, lits)
    assert bool((c1 == c2).all()) and bool((h1 == h2).all())
    assert h1.cpu().tolist()[:2] == [2 ** 12, 2 ** 15 - 2 ** 12]


def _all_positive(n):
    """Every clause (x_a or x_b or x_c) with a < b < c: z = 0 falsifies all of
    them, so the costs reach far beyond m/8 (the levels are counted outside
    the kernels' counting window, one by one)."""
    import itertools
    return np.array([[2 * a, 2 * b, 2 * c] for a, b, c in itertools.combinations(range(n), 3)], dtype=np.int32)


@pytest.mark.parametrize("n", [8, 12])
def test_cost_table_levels_far_from_the_mean(n):
    need_gpu()
    lits = _all_positive(n)
    m = lits.shape[0]
    cost, hist = g.gqaoa_cost_table(n, lits)
    ref = cost_table(n, lits)
    assert ref.max() == m
    np.testing.assert_array_equal(cost.cpu().numpy(), ref.astype(np.uint8))
    np.testing.assert_array_equal(hist.cpu().numpy(), level_histogram(ref, m))


def test_hist_batched_levels_far_from_the_mean():
    need_gpu()
    lits = [_all_positive(n) for n in (8, 9, 12)]
    ns, ms = [8, 9, 12], [l.shape[0] for l in lits]
    hists = g.gqaoa_hist_batched(ns, ms, lits, hist_stride=max(ms) + 1).cpu().numpy()
    for i, n in enumerate(ns):
        ref = level_histogram(cost_table(n, lits[i]), ms[i])
        np.testing.assert_array_equal(hists[i, :ms[i] + 1], ref)


def test_hist_batched_matches_oracle():
    need_gpu()
    insts = inst.batched_scan_instances(3, 24, 4, 14, sat_only=False)
    ns = [it.n for it in insts]
    ms = [it.m for it in insts]
    hists = g.gqaoa_hist_batched(ns, ms, [it.lits for it in insts], hist_stride=80).cpu().numpy()
    for i, it in enumerate(insts):
        ref = level_histogram(cost_table(it.n, it.lits), it.m)
        np.testing.assert_array_equal(hists[i, :it.m + 1], ref)
        assert not hists[i, it.m + 1:].any()
    flat = np.concatenate([np.asarray(it.lits, dtype=np.int32).reshape(-1) for it in insts])
    again = g.gqaoa_hist_batched(ns, ms, flat, hist_stride=80).cpu().numpy()
    np.testing.assert_array_equal(again, hists)


def test_full_size_n28_whole_table_and_histogram():
    """n = 28, m = 118: the whole cost table against the oracle's brute-force
    count of every assignment, in 2^24-entry chunks, and the histogram against
    the counts of those brute-force costs."""
    torch = need_gpu()
    it = c2_instance()
    log(f"n=28 m=118 draw={it.draw}")
    cost, hist = g.gqaoa_cost_table(28, it.lits)
    ref_hist = np.zeros(it.m + 1, dtype=np.int64)
    chunk = 1 << 24
    for z0 in range(0, 1 << 28, chunk):
        ref = brute.cost_range_brute(28, it.lits, z0, chunk)
        got = cost[z0:z0 + chunk].cpu().numpy()
        if not np.array_equal(got, ref):
            bad = np.nonzero(got != ref)[0]
            raise AssertionError(f"{bad.size} costs differ in [{z0}, {z0 + chunk}), first z={z0 + int(bad[0])}")
        ref_hist += np.bincount(ref, minlength=it.m + 1)[:it.m + 1]
    np.testing.assert_array_equal(hist.cpu().numpy(), ref_hist)
    del cost
    torch.cuda.empty_cache()
