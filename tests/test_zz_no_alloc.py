"""GPU: the allocation-free cost table (gqaoa_cost_table_noalloc, scratch in a
static device array) against gqaoa_cost_table, bit for bit, on two calls in a
row with the second input smaller (fewer blocks, fewer levels: the array keeps
the first call's rows, which the second must not read), and without a
histogram. Called through the C ABI by the binding."""
import numpy as np
import pytest

from gpu_common import log, need_gpu, rand_lits
from paper_2402_02585_amd import gqaoa as g

pytestmark = pytest.mark.gpu


def _both(n, lits, with_hist=True):
    torch = need_gpu()
    m = len(lits)
    log(f"noalloc cost table n={n} m={m} hist={with_hist}")
    ref_cost, ref_hist = g.gqaoa_cost_table(n, lits, with_hist=with_hist)
    cost = torch.full((1 << n,), 0xAB, dtype=torch.uint8, device="cuda")
    hist = torch.full((m + 1,), -7, dtype=torch.int64, device="cuda") if with_hist else None
    g.gqaoa_cost_table_noalloc(n, lits, hist=hist, cost=cost)
    torch.cuda.synchronize()
    assert torch.equal(cost, ref_cost)
    if with_hist:
        assert torch.equal(hist, ref_hist)
        assert int(hist.sum().item()) == 1 << n
    return cost, hist


def test_noalloc_two_calls_second_smaller():
    need_gpu()
    _both(24, rand_lits(24, 231, 11))   # 2048 blocks, 232 levels
    _both(12, rand_lits(12, 50, 12))    # one block, 51 levels
    _both(9, rand_lits(9, 17, 13), with_hist=False)
    _both(3, rand_lits(3, 2, 14))


def test_noalloc_headline_size_then_smaller():
    need_gpu()
    _both(28, rand_lits(28, 118, 2))
    _both(20, rand_lits(20, 84, 3))
