"""GPU: the device optimizers pinned to a closed form.

With a two-level cost (solutions at level 0, all other assignments at level
1) the single-pair protocol is a p-query search with a phase oracle, so no
angle pair beats Grover's sin^2((2p+1) theta), sin^2 theta = N0 / 2^n
(optimality of Grover search, Zalka 1999), and (pi, pi) reaches it. Both the
plain optimizer (a device call per pair, float64 level space, L-BFGS-B) and
the batched optimizer (float32 scan, grid then zoom windows) must therefore
return that value: the plain one within 1e-6, the batched one within its
float32 rounding and final window spacing (2e-5), neither above it.
"""
import numpy as np
import pytest

from gpu_common import need_gpu
from paper_2402_02585_amd import optim

pytestmark = pytest.mark.gpu
CASES = [(4, 10), (16, 12), (1, 8)]      # (solutions N0, variables n)
P_LIST = [1, 2, 3]


def _bound(N0, n, p):
    theta = np.arcsin(np.sqrt(N0 / 2 ** n))
    assert (2 * p + 1) * theta <= np.pi / 2
    return float(np.sin((2 * p + 1) * theta) ** 2)


def test_batched_optimizer_reaches_grover_bound():
    need_gpu()
    H = np.array([[N0, 2 ** n - N0] for N0, n in CASES], dtype=np.int64)
    ns = [n for _, n in CASES]
    beta, gamma, psol, _ = optim.batched_single_pair(ns, [1] * len(CASES), H, P_LIST, grid=(72, 37))
    for i, (N0, n) in enumerate(CASES):
        for q, p in enumerate(P_LIST):
            b = _bound(N0, n, p)
            assert b - 2e-5 <= psol[i, q] <= b + 2e-6, (N0, n, p, psol[i, q], b)


def test_plain_optimizer_reaches_grover_bound():
    torch = need_gpu()
    gb, gg = optim.fundamental_grid(40, 21)
    gb = gb + 0.05                        # a grid that misses (pi, pi): the refinement must climb
    gg = np.clip(gg + 0.03, 0, np.pi)
    for N0, n in CASES[:2]:
        hist = torch.tensor([N0, 2 ** n - N0], dtype=torch.int64, device="cuda")
        for p in P_LIST:
            r = optim.plain_single_pair(n, 1, hist, p, gb, gg)
            b = _bound(N0, n, p)
            assert r["psol"] == pytest.approx(b, abs=1e-6) and r["psol"] <= b + 1e-12, (N0, n, p, r["psol"], b)
