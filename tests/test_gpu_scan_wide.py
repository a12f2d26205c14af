"""GPU parity of the batched scan on every register-array size of the scan
kernel: "narrow", 1..40 occupied levels, every size from 4 to 40 (multiples
of 4) with K at a size and next to it; "wide", 41..128 levels, the sizes
above 40 (48, 56, 64, 80, 96, 112, 128) that random 3-SAT instances of the
scan workload (n <= 20) do not reach but unsatisfiable paper-scale sets (m
up to 208) do. Histograms are synthetic (K occupied levels out of 0..m, counts
summing to 2^n; the level-space method does not care which formula produced
them), fed straight into gqaoa_scan_batched and gqaoa_scan_crossing and
compared with the oracle's level-space evolution (float64) at the
single-precision bar: 1e-5 on P_sol and 1e-5 * m on E."""
import numpy as np
import pytest

from gpu_common import log, need_gpu, synthetic_hist
from oracle.evolve import evolve_hist
from oracle.rounds import crossing_trace, first_crossing
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import optim

pytestmark = pytest.mark.gpu

# (levels per instance, m, n) of each set
SETS = {
    "narrow": ([1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 13, 15, 17, 19, 20, 21, 23, 25, 27, 29, 31, 33, 35, 36, 37, 39, 40],
               60, 20),
    "wide": ([41, 47, 48, 49, 56, 63, 64, 65, 79, 80, 81, 96, 100, 112, 127, 128], 200, 30),
}
P_LIST = [1, 4, 16, 64]


def _inputs(name, seed):
    KS, M, N = SETS[name]
    H = np.stack([synthetic_hist(K, M, N, seed + K) for K in KS])
    rng = np.random.Generator(np.random.PCG64(seed))
    targets = np.zeros(len(KS), dtype=np.int32)
    for i in range(1, len(KS), 3):        # every third instance targets another occupied level
        targets[i] = int(rng.choice(np.nonzero(H[i])[0]))
    return KS, M, N, H, targets


@pytest.mark.parametrize("name", list(SETS))
@pytest.mark.parametrize("tile", [None, [1, 4], [4, 2]])
def test_scan_buckets_match_oracle(tile, name):
    need_gpu()
    KS, M, N, H, targets = _inputs(name, 900)
    ns, ms = [N] * len(KS), [M] * len(KS)
    gb, gg = optim.fundamental_grid(64, 5)
    log(f"scan K={KS[0]}..{KS[-1]} tile={tile}")
    psol, energy = g.gqaoa_scan_batched(ns, ms, H, gb, gg, P_LIST, targets=targets, tile=tile)
    psol, energy = psol.cpu().numpy(), energy.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(901))
    worst = 0.0
    for i, K in enumerate(KS):
        for _ in range(6):
            bi, gi = int(rng.integers(0, gb.size)), int(rng.integers(0, gg.size))
            _, rp, re, _ = evolve_hist(H[i], np.full(64, gb[bi]), np.full(64, gg[gi]), int(targets[i]))
            for q, p in enumerate(P_LIST):
                d = abs(psol[i, q, gi, bi] - rp[p])
                worst = max(worst, d)
                assert d < 1e-5, (K, p, gi, bi, psol[i, q, gi, bi], rp[p])
                assert abs(energy[i, q, gi, bi] - re[p]) < 1e-5 * M, (K, p, gi, bi)
    log(f"worst |dP| {worst:.2e}")


@pytest.mark.parametrize("name", list(SETS))
def test_crossing_buckets_match_oracle(name):
    need_gpu()
    KS, M, N, H, targets = _inputs(name, 910)
    ns, ms = [N] * len(KS), [M] * len(KS)
    gb, gg = optim.fundamental_grid(16, 6)
    S, p_max, margin = 0.05, 64, 1e-4
    log(f"crossing K={KS[0]}..{KS[-1]} S={S}")
    first = g.gqaoa_scan_crossing(ns, ms, H, gb, gg, p_max, S, targets=targets).cpu().numpy()
    exact = total = crossed = 0
    for i, K in enumerate(KS):
        t = int(targets[i])
        for gi, gm in enumerate(gg):
            for bi, b in enumerate(gb):
                j_ref = first_crossing(H[i], b, gm, S, p_max, t)
                j_gpu = int(first[i, gi, bi])
                total += 1
                crossed += j_ref > 0
                if j_gpu == j_ref:
                    exact += 1
                    continue
                # a different answer only where the oracle's P lies within the
                # margin of S at every round between the two answers
                tr = crossing_trace(H[i], b, gm, p_max, t)
                before = tr[1:j_gpu] if j_gpu else tr[1:]
                assert not (before >= S + margin).any(), (K, gi, bi, j_gpu, j_ref)
                assert j_gpu == 0 or tr[j_gpu] >= S - margin, (K, gi, bi, j_gpu, j_ref)
    assert exact >= 0.99 * total, (exact, total)
    assert crossed >= total // 10, "too few pairs cross S to exercise the crossing test"
