"""Fair-sampling kernels against the oracle (oracle/fairness.py): identical
per-run shot counts and per-trial rejection draws on the same counter-based
random numbers, for uniform, skewed and edge-size distributions; and the
G-QAOA solution distribution of the paper's 4-variable instance."""
import json
import math
import os

import numpy as np
import pytest

from oracle.fairness import draws_to_reject, expected_shots_to_all, shots_to_all
from paper_2402_02585_amd import fairness
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst

from gpu_common import log, need_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dists():
    rng = np.random.Generator(np.random.PCG64(5))
    skew = rng.exponential(size=5)
    return {
        "uniform4": np.full(4, 0.9 / 4),
        "skewed5": 0.7 * skew / skew.sum(),
        "single": np.array([0.3]),
        "k64": np.full(64, 0.5 / 64),
    }


@pytest.mark.parametrize("name", ["uniform4", "skewed5", "single", "k64"])
def test_shots_to_all_match_oracle(name):
    need_gpu()
    p = _dists()[name]
    runs = 150 if name == "k64" else 1500
    log(f"shots {name}")
    got = g.gqaoa_shots_to_all(p, runs, seed=21, max_shots=5000).cpu().numpy()
    ref = shots_to_all(p, runs, seed=21, max_shots=5000)
    assert (got == ref).all()


def test_shots_cap_reports_zero():
    need_gpu()
    p = np.array([0.01, 0.01])
    got = g.gqaoa_shots_to_all(p, 300, seed=4, max_shots=20).cpu().numpy()
    ref = shots_to_all(p, 300, seed=4, max_shots=20)
    assert (got == ref).all() and (got == 0).any()


@pytest.mark.parametrize("name", ["uniform4", "skewed5", "k64"])
def test_draws_to_reject_match_oracle(name):
    need_gpu()
    q = _dists()[name]
    K = q.size
    crit = fairness.chi2_critical(K)
    trials = 40 if name == "k64" else 300
    log(f"reject {name}")
    got = g.gqaoa_draws_to_reject(q, trials, seed=8, crit=crit, n_min=5 * K, max_draws=1500).cpu().numpy()
    ref = draws_to_reject(q, trials, seed=8, crit=crit, n_min=5 * K, max_draws=1500)
    assert (got == ref).all()


def test_gqaoa_solutions_are_uniform_and_mean_shots_match_exact():
    """G-QAOA on the 4-variable instance of Sec. IV: every solution has the
    same probability; the Monte Carlo mean of shots-to-all-solutions agrees
    with the exact coupon-collector mean within its 95% interval (x 2)."""
    torch = need_gpu()
    with open(os.path.join(GOLDEN, "paper_instances.json")) as f:
        gi = json.load(f)["4var"]
    lits = inst.parse_paper_clauses(gi["clauses"])
    n, m = gi["n"], lits.shape[0]
    cost, hist = g.gqaoa_cost_table(n, lits)
    psi, psol, _, _ = g.gqaoa_evolve(n, m, cost, [2.1, 1.3], [0.9, 2.4], dtype=g.C128)
    z, pr = fairness.solution_probs(cost, psi)
    assert z.size == int(hist[0].item()) and abs(pr.sum() - psol[-1]) < 1e-13
    assert np.abs(pr - pr.mean()).max() < 1e-14
    r = fairness.shots_to_all_solutions(pr, runs=100000, seed=3)
    assert abs(r["mean"] - expected_shots_to_all(pr)) < 2 * r["ci95"]
    torch.cuda.synchronize()
