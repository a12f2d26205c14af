"""Host logic of the lockstep optimizer (optim.lockstep_lbfgsb): many scipy
L-BFGS-B runs whose objective evaluations are served in batches take exactly
the steps of separate scipy calls, and an evaluation error ends every run.
The objective here is the oracle's level-space P_sol and adjoint gradient
(CPU), standing in for the device's batched gradient."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle.cost import cost_table, level_histogram
from oracle.grad import grad_hist
from paper_2402_02585_amd import instances as inst
from paper_2402_02585_amd.optim import lockstep_lbfgsb


def _problems():
    probs = []
    for k, (n, m, p) in enumerate([(8, 34, 3), (9, 38, 5), (10, 42, 2), (8, 30, 6), (9, 40, 4)]):
        lits = inst.random_3sat(np.random.Generator(np.random.PCG64(50 + k)), n, m)
        h = level_histogram(cost_table(n, lits), m)
        rng = np.random.Generator(np.random.PCG64(60 + k))
        probs.append((h, p, np.concatenate([np.full(p, rng.uniform(3, 5)), np.full(p, rng.uniform(0.1, 0.6))])))
    return probs


def _fg(h, p, x):
    P, db, dg = grad_hist(h, x[:p], x[p:])
    return -P, -np.concatenate([db, dg])


def test_lockstep_equals_separate_runs():
    probs = _problems()
    calls = []

    def evaluate(idx, xs):
        calls.append(len(idx))
        out = [_fg(probs[i][0], probs[i][1], x) for i, x in zip(idx, xs)]
        return [o[0] for o in out], [o[1] for o in out]

    res = lockstep_lbfgsb(evaluate, [pr[2] for pr in probs], max_workers=3)
    for (h, p, x0), r in zip(probs, res):
        ref = minimize(lambda x: _fg(h, p, x), x0, jac=True, method="L-BFGS-B", options={"ftol": 1e-6})
        np.testing.assert_array_equal(r.x, ref.x)
        assert r.fun == ref.fun and r.nfev == ref.nfev
    assert max(calls) > 1, "evaluations were never batched"


def test_evaluation_error_ends_all_runs():
    probs = _problems()
    n = {"calls": 0}

    def evaluate(idx, xs):
        n["calls"] += 1
        if n["calls"] == 3:
            raise ValueError("device call failed")
        out = [_fg(probs[i][0], probs[i][1], x) for i, x in zip(idx, xs)]
        return [o[0] for o in out], [o[1] for o in out]

    with pytest.raises(ValueError):
        lockstep_lbfgsb(evaluate, [pr[2] for pr in probs])
