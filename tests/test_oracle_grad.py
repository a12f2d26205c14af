"""Pins for the oracle's reverse-sweep gradient (CPU only).

The sweep is checked against three things it does not use:
  * the parameter-shift rule for beta_k, exact because H_M has eigenvalues
    {0, 1} so P is a first-order trigonometric polynomial in beta_k;
  * trigonometric interpolation in gamma_k, exact because P is a
    trigonometric polynomial in gamma_k with integer frequencies bounded by
    the spread of occupied levels;
  * central finite differences (h = 1e-4) of the forward evolution.
"""
import numpy as np
import pytest

from oracle.cost import cost_table, level_histogram, min_level
from oracle.evolve import evolve_hist, evolve_sv
from oracle.grad import grad_hist, grad_sv
from paper_2402_02585_amd import instances as inst


def _rand(n, m, seed):
    return inst.random_3sat(np.random.Generator(np.random.PCG64(seed)), n, m)


def _P(hist, beta, gamma, target):
    return float(evolve_hist(hist, beta, gamma, target)[1][-1])


def _shift_beta(hist, beta, gamma, k, target):
    bp, bm = beta.copy(), beta.copy()
    bp[k] += np.pi / 2
    bm[k] -= np.pi / 2
    return 0.5 * (_P(hist, bp, gamma, target) - _P(hist, bm, gamma, target))


def _trig_interp_gamma(hist, beta, gamma, k, target):
    occ = np.nonzero(hist)[0]
    R = int(occ.max() - occ.min())
    S = 2 * R + 1
    ts = 2 * np.pi * np.arange(S) / S
    vals = []
    for t in ts:
        g = gamma.copy()
        g[k] = gamma[k] + t
        vals.append(_P(hist, beta, g, target))
    c = np.fft.fft(vals) / S                    # P(gamma_k + t) = sum_f c_f e^{i f t}
    freqs = np.fft.fftfreq(S, d=1.0 / S)
    return float(np.real((1j * freqs * c).sum()))


@pytest.mark.parametrize("n,m,p,seed,use_kmin", [(9, 38, 7, 1, False), (9, 45, 7, 2, True),
                                                 (10, 42, 5, 3, False)])
def test_grad_hist_exact_rules(n, m, p, seed, use_kmin):
    cost = cost_table(n, _rand(n, m, seed))
    hist = level_histogram(cost, m)
    t = min_level(hist) if use_kmin else 0
    beta, gamma = inst.uniform_angles(seed, p)
    P, db, dg = grad_hist(hist, beta, gamma, t)
    assert P == pytest.approx(_P(hist, beta, gamma, t), abs=1e-15)
    for k in range(p):
        assert db[k] == pytest.approx(_shift_beta(hist, beta, gamma, k, t), abs=1e-12)
        assert dg[k] == pytest.approx(_trig_interp_gamma(hist, beta, gamma, k, t), abs=1e-11)


@pytest.mark.parametrize("n,m,p,seed", [(8, 34, 6, 4), (10, 42, 8, 5)])
def test_grad_sv_vs_central_fd_and_hist(n, m, p, seed):
    cost = cost_table(n, _rand(n, m, seed))
    hist = level_histogram(cost, m)
    beta, gamma = inst.uniform_angles(seed + 9, p)
    P, db, dg = grad_sv(n, cost, beta, gamma)
    h = 1e-4
    for k in range(p):
        for arr, d in ((beta, db), (gamma, dg)):
            ap, am = arr.copy(), arr.copy()
            ap[k] += h
            am[k] -= h
            if arr is beta:
                fp = evolve_sv(n, cost, ap, gamma)[1][-1]
                fm = evolve_sv(n, cost, am, gamma)[1][-1]
            else:
                fp = evolve_sv(n, cost, beta, ap)[1][-1]
                fm = evolve_sv(n, cost, beta, am)[1][-1]
            assert d[k] == pytest.approx((fp - fm) / (2 * h), abs=1e-6)
    Ph, dbh, dgh = grad_hist(hist, beta, gamma)
    assert P == pytest.approx(Ph, abs=1e-14)
    np.testing.assert_allclose(db, dbh, atol=1e-12)
    np.testing.assert_allclose(dg, dgh, atol=1e-11)


def test_grad_sv_random_initial_state_fd():
    """The statevector sweep also holds from a state that is not |s>."""
    n, m, p = 7, 30, 5
    cost = cost_table(n, _rand(n, m, 6))
    rng = np.random.Generator(np.random.PCG64(6))
    psi0 = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    psi0 /= np.linalg.norm(psi0)
    beta, gamma = inst.uniform_angles(66, p)
    P, db, dg = grad_sv(n, cost, beta, gamma, psi0=psi0)
    h = 1e-5
    for k in range(p):
        bp, bm = beta.copy(), beta.copy()
        bp[k] += h
        bm[k] -= h
        fd = (evolve_sv(n, cost, bp, gamma, psi0)[1][-1] - evolve_sv(n, cost, bm, gamma, psi0)[1][-1]) / (2 * h)
        assert db[k] == pytest.approx(fd, abs=1e-8)
        gp, gm = gamma.copy(), gamma.copy()
        gp[k] += h
        gm[k] -= h
        fd = (evolve_sv(n, cost, beta, gp, psi0)[1][-1] - evolve_sv(n, cost, beta, gm, psi0)[1][-1]) / (2 * h)
        assert dg[k] == pytest.approx(fd, abs=1e-7)


def test_unsat_gradient_is_zero():
    lits = np.concatenate([inst.two_level_instance(5, 0), [[0, 2, 4]]])   # all 8 patterns
    cost = cost_table(5, lits)
    hist = level_histogram(cost, lits.shape[0])
    assert hist[0] == 0
    beta, gamma = inst.uniform_angles(3, 4)
    P, db, dg = grad_hist(hist, beta, gamma, 0)
    assert P == 0.0 and not db.any() and not dg.any()
