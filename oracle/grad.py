"""Gradient of P_sol with respect to all 2p angles (oracle, test only).

Forward (Eq. (3)): phi_k = D_k psi_{k-1}, psi_k = M_k phi_k with
D_k = diag(exp(-i gamma_k C)) and M_k = I + (exp(-i beta_k) - 1)|s><s|.
Objective P = <psi_p| Pi_t |psi_p>, Pi_t the projector on level t.

Reverse sweep (adjoint states): lambda_p = Pi_t psi_p and, for k = p..1,
    mu_k          = M_k^dagger lambda_k = lambda_k + (exp(+i beta_k) - 1)|s><s|lambda_k>
    dP/dbeta_k    = 2 Re( -i exp(-i beta_k) <lambda_k|s> <s|phi_k> )
    dP/dgamma_k   = 2 Re( <mu_k| (-i C) |phi_k> ) = 2 Im( sum_z conj(mu_z) C(z) phi_z )
    lambda_{k-1}  = D_k^dagger mu_k = exp(+i gamma_k C) mu_k.
These follow from dM_k/dbeta_k = -i exp(-i beta_k)|s><s| and
dD_k/dgamma_k = -i C D_k, with dP/dtheta = 2 Re <lambda_p| d psi_p/d theta>.

``grad_sv`` works on the statevector; ``grad_hist`` is the same sweep in the
level space (inner products weighted by w_k = N_k / 2^n).
"""
from __future__ import annotations

import numpy as np

from .evolve import uniform_state


def grad_sv(n: int, cost, betas, gammas, target: int = 0, psi0=None):
    """Returns (P, dP/dbeta[p], dP/dgamma[p]) by the reverse sweep."""
    cost = np.asarray(cost, dtype=np.int64)
    N = 1 << n
    betas = np.asarray(betas, dtype=np.float64)
    gammas = np.asarray(gammas, dtype=np.float64)
    p = len(betas)
    psi = uniform_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    phis = []
    for k in range(p):
        phi = np.exp(-1j * gammas[k] * cost) * psi
        phis.append(phi)
        psi = phi + (np.exp(-1j * betas[k]) - 1.0) * phi.sum() / N
    mask = cost == target
    P = float((np.abs(psi[mask]) ** 2).sum())
    lam = np.where(mask, psi, 0.0)
    dbeta = np.empty(p)
    dgamma = np.empty(p)
    for k in range(p - 1, -1, -1):
        phi = phis[k]
        s_lam = lam.sum()
        s_phi = phi.sum()
        # <lambda|s><s|phi> = conj(sum lambda) * sum phi / N
        dbeta[k] = 2.0 * np.real(-1j * np.exp(-1j * betas[k]) * np.conj(s_lam) * s_phi / N)
        mu = lam + (np.exp(1j * betas[k]) - 1.0) * s_lam / N
        dgamma[k] = 2.0 * np.imag((np.conj(mu) * cost * phi).sum())
        lam = np.exp(1j * gammas[k] * cost) * mu
    return P, dbeta, dgamma


def grad_hist(hist, betas, gammas, target: int = 0):
    """The reverse sweep in the level space, from |s>.

    Returns (P, dP/dbeta[p], dP/dgamma[p]).
    """
    hist = np.asarray(hist, dtype=np.float64)
    w = hist / hist.sum()
    lev = np.arange(len(hist), dtype=np.float64)
    betas = np.asarray(betas, dtype=np.float64)
    gammas = np.asarray(gammas, dtype=np.float64)
    p = len(betas)
    b = np.ones(len(hist), dtype=np.complex128)
    phis = []
    for k in range(p):
        phi = np.exp(-1j * gammas[k] * lev) * b
        phis.append(phi)
        b = phi + (np.exp(-1j * betas[k]) - 1.0) * (w * phi).sum()
    P = float(w[target] * abs(b[target]) ** 2) if target < len(w) else 0.0
    lam = np.zeros_like(b)
    if target < len(w):
        lam[target] = b[target]
    dbeta = np.empty(p)
    dgamma = np.empty(p)
    for k in range(p - 1, -1, -1):
        phi = phis[k]
        s_lam = (w * lam).sum()
        s_phi = (w * phi).sum()
        dbeta[k] = 2.0 * np.real(-1j * np.exp(-1j * betas[k]) * np.conj(s_lam) * s_phi)
        mu = lam + (np.exp(1j * betas[k]) - 1.0) * s_lam
        dgamma[k] = 2.0 * np.imag((w * np.conj(mu) * lev * phi).sum())
        lam = np.exp(1j * gammas[k] * lev) * mu
    return P, dbeta, dgamma
