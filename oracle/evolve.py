"""G-QAOA evolution in complex128 (oracle, test infrastructure only).

Statevector form (Eq. (3)): starting from psi_0 (default |+> = |s>, the
uniform superposition of Eq. (2)), round j applies
    exp(-i gamma_j H_P)  -- diagonal, phase exp(-i gamma_j C(z)) on |z>,
    exp(-i beta_j  H_M)  -- H_M = |s><s| is a projector (Eq. (2)), so
                            exp(-i beta H_M) = I + (exp(-i beta) - 1)|s><s|.
Single-angle-pair form (Eq. (5)) is the same with beta_j = beta, gamma_j = gamma.

Level-space form (App. C, "Optimization"): from |s>, every amplitude depends
on z only through C(z), so the state is one amplitude b_k per occupied energy
level k with weight w_k = N_k / 2^n, and psi_z = 2^(-n/2) b_{C(z)}.

Readouts after each round j (index 0 = the initial state):
    P_sol(j) = sum_{z: C(z)=t} |psi_z|^2  (t = 0: solutions, App. B; t = k_min:
               Max-SAT assignments),
    E(j)     = <psi| H_P |psi> = sum_z C(z) |psi_z|^2  (Eq. (4)),
    norm(j)  = sum_z |psi_z|^2.
"""
from __future__ import annotations

import numpy as np


def _readout(psi: np.ndarray, cost: np.ndarray, target: int):
    prob = np.abs(psi) ** 2
    return (float(prob[cost == target].sum()), float((cost * prob).sum()), float(prob.sum()))


def uniform_state(n: int) -> np.ndarray:
    """|+>^n = |s>, amplitude 2^(-n/2) on every z (Eq. (2))."""
    return np.full(1 << n, 2.0 ** (-n / 2.0), dtype=np.complex128)


def evolve_sv(n: int, cost, betas, gammas, psi0=None, target: int = 0):
    """Statevector G-QAOA, Eq. (3).

    Returns (psi_p, psol[p+1], energy[p+1], norm[p+1]).
    """
    cost = np.asarray(cost, dtype=np.int64)
    N = 1 << n
    psi = uniform_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    betas = np.asarray(betas, dtype=np.float64)
    gammas = np.asarray(gammas, dtype=np.float64)
    p = len(betas)
    psol, energy, norm = np.empty(p + 1), np.empty(p + 1), np.empty(p + 1)
    psol[0], energy[0], norm[0] = _readout(psi, cost, target)
    for j in range(p):
        psi = np.exp(-1j * gammas[j] * cost) * psi           # exp(-i gamma H_P)
        overlap_sum = psi.sum()                              # 2^(n/2) <s|psi>
        psi = psi + (np.exp(-1j * betas[j]) - 1.0) * overlap_sum / N  # mixer
        psol[j + 1], energy[j + 1], norm[j + 1] = _readout(psi, cost, target)
    return psi, psol, energy, norm


def evolve_hist(hist, betas, gammas, target: int = 0):
    """Level-space G-QAOA from |s> (the effective space of App. C).

    hist[k] = N_k. Returns (b_p[m+1], psol[p+1], energy[p+1], norm[p+1]);
    b_k is meaningful only on occupied levels (N_k > 0).
    """
    hist = np.asarray(hist, dtype=np.float64)
    w = hist / hist.sum()
    k = np.arange(len(hist), dtype=np.float64)
    b = np.ones(len(hist), dtype=np.complex128)
    betas = np.asarray(betas, dtype=np.float64)
    gammas = np.asarray(gammas, dtype=np.float64)
    p = len(betas)

    def readout(b):
        prob = w * np.abs(b) ** 2
        return float(prob[target]) if target < len(prob) else 0.0, float((k * prob).sum()), float(prob.sum())

    psol, energy, norm = np.empty(p + 1), np.empty(p + 1), np.empty(p + 1)
    psol[0], energy[0], norm[0] = readout(b)
    for j in range(p):
        b = np.exp(-1j * gammas[j] * k) * b
        s = (w * b).sum()                                    # = <s|psi>
        b = b + (np.exp(-1j * betas[j]) - 1.0) * s
        psol[j + 1], energy[j + 1], norm[j + 1] = readout(b)
    return b, psol, energy, norm


def psol_single_pair_hist(hist, beta: float, gamma: float, p: int, target: int = 0) -> float:
    """P_sol after p rounds of the single-angle-pair protocol, Eq. (5)."""
    _, psol, _, _ = evolve_hist(hist, np.full(p, beta), np.full(p, gamma), target)
    return float(psol[-1])


def energy_single_pair_hist(hist, beta: float, gamma: float, p: int) -> float:
    """Eq. (4) after p rounds of the single-angle-pair protocol."""
    _, _, energy, _ = evolve_hist(hist, np.full(p, beta), np.full(p, gamma))
    return float(energy[-1])
