"""X-QAOA: QAOA with the transverse-field mixer (oracle, test only).

Sec. II.B compares G-QAOA with the usual QAOA whose mixer is H_X = sum_i X_i
(Table I, rows "X"). One round applies exp(-i gamma H_P), then
exp(-i beta H_X) = prod_i exp(-i beta X_i), each factor acting on the pair of
amplitudes that differ in bit i: (a, b) -> (cos beta a - i sin beta b,
cos beta b - i sin beta a). The initial state is |+>. Readouts as for
G-QAOA (P_sol at the target level, E of Eq. (4), norm). There is no level
symmetry, so this is statevector only.
"""
from __future__ import annotations

import numpy as np

from .evolve import uniform_state


def apply_x_mixer(psi: np.ndarray, n: int, beta: float) -> np.ndarray:
    """prod_q exp(-i beta X_q) on a statevector whose index bit q is qubit q."""
    c, s = np.cos(beta), np.sin(beta)
    psi = psi.copy()
    for q in range(n):
        v = psi.reshape(-1, 2, 1 << q)          # axis 1 is bit q
        a = v[:, 0, :].copy()
        b = v[:, 1, :].copy()
        v[:, 0, :] = c * a - 1j * s * b
        v[:, 1, :] = c * b - 1j * s * a
    return psi


def evolve_x(n: int, cost, betas, gammas, psi0=None, target: int = 0):
    """X-QAOA statevector evolution. Returns (psi_p, psol[p+1], energy[p+1], norm[p+1])."""
    cost = np.asarray(cost, dtype=np.int64)
    psi = uniform_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    betas = np.asarray(betas, dtype=np.float64)
    gammas = np.asarray(gammas, dtype=np.float64)
    p = len(betas)

    def readout(v):
        pr = np.abs(v) ** 2
        return float(pr[cost == target].sum()), float((cost * pr).sum()), float(pr.sum())

    psol, energy, norm = np.empty(p + 1), np.empty(p + 1), np.empty(p + 1)
    psol[0], energy[0], norm[0] = readout(psi)
    for j in range(p):
        psi = np.exp(-1j * gammas[j] * cost) * psi
        psi = apply_x_mixer(psi, n, betas[j])
        psol[j + 1], energy[j + 1], norm[j + 1] = readout(psi)
    return psi, psol, energy, norm
