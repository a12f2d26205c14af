"""Clause cost table and level histogram (oracle, test infrastructure only).

Definitions (Sec. II.A and App. B):
  * assignment tau <-> basis index z, variable v <-> bit v of z (LSB first);
  * a literal on v is satisfied when tau(v) = 1 (plain) or tau(v) = 0
    (negated); with lit = 2*v + neg it is therefore FALSE iff bit_v(z) == neg;
  * a clause is unsatisfied iff all its literals are false;
  * the diagonal of H_P = sum_i H_C^(i) at |tau> is the number of clauses that
    tau leaves unsatisfied (the case table that follows Eq. (1)).

The text's reading is used throughout. ``cost_eq1_pauli`` builds H_P from the
Pauli form of Eq. (1) instead; it equals the text's cost at the bitwise
complement of z (a sign-convention difference in Eq. (1), see the tests).
"""
from __future__ import annotations

import itertools

import numpy as np


def cost_of(z, lits) -> np.ndarray:
    """C(z) for the given assignments z (any int array): the number of
    clauses whose three literals are all false."""
    z = np.asarray(z, dtype=np.int64)
    lits = np.asarray(lits, dtype=np.int64).reshape(-1, 3)
    c = np.zeros(z.shape, dtype=np.int64)
    for clause in lits:
        unsat = np.ones(z.shape, dtype=bool)
        for lit in clause:
            var, neg = lit >> 1, lit & 1
            unsat &= ((z >> var) & 1) == neg
        c += unsat
    return c


def cost_table(n: int, lits, chunk_bits: int = 22) -> np.ndarray:
    """C(z) for z in [0, 2^n): the number of unsatisfied clauses (int64)."""
    N = 1 << n
    out = np.empty(N, dtype=np.int64)
    step = 1 << min(n, chunk_bits)
    for lo in range(0, N, step):
        out[lo:lo + step] = cost_of(np.arange(lo, lo + step, dtype=np.int64), lits)
    return out


def level_histogram(cost: np.ndarray, m: int) -> np.ndarray:
    """N_k = #{z : C(z) = k}, k = 0..m (the state count of each energy
    manifold, App. C "Optimization")."""
    return np.bincount(np.asarray(cost, dtype=np.int64), minlength=m + 1).astype(np.int64)


def satisfying_probability(hist: np.ndarray, n: int) -> float:
    """P = |R_phi| / 2^n with |R_phi| = N_0 (App. B)."""
    return float(hist[0]) / float(1 << n)


def min_level(hist: np.ndarray) -> int:
    """k_min, the lowest occupied level (the Max-SAT level, App. B)."""
    return int(np.nonzero(np.asarray(hist))[0][0])


def count_solutions_enum(n: int, lits) -> int:
    """|R_phi| by enumerating every assignment with Python booleans.

    Independent of ``cost_table``: evaluates phi(tau) as AND over clauses of
    OR over literals (App. B), for small n only.
    """
    clauses = [tuple(int(x) for x in c) for c in np.asarray(lits).reshape(-1, 3)]
    count = 0
    for tau in itertools.product((False, True), repeat=n):
        # tau[v] is the value of variable v
        ok = True
        for c in clauses:
            clause_true = False
            for lit in c:
                v, neg = lit >> 1, bool(lit & 1)
                if tau[v] != neg:          # x with tau=1, or x-bar with tau=0
                    clause_true = True
                    break
            if not clause_true:
                ok = False
                break
        count += ok
    return count


def cost_eq1_pauli(n: int, lits) -> np.ndarray:
    """Diagonal of H_P built literally from Eq. (1):
    H_C = (1/8) prod_j (1 - s_j Z_{v_j}), Z = |0><0| - |1><1| on qubit v,
    s = +1 for a plain literal and -1 for a negated one.

    Qubit v is bit v of z, so Z_v has diagonal 1 - 2*bit_v(z).
    """
    lits = np.asarray(lits, dtype=np.int64).reshape(-1, 3)
    z = np.arange(1 << n, dtype=np.int64)
    diag = np.zeros(1 << n, dtype=np.float64)
    for clause in lits:
        term = np.full(1 << n, 1.0 / 8.0)
        for lit in clause:
            v, neg = lit >> 1, lit & 1
            s = -1.0 if neg else 1.0
            zdiag = 1.0 - 2.0 * ((z >> v) & 1)
            term = term * (1.0 - s * zdiag)
        diag += term
    return diag
