"""Seeded synthetic random 3-SAT workloads and angle draws.

This module is the only code shared by the HIP path and the CPU oracle. It
holds no part of the G-QAOA arithmetic: it draws clauses and angles from
seeded numpy generators, parses the paper's clause notation, and decides
satisfiability with a small DPLL search (a filter on inputs, used because the
paper keeps only satisfiable instances below the threshold, Sec. III).

Clause encoding (shared by every interface of the library): a literal is the
int32 ``2*var + neg``, ``var`` in [0, n), ``neg`` = 1 for a negated variable.
A clause is three literals over three distinct variables (App. B, Eq. (B2)
with k_i = 3).

Instance recipe (Sec. III and App. C, "Optimization"):
  * the three variables of a clause are distinct and drawn uniformly, each
    literal negated with probability 1/2;
  * m = floor(n*d + 1/2) clauses for density d ("appropriate rounding");
  * a duplicate clause (same set of (var, neg) pairs in any order) is
    redrawn, so m is exact; ``dup="drop"`` keeps the paper's behaviour of
    retaining one copy, which can leave fewer than m clauses;
  * satisfiable instances only are kept where the paper does (d in (2, 4.5)).
"""
from __future__ import annotations

import re
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Instance", "m_from_density", "random_3sat", "dpll_satisfiable",
    "first_satisfiable", "sat_stream", "uniform_angles", "parse_paper_clauses",
    "PAPER_4VAR", "PAPER_5VAR", "batched_scan_instances", "two_level_instance",
]


@dataclass(frozen=True)
class Instance:
    n: int
    lits: np.ndarray        # int32 [m, 3], lit = 2*var + neg
    seed: int = -1          # generator seed (or spawn key index)
    draw: int = -1          # index of this draw in the seeded stream
    d: float = float("nan")

    @property
    def m(self) -> int:
        return int(self.lits.shape[0])


def m_from_density(n: int, d: float) -> int:
    """Clause count for density d = m/n, rounded half up (App. C)."""
    return int(np.floor(n * d + 0.5))


def _canon(clause) -> tuple:
    return tuple(sorted(int(x) for x in clause))


def random_3sat(rng: np.random.Generator, n: int, m: int, dup: str = "redraw") -> np.ndarray:
    """Draw m random 3-literal clauses over n >= 3 variables."""
    if n < 3:
        raise ValueError("a 3-SAT clause needs n >= 3 variables")
    if dup not in ("redraw", "drop"):
        raise ValueError("dup must be 'redraw' or 'drop'")
    distinct = 8 * (n * (n - 1) * (n - 2) // 6)   # 3-variable sets times sign patterns
    if dup == "redraw" and m > distinct:
        raise ValueError(f"only {distinct} distinct 3-literal clauses exist over {n} variables, asked for {m}")
    seen: set = set()
    out = []
    while len(out) < m:
        var = rng.choice(n, size=3, replace=False)
        neg = rng.integers(0, 2, size=3)
        clause = 2 * var + neg
        key = _canon(clause)
        if key in seen:
            if dup == "drop":
                m -= 1
            continue
        seen.add(key)
        out.append(clause)
    return np.asarray(out, dtype=np.int32).reshape(-1, 3)


def dpll_satisfiable(n: int, lits: np.ndarray) -> bool:
    """Decide satisfiability by DPLL with unit propagation.

    A literal (var, neg) is true under assignment a iff a[var] != neg
    (App. B: x is satisfied by tau(x) = 1, its negation by tau(x) = 0).
    """
    clauses = [tuple(int(x) for x in c) for c in np.asarray(lits).reshape(-1, 3)]
    occ = [[] for _ in range(2 * n)]       # clauses containing each literal
    for ci, c in enumerate(clauses):
        for lit in c:
            occ[lit].append(ci)
    assign = [-1] * n

    def lit_val(lit):
        a = assign[lit >> 1]
        return -1 if a < 0 else int(a != (lit & 1))

    def propagate(trail):
        i = 0
        while i < len(trail):
            var = trail[i]
            i += 1
            # literal that just became false: var with neg == assign[var]
            false_lit = 2 * var + assign[var]
            for ci in occ[false_lit]:
                unassigned = None
                nun = 0
                sat = False
                for lit in clauses[ci]:
                    v = lit_val(lit)
                    if v == 1:
                        sat = True
                        break
                    if v < 0:
                        nun += 1
                        unassigned = lit
                if sat:
                    continue
                if nun == 0:
                    return False
                if nun == 1:
                    u = unassigned >> 1
                    assign[u] = 1 - (unassigned & 1)
                    trail.append(u)
        return True

    def choose():
        best, score = -1, -1
        for v in range(n):
            if assign[v] < 0:
                s = len(occ[2 * v]) + len(occ[2 * v + 1])
                if s > score:
                    best, score = v, s
        return best

    def solve(trail_start):
        v = choose()
        if v < 0:
            return True
        for val in (1, 0):
            assign[v] = val
            trail = [v]
            if propagate(trail) and solve(None):
                return True
            for u in trail:
                assign[u] = -1
        return False

    # initial unit clauses cannot exist (all clauses have 3 literals)
    return solve(None)


def sat_stream(seed: int, n: int, m: int, dup: str = "redraw"):
    """Yield (draw_index, lits) from the seeded stream PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = 0
    while True:
        yield k, random_3sat(rng, n, m, dup)
        k += 1


def first_satisfiable(seed: int, n: int, m: int, accept=None, max_draws: int = 10000) -> Instance:
    """First draw of the seeded stream that ``accept(n, lits)`` accepts.

    ``accept`` defaults to the DPLL satisfiability check.
    """
    accept = accept or dpll_satisfiable
    for k, lits in sat_stream(seed, n, m):
        if accept(n, lits):
            return Instance(n=n, lits=lits, seed=seed, draw=k, d=m / n)
        if k + 1 >= max_draws:
            break
    raise RuntimeError(f"no accepted draw in {max_draws} for seed={seed} n={n} m={m}")


def draw_at(seed: int, n: int, m: int, draw: int) -> Instance:
    """Re-create draw number ``draw`` of the seeded stream."""
    for k, lits in sat_stream(seed, n, m):
        if k == draw:
            return Instance(n=n, lits=lits, seed=seed, draw=k, d=m / n)


def uniform_angles(seed: int, p: int, lo: float = 0.0, hi: float = np.pi):
    """Independent per-round angles beta_j, gamma_j ~ U[lo, hi] (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    beta = rng.uniform(lo, hi, size=p)
    gamma = rng.uniform(lo, hi, size=p)
    return beta, gamma


def _draw_density(rng, densities, density_range):
    if density_range is not None:
        return float(rng.uniform(density_range[0], density_range[1]))
    return float(densities[int(rng.integers(0, len(densities)))])


def _keep(n, lits, want):
    if want == "any":
        return True
    sat = dpll_satisfiable(n, lits)
    return sat if want == "sat" else not sat


def _child_instance(args):
    seed, count, k, n_lo, n_hi, densities, want, density_range, dup = args
    # child k of SeedSequence(seed).spawn(count), built directly
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(k,))))
    n = int(rng.integers(n_lo, n_hi + 1))
    d = _draw_density(rng, densities, density_range)
    m = m_from_density(n, d)
    draw = 0
    while True:
        lits = random_3sat(rng, n, m, dup=dup)
        if _keep(n, lits, want):
            break
        draw += 1
    return Instance(n=n, lits=lits, seed=k, draw=draw, d=d)


def batched_scan_instances(seed: int, count: int, n_lo: int, n_hi: int,
                           densities=(3.0, 4.2, 5.0), sat_only: bool = True,
                           accept=None, workers: int = 1, want: str | None = None,
                           density_range=None, dup: str = "redraw") -> list:
    """``count`` instances; child k draws from SeedSequence(seed) child k.

    Each child draws n ~ U{n_lo..n_hi}, d ~ U(densities) (or d ~ U(lo, hi)
    with ``density_range=(lo, hi)``, the paper's recipe), m = round(n d), then
    clause sets until one is kept: ``want`` = "sat" (the default when
    ``sat_only``), "unsat" (the Max-SAT set above the threshold) or "any".
    ``dup`` as in ``random_3sat``. ``workers`` > 1 splits the children over
    processes (same instances for any value).
    """
    want = want or ("sat" if sat_only else "any")
    if want not in ("sat", "unsat", "any"):
        raise ValueError("want must be 'sat', 'unsat' or 'any'")
    if accept is not None:
        out = []
        for k, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
            rng = np.random.Generator(np.random.PCG64(child))
            n = int(rng.integers(n_lo, n_hi + 1))
            d = _draw_density(rng, densities, density_range)
            m = m_from_density(n, d)
            draw = 0
            while True:
                lits = random_3sat(rng, n, m, dup=dup)
                if want == "any" or accept(n, lits):
                    break
                draw += 1
            out.append(Instance(n=n, lits=lits, seed=k, draw=draw, d=d))
        return out
    args = [(seed, count, k, n_lo, n_hi, tuple(densities), want, density_range, dup) for k in range(count)]
    if workers <= 1:
        return [_child_instance(a) for a in args]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_child_instance, args, chunksize=max(1, count // (8 * workers)))


# --- the paper's two worked instances (footnote of Sec. IV) -----------------

_LIT_RE = re.compile(r"([+-]?)\s*(\d+)")


def parse_paper_clauses(text: str) -> np.ndarray:
    """Parse the paper's notation '[-0, +2, +3], ...' into int32 [m, 3].

    A minus sign negates the variable; a missing sign reads as '+' (the
    5-variable example prints one literal without a sign).
    """
    clauses = []
    for group in re.findall(r"\[([^\]]*)\]", text):
        lits = []
        for sign, var in _LIT_RE.findall(group):
            lits.append(2 * int(var) + (1 if sign == "-" else 0))
        if len(lits) != 3:
            raise ValueError(f"clause {group!r} does not have three literals")
        clauses.append(lits)
    return np.asarray(clauses, dtype=np.int32)


PAPER_4VAR = ("[-0, +2, +3], [+0, +2, -3], [-1, +2, -3], [-1, -2, -3], "
              "[-1, -2, +3], [+1, +2, -3], [+0, +2, +3], [-0, +1, -3]")
PAPER_5VAR = ("[+1, -2, -3], [-1, -3, +4], [+0, -2, -4], [-0, -2, +3], "
              "[+2, +3, +4], [-0, +1, +2], [+0, -2, 4], [-1, +2, -4]")


def two_level_instance(n: int, keep_pattern: int = 0) -> np.ndarray:
    """The 7 clauses over variables {0,1,2} that forbid every bit pattern of
    (x0, x1, x2) except ``keep_pattern``: the cost takes only the values 0
    (on 2^(n-3) assignments) and 1, a two-valued cost for any n >= 3."""
    out = []
    for pat in range(8):
        if pat == keep_pattern:
            continue
        # the clause that is false exactly on pattern `pat`: literal on var v
        # is false iff bit_v == neg, so neg = bit v of pat
        out.append([2 * v + ((pat >> v) & 1) for v in range(3)])
    return np.asarray(out, dtype=np.int32)
