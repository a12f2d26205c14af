"""Rounds-to-target search and Max-SAT targets (Sec. III.A, App. B).

The paper counts the G-QAOA rounds p needed for the final state to hold at
least S (50%; 25% and 75% in the angle-optimization appendix) of its
probability on the target level, and finds p ~ 1/sqrt(P) against the 1/P of
random guessing:
  * satisfiable instances (d in (2, 4.5)): target level 0, P = N_0 / 2^n;
  * unsatisfiable instances (d in (4.6, 8)), the Max-SAT problem: target
    level k_min (the lowest occupied one), probability D = N_{k_min} / 2^n.

Single angle pair: the least p for which some (beta, gamma) reaches S is the
minimum over a grid of the first round at which each pair crosses S
(``gqaoa_scan_crossing``, one launch for all instances and pairs), refined
by windows of finer pairs around the best ones (per-instance grids, bounded
by the best p so far). Full G-QAOA (angles per round): the least p at
which all 2p angles, optimized with the level-space adjoint gradient from the
best single pair at that p, reach S, by bisection below the single-pair count
(many instances in lockstep).
"""
from __future__ import annotations

import math

import numpy as np

from . import gqaoa as g
from . import optim


def maxsat_targets(ns, hists):
    """(k_min[I], D[I]) from host histograms [I, stride]."""
    hists = np.asarray(hists)
    occupied = hists > 0
    k = occupied.argmax(axis=1)
    D = hists[np.arange(len(k)), k].astype(np.float64) / np.exp2(np.asarray(ns, dtype=np.float64))
    return k.astype(np.int32), D


def _min_first(first):
    """Per instance: (least nonzero first-crossing round or 0, its flat grid
    index, ties to the lowest)."""
    jd, vd = g.gqaoa_row_best(first.reshape(first.shape[0], -1), g.ROW_MIN_POSITIVE_I32)
    return vd.cpu().numpy().astype(np.int64), jd.cpu().numpy()


def single_pair_rounds(ns, ms, hists, S: float, p_max, targets=None, grid=None, zoom: int = 16,
                       zoom_levels: int = 2, max_out_bytes: float = 1e9, tile=None):
    """Least single-pair rounds reaching S for every instance.

    p_max: one cap, or one per instance. Returns (p_star[I] (0: not reached
    within the cap), beta[I], gamma[I]).
    Grid stage over the fundamental domain (default: the paper's pi/180
    spacing), then ``zoom_levels`` windows of zoom x zoom pairs around each
    instance's best pair, each half as wide as the last grid step allows."""
    hists = np.asarray(hists)
    ns = np.asarray(ns)
    ms = np.asarray(ms)
    I = hists.shape[0]
    tg = None if targets is None else np.asarray(targets, dtype=np.int32)
    caps = np.broadcast_to(np.asarray(p_max, dtype=np.int32), (I,)).copy()
    gb, gg = optim.fundamental_grid(*(grid or optim.paper_grid()))
    chunk = max(1, int(max_out_bytes // (4 * gb.size * gg.size)))
    p_star = np.zeros(I, dtype=np.int64)
    beta = np.zeros(I)
    gamma = np.zeros(I)
    for c0 in range(0, I, chunk):
        sl = slice(c0, min(I, c0 + chunk))
        first = g.gqaoa_scan_crossing(ns[sl], ms[sl], hists[sl], gb, gg, caps[sl], S,
                                      targets=None if tg is None else tg[sl], tile=tile)
        v, idx = _min_first(first)
        p_star[sl] = v
        beta[sl] = gb[idx % gb.size]
        gamma[sl] = gg[idx // gb.size]
        del first
    db, dg = gb[1] - gb[0], gg[1] - gg[0]
    offs = (np.arange(zoom) - (zoom - 1) / 2.0) * (2.0 / zoom)
    for _ in range(zoom_levels):
        live = np.nonzero(p_star > 0)[0]
        if live.size == 0:
            break
        bgrid = beta[live, None] + offs[None, :] * db
        ggrid = np.clip(gamma[live, None] + offs[None, :] * dg, 0.0, math.pi)
        first = g.gqaoa_scan_crossing(ns[live], ms[live], hists[live], bgrid, ggrid, p_star[live], S,
                                      targets=None if tg is None else tg[live], tile=tile)
        v, idx = _min_first(first)
        better = (v > 0) & (v < p_star[live])
        sel = live[better]
        p_star[sel] = v[better]
        beta[sel] = bgrid[better, idx[better] % zoom]
        gamma[sel] = ggrid[better, idx[better] // zoom]
        db, dg = db * 2.0 / zoom, dg * 2.0 / zoom
    return p_star, np.mod(beta, 2 * math.pi), gamma


def _best_pairs_at(ns, ms, hists, tg, p, gb, gg):
    """Best single pair of the grid at each instance's own round count p[i]
    (one scan per distinct p). Returns (beta[I], gamma[I])."""
    I = len(p)
    beta = np.zeros(I)
    gamma = np.zeros(I)
    for pv in np.unique(p):
        sel = np.nonzero(p == pv)[0]
        ps, _ = g.gqaoa_scan_batched(ns[sel], ms[sel], hists[sel], gb, gg, [int(pv)], targets=tg[sel],
                                     with_energy=False)
        j = _argbest(ps.reshape(sel.size, -1))
        beta[sel] = gb[j % gb.size]
        gamma[sel] = gg[j // gb.size]
    return beta, gamma


def _argbest(v):
    """Per row: index of the largest entry, ties to the lowest index."""
    return g.gqaoa_row_best(v, g.ROW_ARGMAX_F32, with_value=False)[0].cpu().numpy()


def full_rounds_batched(ns, ms, hists, S: float, p_single, targets=None, grid=(120, 61), p_floor: int = 1,
                        progress=None, on_batch=None):
    """Least full-G-QAOA rounds reaching S for every instance.

    For a candidate p the seed is the best single pair of a (beta, gamma) grid
    at that p, then all 2p angles are optimized (``optim.full_gqaoa_batched``,
    all candidates of one step in lockstep). The best P over all 2p angles
    cannot fall when p grows (a round with beta = gamma = 0 is the identity),
    so the least p with P >= S is found by bisection on [p_floor, p_single],
    p_single (the single-pair rounds, reached by one pair) being the upper
    end. Instances with p_single = 0 (not reached) are skipped.
    Returns (p_full[I] (0 where skipped), betas [I, p_max], gammas [I, p_max],
    psol[I], optimized[I]) at p_full; optimized[i] is False where no p below
    p_single reached S (then the angles are zero and psol NaN).
    progress(step, candidates, reached) is called after every bisection step,
    on_batch(k, waiting) after every batched gradient of the optimizations."""
    hists = np.asarray(hists)
    ns = np.asarray(ns, dtype=np.int32)
    ms = np.asarray(ms, dtype=np.int32)
    I = hists.shape[0]
    tg = np.zeros(I, dtype=np.int32) if targets is None else np.asarray(targets, dtype=np.int32)
    hi = np.asarray(p_single, dtype=np.int64).copy()
    lo = np.minimum(np.full(I, p_floor, dtype=np.int64), hi)
    pmax = int(max(1, hi.max()))
    betas = np.zeros((I, pmax))
    gammas = np.zeros((I, pmax))
    psol = np.full(I, np.nan)
    opt = np.zeros(I, dtype=bool)
    gb, gg = optim.fundamental_grid(*grid)
    step = 0
    while True:
        act = np.nonzero((hi > 0) & (lo < hi))[0]
        if act.size == 0:
            break
        step += 1
        mid = (lo[act] + hi[act]) // 2
        b0, g0 = _best_pairs_at(ns[act], ms[act], hists[act], tg[act], mid, gb, gg)
        bs, gs, P = optim.full_gqaoa_batched(ns[act], ms[act], hists[act], mid, b0, g0, tg[act], on_batch=on_batch)
        ok = P >= S
        for k, i in enumerate(act):
            if ok[k]:
                hi[i] = mid[k]
                betas[i] = 0.0
                gammas[i] = 0.0
                betas[i, :mid[k]] = bs[k, :mid[k]]
                gammas[i, :mid[k]] = gs[k, :mid[k]]
                psol[i] = P[k]
                opt[i] = True
            else:
                lo[i] = mid[k] + 1
        if progress is not None:
            progress(step, int(act.size), int(ok.sum()))
    return hi, betas, gammas, psol, opt


def full_rounds(n: int, m: int, hist, S: float, p_single: int, target: int = 0, grid=(120, 61), p_floor: int = 1):
    """``full_rounds_batched`` for one instance: (p_full, betas, gammas, psol)
    at the least p reached, with None angles and psol when no p below
    p_single reaches S."""
    pf, bs, gs, P, ok = full_rounds_batched([n], [m], np.asarray(hist).reshape(1, -1), S, [p_single], [target],
                                            grid, p_floor)
    if not ok[0]:
        return int(pf[0]), None, None, None
    return int(pf[0]), bs[0, :pf[0]].copy(), gs[0, :pf[0]].copy(), float(P[0])


def sqrt_fit(P, p):
    """Least-squares log p = a + b log(1/P) and the median of p sqrt(P):
    (b, a, c) with c the constant of p ~ c / sqrt(P)."""
    P = np.asarray(P, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    b, a = np.polyfit(np.log(1.0 / P), np.log(p), 1)
    return float(b), float(a), float(np.median(p * np.sqrt(P)))
