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
by the best p so far). Full G-QAOA (angles per round): starting one round
below the single-pair count, all 2p angles are optimized with the adjoint
gradient from the best single pair at that p, stepping down while the
optimum still reaches S.
"""
from __future__ import annotations

import math

import numpy as np

from . import gqaoa as g
from . import optim


def _torch():
    import torch
    return torch


def maxsat_targets(ns, hists):
    """(k_min[I], D[I]) from host histograms [I, stride]."""
    hists = np.asarray(hists)
    occupied = hists > 0
    k = occupied.argmax(axis=1)
    D = hists[np.arange(len(k)), k].astype(np.float64) / np.exp2(np.asarray(ns, dtype=np.float64))
    return k.astype(np.int32), D


def _min_first(first, nb):
    """Per instance: (least nonzero first-crossing round or 0, flat argmin)."""
    torch = _torch()
    big = torch.iinfo(torch.int32).max
    f = first.reshape(first.shape[0], -1)
    f = torch.where(f > 0, f, torch.full_like(f, big))
    val, idx = f.min(dim=1)
    val = torch.where(val == big, torch.zeros_like(val), val)
    return val.cpu().numpy().astype(np.int64), idx.cpu().numpy()


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
        v, idx = _min_first(first, gb.size)
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
        v, idx = _min_first(first, zoom)
        better = (v > 0) & (v < p_star[live])
        sel = live[better]
        p_star[sel] = v[better]
        beta[sel] = bgrid[better, idx[better] % zoom]
        gamma[sel] = ggrid[better, idx[better] // zoom]
        db, dg = db * 2.0 / zoom, dg * 2.0 / zoom
    return p_star, np.mod(beta, 2 * math.pi), gamma


def full_rounds(n: int, m: int, cost, hist, S: float, p_single: int, target: int = 0, grid=(120, 61),
                dtype=g.C128, p_floor: int = 1):
    """Least full-G-QAOA rounds reaching S, searching down from p_single - 1.

    At each p the seed is the best single pair of a (beta, gamma) grid at
    that p (one batched-scan launch), then all 2p angles are optimized
    (``optim.full_gqaoa``). Returns (p_full, betas, gammas, psol) at the
    least p reached (p_single with None angles if no smaller p reaches S)."""
    hist = np.asarray(hist).reshape(1, -1)
    gb, gg = optim.fundamental_grid(*grid)
    best = (p_single, None, None, None)
    for p in range(p_single - 1, p_floor - 1, -1):
        ps, _ = g.gqaoa_scan_batched([n], [m], hist, gb, gg, [p], targets=[target], with_energy=False)
        j = int(ps.reshape(-1).argmax().item())
        b0, g0 = gb[j % gb.size], gg[j // gb.size]
        bs, gs, P = optim.full_gqaoa(n, m, cost, p, b0, g0, target=target, dtype=dtype)
        if P < S:
            break
        best = (p, bs, gs, P)
    return best


def sqrt_fit(P, p):
    """Least-squares log p = a + b log(1/P) and the median of p sqrt(P):
    (b, a, c) with c the constant of p ~ c / sqrt(P)."""
    P = np.asarray(P, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    b, a = np.polyfit(np.log(1.0 / P), np.log(p), 1)
    return float(b), float(a), float(np.median(p * np.sqrt(P)))
