"""Angle optimization with device evaluations (App. C, "Optimization").

The paper evaluates its objective on a uniform (beta, gamma) grid (spacing
pi/180 for n <= 20, sampled pairs beyond), then refines with scipy's L-BFGS-B
to a 1e-6 relative change; full G-QAOA relaxes all 2p angles from the same
seed. Here every evaluation runs on the GPU:

* ``plain_single_pair``: the plain per-instance optimizer - one device call
  per angle pair (``gqaoa_hist_evolve``), grid then L-BFGS-B. This is the
  comparator for the batched and learned forms.
* ``batched_single_pair``: all instances at once - the fundamental-domain grid
  through one ``gqaoa_scan_batched`` call, then two rounds of per-instance
  zoomed grids around each best point (per p, one graph-captured scan plan
  replayed at each zoom level).
* ``full_gqaoa``: all 2p angles by L-BFGS-B with the adjoint gradient
  (``gqaoa_grad``).

Objective: ``"psol"`` maximizes P_sol (the headline quantity of Sec. III);
``"energy"`` minimizes Eq. (4), the paper's stated cost function.
P is 2 pi-periodic in beta and gamma and invariant under
(beta, gamma) -> (-beta, -gamma), so beta in [0, 2 pi), gamma in [0, pi]
covers every distinct pair.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import minimize

from . import gqaoa as g


def fundamental_grid(nb: int = 128, ng: int = 64):
    """beta in [0, 2 pi) (nb points), gamma in [0, pi] (ng points)."""
    return np.linspace(0.0, 2 * math.pi, nb, endpoint=False), np.linspace(0.0, math.pi, ng)


def _value(psol, energy, objective):
    return -psol if objective == "psol" else energy


def plain_single_pair(n: int, m: int, hist_dev, p: int, betas_grid, gammas_grid, objective: str = "psol",
                      target: int = 0, refine: bool = True):
    """Grid (one device call per pair), then L-BFGS-B from the best point.

    Returns dict(beta, gamma, psol, energy, evals)."""
    evals = 0

    def f(x):
        nonlocal evals
        evals += 1
        ps, en, _ = g.gqaoa_hist_evolve(n, m, hist_dev, np.full(p, x[0]), np.full(p, x[1]), target)
        return _value(ps[-1], en[-1], objective)

    best, x0 = math.inf, None
    for b in betas_grid:
        for gm in gammas_grid:
            v = f((b, gm))
            if v < best:
                best, x0 = v, np.array([b, gm])
    x = x0
    if refine:
        res = minimize(f, x0, method="L-BFGS-B", options={"ftol": 1e-6})
        if res.fun < best:
            x, best = res.x, float(res.fun)
    ps, en, _ = g.gqaoa_hist_evolve(n, m, hist_dev, np.full(p, x[0]), np.full(p, x[1]), target)
    return {"beta": float(x[0]), "gamma": float(x[1]), "psol": float(ps[-1]), "energy": float(en[-1]),
            "evals": evals}


def paper_grid():
    """The paper's pi/180 spacing over the fundamental domain: 360 x 181 pairs."""
    return 360, 181


def batched_single_pair(ns, ms, hists, p_list, grid=None, zoom_levels: int = 2, zoom: int = 16,
                        objective: str = "psol", targets=None, tile=None, max_out_bytes: float = 2e9):
    """Single-pair optimum of every instance and p in ``p_list``.

    Grid stage over the fundamental domain (default: the paper's pi/180
    spacing), instances taken in chunks so the [chunk, P, ng, nb] output stays
    under ``max_out_bytes``; then ``zoom_levels`` rounds of a zoom x zoom
    window around each best pair (one launch per p and round, all instances).
    Returns arrays beta[I, P], gamma[I, P], psol[I, P], energy[I, P]."""
    hists = np.asarray(hists)
    ns = np.asarray(ns)
    ms = np.asarray(ms)
    I = hists.shape[0]
    P = len(p_list)
    gb, gg = fundamental_grid(*(grid or paper_grid()))
    tg = None if targets is None else np.asarray(targets)
    want_e = objective != "psol"
    per_inst = P * gb.size * gg.size * 4 * (2 if want_e else 1)
    chunk = max(1, int(max_out_bytes // per_inst))
    beta = np.empty((I, P))
    gamma = np.empty((I, P))
    best_v = np.empty((I, P))
    for c0 in range(0, I, chunk):
        sl = slice(c0, min(I, c0 + chunk))
        psol, energy = g.gqaoa_scan_batched(ns[sl], ms[sl], hists[sl], gb, gg, p_list,
                                            targets=None if tg is None else tg[sl], tile=tile, with_energy=want_e)
        val = -psol if objective == "psol" else energy
        flat = val.reshape(sl.stop - sl.start, P, -1)
        idx = flat.argmin(dim=2)                       # ties -> lowest (gamma, beta) index
        best_v[sl] = flat.gather(2, idx[:, :, None])[:, :, 0].cpu().numpy()
        idx = idx.cpu().numpy()
        beta[sl] = gb[idx % gb.size]
        gamma[sl] = gg[idx // gb.size]
        del psol, energy, val, flat
    db, dg = gb[1] - gb[0], gg[1] - gg[0]
    plans = {}                       # per p: a graph-captured scan replayed at every zoom level
    for _ in range(zoom_levels):
        offs = (np.arange(zoom) - (zoom - 1) / 2.0) * (2.0 / zoom)
        for q, p in enumerate(p_list):
            bgrid = beta[:, q:q + 1] + offs[None, :] * db
            ggrid = np.clip(gamma[:, q:q + 1] + offs[None, :] * dg, 0.0, math.pi)
            if p not in plans:
                plans[p] = g.ScanPlan(ns, ms, hists, bgrid, ggrid, [p], targets=targets, tile=tile,
                                      with_energy=want_e)
                ps, en = plans[p].run()
            else:
                ps, en = plans[p].run(bgrid, ggrid)
            v = (-ps if objective == "psol" else en)[:, 0].reshape(I, -1)
            j = v.argmin(dim=1).cpu().numpy()
            vj = v.cpu().numpy()[np.arange(I), j]
            better = vj < best_v[:, q]
            beta[better, q] = bgrid[better, j[better] % zoom]
            gamma[better, q] = ggrid[better, j[better] // zoom]
            best_v[better, q] = vj[better]
        db, dg = db * 2.0 / zoom, dg * 2.0 / zoom
    for pl in plans.values():
        pl.close()
    # final readout at the chosen pairs
    ps, en = g.gqaoa_scan_batched(ns, ms, hists, beta, gamma, p_list, targets=targets, tile=tile)
    ps = ps.cpu().numpy()
    en = en.cpu().numpy()
    out_p = np.stack([ps[:, q, q, q] for q in range(P)], axis=1).astype(np.float64)
    out_e = np.stack([en[:, q, q, q] for q in range(P)], axis=1).astype(np.float64)
    return np.mod(beta, 2 * math.pi), gamma, out_p, out_e


def full_gqaoa(n: int, m: int, cost, p: int, beta0: float, gamma0: float, target: int = 0, dtype=g.C128,
               ckpt_every: int | None = None):
    """All 2p angles by L-BFGS-B (maximizing P_sol) with the adjoint gradient,
    from the single-pair seed. Returns (betas, gammas, psol)."""
    x0 = np.concatenate([np.full(p, beta0), np.full(p, gamma0)])

    def f(x):
        P, db, dgm = g.gqaoa_grad(n, m, cost, x[:p], x[p:], dtype, target, ckpt_every)
        return -P, -np.concatenate([db, dgm])

    res = minimize(f, x0, jac=True, method="L-BFGS-B", options={"ftol": 1e-6})
    return res.x[:p].copy(), res.x[p:].copy(), float(-res.fun)
