"""Angle optimization with device evaluations (App. C, "Optimization").

The paper evaluates its objective on a uniform (beta, gamma) grid (spacing
pi/180 for n <= 20, sampled pairs beyond), then refines with scipy's L-BFGS-B
to a 1e-6 relative change; full G-QAOA relaxes all 2p angles from the same
seed. Here every evaluation runs on the GPU:

* ``plain_single_pair``: the plain per-instance optimizer - one device call
  per angle pair (``gqaoa_hist_evolve``), grid then L-BFGS-B. This is the
  comparator for the batched and learned forms.
* ``plain_batched_grid``: the plain optimizer's steps for several instances
  with the grid stage as one batched scan (the learned form's fallback).
* ``batched_single_pair``: all instances at once - the fundamental-domain grid
  through one ``gqaoa_scan_batched`` call, then two rounds of per-instance
  zoomed grids around each best point (per p, one graph-captured scan plan
  replayed at each zoom level).
* ``full_gqaoa_batched`` / ``full_gqaoa``: all 2p angles by L-BFGS-B with the
  level-space adjoint gradient (``gqaoa_hist_grad_batched``), many instances
  in lockstep; ``full_gqaoa_statevector`` does the same with the statevector
  adjoint (``gqaoa_grad``).

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


def plain_batched_grid(ns, ms, hists, hists_dev, p: int, betas_grid, gammas_grid, objective: str = "psol",
                       targets=None, max_out_bytes: float = 2e9):
    """The plain optimizer's steps (``plain_single_pair``: the grid, then
    L-BFGS-B from its best point) for several instances, with the grid stage
    evaluated for all of them at once: one batched scan (the best cell per
    instance, ties to the lowest (gamma, beta) index), then per instance the
    grid point's value and L-BFGS-B with one float64 device call per
    evaluation, as in ``plain_single_pair``. ``hists_dev[i, :ms[i] + 1]`` is
    instance i's histogram on the device. Returns beta[I], gamma[I], psol[I]."""
    hists = np.asarray(hists)
    ns = np.asarray(ns)
    ms = np.asarray(ms)
    I = hists.shape[0]
    gb, gg = np.asarray(betas_grid, dtype=np.float64), np.asarray(gammas_grid, dtype=np.float64)
    tg = np.zeros(I, dtype=np.int32) if targets is None else np.asarray(targets, dtype=np.int32)
    want_e = objective != "psol"
    mode = g.ROW_ARGMIN_F32 if want_e else g.ROW_ARGMAX_F32
    chunk = max(1, int(max_out_bytes // (gb.size * gg.size * 4 * (2 if want_e else 1))))
    x0 = np.empty((I, 2))
    for c0 in range(0, I, chunk):
        sl = slice(c0, min(I, c0 + chunk))
        psol, energy = g.gqaoa_scan_batched(ns[sl], ms[sl], hists[sl], gb, gg, [p], targets=tg[sl],
                                            with_energy=want_e)
        jd, _ = g.gqaoa_row_best((energy if want_e else psol).reshape(sl.stop - sl.start, -1), mode)
        j = jd.cpu().numpy()
        x0[sl, 0] = gb[j % gb.size]
        x0[sl, 1] = gg[j // gb.size]
        del psol, energy
    beta, gamma, ps_out = np.empty(I), np.empty(I), np.empty(I)
    for i in range(I):
        hdev = hists_dev[i, :int(ms[i]) + 1].contiguous()
        n, m, t = int(ns[i]), int(ms[i]), int(tg[i])

        def f(x):
            ps, en, _ = g.gqaoa_hist_evolve(n, m, hdev, np.full(p, x[0]), np.full(p, x[1]), t)
            return _value(ps[-1], en[-1], objective)

        x, best = x0[i], f(x0[i])
        res = minimize(f, x0[i], method="L-BFGS-B", options={"ftol": 1e-6})
        if res.fun < best:
            x = res.x
        ps, _, _ = g.gqaoa_hist_evolve(n, m, hdev, np.full(p, x[0]), np.full(p, x[1]), t)
        beta[i], gamma[i], ps_out[i] = x[0], x[1], ps[-1]
    return beta, gamma, ps_out


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
    mode = g.ROW_ARGMIN_F32 if want_e else g.ROW_ARGMAX_F32
    per_inst = P * gb.size * gg.size * 4 * (2 if want_e else 1)
    chunk = max(1, int(max_out_bytes // per_inst))
    beta = np.empty((I, P))
    gamma = np.empty((I, P))
    best_v = np.empty((I, P))
    for c0 in range(0, I, chunk):
        sl = slice(c0, min(I, c0 + chunk))
        psol, energy = g.gqaoa_scan_batched(ns[sl], ms[sl], hists[sl], gb, gg, p_list,
                                            targets=None if tg is None else tg[sl], tile=tile, with_energy=want_e)
        rows = (sl.stop - sl.start) * P
        # best cell per (instance, p), ties -> lowest (gamma, beta) index
        jd, vd = g.gqaoa_row_best((psol if objective == "psol" else energy).reshape(rows, -1), mode)
        idx = jd.cpu().numpy().reshape(-1, P)
        v = vd.cpu().numpy().reshape(-1, P).astype(np.float64)
        best_v[sl] = -v if objective == "psol" else v
        beta[sl] = gb[idx % gb.size]
        gamma[sl] = gg[idx // gb.size]
        del psol, energy
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
            jd, vd = g.gqaoa_row_best((en if want_e else ps).reshape(I, -1), mode)
            j = jd.cpu().numpy()
            vj = vd.cpu().numpy().astype(np.float64)
            vj = vj if want_e else -vj
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


def lockstep_lbfgsb(evaluate, x0s, ftol: float = 1e-6, max_workers: int = 512, on_batch=None):
    """scipy L-BFGS-B from every start point of ``x0s``, run in lockstep.

    Each optimization runs in its own host thread and asks for its objective
    through ``evaluate(idx, xs) -> (F, G)``, which the calling thread serves
    for all waiting optimizations at once (idx: their positions in x0s, xs
    their points; F[k] the value and G[k] the gradient at xs[k]). Every
    optimization takes the same steps as a scipy call of its own, as long as
    evaluate's result for one point does not depend on the others in the
    batch. At most ``max_workers`` optimizations run at a time; on_batch(k,
    waiting), when given, is called after the k-th batched evaluation. Returns
    the scipy results in the order of x0s."""
    import threading

    x0s = [np.asarray(x, dtype=np.float64) for x in x0s]
    results = [None] * len(x0s)
    for c0 in range(0, len(x0s), max_workers):
        idx = list(range(c0, min(len(x0s), c0 + max_workers)))
        W = len(idx)
        cv = threading.Condition()
        req = [None] * W            # point a worker waits on
        ans = [None] * W
        ready = [threading.Event() for _ in range(W)]
        state = {"posted": 0, "done": 0, "error": None}

        def worker(w):
            def fun(x):
                with cv:
                    req[w] = np.array(x, dtype=np.float64)
                    state["posted"] += 1
                    cv.notify()
                ready[w].wait()
                ready[w].clear()
                if state["error"] is not None:
                    raise RuntimeError("batched evaluation failed")
                return ans[w]
            try:
                results[idx[w]] = minimize(fun, x0s[idx[w]], jac=True, method="L-BFGS-B", options={"ftol": ftol})
            except Exception:
                pass
            finally:
                with cv:
                    state["done"] += 1
                    cv.notify()

        threads = [threading.Thread(target=worker, args=(w,), daemon=True) for w in range(W)]
        for t in threads:
            t.start()
        nbatch = 0
        while True:
            with cv:
                cv.wait_for(lambda: state["posted"] + state["done"] >= W)
                waiting = [w for w in range(W) if req[w] is not None]
                if not waiting:
                    break
                xs = [req[w] for w in waiting]
                for w in waiting:
                    req[w] = None
                state["posted"] -= len(waiting)
            try:
                F, G = evaluate([idx[w] for w in waiting], xs)
            except Exception as e:
                state["error"] = e
                for w in waiting:
                    ready[w].set()
                for t in threads:
                    t.join()
                raise
            for k, w in enumerate(waiting):
                ans[w] = (float(F[k]), np.asarray(G[k], dtype=np.float64))
                ready[w].set()
            nbatch += 1
            if on_batch is not None:
                on_batch(nbatch, len(waiting))
        for t in threads:
            t.join()
    return results


def full_gqaoa_batched(ns, ms, hists, p, beta0, gamma0, targets=None, on_batch=None):
    """Full G-QAOA (App. C, "Optimization"): all 2 p_i angles of every instance
    by L-BFGS-B (maximizing P_sol, ftol 1e-6) from its single pair (beta0_i,
    gamma0_i) broadcast to every round, with the level-space adjoint gradient
    (``gqaoa_hist_grad_batched``); the instances' optimizations run in
    lockstep, one batched gradient call per step. p: one round count or one
    per instance. Returns (betas [I, p_max], gammas [I, p_max], psol [I]),
    entries past p_i zero."""
    hists = np.asarray(hists)
    ns = np.asarray(ns, dtype=np.int32)
    ms = np.asarray(ms, dtype=np.int32)
    I = hists.shape[0]
    p = np.broadcast_to(np.asarray(p, dtype=np.int32), (I,)).copy()
    tg = np.zeros(I, dtype=np.int32) if targets is None else np.asarray(targets, dtype=np.int32)
    beta0 = np.broadcast_to(np.asarray(beta0, dtype=np.float64), (I,))
    gamma0 = np.broadcast_to(np.asarray(gamma0, dtype=np.float64), (I,))
    pmax = int(p.max())
    x0s = [np.concatenate([np.full(p[i], beta0[i]), np.full(p[i], gamma0[i])]) for i in range(I)]

    def evaluate(idx, xs):
        idx = np.asarray(idx)
        B = np.zeros((idx.size, pmax))
        G = np.zeros((idx.size, pmax))
        for k, i in enumerate(idx):
            B[k, :p[i]] = xs[k][:p[i]]
            G[k, :p[i]] = xs[k][p[i]:]
        P, db, dg = g.gqaoa_hist_grad_batched(ns[idx], ms[idx], hists[idx], B, G, targets=tg[idx], p=p[idx])
        grads = [-np.concatenate([db[k, :p[i]], dg[k, :p[i]]]) for k, i in enumerate(idx)]
        return -P, grads

    res = lockstep_lbfgsb(evaluate, x0s, on_batch=on_batch)
    betas = np.zeros((I, pmax))
    gammas = np.zeros((I, pmax))
    psol = np.zeros(I)
    for i, r in enumerate(res):
        if r is None:
            raise RuntimeError(f"the optimization of instance {i} failed")
        betas[i, :p[i]] = r.x[:p[i]]
        gammas[i, :p[i]] = r.x[p[i]:]
        psol[i] = -r.fun
    return betas, gammas, psol


def full_gqaoa(n: int, m: int, hist, p: int, beta0: float, gamma0: float, target: int = 0):
    """``full_gqaoa_batched`` for one instance: (betas[p], gammas[p], psol)."""
    b, gm, P = full_gqaoa_batched([n], [m], np.asarray(hist).reshape(1, -1), [p], [beta0], [gamma0], [target])
    return b[0], gm[0], float(P[0])


def full_gqaoa_statevector(n: int, m: int, cost, p: int, beta0: float, gamma0: float, target: int = 0,
                           dtype=g.C128, ckpt_every: int | None = None):
    """``full_gqaoa`` with the statevector adjoint (``gqaoa_grad``, O(2^n p) per
    gradient) instead of the level space; the same optimum from |s>, kept as
    its amplitude-level check. Returns (betas, gammas, psol)."""
    x0 = np.concatenate([np.full(p, beta0), np.full(p, gamma0)])

    def f(x):
        P, db, dgm = g.gqaoa_grad(n, m, cost, x[:p], x[p:], dtype, target, ckpt_every)
        return -P, -np.concatenate([db, dgm])

    res = minimize(f, x0, jac=True, method="L-BFGS-B", options={"ftol": 1e-6})
    return res.x[:p].copy(), res.x[p:].copy(), float(-res.fun)
