"""Learned single-angle-pair G-QAOA angles.

The paper observes that optimized single-pair angles cluster, more tightly as
the clause count grows (Sec. III.B), and suggests determining angles from
statistics of the density of states (Sec. V). ``AngleMLP`` maps an
instance's normalized level histogram and (n, d = m/n, p) to one (beta,
gamma) pair with the device MLP (bfloat16 MFMA forward/backward, float32
Adam); labels come from ``optim.batched_single_pair``. All arithmetic runs in
libgqaoa kernels; this module only orders the calls.

Reference points for judging the network:
  * ``cluster_median``: one fixed pair per p (the median of the training
    labels), i.e. what parameter clustering alone gives;
  * the plain and batched optimizers of ``optim``.

``solve`` is the learned form end to end for one round count: the network's
pair, local window scans around it, and the plain per-instance optimizer for
every instance whose result stays below 0.99 of the cluster-median pair.
The labels come from the batched optimizer, which runs the plain optimizer's
grid and refines by zoomed grid windows instead of L-BFGS-B: labelling the
20,000 x 4 training instance-p pairs with the plain optimizer (one device
call per evaluation, seconds per pair) would take days.
"""
from __future__ import annotations

import math

import numpy as np

from . import gqaoa as g
from . import optim


def _torch():
    import torch
    return torch


class AngleMLP:
    def __init__(self, seed: int = 0):
        torch = _torch()
        rng = np.random.Generator(np.random.PCG64(seed))
        flat = np.zeros(g.MLP_NPARAMS, dtype=np.float32)
        for key, fan_in in (("W1", 131), ("W2", 256), ("W3", 256)):
            off, shape = g.MLP_OFFSETS[key]
            bound = 1.0 / math.sqrt(fan_in)
            w = np.zeros(shape, dtype=np.float32)
            w[:fan_in] = rng.uniform(-bound, bound, size=(fan_in, shape[1]))
            flat[off:off + w.size] = w.ravel()
        self.params = torch.tensor(flat, device="cuda")
        self.state = torch.zeros(2 * g.MLP_NPARAMS, dtype=torch.float32, device="cuda")
        self.grads = torch.empty(g.MLP_NPARAMS, dtype=torch.float32, device="cuda")
        self.step = 0

    def save(self, path):
        """Checkpoint of the network and its optimizer: parameters, Adam
        moments and step count, as a plain .npz (no pickled objects)."""
        np.savez(path, params=self.params.cpu().numpy(), state=self.state.cpu().numpy(),
                 step=np.array([self.step], dtype=np.int64))

    @classmethod
    def load(cls, path):
        """A model restored from save(); training continues from the saved step."""
        torch = _torch()
        with np.load(path, allow_pickle=False) as f:
            params, state, step = f["params"], f["state"], int(f["step"][0])
        if params.shape != (g.MLP_NPARAMS,) or state.shape != (2 * g.MLP_NPARAMS,):
            raise ValueError(f"{path}: not an angle-network checkpoint")
        m = cls.__new__(cls)
        m.params = torch.tensor(params, dtype=torch.float32, device="cuda")
        m.state = torch.tensor(state, dtype=torch.float32, device="cuda")
        m.grads = torch.empty(g.MLP_NPARAMS, dtype=torch.float32, device="cuda")
        m.step = step
        return m

    def outputs(self, x):
        """Raw outputs [B, 2] by the inference kernels (no activation cache)."""
        return g.gqaoa_mlp_infer(self.params, x.contiguous())

    def angles(self, x):
        """(beta, gamma) numpy arrays: beta = 2 pi sigmoid(o0), gamma = pi sigmoid(o1)
        (the map runs on the device)."""
        beta, gamma = g.gqaoa_mlp_angles(self.outputs(x))
        return beta.cpu().numpy(), gamma.cpu().numpy()

    def train(self, X, Y, steps: int = 2000, batch: int = 512, lr: float = 1e-3, seed: int = 0, log_every: int = 0):
        """Adam on the angle-regression loss. X [N, 131], Y [N, 2] device tensors.
        Batches are drawn with replacement by a seeded host generator and
        gathered on the device."""
        torch = _torch()
        rng = np.random.Generator(np.random.PCG64(seed))
        N = X.shape[0]
        B = min(batch, N)
        xb = torch.empty((B, X.shape[1]), dtype=X.dtype, device="cuda")
        yb = torch.empty((B, Y.shape[1]), dtype=Y.dtype, device="cuda")
        losses = []
        for s in range(steps):
            idx = torch.from_numpy(rng.integers(0, N, B).astype(np.int32)).to("cuda")
            g.gqaoa_gather_rows(X, idx, out=xb)
            g.gqaoa_gather_rows(Y, idx, out=yb)
            out, act = g.gqaoa_mlp_forward(self.params, xb)
            dout, loss = g.gqaoa_mlp_loss(out, yb)
            g.gqaoa_mlp_backward(self.params, act, dout, grads=self.grads)
            self.step += 1
            g.gqaoa_mlp_adam(self.params, self.grads, self.state, self.step, lr=lr)
            if log_every and (s % log_every == 0 or s == steps - 1):
                losses.append((s, float(loss.item())))
        return losses


def features_for(hists_dev, ns, ms, p: int):
    """Network inputs of every instance for round count p (device kernel)."""
    torch = _torch()
    I = hists_dev.shape[0]
    nd = torch.tensor(np.asarray(ns, dtype=np.int32), device="cuda")
    md = torch.tensor(np.asarray(ms, dtype=np.int32), device="cuda")
    pd = torch.tensor(np.full(I, p, dtype=np.int32), device="cuda")
    return g.gqaoa_mlp_features(hists_dev.contiguous(), nd, md, pd)


def training_set(insts, p_list, grid=None):
    """(X [I*P, 131], Y [I*P, 2], labels dict) from batched-optimizer labels."""
    torch = _torch()
    ns = [it.n for it in insts]
    ms = [it.m for it in insts]
    stride = max(max(ms) + 1, 2)
    hists_dev = g.gqaoa_hist_batched(ns, ms, [it.lits for it in insts], hist_stride=stride)
    hists = hists_dev.cpu().numpy()
    beta, gamma, psol, _ = optim.batched_single_pair(ns, ms, hists, p_list, grid=grid)
    X = torch.cat([features_for(hists_dev, ns, ms, p) for p in p_list], dim=0)
    Y = torch.tensor(np.concatenate([np.stack([beta[:, q], gamma[:, q]], 1) for q in range(len(p_list))]),
                     dtype=torch.float32, device="cuda")
    return X, Y, {"beta": beta, "gamma": gamma, "psol": psol, "hists": hists, "hists_dev": hists_dev,
                  "ns": ns, "ms": ms}


def cluster_median(labels, p_list):
    """One (beta, gamma) per p: the median of the optimized training pairs."""
    return {p: (float(np.median(labels["beta"][:, q])), float(np.median(labels["gamma"][:, q])))
            for q, p in enumerate(p_list)}


def evaluate_pairs(ns, ms, hists, betas, gammas, p: int):
    """P_sol of every instance at its own (beta, gamma) after p rounds."""
    I = len(ns)
    b = np.asarray(betas, dtype=np.float64).reshape(I, 1)
    gm = np.asarray(gammas, dtype=np.float64).reshape(I, 1)
    ps, _ = g.gqaoa_scan_batched(ns, ms, hists, b, gm, [p], with_energy=False)
    return ps.reshape(I).cpu().numpy().astype(np.float64)


def solve(model, hists_dev, ns, ms, hists, p: int, median_pair, plain_grid=None, fallback_ratio: float = 0.99):
    """The learned form for round count p on every instance: the network's
    pair, refined by ``refine_local``; where the result stays below
    ``fallback_ratio`` times the P_sol of the fixed cluster-median pair, the
    plain optimizer's steps (``optim.plain_batched_grid`` over ``plain_grid``,
    default the paper's pi/180 grid: the grid, then L-BFGS-B from its best
    point) replace it, with the grid stage of all such instances in one
    batched scan.
    Returns dict(beta, gamma, psol, fallback (bool mask), psol_learned (the
    network's pair alone), psol_median)."""
    I = len(ns)
    x = features_for(hists_dev, ns, ms, p)
    bl, gl = model.angles(x)
    # the network's pair and the cluster-median pair in one scan: a 2 x 2 grid
    # per instance whose diagonal holds the two pairs (every cell is computed
    # on its own, so the values are those of two separate scans)
    b2 = np.stack([np.asarray(bl, dtype=np.float64), np.full(I, float(median_pair[0]))], axis=1)
    g2 = np.stack([np.asarray(gl, dtype=np.float64), np.full(I, float(median_pair[1]))], axis=1)
    ps2, _ = g.gqaoa_scan_batched(ns, ms, hists, b2, g2, [p], with_energy=False)
    ps2 = ps2.cpu().numpy().astype(np.float64)
    p_learn, p_med = ps2[:, 0, 0, 0], ps2[:, 0, 1, 1]
    b, gm, ps = refine_local(ns, ms, hists, bl, gl, p, start_psol=p_learn)
    fb = ps < fallback_ratio * p_med
    if fb.any():
        gb, gg = optim.fundamental_grid(*(plain_grid or optim.paper_grid()))
        ix = np.nonzero(fb)[0]
        b[ix], gm[ix], ps[ix] = optim.plain_batched_grid(np.asarray(ns)[ix], np.asarray(ms)[ix],
                                                         np.asarray(hists)[ix], hists_dev[ix], p, gb, gg)
    return {"beta": np.mod(b, 2 * math.pi), "gamma": gm, "psol": ps, "fallback": fb, "psol_learned": p_learn,
            "psol_median": p_med}


def refine_local(ns, ms, hists, betas, gammas, p: int, widths=(0.5, 0.25, 0.06, 0.015), zoom: int = 24,
                 start_psol=None):
    """Best pair after one zoom x zoom window scan per width, each centred on the
    previous best (one replay of a graph-captured scan per width, all
    instances). The peak narrows as p grows, hence shrinking windows; at
    p = 64 the network's pair can sit a few tenths of a radian in beta from
    the optimum, hence the first window's half-width of 0.5, and the peak is
    then narrow in both angles, hence 24 points a side: with 16 the first
    window's spacing steps over it on 18% of the instances (below 0.99 of
    the batched optimizer's P_sol), with 24 on 4%."""
    I = len(ns)
    b = np.asarray(betas, dtype=np.float64).copy()
    gm = np.asarray(gammas, dtype=np.float64).copy()
    # P_sol at the starting pairs (the caller's, when it has them already)
    best = (evaluate_pairs(ns, ms, hists, b, gm, p) if start_psol is None
            else np.asarray(start_psol, dtype=np.float64).copy())
    plan = None                      # one graph-captured scan, replayed per window
    for w in widths:
        offs = np.linspace(-w, w, zoom)
        bgrid = b[:, None] + offs[None, :]
        ggrid = np.clip(gm[:, None] + offs[None, :] / 2, 0.0, math.pi)
        if plan is None:
            plan = g.ScanPlan(ns, ms, hists, bgrid, ggrid, [p], with_energy=False)
            ps, _ = plan.run()
        else:
            ps, _ = plan.run(bgrid, ggrid)
        jd, vd = g.gqaoa_row_best(ps.reshape(I, -1), g.ROW_ARGMAX_F32)   # only the best cell leaves the GPU
        j = jd.cpu().numpy()
        vj = vd.cpu().numpy().astype(np.float64)
        better = vj > best
        b[better] = bgrid[better, j[better] % zoom]
        gm[better] = ggrid[better, j[better] // zoom]
        best[better] = vj[better]
    if plan is not None:
        plan.close()
    return b, gm, best
