"""P_sol as a differentiable function of the G-QAOA angles.

``GQAOAProb.apply(betas, gammas, cost, n, m, ...)`` returns P_sol after
len(betas) rounds of Eq. (3) from |s> (float64 scalar tensor); its backward
returns dP/dbeta_k and dP/dgamma_k from the device adjoint sweep
(``gqaoa_grad``: reverse sweep with checkpoints every ``ckpt_every`` rounds;
None keeps every round's state when that fits in device memory and
checkpoints only when it does not).
The forward call computes the gradient too (one adjoint sweep) and keeps it
for the backward. ``GQAOAProbBatched`` does the same for a batch of
instances with equal n (betas, gammas: [I, p]; returns P_sol[I]).
The cost table is not differentiable.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gqaoa as g


class GQAOAProb(torch.autograd.Function):
    @staticmethod
    def forward(ctx, betas, gammas, cost, n: int, m: int, target_level: int = 0, dtype=g.C128,
                ckpt_every: int | None = None):
        b = betas.detach().cpu().double().numpy()
        gm = gammas.detach().cpu().double().numpy()
        P, db, dg = g.gqaoa_grad(n, m, cost, b, gm, dtype, target_level, ckpt_every)
        ctx.save_for_backward(torch.from_numpy(db).to(betas.device, betas.dtype),
                              torch.from_numpy(dg).to(gammas.device, gammas.dtype))
        return torch.tensor(P, dtype=torch.float64, device=betas.device)

    @staticmethod
    def backward(ctx, grad_out):
        db, dg = ctx.saved_tensors
        return grad_out * db, grad_out * dg, None, None, None, None, None, None


class GQAOAProbBatched(torch.autograd.Function):
    @staticmethod
    def forward(ctx, betas, gammas, costs, n: int, ms, targets=None, dtype=g.C128, ckpt_every: int | None = None):
        b = betas.detach().cpu().double().numpy()
        gm = gammas.detach().cpu().double().numpy()
        P, db, dg = g.gqaoa_grad_batched(n, ms, costs, b, gm, dtype, targets, ckpt_every)
        ctx.save_for_backward(torch.from_numpy(db).to(betas.device, betas.dtype),
                              torch.from_numpy(dg).to(gammas.device, gammas.dtype))
        return torch.from_numpy(np.asarray(P)).to(betas.device)

    @staticmethod
    def backward(ctx, grad_out):
        db, dg = ctx.saved_tensors
        go = grad_out.to(db.dtype)[:, None]
        return go * db, go * dg, None, None, None, None, None, None
