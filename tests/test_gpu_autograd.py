"""GPU: P_sol as a torch.autograd.Function (autograd.GQAOAProb and
GQAOAProbBatched), the adjoint sweep behind .backward(), against the oracle's
reverse sweep (oracle.grad.grad_sv, statevector, complex128). Checks the
forward value, that backward scales the adjoint gradient by grad_out (a
non-unit one from a loss built on top of P_sol, and per-instance weights in the
batched form), and the dtype and device of the returned gradients for float64
and float32 angle tensors."""
import numpy as np
import pytest

from gpu_common import log, need_gpu, rand_lits
from oracle.cost import cost_table
from oracle.grad import grad_sv
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst
from paper_2402_02585_amd.autograd import GQAOAProb, GQAOAProbBatched

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("adt", ["float64", "float32"])
def test_single_instance_backward(adt):
    torch = need_gpu()
    n, m, p = 11, 46, 7
    lits = rand_lits(n, m, 401)
    ref_cost = cost_table(n, lits)
    t = int(np.nonzero(np.bincount(ref_cost, minlength=m + 1))[0][0])   # lowest occupied level
    beta0, gamma0 = inst.uniform_angles(402, p)
    log(f"autograd single n={n} p={p} angles {adt} target={t}")
    cost, _ = g.gqaoa_cost_table(n, lits)
    tdt = getattr(torch, adt)
    betas = torch.tensor(beta0, dtype=tdt, device="cuda", requires_grad=True)
    gammas = torch.tensor(gamma0, dtype=tdt, device="cuda", requires_grad=True)
    P = GQAOAProb.apply(betas, gammas, cost, n, m, t, g.C128)
    Pr, db, dg = grad_sv(n, ref_cost, betas.detach().cpu().double().numpy(),
                         gammas.detach().cpu().double().numpy(), t)
    assert P.dtype == torch.float64 and P.is_cuda
    assert abs(P.item() - Pr) < 1e-12
    loss = (P - 0.9) ** 2               # dloss/dP = 2 (P - 0.9), far from 1
    loss.backward()
    go = 2.0 * (Pr - 0.9)
    assert abs(go) > 0.5
    assert betas.grad.dtype == tdt and gammas.grad.dtype == tdt and betas.grad.is_cuda
    atol = 1e-12 if adt == "float64" else 1e-6
    np.testing.assert_allclose(betas.grad.cpu().double().numpy(), go * db, rtol=1e-6 if adt == "float32" else 0,
                               atol=atol)
    np.testing.assert_allclose(gammas.grad.cpu().double().numpy(), go * dg, rtol=1e-6 if adt == "float32" else 0,
                               atol=atol * m)


def test_batched_backward_with_instance_weights():
    torch = need_gpu()
    n, p, I = 10, 5, 4
    ms = [42, 40, 44, 38]
    lits = [rand_lits(n, ms[i], 410 + i) for i in range(I)]
    ref_costs = [cost_table(n, l) for l in lits]
    costs = torch.stack([g.gqaoa_cost_table(n, l, with_hist=False)[0] for l in lits]).contiguous()
    targets = [0, int(np.nonzero(np.bincount(ref_costs[1], minlength=ms[1] + 1))[0][0]), 0, 1]
    b0 = np.stack([inst.uniform_angles(420 + i, p)[0] for i in range(I)])
    g0 = np.stack([inst.uniform_angles(420 + i, p)[1] for i in range(I)])
    log(f"autograd batched I={I} n={n} p={p}")
    betas = torch.tensor(b0, dtype=torch.float64, device="cuda", requires_grad=True)
    gammas = torch.tensor(g0, dtype=torch.float64, device="cuda", requires_grad=True)
    P = GQAOAProbBatched.apply(betas, gammas, costs, n, ms, targets, g.C128)
    wts = torch.tensor([1.0, -2.5, 0.25, 4.0], dtype=torch.float64, device="cuda")
    (wts * P).sum().backward()
    for i in range(I):
        Pr, db, dg = grad_sv(n, ref_costs[i], b0[i], g0[i], targets[i])
        assert abs(P[i].item() - Pr) < 1e-12, i
        w = float(wts[i])
        np.testing.assert_allclose(betas.grad[i].cpu().numpy(), w * db, rtol=0, atol=1e-12)
        np.testing.assert_allclose(gammas.grad[i].cpu().numpy(), w * dg, rtol=0, atol=1e-12 * ms[i])
