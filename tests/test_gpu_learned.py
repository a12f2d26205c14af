"""GPU: the learned angle predictor against the methods without it.

Trains the device MLP on batched-optimizer labels of small seeded instances
at p in {1, 4, 16, 64} and checks on held-out instances that
  * training reduces the loss,
  * the predicted pairs beat the single fixed cluster-median pair per p (the
    clustering-only baseline) in mean P_sol,
  * the learned form (network pair, local window scans, plain-optimizer
    fallback: learned.solve) reaches >= 0.99 of the batched optimizer's mean
    P_sol, and >= 0.99 of the plain per-instance optimizer's on a seeded
    subsample, at every p including 64,
  * the fallback runs the plain optimizer's steps (grid, then L-BFGS-B) and
    matches optim.plain_single_pair,
  * the batched optimizer agrees with the plain per-call optimizer,
  * a checkpoint restores the network and its optimizer exactly, and
    training resumed from it continues bit for bit.
"""
import math

import numpy as np
import pytest

from gpu_common import log, need_gpu
from oracle.cost import cost_table, level_histogram
from oracle.evolve import psol_single_pair_hist
from paper_2402_02585_amd import gqaoa as g
from paper_2402_02585_amd import instances as inst
from paper_2402_02585_amd import learned, optim

pytestmark = pytest.mark.gpu
P_LIST = [1, 4, 16, 64]


@pytest.fixture(scope="module")
def trained():
    torch = need_gpu()
    train = inst.batched_scan_instances(5, 1600, 10, 16)
    X, Y, lab = learned.training_set(train, P_LIST, grid=(64, 32))
    model = learned.AngleMLP(seed=0)
    losses = model.train(X, Y, steps=2000, batch=256, lr=2e-3, log_every=500)
    log(f"losses {losses}")
    test = inst.batched_scan_instances(6, 200, 10, 16)
    ns = [it.n for it in test]
    ms = [it.m for it in test]
    hd = g.gqaoa_hist_batched(ns, ms, [it.lits for it in test], hist_stride=max(ms) + 1)
    return dict(model=model, losses=losses, lab=lab, test=test, ns=ns, ms=ms, hists_dev=hd,
                hists=hd.cpu().numpy(), torch=torch, X=X, Y=Y)


def test_training_reduces_loss(trained):
    losses = trained["losses"]
    assert losses[-1][1] < 0.5 * losses[0][1], losses


def test_labels_match_oracle(trained):
    """The batched optimizer's reported P_sol at its chosen pair is the oracle's."""
    lab = trained["lab"]
    rng = np.random.Generator(np.random.PCG64(1))
    for i in rng.choice(len(lab["ns"]), 5, replace=False):
        h = lab["hists"][i, :lab["ms"][i] + 1]
        for q, p in enumerate(P_LIST):
            ref = psol_single_pair_hist(h, lab["beta"][i, q], lab["gamma"][i, q], p)
            assert abs(lab["psol"][i, q] - ref) < 1e-5


def test_learned_beats_cluster_median_and_tracks_optimizer(trained):
    model, lab = trained["model"], trained["lab"]
    ns, ms, H, hd = trained["ns"], trained["ms"], trained["hists"], trained["hists_dev"]
    med = learned.cluster_median(lab, P_LIST)
    opt_b, opt_g, opt_p, _ = optim.batched_single_pair(ns, ms, H, P_LIST, grid=(64, 32))
    for q, p in enumerate(P_LIST):
        x = learned.features_for(hd, ns, ms, p)
        bl, gl = model.angles(x)
        p_learn = learned.evaluate_pairs(ns, ms, H, bl, gl, p)
        p_med = learned.evaluate_pairs(ns, ms, H, np.full(len(ns), med[p][0]), np.full(len(ns), med[p][1]), p)
        sol = learned.solve(model, hd, ns, ms, H, p, med[p], plain_grid=(96, 48))
        p_ref = sol["psol"]
        log(f"p={p}: learned {p_learn.mean():.4f}  cluster-median {p_med.mean():.4f}  "
            f"learned form {p_ref.mean():.4f} ({int(sol['fallback'].sum())} fallbacks)  "
            f"optimizer {opt_p[:, q].mean():.4f}")
        assert p_learn.mean() > p_med.mean()
        # solve evaluates the two pairs in one scan (the diagonal of a 2 x 2
        # grid per instance): the same values as the separate scans
        assert np.array_equal(sol["psol_learned"], p_learn) and np.array_equal(sol["psol_median"], p_med)
        assert p_ref.mean() >= 0.99 * opt_p[:, q].mean()
        # every instance's result is the P_sol of its returned pair
        for i in (0, 7, 50):
            ref = psol_single_pair_hist(H[i, :ms[i] + 1], sol["beta"][i], sol["gamma"][i], p)
            assert abs(ref - p_ref[i]) < 1e-5


def test_learned_form_within_one_percent_of_plain_optimizer(trained):
    """The learned form is held to the plain per-instance optimizer (a grid,
    one device call per evaluation, then L-BFGS-B): within 1% of its mean
    P_sol on a seeded subsample, at every p including 64."""
    torch = trained["torch"]
    model, lab = trained["model"], trained["lab"]
    ns, ms, H, hd = trained["ns"], trained["ms"], trained["hists"], trained["hists_dev"]
    med = learned.cluster_median(lab, P_LIST)
    sub = np.random.Generator(np.random.PCG64(11)).choice(len(ns), 5, replace=False)
    gb, gg = optim.fundamental_grid(96, 48)
    for p in P_LIST:
        sol = learned.solve(model, hd, ns, ms, H, p, med[p], plain_grid=(96, 48))
        plain = [optim.plain_single_pair(ns[i], ms[i], hd[i, :ms[i] + 1].contiguous(), p, gb, gg)["psol"]
                 for i in sub]
        log(f"p={p}: learned form {sol['psol'][sub].mean():.4f}  plain {np.mean(plain):.4f}")
        assert sol["psol"][sub].mean() >= 0.99 * np.mean(plain), (p, sol["psol"][sub], plain)


def test_fallback_runs_the_plain_optimizer_steps(trained):
    """Every instance forced to the fallback (ratio far above 1): its pair is
    the plain optimizer's (grid, then L-BFGS-B) with the grid evaluated in one
    batched scan, so its P_sol matches optim.plain_single_pair's over the same
    grid, and equals the oracle's at the returned pair."""
    torch = trained["torch"]
    model, lab = trained["model"], trained["lab"]
    ns, ms, H, hd = trained["ns"], trained["ms"], trained["hists"], trained["hists_dev"]
    med = learned.cluster_median(lab, P_LIST)
    sub = np.random.Generator(np.random.PCG64(12)).choice(len(ns), 6, replace=False)
    ns6, ms6 = [ns[i] for i in sub], [ms[i] for i in sub]
    gb, gg = optim.fundamental_grid(96, 48)
    for p in (4, 16):
        sol = learned.solve(model, hd[sub], ns6, ms6, H[sub], p, med[p], plain_grid=(96, 48), fallback_ratio=1e9)
        assert sol["fallback"].all()
        for k, i in enumerate(sub):
            r = optim.plain_single_pair(ns[i], ms[i], hd[i, :ms[i] + 1].contiguous(), p, gb, gg)
            log(f"p={p} instance {i}: fallback {sol['psol'][k]:.6f}  plain {r['psol']:.6f}")
            assert sol["psol"][k] == pytest.approx(r["psol"], rel=1e-5, abs=1e-7)
            ref = psol_single_pair_hist(H[i, :ms[i] + 1], sol["beta"][k], sol["gamma"][k], p)
            assert sol["psol"][k] == pytest.approx(ref, abs=1e-12)


def test_plain_optimizer_agrees_with_batched():
    torch = need_gpu()
    its = inst.batched_scan_instances(9, 3, 9, 11)
    ns = [it.n for it in its]
    ms = [it.m for it in its]
    H = np.zeros((3, max(ms) + 1), dtype=np.int64)
    for i, it in enumerate(its):
        H[i, :it.m + 1] = level_histogram(cost_table(it.n, it.lits), it.m)
    gb, gg = optim.fundamental_grid(48, 24)
    ob, og, op, _ = optim.batched_single_pair(ns, ms, H, [4], grid=(48, 24))
    for i, it in enumerate(its):
        hdev = torch.tensor(H[i, :it.m + 1], device="cuda")
        r = optim.plain_single_pair(it.n, it.m, hdev, 4, gb, gg)
        assert r["psol"] >= op[i, 0] - 2e-3
        assert r["psol"] == pytest.approx(psol_single_pair_hist(H[i, :it.m + 1], r["beta"], r["gamma"], 4), abs=1e-12)
        assert op[i, 0] >= r["psol"] - 2e-3


def test_checkpoint_resume(trained, tmp_path):
    """save() / load() keep parameters, Adam moments and the step count
    exactly; two models restored from one checkpoint and trained on with the
    same seed end bit-identical (the fixture's model is left untouched)."""
    torch = trained["torch"]
    model = trained["model"]
    path = tmp_path / "angle_mlp.npz"
    model.save(path)
    a = learned.AngleMLP.load(path)
    b = learned.AngleMLP.load(path)
    assert torch.equal(a.params, model.params) and torch.equal(a.state, model.state) and a.step == model.step
    la = a.train(trained["X"], trained["Y"], steps=50, batch=256, lr=1e-3, seed=3, log_every=49)
    lb = b.train(trained["X"], trained["Y"], steps=50, batch=256, lr=1e-3, seed=3, log_every=49)
    assert a.step == b.step == model.step + 50
    assert torch.equal(a.params, b.params) and torch.equal(a.state, b.state)
    assert la == lb
    assert not torch.equal(a.params, model.params)
