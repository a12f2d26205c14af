#!/usr/bin/env python3
"""Benchmark of the G-QAOA hot path on one MI355X.

Headline workload: one random 3-SAT instance with n = 28 variables and
m = 118 clauses (d ~ 4.2), complex64 state of 2^28 amplitudes (2 GiB) plus a
uint8 cost table, p = 64 rounds with independent per-round angles drawn from
a seed. One step = clause ingest + bit-sliced cost table + level histogram +
64 statevector rounds (phase, Grover mixer, readouts) + the final readout
pass. ``value`` is amplitude-rounds per second: 2^28 * 64 / step time.

Also reported (extra keys of the same JSON line):
  * ``roofline`` of the dominant kernel (the statevector round pass),
  * ``cpu_baseline``: the CPU oracle timed on a bounded sample,
  * ``batched``: the single-angle-pair scan over 4096 instances (n in 8..20,
    d in {3, 4.2, 5}, 64 x 64 angle grid, p in {1, 4, 16, 64}) against the
    plain one-instance-one-angle-pair path on the same GPU,
  * ``cost_table``: clause evaluations per second of the cost-table kernel,
  * ``adjoint``: batched adjoint gradients (256 instances, n = 20, p = 32),
  * ``xqaoa``: the X-QAOA comparator on the headline instance (p = 16),
  * ``rounds_to_target``: the single-pair rounds-to-target search over 512
    instances,
  * ``mlp``: angle-network inference over 65,536 instances and training steps,
  * ``small_n_graph``: small states, eager calls against evolve-plan replays,
  * ``fairness``: the fair-sampling Monte Carlo on the 5-variable worked
    instance of Sec. IV.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3   # published; an FMA counts two flops
# 256 CUs x 4 SIMDs x 32 lane-operations per cycle x 2.4 GHz: gfx950 issues
# two-operand 32-bit VALU instructions on VGPR operands at twice the rate of
# those with an SGPR operand (measured 7.5e13 adds or multiplies per second,
# 3.9e13 with an SGPR operand), so this is reachable without packed math
VALU_LANE_OPS_PEAK = 78.6e12
SCAN_WARM_REPLAYS = 10            # untimed scan replays before the timed ones
PROFILE_EVERY = 7   # coprime with the 64 rounds of a step: the sampled launches cover every round index
N_VARS, M_CLAUSES, P_ROUNDS = 28, 118, 64


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha(*files) -> str:
    """Hash of kernel sources (csrc file names), stored beside counter summaries."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2402_02585_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_json(name: str, *files):
    """The JSON block of a committed counter summary under profiles/, or None
    when it is missing or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    return d if d.get("source_sha") == source_sha(*files) else None


def read_traffic():
    """HBM bytes per launch of the round kernel (counters), or None."""
    d = profile_json("sv_round_c64_n28_counters.md", "sv.hip", "internal.h")
    return None if d is None else d.get("hbm_bytes_per_launch")


def read_scan_counters():
    """Issued VALU lane-operations per scan replay (counters), or None."""
    d = profile_json("scan_c3_counters_and_trace.md", "hist.hip", "batch.h", "internal.h")
    return None if d is None else d.get("valu_lane_ops_per_replay")


def read_cost_table_counters():
    """Issued VALU lane-operations per cost-table launch (counters), or None."""
    d = profile_json("cost_table_n28_counters.md", "cost_table.hip", "cost_bits.h", "internal.h")
    return None if d is None else d.get("valu_lane_ops_per_launch")


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "cpu_model": model}


CPU_WORKERS_MAX = 16   # the host's CPU share on a one-GPU machine


def _oracle_sv_worker(k, n, m, p, barrier, results):
    """One oracle statevector evolution (complex128, numpy, one thread) in a
    worker process, timed from a barrier shared with the other workers."""
    from oracle.cost import cost_table
    from oracle.evolve import evolve_sv
    from paper_2402_02585_amd import instances as inst
    lits = inst.random_3sat(np.random.Generator(np.random.PCG64(500 + k)), n, m)
    cost = cost_table(n, lits)
    beta, gamma = inst.uniform_angles(500 + k, p)
    barrier.wait()
    t0 = time.perf_counter()
    evolve_sv(n, cost, beta, gamma)
    results.put((k, time.perf_counter() - t0))


def oracle_sv_parallel(n: int, m: int, p: int, workers: int):
    """Aggregate amplitude-rounds/s of ``workers`` oracle evolutions running at
    once, one per process (one instance each: the oracle as it stands, run
    over the host's cores instance by instance). Returns (rate, seconds)."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    barrier = ctx.Barrier(workers)
    results = ctx.Queue()
    procs = [ctx.Process(target=_oracle_sv_worker, args=(k, n, m, p, barrier, results)) for k in range(workers)]
    for pr in procs:
        pr.start()
    times = [results.get()[1] for _ in range(workers)]
    for pr in procs:
        pr.join()
    wall = max(times)
    return workers * (2 ** n) * p / wall, wall


def cpu_baseline(legs: bool = True, fair=None):
    """The oracle on bounded samples of each workload.

    Headline: its statevector evolution (complex128, numpy) at n = 22, m = 92,
    p = 64 rounds, one instance per process on up to 16 host cores at once
    (the aggregate rate), and one seed-2 instance on one thread beside it.
    With ``legs``, beside it (one thread each): the level-space path on 64
    instances of the scan workload, the adjoint at the gradient workload's
    size, the MLP on one batch of 256, the X mixer and, given the fairness
    leg's distribution, the fair-sampling Monte Carlo."""
    from oracle.cost import cost_table, level_histogram
    from oracle.evolve import evolve_hist, evolve_sv
    from paper_2402_02585_amd import instances as inst

    n, m, p = 22, 92, 64
    it = inst.first_satisfiable(2, n, m)
    beta, gamma = inst.uniform_angles(2, p)
    cost = cost_table(n, it.lits)
    t0 = time.perf_counter()
    evolve_sv(n, cost, beta, gamma)
    dt = time.perf_counter() - t0
    workers = max(1, min(os.cpu_count() or 1, CPU_WORKERS_MAX))
    rate, wall = oracle_sv_parallel(n, m, p, workers)
    out = {"value": rate, "unit": "amplitude-rounds/s", "cores": workers, "kind": "oracle",
           "sample": f"oracle statevector evolution, n={n} m={m} p={p}, complex128 numpy: {workers} random "
                     f"instances at once, one process (one thread) each, {wall:.1f} s wall",
           "single_thread": {"value": (2 ** n) * p / dt, "seconds": dt,
                             "sample": "the seed-2 instance alone on one thread"}}
    if not legs:
        return out
    out["legs"] = {}
    # scan workload: cost tables + histograms of its first 64 instances, then
    # one 64-round level-space run (4 readouts) at 8 grid cells per instance
    its = inst.batched_scan_instances(3, 64, 8, 20)
    t0 = time.perf_counter()
    hists = [level_histogram(cost_table(x.n, x.lits), x.m) for x in its]
    t_hist = time.perf_counter() - t0
    grid = np.linspace(0.0, math.pi, 64)
    rng = np.random.Generator(np.random.PCG64(35))
    cells = [(h, grid[rng.integers(0, 64)], grid[rng.integers(0, 64)]) for h in hists for _ in range(8)]
    t0 = time.perf_counter()
    for h, b, gm in cells:
        evolve_hist(h, np.full(64, b), np.full(64, gm))
    t_scan = time.perf_counter() - t0
    out["legs"]["batched"] = {
        "value": len(cells) * 4 / t_scan, "unit": "instance-angle evals/s",
        "histograms_clause_evals_per_s": sum(x.m * 2 ** x.n for x in its) / t_hist,
        "sample": f"oracle level-space evolution, 64 instances of the scan workload x 8 grid cells, p = 64 with "
                  f"4 readouts ({t_scan:.1f} s); their cost tables and histograms ({t_hist:.1f} s)"}
    # adjoint workload size: one statevector gradient (n = 20, p = 32) and
    # level-space gradients of 4 instances
    from oracle.grad import grad_hist, grad_sv
    n, m, p = 20, 85, 32
    lits = []
    for _, l in inst.sat_stream(4, n, m):
        if inst.dpll_satisfiable(n, l):
            lits.append(l)
        if len(lits) == 4:
            break
    costs = [cost_table(n, l) for l in lits]
    angles = [inst.uniform_angles(100 + i, p) for i in range(4)]
    t0 = time.perf_counter()
    grad_sv(n, costs[0], angles[0][0], angles[0][1])
    t_sv = time.perf_counter() - t0
    hs = [level_histogram(c, m) for c in costs]
    t0 = time.perf_counter()
    for h, (b, gm) in zip(hs, angles):
        grad_hist(h, b, gm)
    t_h = (time.perf_counter() - t0) / len(hs)
    out["legs"]["adjoint"] = {
        "statevector_gradients_per_s": 1.0 / t_sv, "statevector_amplitude_rounds_per_s": (1 << n) * p / t_sv,
        "level_space_gradients_per_s": 1.0 / t_h,
        "sample": f"oracle reverse sweep, n={n} m={m} p={p}: one statevector gradient ({t_sv:.1f} s), "
                  f"level-space gradients of 4 instances"}
    # MLP: one forward + backward of a batch of 256
    from oracle import mlp as omlp
    prm = omlp.init_params(5)
    x = np.random.Generator(np.random.PCG64(36)).uniform(0.0, 0.2, (256, omlp.D_IN))
    t0 = time.perf_counter()
    o, cache = omlp.forward(prm, x)
    _, dout = omlp.loss_and_dout(o, np.full(256, 1.0), np.full(256, 0.5))
    omlp.backward(prm, cache, dout)
    t_mlp = time.perf_counter() - t0
    out["legs"]["mlp"] = {"training_samples_per_s": 256 / t_mlp,
                          "sample": "oracle MLP forward + loss + backward, one batch of 256 (float64, bfloat16 "
                                    "storage emulated)"}
    # X mixer: the comparator's statevector rounds
    from oracle.xqaoa import evolve_x
    n, m, p = 20, 84, 4
    itx = inst.first_satisfiable(2, n, m)
    bx, gx = inst.uniform_angles(3, p)
    cx = cost_table(n, itx.lits)
    t0 = time.perf_counter()
    evolve_x(n, cx, bx, gx)
    t_x = time.perf_counter() - t0
    out["legs"]["xqaoa"] = {"value": (1 << n) * p / t_x, "unit": "amplitude-rounds/s",
                            "sample": f"oracle X-mixer evolution, n={n} m={m} p={p}, complex128 ({t_x:.1f} s)"}
    if fair is not None:
        # fair sampling: the oracle's Monte Carlo on the leg's distribution
        from oracle.fairness import draws_to_reject, shots_to_all
        t0 = time.perf_counter()
        so = shots_to_all(fair["p_sol"], 5000, 102, 1 << 30)
        t_so = time.perf_counter() - t0
        t0 = time.perf_counter()
        do = draws_to_reject(fair["p_sol"], 3, 202, fair["crit"], fair["n_min"], fair["max_draws"])
        t_do = time.perf_counter() - t0
        d_draws = int(do.sum()) + int((do == 0).sum()) * fair["max_draws"]
        out["legs"]["fairness"] = {
            "shots_per_s": int(so.sum()) / t_so, "draws_per_s": d_draws / t_do,
            "gpu_over_oracle_shots": fair["gpu_shots_per_s"] / (int(so.sum()) / t_so),
            "gpu_over_oracle_draws": fair["gpu_draws_per_s"] / (d_draws / t_do),
            "sample": f"oracle Monte Carlo on the leg's distribution: 5000 shots-to-all runs ({t_so:.1f} s), "
                      f"3 chi-squared trials ({d_draws} draws, {t_do:.1f} s), same seeds as the device runs"}
    return out


def batched_leg(torch, g, inst, steps: int):
    """Single-angle-pair scan of 4096 instances vs the plain per-call path."""
    from paper_2402_02585_amd import instances as _inst  # noqa: F401

    t0 = time.perf_counter()
    insts = inst.batched_scan_instances(3, 4096, 8, 20)
    log(f"generated 4096 satisfiable instances in {time.perf_counter() - t0:.1f} s")
    ns = [it.n for it in insts]
    ms = [it.m for it in insts]
    stride = max(ms) + 1
    hists_dev = g.gqaoa_hist_batched(ns, ms, [it.lits for it in insts], hist_stride=stride)
    hists = hists_dev.cpu().numpy()
    grid = np.linspace(0.0, math.pi, 64)
    plist = [1, 4, 16, 64]
    evals = len(insts) * 64 * 64 * len(plist)
    out = g.gqaoa_scan_batched(ns, ms, hists, grid, grid, plist)       # autotunes, warms up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.gqaoa_scan_batched(ns, ms, hists, grid, grid, plist, out=out)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / steps
    # the same scan as a captured graph: level tables resident, each step
    # uploads the grid and replays one graph
    t0 = time.perf_counter()
    plan = g.ScanPlan(ns, ms, hists, grid, grid, plist)
    torch.cuda.synchronize()
    t_plan_create = time.perf_counter() - t0
    for _ in range(SCAN_WARM_REPLAYS):   # the clock ramps up over the first replays
        plan.run(grid, grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(grid, grid)
    torch.cuda.synchronize()
    t_scan = (time.perf_counter() - t0) / steps
    graph_equal = bool(torch.equal(plan.psol, out[0]) and torch.equal(plan.energy, out[1]))
    plan.close()
    # histogram step of the batched path (all 4096 instances; the clauses as one
    # host array, uploaded and ingested on the device by every call)
    flat_lits = np.concatenate([np.asarray(it.lits, dtype=np.int32).reshape(-1) for it in insts])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.gqaoa_hist_batched(ns, ms, flat_lits, hist_stride=stride)
    torch.cuda.synchronize()
    t_hist = (time.perf_counter() - t0) / steps
    psol = out[0].cpu().numpy()

    # plain path: one instance and one angle pair per call, statevector and level space
    rng = np.random.Generator(np.random.PCG64(33))
    sample = rng.choice(len(insts), 32, replace=False)
    cells = [(int(i), int(rng.integers(0, 64)), int(rng.integers(0, 64))) for i in sample for _ in range(2)]
    costs = {int(i): g.gqaoa_cost_table(insts[i].n, insts[i].lits)[0] for i in sample}
    max_dev = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, bi, gi in cells:
        it = insts[i]
        _, ps, _, _ = g.gqaoa_evolve(it.n, it.m, costs[i], np.full(64, grid[bi]), np.full(64, grid[gi]), dtype=g.C64)
        max_dev = max(max_dev, max(abs(ps[p] - psol[i, q, gi, bi]) for q, p in enumerate(plist)))
    t_sv = (time.perf_counter() - t0) / len(cells)
    hdev = {int(i): hists_dev[i, :insts[i].m + 1].contiguous() for i in sample}
    cells_h = [(int(i), int(rng.integers(0, 64)), int(rng.integers(0, 64))) for i in sample for _ in range(8)]
    t0 = time.perf_counter()
    for i, bi, gi in cells_h:
        it = insts[i]
        ps, _, _ = g.gqaoa_hist_evolve(it.n, it.m, hdev[i], np.full(64, grid[bi]), np.full(64, grid[gi]))
        max_dev = max(max_dev, max(abs(ps[p] - psol[i, q, gi, bi]) for q, p in enumerate(plist)))
    t_h = (time.perf_counter() - t0) / len(cells_h)
    # statevector work items on a seeded subset: every instance with n <= 14
    # (its state fits one block's LDS), 16 random grid cells and the 4 cells
    # where the scan's P_sol peaks (one per p), all in one call
    small = [i for i, it in enumerate(insts) if it.n <= 14]
    s_ns = [insts[i].n for i in small]
    s_ms = [insts[i].m for i in small]
    s_costs, s_offsets, _ = g.gqaoa_cost_batched(s_ns, s_ms, [insts[i].lits for i in small], with_hist=False)
    item_inst, item_cells = [], []   # cells: (instance, gamma index, beta index) of the scan output
    for k, i in enumerate(small):
        peaks = [np.unravel_index(int(np.argmax(psol[i, q])), psol[i, q].shape) for q in range(len(plist))]
        rnd = [(int(rng.integers(0, 64)), int(rng.integers(0, 64))) for _ in range(16)]
        for gi, bi in rnd + [(int(a), int(b)) for a, b in peaks]:
            item_inst.append(k)
            item_cells.append((i, gi, bi))
    item_b = [grid[bi] for _, _, bi in item_cells]
    item_g = [grid[gi] for _, gi, _ in item_cells]
    g.gqaoa_sv_items(s_ns, s_ms, s_costs, item_inst[:64], item_b[:64], item_g[:64], plist)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv_ps, _ = g.gqaoa_sv_items(s_ns, s_ms, s_costs, item_inst, item_b, item_g, plist)
    torch.cuda.synchronize()
    t_items = time.perf_counter() - t0
    sv_ps = sv_ps.cpu().numpy()
    scan_at = np.stack([psol[i, :, gi, bi] for i, gi, bi in item_cells])
    items_dev = float(np.abs(sv_ps - scan_at).max())
    # the larger instances (n = 15..20): the 4 peak cells of each, their
    # states streamed from HBM (all items of one n in one batch)
    large = [i for i, it in enumerate(insts) if it.n > 14]
    l_ns = [insts[i].n for i in large]
    l_ms = [insts[i].m for i in large]
    l_costs, _, _ = g.gqaoa_cost_batched(l_ns, l_ms, [insts[i].lits for i in large], with_hist=False)
    l_inst, l_cells = [], []
    for k, i in enumerate(large):
        for q in range(len(plist)):
            gi, bi = np.unravel_index(int(np.argmax(psol[i, q])), psol[i, q].shape)
            l_inst.append(k)
            l_cells.append((i, int(gi), int(bi)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l_ps, _ = g.gqaoa_sv_items(l_ns, l_ms, l_costs, l_inst, [grid[b] for _, _, b in l_cells],
                               [grid[c] for _, c, _ in l_cells], plist)
    torch.cuda.synchronize()
    t_large = time.perf_counter() - t0
    l_ps = l_ps.cpu().numpy()
    l_dev = float(np.abs(l_ps - np.stack([psol[i, :, c, b] for i, c, b in l_cells])).max())
    l_amp_rounds = sum(2 ** insts[i].n for i, _, _ in l_cells) * plist[-1]
    del l_costs
    # both paths in one graph: the scan on one branch, the items (on the
    # scan's own grid cells) on a parallel one
    cost_off = np.zeros(len(insts), dtype=np.uint64)
    cost_off[small] = s_offsets[:-1]
    both = g.ScanPlan(ns, ms, hists, grid, grid, plist, items=np.array(item_cells, dtype=np.int32), costs=s_costs,
                      cost_off=cost_off)
    both.run(grid, grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        both.run(grid, grid)
    torch.cuda.synchronize()
    t_both = (time.perf_counter() - t0) / 2
    both_equal = bool(torch.equal(both.psol, out[0]) and np.array_equal(both.item_psol.cpu().numpy(), sv_ps))
    both.close()
    rate = evals / t_scan
    # the scan's arithmetic: per occupied level, round and angle pair a complex
    # phase multiply (6 flops), the weighted sum for the mixer (4) and the
    # mixer update (2), issued as 8 two-operand VALU instructions
    levels = (hists > 0).sum(axis=1).astype(np.float64)
    padded = np.ceil(levels / 4) * 4
    scan_flops = float(levels.sum()) * 64 * 64 * plist[-1] * 12
    ops_alg = float(levels.sum()) * 64 * 64 * plist[-1] * 8
    ops_pad = float(padded.sum()) * 64 * 64 * plist[-1] * 8
    ops_issued = read_scan_counters()
    plain_sv = len(plist) / t_sv
    plain_h = len(plist) / t_h
    return {
        "metric": "instance-angle evals/s", "value": rate, "ms_per_scan": t_scan * 1e3,
        "timed": "graph replays of gqaoa_scan_plan (grid upload + one hipGraphLaunch per scan)",
        "ms_per_scan_eager_call": t_eager * 1e3, "plan_create_s": t_plan_create,
        "graph_equals_eager": graph_equal,
        "roofline": {"bound": "alu", "kernel": "scan_kernel", "achieved": scan_flops / t_scan / 1e12,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": scan_flops / t_scan / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                     "flops_per_scan": scan_flops, "mean_levels": float(levels.mean()),
                     "mean_levels_padded": float(padded.mean()),
                     "lane_ops_per_scan": {"algorithmic": ops_alg, "padded": ops_pad, "issued": ops_issued},
                     "valu_lane_ops_peak_per_s": VALU_LANE_OPS_PEAK,
                     "issued_frac_of_valu_peak": None if ops_issued is None else
                     ops_issued / t_scan / VALU_LANE_OPS_PEAK,
                     "note": "achieved counts 12 flops per occupied level-round; issued lane-operations are "
                             "the VALU instructions of one replay from the committed counter summary "
                             "(profiles/scan_c3_counters_and_trace.md, null once the kernel changes) x 64 "
                             "lanes, against two-operand VGPR instructions at 2 per SIMD-cycle"},
        "workload": "4096 satisfiable random 3-SAT, n~U{8..20}, d in {3.0,4.2,5.0}, beta,gamma=linspace(0,pi,64), "
                    "p in {1,4,16,64}, float32",
        "hist_batched_ms": t_hist * 1e3,
        "plain_statevector": {"value": plain_sv, "calls_timed": len(cells), "kind": "gqaoa_evolve complex64 per "
                              "(instance, angle pair), one call gives the 4 readouts"},
        "plain_level_space": {"value": plain_h, "calls_timed": len(cells_h), "kind": "gqaoa_hist_evolve float64 per "
                              "(instance, angle pair)"},
        "speedup_vs_plain_statevector": rate / plain_sv,
        "speedup_vs_plain_level_space": rate / plain_h,
        "max_abs_psol_diff_vs_plain": max_dev,
        "statevector_items_streamed": {"items": len(l_inst), "instances": len(large), "seconds": t_large,
                                       "instance_angle_evals_per_s": len(l_inst) * len(plist) / t_large,
                                       "amplitude_rounds_per_s": l_amp_rounds / t_large,
                                       "max_abs_psol_diff_vs_scan": l_dev,
                                       "kind": "gqaoa_sv_items on instances with n = 15..20: the 4 scan peaks "
                                               "per instance, complex64 states streamed, batched per n"},
        "statevector_items": {"items": len(item_inst), "instances": len(small), "seconds": t_items,
                              "instance_angle_evals_per_s": len(item_inst) * len(plist) / t_items,
                              "speedup_vs_plain_statevector": len(item_inst) * len(plist) / t_items / plain_sv,
                              "max_abs_psol_diff_vs_scan": items_dev,
                              "graph_scan_plus_items_ms": t_both * 1e3, "graph_equals_eager": both_equal,
                              "kind": "gqaoa_sv_items: complex64 state in registers, one block per (instance, angle pair), "
                                      "n <= 14, 16 random cells + the 4 scan peaks per instance"},
    }


def adjoint_leg(torch, g, inst, reps: int = 2):
    """Adjoint workload: 256 satisfiable instances, n = 20, m = 85, p = 32
    independent angles, complex128, checkpoints every 8 rounds. When the
    device has room for every round's state (about 142 GB), the same batch is
    also timed with all states kept (no segment recomputation)."""
    n, m, p, I, ckpt = 20, 85, 32, 256, 8
    lits = []
    for _, l in inst.sat_stream(4, n, m):
        if inst.dpll_satisfiable(n, l):
            lits.append(l)
        if len(lits) == I:
            break
    costs = torch.empty((I, 1 << n), dtype=torch.uint8, device="cuda")
    for i, l in enumerate(lits):
        g.gqaoa_cost_table(n, l, with_hist=False, cost=costs[i])
    betas = np.stack([inst.uniform_angles(100 + i, p)[0] for i in range(I)])
    gammas = np.stack([inst.uniform_angles(100 + i, p)[1] for i in range(I)])
    N = I * (1 << n)
    amp_rounds = N * p

    def timed(every):
        ws = torch.empty(g.gqaoa_grad_workspace_bytes(I, n, p, g.C128, every), dtype=torch.uint8, device="cuda")
        out = g.gqaoa_grad_batched(n, [m] * I, costs, betas, gammas, g.C128, None, every, workspace=ws)  # warm-up
        torch.cuda.synchronize()
        g.gqaoa_profile_reset()
        g.gqaoa_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            out = g.gqaoa_grad_batched(n, [m] * I, costs, betas, gammas, g.C128, None, every, workspace=ws)
        dt = (time.perf_counter() - t0) / reps
        g.gqaoa_profile_enable(False)
        prof = {k: g.gqaoa_profile_read(k) for k in ("sv_reverse_c128", "sv_round_c128")}
        del ws
        torch.cuda.empty_cache()
        return dt, out, prof

    dt, (P, db, dg), prof = timed(ckpt)
    (rev_ms, rev_cnt), (fwd_ms, fwd_cnt) = prof["sv_reverse_c128"], prof["sv_round_c128"]
    # algorithmic bytes: forward 33 B, segment recompute 33 B, reverse 49 B per amplitude-round
    rev_bytes = N * 49
    fwd_bytes = N * 33
    res = {
        "workload": f"{I} satisfiable instances n={n} m={m} (seed 4 stream), p={p} independent angles, complex128, "
                    f"checkpoint every {ckpt} rounds",
        "seconds_per_gradient_batch": dt, "amplitude_rounds_per_s": amp_rounds / dt,
        "reverse_pass": {"avg_launch_ms": rev_ms / max(rev_cnt, 1),
                         "GBps": rev_bytes / (rev_ms / max(rev_cnt, 1) * 1e-3) / 1e9},
        "forward_pass": {"avg_launch_ms": fwd_ms / max(fwd_cnt, 1),
                         "GBps": fwd_bytes / (fwd_ms / max(fwd_cnt, 1) * 1e-3) / 1e9},
        "mean_psol": float(np.mean(P)),
    }
    need = g.gqaoa_grad_workspace_bytes(I, n, p, g.C128, 0)
    free = torch.cuda.mem_get_info()[0]
    if need + (4 << 30) <= free:
        dt0, (P0, db0, dg0), _ = timed(0)
        res["store_all"] = {
            "workspace_GB": need / 1e9, "seconds_per_gradient_batch": dt0,
            "amplitude_rounds_per_s": amp_rounds / dt0, "speedup_vs_checkpointed": dt / dt0,
            # both schedules compute the same forward and reverse rounds
            "max_abs_diff_vs_checkpointed": float(max(np.abs(P0 - P).max(), np.abs(db0 - db).max(),
                                                      np.abs(dg0 - dg).max())),
        }
    else:
        res["store_all"] = {"skipped": f"needs {need / 1e9:.1f} GB, {free / 1e9:.1f} GB free"}
    return res


def fairness_leg(torch, g, inst):
    """Fair-sampling Monte Carlo (Sec. IV): the 5-variable worked instance under
    G-QAOA at p = 2 with its energy-minimizing angles; 100,000 runs of
    shots-to-all-solutions and 10,000 chi-squared trials of at most 1e5 draws.
    Returns the leg and the solution probabilities (for the oracle's timing)."""
    from paper_2402_02585_amd import fairness, fairness_eval

    n, text = fairness_eval.PAPER_INSTANCES["5var"]
    lits = inst.parse_paper_clauses(text)
    m = lits.shape[0]
    cost, hist = g.gqaoa_cost_table(n, lits)
    x = fairness_eval.angles("G", n, m, cost, hist)[2]
    psi, psol, _, _ = g.gqaoa_evolve(n, m, cost, x[:2], x[2:], dtype=g.C128)
    _, pr = fairness.solution_probs(cost, psi)
    K = pr.size
    runs, trials, max_draws = 100000, 10000, 100000
    crit = fairness.chi2_critical(K)
    g.gqaoa_shots_to_all(pr, 1000, 7, 1 << 30)           # warm-up
    g.gqaoa_draws_to_reject(pr, 64, 7, crit, 5 * K, 1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    shots = g.gqaoa_shots_to_all(pr, runs, 102, 1 << 30)
    torch.cuda.synchronize()
    t_shots = time.perf_counter() - t0
    t0 = time.perf_counter()
    rej = g.gqaoa_draws_to_reject(pr, trials, 202, crit, 5 * K, max_draws)
    torch.cuda.synchronize()
    t_rej = time.perf_counter() - t0
    s = shots.cpu().numpy().astype(np.int64)
    d = rej.cpu().numpy().astype(np.int64)
    never = int((d == 0).sum())
    draws = int(d.sum()) + never * max_draws
    res = {
        "workload": f"Sec. IV 5-variable instance (K={K} solutions), G-QAOA p=2 at its energy-minimizing angles "
                    f"(P_sol {psol[-1]:.4f}); {runs} shots-to-all runs, {trials} chi-squared trials "
                    f"(n_min 5K, at most {max_draws} draws)",
        "shots_to_all": {"seconds": t_shots, "runs_per_s": runs / t_shots, "shots_per_s": int(s.sum()) / t_shots,
                         "mean_shots": float(s.mean())},
        "draws_to_reject": {"seconds": t_rej, "trials_per_s": trials / t_rej, "draws_per_s": draws / t_rej,
                            "median_draws": float(np.median(np.where(d > 0, d, np.inf))),
                            "never_rejected": never},
    }
    return res, {"p_sol": pr, "crit": crit, "n_min": 5 * K, "max_draws": max_draws,
                 "gpu_shots_per_s": res["shots_to_all"]["shots_per_s"],
                 "gpu_draws_per_s": res["draws_to_reject"]["draws_per_s"]}


def xqaoa_leg(torch, g, inst, it, reps: int = 3):
    """X-QAOA comparator (transverse-field mixer) on the headline instance:
    n = 28, complex64, p = 16 (the first 16 headline angle pairs)."""
    n, m, p = N_VARS, M_CLAUSES, 16
    beta, gamma = inst.uniform_angles(2, P_ROUNDS)
    beta, gamma = beta[:p], gamma[:p]
    N = 1 << n
    cost, _ = g.gqaoa_cost_table(n, it.lits, with_hist=False)
    psi = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(g.gqaoa_x_workspace_bytes(n, p, g.C64), dtype=torch.uint8, device="cuda")
    g.gqaoa_evolve_x(n, m, cost, beta, gamma, dtype=g.C64, psi=psi, workspace=ws)   # warm-up
    torch.cuda.synchronize()
    g.gqaoa_profile_reset()
    g.gqaoa_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        _, psol, _, norm = g.gqaoa_evolve_x(n, m, cost, beta, gamma, dtype=g.C64, psi=psi, workspace=ws)
    dt = (time.perf_counter() - t0) / reps
    g.gqaoa_profile_enable(False)
    pass_ms, pass_cnt = g.gqaoa_profile_read("x_pass_c64")
    passes = pass_cnt // reps
    # groups at n = 28: qubits 0-11, 12-19, 20-27, taken in the order 1 0 2,
    # then 2 0 1; a round is two passes (group 0 mixing only, and a fused
    # boundary pass). The first pass starts from |s> (writes 8 B, reads 1 B of
    # cost), every other pass reads and writes 16 B, and the p later readout
    # passes (p - 1 fused round boundaries and the last pass) read 1 B of cost;
    # the two cost copies of a call (2 B per amplitude each) are not passes
    pass_bytes = N * (9 + (passes - 1) * 16 + p * 1)
    del psi, ws, cost
    torch.cuda.empty_cache()
    return {
        "workload": f"X-QAOA statevector, the headline instance n={n} m={m}, complex64, p={p} (first {p} headline angle pairs)",
        "seconds_per_call": dt, "amplitude_rounds_per_s": N * p / dt, "passes_per_call": passes,
        "pass": {"kernel": "x_pass_kernel<float>", "avg_launch_ms": pass_ms / max(pass_cnt, 1),
                 "GBps": pass_bytes / (pass_ms / reps * 1e-3) / 1e9,
                 "frac_of_hbm_peak": pass_bytes / (pass_ms / reps * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "round_algorithmic_GBps": 17.0 * N * p / dt / 1e9,
        "final_psol": float(psol[-1]), "max_norm_error": float(np.abs(norm - 1).max()),
    }


def small_n_leg(torch, g, inst, calls: int = 200):
    """Launch-bound statevector calls: one instance evolved again and again
    with new angles, through the eager gqaoa_evolve and through a
    graph-captured plan (one hipGraphLaunch per call). n = 10 and 14 take the
    one-launch resident evolution; n = 20 the streaming round passes."""
    out = {}
    for n, m, p, dt, name in ((10, 42, 20, g.C128, "n10_p20_c128"), (14, 59, 64, g.C64, "n14_p64_c64"),
                              (20, 84, 32, g.C64, "n20_p32_c64")):
        it = inst.first_satisfiable(1, n, m)
        cost, _ = g.gqaoa_cost_table(n, it.lits)
        angles = [inst.uniform_angles(200 + k, p) for k in range(calls)]
        psi = torch.empty(1 << n, dtype=torch.complex64 if dt == g.C64 else torch.complex128, device="cuda")
        ws = torch.empty(g.gqaoa_workspace_bytes(n, p, dt), dtype=torch.uint8, device="cuda")
        g.gqaoa_evolve(n, m, cost, *angles[0], dtype=dt, psi=psi, workspace=ws)
        t0 = time.perf_counter()
        for b, gm in angles:
            ps_e = g.gqaoa_evolve(n, m, cost, b, gm, dtype=dt, psi=psi, workspace=ws)[1]
        t_e = (time.perf_counter() - t0) / calls
        plan = g.EvolvePlan(n, m, cost, p, dtype=dt)
        plan.run(*angles[0])
        t0 = time.perf_counter()
        for b, gm in angles:
            ps_g = plan.run(b, gm)[0]
        t_g = (time.perf_counter() - t0) / calls
        plan.close()
        out[name] = {"eager_ms_per_call": t_e * 1e3, "graph_ms_per_call": t_g * 1e3, "speedup": t_e / t_g,
                     "last_call_max_abs_psol_diff": float(np.abs(ps_g - ps_e).max()),
                     "round_ms_graph": t_g * 1e3 / p}
    out["workload"] = ("one satisfiable instance (seed 1) per size, a new set of p independent angle pairs per call "
                       f"({calls} calls), readouts returned to the host every call")
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0


def mlp_leg(torch, g):
    """Angle MLP (bfloat16 MFMA): inference over 65,536 instances' features
    and training steps (forward, loss, backward, Adam) at batch 512."""
    flops_fwd = 2 * (131 * 256 + 256 * 256 + 256 * 2)       # per sample, the network's own sizes
    rng = np.random.Generator(np.random.PCG64(37))
    params = torch.from_numpy(rng.normal(0.0, 0.05, g.MLP_NPARAMS).astype(np.float32)).cuda()
    B = 65536
    x = torch.from_numpy(rng.uniform(0.0, 0.2, (B, 131)).astype(np.float32)).cuda()
    out = torch.empty((B, 2), dtype=torch.float32, device="cuda")
    act = torch.empty(g.gqaoa_mlp_act_bytes(B), dtype=torch.uint8, device="cuda")
    ws = torch.empty(g.gqaoa_mlp_infer_bytes(B), dtype=torch.uint8, device="cuda")
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_fwd = timed(lambda: g.gqaoa_mlp_forward(params, x, out=out, act=act))
    t_inf = timed(lambda: g.gqaoa_mlp_infer(params, x, out=out, workspace=ws))
    # HBM bytes the inference kernels must move: x (float32) in, h1 (bfloat16) out and back in, outputs out
    inf_bytes = B * (131 * 4 + 2 * 256 * 2 + 2 * 4)
    # training steps at batch 512
    b = 512
    xb = x[:b].contiguous()
    yb = torch.from_numpy(np.stack([rng.uniform(0, 2 * math.pi, b), rng.uniform(0, math.pi, b)], axis=1)
                          .astype(np.float32)).cuda()
    grads = torch.empty(g.MLP_NPARAMS, dtype=torch.float32, device="cuda")
    state = torch.zeros(2 * g.MLP_NPARAMS, dtype=torch.float32, device="cuda")
    ob = torch.empty((b, 2), dtype=torch.float32, device="cuda")
    actb = torch.empty(g.gqaoa_mlp_act_bytes(b), dtype=torch.uint8, device="cuda")

    def step(k):
        g.gqaoa_mlp_forward(params, xb, out=ob, act=actb)
        dout, _ = g.gqaoa_mlp_loss(ob, yb)
        g.gqaoa_mlp_backward(params, actb, dout, grads=grads)
        g.gqaoa_mlp_adam(params, grads, state, k)

    step(1)
    torch.cuda.synchronize()
    steps = 200
    e0.record()
    for k in range(steps):
        step(2 + k)
    e1.record()
    torch.cuda.synchronize()
    t_step = e0.elapsed_time(e1) / steps * 1e-3
    inf_tflops = B * flops_fwd / t_inf / 1e12
    return {
        "workload": "angle MLP 131-256-256-2, bfloat16 weights and activations, float32 accumulation; "
                    "inference batch 65536, training batch 512",
        "inference": {"ms_per_batch": t_inf * 1e3, "instances_per_s": B / t_inf, "TFLOPs": inf_tflops,
                      "frac_of_bf16_mfma_peak": inf_tflops / MFMA_BF16_PEAK_TFLOPS,
                      "hbm_GBps": inf_bytes / t_inf / 1e9, "kind": "gqaoa_mlp_infer (weights in LDS, two launches)",
                      "training_forward_ms": t_fwd * 1e3},
        "training": {"ms_per_step": t_step * 1e3, "samples_per_s": b / t_step,
                     "TFLOPs": 3 * b * flops_fwd / t_step / 1e12},
        "note": "65,536 x 2e5 flops is about 5 us of MFMA work at peak and the inference moves about 100 MB; "
                "training steps at batch 512 are launch-bound (13 launches per step)",
    }


def scan_replays(torch, g, inst, k: int):
    """Only the batched scan of the batched leg, as 1 + k graph replays of its
    scan plan (the dispatches a counter run over scan_kernel sees when the
    autotuner's choices come from GQAOA_TUNE_CACHE). Returns its JSON."""
    insts = inst.batched_scan_instances(3, 4096, 8, 20)
    ns = [it.n for it in insts]
    ms = [it.m for it in insts]
    hists = g.gqaoa_hist_batched(ns, ms, [it.lits for it in insts], hist_stride=max(ms) + 1).cpu().numpy()
    grid = np.linspace(0.0, math.pi, 64)
    plist = [1, 4, 16, 64]
    plan = g.ScanPlan(ns, ms, hists, grid, grid, plist)
    plan.run(grid, grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k):
        plan.run(grid, grid)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / max(k, 1)
    plan.close()
    levels = (hists > 0).sum(axis=1)
    return {"profile": "scan replays", "replays": 1 + k, "timed_replays": k, "ms_per_scan": t * 1e3,
            "mean_levels": float(levels.mean())}


def optimizers_leg(torch, g, inst, plain_instances: int = 4):
    """The three ways to pick single-pair angles, on the same GPU, at p in
    {1, 4, 16, 64}: the plain per-instance optimizer (the paper's pi/180 grid,
    one device call per evaluation, then L-BFGS-B), the batched optimizer (the
    same grid for all instances at once, then two zoom windows) and the
    learned form (the angle network trained here on 20,000 generated
    instances with batched-optimizer labels, then four local windows, and the
    plain optimizer where the result stays below 0.99 of the cluster-median
    pair). 4096 test instances (SeedSequence(6), n ~ U{12..24}); the plain
    optimizer runs on a seeded subsample, where the three are compared."""
    from paper_2402_02585_amd import learned, optim
    P_LIST = [1, 4, 16, 64]
    t0 = time.perf_counter()
    train = inst.batched_scan_instances(5, 20000, 12, 20, workers=CPU_WORKERS_MAX)
    test = inst.batched_scan_instances(6, 4096, 12, 24, workers=CPU_WORKERS_MAX)
    log(f"optimizers leg: generated 20000 + 4096 instances in {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, Y, lab = learned.training_set(train, P_LIST)
    model = learned.AngleMLP(seed=0)
    model.train(X, Y, steps=4000, batch=1024, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    med = learned.cluster_median(lab, P_LIST)
    ns = np.array([it.n for it in test])
    ms = np.array([it.m for it in test])
    I = len(test)
    hd = g.gqaoa_hist_batched(ns, ms, [it.lits for it in test], hist_stride=int(ms.max()) + 1)
    H = hd.cpu().numpy()
    # warm the scan autotuner for every shape both forms use, outside the timed regions
    optim.batched_single_pair(ns[:64], ms[:64], H[:64], P_LIST)
    for p in P_LIST:
        learned.solve(model, hd[:64], ns[:64], ms[:64], H[:64], p, med[p])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, p_batched, _ = optim.batched_single_pair(ns, ms, H, P_LIST)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    p_learned = np.empty((I, len(P_LIST)))
    fallbacks = 0
    t0 = time.perf_counter()
    for q, p in enumerate(P_LIST):
        sol = learned.solve(model, hd, ns, ms, H, p, med[p])
        p_learned[:, q] = sol["psol"]
        fallbacks += int(sol["fallback"].sum())
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    sub = np.random.Generator(np.random.PCG64(8)).choice(I, plain_instances, replace=False)
    gb, gg = optim.fundamental_grid(*optim.paper_grid())
    p_plain = np.empty((plain_instances, len(P_LIST)))
    t0 = time.perf_counter()
    for k, i in enumerate(sub):
        hdev = hd[i, :ms[i] + 1].contiguous()
        for q, p in enumerate(P_LIST):
            p_plain[k, q] = optim.plain_single_pair(int(ns[i]), int(ms[i]), hdev, p, gb, gg)["psol"]
    t_plain = time.perf_counter() - t0
    per_p = {}
    for q, p in enumerate(P_LIST):
        per_p[str(p)] = {
            "subsample_mean_psol": {"plain": float(p_plain[:, q].mean()), "batched": float(p_batched[sub, q].mean()),
                                    "learned": float(p_learned[sub, q].mean())},
            "ratio_batched_to_plain": float(p_batched[sub, q].mean() / p_plain[:, q].mean()),
            "ratio_learned_to_plain": float(p_learned[sub, q].mean() / p_plain[:, q].mean()),
            "all_instances_mean_psol": {"batched": float(p_batched[:, q].mean()),
                                        "learned": float(p_learned[:, q].mean())},
            "ratio_learned_to_batched_all": float(p_learned[:, q].mean() / p_batched[:, q].mean())}
    rate = {"plain": plain_instances * len(P_LIST) / t_plain, "batched": I * len(P_LIST) / t_batched,
            "learned": I * len(P_LIST) / t_learned}
    return {"workload": "4096 satisfiable random 3-SAT (SeedSequence(6)), n~U{12..24}, d in {3.0,4.2,5.0}, "
                        "p in {1,4,16,64}, maximize P_sol; network trained on 20000 instances (SeedSequence(5), "
                        f"n~U{{12..20}}); plain optimizer on {plain_instances} of the test instances",
            "instance_p_per_s": rate, "speedup_vs_plain": {"batched": rate["batched"] / rate["plain"],
                                                           "learned": rate["learned"] / rate["plain"]},
            "per_p": per_p,
            "min_ratio_to_plain": {"batched": min(v["ratio_batched_to_plain"] for v in per_p.values()),
                                   "learned": min(v["ratio_learned_to_plain"] for v in per_p.values())},
            "learned_fallbacks": fallbacks, "train_seconds": t_train, "plain_seconds": t_plain}


def rounds_leg(torch, g, inst):
    """Rounds-to-target search (single angle pair, S = 50%) for 512
    satisfiable instances, n in 12..20, d ~ U(2, 4.5), the pi/180 grid."""
    from paper_2402_02585_amd import rounds
    its = inst.batched_scan_instances(41, 512, 12, 20, density_range=(2.0, 4.5), dup="drop", workers=8)
    ns = np.array([x.n for x in its])
    ms = np.array([x.m for x in its])
    H = g.gqaoa_hist_batched(ns, ms, [x.lits for x in its], hist_stride=int(ms.max()) + 1).cpu().numpy()
    P = H[:, 0] / np.exp2(ns)
    caps = np.clip(np.ceil(3.0 / np.sqrt(P)), 8, 100000).astype(np.int32)
    rounds.single_pair_rounds(ns, ms, H, 0.5, caps)   # warm-up: the scan autotuner sees every bucket the timed call uses
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p_star, _, _ = rounds.single_pair_rounds(ns, ms, H, 0.5, caps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = p_star > 0
    b, _, c = rounds.sqrt_fit(P[ok], p_star[ok])
    return {"workload": "512 satisfiable random 3-SAT (seed 41), n~U{12..20}, d~U(2,4.5), S=0.5, pi/180 grid, "
                        "two zoom levels, cap 3/sqrt(P)",
            "seconds": dt, "instances_per_s": len(its) / dt, "reached": int(ok.sum()),
            "fit_slope_log_p_vs_log_inv_P": b, "median_p_sqrtP": c}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the cpu_baseline leg")
    ap.add_argument("--skip-batched", action="store_true", help="omit the batched-scan leg")
    ap.add_argument("--skip-adjoint", action="store_true", help="omit the adjoint-gradient leg")
    ap.add_argument("--skip-x", action="store_true", help="omit the X-QAOA leg")
    ap.add_argument("--skip-rounds", action="store_true", help="omit the rounds-to-target leg")
    ap.add_argument("--skip-mlp", action="store_true", help="omit the angle-MLP leg")
    ap.add_argument("--skip-small", action="store_true", help="omit the small-n eager vs graph leg")
    ap.add_argument("--skip-fairness", action="store_true", help="omit the fair-sampling Monte Carlo leg")
    ap.add_argument("--skip-optimizers", action="store_true",
                    help="omit the plain vs batched vs learned optimizer comparison")
    ap.add_argument("--profile-scan", type=int, default=0, metavar="K",
                    help="run only 1 + K graph replays of the batched scan and print their timing (counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three 2 GiB device copies (the reference dispatch for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU; --gpus must be 1 (multi-GPU sharding is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2402_02585_amd import gqaoa as g
    from paper_2402_02585_amd import instances as inst

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.profile_scan:
        print(json.dumps(scan_replays(torch, g, inst, args.profile_scan)), flush=True)
        return

    if args.copy_calibration:
        src = torch.empty(2 ** 28, dtype=torch.complex64, device="cuda")
        src.zero_()
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 3 x 2 GiB (2^31 bytes read and written per copy)")
        del src, dst
        torch.cuda.empty_cache()

    it = inst.first_satisfiable(2, N_VARS, M_CLAUSES)
    beta, gamma = inst.uniform_angles(2, P_ROUNDS)
    N = 1 << N_VARS
    cost = torch.empty(N, dtype=torch.uint8, device="cuda")
    psi = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(g.gqaoa_workspace_bytes(N_VARS, P_ROUNDS, g.C64), dtype=torch.uint8, device="cuda")

    def step():
        _, hist = g.gqaoa_cost_table(N_VARS, it.lits, cost=cost)
        _, psol, _, _ = g.gqaoa_evolve(N_VARS, M_CLAUSES, cost, beta, gamma, dtype=g.C64, psi=psi, workspace=ws)
        return hist, psol

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    g.gqaoa_profile_reset()
    # HIP events bracket one round pass in PROFILE_EVERY (an event pair around
    # every pass would add ~1% to the step); the bytes of exactly the sampled
    # launches are counted below
    g.gqaoa_profile_enable(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = []
    for _ in range(args.steps):
        hist, psol = step()   # ends with the host copy of the readouts (the stream is synchronized)
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_step = np.diff(np.array([t0] + marks)) * 1e3
    g.gqaoa_profile_enable(False)
    round_ms, round_cnt = g.gqaoa_profile_read("sv_round_c64")
    ct_ms, ct_cnt = g.gqaoa_profile_read("cost_table")
    ms_per_step = elapsed / args.steps * 1e3
    value = N * P_ROUNDS / (elapsed / args.steps)
    log(f"step {ms_per_step:.2f} ms; P_sol(64) = {psol[-1]:.6f}; #SAT = {int(hist[0].item())}")

    # roofline of the round pass: algorithmic bytes = 16 B of state + 1 B of cost
    # per amplitude, except round 1, which starts from |s> and reads no state
    avg_round_ms = round_ms / max(round_cnt, 1)
    sampled = range(0, args.steps * P_ROUNDS, PROFILE_EVERY)   # launch L is round (L mod 64) + 1 of its step
    if len(sampled) != round_cnt:
        raise RuntimeError(f"expected {len(sampled)} timed round passes, the library recorded {round_cnt}")
    sampled_bytes = N * sum(9 if L % P_ROUNDS == 0 else 17 for L in sampled)
    bytes_per_launch = sampled_bytes / max(round_cnt, 1)
    achieved = sampled_bytes / (round_ms * 1e-3) / 1e9
    traffic = read_traffic()
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "sv_forward_kernel<float, true, true, 2, 4, 1, false>", "avg_launch_ms": avg_round_ms,
                "launches": args.steps * P_ROUNDS, "launches_timed": round_cnt,
                "algorithmic_bytes_per_launch": bytes_per_launch}
    ct_avg = ct_ms / max(ct_cnt, 1)
    ct_ops = read_cost_table_counters()
    cost_table = {"avg_launch_ms": ct_avg, "clause_evals_per_s": M_CLAUSES * N / (ct_avg * 1e-3),
                  "valu_lane_ops_per_launch": ct_ops,
                  "issued_frac_of_valu_peak": None if ct_ops is None else ct_ops / (ct_avg * 1e-3) / VALU_LANE_OPS_PEAK,
                  "note": "issued lane-operations from the committed counter summary "
                          "(profiles/cost_table_n28_counters.md; null once the kernel changes)"}

    out = {
        "metric": "amplitude-rounds/s (n=28,p=64) + batched instance-angle evals/s vs plain, same GPU",
        "value": value, "unit": "amplitude-rounds/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "ms_per_step_median": float(np.median(per_step)), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": "G-QAOA statevector, one random 3-SAT instance n=28 m=118 (seed 2, first satisfiable "
                               "draw), complex64, p=64 independent per-round angles U[0,pi] (seed 2)",
                   "n": N_VARS, "m": M_CLAUSES, "p": P_ROUNDS, "amplitudes": N, "parallelism": "single GPU"},
        "roofline": roofline,
        "cost_table": cost_table,
        "host": host_info(),
        "gpu": {"name": torch.cuda.get_device_name(0),
                "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", "")},
    }
    del psi, ws
    torch.cuda.empty_cache()
    if not args.skip_batched:
        out["batched"] = batched_leg(torch, g, inst, max(3, args.steps // 2))
    if not args.skip_adjoint:
        out["adjoint"] = adjoint_leg(torch, g, inst)
    if not args.skip_x:
        out["xqaoa"] = xqaoa_leg(torch, g, inst, it)
    if not args.skip_rounds:
        out["rounds_to_target"] = rounds_leg(torch, g, inst)
    if not args.skip_mlp:
        out["mlp"] = mlp_leg(torch, g)
    if not args.skip_small:
        out["small_n_graph"] = small_n_leg(torch, g, inst)
    if not args.skip_optimizers:
        out["optimizers"] = optimizers_leg(torch, g, inst)
    fair = None
    if not args.skip_fairness:
        out["fairness"], fair = fairness_leg(torch, g, inst)
    if not args.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(fair=fair)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
