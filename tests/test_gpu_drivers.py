"""The evaluation drivers end to end on small configurations (their
paper-scale runs are reported in the design notes): each produces its JSON
report with the fields the notes quote, and the numbers obey the checks that
hold at any size."""
import json

import numpy as np
import pytest

from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


def test_rounds_eval_small(tmp_path, capsys):
    need_gpu()
    from paper_2402_02585_amd import rounds_eval
    out = tmp_path / "rounds.json"
    rounds_eval.main(["--n-lo", "9", "--n-hi", "11", "--per-n", "6", "--per-n-large", "2", "--conv-n", "10",
                      "--full", "2", "--full-n-max", "11", "--grid", "60", "31", "--workers", "1",
                      "--out", str(out)])
    r = json.loads(out.read_text())
    for kind in ("sat", "unsat"):
        e = r[kind]["per_S"]["0.5"]
        assert e["instances"] == 18 and 0 < e["reached"] <= 18
        if "fit_slope_log_p_vs_log_inv_P" in e:
            assert 0.0 < e["fit_slope_log_p_vs_log_inv_P"] < 1.5


def test_rounds_eval_set_range_slice_and_convergence_options(tmp_path):
    """One set, an n range for the full-angle search, every second eligible
    instance of it, and full G-QAOA at S = 25% and 75% on the conv-n
    instances: full-angle rounds never exceed the single-pair ones."""
    need_gpu()
    from paper_2402_02585_amd import rounds_eval
    out = tmp_path / "rounds_opts.json"
    rounds_eval.main(["--kinds", "sat", "--n-lo", "9", "--n-hi", "11", "--per-n", "6", "--per-n-large", "2",
                      "--conv-n", "10", "--full-n-min", "10", "--full-n-max", "11", "--full-slice", "1", "2",
                      "--full-conv", "--full-grid", "40", "21", "--grid", "60", "31", "--workers", "1",
                      "--out", str(out)])
    r = json.loads(out.read_text())
    assert set(r) == {"workload", "sat"}
    e = r["sat"]
    rec = e["per_S"]["0.5"]["records"]          # [n, m, d, P, p_single, cap]
    eligible = [x for x in rec if 10 <= x[0] <= 11 and x[4] > 1]
    full = e["full_gqaoa"]
    assert full["instances"] == len(eligible[1::2])
    assert all(f["n"] in (10, 11) and 1 <= f["p_full"] <= f["p_single"] for f in full["records"])
    for S in ("0.25", "0.75"):
        fc = e["per_S"][S].get("full_gqaoa")
        if fc is not None:
            assert 0 < fc["mean_ratio_full_to_single"] <= 1.0
            assert fc["median_p_full"] <= fc["median_p_single"]


def test_fairness_eval_small(tmp_path):
    need_gpu()
    from paper_2402_02585_amd import fairness_eval
    out = tmp_path / "fair.json"
    fairness_eval.main(["--runs", "4000", "--trials", "400", "--max-draws", "4000", "--out", str(out)])
    rows = json.loads(out.read_text())["rows"]
    assert len(rows) == 8
    paper = {("4var", "X", 1): 52.0, ("4var", "X", 2): 83.7, ("4var", "G", 1): 56.1, ("4var", "G", 2): 99.9,
             ("5var", "X", 1): 38.1, ("5var", "X", 2): 68.9, ("5var", "G", 1): 43.1, ("5var", "G", 2): 98.7}
    for r in rows:
        assert abs(r["solution_percent"] - paper[(r["instance"], r["protocol"], r["p"])]) < 0.3
        if r["protocol"] == "G":   # every solution has the same amplitude
            assert r["max_over_min_solution_prob"] < 1 + 1e-9
        assert r["shots_to_all_solutions"]["mean"] >= r["solutions"]


def test_learned_eval_small(tmp_path):
    need_gpu()
    from paper_2402_02585_amd import learned_eval
    out = tmp_path / "learned.json"
    learned_eval.main(["--train", "300", "--test", "256", "--plain", "2", "--plain-grid", "36", "18",
                       "--steps", "300", "--batch", "256", "--workers", "1", "--out", str(out)])
    r = json.loads(out.read_text())
    assert r["loss_first_last"][1] < r["loss_first_last"][0]
    for p, e in r["per_p"].items():
        # the windows never lose P_sol against the pair they start from
        assert e["mean_psol_learned_window"] >= e["mean_psol_learned"] - 1e-6
        assert 0 < e["mean_psol_batched_optimizer"] <= 1
