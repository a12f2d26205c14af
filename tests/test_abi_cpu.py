"""The C-ABI library on a machine without a GPU: it loads, exports every entry
point that include/gqaoa.h declares, and rejects invalid arguments before any
device call (no compute call runs here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2402_02585_amd import gqaoa as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gqaoa.h")

pytestmark = pytest.mark.skipif(not os.path.exists(g.LIB_PATH), reason="libgqaoa.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gqaoa_\w+)\s*\(", text)))


def test_header_symbols_exported():
    lib = ctypes.CDLL(g.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(g._SIGS), "binding and header disagree"


def test_status_strings_and_version():
    lib = g.load_library()
    assert lib.gqaoa_abi_version() == 1
    assert lib.gqaoa_status_string(0) == b"ok"
    assert lib.gqaoa_status_string(-3) == b"workspace too small"


def _lits(rows):
    return np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1))


def test_cost_table_rejects_bad_clauses():
    lib = g.load_library()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    bad_repeat = _lits([[0, 2, 1]])              # variable 0 twice
    assert lib.gqaoa_cost_table(5, 1, g._np_ptr(bad_repeat), dummy, None, None) == -1
    assert b"repeats" in lib.gqaoa_last_error()
    bad_range = _lits([[0, 2, 10]])              # literal 10 = var 5 >= n
    assert lib.gqaoa_cost_table(5, 1, g._np_ptr(bad_range), dummy, None, None) == -1
    ok = _lits([[0, 2, 4]])
    assert lib.gqaoa_cost_table(2, 1, g._np_ptr(ok), dummy, None, None) == -2   # n < 3
    assert lib.gqaoa_cost_table(35, 1, g._np_ptr(ok), dummy, None, None) == -2  # n > 34
    assert lib.gqaoa_cost_table(5, 0, g._np_ptr(ok), dummy, None, None) == -2   # m < 1
    assert lib.gqaoa_cost_table(5, 1, None, dummy, None, None) == -1
    assert lib.gqaoa_cost_table(5, 1, g._np_ptr(ok), None, None, None) == -1


def test_evolve_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    b = np.zeros(3)
    bp = g._np_ptr(b)
    need = lib.gqaoa_workspace_bytes(10, 3, 0, 0)
    assert need > 0
    assert lib.gqaoa_workspace_bytes(10, 3, 7, 0) == 0
    args = dict(n=10, m=42, cost=d, p=3, beta=bp, gamma=bp, dt=0, uni=1, psi=d, t=0, ws=d, wsb=need)

    def call(**kw):
        a = dict(args, **kw)
        return lib.gqaoa_evolve(a["n"], a["m"], a["cost"], a["p"], a["beta"], a["gamma"], a["dt"], a["uni"],
                                a["psi"], a["t"], None, None, None, a["ws"], a["wsb"], None)

    assert call(n=2) == -2
    assert call(n=35) == -2
    assert call(m=256) == -2
    assert call(p=-1) == -2
    assert call(t=43) == -2
    assert call(dt=3) == -1
    assert call(cost=None) == -1
    assert call(psi=None) == -1
    assert call(beta=None) == -1
    assert call(wsb=need - 1) == -3


def test_evolve_x_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    b = np.zeros(3)
    bp = g._np_ptr(b)
    need = lib.gqaoa_x_workspace_bytes(10, 3, 1)
    assert need > lib.gqaoa_x_workspace_bytes(10, 3, 0) > 0
    assert lib.gqaoa_x_workspace_bytes(2, 3, 0) == 0
    assert lib.gqaoa_x_workspace_bytes(10, -1, 0) == 0

    def call(n=10, m=42, p=3, t=0, dt=1, cost=d, psi=d, beta=bp, wsb=need):
        return lib.gqaoa_evolve_x(n, m, cost, p, beta, bp, dt, 1, psi, t, None, None, None, d, wsb, None)

    assert call(n=2) == -2
    assert call(n=35) == -2
    assert call(m=0) == -2
    assert call(p=-1) == -2
    assert call(t=43) == -2
    assert call(dt=2) == -1
    assert call(cost=None) == -1
    assert call(psi=None) == -1
    assert call(beta=None) == -1
    assert call(wsb=need - 1) == -3


def test_grad_and_scan_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    b = np.zeros(4)
    m = np.array([42], dtype=np.int32)
    t = np.array([43], dtype=np.int32)
    need = lib.gqaoa_grad_workspace_bytes(1, 10, 4, 1, 2)
    assert need > lib.gqaoa_grad_workspace_bytes(1, 10, 4, 1, 0) - 1 or need > 0
    assert lib.gqaoa_grad_batched(1, 10, g._np_ptr(m), d, 0, g._np_ptr(b), g._np_ptr(b), 1, None, 0, None, None,
                                  None, d, need, None) == -2      # p < 1
    assert lib.gqaoa_grad_batched(1, 10, g._np_ptr(m), d, 4, g._np_ptr(b), g._np_ptr(b), 1, g._np_ptr(t), 0, None,
                                  None, None, d, need, None) == -2  # target > m
    ns = np.array([10], dtype=np.int32)
    hist = np.zeros((1, 43), dtype=np.uint64)
    hist[0, :5] = 1
    pl = np.array([4, 2], dtype=np.int32)                      # not ascending
    ws = lib.gqaoa_scan_workspace_bytes(1, 43, 4, 4, 2, 0)
    assert lib.gqaoa_scan_batched(1, g._np_ptr(ns), g._np_ptr(m), g._np_ptr(hist), 43, None, 4, g._np_ptr(b), 4,
                                  g._np_ptr(b), 0, 2, g._np_ptr(pl), d, None, None, d, ws, None) == -1
    pl = np.array([2, 4], dtype=np.int32)
    tile = np.array([3, 4], dtype=np.int32)                    # 3 waves per block is not offered
    assert lib.gqaoa_scan_batched(1, g._np_ptr(ns), g._np_ptr(m), g._np_ptr(hist), 43, None, 4, g._np_ptr(b), 4,
                                  g._np_ptr(b), 0, 2, g._np_ptr(pl), d, None, g._np_ptr(tile), d, ws, None) == -1
    assert lib.gqaoa_scan_batched(1, g._np_ptr(ns), g._np_ptr(m), g._np_ptr(hist), 43, None, 4, g._np_ptr(b), 4,
                                  g._np_ptr(b), 0, 2, g._np_ptr(pl), d, None, None, d, ws - 1, None) == -3
    assert lib.gqaoa_scan_workspace_bytes(1, 43, 4, 4, 2, 1) >= ws


def test_scan_rejects_more_than_128_occupied_levels():
    """128 occupied levels is the largest register array of the scan kernels:
    an instance with 129 gets ERANGE from both scan forms, before any device
    call; 128 passes validation (the call then fails only for want of a GPU)."""
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    ns = np.array([30], dtype=np.int32)
    m = np.array([200], dtype=np.int32)
    b = np.zeros(4)
    pl = np.array([1, 4], dtype=np.int32)
    for K, want in ((129, -2), (128, None)):
        hist = np.zeros((1, 201), dtype=np.uint64)
        hist[0, :K] = 1
        hist[0, 0] += (1 << 30) - K
        ws = lib.gqaoa_scan_workspace_bytes(1, 201, 4, 4, 2, 0)
        s1 = lib.gqaoa_scan_batched(1, g._np_ptr(ns), g._np_ptr(m), g._np_ptr(hist), 201, None, 4, g._np_ptr(b), 4,
                                    g._np_ptr(b), 0, 2, g._np_ptr(pl), d, None, None, d, ws, None)
        s2 = lib.gqaoa_scan_crossing(1, g._np_ptr(ns), g._np_ptr(m), g._np_ptr(hist), 201, None, 4, g._np_ptr(b), 4,
                                     g._np_ptr(b), 0, 8, None, ctypes.c_float(0.5), d, None, d, ws, None)
        if want is not None:
            assert s1 == want and s2 == want, (K, s1, s2)
            assert b"occupied levels" in lib.gqaoa_last_error()
        else:
            assert s1 not in (-1, -2, -3) and s2 not in (-1, -2, -3), (K, s1, s2)


def test_fairness_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    p = np.array([0.2, 0.3])
    pp = g._np_ptr(p)
    assert lib.gqaoa_shots_to_all(0, pp, 10, 1, 100, d, None) == -2
    assert lib.gqaoa_shots_to_all(65, pp, 10, 1, 100, d, None) == -2
    assert lib.gqaoa_shots_to_all(2, pp, 0, 1, 100, d, None) == -2
    assert lib.gqaoa_shots_to_all(2, None, 10, 1, 100, d, None) == -1
    bad = np.array([0.7, 0.6])
    assert lib.gqaoa_shots_to_all(2, g._np_ptr(bad), 10, 1, 100, d, None) == -1   # sum > 1
    neg = np.array([0.5, -0.1])
    assert lib.gqaoa_shots_to_all(2, g._np_ptr(neg), 10, 1, 100, d, None) == -1
    assert lib.gqaoa_draws_to_reject(1, pp, 10, 1, 3.8, 5, 100, d, None) == -2     # chi-squared needs K >= 2
    assert lib.gqaoa_draws_to_reject(2, pp, 10, 1, 3.8, 5, 10 ** 7 + 1, d, None) == -2
    assert lib.gqaoa_draws_to_reject(2, pp, 10, 1, 0.0, 5, 100, d, None) == -1
    assert lib.gqaoa_draws_to_reject(2, pp, 10, 1, 3.8, 0, 100, d, None) == -2


def test_mlp_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    assert lib.gqaoa_mlp_forward(d, 0, d, d, d, None) == -2
    assert lib.gqaoa_mlp_adam(d, d, d, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -2
    assert lib.gqaoa_mlp_adam(d, d, d, 1, 1e-3, 1.0, 0.999, 1e-8, None) == -2
    assert lib.gqaoa_mlp_act_bytes(256) > 256 * 256 * 4
    need = lib.gqaoa_mlp_infer_bytes(1000)
    assert need >= 1000 * 256 * 2 and lib.gqaoa_mlp_infer_bytes(0) == 0
    assert lib.gqaoa_mlp_infer(d, 0, d, d, d, need, None) == -2
    assert lib.gqaoa_mlp_infer(d, 1000, None, d, d, need, None) == -1
    assert lib.gqaoa_mlp_infer(d, 1000, d, d, d, need - 1, None) == -3


def test_batched_cost_and_items_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    ns = np.array([10, 15], dtype=np.int32)
    ms = np.array([5, 5], dtype=np.int32)
    lits = np.tile(np.array([0, 2, 4], dtype=np.int32), 10)
    big = np.array([27], dtype=np.int32)
    assert lib.gqaoa_cost_batched(1, g._np_ptr(big), g._np_ptr(ms), g._np_ptr(lits), d, None, 6, None) == -2
    assert lib.gqaoa_cost_batched(2, g._np_ptr(ns), g._np_ptr(ms), g._np_ptr(lits), None, None, 6, None) == -1
    assert lib.gqaoa_cost_batched_offset(2, g._np_ptr(ns)) == 1024 + 32768
    b = np.zeros(2)
    pl = np.array([1, 4], dtype=np.int32)
    big2 = np.array([10, 27], dtype=np.int32)    # instance 1 has n = 27 > 26
    items = np.array([0, 1], dtype=np.int32)
    assert lib.gqaoa_sv_items(2, g._np_ptr(big2), g._np_ptr(ms), None, d, 2, g._np_ptr(items), g._np_ptr(b),
                              g._np_ptr(b), 2, g._np_ptr(pl), d, None, None) == -2
    items = np.array([0, 2], dtype=np.int32)     # no instance 2
    assert lib.gqaoa_sv_items(2, g._np_ptr(ns), g._np_ptr(ms), None, d, 2, g._np_ptr(items), g._np_ptr(b),
                              g._np_ptr(b), 2, g._np_ptr(pl), d, None, None) == -2
    items = np.array([0, 0], dtype=np.int32)
    bad = np.array([4, 1], dtype=np.int32)
    assert lib.gqaoa_sv_items(2, g._np_ptr(ns), g._np_ptr(ms), None, d, 2, g._np_ptr(items), g._np_ptr(b),
                              g._np_ptr(b), 2, g._np_ptr(bad), d, None, None) == -1


def test_evolve_plan_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    out = ctypes.c_void_p()
    need = lib.gqaoa_workspace_bytes(10, 4, 0, 0)
    assert lib.gqaoa_evolve_plan_create(10, 42, d, 4, 0, 1, d, 0, d, need, None, None) == -1        # no plan_out
    assert lib.gqaoa_evolve_plan_create(10, 42, d, 0, 0, 1, d, 0, d, need, None, ctypes.byref(out)) == -2   # p = 0
    assert lib.gqaoa_evolve_plan_create(10, 42, d, 4, 0, 1, d, 43, d, need, None, ctypes.byref(out)) == -2  # target > m
    assert lib.gqaoa_evolve_plan_create(10, 42, d, 4, 2, 1, d, 0, d, need, None, ctypes.byref(out)) == -1   # dtype
    assert lib.gqaoa_evolve_plan_create(10, 42, d, 4, 0, 1, d, 0, d, need - 1, None, ctypes.byref(out)) == -3
    assert not out.value
    assert lib.gqaoa_evolve_plan_run(None, d, d, None, None, None, None) == -1
    lib.gqaoa_evolve_plan_destroy(None)


def test_scan_plan_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    ns = np.array([10, 15], dtype=np.int32)
    ms = np.array([42, 42], dtype=np.int32)
    hist = np.zeros((2, 43), dtype=np.uint64)
    hist[:, :5] = 1
    b = np.zeros(4)
    pl = np.array([1, 4], dtype=np.int32)
    off = np.zeros(2, dtype=np.uint64)
    out = ctypes.c_void_p()

    def create(items, k, grid=b, plan=ctypes.byref(out), costs=d):
        return lib.gqaoa_scan_plan_create(2, g._np_ptr(ns), g._np_ptr(ms), g._np_ptr(hist), 43, None, 4,
                                          g._np_ptr(grid), 4, g._np_ptr(b), 0, 2, g._np_ptr(pl), d, None, None, k,
                                          g._np_ptr(items), costs, g._np_ptr(off), d, None, None, plan)

    ok = np.array([0, 1, 2], dtype=np.int32)
    assert create(ok, 1, plan=None) == -1                                   # no place for the plan
    assert create(np.array([0, 4, 0], dtype=np.int32), 1) == -1             # gamma index outside the grid
    assert create(np.array([0, 0, -1], dtype=np.int32), 1) == -1            # beta index outside the grid
    assert create(np.array([2, 0, 0], dtype=np.int32), 1) == -2             # no instance 2
    assert create(np.array([1, 0, 0], dtype=np.int32), 1) == -2             # n = 15 is past the LDS items
    assert create(ok, 1, costs=None) == -1                                  # items need cost tables
    assert create(ok, -1) == -2
    assert create(ok, 1, grid=np.array([0.0, np.nan, 0.0, 0.0])) == -1      # non-finite angle
    assert not out.value
    assert lib.gqaoa_scan_plan_run(None, None, None, None) == -1
    lib.gqaoa_scan_plan_destroy(None)                                       # a no-op


def test_profile_interval_checks():
    lib = g.load_library()
    assert lib.gqaoa_profile_enable(-1) == -1
    assert lib.gqaoa_profile_enable(3) == 0
    assert lib.gqaoa_profile_enable(0) == 0


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(g.GQAOAError):
        g.gqaoa_cost_table(5, [[0, 2, 4]])


def test_checkpoint_interval_choice():
    """ckpt_every=None: every state kept when that workspace fits the budget,
    else the largest interval that fits (fewest recomputed rounds)."""
    I, n, p = 4, 16, 32
    ws = lambda c: g.gqaoa_grad_workspace_bytes(I, n, p, g.C128, c)
    assert g.choose_ckpt_every(I, n, p, g.C128, budget_bytes=ws(0)) == 0
    budget = ws(0) - 1
    c = g.choose_ckpt_every(I, n, p, g.C128, budget_bytes=budget)
    assert 1 <= c < p and ws(c) <= budget
    assert all(ws(k) > budget for k in range(c + 1, p))
    smallest = min(ws(k) for k in range(1, p))
    c = g.choose_ckpt_every(I, n, p, g.C128, budget_bytes=smallest)
    assert ws(c) == smallest and all(ws(k) > smallest for k in range(c + 1, p))
    with pytest.raises(g.GQAOAError):
        g.choose_ckpt_every(I, n, p, g.C128, budget_bytes=smallest - 1)


def test_hist_grad_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    ns = np.array([10, 12], dtype=np.int32)
    ms = np.array([42, 50], dtype=np.int32)
    hist = np.zeros((2, 51), dtype=np.uint64)
    hist[:, :5] = 1
    ang = np.zeros((2, 6))
    ws = lib.gqaoa_hist_grad_workspace_bytes(2, 51, 6)
    assert ws > 0 and lib.gqaoa_hist_grad_workspace_bytes(2, 51, 0) == 0

    def call(p_max=6, p=None, t=None, wsb=ws, m=ms, stride=51):
        return lib.gqaoa_hist_grad_batched(2, g._np_ptr(ns), g._np_ptr(m), g._np_ptr(hist), stride, g._np_ptr(t),
                                           p_max, g._np_ptr(p), g._np_ptr(ang), g._np_ptr(ang), None, None, None,
                                           d, wsb, None)
    assert call(p_max=0) == -2
    assert call(p=np.array([3, 7], dtype=np.int32)) == -2          # p_i > p_max
    assert call(p=np.array([0, 2], dtype=np.int32)) == -2          # p_i < 1
    assert call(t=np.array([0, 51], dtype=np.int32)) == -2         # target > m
    assert call(m=np.array([42, 51], dtype=np.int32)) == -2        # m + 1 > stride
    assert call(wsb=ws - 1) == -3
    assert lib.gqaoa_hist_grad_batched(2, g._np_ptr(ns), g._np_ptr(ms), None, 51, None, 6, None, g._np_ptr(ang),
                                       g._np_ptr(ang), None, None, None, d, ws, None) == -1


def test_cost_table_noalloc_rejects_bad_arguments():
    """The allocation-free cost table validates like gqaoa_cost_table, before
    any device call."""
    lib = g.load_library()
    dummy = ctypes.c_void_p(16)
    ok = _lits([[0, 2, 4]])
    assert lib.gqaoa_cost_table_noalloc(2, 1, g._np_ptr(ok), dummy, None, None) == -2    # n < 3
    assert lib.gqaoa_cost_table_noalloc(35, 1, g._np_ptr(ok), dummy, None, None) == -2   # n > 34
    assert lib.gqaoa_cost_table_noalloc(5, 256, g._np_ptr(ok), dummy, None, None) == -2  # m > 255
    assert lib.gqaoa_cost_table_noalloc(5, 1, None, dummy, None, None) == -1
    assert lib.gqaoa_cost_table_noalloc(5, 1, g._np_ptr(ok), None, None, None) == -1
    assert lib.gqaoa_cost_table_noalloc(5, 1, g._np_ptr(_lits([[0, 1, 4]])), dummy, None, None) == -1  # var 0 twice


def test_selection_argument_checks():
    lib = g.load_library()
    d = ctypes.c_void_p(16)
    assert lib.gqaoa_row_best(4, 8, d, 3, d, None, None) == -1            # unknown mode
    assert lib.gqaoa_row_best(4, 0, d, 0, d, None, None) == -2
    assert lib.gqaoa_row_best(0, 8, d, 0, d, None, None) == -2
    assert lib.gqaoa_row_best(4, 8, None, 0, d, None, None) == -1
    cnt = np.zeros(1, dtype=np.int64)
    ws = lib.gqaoa_level_probs_workspace_bytes(20)
    assert ws == 8 * ((1 << 20) // 16384 + 1) and lib.gqaoa_level_probs_workspace_bytes(2) == 0
    assert lib.gqaoa_level_probs(2, d, d, 0, 0, 4, d, d, g._np_ptr(cnt), d, ws, None) == -2
    assert lib.gqaoa_level_probs(20, d, d, 0, 256, 4, d, d, g._np_ptr(cnt), d, ws, None) == -2
    assert lib.gqaoa_level_probs(20, d, d, 0, 0, -1, d, d, g._np_ptr(cnt), d, ws, None) == -2
    assert lib.gqaoa_level_probs(20, d, d, 2, 0, 4, d, d, g._np_ptr(cnt), d, ws, None) == -1
    assert lib.gqaoa_level_probs(20, d, d, 0, 0, 4, d, d, g._np_ptr(cnt), d, ws - 1, None) == -3
    assert lib.gqaoa_mlp_angles(0, d, d, d, None) == -2
    assert lib.gqaoa_mlp_angles(4, d, None, d, None) == -1
    assert lib.gqaoa_gather_rows(4, d, 10, d, 6, d, None) == -2             # not a multiple of 4
    assert lib.gqaoa_gather_rows(4, d, 0, d, 8, d, None) == -2
