"""Python binding of libgqaoa (the C ABI in include/gqaoa.h).

Argument marshalling only: every function forwards to the entry point of the
same name, passing torch device pointers and the current HIP stream. Device
buffers are torch tensors on ``cuda`` (ROCm); host arrays are numpy. There is
no CPU fallback: the functions raise ``GQAOAError`` when the library or a
gfx950 device is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgqaoa.so")

C64, C128 = 0, 1
ROW_ARGMAX_F32, ROW_ARGMIN_F32, ROW_MIN_POSITIVE_I32 = 0, 1, 2   # modes of gqaoa_row_best
SV_ITEMS_MAX_N = 14          # GQAOA_SV_ITEMS_MAX_N: largest n of a statevector work item (state in registers)
MLP_NPARAMS = 160 * 256 + 256 + 256 * 256 + 256 + 256 * 2 + 2
MLP_OFFSETS = {"W1": (0, (160, 256)), "b1": (40960, (256,)), "W2": (41216, (256, 256)),
               "b2": (106752, (256,)), "W3": (107008, (256, 2)), "b3": (107520, (2,))}

_lib = None
_c = ctypes
_vp, _i32, _sz, _f32 = _c.c_void_p, _c.c_int, _c.c_size_t, _c.c_float

_SIGS = {
    "gqaoa_status_string": ([_i32], _c.c_char_p),
    "gqaoa_last_error": ([], _c.c_char_p),
    "gqaoa_abi_version": ([], _i32),
    "gqaoa_cost_table": ([_i32, _i32, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_cost_table_noalloc": ([_i32, _i32, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_hist_batched": ([_i32, _vp, _vp, _vp, _vp, _i32, _vp], _i32),
    "gqaoa_cost_batched_offset": ([_i32, _vp], _c.c_uint64),
    "gqaoa_cost_batched": ([_i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp], _i32),
    "gqaoa_sv_items": ([_i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_workspace_bytes": ([_i32, _i32, _i32, _i32], _sz),
    "gqaoa_evolve": ([_i32, _i32, _vp, _i32, _vp, _vp, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "gqaoa_evolve_plan_create": ([_i32, _i32, _vp, _i32, _i32, _i32, _vp, _i32, _vp, _sz, _vp, _vp], _i32),
    "gqaoa_evolve_plan_run": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_evolve_plan_destroy": ([_vp], None),
    "gqaoa_solution_prob": ([_i32, _vp, _vp, _i32, _i32, _vp, _vp, _sz, _vp], _i32),
    "gqaoa_x_workspace_bytes": ([_i32, _i32, _i32], _sz),
    "gqaoa_evolve_x": ([_i32, _i32, _vp, _i32, _vp, _vp, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "gqaoa_grad_workspace_bytes": ([_i32, _i32, _i32, _i32, _i32], _sz),
    "gqaoa_grad": ([_i32, _i32, _vp, _i32, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "gqaoa_grad_batched": ([_i32, _i32, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "gqaoa_hist_evolve": ([_i32, _i32, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_hist_grad_workspace_bytes": ([_i32, _i32, _i32], _sz),
    "gqaoa_hist_grad_batched": ([_i32, _vp, _vp, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
                                _i32),
    "gqaoa_scan_workspace_bytes": ([_i32, _i32, _i32, _i32, _i32, _i32], _sz),
    "gqaoa_scan_batched": ([_i32, _vp, _vp, _vp, _i32, _vp, _i32, _vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                            _sz, _vp], _i32),
    "gqaoa_scan_crossing": ([_i32, _vp, _vp, _vp, _i32, _vp, _i32, _vp, _i32, _vp, _i32, _i32, _vp, _f32, _vp, _vp,
                             _vp, _sz, _vp], _i32),
    "gqaoa_scan_plan_create": ([_i32, _vp, _vp, _vp, _i32, _vp, _i32, _vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp, _vp,
                                _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_scan_plan_run": ([_vp, _vp, _vp, _vp], _i32),
    "gqaoa_scan_plan_destroy": ([_vp], None),
    "gqaoa_shots_to_all": ([_i32, _vp, _i32, _c.c_uint64, _i32, _vp, _vp], _i32),
    "gqaoa_draws_to_reject": ([_i32, _vp, _i32, _c.c_uint64, _c.c_double, _i32, _i32, _vp, _vp], _i32),
    "gqaoa_mlp_act_bytes": ([_i32], _sz),
    "gqaoa_mlp_forward": ([_vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_mlp_infer_bytes": ([_i32], _sz),
    "gqaoa_mlp_infer": ([_vp, _i32, _vp, _vp, _vp, _sz, _vp], _i32),
    "gqaoa_mlp_backward": ([_vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_mlp_adam": ([_vp, _vp, _vp, _i32, _f32, _f32, _f32, _f32, _vp], _i32),
    "gqaoa_mlp_loss": ([_i32, _vp, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_mlp_features": ([_i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_row_best": ([_i32, _i32, _vp, _i32, _vp, _vp, _vp], _i32),
    "gqaoa_level_probs_workspace_bytes": ([_i32], _sz),
    "gqaoa_level_probs": ([_i32, _vp, _vp, _i32, _i32, _c.c_int64, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "gqaoa_mlp_angles": ([_i32, _vp, _vp, _vp, _vp], _i32),
    "gqaoa_gather_rows": ([_i32, _vp, _i32, _vp, _i32, _vp, _vp], _i32),
    "gqaoa_profile_enable": ([_i32], _i32),
    "gqaoa_profile_reset": ([], None),
    "gqaoa_profile_read": ([_c.c_char_p, _vp, _vp], _i32),
}


class GQAOAError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        super().__init__(f"{what} (status {status}){': ' + detail if detail else ''}")
        self.status = status


def load_library():
    """Load libgqaoa.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GQAOAError(-5, "libgqaoa.so is not built", LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(status: int):
    if status != 0:
        lib = load_library()
        raise GQAOAError(status, lib.gqaoa_status_string(status).decode(), lib.gqaoa_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise GQAOAError(-5, "no GPU visible to torch; libgqaoa has no CPU path")
    return torch


def _stream(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _dtype_code(dtype) -> int:
    if dtype in (C64, "c64", "complex64"):
        return C64
    if dtype in (C128, "c128", "complex128"):
        return C128
    raise ValueError(f"unknown dtype {dtype!r}")


def _lits(lits) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(lits, dtype=np.int32).reshape(-1))


# ---- cost table -----------------------------------------------------------------------
def gqaoa_cost_table(n: int, lits, with_hist: bool = True, cost=None, stream=None):
    """Returns (cost uint8[2^n], hist int64[m+1] or None) as device tensors."""
    torch = _torch()
    lib = load_library()
    flat = _lits(lits)
    m = flat.size // 3
    if cost is None:
        cost = torch.empty(1 << n, dtype=torch.uint8, device="cuda")
    hist = torch.empty(m + 1, dtype=torch.int64, device="cuda") if with_hist else None
    _check(lib.gqaoa_cost_table(n, m, _np_ptr(flat), _ptr(cost), _ptr(hist), _stream(torch, stream)))
    return cost, hist


def gqaoa_cost_table_noalloc(n: int, lits, hist=None, cost=None, stream=None):
    """gqaoa_cost_table with the library's static scratch (no device
    allocation inside the call). cost: uint8 [2^n] device tensor, hist: int64
    [m+1] device tensor or None; allocated here when not given. Returns (cost, hist)."""
    torch = _torch()
    lib = load_library()
    flat = _lits(lits)
    m = flat.size // 3
    if cost is None:
        cost = torch.empty(1 << n, dtype=torch.uint8, device="cuda")
    if cost.dtype != torch.uint8 or cost.numel() < (1 << n) or not cost.is_cuda:
        raise ValueError(f"cost must be a device uint8 tensor of 2^{n} entries")
    if hist is not None and (hist.dtype != torch.int64 or hist.numel() < m + 1 or not hist.is_cuda):
        raise ValueError(f"hist must be a device int64 tensor of {m + 1} entries")
    _check(lib.gqaoa_cost_table_noalloc(n, m, _np_ptr(flat), _ptr(cost), _ptr(hist), _stream(torch, stream)))
    return cost, hist


def gqaoa_hist_batched(ns, ms, lits_list, hist_stride: int | None = None, stream=None):
    """Level histograms of many instances: int64 device tensor [I, hist_stride].
    lits_list: one literal array per instance, or all of them already
    concatenated in instance order (an int32 array of sum(ms) * 3 literals)."""
    torch = _torch()
    lib = load_library()
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int32))
    flat = _flat_lits(lits_list, ms)
    stride = int(hist_stride or (int(ms.max()) + 1))
    hists = torch.empty((len(ns), stride), dtype=torch.int64, device="cuda")
    _check(lib.gqaoa_hist_batched(len(ns), _np_ptr(ns), _np_ptr(ms), _np_ptr(flat), _ptr(hists), stride,
                                  _stream(torch, stream)))
    return hists


def _flat_lits(lits_list, ms):
    if isinstance(lits_list, np.ndarray):
        flat = _lits(lits_list)
    else:
        flat = np.ascontiguousarray(np.concatenate([_lits(l) for l in lits_list]))
    if flat.size != 3 * int(np.asarray(ms, dtype=np.int64).sum()):
        raise ValueError(f"{flat.size} literals for {int(np.sum(ms))} clauses")
    return flat


def gqaoa_cost_batched(ns, ms, lits_list, with_hist: bool = True, hist_stride: int | None = None, stream=None):
    """Cost tables of many instances (n <= 26) in one launch.

    Returns (costs uint8 device tensor, offsets int64 numpy array [I + 1],
    hists int64 device tensor [I, stride] or None); instance i's table is
    costs[offsets[i] : offsets[i] + 2^n_i]."""
    torch = _torch()
    lib = load_library()
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int32))
    flat = _flat_lits(lits_list, ms)
    offsets = np.array([lib.gqaoa_cost_batched_offset(i, _np_ptr(ns)) for i in range(len(ns) + 1)], dtype=np.int64)
    costs = torch.empty(max(int(offsets[-1]), 1), dtype=torch.uint8, device="cuda")
    stride = int(hist_stride or (int(ms.max()) + 1))
    hists = torch.empty((len(ns), stride), dtype=torch.int64, device="cuda") if with_hist else None
    _check(lib.gqaoa_cost_batched(len(ns), _np_ptr(ns), _np_ptr(ms), _np_ptr(flat), _ptr(costs), _ptr(hists), stride,
                                  _stream(torch, stream)))
    return costs, offsets, hists


def gqaoa_sv_items(ns, ms, costs, item_inst, betas, gammas, p_list, targets=None, with_energy: bool = False,
                   stream=None):
    """Statevector single-pair items on costs from gqaoa_cost_batched.
    Returns (psol, energy) float32 device tensors [num_items, num_p] (energy None
    unless requested)."""
    torch = _torch()
    lib = load_library()
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int32))
    ii = np.ascontiguousarray(np.asarray(item_inst, dtype=np.int32).ravel())
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).ravel())
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64).ravel())
    if not (ii.size == b.size == g.size):
        raise ValueError("item_inst, betas and gammas must have one entry per item")
    pl = np.ascontiguousarray(np.asarray(p_list, dtype=np.int32))
    tg = None if targets is None else np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    psol = torch.empty((ii.size, pl.size), dtype=torch.float32, device="cuda")
    energy = torch.empty((ii.size, pl.size), dtype=torch.float32, device="cuda") if with_energy else None
    _check(lib.gqaoa_sv_items(len(ns), _np_ptr(ns), _np_ptr(ms), _np_ptr(tg), _ptr(costs), ii.size, _np_ptr(ii),
                              _np_ptr(b), _np_ptr(g), pl.size, _np_ptr(pl), _ptr(psol), _ptr(energy),
                              _stream(torch, stream)))
    return psol, energy


# ---- statevector ----------------------------------------------------------------------
def gqaoa_workspace_bytes(n: int, p: int, dtype=C64, ckpt_every: int = 0) -> int:
    return int(load_library().gqaoa_workspace_bytes(n, p, _dtype_code(dtype), ckpt_every))


def _workspace(torch, nbytes: int):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


def _state_args(torch, n, cost, betas, gammas, dt, psi):
    """Host-side shape checks shared by the statevector entry points."""
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).ravel())
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64).ravel())
    if b.size != g.size:
        raise ValueError(f"{b.size} betas but {g.size} gammas")
    cdt = torch.complex64 if dt == C64 else torch.complex128
    if psi is None:
        psi = torch.empty(1 << n, dtype=cdt, device="cuda")
    if psi.dtype != cdt or psi.numel() != (1 << n) or not psi.is_contiguous() or not psi.is_cuda:
        raise ValueError(f"psi must be a contiguous device {cdt} tensor of 2^{n} entries")
    if cost.numel() < (1 << n) or cost.dtype != torch.uint8 or not cost.is_cuda:
        raise ValueError(f"cost must be a device uint8 tensor of 2^{n} entries")
    return b, g, psi


def gqaoa_evolve(n: int, m: int, cost, betas, gammas, dtype=C64, psi=None, init_uniform: bool = True,
                 target_level: int = 0, workspace=None, stream=None):
    """Eq. (3) on the device. Returns (psi, psol[p+1], energy[p+1], norm[p+1])."""
    torch = _torch()
    lib = load_library()
    dt = _dtype_code(dtype)
    b, g, psi = _state_args(torch, n, cost, betas, gammas, dt, psi)
    p = b.size
    need = lib.gqaoa_workspace_bytes(n, p, dt, 0)
    ws = workspace if workspace is not None else _workspace(torch, need)
    psol, energy, norm = np.empty(p + 1), np.empty(p + 1), np.empty(p + 1)
    _check(lib.gqaoa_evolve(n, m, _ptr(cost), p, _np_ptr(b), _np_ptr(g), dt, int(bool(init_uniform)), _ptr(psi),
                            target_level, _np_ptr(psol), _np_ptr(energy), _np_ptr(norm), _ptr(ws),
                            ws.numel(), _stream(torch, stream)))
    return psi, psol, energy, norm


class EvolvePlan:
    """Graph-captured gqaoa_evolve (gqaoa_evolve_plan_*) for one instance and a
    fixed p: each run(betas, gammas) uploads the angles, replays the graph and
    returns (psol, energy, norm) numpy arrays [p+1]; the final state is left
    in ``psi``. The plan holds the cost table, state and workspace tensors."""

    def __init__(self, n: int, m: int, cost, p: int, dtype=C64, init_uniform: bool = True, target_level: int = 0,
                 psi=None, stream=None):
        torch = _torch()
        lib = load_library()
        self._lib = lib
        self._handle = ctypes.c_void_p()
        self.p = int(p)
        dt = _dtype_code(dtype)
        _, _, psi = _state_args(torch, n, cost, np.zeros(self.p), np.zeros(self.p), dt, psi)
        self.psi, self.cost = psi, cost
        self.workspace = _workspace(torch, lib.gqaoa_workspace_bytes(n, self.p, dt, 0))
        _check(lib.gqaoa_evolve_plan_create(n, m, _ptr(cost), self.p, dt, int(bool(init_uniform)), _ptr(psi),
                                            target_level, _ptr(self.workspace), self.workspace.numel(),
                                            _stream(torch, stream), ctypes.byref(self._handle)))

    def run(self, betas, gammas, stream=None):
        torch = _torch()
        b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).ravel())
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64).ravel())
        if b.size != self.p or g.size != self.p:
            raise ValueError(f"the plan runs p={self.p} rounds: {b.size} betas, {g.size} gammas given")
        if not self._handle:
            raise GQAOAError(-1, "plan already closed")
        psol, energy, norm = np.empty(self.p + 1), np.empty(self.p + 1), np.empty(self.p + 1)
        _check(self._lib.gqaoa_evolve_plan_run(self._handle, _np_ptr(b), _np_ptr(g), _np_ptr(psol), _np_ptr(energy),
                                               _np_ptr(norm), _stream(torch, stream)))
        return psol, energy, norm

    def close(self):
        if self._handle:
            self._lib.gqaoa_evolve_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gqaoa_x_workspace_bytes(n: int, p: int, dtype=C64) -> int:
    return int(load_library().gqaoa_x_workspace_bytes(n, p, _dtype_code(dtype)))


def gqaoa_evolve_x(n: int, m: int, cost, betas, gammas, dtype=C64, psi=None, init_uniform: bool = True,
                   target_level: int = 0, workspace=None, stream=None):
    """X-QAOA rounds (transverse-field mixer) on the device.
    Returns (psi, psol[p+1], energy[p+1], norm[p+1])."""
    torch = _torch()
    lib = load_library()
    dt = _dtype_code(dtype)
    b, g, psi = _state_args(torch, n, cost, betas, gammas, dt, psi)
    p = b.size
    ws = workspace if workspace is not None else _workspace(torch, lib.gqaoa_x_workspace_bytes(n, p, dt))
    psol, energy, norm = np.empty(p + 1), np.empty(p + 1), np.empty(p + 1)
    _check(lib.gqaoa_evolve_x(n, m, _ptr(cost), p, _np_ptr(b), _np_ptr(g), dt, int(bool(init_uniform)), _ptr(psi),
                              target_level, _np_ptr(psol), _np_ptr(energy), _np_ptr(norm), _ptr(ws),
                              ws.numel(), _stream(torch, stream)))
    return psi, psol, energy, norm


def gqaoa_solution_prob(n: int, cost, psi, dtype=C64, target_level: int = 0, workspace=None, stream=None) -> float:
    torch = _torch()
    lib = load_library()
    dt = _dtype_code(dtype)
    ws = workspace if workspace is not None else _workspace(torch, lib.gqaoa_workspace_bytes(n, 0, dt, 0))
    out = np.zeros(1)
    _check(lib.gqaoa_solution_prob(n, _ptr(cost), _ptr(psi), dt, target_level, _np_ptr(out), _ptr(ws), ws.numel(),
                                   _stream(torch, stream)))
    return float(out[0])


def gqaoa_grad_workspace_bytes(num_inst: int, n: int, p: int, dtype=C128, ckpt_every: int = 0) -> int:
    return int(load_library().gqaoa_grad_workspace_bytes(num_inst, n, p, _dtype_code(dtype), ckpt_every))


def choose_ckpt_every(num_inst: int, n: int, p: int, dtype=C128, budget_bytes: int | None = None) -> int:
    """Checkpoint interval of the adjoint sweep for a workspace budget: 0
    (every round's state kept, nothing recomputed) when that fits, else the
    largest interval whose workspace fits, which recomputes the fewest rounds
    (the rounds of every segment but the last). The budget defaults to 90% of
    the device's free memory. Raises GQAOAError (EWORKSPACE) when no interval
    fits."""
    lib = load_library()
    dt = _dtype_code(dtype)
    if budget_bytes is None:
        free, _ = _torch().cuda.mem_get_info()
        budget_bytes = int(0.9 * free)
    if lib.gqaoa_grad_workspace_bytes(num_inst, n, p, dt, 0) <= budget_bytes:
        return 0
    for c in range(p - 1, 0, -1):
        if lib.gqaoa_grad_workspace_bytes(num_inst, n, p, dt, c) <= budget_bytes:
            return c
    raise GQAOAError(-3, "no checkpoint interval fits the workspace budget",
                     f"{num_inst} instances, n={n}, p={p}, budget {budget_bytes} bytes")


def gqaoa_grad(n: int, m: int, cost, betas, gammas, dtype=C128, target_level: int = 0, ckpt_every: int | None = None,
               workspace=None, stream=None):
    """Returns (P, dP/dbeta[p], dP/dgamma[p]) by the adjoint sweep (ckpt_every
    as in gqaoa_grad_batched)."""
    P, db, dg = gqaoa_grad_batched(n, [m], cost, np.asarray(betas)[None, :], np.asarray(gammas)[None, :], dtype,
                                   [target_level], ckpt_every, workspace, stream)
    return float(P[0]), db[0], dg[0]


def gqaoa_grad_batched(n: int, ms, costs, betas, gammas, dtype=C128, targets=None, ckpt_every: int | None = None,
                       workspace=None, stream=None):
    """Batched adjoint: costs uint8 [I, 2^n] (contiguous), betas/gammas [I, p].
    ckpt_every: rounds between stored states (0: every state kept); None
    chooses it with choose_ckpt_every, within the given workspace's size or
    the device's free memory, so states are recomputed only when keeping them
    all would not fit. Returns (P[I], dbeta[I, p], dgamma[I, p])."""
    torch = _torch()
    lib = load_library()
    dt = _dtype_code(dtype)
    ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int32))
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
    I, p = b.shape
    tg = None if targets is None else np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    if ckpt_every is None:
        ckpt_every = choose_ckpt_every(I, n, p, dtype, None if workspace is None else workspace.numel())
    need = lib.gqaoa_grad_workspace_bytes(I, n, p, dt, ckpt_every)
    ws = workspace if workspace is not None else _workspace(torch, need)
    P, db, dg = np.empty(I), np.empty((I, p)), np.empty((I, p))
    _check(lib.gqaoa_grad_batched(I, n, _np_ptr(ms), _ptr(costs), p, _np_ptr(b), _np_ptr(g), dt, _np_ptr(tg),
                                  ckpt_every, _np_ptr(P), _np_ptr(db), _np_ptr(dg), _ptr(ws), ws.numel(),
                                  _stream(torch, stream)))
    return P, db, dg


# ---- level space ------------------------------------------------------------------------
def gqaoa_hist_evolve(n: int, m: int, hist, betas, gammas, target_level: int = 0, stream=None):
    """Level-space evolution of one instance (float64). Returns (psol, energy, norm), each [p+1]."""
    torch = _torch()
    lib = load_library()
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
    p = b.size
    psol, energy, norm = np.empty(p + 1), np.empty(p + 1), np.empty(p + 1)
    _check(lib.gqaoa_hist_evolve(n, m, _ptr(hist), p, _np_ptr(b), _np_ptr(g), target_level, _np_ptr(psol),
                                 _np_ptr(energy), _np_ptr(norm), _stream(torch, stream)))
    return psol, energy, norm


def gqaoa_hist_grad_batched(ns, ms, hists, betas, gammas, targets=None, p=None, workspace=None, stream=None):
    """Level-space adjoint gradient of P_sol for many instances (float64).
    hists: host int64/uint64 [I, stride]; betas, gammas: [I, p_max] (instance
    i uses its first p[i] angles; p None: all p_max). Returns numpy
    (P[I], dP/dbeta[I, p_max], dP/dgamma[I, p_max]); entries beyond p[i] are 0."""
    torch = _torch()
    lib = load_library()
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int32))
    h = np.asarray(hists)
    if h.dtype == np.int64:
        h = h.view(np.uint64)
    h = np.ascontiguousarray(h, dtype=np.uint64)
    I, stride = h.shape
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).reshape(I, -1))
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64).reshape(I, -1))
    if b.shape != g.shape:
        raise ValueError(f"betas {b.shape} and gammas {g.shape} differ")
    pmax = b.shape[1]
    tg = None if targets is None else np.ascontiguousarray(np.asarray(targets, dtype=np.int32).reshape(I))
    pp = None if p is None else np.ascontiguousarray(np.asarray(p, dtype=np.int32).reshape(I))
    need = lib.gqaoa_hist_grad_workspace_bytes(I, stride, pmax)
    ws = workspace if workspace is not None else _workspace(torch, need)
    P, db, dg = np.empty(I), np.empty((I, pmax)), np.empty((I, pmax))
    _check(lib.gqaoa_hist_grad_batched(I, _np_ptr(ns), _np_ptr(ms), _np_ptr(h), stride, _np_ptr(tg), pmax,
                                       _np_ptr(pp), _np_ptr(b), _np_ptr(g), _np_ptr(P), _np_ptr(db), _np_ptr(dg),
                                       _ptr(ws), ws.numel(), _stream(torch, stream)))
    return P, db, dg


def gqaoa_scan_workspace_bytes(num_inst: int, hist_stride: int, nb: int, ng: int, num_p: int,
                               per_instance_grid: bool = False) -> int:
    return int(load_library().gqaoa_scan_workspace_bytes(num_inst, hist_stride, nb, ng, num_p,
                                                         int(bool(per_instance_grid))))


def _scan_common(ns, ms, hists, betas, gammas, targets, tile):
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int32))
    h = np.asarray(hists)
    if h.dtype == np.int64:
        h = h.view(np.uint64)        # counts: the same bits, no copy of a [I][stride] table
    h = np.ascontiguousarray(h, dtype=np.uint64)
    I, stride = h.shape
    if ns.shape != (I,) or ms.shape != (I,):
        raise ValueError(f"ns and ms must have {I} entries")
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
    per_inst = b.ndim == 2
    if per_inst != (g.ndim == 2) or (per_inst and (b.shape[0] != I or g.shape[0] != I)):
        raise ValueError("betas and gammas must both be 1-D, or both [num_inst, *]")
    tg = None if targets is None else np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    if tg is not None and tg.shape != (I,):
        raise ValueError(f"targets must have {I} entries")
    tl = None if tile is None else np.ascontiguousarray(np.asarray(tile, dtype=np.int32))
    return ns, ms, h, I, stride, b, g, per_inst, b.shape[-1], g.shape[-1], tg, tl


def gqaoa_scan_batched(ns, ms, hists, betas, gammas, p_list, targets=None, tile=None, with_energy: bool = True,
                       out=None, workspace=None, stream=None):
    """Single-angle-pair scan. hists: host int64/uint64 [I, stride]. betas, gammas:
    1-D (one grid shared by all instances) or 2-D [I, nb] / [I, ng] (a grid per
    instance). Returns (psol, energy) float32 device tensors [I, num_p, ng, nb]."""
    torch = _torch()
    lib = load_library()
    ns, ms, h, I, stride, b, g, per_inst, nb, ng, tg, tl = _scan_common(ns, ms, hists, betas, gammas, targets, tile)
    pl = np.ascontiguousarray(np.asarray(p_list, dtype=np.int32))
    shape = (I, pl.size, ng, nb)
    if out is None:
        psol = torch.empty(shape, dtype=torch.float32, device="cuda")
        energy = torch.empty(shape, dtype=torch.float32, device="cuda") if with_energy else None
    else:
        psol, energy = out
    for t in (psol, energy):
        if t is not None and (tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_contiguous()):
            raise ValueError(f"scan outputs must be contiguous float32 {shape}")
    need = lib.gqaoa_scan_workspace_bytes(I, stride, nb, ng, pl.size, int(per_inst))
    ws = workspace if workspace is not None else _workspace(torch, need)
    _check(lib.gqaoa_scan_batched(I, _np_ptr(ns), _np_ptr(ms), _np_ptr(h), stride, _np_ptr(tg), nb, _np_ptr(b),
                                  ng, _np_ptr(g), int(per_inst), pl.size, _np_ptr(pl), _ptr(psol), _ptr(energy),
                                  _np_ptr(tl), _ptr(ws), ws.numel(), _stream(torch, stream)))
    return psol, energy


def gqaoa_scan_crossing(ns, ms, hists, betas, gammas, p_max, threshold: float, targets=None, tile=None,
                        workspace=None, stream=None):
    """First round j <= p_max with P_sol >= threshold for every (instance, gamma,
    beta) of the grid (0 if none): int32 device tensor [I, ng, nb]. p_max is
    one int or one per instance."""
    torch = _torch()
    lib = load_library()
    ns, ms, h, I, stride, b, g, per_inst, nb, ng, tg, tl = _scan_common(ns, ms, hists, betas, gammas, targets, tile)
    pm = np.ascontiguousarray(np.asarray(p_max, dtype=np.int32).reshape(-1))
    if pm.size not in (1, I):
        raise ValueError(f"p_max must be one value or {I}")
    pm_all = None if pm.size == 1 else pm
    first = torch.empty((I, ng, nb), dtype=torch.int32, device="cuda")
    need = lib.gqaoa_scan_workspace_bytes(I, stride, nb, ng, 1, int(per_inst))
    ws = workspace if workspace is not None else _workspace(torch, need)
    _check(lib.gqaoa_scan_crossing(I, _np_ptr(ns), _np_ptr(ms), _np_ptr(h), stride, _np_ptr(tg), nb, _np_ptr(b),
                                   ng, _np_ptr(g), int(per_inst), int(pm.max()), _np_ptr(pm_all), float(threshold),
                                   _ptr(first),
                                   _np_ptr(tl), _ptr(ws), ws.numel(), _stream(torch, stream)))
    return first


class ScanPlan:
    """Graph-captured scan (gqaoa_scan_plan_*): the instances' level tables and
    launch shapes are fixed at construction, each run() uploads a grid of the
    same shape and replays one HIP graph. Optional statevector items run on
    grid cells in the same graph.

    items: int array [K, 3] of (instance, gamma index, beta index); costs and
    cost_off: the uint8 cost tables and per-instance byte offsets (e.g. from
    gqaoa_cost_batched; instances without items may have any offset).
    Outputs live on the plan: psol/energy [I, num_p, ng, nb] and
    item_psol/item_energy [K, num_p], complete once the run's stream reaches
    the end of the replay."""

    def __init__(self, ns, ms, hists, betas, gammas, p_list, targets=None, tile=None, with_energy: bool = True,
                 items=None, costs=None, cost_off=None, stream=None):
        torch = _torch()
        lib = load_library()
        self._lib = lib
        self._handle = ctypes.c_void_p()
        ns, ms, h, I, stride, b, g, per_inst, nb, ng, tg, tl = _scan_common(ns, ms, hists, betas, gammas, targets,
                                                                            tile)
        self.shape_b, self.shape_g = b.shape, g.shape
        pl = np.ascontiguousarray(np.asarray(p_list, dtype=np.int32))
        self.psol = torch.empty((I, pl.size, ng, nb), dtype=torch.float32, device="cuda")
        self.energy = torch.empty_like(self.psol) if with_energy else None
        it = np.zeros((0, 3), dtype=np.int32) if items is None else np.asarray(items, dtype=np.int32).reshape(-1, 3)
        it = np.ascontiguousarray(it)
        K = it.shape[0]
        self.item_psol = torch.empty((K, pl.size), dtype=torch.float32, device="cuda") if K else None
        self.item_energy = torch.empty((K, pl.size), dtype=torch.float32, device="cuda") if K and with_energy else None
        co = None
        if K:
            co = np.ascontiguousarray(np.asarray(cost_off, dtype=np.uint64).reshape(-1)[:I])
            if co.size != I:
                raise ValueError(f"cost_off must have {I} entries")
        self._keep = (costs,)
        _check(lib.gqaoa_scan_plan_create(I, _np_ptr(ns), _np_ptr(ms), _np_ptr(h), stride, _np_ptr(tg), nb,
                                          _np_ptr(b), ng, _np_ptr(g), int(per_inst), pl.size, _np_ptr(pl),
                                          _ptr(self.psol), _ptr(self.energy), _np_ptr(tl), K,
                                          _np_ptr(it) if K else None, _ptr(costs) if K else None,
                                          _np_ptr(co), _ptr(self.item_psol), _ptr(self.item_energy),
                                          _stream(torch, stream), ctypes.byref(self._handle)))

    def run(self, betas=None, gammas=None, stream=None):
        """Replay with a new grid (same shapes), or the current one when both are None."""
        torch = _torch()
        if (betas is None) != (gammas is None):
            raise ValueError("give both grids or neither")
        b = g = None
        if betas is not None:
            b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
            g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
            if b.shape != self.shape_b or g.shape != self.shape_g:
                raise ValueError(f"grid shapes {b.shape}, {g.shape} differ from the plan's "
                                 f"{self.shape_b}, {self.shape_g}")
        if not self._handle:
            raise GQAOAError(-1, "plan already closed")
        _check(self._lib.gqaoa_scan_plan_run(self._handle, _np_ptr(b), _np_ptr(g), _stream(torch, stream)))
        return self.psol, self.energy

    def close(self):
        if self._handle:
            self._lib.gqaoa_scan_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- fair-sampling metrics ------------------------------------------------------------
def gqaoa_shots_to_all(p_sol, runs: int, seed: int, max_shots: int, stream=None):
    """Shots until every solution is seen, per run: int32 device tensor [runs]."""
    torch = _torch()
    p = np.ascontiguousarray(np.asarray(p_sol, dtype=np.float64).ravel())
    out = torch.empty(runs, dtype=torch.int32, device="cuda")
    _check(load_library().gqaoa_shots_to_all(p.size, _np_ptr(p), runs, seed, max_shots, _ptr(out),
                                             _stream(torch, stream)))
    return out


def gqaoa_draws_to_reject(q_sol, trials: int, seed: int, crit: float, n_min: int, max_draws: int, stream=None):
    """Draws until the chi-squared test rejects uniform solution sampling, per
    trial: int32 device tensor [trials] (0: not within max_draws)."""
    torch = _torch()
    q = np.ascontiguousarray(np.asarray(q_sol, dtype=np.float64).ravel())
    out = torch.empty(trials, dtype=torch.int32, device="cuda")
    _check(load_library().gqaoa_draws_to_reject(q.size, _np_ptr(q), trials, seed, float(crit), n_min, max_draws,
                                                _ptr(out), _stream(torch, stream)))
    return out


# ---- MLP ---------------------------------------------------------------------------------
def gqaoa_mlp_act_bytes(batch: int) -> int:
    return int(load_library().gqaoa_mlp_act_bytes(batch))


def gqaoa_mlp_forward(params, x, out=None, act=None, stream=None):
    """params float32 [MLP_NPARAMS], x float32 [B, 131] -> (out [B, 2], act cache)."""
    torch = _torch()
    lib = load_library()
    B = x.shape[0]
    out = out if out is not None else torch.empty((B, 2), dtype=torch.float32, device="cuda")
    act = act if act is not None else _workspace(torch, lib.gqaoa_mlp_act_bytes(B))
    _check(lib.gqaoa_mlp_forward(_ptr(params), B, _ptr(x), _ptr(out), _ptr(act), _stream(torch, stream)))
    return out, act


def gqaoa_mlp_infer_bytes(batch: int) -> int:
    return int(load_library().gqaoa_mlp_infer_bytes(batch))


def gqaoa_mlp_infer(params, x, out=None, workspace=None, stream=None):
    """Inference only: params float32 [MLP_NPARAMS], x float32 [B, 131] -> out [B, 2]."""
    torch = _torch()
    lib = load_library()
    B = x.shape[0]
    if tuple(x.shape) != (B, 131) or x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be contiguous float32 [B, 131]")
    out = out if out is not None else torch.empty((B, 2), dtype=torch.float32, device="cuda")
    ws = workspace if workspace is not None else _workspace(torch, lib.gqaoa_mlp_infer_bytes(B))
    _check(lib.gqaoa_mlp_infer(_ptr(params), B, _ptr(x), _ptr(out), _ptr(ws), ws.numel(), _stream(torch, stream)))
    return out


def gqaoa_mlp_backward(params, act, dout, grads=None, stream=None):
    torch = _torch()
    lib = load_library()
    B = dout.shape[0]
    grads = grads if grads is not None else torch.empty(MLP_NPARAMS, dtype=torch.float32, device="cuda")
    _check(lib.gqaoa_mlp_backward(_ptr(params), B, _ptr(act), _ptr(dout), _ptr(grads), _stream(torch, stream)))
    return grads


def gqaoa_mlp_adam(params, grads, state, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    torch = _torch()
    lib = load_library()
    _check(lib.gqaoa_mlp_adam(_ptr(params), _ptr(grads), _ptr(state), step, lr, beta1, beta2, eps,
                              _stream(torch, stream)))


def gqaoa_mlp_loss(out, targets, dout=None, loss=None, stream=None):
    torch = _torch()
    lib = load_library()
    B = out.shape[0]
    dout = dout if dout is not None else torch.empty_like(out)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib.gqaoa_mlp_loss(B, _ptr(out), _ptr(targets), _ptr(dout), _ptr(loss), _stream(torch, stream)))
    return dout, loss


def gqaoa_mlp_features(hists, ns, ms, ps, x=None, stream=None):
    """hists int64 device [B, stride]; ns, ms, ps int32 device [B] -> x float32 [B, 131]."""
    torch = _torch()
    lib = load_library()
    B, stride = hists.shape
    x = x if x is not None else torch.empty((B, 131), dtype=torch.float32, device="cuda")
    _check(lib.gqaoa_mlp_features(B, _ptr(hists), stride, _ptr(ns), _ptr(ms), _ptr(ps), _ptr(x),
                                  _stream(torch, stream)))
    return x


# ---- selections on device data --------------------------------------------------------------
def gqaoa_row_best(x, mode: int, with_value: bool = True, stream=None):
    """Best entry of every row of a contiguous device matrix x (any shape:
    rows = x.shape[0], the rest flattened): float32 for ROW_ARGMAX_F32 /
    ROW_ARGMIN_F32, int32 for ROW_MIN_POSITIVE_I32. Returns (idx int32 [rows],
    value [rows] or None) as device tensors; ties go to the lowest column."""
    torch = _torch()
    want = torch.int32 if mode == ROW_MIN_POSITIVE_I32 else torch.float32
    if x.dtype != want or not x.is_contiguous() or not x.is_cuda:
        raise ValueError(f"x must be a contiguous device {want} tensor")
    rows = int(x.shape[0])
    cols = int(x.numel() // max(rows, 1))
    idx = torch.empty(rows, dtype=torch.int32, device="cuda")
    val = torch.empty(rows, dtype=want, device="cuda") if with_value else None
    _check(load_library().gqaoa_row_best(rows, cols, _ptr(x), int(mode), _ptr(idx), _ptr(val), _stream(torch, stream)))
    return idx, val


def gqaoa_level_probs(n: int, cost, psi, dtype=C64, level: int = 0, max_out: int | None = None, stream=None):
    """(z int64, |psi_z|^2 float64) numpy arrays of the assignments with
    C(z) = level, z ascending (all of them when max_out is None)."""
    torch = _torch()
    lib = load_library()
    dt = _dtype_code(dtype)
    ws = _workspace(torch, lib.gqaoa_level_probs_workspace_bytes(n))
    cap = 4096 if max_out is None else int(max_out)
    cnt = np.zeros(1, dtype=np.int64)
    while True:
        z = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
        pr = torch.empty(max(cap, 1), dtype=torch.float64, device="cuda")
        _check(lib.gqaoa_level_probs(n, _ptr(cost), _ptr(psi), dt, int(level), cap, _ptr(z), _ptr(pr),
                                     _np_ptr(cnt), _ptr(ws), ws.numel(), _stream(torch, stream)))
        total = int(cnt[0])
        if max_out is not None or total <= cap:
            k = min(total, cap)
            return z[:k].cpu().numpy(), pr[:k].cpu().numpy()
        cap = total


def gqaoa_mlp_angles(out, stream=None):
    """Network outputs [B, 2] (float32, device) -> (beta, gamma) float64 device tensors."""
    torch = _torch()
    B = int(out.shape[0])
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != 2 * B:
        raise ValueError("out must be contiguous float32 [B, 2]")
    beta = torch.empty(B, dtype=torch.float64, device="cuda")
    gamma = torch.empty(B, dtype=torch.float64, device="cuda")
    _check(load_library().gqaoa_mlp_angles(B, _ptr(out), _ptr(beta), _ptr(gamma), _stream(torch, stream)))
    return beta, gamma


def gqaoa_gather_rows(src, idx, out=None, stream=None):
    """Rows src[idx[r]] of a contiguous device tensor (first dimension = rows)
    into out [len(idx), *src.shape[1:]]; idx: int32 device tensor."""
    torch = _torch()
    R = int(idx.numel())
    row_bytes = src[0].numel() * src.element_size()
    if out is None:
        out = torch.empty((R,) + tuple(src.shape[1:]), dtype=src.dtype, device="cuda")
    if idx.dtype != torch.int32 or not src.is_contiguous() or not out.is_contiguous():
        raise ValueError("idx must be int32, src and out contiguous")
    _check(load_library().gqaoa_gather_rows(R, _ptr(idx), int(src.shape[0]), _ptr(src), int(row_bytes), _ptr(out),
                                            _stream(torch, stream)))
    return out


# ---- instrumentation ------------------------------------------------------------------------
def gqaoa_profile_enable(on=True, every: int = 1):
    """Time one launch in ``every`` (per kernel name) while ``on``."""
    _check(load_library().gqaoa_profile_enable(int(every) if on else 0))


def gqaoa_profile_reset():
    load_library().gqaoa_profile_reset()


def gqaoa_profile_read(name: str):
    """(total_ms, count) of the launches recorded under ``name``."""
    ms = np.zeros(1)
    cnt = np.zeros(1, dtype=np.int64)
    _check(load_library().gqaoa_profile_read(name.encode(), _np_ptr(ms), _np_ptr(cnt)))
    return float(ms[0]), int(cnt[0])
