"""Helpers shared by the GPU parity tests (inputs come from the seeded
generators; expected values only from the oracle)."""
import functools
import sys

import numpy as np
import pytest

from paper_2402_02585_amd import instances as inst


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def rand_lits(n, m, seed):
    return inst.random_3sat(np.random.Generator(np.random.PCG64(seed)), n, m)


def rand_state(n, seed, dtype=np.complex128):
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    return (v / np.linalg.norm(v)).astype(dtype)


@functools.lru_cache(maxsize=None)
def c2_instance():
    """Seed-2 stream, n = 28, m = 118 (d ~ 4.2): first satisfiable draw."""
    return inst.first_satisfiable(2, 28, 118)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def synthetic_hist(K: int, m: int, n: int, seed: int) -> np.ndarray:
    """A level histogram with exactly K occupied levels out of 0..m (level 0
    always among them) and counts summing to 2^n: a level-space input with
    more occupied levels than random 3-SAT instances of the tested sizes reach.
    uint64 [m + 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lev = np.concatenate([[0], rng.choice(np.arange(1, m + 1), K - 1, replace=False)])
    w = rng.dirichlet(np.ones(K))
    cnt = np.maximum(1, np.floor(w * 2.0 ** n)).astype(np.int64)
    cnt[np.argmax(cnt)] += (1 << n) - int(cnt.sum())
    h = np.zeros(m + 1, dtype=np.uint64)
    h[lev] = cnt.astype(np.uint64)
    assert int(h.sum()) == 1 << n and int((h > 0).sum()) == K
    return h
