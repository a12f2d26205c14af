"""The benchmark's command-line contract and the product path's refusal to run
without its GPU library, on a machine without a GPU."""
import os
import subprocess
import sys

import pytest

from paper_2402_02585_amd import gqaoa as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_without_gpu_exits_instead_of_falling_back():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = _bench("--steps", "1", "--warmup", "0")
    assert r.returncode == 1
    assert "needs a GPU" in r.stderr
    assert r.stdout == ""


def test_missing_library_is_an_error(monkeypatch):
    monkeypatch.setattr(g, "_lib", None)
    monkeypatch.setattr(g, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libgqaoa.so"))
    with pytest.raises(g.GQAOAError, match="not built"):
        g.load_library()
    with pytest.raises(g.GQAOAError):
        g.gqaoa_workspace_bytes(10, 4, g.C64)
