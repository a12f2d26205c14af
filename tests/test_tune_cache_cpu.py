"""The scan autotuner's cache file (GQAOA_TUNE_CACHE) on the host: entries
whose launch shape the scan kernels do not accept are dropped when the file is
read (the bucket is then timed again), valid ones are kept. The parser is
host-only C++ (csrc/tune_cache.h), compiled here with g++ into a small test
driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_02585_amd", "csrc")

DRIVER = r"""
#include "tune_cache.h"
#include <cstdio>
int main(int argc, char **argv) {
    std::map<std::string, gqaoa::TileChoice> m;
    FILE *f = std::fopen(argv[1], "r");
    if (!f) return 2;
    const int skipped = gqaoa::tune_cache_read(f, m);
    std::fclose(f);
    std::printf("skipped %d\n", skipped);
    for (const auto &kv : m) std::printf("%s %d %d\n", kv.first.c_str(), kv.second.waves, kv.second.blocks_per_cu);
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("tune")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return exe


def _read(driver, tmp_path, text):
    path = tmp_path / "cache.txt"
    path.write_text(text)
    out = subprocess.run([str(driver), str(path)], capture_output=True, text=True, check=True).stdout.splitlines()
    skipped = int(out[0].split()[1])
    return skipped, {l.split()[0]: (int(l.split()[1]), int(l.split()[2])) for l in out[1:]}


def test_valid_entries_kept(driver, tmp_path):
    skipped, m = _read(driver, tmp_path, "gfx950:k8:t1:p64 4 8\ngfx950:k16:t2:p16 1 32\ngfx950:k24:t1:p64:x 2 1\n")
    assert skipped == 0
    assert m == {"gfx950:k8:t1:p64": (4, 8), "gfx950:k16:t2:p16": (1, 32), "gfx950:k24:t1:p64:x": (2, 1)}


def test_malformed_shapes_dropped(driver, tmp_path):
    text = ("gfx950:k8:t1:p64 0 8\n"       # zero waves: a division by zero in the grid size
            "gfx950:k16:t1:p64 8 4\n"      # more waves than the kernels are compiled for
            "gfx950:k24:t1:p64 3 4\n"      # not a power of two
            "gfx950:k32:t1:p64 4 0\n"      # no blocks
            "gfx950:k40:t1:p64 2 33\n"     # beyond 32 blocks per CU
            "gfx950:k48:t1:p64 -4 -1\n"
            "gfx950:k56:t1:p64 2 16\n")    # the one valid entry
    skipped, m = _read(driver, tmp_path, text)
    assert skipped == 6
    assert m == {"gfx950:k56:t1:p64": (2, 16)}


def test_garbage_stops_reading(driver, tmp_path):
    skipped, m = _read(driver, tmp_path, "gfx950:k8:t1:p64 4 8\nnot a number\ngfx950:k16:t1:p64 2 2\n")
    assert m == {"gfx950:k8:t1:p64": (4, 8)}
