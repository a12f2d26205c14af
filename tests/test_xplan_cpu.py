"""The X-QAOA passes' chunk plans on the host (csrc/xplan.h, compiled here
with g++ into a small driver that prints every plan): for every tile size,
register count and group the passes use, the chunks apply each of the group's
qubits exactly once and no other, every chunk's register window lies inside
the tile, the forward mixers start from the load layout, group 0's plan ends
where its costs are read straight from the cost table, and the mixing-only
plan of group 0 ends where lanes cover runs of at least 128 bytes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_02585_amd", "csrc")

DRIVER = r"""
#include "xplan.h"
#include <cstdio>
#include <cstdlib>
static void show(const char *kind, int tb, int r, int mlo, const gqaoa::XPlan &p) {
    std::printf("%s %d %d %d %d", kind, tb, r, mlo, p.nchunks);
    for (int k = 0; k < p.nchunks; ++k) std::printf(" %d:%d", p.rb[k], p.mask[k]);
    std::printf("\n");
}
int main(int argc, char **argv) {
    const int tb = std::atoi(argv[1]), r = std::atoi(argv[2]);
    for (int mlo = 0; mlo < tb; ++mlo) show("group", tb, r, mlo, gqaoa::x_plan(tb, r, mlo));
    show("mix0", tb, r, 0, gqaoa::x_plan_mix0(tb, r));
    return 0;
}
"""

# (tile bits, register bits, amplitude bytes): group 0 and the high groups,
# complex64 and complex128
CONFIGS = [(12, 4, 8), (13, 4, 8), (11, 3, 16), (12, 3, 16)]
MAX_CHUNKS = 6


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("xplan")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return exe


def _plans(driver, tb, r):
    out = subprocess.run([str(driver), str(tb), str(r)], capture_output=True, text=True, check=True).stdout
    plans = []
    for line in out.splitlines():
        f = line.split()
        chunks = [tuple(int(v) for v in c.split(":")) for c in f[5:]]
        assert len(chunks) == int(f[4])
        plans.append((f[0], int(f[3]), chunks))
    return plans


def _covered(chunks, tb, r):
    """Tile bits each chunk applies, checking the register window."""
    seen = []
    for rb, mask in chunks:
        assert 0 <= rb <= tb - r, (rb, tb, r)
        assert 0 <= mask < (1 << r)
        seen += [rb + q for q in range(r) if (mask >> q) & 1]
    return seen


@pytest.mark.parametrize("tb,r,cs", CONFIGS)
def test_every_group_plan_applies_each_qubit_once(driver, tb, r, cs):
    for kind, mlo, chunks in _plans(driver, tb, r):
        if kind != "group":
            continue
        assert 1 <= len(chunks) <= MAX_CHUNKS
        seen = _covered(chunks, tb, r)
        assert sorted(seen) == list(range(mlo, tb)), (tb, r, mlo, chunks)
        assert chunks[0][0] == tb - r          # the forward mixers start in the load layout
        if mlo == 0:
            assert chunks[-1][0] == 0          # group 0 ends with its costs consecutive in the table


@pytest.mark.parametrize("tb,r,cs", CONFIGS)
def test_mixing_only_plan_of_group_zero(driver, tb, r, cs):
    (kind, _, chunks), = [p for p in _plans(driver, tb, r) if p[0] == "mix0"]
    assert 1 <= len(chunks) <= MAX_CHUNKS
    assert sorted(_covered(chunks, tb, r)) == list(range(tb))
    assert chunks[0][0] == tb - r
    assert cs << chunks[-1][0] >= 128           # stored from lanes over runs of >= 128 bytes


def test_plans_have_teeth(driver):
    """A plan that dropped or repeated a bit would fail the coverage check:
    the check rejects both on a hand-made plan."""
    with pytest.raises(AssertionError):
        assert sorted(_covered([(8, 0b1111), (0, 0b1111)], 12, 4)) == list(range(12))
    with pytest.raises(AssertionError):
        assert sorted(_covered([(8, 0b1111), (4, 0b1111), (5, 0b0001), (0, 0b1111)], 12, 4)) == list(range(12))
