"""GPU: the selections the drivers run on device data (gqaoa_row_best,
gqaoa_level_probs, gqaoa_mlp_angles, gqaoa_gather_rows), against plain numpy
on the same inputs and the oracle's angle map: exact for indices, integers and
gathered rows, ties to the lowest column, NaNs never chosen over numbers."""
import numpy as np
import pytest

from gpu_common import log, need_gpu, rand_lits, rand_state
from oracle import mlp as omlp
from oracle.cost import cost_table
from paper_2402_02585_amd import gqaoa as g

pytestmark = pytest.mark.gpu


def _ref_best(x, mode):
    if mode == g.ROW_MIN_POSITIVE_I32:
        v = np.where(x > 0, x.astype(np.int64), np.iinfo(np.int64).max)
        j = v.argmin(axis=1)
        val = v[np.arange(len(j)), j]
        none = val == np.iinfo(np.int64).max
        return np.where(none, 0, j), np.where(none, 0, val)
    fill = -np.inf if mode == g.ROW_ARGMAX_F32 else np.inf
    v = np.where(np.isnan(x), fill, x)
    j = v.argmax(axis=1) if mode == g.ROW_ARGMAX_F32 else v.argmin(axis=1)
    allnan = np.isnan(x).all(axis=1)
    j = np.where(allnan, 0, j)
    return j, x[np.arange(len(j)), j]


@pytest.mark.parametrize("rows,cols", [(1, 1), (7, 300), (33, 65160), (4096, 256), (5, 257)])
@pytest.mark.parametrize("mode", [g.ROW_ARGMAX_F32, g.ROW_ARGMIN_F32, g.ROW_MIN_POSITIVE_I32])
def test_row_best_matches_numpy(rows, cols, mode):
    torch = need_gpu()
    rng = np.random.Generator(np.random.PCG64(rows * 7 + cols + mode))
    if mode == g.ROW_MIN_POSITIVE_I32:
        x = rng.integers(-3, 40, (rows, cols)).astype(np.int32)
        x[rng.random((rows, cols)) < 0.5] = 0
        x[0] = 0                                           # a row without a positive entry
        if cols > 3:
            x[-1, :] = 0
            x[-1, [cols // 2, cols - 1, 2]] = 5            # ties: the lowest column wins
    else:
        x = rng.integers(0, 50, (rows, cols)).astype(np.float32)   # many ties
        x[rng.random((rows, cols)) < 0.05] = np.nan
        x[0] = np.nan if rows > 1 else x[0]                # a row of NaNs only
        if cols > 2:
            x[-1, :] = np.nan
            x[-1, cols - 1] = 3.0
            x[-1, 1] = 3.0
    xd = torch.tensor(x, device="cuda")
    log(f"row_best rows={rows} cols={cols} mode={mode}")
    jd, vd = g.gqaoa_row_best(xd, mode)
    j, v = _ref_best(x, mode)
    np.testing.assert_array_equal(jd.cpu().numpy(), j)
    np.testing.assert_array_equal(vd.cpu().numpy(), v.astype(x.dtype))


@pytest.mark.parametrize("n,dt", [(5, g.C64), (12, g.C128), (16, g.C64), (22, g.C128)])
def test_level_probs_matches_numpy(n, dt):
    torch = need_gpu()
    m = max(1, int(round(4.2 * n)))
    lits = rand_lits(n, m, 500 + n)
    cost_h = cost_table(n, lits)
    cost, _ = g.gqaoa_cost_table(n, lits, with_hist=False)
    psi0 = rand_state(n, 501 + n)
    tdt = torch.complex64 if dt == g.C64 else torch.complex128
    psi = torch.tensor(psi0, dtype=tdt, device="cuda")
    comp = psi.cpu().numpy()
    log(f"level_probs n={n} dt={dt}")
    for level in sorted(set([int(cost_h.min()), int(np.median(cost_h)), m])):
        z, pr = g.gqaoa_level_probs(n, cost, psi, dt, level)
        zr = np.nonzero(cost_h == level)[0]
        np.testing.assert_array_equal(z, zr)
        re = comp.real[zr].astype(np.float64)
        im = comp.imag[zr].astype(np.float64)
        np.testing.assert_allclose(pr, re * re + im * im, rtol=1e-15, atol=0)
    zr = np.nonzero(cost_h == int(np.median(cost_h)))[0]
    if zr.size > 3:
        z, pr = g.gqaoa_level_probs(n, cost, psi, dt, int(np.median(cost_h)), max_out=3)
        np.testing.assert_array_equal(z, zr[:3])


def test_mlp_angles_match_oracle():
    torch = need_gpu()
    rng = np.random.Generator(np.random.PCG64(510))
    o = (rng.normal(size=(1000, 2)) * 4).astype(np.float32)
    o[0] = [0.0, 0.0]
    o[1] = [40.0, -40.0]
    b, gm = g.gqaoa_mlp_angles(torch.tensor(o, device="cuda"))
    rb, rg = omlp.angles(o.astype(np.float64))
    np.testing.assert_allclose(b.cpu().numpy(), rb, rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(gm.cpu().numpy(), rg, rtol=1e-14, atol=1e-300)


def test_gather_rows_exact():
    torch = need_gpu()
    rng = np.random.Generator(np.random.PCG64(520))
    src = rng.normal(size=(300, 131)).astype(np.float32)
    idx = rng.integers(0, 300, 512).astype(np.int32)
    idx[5] = 300                                          # out of range: a row of zeros
    idx[6] = -1
    out = g.gqaoa_gather_rows(torch.tensor(src, device="cuda"), torch.tensor(idx, device="cuda")).cpu().numpy()
    ok = (idx >= 0) & (idx < 300)
    np.testing.assert_array_equal(out[ok], src[idx[ok]])
    assert not out[~ok].any()
