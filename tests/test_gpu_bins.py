"""The binning (index work) of fse_set_points, bit for bit: window starts and
window-centre offsets against the oracle's se.window (Section 5.1's support of
eq. Hx, FP64), the spread and real-space orders against a plain stable counting
sort of the bin and cell keys, and the bin and cell offsets against the key
counts.  Points include the box corners and faces, a dense cluster (many
points per bin) and exact duplicates (ties keep input order)."""
import numpy as np
import pytest

import workloads as W
from oracle import se

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1607_04808_amd as F  # noqa: E402

DEV = "cuda:0"


def _points(n, seed, L):
    x = W.uniform_cube(n, seed, L=L)
    r = W.rng(seed + 1)
    k = n // 8
    x[:k] = 0.3 * L + 0.01 * L * r.random((k, 3))           # a cluster
    x[k:k + 8] = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], float) * L * (1 - 1e-12)
    x[k + 8:k + 16] = x[k + 16:k + 24]                      # duplicates
    x[k + 24:k + 30, 0] = 0.0                               # on a face
    return x


def _expected(x, prm_geo, nbins, TS, ncell, cell, lo, dtype):
    g = prm_geo
    t, b = se.window(x, g)
    coff = t - b - 0.5 * (g.P - 1)
    if dtype == "f32":
        coff = coff.astype(np.float32).astype(np.float64)
    tb = b // TS
    key_s = (tb[:, 2] * nbins + tb[:, 1]) * nbins + tb[:, 0]
    c = np.clip(np.floor((x - np.asarray(lo)) / cell), 0, ncell - 1).astype(np.int64)
    key_r = (c[:, 2] * ncell + c[:, 1]) * ncell + c[:, 0]
    perm_s = np.argsort(key_s, kind="stable")
    perm_r = np.argsort(key_r, kind="stable")
    tile_start = np.concatenate([[0], np.cumsum(np.bincount(key_s, minlength=nbins ** 3))])
    cell_start = np.concatenate([[0], np.cumsum(np.bincount(key_r, minlength=ncell ** 3))])
    bpack = b[:, 0] | (b[:, 1] << 10) | (b[:, 2] << 20)
    return dict(perm_s=perm_s, bpack_s=bpack[perm_s], coff_s=coff[perm_s], tile_start=tile_start,
                perm_r=perm_r, cell_start=cell_start)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bin_side", [7, 5])
def test_bins_match_counting_sort(dtype, bin_side):
    n, L = 20_000, 2.0
    xi, rc, M, P = 10.0, 0.3, 60, 12
    x = _points(n, 420, L)
    if dtype == "f32":
        x = np.minimum(x.astype(np.float32).astype(np.float64), np.nextafter(L, 0))
    lo = (-0.5, 0.25, 0.0)
    x = x + np.asarray(lo)
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    Lbox = L * (1 + 2.0 ** -20)
    prm = F.make_params(xi, rc, M, P, box_lo=lo, L=Lbox)
    # the library takes the smallest Mt whose 2 Mt factors into 2, 3, 5, 7
    g = se.geometry(xi, rc, M, P, box_lo=lo, L=Lbox, Mt=F.geometry("stokeslet", prm).Mt)
    plan = F.Plan("stokeslet", dtype, prm, nmax=n, tuned=False)
    try:
        plan.set_tuning({"bin_side": bin_side})
        xt = torch.tensor(x, dtype=torch.float32 if dtype == "f32" else torch.float64, device=DEV)
        plan.set_points(xt)
        got = plan.bins()
        assert plan.geometry.Mt == g.Mt
        ncell = plan.geometry.ncell
        nbins = got["nbins"]
        assert nbins == -(-g.Mt // bin_side)
        exp = _expected(x, g, nbins, bin_side, ncell, Lbox / ncell, lo, dtype)
        for k in ("perm_s", "bpack_s", "tile_start", "perm_r", "cell_start"):
            assert np.array_equal(got[k], exp[k]), k
        assert np.array_equal(got["coff_s"], exp["coff_s"])
        # the same points again give the same order (no run-to-run change)
        plan.set_points(xt)
        again = plan.bins()
        assert all(np.array_equal(again[k], got[k]) for k in ("perm_s", "perm_r"))
    finally:
        plan.close()
