"""The paper's error figures, reproduced on synthetic data with the GPU path and
the oracle's exact parts, and checked against the estimates they illustrate:

* Fig. fourier_err (Section 7.1): RMS of the relative Fourier-space truncation
  error against Table est_fourier; N = 1e4 random points in a cube of side
  L = 3, xi = 3.49, P = 32, M = 2 .. 50.
* Fig. real_err (Section 7.2): RMS of the relative real-space truncation error
  against Table est_real; N = 2000, L = 3, xi = 4.67, r_c in (0, L/2].
* Fig. P_errors (Section 5.3): the Fourier part's error for several P with the
  box extended by eq. deltaL_cond and by deltaL = d; 1000 sources in the unit
  cube, xi = 2 pi, Mt = 2 .. 40.

"Relative" is relative to the RMS of the part itself, as in the paper's plots.
Set FSE_FIGURE_DIR to write the curves as JSON there.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import direct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1607_04808_amd as F  # noqa: E402

DEV = "cuda:0"


def _dump(name, data):
    d = os.environ.get("FSE_FIGURE_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, name + ".json"), "w") as fh:
            json.dump(data, fh, indent=1)


def _rms(a):
    return float(np.sqrt(np.sum(np.asarray(a) ** 2) / len(a)))


def _parts(kernel, x, a, b, prm):
    plan = F.Plan(kernel, "f64", prm, nmax=len(x))
    try:
        plan.set_points(torch.tensor(x, device=DEV))
        uR, uF = plan.eval_parts(torch.tensor(a, device=DEV), None if b is None else torch.tensor(b, device=DEV))
        return uR.cpu().numpy()[0], uF.cpu().numpy()[0], plan.geometry
    finally:
        plan.close()


def _src(kernel, n, seed):
    a = W.uniform_strengths(n, seed)
    b = W.uniform_strengths(n, seed + 1) if kernel == "stresslet" else None
    Q = float(np.sum(a * a)) if b is None else float(np.sum(np.sum(a * a, 1) * np.sum(b * b, 1)))
    return a, b, Q


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_fig_fourier_err(kernel):
    N, L, xi, P = 10_000, 3.0, 3.49, 32
    x = W.uniform_cube(N, 900, L=L)
    a, b, Q = _src(kernel, N, 901)
    ref = direct.fourier_dir(kernel, xi, x, a, b)
    scale = _rms(ref)
    rows = []
    for M in range(2, 51, 4):
        prm = F.make_params(xi, 1.0, M, P, L=L, deltaL_rule=1)
        _, uF, g = _parts(kernel, x, a, b, prm)
        meas = _rms(uF - ref) / scale
        est = F.error_estimates(kernel, prm, Q)[1] / scale
        rows.append(dict(M=M, Mt=g.Mt, kinf=g.kinf, measured=meas, estimate=est))
        print(kernel, "M %2d Mt %3d measured %.2e estimate %.2e" % (M, g.Mt, meas, est))
    _dump("fourier_err_" + kernel, rows)
    # where the estimate is meaningful (the Gaussian factor has set in, above
    # roundoff), it tracks the measurement within a factor of 10 and the errors
    # fall by at least 8 decades over the sweep
    used = [r for r in rows if 1e-13 < r["estimate"] < 1e-1]
    assert len(used) >= 4
    assert all(0.05 < r["measured"] / r["estimate"] < 10 for r in used), used
    assert rows[0]["measured"] / min(r["measured"] for r in rows) > 1e8


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_fig_real_err(kernel):
    N, L, xi = 2000, 3.0, 4.67
    x = W.uniform_cube(N, 910, L=L)
    a, b, Q = _src(kernel, N, 911)
    full = direct.real_trunc(kernel, xi, 10.0, x, a, b)
    scale = _rms(full)
    rows = []
    for rc in (0.2, 0.35, 0.5, 0.65, 0.8, 1.0, 1.25, 1.5):
        prm = F.make_params(xi, rc, 30, 12, L=L)
        uR, _, _ = _parts(kernel, x, a, b, prm)
        if kernel == "stokeslet":  # the real part of fse_eval_parts carries the self term
            uR = uR + 4.0 * xi / math.sqrt(math.pi) * a
        meas = _rms(uR - full) / scale
        est = F.error_estimates(kernel, prm, Q)[0] / scale
        rows.append(dict(rc=rc, measured=meas, estimate=est))
        print(kernel, "rc %.2f measured %.2e estimate %.2e" % (rc, meas, est))
    _dump("real_err_" + kernel, rows)
    used = [r for r in rows if 1e-13 < r["estimate"] < 1e-1]
    assert len(used) >= 4
    # the free-space box leaves targets near the faces fewer neighbours beyond r_c
    # than the estimate's unbounded medium, so the measurement sits at or below it
    assert all(0.1 < r["measured"] / r["estimate"] < 2.0 for r in used), used


def test_fig_P_errors():
    """Stokeslet Fourier part, 1000 sources in the unit cube, xi = 2 pi, total grid Mt
    from 24 to 72: with eq. deltaL_cond's extension the error keeps falling with Mt
    to the floor that P sets (about 2.5 digits per 4 points of P), while deltaL = d
    leaves the remainder Gaussians cut at the box edge and the error grows once Mt
    exceeds what the tolerance needs (Section 5.3)."""
    N, xi = 1000, 2.0 * math.pi
    x = W.uniform_cube(N, 920)
    a, _, _ = _src("stokeslet", N, 921)
    ref = direct.fourier_dir("stokeslet", xi, x, a)
    scale = _rms(ref)
    rows = []
    err = {}
    for P in (8, 12, 16):
        for rule in (1, 0):
            for Mt in range(24, 73, 8):
                # the M whose extended grid first reaches Mt nodes
                M = next(m for m in range(1, Mt) if F.geometry("stokeslet", F.make_params(
                    xi, 0.5, m, P, L=1.0, deltaL_rule=rule)).Mt >= Mt)
                prm = F.make_params(xi, 0.5, M, P, L=1.0, deltaL_rule=rule)
                _, uF, g = _parts("stokeslet", x, a, None, prm)
                e = _rms(uF - ref) / scale
                err[(P, rule, Mt)] = e
                rows.append(dict(P=P, rule=rule, M=M, Mt=g.Mt, error=e))
                print("P %2d rule %d M %2d Mt %2d error %.2e" % (P, rule, M, g.Mt, e))
    _dump("P_errors", rows)
    for P in (8, 12, 16):
        assert err[(P, 1, 72)] <= 1.1 * err[(P, 1, 40)]          # no growth with eq. deltaL_cond
        assert err[(P, 0, 72)] > 100 * err[(P, 1, 72)]           # deltaL = d with an oversized grid
    assert err[(8, 1, 72)] > 30 * err[(12, 1, 72)] > 30 * 30 * err[(16, 1, 72)]
