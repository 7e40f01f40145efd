"""Separate targets (fse_set_targets / fse_eval_targets; Section 2: sums at the
sources or at any other points) against the oracle, element by element.

u^R at the targets against the oracle's truncated real-space sum there, u^F
against the oracle's FSE field gathered at the targets (same windows and
multiplier: FP64 to 1e-10), and the total against the direct sum at the
targets within the method's truncation."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, se

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1607_04808_amd as F  # noqa: E402

DEV = "cuda:0"
TOL = {"f64": 1e-10, "f32": 2e-6}
TOL_REAL = {"f64": 1e-10, "f32": 5e-6}


def relmax(u, ref):
    return float(np.abs(np.asarray(u, np.float64) - ref).max() / np.abs(ref).max())


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=torch.float32 if dtype == "f32" else torch.float64, device=DEV)


def _as64(a, dtype):
    if a is None:
        return None
    return np.asarray(a, dtype=np.float32).astype(np.float64) if dtype == "f32" else np.asarray(a)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("n,nt,batch", [(1500, 999, 1), (700, 2100, 2)])
def test_targets_parts_match_oracle(kernel, dtype, n, nt, batch):
    xi, rc, M, P = 9.0, 0.35, 22, 12
    prm = F.make_params(xi, rc, M, P, L=1.0)
    x = W.uniform_cube(n, 501)
    y = W.uniform_cube(nt, 502)  # free targets, none on a source
    nb = None if batch == 1 else batch
    a = W.normal_strengths(n, 503, nb)
    b = W.normal_strengths(n, 504, nb) if kernel == "stresslet" else None
    plan = F.Plan(kernel, dtype, prm, batch=batch, nmax=n)
    try:
        plan.set_points(_t(x, dtype))
        plan.set_targets(_t(y, dtype))
        uR, uF = plan.eval_targets(_t(a, dtype), None if b is None else _t(b, dtype), parts=True)
        u = plan.eval_targets(_t(a, dtype), None if b is None else _t(b, dtype))
        uR, uF, u = (v.cpu().numpy().reshape(batch, nt, 3) for v in (uR, uF, u))
        g = se.geometry(xi, rc, M, P, L=1.0, Mt=plan.geometry.Mt)
    finally:
        plan.close()
    x64, y64 = _as64(x, dtype), _as64(y, dtype)
    for bm in range(batch):
        ab = _as64(a if batch == 1 else a[bm], dtype)
        bb = None if b is None else _as64(b if batch == 1 else b[bm], dtype)
        refR = direct.real_trunc(kernel, xi, rc, x64, ab, bb, y=y64)
        _, field = se.fourier_part(kernel, x64, ab, bb, g, return_field=True)
        refF = se.gather(field, y64, g)
        eR, eF = relmax(uR[bm], refR), relmax(uF[bm], refF)
        eT = relmax(u[bm], refR + refF)
        print(kernel, dtype, n, nt, bm, "real %.1e fourier %.1e total %.1e" % (eR, eF, eT))
        assert eR < TOL_REAL[dtype] and eF < TOL[dtype] and eT < TOL[dtype]
        if bm == 0:
            ed = direct.rel_errors(u[bm], direct.direct(kernel, x64, ab, bb, y=y64))[0]
            assert ed < 1e-4, ed  # the method's truncation at these parameters


def test_targets_equal_sources_reduce_to_eval():
    """Targets at the source positions (stresslet and rotlet: no self term, and the
    coincident pair is skipped, exactly as fse_eval excludes n = m)."""
    n = 1200
    prm = F.make_params(9.0, 0.35, 22, 12, L=1.0)
    x = W.uniform_cube(n, 511)
    a = W.normal_strengths(n, 512)
    b = W.normal_strengths(n, 513)
    for kernel in ("rotlet", "stresslet"):
        plan = F.Plan(kernel, "f64", prm, nmax=n)
        try:
            plan.set_points(_t(x, "f64"))
            plan.set_targets(_t(x[::-1].copy(), "f64"))
            bb = _t(b, "f64") if kernel == "stresslet" else None
            ut = plan.eval_targets(_t(a, "f64"), bb).cpu().numpy()[0][::-1]
            u = plan.eval(_t(a, "f64"), bb).cpu().numpy()[0]
        finally:
            plan.close()
        assert relmax(ut, u) < 1e-12


def test_targets_outside_box_rejected():
    prm = F.make_params(9.0, 0.35, 22, 12, L=1.0)
    plan = F.Plan("stokeslet", "f64", prm, nmax=100)
    try:
        plan.set_points(_t(W.uniform_cube(100, 1), "f64"))
        with pytest.raises(F.FseError):
            plan.set_targets(_t(np.array([[0.5, 0.5, 1.5]]), "f64"))
    finally:
        plan.close()
