"""Stresslet adjoint (fse_eval_adjoint_stresslet): dL/dq and dL/dn of
L = sum_m w_m . u(x_m) by the transposed chain.

1. Transpose identity of the discrete operator: u is linear in q and in n, so
   sum dL/dq . dq' = w . u(dq', n) and sum dL/dn . dn' = w . u(q, dn') with u from
   fse_eval on the same plan (FP64 to rounding).
2. Against the oracle's adjoint of the direct sum (eq. def_stresslet), within the
   method's truncation, at sampled points; FP32 and FP64.
"""
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


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=torch.float32 if dtype == "f32" else torch.float64, device=DEV)


def _as64(a, dtype):
    return np.asarray(a, dtype=np.float32).astype(np.float64) if dtype == "f32" else np.asarray(a)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
@pytest.mark.parametrize("batch", [1, 2])
def test_stresslet_adjoint_transpose_identity(dtype, tol, batch):
    n = 3000
    prm = F.make_params(9.0, 0.35, 22, 12, L=1.0)
    x = W.uniform_cube(n, 601)
    q, nn, w, dq1, dn1 = (W.normal_strengths(n, 602 + k, batch) for k in range(5))
    plan = F.Plan("stresslet", dtype, prm, batch=batch, nmax=n)
    try:
        plan.set_points(_t(x, dtype))
        dq, dn = plan.adjoint_stresslet(_t(q, dtype), _t(nn, dtype), _t(w, dtype))
        uq = plan.eval(_t(dq1, dtype), _t(nn, dtype))
        un = plan.eval(_t(q, dtype), _t(dn1, dtype))
        dq, dn, uq, un = (v.cpu().numpy().astype(np.float64).reshape(batch, n, 3) for v in (dq, dn, uq, un))
    finally:
        plan.close()
    wv = np.asarray(w, np.float64).reshape(batch, n, 3)
    for bm in range(batch):
        lhs_q = np.sum(dq[bm] * np.reshape(dq1, (batch, n, 3))[bm])
        rhs_q = np.sum(wv[bm] * uq[bm])
        lhs_n = np.sum(dn[bm] * np.reshape(dn1, (batch, n, 3))[bm])
        rhs_n = np.sum(wv[bm] * un[bm])
        scale_q = np.linalg.norm(dq[bm]) * np.linalg.norm(dq1)
        scale_n = np.linalg.norm(dn[bm]) * np.linalg.norm(dn1)
        print(dtype, batch, bm, "q %.2e n %.2e" % (abs(lhs_q - rhs_q) / scale_q, abs(lhs_n - rhs_n) / scale_n))
        assert abs(lhs_q - rhs_q) < tol * scale_q
        assert abs(lhs_n - rhs_n) < tol * scale_n


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-8), ("f32", 1e-6)])
def test_stresslet_adjoint_matches_oracle(dtype, tol):
    n = 20_000
    x = W.uniform_cube(n, 611, L=2.0) - 1.0
    q, nn, w = (W.normal_strengths(n, 612 + k) for k in range(3))
    xt, qt, nt, wt = (_t(a, dtype) for a in (x, q, nn, w))
    qt.requires_grad_(True)
    nt.requires_grad_(True)
    u = F.stresslet(xt, qt, nt, tol=tol)
    (u * wt).sum().backward()
    tg = np.sort(W.rng(613).choice(n, size=200, replace=False))
    xs, qs, ns, ws = (_as64(a, dtype) for a in (x, q, nn, w))
    rq, rn = direct.stresslet_adjoint(xs, qs, ns, ws, targets=tg)
    eq = direct.rel_errors(qt.grad.cpu().numpy()[tg], rq)[0]
    en = direct.rel_errors(nt.grad.cpu().numpy()[tg], rn)[0]
    print(dtype, "dL/dq %.2e dL/dn %.2e" % (eq, en))
    # the parameters hold u at `tol`; the adjoint's relative error runs about twice
    # the forward's (measured: FP64 1.8e-8 / 2.5e-8 at the 1e-8 parameters, FP32
    # 8.1e-7 / 7.0e-7 at 1e-6)
    assert eq < 3 * tol and en < 3 * tol
