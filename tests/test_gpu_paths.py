"""Parity on every code path the ABI admits, element by element against the oracle:

* Gaussian supports that select each quadrature kernel: P = 8 (the generic
  row walk), P = 11 and 18 (the headline forms' widths, whose x-sums run 11
  and 18 terms), P = 24 and 28 in FP64 (the column kernel's widest ring, then
  the block and global-memory kernels), P = 32 in both precisions;
* FFT sizes whose stages run fused in FP32: n = 50 (5 5 | 2) and n = 60 (5 4 | 3);
* the batched adjoint against single adjoints;
* the FP32 adjoints (stokeslet and rotlet) against the oracle's discrete gradient.
"""
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


def _geo(plan, p):
    return se.geometry(p.xi, p.rc, p.M, p.P, tuple(p.box_lo), p.L, Mt=plan.geometry.Mt, deltaL_rule=p.deltaL_rule)


# (P, xi, M, Mt, dtypes): eta < 0.7 in every case
PCASES = [
    (8, 10.0, 20, 0, ("f64", "f32")),
    (11, 8.5, 20, 0, ("f64", "f32")),   # odd P, the FP32 headline's (FP32: 11-term x-sums)
    (18, 6.5, 20, 0, ("f64",)),         # the FP64 headline's P (18-term x-sums)
    (24, 5.5, 20, 0, ("f64", "f32")),
    (28, 5.0, 20, 0, ("f64",)),
    (32, 4.0, 20, 54, ("f64", "f32")),
]


@pytest.mark.parametrize("case", range(len(PCASES)))
@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet"])
def test_parts_parity_across_P(kernel, case):
    P, xi, M, Mt, dtypes = PCASES[case]
    n = 700
    rc = 3.5 / xi
    prm = F.make_params(xi, rc, M, P, L=1.0, Mt=Mt)
    x = W.uniform_cube(n, 300 + case)
    a = W.normal_strengths(n, 310 + case)
    b = W.normal_strengths(n, 320 + case) if kernel == "stresslet" else None
    for dtype in dtypes:
        plan = F.Plan(kernel, dtype, prm, nmax=n)
        try:
            plan.set_points(_t(x, dtype))
            uR, uF = plan.eval_parts(_t(a, dtype), None if b is None else _t(b, dtype))
            g = _geo(plan, prm)
        finally:
            plan.close()
        x64, a64, b64 = _as64(x, dtype), _as64(a, dtype), _as64(b, dtype)
        refF = se.fourier_part(kernel, x64, a64, b64, g)
        refR = direct.real_trunc(kernel, xi, rc, x64, a64, b64) + se.self_term(kernel, xi, a64)
        eF, eR = relmax(uF.cpu().numpy()[0], refF), relmax(uR.cpu().numpy()[0], refR)
        print(kernel, dtype, "P", P, "Mt", g.Mt, "errF %.2e errR %.2e" % (eF, eR))
        assert eF < TOL[dtype] and eR < TOL_REAL[dtype]


@pytest.mark.parametrize("case", range(len(PCASES)))
def test_adjoint_across_P(case):
    """dL/dx (window derivatives in spreading and quadrature, every quadrature path)
    against the oracle's discrete gradient, FP64."""
    P, xi, M, Mt, _ = PCASES[case]
    n = 500
    prm = F.make_params(xi, 3.5 / xi, M, P, L=1.0, Mt=Mt)
    x = W.uniform_cube(n, 330 + case)
    f = W.normal_strengths(n, 340 + case)
    w = W.normal_strengths(n, 350 + case)
    plan = F.Plan("stokeslet", "f64", prm, nmax=n)
    try:
        plan.set_points(_t(x, "f64"))
        df, dx = plan.adjoint(_t(f, "f64"), _t(w, "f64"))
        uw = plan.eval(_t(w, "f64")).cpu().numpy()[0]
        g = _geo(plan, prm)
    finally:
        plan.close()
    assert relmax(df.cpu().numpy()[0], uw) < 1e-12
    e = relmax(dx.cpu().numpy(), se.grad_x("stokeslet", x, f, w, g))
    print("P", P, "dL/dx err %.2e" % e)
    assert e < 1e-10


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("Mt", [25, 30])
def test_fused_fft_stages_fp32(kernel, Mt):
    """n = 2 Mt = 50 (radices 5, 5, 2: the 5 x 5 stages fused) and 60 (5, 4, 3: 5 x 4
    fused) in FP32, element by element against the oracle."""
    n = 900
    xi, M, P = 5.0, 16, 8
    prm = F.make_params(xi, 0.6, M, P, L=1.0, Mt=Mt)
    x = W.uniform_cube(n, 360 + Mt)
    a = W.normal_strengths(n, 361 + Mt)
    b = W.normal_strengths(n, 362 + Mt) if kernel == "stresslet" else None
    plan = F.Plan(kernel, "f32", prm, nmax=n)
    try:
        assert plan.geometry.n_fft == 2 * Mt
        plan.set_points(_t(x, "f32"))
        uR, uF = plan.eval_parts(_t(a, "f32"), None if b is None else _t(b, "f32"))
        g = _geo(plan, prm)
    finally:
        plan.close()
    x64, a64, b64 = _as64(x, "f32"), _as64(a, "f32"), _as64(b, "f32")
    eF = relmax(uF.cpu().numpy()[0], se.fourier_part(kernel, x64, a64, b64, g))
    print(kernel, "n", 2 * Mt, "errF %.2e" % eF)
    assert eF < TOL["f32"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_batched_adjoint_matches_single(kernel, dtype):
    """batch = 3: dL/df of each member equals that member's single adjoint, and dL/dx
    is the sum of the members' gradients."""
    n, B = 800, 3
    prm = F.make_params(9.0, 0.35, 22, 12, L=1.0)
    x = W.uniform_cube(n, 370)
    f = W.normal_strengths(n, 371, B)
    w = W.normal_strengths(n, 372, B)
    pb = F.Plan(kernel, dtype, prm, batch=B, nmax=n)
    p1 = F.Plan(kernel, dtype, prm, nmax=n)
    try:
        pb.set_points(_t(x, dtype))
        dfb, dxb = pb.adjoint(_t(f, dtype), _t(w, dtype))
        dfb, dxb = dfb.double().cpu().numpy(), dxb.double().cpu().numpy()
        p1.set_points(_t(x, dtype))
        dx_sum = np.zeros((n, 3))
        for k in range(B):
            df1, dx1 = p1.adjoint(_t(f[k], dtype), _t(w[k], dtype))
            assert relmax(dfb[k], df1.double().cpu().numpy()[0]) < (1e-13 if dtype == "f64" else 1e-6)
            dx_sum += dx1.double().cpu().numpy()
    finally:
        pb.close()
        p1.close()
    e = relmax(dxb, dx_sum)
    print(kernel, dtype, "batched dL/dx vs summed singles %.2e" % e)
    assert e < (1e-12 if dtype == "f64" else 2e-6)


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_fp32_adjoint_matches_oracle(kernel):
    n = 1000
    prm = F.make_params(8.0, 0.4, 20, 12, L=1.0)
    x, f, w = W.uniform_cube(n, 380), W.normal_strengths(n, 381), W.normal_strengths(n, 382)
    plan = F.Plan(kernel, "f32", prm, nmax=n)
    try:
        plan.set_points(_t(x, "f32"))
        df, dx = plan.adjoint(_t(f, "f32"), _t(w, "f32"))
        g = _geo(plan, prm)
    finally:
        plan.close()
    x64, f64, w64 = (_as64(a, "f32") for a in (x, f, w))
    ex = relmax(dx.cpu().numpy(), se.grad_x(kernel, x64, f64, w64, g))
    ef = relmax(df.cpu().numpy()[0], se.evaluate(kernel, x64, w64, g=g)["u"])
    print(kernel, "FP32 dL/dx %.2e dL/df %.2e" % (ex, ef))
    assert ex < 2e-6 and ef < 2e-6


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tuning_changes_shapes_not_results(dtype):
    """Every bin side, queue depth and wave count gives the same sums (FP64 to
    rounding; FP32 within its rounding), and autotune leaves a working plan and
    changes no queue depth whose pass the timed calls do not run."""
    n = 4000
    prm = F.make_params(9.0, 0.35, 22, 12, L=1.0)
    x, f, w = W.uniform_cube(n, 390), W.normal_strengths(n, 391), W.normal_strengths(n, 392)
    plan = F.Plan("stokeslet", dtype, prm, nmax=n, tuned=False)
    try:
        xt, ft, wt = _t(x, dtype), _t(f, dtype), _t(w, dtype)
        plan.set_points(xt)
        u0 = plan.eval(ft).double().cpu().numpy()
        d0 = plan.adjoint(ft, wt)[1].double().cpu().numpy()
        tol = 1e-12 if dtype == "f64" else 2e-6
        for t in ({"bin_side": 5, "real_queue": 24, "real_queue_grad": 32, "real_waves": 1, "fft_lines": 1},
                  {"bin_side": 8, "real_queue": 64, "real_queue_grad": 64, "real_waves": 2, "fft_lines": 4},
                  {"bin_side": 6, "real_queue": 48, "real_queue_grad": 48, "real_waves": 4, "fft_lines": 0}):
            plan.set_tuning(t)
            with pytest.raises(F.FseError):
                plan.eval(ft)  # the points must be set again
            plan.set_points(xt)
            assert plan.tuning() == t
            assert relmax(plan.eval(ft).double().cpu().numpy(), u0) < tol
            assert relmax(plan.adjoint(ft, wt)[1].double().cpu().numpy(), d0) < tol
        # queue depths outside the candidate sets: a knob the timed calls never
        # exercise must keep its value (the fused call runs no value-only pass,
        # and without w no gradient pass runs)
        plan.set_tuning(dict(plan.tuning(), real_queue=40, real_queue_grad=40))
        best = plan.autotune(xt, ft, None, wt, repeats=1)
        assert plan.tuning() == best
        assert best["real_queue"] == 40
        assert relmax(plan.eval(ft).double().cpu().numpy(), u0) < tol
        plan.set_tuning(dict(best, real_queue_grad=40))
        best = plan.autotune(xt, ft, repeats=1)
        assert best["real_queue_grad"] == 40
        assert relmax(plan.eval(ft).double().cpu().numpy(), u0) < tol
        with pytest.raises(F.FseError):
            plan.set_tuning(dict(best, bin_side=3))
        with pytest.raises(F.FseError):
            plan.set_tuning(dict(best, fft_lines=3))
    finally:
        plan.close()


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet", "stresslet"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fft_line_counts_agree(kernel, dtype):
    """Each FFT pass transforms its lines one by one, whatever the number of lines
    a workgroup holds, and the z-pass multiplies each wavevector alike, one column
    or three at a time: every line count (the variants that long lines fall back
    to) gives the default's field to within a few units of rounding."""
    n = 3000
    prm = F.make_params(9.0, 0.35, 22, 12, L=1.0)
    x = W.uniform_cube(n, 395)
    f = W.normal_strengths(n, 396)
    nrm = W.normal_strengths(n, 397) if kernel == "stresslet" else None
    plan = F.Plan(kernel, dtype, prm, nmax=n, tuned=False)
    try:
        xt, ft = _t(x, dtype), _t(f, dtype)
        bt = None if nrm is None else _t(nrm, dtype)
        plan.set_points(xt)
        u0 = plan.eval_parts(ft, bt)[1].double().cpu().numpy()
        worst = 0.0
        for lines in (16, 8, 4, 2, 1):
            plan.set_tuning({"fft_lines": lines})
            plan.set_points(xt)
            u = plan.eval_parts(ft, bt)[1].double().cpu().numpy()
            worst = max(worst, relmax(u, u0))
        print(kernel, dtype, "largest change of u^F over line counts %.1e" % worst)
        assert worst < (1e-14 if dtype == "f64" else 1e-6)
    finally:
        plan.close()
