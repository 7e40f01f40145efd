"""GPU parity: the HIP path (through the C ABI) against the oracle, element by element.

Tolerances (relative to the largest component of the reference, the max-norm
of the Results section's "relative error" reading):
  FP64: the HIP path and the oracle run the same steps (same windows, same
        mollified kernel, same multipliers); only summation order and the FFT
        algorithm differ, so they agree to ~1e-13; 1e-10 is asserted.
  FP32: unit roundoff 6e-8; the spread sums ~P^3 terms per node, the FFTs add
        ~log2(n) rounding steps, the quadrature ~P^3 terms; the observed error
        is a few 1e-7; 2e-6 is asserted for the Fourier part and the total,
        5e-6 for the real-space part alone (sums of ~1/r terms with cancellation).
"""
import math

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
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(u - ref).max() / np.abs(ref).max())


def _inputs(kernel, n, seed, L=1.0, lo=(0.0, 0.0, 0.0), positions="uniform", batch=None):
    if positions == "uniform":
        x = W.uniform_cube(n, seed, lo=0.0, L=L) + np.asarray(lo)
    elif positions == "blobs":
        x = np.clip(W.gaussian_blobs(n, seed, nblobs=8, sigma=0.03), 0.0, 1.0 - 1e-9) * L + np.asarray(lo)
    a = W.normal_strengths(n, seed + 1, batch)
    b = W.normal_strengths(n, seed + 2, batch) if kernel == "stresslet" else None
    return x, a, b


def _plan(kernel, dtype, params, n, batch=1):
    return F.Plan(kernel, dtype, params, batch=batch, nmax=n)


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=torch.float32 if dtype == "f32" else torch.float64, device=DEV)


def _oracle_geo(plan, params):
    p = params
    return se.geometry(p.xi, p.rc, p.M, p.P, tuple(p.box_lo), p.L, Mt=plan.geometry.Mt,
                       deltaL_rule=p.deltaL_rule)


def _as64(x, dtype):
    """The FP32 form evaluates the FP32-rounded inputs; the oracle gets those exactly."""
    if x is None:
        return None
    return np.asarray(x, dtype=np.float32).astype(np.float64) if dtype == "f32" else np.asarray(x)


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("Mt", [0, 28, 30, 35])
def test_multiplier_matches_mollified_kernel(kernel, Mt):
    """The precomputed scalar multiplier = eq. gridfcnsc factor x eqs. AS/AT/AR scalar x
    the mollified kernel of Section 4.3 (oracle: literal IFFT/crop/FFT) x normalisations."""
    params = F.make_params(6.0, 0.4, 16, 8, L=1.0, Mt=Mt)
    plan = _plan(kernel, "f64", params, 16)
    sig = plan.multiplier()
    g = _oracle_geo(plan, params)
    Kt = se.mollified_kernel(se.kernel_family(kernel), g)
    Mp = g.Mt + 1
    oct_ = Kt[:Mp, :Mp, :Mp]
    kb = np.arange(Mp)
    k2 = (math.pi / g.Lt) ** 2 * (kb[:, None, None] ** 2 + kb[None, :, None] ** 2 + kb[None, None, :] ** 2)
    E = np.exp(-(1 - g.eta) * k2 / (4 * g.xi ** 2))
    fac = {"stokeslet": -(1 + k2 / (4 * g.xi ** 2)) * E, "stresslet": (1 + k2 / (4 * g.xi ** 2)) * E,
           "rotlet": E}[kernel]
    norm = (g.alpha / math.pi) ** 3 * g.h ** 3 / g.n ** 3
    ref = fac * oct_ * norm
    assert relmax(sig, ref) < 1e-11
    plan.close()


def _multiplier_ref(kernel, plan, params):
    g = _oracle_geo(plan, params)
    Kt = se.mollified_kernel(se.kernel_family(kernel), g)
    Mp = g.Mt + 1
    kb = np.arange(Mp)
    k2 = (math.pi / g.Lt) ** 2 * (kb[:, None, None] ** 2 + kb[None, :, None] ** 2 + kb[None, None, :] ** 2)
    E = np.exp(-(1 - g.eta) * k2 / (4 * g.xi ** 2))
    fac = {"stokeslet": -(1 + k2 / (4 * g.xi ** 2)) * E, "stresslet": (1 + k2 / (4 * g.xi ** 2)) * E,
           "rotlet": E}[kernel]
    return fac * Kt[:Mp, :Mp, :Mp] * (g.alpha / math.pi) ** 3 * g.h ** 3 / g.n ** 3


def test_precompute_cache_scales_the_transform():
    """Plans with the grid side and kernel family of an earlier plan reuse its
    mollified transform, scaled for their own grid spacing ((h/h0)^4 biharmonic,
    (h/h0)^2 harmonic): each multiplier still matches the oracle's, computed afresh
    for its own geometry, and the second plan of each family is a cache hit."""
    for fam in (["stokeslet", "stresslet", "stokeslet"], ["rotlet", "rotlet"]):
        for i, (kernel, L) in enumerate(zip(fam, (1.0, 2.5, 0.7))):
            before = F.precompute_cache_stats()
            params = F.make_params(6.0 / L, 0.4 * L, 16, 8, L=L, Mt=27)  # Mt 27: no other test's grid
            plan = _plan(kernel, "f64", params, 16)
            try:
                assert plan.geometry.Mt == 27
                sig = plan.multiplier()
                ref = _multiplier_ref(kernel, plan, params)
            finally:
                plan.close()
            after = F.precompute_cache_stats()
            assert after["hits"] + after["misses"] == before["hits"] + before["misses"] + 1
            if i > 0:
                assert after["hits"] == before["hits"] + 1, (kernel, L)
            e = relmax(sig, ref)
            print(kernel, "L", L, "multiplier error %.1e" % e, after)
            assert e < 1e-11


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_stage_grids(kernel):
    """Stage by stage: the spread grid (step 1) and the scaled inverse-transformed
    grid (steps 2-4) against the oracle's, FP64."""
    n = 700
    params = F.make_params(10.0, 0.32, 24, 10, L=1.0, Mt=35)
    x, a, b = _inputs(kernel, n, 70)
    plan = _plan(kernel, "f64", params, n)
    plan.set_points(_t(x, "f64"))
    plan.eval_parts(_t(a, "f64"), None if b is None else _t(b, "f64"))
    g = _oracle_geo(plan, params)
    src = se.sources_grid(kernel, a, b)
    grid_o = se.spread(x, src, g)  # (c, ix, iy, iz)
    norm = (g.alpha / math.pi) ** 1.5
    G = plan.grid(0)[0]            # (c, z, y, x)
    if kernel == "stresslet":      # symmetric components (00, 11, 22, 01, 02, 12) of n_l q_m
        sym = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
        grid_o = np.array([0.5 * (grid_o[3 * l + m] + grid_o[3 * m + l]) for l, m in sym])
    e1 = relmax(np.transpose(G, (0, 3, 2, 1)) * norm, grid_o)
    Kt = se.mollified_kernel(se.kernel_family(kernel), g)
    field_o = se.fourier_step(kernel, se.spread(x, src, g), g, Kt)
    Phi = plan.grid(1)[0]
    e2 = relmax(np.transpose(Phi, (0, 3, 2, 1)) / (norm * g.h ** 3), field_o)
    print(kernel, "spread err %.2e  field err %.2e" % (e1, e2))
    assert e1 < 1e-12
    assert e2 < 1e-11
    plan.close()


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("M,P,Mt", [(24, 10, 35), (20, 12, 0), (8, 7, 0)])
def test_spread_grid_f32(kernel, M, P, Mt):
    """FP32 spreading (the matrix-core kernel) node by node against the oracle's grid
    of the FP32-rounded inputs: cores cut by the grid edge (Mt not a multiple of 16),
    the headline P, and a grid about one core wide with odd P."""
    n = 900
    # xi = 4 keeps eta < 1 (the FP32 form's bound) for every case; the spread grid
    # itself does not depend on xi (alpha = 2 m^2 / d^2)
    params = F.make_params(4.0, 0.32, M, P, L=1.0, Mt=Mt)
    x, a, b = _inputs(kernel, n, 90)
    plan = _plan(kernel, "f32", params, n)
    plan.set_points(_t(x, "f32"))
    plan.eval_parts(_t(a, "f32"), None if b is None else _t(b, "f32"))
    g = _oracle_geo(plan, params)
    x64, a64, b64 = _as64(x, "f32"), _as64(a, "f32"), _as64(b, "f32")
    grid_o = se.spread(x64, se.sources_grid(kernel, a64, b64), g)
    if kernel == "stresslet":
        sym = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
        grid_o = np.array([0.5 * (grid_o[3 * l + m] + grid_o[3 * m + l]) for l, m in sym])
    norm = (g.alpha / math.pi) ** 1.5
    G = plan.grid(0)[0].astype(np.float64)
    e = relmax(np.transpose(G, (0, 3, 2, 1)) * norm, grid_o)
    print(kernel, "Mt", g.Mt, "P", P, "FP32 spread err %.2e" % e)
    assert e < 2e-6
    plan.close()


CASES = [
    # (n, xi, rc, M, P, Mt, L, lo); eta = xi^2 h^2 P / (C^2 pi) < 0.7 in every case, so
    # the middle factor exp(-(1-eta) k^2/4xi^2) of the Gaussian splitting is a
    # smoothing (eta > 1 turns it into a deconvolution that amplifies FP32 rounding)
    (1500, 10.0, 0.32, 24, 10, 0, 1.0, (0.0, 0.0, 0.0)),    # eta 0.58, radices 7,5,2
    (777, 6.0, 0.6, 20, 13, 42, 1.3, (-0.5, 0.25, 2.0)),    # eta 0.66, odd P, ragged n, radices 7,4,3
    (2048, 10.0, 0.3, 30, 16, 60, 1.0, (0.0, 0.0, 0.0)),    # eta 0.59, padded grid, radices 8,5,3
    (1200, 10.0, 0.32, 24, 10, 64, 1.0, (0.0, 0.0, 0.0)),   # eta 0.58, n = 128: radices 8,8,2 (8,2 fused)
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_parts_parity(kernel, dtype, case):
    n, xi, rc, M, P, Mt, L, lo = CASES[case]
    params = F.make_params(xi, rc, M, P, lo, L, Mt=Mt)
    x, a, b = _inputs(kernel, n, 100 + case, L=L, lo=lo)
    plan = _plan(kernel, dtype, params, n)
    plan.set_points(_t(x, dtype))
    uR, uF = plan.eval_parts(_t(a, dtype), None if b is None else _t(b, dtype))
    uR, uF = uR.cpu().numpy()[0], uF.cpu().numpy()[0]
    g = _oracle_geo(plan, params)
    x64, a64, b64 = _as64(x, dtype), _as64(a, dtype), _as64(b, dtype)
    refF = se.fourier_part(kernel, x64, a64, b64, g)
    refR = direct.real_trunc(kernel, xi, rc, x64, a64, b64) + se.self_term(kernel, xi, a64)
    eF, eR = relmax(uF, refF), relmax(uR, refR)
    print("case", case, kernel, dtype, "Mt", g.Mt, "errF %.2e errR %.2e" % (eF, eR))
    assert eF < TOL[dtype]
    assert eR < TOL_REAL[dtype]
    plan.close()


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_total_against_direct_sum(kernel):
    """fse_eval = u^R + u^F + u^self, and with tight parameters it equals the
    direct sum (the method's truncation errors below 1e-9)."""
    n = 1200
    params = F.make_params(6.0, 0.95, 24, 20, L=1.0, deltaL_rule=1)
    x, a, b = _inputs(kernel, n, 7)
    plan = _plan(kernel, "f64", params, n)
    plan.set_points(_t(x, "f64"))
    u = plan.eval(_t(a, "f64"), None if b is None else _t(b, "f64")).cpu().numpy()[0]
    uR, uF = plan.eval_parts(_t(a, "f64"), None if b is None else _t(b, "f64"))
    np.testing.assert_allclose(u, (uR + uF).cpu().numpy()[0], rtol=0, atol=1e-12 * np.abs(u).max())
    ref = direct.direct(kernel, x, a, b)
    mx, rms = direct.rel_errors(u, ref)
    print(kernel, "vs direct: max %.2e rms %.2e" % (mx, rms))
    assert mx < 1e-9
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_matches_single(dtype):
    n, B = 900, 3
    params = F.make_params(9.0, 0.35, 22, 12, L=1.0)
    x, a, _ = _inputs("rotlet", n, 11, batch=B)
    pb = _plan("rotlet", dtype, params, n, batch=B)
    pb.set_points(_t(x, dtype))
    ub = pb.eval(_t(a, dtype)).cpu().numpy()
    p1 = _plan("rotlet", dtype, params, n)
    p1.set_points(_t(x, dtype))
    for k in range(B):
        u1 = p1.eval(_t(a[k], dtype)).cpu().numpy()[0]
        assert relmax(ub[k], u1) < (1e-13 if dtype == "f64" else 1e-6)
    pb.close()
    p1.close()


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_adjoint_matches_oracle(kernel):
    n = 1000
    params = F.make_params(8.0, 0.4, 20, 12, L=1.0)
    x, f, _ = _inputs(kernel, n, 21)
    w = W.normal_strengths(n, 24)
    plan = _plan(kernel, "f64", params, n)
    plan.set_points(_t(x, "f64"))
    u = plan.eval(_t(f, "f64"))
    df, dx = plan.adjoint(_t(f, "f64"), _t(w, "f64"), recompute=False)
    uw = plan.eval(_t(w, "f64")).cpu().numpy()[0]
    # dL/df = K w (the discrete operator is symmetric)
    assert relmax(df.cpu().numpy()[0], uw) < 1e-12
    g = _oracle_geo(plan, params)
    ref = se.grad_x(kernel, x, f, w, g)
    e = relmax(dx.cpu().numpy(), ref)
    print(kernel, "dL/dx err %.2e" % e)
    assert e < 1e-10
    del u
    plan.close()


def test_adjoint_recompute_flag():
    n = 600
    params = F.make_params(8.0, 0.4, 20, 12, L=1.0)
    x, f, _ = _inputs("stokeslet", n, 31)
    w = W.normal_strengths(n, 32)
    plan = _plan("stokeslet", "f64", params, n)
    plan.set_points(_t(x, "f64"))
    plan.eval(_t(f, "f64"))
    d1 = plan.adjoint(_t(f, "f64"), _t(w, "f64"), recompute=False)[1].cpu().numpy()
    plan.eval(_t(w, "f64"))  # overwrite the cached forward grid
    d2 = plan.adjoint(_t(f, "f64"), _t(w, "f64"), recompute=True)[1].cpu().numpy()
    np.testing.assert_allclose(d2, d1, rtol=0, atol=1e-13 * np.abs(d1).max())
    plan.close()


def test_autograd_function():
    n = 500
    params = F.make_params(8.0, 0.4, 20, 12, L=1.0)
    x, f, _ = _inputs("stokeslet", n, 41)
    w = W.normal_strengths(n, 42)
    plan = _plan("stokeslet", "f64", params, n)
    xt = _t(x, "f64").requires_grad_(True)
    ft = _t(f, "f64").requires_grad_(True)
    u = F.fse_sum(xt, ft, plan)
    (u * _t(w, "f64")).sum().backward()
    g = _oracle_geo(plan, params)
    assert relmax(xt.grad.cpu().numpy(), se.grad_x("stokeslet", x, f, w, g)) < 1e-10
    uw = se.evaluate("stokeslet", x, w, g=g)["u"]
    assert relmax(ft.grad.cpu().numpy(), uw) < 1e-10
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_edge_cases_tiny_and_corners(dtype):
    """n = 2 and 3, points on the box's lower corner and just inside its upper faces."""
    params = F.make_params(5.0, 0.6, 12, 8, (0.0, 0.0, 0.0), 1.0)
    top = 1.0 - 2.0 ** -20
    for x in (np.array([[0.0, 0.0, 0.0], [top, top, top]]),
              np.array([[0.0, 0.5, top], [top, 0.0, 0.5], [0.5, top, 0.0]])):
        n = len(x)
        f = W.normal_strengths(n, 50 + n)
        plan = _plan("stokeslet", dtype, params, 8)
        plan.set_points(_t(x, dtype))
        uR, uF = plan.eval_parts(_t(f, dtype))
        g = _oracle_geo(plan, params)
        x64, f64 = _as64(x, dtype), _as64(f, dtype)
        refF = se.fourier_part("stokeslet", x64, f64, None, g)
        refR = direct.real_trunc("stokeslet", 5.0, 0.6, x64, f64) + se.self_term("stokeslet", 5.0, f64)
        assert relmax(uF.cpu().numpy()[0], refF) < TOL[dtype]
        assert relmax(uR.cpu().numpy()[0], refR) < TOL_REAL[dtype]
        plan.close()


def test_clustered_points():
    n = 3000
    params = F.make_params(14.0, 0.2, 32, 12, L=1.0)
    x, a, _ = _inputs("stokeslet", n, 60, positions="blobs")
    plan = _plan("stokeslet", "f64", params, n)
    plan.set_points(_t(x, "f64"))
    uR, uF = plan.eval_parts(_t(a, "f64"))
    g = _oracle_geo(plan, params)
    assert relmax(uF.cpu().numpy()[0], se.fourier_part("stokeslet", x, a, None, g)) < 1e-10
    refR = direct.real_trunc("stokeslet", 14.0, 0.2, x, a) + se.self_term("stokeslet", 14.0, a)
    assert relmax(uR.cpu().numpy()[0], refR) < 1e-10
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_call_order_sizes_and_plan_reuse(dtype):
    """An evaluation before any set_points is refused (FSE_ESTATE), so is a point
    count outside [2, nmax] (FSE_EINVAL); a plan binned again with fewer points
    gives the same bits as a fresh plan given only those points."""
    from paper_1607_04808_amd import fse as FM
    params = F.make_params(6.0, 0.4, 16, 8, L=1.0)
    nmax = 600
    x, a, _ = _inputs("stokeslet", nmax, 70)
    plan = F.Plan("stokeslet", dtype, params, nmax=nmax, tuned=False)
    fresh = F.Plan("stokeslet", dtype, params, nmax=nmax, tuned=False)
    try:
        buf = _t(np.zeros((nmax, 3)), dtype)
        assert FM.lib().fse_eval(plan._h, buf.data_ptr(), None, buf.data_ptr()) == 6
        for bad in (1, nmax + 1):
            xb = _t(W.uniform_cube(bad, 71), dtype)
            with pytest.raises(F.FseError) as e:
                plan.set_points(xb)
            assert e.value.status == 1
        plan.set_points(_t(x, dtype))
        u_big = plan.eval(_t(a, dtype))
        k = 257
        plan.set_points(_t(x[:k], dtype))
        u_small = plan.eval(_t(a[:k], dtype))
        fresh.set_points(_t(x[:k], dtype))
        u_ref = fresh.eval(_t(a[:k], dtype))
        torch.cuda.synchronize()
        assert u_big.shape == (1, nmax, 3) and u_small.shape == (1, k, 3)
        assert torch.equal(u_small, u_ref)
        # and the smaller sum is the oracle's (the first k points alone)
        g = _oracle_geo(plan, params)
        x64, a64 = _as64(x[:k], dtype), _as64(a[:k], dtype)
        ref = (se.fourier_part("stokeslet", x64, a64, None, g) + direct.real_trunc("stokeslet", 6.0, 0.4, x64, a64)
               + se.self_term("stokeslet", 6.0, a64))
        assert relmax(u_small.cpu().numpy()[0], ref) < TOL[dtype]
    finally:
        plan.close()
        fresh.close()


def test_out_of_box_points_rejected():
    params = F.make_params(5.0, 0.6, 12, 8, (0.0, 0.0, 0.0), 1.0)
    plan = _plan("stokeslet", "f64", params, 8)
    for bad in (1.0, -1e-9, float("nan")):
        x = np.array([[0.1, 0.2, 0.3], [0.5, bad, 0.5]])
        with pytest.raises(F.FseError) as e:
            plan.set_points(_t(x, "f64"))
        assert e.value.status == 2
    # unvalidated: the kernels clamp and still run safely
    plan.set_points(_t(np.array([[0.1, 0.2, 0.3], [0.5, 3.0, 0.5]]), "f64"), validate=False)
    plan.eval(_t(np.ones((2, 3)), "f64"))
    torch.cuda.synchronize()
    plan.close()

