"""Run-to-run reproducibility of the whole evaluation.  Binning orders the points
of a bin or cell by index (a stable sort), and spreading, quadrature and the
real-space pass each sum in an order fixed by that binning and by the launch
shape, with no floating-point atomics anywhere.  A second set_points on the same
plan, and a fresh plan with the same parameters, must therefore give the same
bits as the first evaluation, for the forward sums and the adjoints alike (the
fused stokeslet and rotlet call; the stresslet sum and its adjoint).  The
points include a dense cluster, so that a few bins and cells hold thousands of
points and the real-space hit queues flush many times per target."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1607_04808_amd as F  # noqa: E402

DEV = "cuda:0"

# the 100k-point configurations of the paper's timing study, one per precision
PRM = {"f32": (40.0, 0.0945, 124, 12), "f64": (40.0, 0.1215, 153, 20)}


def _points(n, seed):
    x = W.uniform_cube(n, seed)
    r = W.rng(seed + 1)
    k = n // 16
    x[:k] = 0.4 + 0.02 * r.random((k, 3))  # 6250 points within one to eight real-space cells
    return x


def _run(plan, kernel, xt, a, b, w):
    plan.set_points(xt)
    if kernel == "stresslet":
        return (plan.eval(a, b),) + plan.adjoint_stresslet(a, b, w)
    return plan.eval_with_adjoint(a, w)


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet", "stresslet"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_repeated_evaluations_are_bit_identical(kernel, dtype):
    n = 100_000
    td = torch.float32 if dtype == "f32" else torch.float64
    t = lambda v: torch.tensor(np.asarray(v), dtype=td, device=DEV)
    x = _points(n, 450)
    a = W.normal_strengths(n, 451)
    b = None
    if kernel == "stresslet":
        nv = W.normal_strengths(n, 452)
        b = t(nv / np.linalg.norm(nv, axis=1, keepdims=True))
    w = t(W.normal_strengths(n, 453))
    xt, at = t(x), t(a)
    prm = F.make_params(*PRM[dtype], L=1.0)
    plans = [F.Plan(kernel, dtype, prm, nmax=n, tuned=False) for _ in range(2)]
    try:
        first = [o.clone() for o in _run(plans[0], kernel, xt, at, b, w)]
        again = _run(plans[0], kernel, xt, at, b, w)      # same plan, binned again
        fresh = _run(plans[1], kernel, xt, at, b, w)      # new plan and workspace
        torch.cuda.synchronize()
        for o0, o1, o2 in zip(first, again, fresh):
            assert torch.isfinite(o0).all()
            assert torch.equal(o0, o1), "same plan: results differ between runs"
            assert torch.equal(o0, o2), "fresh plan: results differ from the first plan's"
    finally:
        for p in plans:
            p.close()
