"""Pins of the oracle's gradients of L = sum_m w_m . u(x_m) against central finite
differences of the oracle's own sums (no gradient formula is retyped here)."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, se


def _loss_direct(kernel, x, f, w):
    return float(np.sum(w * direct.direct(kernel, x, f)))


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_direct_gradient_vs_finite_differences(kernel):
    x = W.uniform_cube(40, 70)
    f = W.normal_strengths(40, 71)
    w = W.normal_strengths(40, 72)
    tg = np.array([0, 7, 39])
    g = direct.grad_direct(kernel, x, f, w, targets=tg)
    h = 1e-5
    for i, p in enumerate(tg):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[p, k] += h
            xm[p, k] -= h
            fd = (_loss_direct(kernel, xp, f, w) - _loss_direct(kernel, xm, f, w)) / (2 * h)
            assert abs(fd - g[i, k]) <= 1e-6 * max(1.0, abs(fd)), (p, k, fd, g[i, k])


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_real_part_gradient_vs_finite_differences(kernel):
    x = W.uniform_cube(60, 73)
    f = W.normal_strengths(60, 74)
    w = W.normal_strengths(60, 75)
    xi, rc = 5.0, 0.45
    tg = np.array([3, 30])
    g = direct.grad_real_trunc(kernel, xi, rc, x, f, w, targets=tg)
    loss = lambda xx: float(np.sum(w * direct.real_trunc(kernel, xi, rc, xx, f)))
    h = 1e-6
    for i, p in enumerate(tg):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[p, k] += h
            xm[p, k] -= h
            fd = (loss(xp) - loss(xm)) / (2 * h)
            assert abs(fd - g[i, k]) <= 1e-5 * max(1.0, abs(fd)), (p, k, fd, g[i, k])


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_fse_gradient_vs_finite_differences(kernel):
    """dL/dx of the discrete FSE operator (Gaussian windows fixed: steps stay
    inside one grid cell so no window moves)."""
    x = W.uniform_cube(50, 76)
    f = W.normal_strengths(50, 77)
    w = W.normal_strengths(50, 78)
    g = se.geometry(xi=6.0, rc=0.5, M=20, P=12, L=1.0)
    Kt = se.mollified_kernel(se.kernel_family(kernel), g)
    grad = se.grad_x(kernel, x, f, w, g, Kt)
    loss = lambda xx: float(np.sum(w * se.evaluate(kernel, xx, f, g=g, Kt=Kt)["u"]))
    h = 1e-6
    for p in (2, 41):
        t, b = se.window(x[p:p + 1], g)
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[p, k] += h
            xm[p, k] -= h
            for xx in (xp, xm):
                assert np.all(se.window(xx[p:p + 1], g)[1] == b)
            fd = (loss(xp) - loss(xm)) / (2 * h)
            assert abs(fd - grad[p, k]) <= 2e-5 * max(1.0, abs(fd)), (p, k, fd, grad[p, k])


def test_fse_gradient_close_to_exact_gradient():
    """The FSE gradient approximates the exact one (parity within truncation)."""
    x = W.uniform_cube(200, 79)
    f = W.normal_strengths(200, 80)
    w = W.normal_strengths(200, 81)
    g = se.geometry(xi=6.0, rc=1.1, M=30, P=20, L=1.0)
    ga = se.grad_x("stokeslet", x, f, w, g)
    ge = direct.grad_direct("stokeslet", x, f, w)
    assert direct.rel_errors(ga, ge)[1] < 1e-5


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_fse_operator_symmetric(kernel):
    """w . K_FSE f = f . K_FSE w: so dL/df = K_FSE w (the adjoint reuses the forward)."""
    x = W.uniform_cube(80, 82)
    f = W.normal_strengths(80, 83)
    w = W.normal_strengths(80, 84)
    g = se.geometry(xi=6.0, rc=0.5, M=20, P=12, L=1.0)
    Kt = se.mollified_kernel(se.kernel_family(kernel), g)
    a = np.sum(w * se.evaluate(kernel, x, f, g=g, Kt=Kt)["u"])
    b = np.sum(f * se.evaluate(kernel, x, w, g=g, Kt=Kt)["u"])
    assert abs(a - b) <= 1e-12 * abs(a)
