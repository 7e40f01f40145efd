"""Pins of the oracle's Ewald split: real-space parts G^R (Section 3.2), Fourier
parts G^F, limits and the TR2int closed form (Section 7.2)."""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import direct, se

SQPI = math.sqrt(math.pi)


def _probe_full(kernel, rvec):
    """G(r) as a tensor from the oracle's direct sum (one source, one target)."""
    x = np.array([np.zeros(3), -np.asarray(rvec, float)])
    if kernel == "stresslet":
        T = np.zeros((3, 3, 3))
        for l in range(3):
            for m in range(3):
                nn = np.zeros((2, 3)); q = np.zeros((2, 3))
                nn[1, l] = 1.0; q[1, m] = 1.0
                T[:, l, m] = direct.direct(kernel, x, q, nn, targets=[0])[0]
        return T
    S = np.zeros((3, 3))
    for l in range(3):
        f = np.zeros((2, 3)); f[1, l] = 1.0
        S[:, l] = direct.direct(kernel, x, f, targets=[0])[0]
    return S


def _psi_hasimoto(xi):
    """r - Phi_H(r), Phi_H the Hasimoto splitting function of Table 1."""
    return lambda r: r - (r * math.erf(xi * r) + math.exp(-xi * xi * r * r) / (SQPI * xi))


def _fd_hessian(fun, x, h=2e-3):
    """4th-order central-difference Hessian of a scalar function of a 3-vector."""
    H = np.zeros((3, 3))
    e = np.eye(3)
    c = [(-2, 1 / 12.0), (-1, -8 / 12.0), (1, 8 / 12.0), (2, -1 / 12.0)]
    for j in range(3):
        for l in range(3):
            s = 0.0
            for a, ca in c:
                for b, cb in c:
                    s += ca * cb * fun(x + a * h * e[j] + b * h * e[l])
            H[j, l] = s / (h * h)
    return H


def _fd_grad(fun, x, h=1e-3):
    g = np.zeros(3)
    e = np.eye(3)
    for j in range(3):
        g[j] = (-fun(x + 2 * h * e[j]) + 8 * fun(x + h * e[j]) - 8 * fun(x - h * e[j])
                + fun(x - 2 * h * e[j])) / (12 * h)
    return g


def test_stokeslet_real_part_is_operator_on_hasimoto_split():
    """S^R_jl = (d_jl lap - d_j d_l)(r - Phi_H) (Section 3.2), by finite differences."""
    xi = 3.0
    psi = _psi_hasimoto(xi)
    fun = lambda v: psi(float(np.linalg.norm(v)))
    for rvec in ([0.31, -0.12, 0.2], [0.05, 0.4, -0.33]):
        rvec = np.array(rvec)
        H = _fd_hessian(fun, rvec)
        fd = np.trace(H) * np.eye(3) - H
        SR = se.real_kernel_tensor("stokeslet", xi, rvec)
        np.testing.assert_allclose(SR, fd, rtol=0, atol=2e-7 * np.abs(SR).max())


def test_rotlet_real_part_is_gradient_of_ewald_split():
    """Omega^R_jl = -eps_jlm d_m (erfc(xi r)/r): the eq. def_rotlet normalisation
    applied to the Ewald split of 1/r (eq. laplace_decomp)."""
    xi = 2.5
    phi = lambda v: math.erfc(xi * np.linalg.norm(v)) / np.linalg.norm(v)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1
    for rvec in ([0.3, 0.1, -0.25], [-0.11, 0.07, 0.5]):
        rvec = np.array(rvec)
        g = _fd_grad(phi, rvec)
        fd = -np.einsum("jlm,m->jl", eps, g)
        OR = se.real_kernel_tensor("rotlet", xi, rvec)
        np.testing.assert_allclose(OR, fd, rtol=0, atol=1e-8 * np.abs(OR).max())


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_real_part_recovers_kernel_as_xi_to_zero(kernel):
    rvec = np.array([0.2, -0.35, 0.15])
    G = _probe_full(kernel, rvec)
    GR = se.real_kernel_tensor(kernel, 1e-9, rvec)
    np.testing.assert_allclose(GR, G, rtol=0, atol=1e-8 * np.abs(G).max())


def test_stokeslet_self_limit():
    """lim_{r->0} (S^R - S) = -4 xi/sqrt(pi) I (eq. Slimit)."""
    xi = 4.0
    rvec = np.array([1.0, 2.0, -2.0]) / 3.0 * 1e-6
    D = se.real_kernel_tensor("stokeslet", xi, rvec) - _probe_full("stokeslet", rvec)
    np.testing.assert_allclose(D, -4 * xi / SQPI * np.eye(3), rtol=0, atol=1e-6)


def test_stresslet_tr2int_closed_form():
    """int_{r>rc} (1/9)(A1^2 + 6 A1 A2 + 15 A2^2) 4 pi r^2 dr equals eq. TR2int.

    A1, A2 are read off the oracle's T^R at r = (r,0,0): T_xxx = A1 + 3 A2,
    T_xyy = A2.  Holds only with A2 = 4 xi^3 r e^{-xi^2 r^2}/sqrt(pi).
    """
    for xi, rc in ((4.67, 0.8), (3.0, 0.5)):
        def integrand(r):
            T = se.real_kernel_tensor("stresslet", xi, [r, 0.0, 0.0])
            A2 = T[0, 1, 1]
            A1 = T[0, 0, 0] - 3 * A2
            return (A1 * A1 + 6 * A1 * A2 + 15 * A2 * A2) / 9.0 * 4 * math.pi * r * r
        val, _ = integrate.quad(integrand, rc, rc + 12.0 / xi, epsabs=0, epsrel=1e-11, limit=200)
        e1, e2 = math.exp(-xi * xi * rc * rc), math.erfc(xi * rc)
        closed = (-32.0 / 3.0 * SQPI * xi * e1 * e2 + 21 * math.sqrt(2 * math.pi) * xi
                  * math.erfc(math.sqrt(2) * xi * rc) + 16 * math.pi * e2 * e2 / rc
                  + 4.0 / 9.0 * xi * xi * rc * math.exp(-2 * xi * xi * rc * rc) * (28 * xi * xi * rc * rc - 3))
        assert abs(val - closed) <= 1e-9 * abs(closed)


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_real_plus_fourier_is_full(kernel):
    """G^R + G^F = G pointwise; with n = m the Fourier part carries the self value."""
    x = W.uniform_cube(60, 30)
    a = W.normal_strengths(60, 31)
    b = W.normal_strengths(60, 32) if kernel == "stresslet" else None
    xi = 3.5
    uR = direct.real_trunc(kernel, xi, 10.0, x, a, b)
    uF = direct.fourier_dir(kernel, xi, x, a, b)
    us = se.self_term(kernel, xi, a)
    u = direct.direct(kernel, x, a, b)
    np.testing.assert_allclose(uR + uF + us, u, rtol=0, atol=1e-12 * np.abs(u).max())


def test_fourier_part_limits():
    """G^F(0) = 4 xi/sqrt(pi) I for S, 0 for T and Omega (eq. Slimit; oddness)."""
    xi = 2.0
    x = np.zeros((1, 3))
    f = np.array([[1.0, -2.0, 0.5]])
    np.testing.assert_allclose(direct.fourier_dir("stokeslet", xi, x, f), 4 * xi / SQPI * f, rtol=1e-15)
    assert np.all(direct.fourier_dir("rotlet", xi, x, f) == 0)
    assert np.all(direct.fourier_dir("stresslet", xi, x, f, f) == 0)
    # continuity at small r
    x2 = np.array([[0, 0, 0], [1e-7, 0, 0]])
    f2 = np.array([[0, 0, 0], [1.0, -2.0, 0.5]])
    u = direct.fourier_dir("stokeslet", xi, x2, f2, targets=[0])
    np.testing.assert_allclose(u[0], 4 * xi / SQPI * f2[1], rtol=1e-9)


def test_truncated_kernel_transforms():
    """Bhat^R(0) = pi R^4, Hhat^R(0) = 2 pi R^2 (Section 4); the small-k series of
    Bhat^R agrees with eq. BhatR evaluated in 50-digit arithmetic."""
    R = 1.7
    assert se.bhat_trunc(np.array([0.0]), R)[0] == pytest.approx(math.pi * R ** 4, rel=1e-15)
    assert se.hhat_trunc(np.array([0.0]), R)[0] == pytest.approx(2 * math.pi * R * R, rel=1e-15)
    mpmath.mp.dps = 50
    for k in (1e-4, 0.01, 0.1, 0.25, 0.29, 0.3, 0.5, 2.0, 7.0):
        kk, RR = mpmath.mpf(k), mpmath.mpf(R)
        ex = 4 * mpmath.pi * ((2 - RR ** 2 * kk ** 2) * mpmath.cos(RR * kk)
                              + 2 * RR * kk * mpmath.sin(RR * kk) - 2) / kk ** 4
        got = se.bhat_trunc(np.array([k]), R)[0]
        assert abs(got - float(ex)) <= 1e-12 * abs(float(ex)), k
        exh = 8 * mpmath.pi * (mpmath.sin(RR * kk / 2) / kk) ** 2
        assert abs(se.hhat_trunc(np.array([k]), R)[0] - float(exh)) <= 1e-13 * float(exh)
