"""Pins of the triply periodic oracle (Section 1.1): the Hasimoto Ewald formula
(eq. usum_SR_SF_limit with eqs. SR_Hasimoto, ShatH, Slimit) and its spectral
Ewald discretization on one period."""
import math

import numpy as np
import pytest

from oracle import direct
from oracle import periodic as PE


def _system(n, seed, L):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, L, (n, 3)), rng.normal(size=(n, 3))


def test_ewald_sum_independent_of_xi():
    """The split into real and k space must not change the sum (xi only moves work)."""
    x, f = _system(30, 1, 1.3)
    us = [PE.ewald_sum(x, f, 1.3, xi)["u"] for xi in (3.5, 6.0, 10.0)]
    assert np.abs(us[0] - us[1]).max() < 1e-12 * np.abs(us[1]).max()
    assert np.abs(us[2] - us[1]).max() < 1e-12 * np.abs(us[1]).max()


def test_hasimoto_constant_of_the_cubic_lattice():
    """Two points a tiny distance d apart: the periodic sum's regular part at r -> 0
    is the cubic-lattice constant of Hasimoto (1959): u_1 - S(x_1 - x_2) f_2 ->
    -(4/3) 2.837297 / L f_2 (the drag correction 1 - 1.7601 c^{1/3} of a simple
    cubic array of spheres, c^{1/3} = (4 pi / 3)^{1/3} a / L), up to O(d^2 / L^3)."""
    L = 2.0
    f = np.array([[0.0, 0.0, 0.0], [0.3, -1.1, 0.7]])
    x = np.array([[0.9, 1.0, 1.1], [0.9 + 1e-4, 1.0 - 2e-4, 1.1 + 1e-4]])
    u = PE.ewald_sum(x, f, L, 5.0)["u"]
    free = direct.direct("stokeslet", x, f)
    corr = u[0] - free[0]
    assert np.allclose(corr, -(4.0 / 3.0) * 2.837297 / L * f[1], rtol=2e-6, atol=0)


def test_ewald_sum_translation_and_periodicity():
    """Shifting every point (and wrapping it into the cell) leaves the sum unchanged,
    and a point moved by a lattice vector is the same point."""
    L = 1.1
    x, f = _system(25, 2, L)
    u = PE.ewald_sum(x, f, L, 6.0)["u"]
    xs = np.mod(x + np.array([0.37, -0.81, 0.55]), L)
    assert np.abs(PE.ewald_sum(xs, f, L, 6.0)["u"] - u).max() < 1e-12 * np.abs(u).max()
    xl = x.copy()
    xl[3] += np.array([L, 0.0, -L])
    assert np.abs(PE.ewald_sum(xl, f, L, 6.0)["u"] - u).max() < 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("M,P,tol", [(24, 12, 2e-6), (32, 16, 3e-9), (40, 20, 3e-12)])
def test_se_discretization_converges_to_the_k_sum(M, P, tol):
    """The spectral Ewald steps on one period reproduce the k-space sum with the
    accuracy that the Gaussian support P sets (Section 8.2: about 2 digits per 4
    points of P here)."""
    L, xi = 1.3, 6.0
    x, f = _system(40, 3, L)
    ref = PE.ewald_sum(x, f, L, xi)
    uF = PE.se_fourier(x, f, PE.geometry(xi, M, P, L))
    assert np.abs(uF - ref["uF"]).max() < tol * np.abs(ref["u"]).max()


def test_se_discretization_is_translation_invariant_on_the_grid():
    """Shifting every point by whole grid steps (wrapping into the cell) permutes the
    grid, so the discrete u^F is unchanged to rounding: the windows wrap at the
    period exactly as the nodes do."""
    L, xi, M = 1.0, 6.0, 30
    x, f = _system(12, 4, L)
    g = PE.geometry(xi, M, 14, L)
    u0 = PE.se_fourier(x, f, g)
    xs = np.mod(x + g["h"] * np.array([7.0, -3.0, 29.0]), L)
    assert np.abs(PE.se_fourier(xs, f, g) - u0).max() < 1e-12 * np.abs(u0).max()
