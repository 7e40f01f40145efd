"""Pins of the oracle's direct sums (Section 2) against closed forms and invariants."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import direct

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rot(seed):
    """A proper rotation from the QR of a seeded Gaussian matrix."""
    q, r = np.linalg.qr(W.rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _src(kernel, n, seed):
    a = W.normal_strengths(n, seed)
    b = W.normal_strengths(n, seed + 1) if kernel == "stresslet" else None
    return a, b


def test_two_point_closed_forms():
    cases = json.load(open(os.path.join(GOLD, "two_point.json")))["cases"]
    for c in cases:
        u = direct.direct(c["kernel"], np.array(c["x"], float), np.array(c["a"], float),
                          None if "b" not in c else np.array(c["b"], float))
        np.testing.assert_allclose(u, np.array(c["u"]), rtol=0, atol=1e-14)


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_translation_invariance(kernel):
    x = W.uniform_cube(64, 5)
    a, b = _src(kernel, 64, 6)
    u1 = direct.direct(kernel, x, a, b)
    u2 = direct.direct(kernel, x + np.array([0.25, -3.5, 7.0]), a, b)
    np.testing.assert_allclose(u2, u1, rtol=1e-12, atol=1e-12 * np.abs(u1).max())


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_rotation_covariance(kernel):
    """u(Qx, Qf) = Q u(x, f) for proper rotations; the stresslet rotates q and n."""
    x = W.uniform_cube(64, 7)
    a, b = _src(kernel, 64, 8)
    Q = _rot(9)
    u1 = direct.direct(kernel, x, a, b)
    u2 = direct.direct(kernel, x @ Q.T, a @ Q.T, None if b is None else b @ Q.T)
    np.testing.assert_allclose(u2, u1 @ Q.T, rtol=0, atol=1e-12 * np.abs(u1).max())


@pytest.mark.parametrize("kernel,sign", [("stokeslet", -1.0), ("stresslet", -1.0), ("rotlet", 1.0)])
def test_inversion_parity(kernel, sign):
    """x -> -x with strengths fixed: S and T are odd under r -> -r in their action
    on a polar field, so u flips; the rotlet gives a pseudo-vector and does not."""
    x = W.uniform_cube(50, 10)
    a, b = _src(kernel, 50, 11)
    u1 = direct.direct(kernel, x, a, b)
    u2 = direct.direct(kernel, -x, -a, None if b is None else -b)
    # S(-r) = S(r): u(-x, -f) = -u;  T(-r) = -T(r), (-q)(-n) = qn: u -> -u;
    # Omega(-r) = -Omega(r), -f: u unchanged.
    np.testing.assert_allclose(u2, sign * u1, rtol=0, atol=1e-12 * np.abs(u1).max())


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_reciprocity(kernel):
    """w . K f = f . K w: the operator with blocks G(x_m - x_n) is symmetric for S and Omega."""
    x = W.uniform_cube(80, 12)
    f = W.normal_strengths(80, 13)
    w = W.normal_strengths(80, 14)
    lhs = np.sum(w * direct.direct(kernel, x, f))
    rhs = np.sum(f * direct.direct(kernel, x, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_stresslet_index_symmetry():
    """T_jlm is symmetric in (l, m): swapping q and n leaves u unchanged (Section 2)."""
    x = W.uniform_cube(40, 15)
    q, n = W.normal_strengths(40, 16), W.normal_strengths(40, 17)
    np.testing.assert_allclose(direct.direct("stresslet", x, q, n), direct.direct("stresslet", x, n, q),
                               rtol=1e-13, atol=1e-13)


def test_superposition_brute_force():
    """The N-point sum equals the sum of two-point sums, one source at a time."""
    x = W.uniform_cube(12, 18)
    f = W.normal_strengths(12, 19)
    u = direct.direct("stokeslet", x, f)
    acc = np.zeros_like(u)
    for s in range(len(x)):
        fs = np.zeros_like(f)
        fs[s] = f[s]
        acc += direct.direct("stokeslet", x, fs)
    np.testing.assert_allclose(u, acc, rtol=1e-13, atol=1e-13)


def test_free_targets_and_subset():
    """Target subsets and free targets agree with the full self-excluded sum."""
    x = W.uniform_cube(100, 20)
    f = W.normal_strengths(100, 21)
    u = direct.direct("stokeslet", x, f)
    sub = np.array([3, 50, 99])
    np.testing.assert_array_equal(direct.direct("stokeslet", x, f, targets=sub), u[sub])
    y = np.array([[2.0, 2.0, 2.0]])
    uy = direct.direct("stokeslet", x, f, y=y)
    # far field: leading term is S(y - c) sum f
    c = x.mean(axis=0)
    r = y[0] - c
    F = f.sum(axis=0)
    lead = F / np.linalg.norm(r) + r * (r @ F) / np.linalg.norm(r) ** 3
    assert np.linalg.norm(uy[0] - lead) < 0.2 * np.linalg.norm(lead)


def test_coincident_points_rejected():
    x = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    f = np.ones((3, 3))
    with pytest.raises(ValueError):
        direct.direct("stokeslet", x, f)


def test_stresslet_adjoint_is_the_derivative_of_the_direct_sum():
    """dL/dq and dL/dn of L = w . u_T(q, n): u is linear in q and in n, so a
    central difference in any direction is exact up to rounding; brute-force one-hot
    differences on a tiny system and random directions on a larger one."""
    rng = np.random.default_rng(77)
    n = 9
    x = rng.uniform(size=(n, 3))
    q, nn, w = (rng.normal(size=(n, 3)) for _ in range(3))
    dq, dn = direct.stresslet_adjoint(x, q, nn, w)
    L = lambda qq, nv: float(np.sum(w * direct.direct("stresslet", x, qq, nv)))
    for b in range(n):
        for l in range(3):
            e = np.zeros((n, 3))
            e[b, l] = 1.0
            assert abs((L(q + e, nn) - L(q - e, nn)) / 2 - dq[b, l]) < 1e-9 * (1 + abs(dq[b, l]))
            assert abs((L(q, nn + e) - L(q, nn - e)) / 2 - dn[b, l]) < 1e-9 * (1 + abs(dn[b, l]))
    n = 300
    x = rng.uniform(size=(n, 3))
    q, nn, w = (rng.normal(size=(n, 3)) for _ in range(3))
    tg = np.array([0, 17, 123, 299])
    dq, dn = direct.stresslet_adjoint(x, q, nn, w, targets=tg)
    dqa, dna = direct.stresslet_adjoint(x, q, nn, w)
    assert np.allclose(dq, dqa[tg], rtol=1e-13, atol=0) and np.allclose(dn, dna[tg], rtol=1e-13, atol=0)
    for _ in range(3):
        d = rng.normal(size=(n, 3))
        gq = (L(q + d, nn) - L(q - d, nn)) / 2
        gn = (L(q, nn + d) - L(q, nn - d)) / 2
        assert abs(gq - np.sum(dqa * d)) < 1e-10 * abs(gq)
        assert abs(gn - np.sum(dna * d)) < 1e-10 * abs(gn)
