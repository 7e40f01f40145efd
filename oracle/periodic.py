"""TEST INFRASTRUCTURE ONLY: triply periodic stokeslet sums (Section 1.1), FP64.

ewald_sum
    The Hasimoto Ewald formula of Section 1.1 (eq. usum_SR_SF_limit) written out
    directly: the real-space kernel of eq. SR_Hasimoto summed over every periodic
    image within r_c (the n = m, p = 0 term excluded), the k-space kernel of
    eq. ShatH summed over the wavevectors k = 2 pi j / L, j != 0, up to a cutoff
    where its Gaussian factor is below double precision, divided by V, and the
    self term of eq. Slimit.  With r_c and the k cutoff beyond the Gaussian
    decay this is the periodic sum itself (the sum over images of eq. usumper,
    made definite by the mean pressure gradient of Section 1.1), and it does not
    depend on xi.

se_fourier
    The spectral Ewald discretization of that k-space sum on an M^3 grid over
    one period (the periodic form of Section 5.1's steps): Gaussians of exponent
    alpha = 2 xi^2 / eta truncated to P^3 windows that wrap around the period
    (eq. Hx), numpy FFT, the scaling of eq. gridfcnsc with the eq. ShatH kernel
    (k = 0 dropped), inverse FFT, and the trapezoidal quadrature (eq. u_integr)
    with the same wrapped windows.

Plain numpy; only tests import this module.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

C_GAUSS = 0.976  # m = C sqrt(pi P), Section 5.3


def real_kernel(r, xi):
    """S^R(r) of eq. SR_Hasimoto for displacement rows r (n, 3): (n, 3, 3)."""
    r2 = np.einsum("ij,ij->i", r, r)
    rr = np.sqrt(r2)
    e = np.exp(-xi * xi * r2)
    c1 = 2.0 * (xi * e / (math.sqrt(math.pi) * r2) + erfc(xi * rr) / (2.0 * r2 * rr))
    eye = np.eye(3)[None]
    return (c1[:, None, None] * (r2[:, None, None] * eye + r[:, :, None] * r[:, None, :])
            - (4.0 * xi / math.sqrt(math.pi) * e)[:, None, None] * eye)


def ewald_sum(x, f, L, xi, rc=None, box_lo=(0.0, 0.0, 0.0), tol=1e-17):
    """u^{3P}(x_m), eq. usum_SR_SF_limit, for the stokeslet in the periodic cube
    [box_lo, box_lo + L)^3.  rc defaults to the radius where erfc(xi r) < tol;
    the k-space cutoff keeps every k with exp(-k^2/4xi^2) above tol."""
    x = np.asarray(x, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    n = len(x)
    if rc is None:
        rc = math.sqrt(-math.log(tol)) / xi + 1e-12
    # real space: every image p = L j with |x_m - x_n + p| <= rc
    nimg = int(math.ceil(rc / L)) + 1
    rng = range(-nimg, nimg + 1)
    uR = np.zeros((n, 3))
    for m in range(n):
        d0 = x[m] - x
        for j0 in rng:
            for j1 in rng:
                for j2 in rng:
                    d = d0 + L * np.array([j0, j1, j2], dtype=np.float64)
                    r2 = np.einsum("ij,ij->i", d, d)
                    sel = r2 <= rc * rc
                    if j0 == j1 == j2 == 0:
                        sel[m] = False
                    if np.any(sel & (r2 == 0.0)):
                        raise ValueError("coincident distinct points")
                    if np.any(sel):
                        uR[m] += np.einsum("ijk,ik->j", real_kernel(d[sel], xi), f[sel])
    # k space: (1/V) sum_{k != 0} S^F(k) sum_n f_n exp(i k.(x_m - x_n))
    kmax = 2.0 * xi * math.sqrt(-math.log(tol))
    K = int(math.ceil(kmax * L / (2.0 * math.pi)))
    j = np.arange(-K, K + 1)
    J = np.stack(np.meshgrid(j, j, j, indexing="ij"), -1).reshape(-1, 3)
    J = J[np.any(J != 0, axis=1)]
    k = 2.0 * math.pi / L * J.astype(np.float64)
    k2 = np.einsum("ij,ij->i", k, k)
    keep = k2 <= kmax * kmax
    k, k2 = k[keep], k2[keep]
    s = 8.0 * math.pi * (1.0 + k2 / (4.0 * xi * xi)) * np.exp(-k2 / (4.0 * xi * xi)) / (k2 * k2)
    uF = np.zeros((n, 3))
    for c0 in range(0, len(k), 4096):
        kc, sc, k2c = k[c0:c0 + 4096], s[c0:c0 + 4096], k2[c0:c0 + 4096]
        ph = np.exp(-1j * (x @ kc.T))                         # (n, nk): exp(-i k.x_n)
        S = ph.T @ f                                           # (nk, 3): structure factor
        kS = np.einsum("ij,ij->i", kc, S)
        A = sc[:, None] * (k2c[:, None] * S - kc * kS[:, None])   # S^F(k) applied
        uF += np.real(np.conj(ph) @ A)                         # sum_k exp(+i k.x_m) (...)
    uF /= L ** 3
    uself = -4.0 * xi / math.sqrt(math.pi) * f
    return dict(u=uR + uF + uself, uR=uR, uF=uF, uself=uself)


def geometry(xi, M, P, L, C=C_GAUSS):
    """h, eta, alpha of the periodic grid (h = L / M, eta = (xi h P / m)^2,
    m = C sqrt(pi P), alpha = 2 xi^2 / eta; Sections 5.2-5.3)."""
    h = L / M
    m = C * math.sqrt(math.pi * P)
    eta = (xi * h * P / m) ** 2
    return dict(h=h, eta=eta, alpha=2.0 * xi * xi / eta, M=M, P=P, L=L, xi=xi)


def _windows(x, g, box_lo):
    """Window start b = floor(t - P/2 + 1), t = (x - box_lo)/h, and the P node
    offsets' Gaussian factors per direction (as in the free-space windows)."""
    h, P, a = g["h"], g["P"], g["alpha"]
    t = (np.asarray(x, np.float64) - np.asarray(box_lo, np.float64)) / h
    b = np.floor(t - 0.5 * P + 1.0).astype(np.int64)
    i = b[:, :, None] + np.arange(P)[None, None, :]             # (n, 3, P) unwrapped nodes
    w = np.exp(-a * h * h * (t[:, :, None] - i) ** 2)           # (n, 3, P)
    return i % g["M"], w


def se_fourier(x, f, g, box_lo=(0.0, 0.0, 0.0)):
    """u^F at the points by the periodic spectral Ewald steps (see the module doc)."""
    M, h, a, xi, eta = g["M"], g["h"], g["alpha"], g["xi"], g["eta"]
    norm = (a / math.pi) ** 1.5
    idx, w = _windows(x, g, box_lo)
    n = len(x)
    grid = np.zeros((3, M, M, M))
    for p in range(n):
        W = norm * np.einsum("i,j,k->ijk", w[p, 0], w[p, 1], w[p, 2])
        ix = np.ix_(idx[p, 0], idx[p, 1], idx[p, 2])
        for c in range(3):
            grid[c][ix] += f[p, c] * W
    G = np.fft.fftn(grid, axes=(1, 2, 3))
    kk = 2.0 * math.pi * np.fft.fftfreq(M, d=h)
    K = np.stack(np.meshgrid(kk, kk, kk, indexing="ij"), 0)     # (3, M, M, M)
    k2 = np.sum(K * K, 0)
    k2s = np.where(k2 == 0.0, 1.0, k2)
    s = 8.0 * math.pi * (1.0 + k2 / (4 * xi * xi)) * np.exp(-(1.0 - eta) * k2 / (4 * xi * xi)) / (k2s * k2s)
    s[k2 == 0.0] = 0.0
    kG = np.sum(K * G, 0)
    Wk = s[None] * (k2[None] * G - K * kG[None])
    field = np.real(np.fft.ifftn(Wk, axes=(1, 2, 3)))
    u = np.zeros((n, 3))
    for p in range(n):
        Wq = h ** 3 * norm * np.einsum("i,j,k->ijk", w[p, 0], w[p, 1], w[p, 2])
        ix = np.ix_(idx[p, 0], idx[p, 1], idx[p, 2])
        for c in range(3):
            u[p, c] = np.sum(field[c][ix] * Wq)
    return u
