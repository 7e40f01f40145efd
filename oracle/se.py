"""TEST INFRASTRUCTURE ONLY: FP64 numpy implementation of the free-space
spectral Ewald (FSE) method of af Klinteberg, Shamshirgar & Tornberg
(arXiv:1607.04808), step by step in the paper's order and notation.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
use this module.  Library primitives used as steps: numpy's FFT.

Steps (paper section -> function):
  Section 4.3 "Precomputation"        mollified_kernel()  (IFFT on M_g^3, crop to
                                       (2 Mt)^3 centred, FFT)
  Section 5.2 "Discretization", step 1 spread()            (eq. Hx, truncated
                                       Gaussians on a P^3 cube, Section 5.2 FGG)
  step 2 FFT, zero-padded to (2 Mt)^3  fourier_step()
  step 3 scaling by eq. gridfcnsc with eqs. AS/AT/AR (truncated B or H)
  step 4 IFFT and truncation to Mt^3
  step 5 quadrature (eq. u_integr)     gather()
  Section 6 real-space sum             direct.real_trunc()
  eq. Slimit self term                 self_term()
  Section 8.2 parameter choices          geometry()

Readings of the paper taken here (all listed with their pins in the design doc):
  * grid: nodes x0 + j h, j = 0..Mt-1, x0 = box_lo - (Lt - L)/2 (the extended
    domain of Section 5.2 centred on the box), h = L/M, Lt = Mt h.
  * window: P consecutive nodes per dimension starting at
    b = floor(t - P/2 + 1), t = (x - x0)/h, computed in FP64 (Section 5.2 FGG).
  * Fourier convention: forward transform e^{-i k.x}, inverse e^{+i k.x}
    (Section 3.1), so derivatives map to +ik.  The stresslet and rotlet
    multipliers of eqs. AT and AR are used with that convention; the rotlet is
    normalised as in eq. def_rotlet (one half of the operator-form factor 2):
        A^S_jl = -(k^2 d_jl - k_j k_l)(1 + k^2/4xi^2) Bt(k)
        A^T_jlm = -i[(k_m d_jl + k_j d_lm + k_l d_mj) k^2 - 2 k_j k_l k_m](1 + k^2/4xi^2) Bt(k)
        A^O_jl = -i eps_jlm k_m Ht(k)
    with Bt, Ht the mollified truncated kernels of Section 4.3.
  * the FFTs are full complex transforms; the real part of the inverse is kept.
  * normalisation: the inverse FFT carries 1/(2Mt)^3, the quadrature carries h^3
    (Section 4.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import direct

C_GAUSS = 0.976  # the constant C of m = C sqrt(pi P), Section 5.3
KERNELS = ("stokeslet", "stresslet", "rotlet")


def _kname(kernel):
    return KERNELS[kernel] if isinstance(kernel, (int, np.integer)) else kernel


@dataclass
class Geometry:
    xi: float
    rc: float
    M: int
    P: int
    box_lo: np.ndarray
    L: float
    h: float
    d: float
    m: float
    eta: float
    alpha: float
    deltaL_min: float
    Mt: int
    Lt: float
    x0: np.ndarray
    Mg: int
    R: float

    @property
    def n(self):
        return 2 * self.Mt


def geometry(xi, rc, M, P, box_lo=(0.0, 0.0, 0.0), L=1.0, Mt=None, deltaL_rule=0,
             C=C_GAUSS):
    """Derived parameters of Sections 6.2-6.3 and 8.

    h = L/M; d = hP; m = C sqrt(pi P); eta = (xi d / m)^2; Gaussian exponent
    alpha = 2 xi^2 / eta (eq. Hx); deltaL from eq. deltaL_cond (rule 1) or
    deltaL = d (rule 0, the choice of the Results section); Mt grid points on
    Lt = Mt h >= L + deltaL; M_g = the smallest even integer above
    (1 + sqrt 3) Mt (Results section); R = sqrt(3) Lt (Section 4.1).
    ``Mt`` may be given larger than the minimum (zero padding on the grid).
    """
    box_lo = np.asarray(box_lo, dtype=np.float64).reshape(3)
    h = L / M
    d = h * P
    m = C * math.sqrt(math.pi * P)
    eta = (xi * d / m) ** 2
    alpha = 2.0 * xi * xi / eta
    if deltaL_rule == 0 or eta >= 1.0:
        dL = d
    else:
        dL = max(d, math.sqrt(2.0 * (1.0 - eta) * m * m / (xi * xi)))
    Mt_min = M + int(math.ceil(dL / h - 1e-12))
    if Mt is None:
        Mt = Mt_min
    if Mt < Mt_min:
        raise ValueError("Mt=%d below the minimum %d" % (Mt, Mt_min))
    Lt = Mt * h
    x0 = box_lo - 0.5 * (Lt - L)
    Mg = int(math.floor((1.0 + math.sqrt(3.0)) * Mt)) + 1
    if Mg % 2:
        Mg += 1
    R = math.sqrt(3.0) * Lt
    return Geometry(float(xi), float(rc), int(M), int(P), box_lo, float(L), h, d, m, eta,
                    alpha, dL, int(Mt), Lt, x0, Mg, R)


# ---------------------------------------------------------------------------
# Section 4: truncated Green's functions and the mollified kernel
# ---------------------------------------------------------------------------

def _bhat_series_coeffs(nterms=14):
    """c_{2j} of N(x) = (2 - x^2) cos x + 2 x sin x - 2 = sum_j c_{2j} x^{2j}."""
    cs = []
    for j in range(2, 2 + nterms):
        c = 2.0 / math.factorial(2 * j) + 1.0 / math.factorial(2 * j - 2) - 2.0 / math.factorial(2 * j - 1)
        cs.append((-1) ** j * c)
    return cs


_BH_COEFFS = _bhat_series_coeffs()


def bhat_trunc(k, R):
    """Fourier transform of the truncated biharmonic Green's function, eq. BhatR.

    4 pi [(2 - R^2k^2) cos Rk + 2 Rk sin Rk - 2] / k^4, with limit pi R^4 at
    k = 0.  The numerator cancels to (Rk)^4/4 near 0, so for Rk < 0.5 the
    Taylor series of the numerator is summed instead (exact to rounding).
    """
    k = np.asarray(k, dtype=np.float64)
    x = k * R
    out = np.empty_like(x)
    small = x < 0.5
    xs = x[small]
    ser = np.zeros_like(xs)
    for j, c in enumerate(_BH_COEFFS):
        ser += c * xs ** (2 * j)  # c_{2(j+2)} x^{2j} = N(x)/x^4 term
    out[small] = 4.0 * math.pi * R ** 4 * ser
    xl, kl = x[~small], k[~small]
    out[~small] = 4.0 * math.pi * ((2.0 - xl * xl) * np.cos(xl) + 2.0 * xl * np.sin(xl) - 2.0) / kl ** 4
    return out


def hhat_trunc(k, R):
    """Fourier transform of the truncated harmonic Green's function, eq. HhatR.

    8 pi (sin(Rk/2)/k)^2, limit 2 pi R^2 at k = 0.
    """
    k = np.asarray(k, dtype=np.float64)
    out = np.empty_like(k)
    z = k == 0
    out[z] = 2.0 * math.pi * R * R
    kk = k[~z]
    out[~z] = 8.0 * math.pi * (np.sin(R * kk / 2.0) / kk) ** 2
    return out


def kernel_family(kernel):
    """Biharmonic for the stokeslet and stresslet, harmonic for the rotlet (Section 3.2)."""
    return "H" if _kname(kernel) == "rotlet" else "B"


def mollified_kernel(family, g: Geometry, return_imag=False):
    """The transformed mollified Green's function on the (2Mt)^3 grid (Section 4.3).

    1. evaluate Bhat^R (or Hhat^R) at k = 2 pi kbar / (M_g h), kbar in
       [-M_g/2, M_g/2), on an M_g^3 grid (oversampling s_f = M_g / Mt >= 1 + sqrt 3);
    2. inverse FFT (1/M_g^3 built in, no other prefactor);
    3. keep G_j for j in [-Mt, Mt)^3 (the mollified kernel on the doubled grid);
    4. forward FFT of size (2Mt)^3.
    Returns the real array indexed in FFT order (index i <-> kbar = i or i - 2Mt),
    with k = pi kbar / Lt.
    """
    Mg, Mt, h = g.Mg, g.Mt, g.h
    kb = np.fft.fftfreq(Mg, 1.0 / Mg)
    k1 = 2.0 * math.pi * kb / (Mg * h)
    K = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k1[None, None, :] ** 2)
    Gh = bhat_trunc(K, g.R) if family == "B" else hhat_trunc(K, g.R)
    del K
    G = np.fft.ifftn(Gh)
    del Gh
    j = np.arange(-Mt, Mt)
    src = j % Mg
    dst = j % (2 * Mt)
    Gt = np.zeros((2 * Mt,) * 3, dtype=np.complex128)
    Gt[np.ix_(dst, dst, dst)] = G[np.ix_(src, src, src)]
    del G
    Kt = np.fft.fftn(Gt)
    if return_imag:
        return Kt.real, float(np.abs(Kt.imag).max())
    return Kt.real


# ---------------------------------------------------------------------------
# Section 5.2: spreading and quadrature with truncated Gaussians
# ---------------------------------------------------------------------------

def window(x, g: Geometry):
    """Continuous grid coordinate t = (x - x0)/h and window start b (FP64)."""
    t = (np.asarray(x, dtype=np.float64) - g.x0) / g.h
    b = np.floor(t - g.P / 2.0 + 1.0).astype(np.int64)
    return t, b


def gauss_1d(t, b, g: Geometry):
    """exp(-alpha |x_node - x|^2) factors per dimension: array (N, 3, P)."""
    i = np.arange(g.P)
    dist = (t[:, :, None] - (b[:, :, None] + i)) * g.h
    return np.exp(-g.alpha * dist * dist)


def _flat_index(b, g: Geometry):
    Mt, P = g.Mt, g.P
    i = np.arange(P)
    ix = b[:, 0, None] + i
    iy = b[:, 1, None] + i
    iz = b[:, 2, None] + i
    if ix.min() < 0 or max(ix.max(), iy.max(), iz.max()) >= Mt or min(iy.min(), iz.min()) < 0:
        raise ValueError("Gaussian window outside the grid: point outside the box")
    return (ix[:, :, None, None] * Mt + iy[:, None, :, None]) * Mt + iz[:, None, None, :]


def spread(x, src, g: Geometry, chunk=2048):
    """Step 1: grid function H(x_p) of eq. Hx on the Mt^3 grid.

    H(x_p) = sum_n src_n (2 xi^2/(pi eta))^{3/2} exp(-2 xi^2 |x_p - x_n|^2 / eta)
    over the P^3 window of each source.  src: (N, c).  Returns (c, Mt, Mt, Mt),
    axes (x, y, z).
    """
    x = np.asarray(x, dtype=np.float64)
    src = np.asarray(src, dtype=np.float64).reshape(len(x), -1)
    c = src.shape[1]
    Mt = g.Mt
    norm = (g.alpha / math.pi) ** 1.5
    out = np.zeros((c, Mt ** 3))
    for s in range(0, len(x), chunk):
        xs = x[s:s + chunk]
        t, b = window(xs, g)
        w = gauss_1d(t, b, g)
        W = w[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]
        idx = _flat_index(b, g).ravel()
        for comp in range(c):
            vals = (W * src[s:s + chunk, comp, None, None, None]).ravel()
            out[comp] += np.bincount(idx, weights=vals, minlength=Mt ** 3)
    return norm * out.reshape(c, Mt, Mt, Mt)


def gather(grid, x, g: Geometry, chunk=2048):
    """Step 5: quadrature of eq. u_integr with the trapezoidal rule (weight h^3)."""
    x = np.asarray(x, dtype=np.float64)
    c = grid.shape[0]
    flat = grid.reshape(c, -1)
    norm = (g.alpha / math.pi) ** 1.5 * g.h ** 3
    out = np.zeros((len(x), c))
    for s in range(0, len(x), chunk):
        xs = x[s:s + chunk]
        t, b = window(xs, g)
        w = gauss_1d(t, b, g)
        W = w[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]
        idx = _flat_index(b, g)
        for comp in range(c):
            out[s:s + chunk, comp] = (flat[comp][idx] * W).sum(axis=(1, 2, 3))
    return norm * out


# ---------------------------------------------------------------------------
# Section 5.2 steps 2-4: FFT, scaling (eq. gridfcnsc), IFFT
# ---------------------------------------------------------------------------

def wavevectors(g: Geometry):
    """k = pi kbar / Lt on the (2Mt)^3 grid, FFT order; broadcastable arrays."""
    n = g.n
    kb = np.fft.fftfreq(n, 1.0 / n)
    k1 = math.pi * kb / g.Lt
    return k1[:, None, None], k1[None, :, None], k1[None, None, :]


def fourier_step(kernel, grid, g: Geometry, Kt):
    """Steps 2-4 of Section 5.2 for one source set.

    grid: (c, Mt, Mt, Mt) real, c = 3 (stokeslet, rotlet: f_l) or 9 (stresslet:
    f_lm = n_l q_m at index 3l + m).  Kt: mollified kernel (Bt or Ht) on the
    (2Mt)^3 grid.  Returns the scaled, inverse transformed and truncated grid
    function (3, Mt, Mt, Mt).
    """
    kernel = _kname(kernel)
    n, Mt = g.n, g.Mt
    gh = np.fft.fftn(grid, s=(n, n, n), axes=(1, 2, 3))
    kx, ky, kz = wavevectors(g)
    k = (kx, ky, kz)
    k2 = kx * kx + ky * ky + kz * kz
    E = np.exp(-(1.0 - g.eta) * k2 / (4.0 * g.xi * g.xi))
    w = np.empty((3, n, n, n), dtype=np.complex128)
    if kernel == "stokeslet":
        sig = -(1.0 + k2 / (4.0 * g.xi ** 2)) * E * Kt
        kg = kx * gh[0] + ky * gh[1] + kz * gh[2]
        for j in range(3):
            w[j] = sig * (k2 * gh[j] - k[j] * kg)
    elif kernel == "rotlet":
        sig = E * Kt
        # A^O_jl g_l = -i eps_jlm g_l k_m = -i (g x k)_j
        w[0] = -1j * sig * (gh[1] * kz - gh[2] * ky)
        w[1] = -1j * sig * (gh[2] * kx - gh[0] * kz)
        w[2] = -1j * sig * (gh[0] * ky - gh[1] * kx)
    else:
        sig = (1.0 + k2 / (4.0 * g.xi ** 2)) * E * Kt
        G = [[gh[3 * l + m] for m in range(3)] for l in range(3)]
        tr = G[0][0] + G[1][1] + G[2][2]
        kgk = sum(k[l] * k[m] * G[l][m] for l in range(3) for m in range(3))
        for j in range(3):
            a = sum(k[m] * G[j][m] for m in range(3)) + sum(k[l] * G[l][j] for l in range(3))
            w[j] = -1j * sig * (k2 * (a + k[j] * tr) - 2.0 * k[j] * kgk)
    del gh
    out = np.fft.ifftn(w, axes=(1, 2, 3))[:, :Mt, :Mt, :Mt]
    return out.real.copy()


def sources_grid(kernel, a, b=None):
    """Per-point source components spread onto the grid: f (N,3) or n_l q_m (N,9)."""
    if _kname(kernel) == "stresslet":
        q, nn = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
        return (nn[:, :, None] * q[:, None, :]).reshape(len(q), 9)
    return np.asarray(a, dtype=np.float64)


def self_term(kernel, xi, a):
    """u^self = lim (G^R - G) . f_m at the target's own source (eq. Slimit); stokeslet only."""
    if _kname(kernel) == "stokeslet":
        return -4.0 * xi / math.sqrt(math.pi) * np.asarray(a, dtype=np.float64)
    return np.zeros_like(np.asarray(a, dtype=np.float64))


def fourier_part(kernel, x, a, b, g: Geometry, Kt=None, return_field=False):
    """u^F at the sources: spread -> FFT -> scale -> IFFT -> quadrature."""
    if Kt is None:
        Kt = mollified_kernel(kernel_family(kernel), g)
    grid = spread(x, sources_grid(kernel, a, b), g)
    field = fourier_step(kernel, grid, g, Kt)
    uF = gather(field, x, g)
    return (uF, field) if return_field else uF


def evaluate(kernel, x, a, b=None, g: Geometry | None = None, Kt=None, **geo):
    """Full FSE sum at the sources: u = u^R + u^F + u^self (Section 8)."""
    if g is None:
        g = geometry(**geo)
    uR = direct.real_trunc(kernel, g.xi, g.rc, x, a, b)
    uF = fourier_part(kernel, x, a, b, g, Kt)
    us = self_term(kernel, g.xi, a)
    return dict(u=uR + uF + us, uR=uR, uF=uF, uself=us)


def grad_x(kernel, x, f, w, g: Geometry, Kt=None):
    """dL/dx of L = sum_m w_m . u_FSE(x_m) for the discrete FSE operator (S, Omega).

    The Fourier part differentiates the Gaussian windows of both the spreading
    and the quadrature step:
      dL/dx_s = h^3 sum_p grad g(x_s - x_p) [w_s . phi_f(x_p) + f_s . phi_w(x_p)],
    phi_f, phi_w the scaled inverse-transformed grids of f and w (steps 1-4),
    g(r) = (alpha/pi)^{3/2} exp(-alpha r^2).  The real-space part is the
    analytic gradient of the truncated sum.  Valid for kernels whose discrete
    operator is symmetric (stokeslet, rotlet).
    """
    kernel = _kname(kernel)
    if kernel == "stresslet":
        raise NotImplementedError("stresslet adjoint")
    if Kt is None:
        Kt = mollified_kernel(kernel_family(kernel), g)
    x = np.asarray(x, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    phi_f = fourier_step(kernel, spread(x, f, g), g, Kt)
    phi_w = fourier_step(kernel, spread(x, w, g), g, Kt)
    norm = (g.alpha / math.pi) ** 1.5 * g.h ** 3
    t, b = window(x, g)
    wg = gauss_1d(t, b, g)
    i = np.arange(g.P)
    dvec = (t[:, :, None] - (b[:, :, None] + i)) * g.h  # x - x_node per dim
    dg = -2.0 * g.alpha * dvec * wg  # derivative factor per dim
    out = np.zeros((len(x), 3))
    idx = _flat_index(b, g)
    pf = phi_f.reshape(3, -1)
    pw = phi_w.reshape(3, -1)
    psi = sum(w[:, c, None, None, None] * pf[c][idx] + f[:, c, None, None, None] * pw[c][idx]
              for c in range(3))
    gx = dg[:, 0, :, None, None] * wg[:, 1, None, :, None] * wg[:, 2, None, None, :]
    gy = wg[:, 0, :, None, None] * dg[:, 1, None, :, None] * wg[:, 2, None, None, :]
    gz = wg[:, 0, :, None, None] * wg[:, 1, None, :, None] * dg[:, 2, None, None, :]
    out[:, 0] = (psi * gx).sum(axis=(1, 2, 3))
    out[:, 1] = (psi * gy).sum(axis=(1, 2, 3))
    out[:, 2] = (psi * gz).sum(axis=(1, 2, 3))
    return norm * out + direct.grad_real_trunc(kernel, g.xi, g.rc, x, f, w)


# ---------------------------------------------------------------------------
# Section 7 truncation-error estimates (Tables est_fourier and est_real)
# ---------------------------------------------------------------------------

def est_fourier(kernel, Q, xi, L, kinf, R):
    """RMS Fourier truncation error, Table est_fourier."""
    kernel = _kname(kernel)
    e = math.exp(-kinf * kinf / (4.0 * xi * xi))
    if kernel == "stokeslet":
        return math.sqrt(Q) * R * kinf ** 3 / (xi * xi * math.pi * L) * e
    if kernel == "stresslet":
        return math.sqrt(7.0 * Q / 6.0) * R * kinf ** 4 / (xi * xi * math.pi * L) * e
    return math.sqrt(8.0 * xi * xi * Q / (3.0 * math.pi * L ** 3 * kinf)) * e


def est_real(kernel, Q, xi, L, rc):
    """RMS real-space truncation error, Table est_real."""
    kernel = _kname(kernel)
    e = math.exp(-xi * xi * rc * rc)
    if kernel == "stokeslet":
        return math.sqrt(4.0 * Q * rc / L ** 3) * e
    if kernel == "stresslet":
        return math.sqrt(112.0 * Q * xi ** 4 * rc ** 3 / (9.0 * L ** 3)) * e
    return math.sqrt(8.0 * Q / (3.0 * L ** 3 * rc)) * e


def real_kernel_tensor(kernel, xi, rvec):
    """G^R(r) as a tensor (3x3 or 3x3x3) by probing the oracle's real-space sum."""
    kernel = _kname(kernel)
    rvec = np.asarray(rvec, dtype=np.float64)
    x = np.array([np.zeros(3), -rvec])  # target at 0, source at -r -> r = 0 - (-r)
    rc = 2.0 * np.linalg.norm(rvec) + 1.0
    if kernel == "stresslet":
        T = np.zeros((3, 3, 3))
        for l in range(3):
            for m in range(3):
                nn = np.zeros((2, 3)); q = np.zeros((2, 3))
                nn[1, l] = 1.0; q[1, m] = 1.0
                T[:, l, m] = direct.real_trunc(kernel, xi, rc, x, q, nn, targets=[0])[0]
        return T
    S = np.zeros((3, 3))
    for l in range(3):
        f = np.zeros((2, 3)); f[1, l] = 1.0
        S[:, l] = direct.real_trunc(kernel, xi, rc, x, f, targets=[0])[0]
    return S

