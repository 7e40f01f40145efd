"""Fit of the FP32 complementary error function used by the real-space kernels.

erfc(x) = exp(-x^2) * t * Q(t),  t = 1 / (1 + p x),  x >= 0,

the form of the rational-in-t approximations of Abramowitz & Stegun 7.1.25-7.1.28
with a polynomial Q of higher degree.  Q is fitted here by iteratively
reweighted least squares for small relative error of erfcx(x) = exp(x^2) erfc(x)
over all t in (0, 1], i.e. all x >= 0 (Q(0) = p / sqrt(pi) from the asymptote
erfcx(x) ~ 1 / (x sqrt(pi))).  Run it to print the coefficient table and the
achieved maximum relative error in FP64 and with FP32 Horner evaluation.
"""
import numpy as np
from scipy.special import erfc, erfcx

P_T = 0.4
DEGREE = 10


def fit(p=P_T, degree=DEGREE, iters=60):
    t = np.concatenate([np.cos(np.linspace(0, np.pi / 2, 20000)), np.linspace(1e-6, 1, 20000)])
    t = t[(t > 0) & (t <= 1)]
    x = (1 / t - 1) / p
    y = erfcx(x) / t
    w = np.ones_like(t)
    V = np.vander(t, degree + 1, increasing=True)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(V / y[:, None] * w[:, None], w, rcond=None)
        rel = (V @ c) / y - 1
        w = w * (np.abs(rel) / np.abs(rel).max()) ** 0.3 + 1e-3
        w /= w.max()
    rel = (V @ c) / y - 1
    return c, float(np.abs(rel).max())


def fp32_error(c, p=P_T, xmax=9.0):
    f32 = np.float32
    x = np.linspace(0, xmax, 200001).astype(f32)
    t = f32(1) / (f32(1) + f32(p) * x)
    q = np.full_like(x, f32(c[-1]))
    for cc in c[-2::-1]:
        q = (q * t + f32(cc)).astype(f32)
    approx = (t * q).astype(np.float64) * np.exp(-x.astype(np.float64) ** 2)
    ref = erfc(x.astype(np.float64))
    m = ref > 1e-37
    return float(np.abs(approx[m] / ref[m] - 1).max())


if __name__ == "__main__":
    c, e = fit()
    print("p = %.9g, degree %d, max rel err (fp64) %.3g, (fp32 Horner) %.3g" % (P_T, DEGREE, e, fp32_error(c)))
    print(", ".join("%.9gf" % v for v in c))
