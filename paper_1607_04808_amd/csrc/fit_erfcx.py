"""Fits of the complementary error function used by the real-space kernels.

Both write erfc(x) = exp(-x^2) * t * Q(t) with t = 1 / (1 + p x), x >= 0, the
form of the rational-in-t approximations of Abramowitz & Stegun 7.1.25-7.1.28,
with a longer Q fitted here for small relative error of
erfcx(x) = exp(x^2) erfc(x):

* FP32: p = 0.4, Q a degree-10 polynomial in t, fitted by iteratively
  reweighted least squares over all t in (0, 1] (all x >= 0).
* FP64: p = 0.5, Q a degree-20 Chebyshev series in s = 2 (t - t0) / (1 - t0) - 1,
  t0 = 1 / (1 + p XMAX), fitted by weighted least squares at Chebyshev nodes
  against a 40-digit reference, for x in [0, XMAX]; beyond XMAX, erfc(x) is
  below 1e-44 and the kernels evaluate the series at s = -1.

Run it to print both coefficient tables and their maximum relative errors.
"""
import numpy as np
from scipy.special import erfc, erfcx

P32, DEG32 = 0.4, 10
P64, DEG64, XMAX64 = 0.5, 20, 10.0


def fit32(p=P32, degree=DEG32, iters=60):
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


def fp32_error(c, p=P32, xmax=9.0):
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


def fit64(p=P64, degree=DEG64, xmax=XMAX64, nodes=3000):
    import mpmath as mp
    mp.mp.dps = 40
    t0 = 1 / (1 + p * xmax)
    s = np.cos(np.linspace(0, np.pi, nodes))
    t = t0 + (s + 1) / 2 * (1 - t0)
    x = (1 / t - 1) / p
    y = np.array([float(mp.erfc(mp.mpf(v)) * mp.exp(mp.mpf(v) ** 2)) for v in x]) / t
    V = np.polynomial.chebyshev.chebvander(s, degree)
    c, *_ = np.linalg.lstsq(V / y[:, None], np.ones_like(y), rcond=None)
    # check on a dense grid (reference: scipy erfcx, accurate to a few ulp)
    s2 = np.linspace(-1, 1, 20001)
    t2 = t0 + (s2 + 1) / 2 * (1 - t0)
    x2 = (1 / t2 - 1) / p
    rel = np.polynomial.chebyshev.chebval(s2, c) / (erfcx(x2) / t2) - 1
    return c, t0, float(np.abs(rel).max())


if __name__ == "__main__":
    c, e = fit32()
    print("FP32: p = %.9g, degree %d, max rel err (fp64 eval) %.3g, (fp32 Horner) %.3g"
          % (P32, DEG32, e, fp32_error(c)))
    print(", ".join("%.9gf" % v for v in c))
    c, t0, e = fit64()
    print("FP64: p = %.17g, degree %d, t0 = %.17g, max rel err %.3g" % (P64, DEG64, t0, e))
    print(",\n".join("%.17g" % v for v in c))
