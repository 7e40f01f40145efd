"""TEST INFRASTRUCTURE ONLY: ctypes binding of the oracle's FP64 C sums.

The functions mirror ``direct.c``; see that file for the formulas and the
paper passages they follow.  Arrays are converted to C-contiguous float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

KERNELS = {"stokeslet": 0, "stresslet": 1, "rotlet": 2}


def build(force: bool = True, path: str | None = None, native: bool = False) -> str:
    """Compile ``direct.c`` with gcc (FP64, OpenMP) into ``liboracle.so`` (or `path`).

    The default build targets x86-64-v3, so the library built here also runs on
    the GPU host; ``native=True`` compiles for the machine it runs on (the CPU
    baseline's timing build, made on that host)."""
    out = path or _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=native" if native else "-march=x86-64-v3", "-fopenmp", "-fPIC",
               "-shared", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


def use_library(path: str) -> None:
    """Load the oracle from `path` (a build of the same source) for the rest of the process."""
    global _lib
    with _lock:
        _lib = _load(path)


def _load(path):
    L = ctypes.CDLL(path)
    d, i64, vp, i = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    L.oracle_direct.argtypes = [i, i64, vp, vp, vp, i64, vp, vp, vp]
    L.oracle_real_trunc.argtypes = [i, d, d, i64, vp, vp, vp, i64, vp, vp, vp]
    L.oracle_fourier_dir.argtypes = [i, d, i64, vp, vp, vp, i64, vp, vp, vp]
    L.oracle_grad_direct.argtypes = [i, i64, vp, vp, vp, i64, vp, vp]
    L.oracle_grad_real_trunc.argtypes = [i, d, d, i64, vp, vp, vp, i64, vp, vp]
    L.oracle_set_threads.argtypes = [i]
    L.oracle_set_threads.restype = None
    for fn in ("oracle_direct", "oracle_real_trunc", "oracle_fourier_dir",
               "oracle_grad_direct", "oracle_grad_real_trunc", "oracle_num_threads"):
        getattr(L, fn).restype = ctypes.c_int
    return L


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            _lib = _load(_LIB)
    return _lib


def set_threads(t: int) -> None:
    """OpenMP threads of the sums (t <= 0: all cores)."""
    lib().oracle_set_threads(int(t))


def num_threads() -> int:
    return lib().oracle_num_threads()


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _targets(x, targets, y):
    """Resolve target points: indices into the sources (self excluded) or free points."""
    if y is not None:
        y = _c(y)
        skip = np.full(len(y), -1, dtype=np.int64)
        return y, skip
    if targets is None:
        targets = np.arange(len(x), dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    return np.ascontiguousarray(x[targets]), targets


def _kid(kernel):
    return KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def _check(rc):
    if rc == 2:
        raise ValueError("oracle: coincident distinct points (undefined sum)")
    if rc != 0:
        raise ValueError("oracle: invalid arguments")


def direct(kernel, x, a, b=None, targets=None, y=None):
    """u(y_t) = sum_{n != t} G(y_t - x_n) . src_n  (eq. usumfree / eq. usum), FP64."""
    x, a, b = _c(x), _c(a), _c(b)
    yy, skip = _targets(x, targets, y)
    out = np.zeros((len(yy), 3))
    _check(lib().oracle_direct(_kid(kernel), len(x), _p(x), _p(a), _p(b), len(yy), _p(yy),
                               _p(skip), _p(out)))
    return out


def real_trunc(kernel, xi, rc, x, a, b=None, targets=None, y=None):
    """Real-space sum over 0 < |r| <= rc (Section 6), FP64 brute force."""
    x, a, b = _c(x), _c(a), _c(b)
    yy, skip = _targets(x, targets, y)
    out = np.zeros((len(yy), 3))
    _check(lib().oracle_real_trunc(_kid(kernel), float(xi), float(rc), len(x), _p(x), _p(a),
                                   _p(b), len(yy), _p(yy), _p(skip), _p(out)))
    return out


def fourier_dir(kernel, xi, x, a, b=None, targets=None, y=None):
    """sum_n G^F(y_t - x_n) . src_n including the self value G^F(0), FP64."""
    x, a, b = _c(x), _c(a), _c(b)
    yy, skip = _targets(x, targets, y)
    out = np.zeros((len(yy), 3))
    _check(lib().oracle_fourier_dir(_kid(kernel), float(xi), len(x), _p(x), _p(a), _p(b),
                                    len(yy), _p(yy), _p(skip), _p(out)))
    return out


def grad_direct(kernel, x, f, w, targets=None):
    """dL/dx_p of L = sum_m w_m . u(x_m) for the direct sum (S or Omega)."""
    x, f, w = _c(x), _c(f), _c(w)
    if targets is None:
        targets = np.arange(len(x), dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    out = np.zeros((len(targets), 3))
    _check(lib().oracle_grad_direct(_kid(kernel), len(x), _p(x), _p(f), _p(w), len(targets),
                                    _p(targets), _p(out)))
    return out


def grad_real_trunc(kernel, xi, rc, x, f, w, targets=None):
    """dL/dx_p of the truncated real-space part of L (S or Omega)."""
    x, f, w = _c(x), _c(f), _c(w)
    if targets is None:
        targets = np.arange(len(x), dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    out = np.zeros((len(targets), 3))
    _check(lib().oracle_grad_real_trunc(_kid(kernel), float(xi), float(rc), len(x), _p(x),
                                        _p(f), _p(w), len(targets), _p(targets), _p(out)))
    return out


def stresslet_adjoint(x, q, nrm, w, targets=None, chunk=4096):
    """dL/dq and dL/dn of L = sum_m w_m . u(x_m) for the stresslet direct sum.

    u_j(x_m) = sum_{n != m} T_jlm(x_m - x_n) q_l(n) n_m(n) with
    T_jlm(r) = -6 r_j r_l r_m / |r|^5 (eq. def_stresslet).  L is linear in q and
    in n, so at source b: D_lm = sum_{a != b} w_j(a) T_jlm(x_a - x_b) and
    dL/dq_l(b) = D_lm n_m(b), dL/dn_m(b) = D_lm q_l(b).  Plain numpy, FP64, for
    the given target indices b (all by default).
    """
    x, q, nrm, w = (np.asarray(a, dtype=np.float64) for a in (x, q, nrm, w))
    if targets is None:
        targets = np.arange(len(x), dtype=np.int64)
    dq = np.zeros((len(targets), 3))
    dn = np.zeros((len(targets), 3))
    for k, b in enumerate(targets):
        for s0 in range(0, len(x), chunk):
            r = x[s0:s0 + chunk] - x[b]                     # x_a - x_b
            ww = w[s0:s0 + chunk]
            r2 = np.einsum("ij,ij->i", r, r)
            own = (np.arange(s0, s0 + len(r)) == b)
            if np.any((r2 == 0.0) & ~own):
                raise ValueError("oracle: coincident distinct points (undefined sum)")
            r2[own] = 1.0
            c = -6.0 * np.einsum("ij,ij->i", r, ww) / r2 ** 2.5  # w_j r_j times -6/|r|^5
            c[own] = 0.0
            D = np.einsum("i,ij,ik->jk", c, r, r)               # sum_a c_a r_l r_m
            dq[k] += D @ nrm[b]
            dn[k] += D @ q[b]
    return dq, dn


def rel_errors(u, ref):
    """(relative max-norm, relative RMS) of u against ref over all components.

    max-norm: max|u - ref| / max|ref|;  RMS: ||u - ref||_2 / ||ref||_2.
    """
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = u - ref
    return float(np.abs(d).max() / np.abs(ref).max()), float(np.linalg.norm(d) / np.linalg.norm(ref))
