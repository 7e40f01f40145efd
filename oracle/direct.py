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


def build(force: bool = True) -> str:
    """Compile ``direct.c`` with gcc (FP64, OpenMP) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_LIB)
            d, i64, vp, i = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
            L.oracle_direct.argtypes = [i, i64, vp, vp, vp, i64, vp, vp, vp]
            L.oracle_real_trunc.argtypes = [i, d, d, i64, vp, vp, vp, i64, vp, vp, vp]
            L.oracle_fourier_dir.argtypes = [i, d, i64, vp, vp, vp, i64, vp, vp, vp]
            L.oracle_grad_direct.argtypes = [i, i64, vp, vp, vp, i64, vp, vp]
            L.oracle_grad_real_trunc.argtypes = [i, d, d, i64, vp, vp, vp, i64, vp, vp]
            for fn in ("oracle_direct", "oracle_real_trunc", "oracle_fourier_dir",
                       "oracle_grad_direct", "oracle_grad_real_trunc", "oracle_num_threads"):
                getattr(L, fn).restype = ctypes.c_int
            _lib = L
    return _lib


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


def rel_errors(u, ref):
    """(relative max-norm, relative RMS) of u against ref over all components.

    max-norm: max|u - ref| / max|ref|;  RMS: ||u - ref||_2 / ||ref||_2.
    """
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = u - ref
    return float(np.abs(d).max() / np.abs(ref).max()), float(np.linalg.norm(d) / np.linalg.norm(ref))
