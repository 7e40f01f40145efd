"""Python binding of libfse (include/fse.h): argument marshalling only.

Every step of the evaluation runs in the HIP library; torch supplies device
memory and the current stream.  There is no CPU fallback: without the built
library every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libfse.so")

KERNELS = {"stokeslet": 0, "stresslet": 1, "rotlet": 2}
DTYPES = {"f32": 0, "f64": 1}
STATUS = {0: "FSE_OK", 1: "FSE_EINVAL", 2: "FSE_ERANGE", 3: "FSE_ENOMEM", 4: "FSE_EHIP",
          5: "FSE_EUNSUPPORTED", 6: "FSE_ESTATE"}
EXPORTS = ("fse_geometry", "fse_plan_create", "fse_plan_geometry", "fse_plan_set_stream",
           "fse_set_points", "fse_eval", "fse_eval_parts", "fse_eval_adjoint", "fse_plan_multiplier",
           "fse_plan_workspace", "fse_plan_grid", "fse_plan_set_timing", "fse_plan_timings",
           "fse_stage_name", "fse_plan_destroy", "fse_status_string", "fse_last_error", "fse_eval_noalloc",
           "fse_error_estimates", "fse_choose_params", "fse_bounding_box", "fse_set_targets", "fse_eval_targets",
           "fse_eval_adjoint_stresslet", "fse_freespace_solve",
           "fse_plan_get_tuning", "fse_plan_set_tuning", "fse_plan_autotune", "fse_plan_bins",
           "fse_precompute_cache_stats", "fse_eval_with_adjoint")
NOALLOC_MAX_BYTES = 64 << 20  # FSE_NOALLOC_MAX_BYTES
NSTAGES = 12


class FseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("xi", ctypes.c_double), ("rc", ctypes.c_double), ("M", ctypes.c_int32),
                ("P", ctypes.c_int32), ("box_lo", ctypes.c_double * 3), ("L", ctypes.c_double),
                ("deltaL_rule", ctypes.c_int32), ("Mt", ctypes.c_int32), ("C", ctypes.c_double),
                ("periodic", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("bin_side", ctypes.c_int32), ("real_queue", ctypes.c_int32), ("real_queue_grad", ctypes.c_int32),
                ("real_waves", ctypes.c_int32), ("fft_lines", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GeometryC(ctypes.Structure):
    _fields_ = [("Mt", ctypes.c_int32), ("n_fft", ctypes.c_int32), ("Mg", ctypes.c_int32),
                ("ncell", ctypes.c_int32), ("h", ctypes.c_double), ("d", ctypes.c_double),
                ("m", ctypes.c_double), ("eta", ctypes.c_double), ("alpha", ctypes.c_double),
                ("Lt", ctypes.c_double), ("R", ctypes.c_double), ("deltaL", ctypes.c_double),
                ("kinf", ctypes.c_double), ("cell", ctypes.c_double), ("x0", ctypes.c_double * 3),
                ("radices", ctypes.c_int32 * 8)]


_lock = threading.Lock()
_lib = None


def lib():
    """Load libfse.so; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libfse.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
            L.fse_geometry.argtypes = [ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(GeometryC)]
            L.fse_plan_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params), i32, i64, vp,
                                          ctypes.POINTER(vp)]
            L.fse_plan_geometry.argtypes = [vp, ctypes.POINTER(GeometryC)]
            L.fse_plan_set_stream.argtypes = [vp, vp]
            L.fse_set_points.argtypes = [vp, i64, vp, i32]
            L.fse_eval.argtypes = [vp, vp, vp, vp]
            L.fse_eval_parts.argtypes = [vp, vp, vp, vp, vp]
            L.fse_eval_adjoint.argtypes = [vp, vp, vp, vp, vp, i32]
            L.fse_eval_adjoint_stresslet.argtypes = [vp, vp, vp, vp, vp, vp]
            L.fse_eval_with_adjoint.argtypes = [vp, vp, vp, vp, vp, vp]
            L.fse_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
            L.fse_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
            L.fse_plan_autotune.argtypes = [vp, i64, vp, vp, vp, vp, i32, ctypes.POINTER(Tuning)]
            L.fse_freespace_solve.argtypes = [i32, ctypes.c_int, i32, ctypes.c_double, i32, vp, vp, vp]
            L.fse_set_targets.argtypes = [vp, i64, vp, i32]
            L.fse_eval_targets.argtypes = [vp, vp, vp, vp, vp]
            L.fse_plan_multiplier.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
            L.fse_plan_workspace.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
            L.fse_plan_grid.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
            L.fse_plan_bins.argtypes = [vp, ctypes.POINTER(i32), vp, vp, vp, vp, vp, vp]
            L.fse_precompute_cache_stats.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i64),
                                                     ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(i32)]
            L.fse_plan_set_timing.argtypes = [vp, i32]
            L.fse_plan_timings.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
            L.fse_stage_name.argtypes = [i32]
            L.fse_stage_name.restype = ctypes.c_char_p
            L.fse_eval_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params), i32, i64, vp, vp, vp,
                                           vp, i32, vp]
            dp = ctypes.POINTER(ctypes.c_double)
            L.fse_error_estimates.argtypes = [ctypes.c_int, ctypes.POINTER(Params), ctypes.c_double, dp, dp]
            L.fse_choose_params.argtypes = [ctypes.c_int, ctypes.c_int, i64, dp, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.POINTER(Params)]
            L.fse_bounding_box.argtypes = [ctypes.c_int, i64, vp, vp, dp, dp]
            L.fse_plan_destroy.argtypes = [vp]
            L.fse_plan_destroy.restype = None
            L.fse_status_string.argtypes = [ctypes.c_int]
            L.fse_status_string.restype = ctypes.c_char_p
            L.fse_last_error.restype = ctypes.c_char_p
            for name in EXPORTS:
                if name not in ("fse_plan_destroy", "fse_status_string", "fse_last_error", "fse_stage_name"):
                    getattr(L, name).restype = ctypes.c_int
            _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise FseError(status, lib().fse_last_error().decode())


def make_params(xi, rc, M, P, box_lo=(0.0, 0.0, 0.0), L=1.0, deltaL_rule=0, Mt=0, C=0.0, periodic=0) -> Params:
    p = Params()
    p.xi, p.rc, p.M, p.P = float(xi), float(rc), int(M), int(P)
    for d in range(3):
        p.box_lo[d] = float(box_lo[d])
    p.L, p.deltaL_rule, p.Mt, p.C = float(L), int(deltaL_rule), int(Mt), float(C)
    p.periodic = int(periodic)
    return p


@dataclass
class Geometry:
    Mt: int
    n_fft: int
    Mg: int
    ncell: int
    h: float
    d: float
    m: float
    eta: float
    alpha: float
    Lt: float
    R: float
    deltaL: float
    kinf: float
    cell: float
    x0: tuple
    radices: tuple

    @classmethod
    def from_c(cls, g: GeometryC):
        return cls(g.Mt, g.n_fft, g.Mg, g.ncell, g.h, g.d, g.m, g.eta, g.alpha, g.Lt, g.R, g.deltaL,
                   g.kinf, g.cell, tuple(g.x0), tuple(r for r in g.radices if r))


def _kid(kernel):
    return KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def geometry(kernel, params: Params) -> Geometry:
    """Derived geometry (host only, no GPU needed)."""
    g = GeometryC()
    _check(lib().fse_geometry(_kid(kernel), ctypes.byref(params), ctypes.byref(g)))
    return Geometry.from_c(g)


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """An FSE plan on the current HIP device (see fse_plan_create)."""

    def __init__(self, kernel, dtype, params: Params, batch=1, nmax=2, tuned=True):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libfse needs a HIP device")
        self.kernel = kernel if isinstance(kernel, str) else list(KERNELS)[kernel]
        self.dtype = dtype
        self.tdtype = torch.float32 if dtype == "f32" else torch.float64
        self.batch = int(batch)
        self.nmax = int(nmax)
        self.params = params
        self._h = ctypes.c_void_p()
        _check(lib().fse_plan_create(_kid(kernel), DTYPES[dtype], ctypes.byref(params), self.batch,
                                     self.nmax, _stream_ptr(), ctypes.byref(self._h)))
        g = GeometryC()
        _check(lib().fse_plan_geometry(self._h, ctypes.byref(g)))
        self.geometry = Geometry.from_c(g)
        self.n = 0
        self.generation = 0
        if tuned:
            t = tuning_for(self.kernel, dtype, self.batch, params.P, self.geometry.Mt, self.nmax)
            if t is not None:
                self.set_tuning(t)

    def close(self):
        if self._h:
            lib().fse_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(lib().fse_plan_set_stream(self._h, _stream_ptr()))

    def _prep(self, t, shape):
        torch = _torch()
        if t.device.type != "cuda":
            raise ValueError("expected a device tensor")
        t = t.to(self.tdtype).contiguous()
        if tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t

    def set_points(self, x, validate=True):
        x = self._prep(x, (x.shape[0], 3))
        self._sync_stream()
        self._x = x  # keep alive while the plan may read it
        _check(lib().fse_set_points(self._h, x.shape[0], _ptr(x), 1 if validate else 0))
        self.n = x.shape[0]
        self.generation += 1
        return self

    def _src_shape(self):
        return (self.batch, self.n, 3)

    def eval(self, a, b=None, out=None):
        torch = _torch()
        a = self._prep(a, self._src_shape())
        b = None if b is None else self._prep(b, self._src_shape())
        if out is None:
            out = torch.empty(self._src_shape(), dtype=self.tdtype, device=a.device)
        self._sync_stream()
        _check(lib().fse_eval(self._h, _ptr(a), _ptr(b), _ptr(out)))
        self.generation += 1
        return out

    def set_targets(self, y, validate=True):
        """Separate targets (fse_set_targets)."""
        y = self._prep(y, (y.shape[0], 3))
        self._sync_stream()
        self._y = y
        _check(lib().fse_set_targets(self._h, y.shape[0], _ptr(y), 1 if validate else 0))
        self.nt = y.shape[0]
        return self

    def eval_targets(self, a, b=None, parts=False):
        """u at the targets (fse_eval_targets); parts=True gives (u^R, u^F)."""
        torch = _torch()
        a = self._prep(a, self._src_shape())
        b = None if b is None else self._prep(b, self._src_shape())
        shape = (self.batch, self.nt, 3)
        u = torch.empty(shape, dtype=self.tdtype, device=a.device)
        uF = torch.empty(shape, dtype=self.tdtype, device=a.device) if parts else None
        self._sync_stream()
        _check(lib().fse_eval_targets(self._h, _ptr(a), _ptr(b), _ptr(u), _ptr(uF)))
        self.generation += 1
        return (u, uF) if parts else u

    def eval_parts(self, a, b=None):
        torch = _torch()
        a = self._prep(a, self._src_shape())
        b = None if b is None else self._prep(b, self._src_shape())
        uR = torch.empty(self._src_shape(), dtype=self.tdtype, device=a.device)
        uF = torch.empty_like(uR)
        self._sync_stream()
        _check(lib().fse_eval_parts(self._h, _ptr(a), _ptr(b), _ptr(uR), _ptr(uF)))
        self.generation += 1
        return uR, uF

    def adjoint(self, f, w, want_df=True, want_dx=True, recompute=True):
        torch = _torch()
        f = self._prep(f, self._src_shape())
        w = self._prep(w, self._src_shape())
        df = torch.empty(self._src_shape(), dtype=self.tdtype, device=f.device) if want_df else None
        dx = torch.empty((self.n, 3), dtype=self.tdtype, device=f.device) if want_dx else None
        self._sync_stream()
        _check(lib().fse_eval_adjoint(self._h, _ptr(f), _ptr(w), _ptr(df), _ptr(dx), 1 if recompute else 0))
        self.generation += 1
        return df, dx

    def eval_with_adjoint(self, f, w):
        """(u, dL/df, dL/dx) for L = sum w . u in one call (fse_eval_with_adjoint)."""
        torch = _torch()
        f = self._prep(f, self._src_shape())
        w = self._prep(w, self._src_shape())
        u = torch.empty(self._src_shape(), dtype=self.tdtype, device=f.device)
        df = torch.empty_like(u)
        dx = torch.empty((self.n, 3), dtype=self.tdtype, device=f.device)
        self._sync_stream()
        _check(lib().fse_eval_with_adjoint(self._h, _ptr(f), _ptr(w), _ptr(u), _ptr(df), _ptr(dx)))
        self.generation += 1
        return u, df, dx

    def adjoint_stresslet(self, q, nrm, w):
        """(dL/dq, dL/dn) of L = sum w . u for a stresslet plan (fse_eval_adjoint_stresslet)."""
        torch = _torch()
        q = self._prep(q, self._src_shape())
        nrm = self._prep(nrm, self._src_shape())
        w = self._prep(w, self._src_shape())
        dq = torch.empty(self._src_shape(), dtype=self.tdtype, device=q.device)
        dn = torch.empty_like(dq)
        self._sync_stream()
        _check(lib().fse_eval_adjoint_stresslet(self._h, _ptr(q), _ptr(nrm), _ptr(w), _ptr(dq), _ptr(dn)))
        self.generation += 1
        return dq, dn

    def multiplier(self):
        Mp = self.geometry.Mt + 1
        out = np.empty((Mp, Mp, Mp), dtype=np.float64)
        self._sync_stream()
        _check(lib().fse_plan_multiplier(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def grid(self, which):
        """Host copy (float64) of the spread grid (0) or the scaled inverse-transformed grid (1)."""
        Mt = self.geometry.Mt
        nc = (6 if self.kernel == "stresslet" else 3) if which == 0 else 3
        out = np.empty((self.batch, nc, Mt, Mt, Mt), dtype=np.float64)
        _check(lib().fse_plan_grid(self._h, int(which), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def bins(self):
        """Host copies of the binning of the points last set (fse_plan_bins): a dict
        with nbins, perm_s, bpack_s, coff_s (n, 3), tile_start, perm_r, cell_start."""
        nb = ctypes.c_int32(0)
        self._sync_stream()
        _check(lib().fse_plan_bins(self._h, ctypes.byref(nb), None, None, None, None, None, None))
        n, nc = self.n, self.geometry.ncell
        out = dict(nbins=nb.value, perm_s=np.empty(n, np.int32), bpack_s=np.empty(n, np.int32),
                   coff_s=np.empty((n, 3), np.float64), tile_start=np.empty(nb.value ** 3 + 1, np.int32),
                   perm_r=np.empty(n, np.int32), cell_start=np.empty(nc ** 3 + 1, np.int32))
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().fse_plan_bins(self._h, ctypes.byref(nb), p(out["perm_s"]), p(out["bpack_s"]), p(out["coff_s"]),
                                   p(out["tile_start"]), p(out["perm_r"]), p(out["cell_start"])))
        return out

    def set_timing(self, on=True):
        _check(lib().fse_plan_set_timing(self._h, 1 if on else 0))

    def timings(self):
        """{stage: (total ms, launch groups)} since the last call (synchronises)."""
        ms = (ctypes.c_double * NSTAGES)()
        cnt = (ctypes.c_int64 * NSTAGES)()
        _check(lib().fse_plan_timings(self._h, ms, cnt))
        return {lib().fse_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(NSTAGES)}

    def tuning(self):
        t = Tuning()
        _check(lib().fse_plan_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, t):
        """Apply a tuning dict (fse_plan_set_tuning); points must be set again.
        Knobs the dict leaves out keep their current values."""
        cur = self.tuning()
        tt = Tuning(**{k: int(t.get(k, cur[k])) for k, _ in Tuning._fields_})
        _check(lib().fse_plan_set_tuning(self._h, ctypes.byref(tt)))
        self.generation += 1

    def autotune(self, x, a, b=None, w=None, repeats=3):
        """fse_plan_autotune on this workload; leaves the points set; returns the tuning."""
        x = self._prep(x, (x.shape[0], 3))
        n = x.shape[0]
        self.n = n
        a = self._prep(a, self._src_shape())
        b = None if b is None else self._prep(b, self._src_shape())
        w = None if w is None else self._prep(w, self._src_shape())
        self._sync_stream()
        t = Tuning()
        _check(lib().fse_plan_autotune(self._h, n, _ptr(x), _ptr(a), _ptr(b), _ptr(w), int(repeats),
                                       ctypes.byref(t)))
        self._x = x
        self.generation += 1
        return t.as_dict()

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        _check(lib().fse_plan_workspace(self._h, ctypes.byref(b)))
        return b.value


def freespace_solve(f, h, family="harmonic"):
    """fse_freespace_solve: u = G * f on the grid (G = 1/r harmonic, r biharmonic).
    f: device tensor (M, M, M) or (ncomp, M, M, M) indexed [z][y][x]; returns u alike."""
    torch = _torch()
    dtype = "f32" if f.dtype == torch.float32 else "f64"
    single = f.dim() == 3
    g = (f[None] if single else f).contiguous()
    M = g.shape[-1]
    if tuple(g.shape[1:]) != (M, M, M):
        raise ValueError("f must be (M, M, M) or (ncomp, M, M, M)")
    u = torch.empty_like(g)
    fam = {"biharmonic": 0, "harmonic": 1}[family]
    _check(lib().fse_freespace_solve(fam, DTYPES[dtype], M, float(h), g.shape[0], _ptr(g), _ptr(u), _stream_ptr()))
    return u[0] if single else u


def error_estimates(kernel, params: Params, Q):
    """(est_real, est_fourier): Tables est_real and est_fourier (absolute RMS), host only."""
    er, ef = ctypes.c_double(), ctypes.c_double()
    _check(lib().fse_error_estimates(_kid(kernel), ctypes.byref(params), float(Q), ctypes.byref(er),
                                     ctypes.byref(ef)))
    return er.value, ef.value


def choose_params(kernel, dtype, n, box_lo, L, tol, Q, u_rms=0.0) -> Params:
    """fse_choose_params (Section 8.2): parameters for a relative max-norm tolerance, host only."""
    p = Params()
    lo = (ctypes.c_double * 3)(*[float(v) for v in box_lo])
    _check(lib().fse_choose_params(_kid(kernel), DTYPES[dtype], int(n), lo, float(L), float(tol), float(Q),
                                   float(u_rms), ctypes.byref(p)))
    return p


def bounding_box(x):
    """fse_bounding_box: (box_lo, L) of the bounding cube of the device points x (n, 3)."""
    torch = _torch()
    dtype = "f32" if x.dtype == torch.float32 else "f64"
    x = x.contiguous()
    lo = (ctypes.c_double * 3)()
    L = ctypes.c_double()
    _check(lib().fse_bounding_box(DTYPES[dtype], x.shape[0], _ptr(x), _stream_ptr(), lo, ctypes.byref(L)))
    return tuple(lo), L.value


def eval_noalloc(kernel, dtype, params: Params, x, a, b=None, out=None, batch=1, validate=False):
    """fse_eval_noalloc: one evaluation with no device allocation inside the library
    (workspace from its static per-GPU scratch array).  `out` may be preallocated."""
    torch = _torch()
    td = torch.float32 if dtype == "f32" else torch.float64
    n = x.shape[0]
    shape = (int(batch), n, 3)
    x = x.to(td).contiguous()
    a = a.to(td).contiguous().reshape(shape)
    b = None if b is None else b.to(td).contiguous().reshape(shape)
    if out is None:
        out = torch.empty(shape, dtype=td, device=x.device)
    _check(lib().fse_eval_noalloc(_kid(kernel), DTYPES[dtype], ctypes.byref(params), int(batch), n, _ptr(x),
                                  _ptr(a), _ptr(b), _ptr(out), 1 if validate else 0, _stream_ptr()))
    return out


def precompute_cache_stats():
    """fse_precompute_cache_stats: dict of hits, misses, bytes and entries."""
    h, m, b, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_int32()
    _check(lib().fse_precompute_cache_stats(ctypes.byref(h), ctypes.byref(m), ctypes.byref(b), ctypes.byref(e)))
    return dict(hits=h.value, misses=m.value, bytes=b.value, entries=e.value)


TUNING_PATH = os.path.join(_HERE, "tuning.json")
_TUNING = None


def tuning_for(kernel, dtype, batch, P, Mt, n):
    """The autotuner's entry for the closest recorded workload (same kernel, dtype,
    batch and P; grid size and point count within a factor of 2), or None."""
    global _TUNING
    if _TUNING is None:
        try:
            import json
            with open(TUNING_PATH) as fh:
                _TUNING = json.load(fh).get("entries", [])
        except (OSError, ValueError):
            _TUNING = []
    import math
    best, dist = None, None
    for e in _TUNING:
        if (e["kernel"], e["dtype"], e["batch"], e["P"]) != (kernel, dtype, batch, P):
            continue
        d = abs(math.log(e["Mt"] / Mt)) + abs(math.log(e["n"] / max(n, 2)))
        if abs(math.log(e["Mt"] / Mt)) <= math.log(2) and abs(math.log(e["n"] / max(n, 2))) <= math.log(2) \
                and (dist is None or d < dist):
            best, dist = e["tuning"], d
    return best


def _autograd():
    torch = _torch()

    class FSEFunction(torch.autograd.Function):
        """u = FSE sum of f at x; backward gives dL/dx and dL/df (stokeslet, rotlet)."""

        @staticmethod
        def forward(ctx, x, f, plan: Plan):
            plan.set_points(x.detach())
            u = plan.eval(f.detach())
            ctx.plan = plan
            ctx.gen = plan.generation
            ctx.save_for_backward(x, f)
            return u.reshape(f.shape)

        @staticmethod
        def backward(ctx, gu):
            x, f = ctx.saved_tensors
            plan = ctx.plan
            recompute = plan.generation != ctx.gen
            if recompute:
                plan.set_points(x.detach())
            df, dx = plan.adjoint(f.detach(), gu.detach(), want_df=ctx.needs_input_grad[1],
                                  want_dx=ctx.needs_input_grad[0], recompute=recompute)
            return (None if dx is None else dx.reshape(x.shape),
                    None if df is None else df.reshape(f.shape), None)

    return FSEFunction


def _autograd_stresslet():
    torch = _torch()

    class FSEStressletFunction(torch.autograd.Function):
        """u = FSE stresslet sum of (q, n) at x; backward gives dL/dq and dL/dn."""

        @staticmethod
        def forward(ctx, x, q, nrm, plan: Plan):
            plan.set_points(x.detach())
            u = plan.eval(q.detach(), nrm.detach())
            ctx.plan = plan
            ctx.gen = plan.generation
            ctx.save_for_backward(x, q, nrm)
            return u.reshape(q.shape)

        @staticmethod
        def backward(ctx, gu):
            x, q, nrm = ctx.saved_tensors
            if ctx.needs_input_grad[0]:
                raise NotImplementedError("dL/dx of the stresslet sum is not implemented")
            plan = ctx.plan
            if plan.generation != ctx.gen:
                plan.set_points(x.detach())
            dq, dn = plan.adjoint_stresslet(q.detach(), nrm.detach(), gu.detach())
            return None, dq.reshape(q.shape), dn.reshape(nrm.shape), None

    return FSEStressletFunction


_FN = None
_FNT = None


def fse_sum(x, f, plan: Plan, nrm=None):
    """Differentiable FSE sum u(x_m) = sum_{n != m} G(x_m - x_n) f_n (stokeslet or
    rotlet plan: gradients in x and f), or, with the normals nrm, the stresslet sum
    of (q = f, n) (gradients in q and n)."""
    global _FN, _FNT
    if nrm is not None:
        if _FNT is None:
            _FNT = _autograd_stresslet()
        return _FNT.apply(x, f, nrm, plan)
    if _FN is None:
        _FN = _autograd()
    return _FN.apply(x, f, plan)


# ---------------------------------------------------------------------------
# Tolerance-driven sums: the box is the points' bounding cube, the parameters
# come from fse_choose_params, and the scale u_rms it needs comes from one coarse
# evaluation (relative tolerance 1e-3) of the same sum.  Plans are cached by
# kernel, dtype, batch, size and parameters.
# ---------------------------------------------------------------------------
_PLANS = {}
_PLAN_CACHE = 4


def _cached_plan(kernel, dtype, params: Params, batch, n):
    key = (kernel, dtype, batch, n, params.xi, params.rc, params.M, params.P, tuple(params.box_lo), params.L,
           params.Mt, params.deltaL_rule)
    plan = _PLANS.get(key)
    if plan is None:
        while len(_PLANS) >= _PLAN_CACHE:
            _PLANS.pop(next(iter(_PLANS))).close()
        plan = Plan(kernel, dtype, params, batch=batch, nmax=n)
        _PLANS[key] = plan
    return plan


def _source_norm(a, b):
    """Q of eq. Q_stokeslet (sum |f|^2) or eq. Q_stresslet (sum |q|^2 |n|^2), summed over the batch."""
    if b is None:
        return float((a.double() * a.double()).sum())
    return float(((a.double() ** 2).sum(-1) * (b.double() ** 2).sum(-1)).sum())


def plan_for(kernel, x, a, b=None, tol=1e-6, dtype=None, u_rms=None):
    """The cached plan fse_choose_params picks for these points and sources (and the points set)."""
    torch = _torch()
    if dtype is None:
        dtype = "f32" if x.dtype == torch.float32 else "f64"
    n = x.shape[0]
    batch = 1 if a.dim() == 2 else a.shape[0]
    box_lo, L = bounding_box(x.detach().to(torch.float32 if dtype == "f32" else torch.float64))
    Q = _source_norm(a.detach(), None if b is None else b.detach()) / batch
    if u_rms is None:
        coarse = _cached_plan(kernel, dtype, choose_params(kernel, dtype, n, box_lo, L, 1e-3, Q), batch, n)
        coarse.set_points(x.detach())
        uc = coarse.eval(a.detach(), None if b is None else b.detach())
        u_rms = float((uc.double() ** 2).sum(-1).mean().sqrt())
    prm = choose_params(kernel, dtype, n, box_lo, L, tol, Q, u_rms)
    return _cached_plan(kernel, dtype, prm, batch, n)


def stokeslet(x, f, tol=1e-6, dtype=None, u_rms=None):
    """u(x_m) = sum_{n != m} S(x_m - x_n) f_n at relative max-norm tolerance `tol`
    (differentiable in x and f).  f: (n, 3) or (batch, n, 3)."""
    plan = plan_for("stokeslet", x, f, None, tol, dtype, u_rms)
    return fse_sum(x, f, plan)


def rotlet(x, f, tol=1e-6, dtype=None, u_rms=None):
    """u(x_m) = sum_{n != m} Omega(x_m - x_n) f_n at relative tolerance `tol` (differentiable in x and f)."""
    plan = plan_for("rotlet", x, f, None, tol, dtype, u_rms)
    return fse_sum(x, f, plan)


def stresslet(x, q, nrm, tol=1e-6, dtype=None, u_rms=None):
    """u_j(x_m) = sum_{n != m} T_jlm(x_m - x_n) q_l n_m at relative tolerance `tol`
    (differentiable in q and n)."""
    plan = plan_for("stresslet", x, q, nrm, tol, dtype, u_rms)
    return fse_sum(x, q, plan, nrm)
