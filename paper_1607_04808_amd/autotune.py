"""Autotune the launch shapes (fse_plan_autotune) on the standard workloads and
write the table that Plan() loads (tuning.json beside this file).

    python -m paper_1607_04808_amd.autotune [--out PATH] [--repeats R] [--only NAME ...]

Each workload is the seeded synthetic input of a measured configuration; the
timed unit is one set_points + eval, or set_points + eval_with_adjoint where the
configuration has an adjoint, on a plan with exactly that configuration's
parameters.  Runs on the GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

_HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(_HERE))

import workloads as W  # noqa: E402

from . import fse as F  # noqa: E402

L_UNIT = 1.0 + 2.0 ** -20

# name: (kernel, dtype, n, batch, (xi, rc, M, P), deltaL_rule, positions, adjoint); parameters
# None: chosen for a 1e-6 tolerance (fse_choose_params, bounding-cube box); "blobs": the
# 64-blob cloud in its bounding cube with xi = 165, r_c = 3.93 / xi, M = 3.15 xi L
WORKLOADS = {
    "c1_f64": ("stokeslet", "f64", 1000, 1, None, 1, "cube", True),
    "headline_f32": ("stokeslet", "f32", 1_000_000, 1, (75.0, 0.0476, 236, 11), 0, "cube", True),
    "headline_f64": ("stokeslet", "f64", 1_000_000, 1, (80.0, 0.06075, 304, 18), 0, "cube", True),
    "batched16_f32": ("stokeslet", "f32", 1_000_000, 16, (75.0, 0.0476, 236, 11), 0, "cube", True),
    "c4_rotlet16_f32": ("rotlet", "f32", 1_000_000, 16, (80.0, 0.04725, 246, 12), 0, "cube", False),
    "c2_f32": ("stokeslet", "f32", 100_000, 1, (40.0, 0.0945, 124, 12), 0, "cube", True),
    "c2_f64": ("stokeslet", "f64", 100_000, 1, (40.0, 0.1215, 153, 20), 0, "cube", True),
    "c3_f32": ("stresslet", "f32", 200_000, 1, (30.0, 0.14, 240, 14), 1, "sphere", False),
    "c3_f64": ("stresslet", "f64", 200_000, 1, (40.0, 0.11, 300, 14), 1, "sphere", False),
    "c5_blobs4m_f32": ("stokeslet", "f32", 4_000_000, 1, "blobs", 0, "blobs", True),
}


def _inputs(name, kernel, n, batch, positions):
    seed = 1000 + sum(map(ord, name)) % 997
    if positions == "sphere":
        x, nrm = W.sphere_surface(n, seed)
        lo, L = (-L_UNIT,) * 3, 2.0 * L_UNIT
    elif positions == "blobs":
        import numpy as np
        x, nrm = W.gaussian_blobs(n, seed), None
        xs = np.asarray(x, np.float32).astype(np.float64)
        lo = tuple(float(v) for v in xs.min(axis=0))
        L = float((xs.max(axis=0) - xs.min(axis=0)).max()) * L_UNIT + 1e-6
    else:
        x, nrm = W.uniform_cube(n, seed), None
        lo, L = (0.0, 0.0, 0.0), L_UNIT
    bb = None if batch == 1 else batch
    a = W.normal_strengths(n, seed + 1, bb)
    b = None
    if kernel == "stresslet":
        b = nrm if batch == 1 else [nrm] * batch
    w = W.normal_strengths(n, seed + 2, bb)
    return x, a, b, w, lo, L


def tune(name, repeats=3):
    import numpy as np
    import torch
    kernel, dtype, n, batch, prm, rule, positions, adjoint = WORKLOADS[name]
    td = torch.float32 if dtype == "f32" else torch.float64
    x, a, b, w, lo, L = _inputs(name, kernel, n, batch, positions)
    t = lambda v: None if v is None else torch.tensor(np.asarray(v), dtype=td, device="cuda:0")
    if prm is None:
        params = F.plan_for(kernel, t(x), t(a), t(b), tol=1e-6).params
        prm = (params.xi, params.rc, params.M, params.P)
    else:
        if prm == "blobs":
            xi = 165.0
            prm = (xi, 3.93 / xi, int(math.ceil(3.15 * xi * L)), 12)
        params = F.make_params(*prm, box_lo=lo, L=L, deltaL_rule=rule)
    plan = F.Plan(kernel, dtype, params, batch=batch, nmax=n, tuned=False)
    try:
        default = plan.tuning()
        xt, at, bt, wt = t(x), t(a), t(b), t(w if adjoint else None)

        def run(reps):
            torch.cuda.synchronize()
            t0 = time.time()
            for _ in range(reps):
                plan.set_points(xt, validate=False)
                if adjoint:
                    plan.eval_with_adjoint(at, wt)
                else:
                    plan.eval(at, bt)
            torch.cuda.synchronize()
            return (time.time() - t0) / reps * 1e3

        plan.set_points(xt)
        run(1)
        ms_default = run(repeats)
        best = plan.autotune(xt, at, bt, wt, repeats=repeats)
        ms_tuned = run(repeats)
        return dict(name=name, kernel=kernel, dtype=dtype, batch=batch, P=int(prm[3]), Mt=plan.geometry.Mt, n=n,
                    tuning=best, default=default, ms_default=round(ms_default, 3), ms_tuned=round(ms_tuned, 3))
    finally:
        plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=F.TUNING_PATH)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    names = args.only or list(WORKLOADS)
    entries = []
    for name in names:
        e = tune(name, args.repeats)
        print(json.dumps(e), flush=True)
        entries.append(e)
    import torch
    out = {"command": "python -m paper_1607_04808_amd.autotune --repeats %d" % args.repeats,
           "device": torch.cuda.get_device_name(0), "entries": entries}
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
