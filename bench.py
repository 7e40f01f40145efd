"""Benchmark: stokeslet targets/s at 1e-6 relative error, N = 1M, forward + adjoint,
FP32 form (headline) and FP64 form, on one MI355X.

One step = the whole hot path over one batch of synthetic input already in HBM:
bin/sort the points, forward FSE sum (spread, FFT, scale, IFFT, gather, real
space), and the adjoint (dL/df and dL/dx for L = sum_m w_m . u(x_m)).

Prints ONE JSON line.  `value` is the FP32-form forward+adjoint throughput;
the FP64 form, the batched form (16 force vectors over the same points),
forward-only rates, per-stage times, the roofline of the dominant kernel, the
FP32 form's error over all N against the FP64 form at the same (FP32-rounded)
inputs, and the CPU baseline (the oracle on a bounded target sample, which also
gives the sampled relative errors) are extra fields.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK = {"hbm_GBs": 8000.0, "f32_TFLOPs": 157.3, "f64_TFLOPs": 78.6}
MFMA_STAGES = {("f32", "spread")}  # (form, stage) pairs whose kernel is a matrix-core product

# Parameters per form (calibrated against the oracle):
# FP32 form: 1e-6 relative max-norm; FP64 form: 1e-10.
FORMS = {
    "f32": dict(xi=75.0, rc=0.0476, M=236, P=11, Mt=0, tol=1e-6),
    "f64": dict(xi=80.0, rc=0.06075, M=304, P=18, Mt=0, tol=1e-10),
}
N_DEFAULT = 1_000_000
L_BOX = 1.0 + 2.0 ** -20  # the unit cube, enlarged so FP32-rounded points stay inside


def cube_pair_cdf(r):
    """P(|x - y| <= r) for two uniform points in the unit cube, 0 <= r <= 1."""
    return 4 * math.pi / 3 * r ** 3 - 1.5 * math.pi * r ** 4 + 1.6 * r ** 5 - r ** 6 / 6


def stage_work(stage, geo, n, P, dtype, pairs, c_in=3, batch=1, fused=False):
    """Algorithmic (bytes, flops) of one launch group of a stage.  fused: the stage
    groups of fse_eval_with_adjoint (one spread of both source sets; the forward
    quadrature inside gather_grad; the forward real-space pairs inside real_grad)."""
    s = 4 if dtype == "f32" else 8
    Mt, nf = geo.Mt, geo.n_fft
    Mp = Mt + 1
    M3 = Mt ** 3
    nc = batch * c_in
    if stage == "fft_x":
        return nc * (M3 * s + Mp * Mt * Mt * 2 * s), None
    if stage == "fft_y":
        return nc * (Mp * Mt * Mt * 2 * s + Mp * nf * Mt * 2 * s), None
    if stage == "fft_z_scale":
        return batch * (c_in + 3) * Mp * nf * Mt * 2 * s + Mp ** 3 * s, None
    if stage == "fft_yinv":
        return batch * 3 * (Mp * nf * Mt * 2 * s + Mp * Mt * Mt * 2 * s), None
    if stage == "fft_xinv":
        return batch * 3 * (Mp * Mt * Mt * 2 * s + M3 * s), None
    if stage == "spread":
        # per point and window node: 1 weight product + c_in multiply-adds
        if fused:
            return 2 * nc * M3 * s + n * 7 * s, n * P ** 3 * (1 + 2 * 2 * c_in) * batch
        return nc * M3 * s + n * 4 * s, n * P ** 3 * (1 + 2 * c_in) * batch
    if stage == "gather":
        return batch * 3 * M3 * s + n * 4 * s, n * P ** 3 * (2 + 2 * 3) * batch
    if stage == "gather_grad":
        return 2 * batch * 3 * M3 * s, n * P ** 3 * batch * (2 + 12 + 6 + 6 + 6 + (8 if fused else 0))
    if stage in ("real", "real_grad"):
        # per interacting pair: r^2 (5), sqrt+div (2), exp (1), erfc (1), coefficients and
        # the 3x3 application (~25): counted as 34 flops; gradients about twice that
        per = 34 if stage == "real" else (104 if fused else 70)
        return None, pairs * per * batch
    return None, None


# Kernels behind each timed stage (FP32 / FP64 template names as rocprofv3 lists them)
# and the sources that define them, for the counter-based HBM traffic.
# Timed step: fse_eval_with_adjoint, so the spread stage is the six-component launch,
# gather_grad the sweeps of modes 3 and 2, and real_grad the pass that also sums u.
STAGE_KERNELS = {
    "real": (["k_real<{T}, 0, 1, false, false,"], "fse_real.hip"),
    "real_grad": (["k_real<{T}, 0, 1, true, true, true>"], "fse_real.hip"),
    "spread": (["k_spread<{T}, 6,", "k_spread_mfma<6,"], "fse_spread.hip"),
    "gather": (["k_gather_col<{T}, 0, "], "fse_spread.hip"),
    "gather_grad": (["k_gather_col<{T}, 3, ", "k_gather_col<{T}, 2, "], "fse_spread.hip"),
    "fft_x": (["k_fft_x<{T},"], "fse_fft.hip"),
    "fft_y": (["k_fft_y<{T},"], "fse_fft.hip"),
    "fft_z_scale": (["k_fft_z<{T}, 0, 3,", "k_fft_zb<{T}, 0,"], "fse_fft.hip"),
    "fft_yinv": (["k_fft_yinv<{T},"], "fse_fft.hip"),
    "fft_xinv": (["k_fft_xinv<{T},"], "fse_fft.hip"),
}
CSRC = os.path.join(ROOT, "paper_1607_04808_amd", "csrc")


def code_text(text):
    """Source text without // comments, trailing blanks and empty lines: what the
    compiler sees, so that editing a comment keeps the counters valid."""
    lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def source_hash(name):
    """sha256 of a kernel source and the shared header (code only), to tell stale counters."""
    h = hashlib.sha256()
    for f in (name, "fse_common.h"):
        with open(os.path.join(CSRC, f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic_path(form):
    return os.path.join(ROOT, "profiles", "traffic_stokeslet_n1m_%s.json" % form)


def traffic_from_counters(fetch_csv, write_csv, form, copy_bytes):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of each stage's kernels from two
    rocprofv3 --pmc runs, with the plain copy kernel's readings for scaling."""
    def load(path, counter):
        per = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"].replace("fse::(anonymous namespace)::", "").replace("void ", "")
                per.setdefault(name, {}).setdefault(r["Dispatch_Id"], 0.0)
                per[name][r["Dispatch_Id"]] += float(r["Counter_Value"])
        return {k: list(v.values()) for k, v in per.items()}
    fetch_d, write_d = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    # the probe is the largest plain copy; kernels of a stage: mean per dispatch
    copy = "__amd_rocclr_copyBuffer"
    out = {"form": form, "copy_probe": {"bytes": copy_bytes, "fetch_kib": max(fetch_d[copy]),
                                         "write_kib": max(write_d[copy])},
           "stages": {}}
    fetch = {k: sum(v) / len(v) for k, v in fetch_d.items()}
    write = {k: sum(v) / len(v) for k, v in write_d.items()}
    T = "float" if form == "f32" else "double"
    for stage, (pats, src) in STAGE_KERNELS.items():
        f = w = 0.0
        found = False
        for pat in pats:
            pat = pat.format(T=T)
            names = [k for k in fetch if k.startswith(pat)]
            if names:
                found = True
                f += sum(fetch[k] for k in names)
                w += sum(write.get(k, 0.0) for k in names)
        if found:
            out["stages"][stage] = {"fetch_kib": f, "write_kib": w, "source": src, "sha": source_hash(src)}
    return out


def stage_traffic(form, stage):
    """HBM bytes per launch group of `stage` from the committed counter readings,
    scaled by the copy kernel's; None when absent or the kernel source changed."""
    try:
        with open(traffic_path(form)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    st = t.get("stages", {}).get(stage)
    if not st or st["sha"] != source_hash(st["source"]):
        return None
    cp = t["copy_probe"]
    sf = cp["bytes"] / (cp["fetch_kib"] * 1024.0)
    sw = cp["bytes"] / (cp["write_kib"] * 1024.0)
    return st["fetch_kib"] * 1024.0 * sf + st["write_kib"] * 1024.0 * sw


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_DEFAULT)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-form measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-targets", type=int, default=6144, help="oracle target sample size")
    ap.add_argument("--forms", default="f32,f64,batched")
    ap.add_argument("--batch", type=int, default=16, help="force vectors of the batched form")
    ap.add_argument("--set", action="append", default=[], metavar="FORM.KEY=VALUE",
                    help="override a parameter of a form, e.g. f32.xi=90 (repeatable)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter scaling)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-stage HBM traffic file from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.traffic_from:
        form = args.forms.split(",")[0]
        t = traffic_from_counters(args.traffic_from[0], args.traffic_from[1], form,
                                  args.copy_probe_mb * 2 ** 20)
        with open(traffic_path(form), "w") as fh:
            json.dump(t, fh, indent=1, sort_keys=True)
        print("wrote", traffic_path(form))
        return
    for item in args.set:
        key, val = item.split("=", 1)
        form, name = key.split(".", 1)
        if form not in FORMS or name not in FORMS[form]:
            ap.error("unknown parameter %s" % key)
        FORMS[form][name] = type(FORMS[form][name])(float(val))
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus %d is not supported "
              "(sharding over several GPUs is described, not implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1607_04808_amd as F

    dev = torch.device("cuda:0")
    if args.copy_probe_mb > 0:
        src = torch.ones(args.copy_probe_mb * 2 ** 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    cfg_id = 0
    x64 = W.uniform_cube(n, 1000 + cfg_id)
    f64 = W.normal_strengths(n, 2000 + cfg_id)
    w64 = W.normal_strengths(n, 3000 + cfg_id)

    results = {}
    outputs = {}
    results_full = None
    forms = [f for f in args.forms.split(",") if f]
    if args.no_fp64 and "f64" in forms:
        forms.remove("f64")
    B = args.batch
    for form in forms:
        batched = form == "batched"
        dform = "f32" if batched else form  # the batched form is FP32 at the FP32 parameters
        nb = B if batched else 1
        prm = FORMS[dform]
        tdt = torch.float32 if dform == "f32" else torch.float64
        x = torch.tensor(x64, dtype=tdt, device=dev)
        if batched:
            fb = W.normal_strengths(n, 2100, batch=B)
            wb = W.normal_strengths(n, 3100, batch=B)
            f = torch.tensor(fb, dtype=tdt, device=dev)
            w = torch.tensor(wb, dtype=tdt, device=dev)
        else:
            f = torch.tensor(f64, dtype=tdt, device=dev)
            w = torch.tensor(w64, dtype=tdt, device=dev)
        params = F.make_params(prm["xi"], prm["rc"], prm["M"], prm["P"], (0.0, 0.0, 0.0), L_BOX, Mt=prm["Mt"])
        t0 = time.time()
        plan = F.Plan("stokeslet", dform, params, batch=nb, nmax=n)
        torch.cuda.synchronize()
        t_plan = time.time() - t0
        plan.set_points(x, validate=True)
        geo = plan.geometry

        # the timed step: binning, then u = K f, dL/df = K w and dL/dx in one call
        # (fse_eval_with_adjoint); "separate": fse_eval then fse_eval_adjoint reusing
        # the forward field (as torch.autograd does); "forward": fse_eval alone
        def step(kind="fused"):
            plan.set_points(x, validate=False)
            if kind == "fused":
                return plan.eval_with_adjoint(f, w)
            u = plan.eval(f)
            if kind == "separate":
                df, dx = plan.adjoint(f, w, recompute=False)
                return u, df, dx
            return u, None, None

        def timed(kind):
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                out = step(kind)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / args.steps, out

        for _ in range(args.warmup):
            step()
            step("separate")
        torch.cuda.synchronize()
        plan.timings()
        plan.set_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms, (u, df, dx) = timed("fused")
        stages = plan.timings()
        plan.set_timing(False)
        ms_sep, (u_s, df_s, dx_s) = timed("separate")
        ms_fwd, _ = timed("forward")
        # the fused and the separate calls agree to rounding
        agree = max(float((a - b).abs().max() / b.abs().max()) for a, b in ((u, u_s), (df, df_s), (dx, dx_s)))
        del u_s, df_s, dx_s
        if batched:
            # two members for the sampled error check
            outputs[form] = (u.cpu().numpy()[:2], df.cpu().numpy()[:2], fb[:2], wb[:2])
        else:
            outputs[form] = (u.cpu().numpy()[0], df.cpu().numpy()[0], dx.cpu().numpy())
        if form == "f32" and "f64" in forms:
            # the FP64 form at the FP32-rounded inputs (untimed): the reference for the
            # FP32 form's error over all N (the FP64 form is ~1e-11 from the direct sum)
            xs, fs, ws = (np.asarray(a, np.float32).astype(np.float64) for a in (x64, f64, w64))
            p64 = F.make_params(FORMS["f64"]["xi"], FORMS["f64"]["rc"], FORMS["f64"]["M"], FORMS["f64"]["P"],
                                (0.0, 0.0, 0.0), L_BOX, Mt=FORMS["f64"]["Mt"])
            ref_plan = F.Plan("stokeslet", "f64", p64, batch=1, nmax=n)
            xr, fr, wr = (torch.tensor(a, device=dev) for a in (xs, fs, ws))
            ref_plan.set_points(xr)
            ur = ref_plan.eval(fr)
            dfr, dxr = ref_plan.adjoint(fr, wr, recompute=False)
            full = {}
            for key, a32, a64 in (("u", u[0], ur[0]), ("dL_df", df[0], dfr[0]), ("dL_dx", dx, dxr)):
                d = (a32.double() - a64).abs().max() / a64.abs().max()
                full[key] = float("%.3g" % float(d))
            full["targets"] = n
            results_full = full
            ref_plan.close()
            del xr, fr, wr, ur, dfr, dxr
        pairs = n * (n - 1) * cube_pair_cdf(prm["rc"] / L_BOX)
        stage_tab = {}
        for name, (tot, cnt) in stages.items():
            if cnt == 0:
                continue
            per = tot / cnt
            b, fl = stage_work(name, geo, n, prm["P"], dform, pairs / 1.0, batch=nb, fused=True)
            # launches per step of this stage (e.g. two spreads per forward+adjoint step)
            stage_tab[name] = dict(ms_per_step=tot / args.steps, ms_per_launch=per, launches=cnt,
                                   GBs=(b / per / 1e6 if b else None),
                                   TFLOPs=(fl / per / 1e9 if fl else None))
        results[form] = dict(params=dict(prm, Mt=geo.Mt, n_fft=geo.n_fft, eta=round(geo.eta, 4), L=L_BOX),
                             ms_per_step=ms, ms_forward=ms_fwd, targets_per_s=n / (ms / 1e3),
                             ms_per_step_separate_calls=ms_sep,
                             targets_per_s_separate_calls=n / (ms_sep / 1e3),
                             fused_vs_separate_max_rel_diff=float("%.2e" % agree),
                             forward_targets_per_s=n / (ms_fwd / 1e3), plan_seconds=t_plan,
                             workspace_GB=plan.workspace_bytes() / 1e9, stages=stage_tab)
        if batched:
            results[form].update(batch=B, dtype="f32",
                                 vector_targets_per_s=n * B / (ms / 1e3),
                                 forward_vector_targets_per_s=n * B / (ms_fwd / 1e3))
        plan.close()
        del x, f, w
        torch.cuda.empty_cache()

    head = results.get("f32") or next(iter(results.values()))
    head_form = "f32" if "f32" in results else forms[0]
    # dominant kernel (of the stages with an algorithmic work figure) and its roofline
    dom_name, dom = max(((k, v) for k, v in head["stages"].items() if v["GBs"] is not None or v["TFLOPs"] is not None),
                        key=lambda kv: kv[1]["ms_per_step"])
    peak_alu = PEAK["f32_TFLOPs"] if head_form == "f32" else PEAK["f64_TFLOPs"]
    tr = stage_traffic(head_form, dom_name)
    tr = round(tr) if tr is not None else None
    if dom["GBs"] is not None and dom["TFLOPs"] is None:
        roof = dict(kernel=dom_name, bound="hbm", achieved=round(dom["GBs"], 1), peak=PEAK["hbm_GBs"],
                    unit="GB/s", frac=round(dom["GBs"] / PEAK["hbm_GBs"], 4), traffic=tr)
    else:
        # FP32 spreading runs on the matrix cores (dense FP32 MFMA peak, also 157.3 TFLOP/s)
        bound = "mfma" if (head_form, dom_name) in MFMA_STAGES else "alu"
        roof = dict(kernel=dom_name, bound=bound, achieved=round(dom["TFLOPs"], 2), peak=peak_alu,
                    unit="TFLOP/s", frac=round(dom["TFLOPs"] / peak_alu, 4), traffic=tr)

    line = {
        "metric": "stokeslet targets/s at 1e-6 rel err, N=1M; fwd+adjoint; FP32 vs FP64 form",
        "value": round(head["targets_per_s"], 1),
        "unit": "targets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head_form,
        "data": "synthetic",
        "config": {"workload": "stokeslet sum, N=%d points uniform in [0,1)^3, f and w i.i.d. N(0,1), "
                               "forward + adjoint (dL/df, dL/dx), %s form" % (n, head_form),
                   "n": n, "kernel": "stokeslet", "params": head["params"],
                   "step": "fse_set_points + fse_eval_with_adjoint (u, dL/df and dL/dx in one call); "
                           "forms.*.ms_per_step_separate_calls: fse_eval then fse_eval_adjoint"},
        "roofline": roof,
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) and not kk.endswith("_diff") else vv)
                      for kk, vv in v.items() if kk != "stages"}
                  for k, v in results.items()},
        "stages": {k: v["stages"] for k, v in results.items()},
    }

    if "batched" in results:
        br = results["batched"]
        bd, bdom = max(((k, v) for k, v in br["stages"].items() if v["GBs"] is not None or v["TFLOPs"] is not None),
                       key=lambda kv: kv[1]["ms_per_step"])
        if bdom["TFLOPs"] is not None:
            line["forms"]["batched"]["roofline"] = dict(kernel=bd, bound="mfma" if ("f32", bd) in MFMA_STAGES else "alu",
                                                        achieved=round(bdom["TFLOPs"], 2), peak=PEAK["f32_TFLOPs"],
                                                        unit="TFLOP/s", frac=round(bdom["TFLOPs"] / PEAK["f32_TFLOPs"], 4))
        else:
            line["forms"]["batched"]["roofline"] = dict(kernel=bd, bound="hbm", achieved=round(bdom["GBs"], 1),
                                                        peak=PEAK["hbm_GBs"], unit="GB/s",
                                                        frac=round(bdom["GBs"] / PEAK["hbm_GBs"], 4))
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["error"] = cpu_baseline(x64, f64, w64, outputs, args.cpu_targets)
    if results_full is not None:
        line.setdefault("error", {}).setdefault("f32", {})["all_targets_vs_f64_form"] = results_full
    print(json.dumps(line))


def cpu_baseline(x64, f64, w64, outputs, T):
    """The oracle (FP64 direct sum, its K w, and the analytic gradient: the work of
    one GPU step) on a seeded sample of T targets with all N sources, built for the
    host it runs on; gives the CPU rate on all cores and on one core, and the
    sampled errors."""
    import tempfile
    from oracle import direct
    try:
        direct.use_library(direct.build(path=os.path.join(tempfile.mkdtemp(), "liboracle_native.so"), native=True))
        build = "gcc -O3 -march=native -fopenmp"
    except Exception:  # no compiler on this host: the portable build
        build = "gcc -O3 -march=x86-64-v3 -fopenmp"
    n = len(x64)
    tg = np.sort(W.rng(4000).choice(n, size=min(T, n), replace=False)).astype(np.int64)
    errs = {}
    t0 = time.time()
    u_ref = direct.direct("stokeslet", x64, f64, targets=tg)
    t1 = time.time()
    g_ref = direct.grad_direct("stokeslet", x64, f64, w64, targets=tg)
    t2 = time.time()
    df_ref = direct.direct("stokeslet", x64, w64, targets=tg)
    t3 = time.time()
    # one core, on the first 256 sampled targets
    t1c = tg[:256]
    direct.set_threads(1)
    s0 = time.time()
    direct.direct("stokeslet", x64, f64, targets=t1c)
    direct.grad_direct("stokeslet", x64, f64, w64, targets=t1c)
    direct.direct("stokeslet", x64, w64, targets=t1c)
    s1 = time.time()
    direct.set_threads(0)
    for form, out in outputs.items():
        if form == "batched":
            u, df, fb, wb = out
            xs = x64.astype(np.float32).astype(np.float64)
            ts = tg[:512]
            e_u = e_f = 0.0
            for m in range(len(u)):
                fs, ws = (a.astype(np.float32).astype(np.float64) for a in (fb[m], wb[m]))
                e_u = max(e_u, direct.rel_errors(u[m][ts], direct.direct("stokeslet", xs, fs, targets=ts))[0])
                e_f = max(e_f, direct.rel_errors(df[m][ts], direct.direct("stokeslet", xs, ws, targets=ts))[0])
            errs[form] = {"u": {"max": float("%.3g" % e_u)}, "dL_df": {"max": float("%.3g" % e_f)},
                          "members_checked": len(u), "targets_sampled": int(len(ts))}
            continue
        u, df, dx = out
        # the FP32 form evaluates the FP32-rounded inputs; its reference uses them
        if form == "f32":
            xs, fs, ws = (a.astype(np.float32).astype(np.float64) for a in (x64, f64, w64))
            ur = direct.direct("stokeslet", xs, fs, targets=tg)
            gr = direct.grad_direct("stokeslet", xs, fs, ws, targets=tg)
            dr = direct.direct("stokeslet", xs, ws, targets=tg)
        else:
            ur, gr, dr = u_ref, g_ref, df_ref
        errs[form] = {
            "u": dict(zip(("max", "rms"), (float("%.3g" % e) for e in direct.rel_errors(u[tg], ur)))),
            "dL_df": dict(zip(("max", "rms"), (float("%.3g" % e) for e in direct.rel_errors(df[tg], dr)))),
            "dL_dx": dict(zip(("max", "rms"), (float("%.3g" % e) for e in direct.rel_errors(dx[tg], gr)))),
            "targets_sampled": int(len(tg)),
        }
    cores = direct.num_threads()
    rate = len(tg) / (t3 - t0)
    base = {"value": round(rate, 2), "unit": "targets/s", "cores": cores, "kind": "oracle",
            "one_core_value": round(len(t1c) / (s1 - s0), 2),
            "build": build,
            "sample": "%d seeded targets x %d sources, FP64: direct sum u, K w and the analytic gradient "
                      "dL/dx (the GPU step's outputs; %.2fs, %.2fs, %.2fs); one core: the first %d of "
                      "those targets" % (len(tg), n, t1 - t0, t2 - t1, t3 - t2, len(t1c))}
    return base, errs


if __name__ == "__main__":
    main()
