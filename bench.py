"""Benchmark: cell-steps/s of the segregated pressure-based Euler step at
pressure relative residual 1e-8, on one MI355X.

A step is one pass of the whole hot path (Steps 1-3 of Sec. 3 with n_corr
PISO correctors and their pressure solves) over the 3D smooth-bubble
evaluation mesh (256 x 256 x 128 cells over 20 x 20 x 10 km, dt 0.5 s),
built on the device from the analytic initial state (synthetic input, no
dataset).  Every solver form is timed on the same workload and tolerance:
plain FP64 Jacobi-PCG, FP32/FP64 iterative refinement, and the learned
initial guess/preconditioner when its weights are present.

Prints one JSON line (see the design doc for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# algorithmic bytes per cell of one launch of each kernel class (each array
# read or written once; halo re-reads are not counted)
BYTES_PER_CELL = {
    0: 88.0,   # FP64 CG iteration: read r, A p, p (old), x, 1/diag, c, D; write r, p, A p, x
    2: 44.0,   # FP32 CG iteration (same arrays in FP32)
}
CLASS_NAMES = {0: "k_cg_iter<fp64>", 1: "k_cg_scalars<fp64>", 2: "k_cg_iter<fp32>",
               3: "k_cg_scalars<fp32>", 4: "solver set-up kernels",
               5: "explicit step kernels", 6: "learned network"}
# the six forward convolutions of the network (bf16 matrix-core kernels)
LAYER_NAMES = ["k_conv0z L0 (2->16)", "k_conv_z L1 (16->32, 1/2)", "k_conv_t L2 (32->64, 1/4)",
               "k_conv_z L3 ([64,32]->32, 1/2)", "k_conv_z L4 ([32,16]->16)", "k_conv5z L5 (16->1)"]
MFMA_BF16_PEAK_TFLOPS = 2500.0
# vector bf16 pair dot products (layer 5): 256 CUs x 64 lanes x 2.4 GHz x 4 FLOP
VALU_DOT2_PEAK_TFLOPS = 157.3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# solver forms: (library solver, learned_steps)
FORMS = {"pcg64": ("pcg64", 1), "mixed": ("mixed", 1), "learned": ("learned", 1),
         "learned_fcg": ("learned", 25)}


def run_form(cfg, form, steps, warmup, kernel_steps):
    import torch
    from paper_2303_10499_amd import gea

    solver, lsteps = FORMS[form]
    params = dict(cfg["params"], learned_steps=lsteps)
    S = gea.Solver(cfg["mesh"], params, solver=solver)
    if solver == "learned":
        S.load_weights()
    S.init_bubble(**cfg["bubble"])
    stream = S.stream
    nc = S.nc
    t0 = time.time()
    if warmup:
        S.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    st = S.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    log(f"[bench] {cfg['name']} {form}: {steps} steps in {ms:.1f} ms "
        f"({time.time() - t0:.1f} s wall incl. warmup)")
    out = dict(solver=solver, learned_steps=lsteps if solver == "learned" else None,
               ms_per_step=ms / steps, cell_steps_per_s=nc * steps / (ms * 1e-3),
               iters_per_solve=st.total_iters / max(st.total_solves, 1),
               rel_res_last=max(st.solve[k].rel_res for k in range(st.n_solves)),
               fallbacks_last_step=sum(st.solve[k].fallbacks for k in range(st.n_solves)),
               eos_mismatch=st.eos_mismatch)
    # launches per step of each kernel class, from a second window of steps
    # with the per-launch event timer (events around every launch inflate
    # short kernels, so its times are only used for the explicit kernels'
    # share; kept out of the timed region above)
    S.kernel_timing(True, reset=True)
    S.step(kernel_steps)
    kms, kn = S.kernel_times()
    S.kernel_timing(False)
    # accurate per-launch durations of the CG kernels: reps back-to-back
    # launches between two events on the solver's stream
    avg = S.time_solver_kernels(reps=50)
    out["kernel_avg_us"] = {CLASS_NAMES[k]: round(avg[k] * 1e3, 2) for k in range(4)}
    out["launches_per_step"] = {CLASS_NAMES[k]: kn[k] / kernel_steps for k in range(7) if kn[k]}
    out["explicit_ms_per_step_event_timed"] = kms[5] / kernel_steps
    # candidates for the dominant kernel: device time per step = average
    # launch duration x launches per step
    cands = {}
    for k in BYTES_PER_CELL:
        if kn[k]:
            cands[CLASS_NAMES[k]] = dict(bound="hbm", avg_ms=avg[k], per_step_ms=avg[k] * kn[k] / kernel_steps,
                                         work=BYTES_PER_CELL[k] * nc)
    if solver == "learned":
        nms, ngf = S.time_network(reps=20)
        apps = kn[6] / kernel_steps
        out["network_applications_per_step"] = apps
        out["network_layer_avg_us"] = {LAYER_NAMES[l]: round(nms[l] * 1e3, 2) for l in range(6)}
        for l in range(6):
            cands[LAYER_NAMES[l]] = dict(bound="alu" if l == 5 else "mfma", avg_ms=nms[l],
                                         per_step_ms=nms[l] * apps,
                                         work=ngf[l] * 1e9)
    out["kernel_ms_per_step"] = {k: round(v["per_step_ms"], 4) for k, v in cands.items()}
    if cands:
        dom = max(cands, key=lambda k: cands[k]["per_step_ms"])
        out["roofline"] = dict(kernel=dom, **cands[dom])
    S.close()
    return out


def roofline_entry(rr):
    """the roofline object of a kernel candidate (see run_form)"""
    t = rr["avg_ms"] * 1e-3
    if rr["bound"] == "hbm":
        achieved, peak, unit = rr["work"] / t / 1e9, HBM_PEAK_GBS, "GB/s"
        extra = dict(bytes_per_launch=rr["work"])
    else:
        peak = MFMA_BF16_PEAK_TFLOPS if rr["bound"] == "mfma" else VALU_DOT2_PEAK_TFLOPS
        achieved, unit = rr["work"] / t / 1e12, "TFLOP/s"
        extra = dict(flop_per_launch=rr["work"])
    return dict(bound=rr["bound"], kernel=rr["kernel"], achieved=round(achieved, 1), peak=peak,
                unit=unit, frac=round(achieved / peak, 4), avg_launch_us=round(rr["avg_ms"] * 1e3, 2),
                **extra, traffic=read_traffic(rr["kernel"]))


def cpu_baseline(cfg):
    """The oracle as it stands, one step from the initial state, 1 thread."""
    import numpy as np  # noqa: F401
    from oracle import geao
    geao.build(force=False)
    O = geao.Oracle(cfg["mesh"], cfg["params"])
    s = O.init_bubble(**cfg["bubble"])
    t = time.time()
    O.step(s, 1)
    dt = time.time() - t
    return dict(value=O.nc / dt, unit="cell-steps/s", cores=1, kind="oracle",
                sample=f"1 step of {cfg['name']} from the initial state, FP64 Jacobi-PCG at "
                       f"tol {cfg['params']['tol']:g}, single-threaded C (-O2), {dt:.1f} s")


def source_sha(name):
    import hashlib
    src = os.path.join(ROOT, "paper_2303_10499_amd", "csrc", name)
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def read_traffic(kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (profiles/traffic.txt: lines 'kernel = bytes @ source sha'), if
    the counters were taken on the current source of that kernel; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        line = line.strip()
        if line.startswith("#") or "=" not in line or "@" not in line:
            continue
        k, rest = line.split("=", 1)
        val, src = rest.split("@", 1)
        name, sha = src.split()
        if k.strip() == kernel:
            return float(val) if source_sha(name) == sha else None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bubble3d_256x256x128")
    ap.add_argument("--also", default="nonsmooth2d_2048_eval",
                    help="second evaluation mesh reported beside the first ('' for none)")
    ap.add_argument("--forms", default="pcg64,mixed,learned,learned_fcg")
    ap.add_argument("--kernel-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU domain decomposition is a design, not a build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_10499_amd import configs, gea
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    gea.lib()
    forms = [f for f in args.forms.split(",") if f]

    def run_workload(name):
        cfg = configs.get(name)
        cfg["params"]["tol"] = 1e-8
        cfg["params"]["inner_tol"] = 1e-4
        cfg["params"]["max_iter"] = 200000
        res = {}
        for f in forms:
            if FORMS[f][0] == "learned" and not learned_available(cfg):
                log(f"[bench] {f} skipped: no trained weights for this workload")
                continue
            res[f] = run_form(cfg, f, args.steps, args.warmup, args.kernel_steps)
        return cfg, res

    cfg, results = run_workload(args.workload)
    also = None
    if args.also:
        cfg2, res2 = run_workload(args.also)
        also = {"workload": cfg2["name"],
                "cells": cfg2["mesh"]["nx"] * cfg2["mesh"]["ny"] * cfg2["mesh"]["nz"],
                "forms": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv)
                              for kk, vv in v.items() if kk != "roofline"} for k, v in res2.items()}}
        if "pcg64" in res2:
            also["speedup_vs_pcg64"] = {k: round(v["cell_steps_per_s"] / res2["pcg64"]["cell_steps_per_s"], 3)
                                        for k, v in res2.items()}
    primary = "learned" if "learned" in results else ("mixed" if "mixed" in results else forms[0])
    R = results[primary]
    nc = cfg["mesh"]["nx"] * cfg["mesh"]["ny"] * cfg["mesh"]["nz"]
    roof = roofline_entry(R["roofline"]) if "roofline" in R else None
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a one-step sample ...")
        cpu = cpu_baseline(cfg)
    line = {
        "metric": "cell-steps/s at pressure residual 1e-8: learned+mixed vs plain FP64 PCG",
        "value": round(R["cell_steps_per_s"], 1),
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(R["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if primary == "pcg64" else "f64+f32" + ("+bf16" if primary == "learned" else ""),
        "data": "synthetic: analytic 3D smooth-bubble initial state built on the device",
        "config": {"workload": cfg["name"], "cells": nc, "form": primary,
                   "dt": cfg["params"]["dt"], "n_corr": cfg["params"]["n_corr"],
                   "tol": cfg["params"]["tol"], "parallelism": "single GPU"},
        "forms": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv)
                      for kk, vv in v.items() if kk != "roofline"} for k, v in results.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if "pcg64" in results:
        line["speedup_vs_pcg64"] = {k: round(v["cell_steps_per_s"] / results["pcg64"]["cell_steps_per_s"], 3)
                                    for k, v in results.items()}
    line["also"] = also
    print(json.dumps(line), flush=True)


def learned_available(cfg):
    from paper_2303_10499_amd import learned
    ndim = 2 if cfg["mesh"]["ny"] == 1 else 3
    m = cfg["mesh"]
    ok = all(n % 4 == 0 for n in (m["nx"], m["nz"])) and (ndim == 2 or m["ny"] % 4 == 0)
    return ok and os.path.exists(learned.weights_file(ndim))


if __name__ == "__main__":
    main()
