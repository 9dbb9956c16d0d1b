"""Benchmark: cell-steps/s of the segregated pressure-based Euler step at
pressure relative residual 1e-8, on one MI355X.

A step is one pass of the whole hot path (Steps 1-3 of Sec. 3 with n_corr
PISO correctors and their pressure solves) over the 3D smooth-bubble
evaluation mesh (256 x 256 x 128 cells over 20 x 20 x 10 km, dt 0.5 s),
built on the device from the analytic initial state (synthetic input, no
dataset).  Every solver form is timed on the same workload and tolerance:
plain FP64 Jacobi-PCG, FP32/FP64 iterative refinement, and the learned
initial guess/preconditioner when its weights are present.

Two measurements per form:
  * the timed window: W warm-up steps, then exactly K steps between HIP
    events on the solver's stream (`value`, `ms_per_step`);
  * the full run: the whole evaluation run from the initial state (200
    steps in 3D, 500 on the 2D 2048^2 mesh), timed as one piece, the median
    of several repetitions in 3D (`full_run`).
Every solve's exit residual is reported (`max_rel_res`), unrounded.
`implicit_transport`: the same meshes with Steps 1-2 solved implicitly
(transport = 1, BiCGStab; the refinement form for the pressure), in both
energy forms: the timed window only.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell of one Jacobi-PCG iteration: the operator
# (read p, c, D; write A p: 32 B), the update (read x, p, r, A p, 1/diag;
# write x, r: 56 B) and the new direction (read r, 1/diag, p; write p: 32 B)
# with every array read or written once: 120 B in FP64, 60 B in FP32 (the
# refined forms' inner iterations).
ALG_BYTES_PER_CELL = {0: 120.0, 2: 60.0}
# What the fused iteration kernel itself must move: 11 arrays (read r, A p,
# p, x, 1/diag, c, D; write r, p, A p, x).
FUSED_BYTES_PER_CELL = {0: 88.0, 2: 44.0}
CLASS_NAMES = {0: "k_cg_iter<fp64>", 1: "k_cg_scalars<fp64>", 2: "k_cg_iter<fp32>",
               3: "k_cg_scalars<fp32>", 4: "solver set-up kernels",
               5: "explicit step kernels", 6: "learned network", 7: "energy solve kernels"}
# the six forward convolutions of the network (bf16 matrix-core kernels)
LAYER_NAMES = ["k_conv0z L0 (2->16)", "k_conv_z L1 (16->32, 1/2)", "k_conv_t L2 (32->64, 1/4)",
               "k_conv_z L3 ([64,32]->32, 1/2)", "k_conv_z L4 ([32,16]->16)", "k_conv5z L5 (16->1)"]
MFMA_BF16_PEAK_TFLOPS = 2500.0
# vector bf16 pair dot products (layer 5): 256 CUs x 64 lanes x 2.4 GHz x 4 FLOP
VALU_DOT2_PEAK_TFLOPS = 157.3

# solver forms: (library solver, learned_steps, learned_always).  "learned" is
# the production form: its gate runs the network on a corrector only while
# it pays for itself; "learned_always" applies it on every solve.
FORMS = {"pcg64": ("pcg64", 1, 0), "mixed": ("mixed", 1, 0), "learned": ("learned", 1, 0),
         "learned_always": ("learned", 1, 1), "learned_fcg": ("learned", 25, 1)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sig(v, n=6):
    """a float to n significant digits (small values keep their exponent)"""
    return float(f"{v:.{n}g}") if isinstance(v, float) else v


def clean(d):
    return {k: (clean(v) if isinstance(v, dict) else sig(v)) for k, v in d.items()}


def timed_steps(S, n):
    """n steps between two events on the solver's stream: (ms, stats)"""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(S.stream)
    st = S.step(n)
    e1.record(S.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), st


def make_solver(cfg, form):
    from paper_2303_10499_amd import gea
    solver, lsteps, always = FORMS[form]
    params = dict(cfg["params"], learned_steps=lsteps, learned_always=always)
    S = gea.Solver(cfg["mesh"], params, solver=solver)
    if solver == "learned":
        S.load_weights()
    return S


def run_window(cfg, form, steps, warmup, kernel_steps):
    """the timed window of a form, its kernel accounting and roofline candidates"""
    solver, lsteps, _ = FORMS[form]
    S = make_solver(cfg, form)
    nc = S.nc
    S.init_bubble(**cfg["bubble"])
    if warmup:
        S.step(warmup)
    ms, st = timed_steps(S, steps)
    log(f"[bench] {cfg['name']} {form}: {steps} steps in {ms:.1f} ms")
    out = dict(solver=solver, learned_steps=lsteps if solver == "learned" else None,
               ms_per_step=ms / steps, cell_steps_per_s=nc * steps / (ms * 1e-3),
               iters_per_solve=st.total_iters / max(st.total_solves, 1),
               max_rel_res=st.max_rel_res, fallbacks=st.total_fallbacks,
               eos_mismatch=st.eos_mismatch)
    # A second window with the per-launch event timer (events around every
    # launch inflate short kernels; kept out of the timed window above).
    # Launches that find their solve already done return at once: the
    # per-step device time of the CG iteration kernel counts only the
    # launches that did an iteration.
    S.kernel_timing(True, reset=True)
    st_k = S.step(kernel_steps)
    kms, kn = S.kernel_times()
    S.kernel_timing(False)
    iters_per_step = st_k.total_iters / kernel_steps
    avg = S.time_solver_kernels(reps=50)   # back-to-back launches between two events
    out["kernel_avg_us"] = {CLASS_NAMES[k]: round(avg[k] * 1e3, 2) for k in range(4)}
    out["launches_per_step"] = {CLASS_NAMES[k]: kn[k] / kernel_steps for k in range(8) if kn[k]}
    out["energy_iters_per_step"] = st_k.energy_iters / kernel_steps
    out["energy_ms_per_step_event_timed"] = kms[7] / kernel_steps
    out["iterations_per_step"] = iters_per_step
    out["explicit_ms_per_step_event_timed"] = kms[5] / kernel_steps
    cands = {}
    it_class = 0 if solver == "pcg64" else 2
    cands[CLASS_NAMES[it_class]] = dict(bound="hbm", avg_ms=avg[it_class],
                                        per_step_ms=avg[it_class] * iters_per_step,
                                        bytes_alg=ALG_BYTES_PER_CELL[it_class] * nc,
                                        bytes_fused=FUSED_BYTES_PER_CELL[it_class] * nc,
                                        per_cell=(ALG_BYTES_PER_CELL[it_class], FUSED_BYTES_PER_CELL[it_class]))
    if solver == "learned":
        nms, ngf = S.time_network(reps=20)
        apps = kn[6] / kernel_steps
        out["network_applications_per_step"] = apps
        out["network_layer_avg_us"] = {LAYER_NAMES[l]: round(nms[l] * 1e3, 2) for l in range(6)}
        for l in range(6):
            cands[LAYER_NAMES[l]] = dict(bound="alu" if l == 5 else "mfma", avg_ms=nms[l],
                                         per_step_ms=nms[l] * apps, flop=ngf[l] * 1e9)
    out["kernel_ms_per_step"] = {k: round(v["per_step_ms"], 4) for k, v in cands.items()}
    dom = max(cands, key=lambda k: cands[k]["per_step_ms"])
    out["_roofline"] = dict(kernel=dom, **cands[dom])
    S.close()
    return out


def run_transport(cfg, steps, warmup, solver="mixed"):
    """the implicit-transport variant of the step (Steps 1-2 solved by BiCGStab,
    transport = 1) in both energy forms: the timed window of one solver form"""
    from paper_2303_10499_amd import gea
    out = {}
    for name, form in (("total_energy", 0), ("enthalpy", 1)):
        params = dict(cfg["params"], transport=1, energy_form=form)
        S = gea.Solver(cfg["mesh"], params, solver=solver)
        S.init_bubble(**cfg["bubble"])
        if warmup:
            S.step(warmup)
        ms, st = timed_steps(S, steps)
        log(f"[bench] {cfg['name']} {solver}, implicit transport, {name}: {steps} steps in {ms:.1f} ms")
        out[name] = dict(solver=solver, ms_per_step=ms / steps,
                         cell_steps_per_s=S.nc * steps / (ms * 1e-3),
                         transport_iters_per_step=st.transport_iters / steps,
                         iters_per_solve=st.total_iters / max(st.total_solves, 1),
                         max_rel_res=st.max_rel_res)
        S.close()
    return {k: clean(v) for k, v in out.items()}


def run_full(cfg, form, nsteps, reps):
    """the whole evaluation run from the initial state, reps times"""
    S = make_solver(cfg, form)
    nc = S.nc
    runs = []
    for r in range(reps):
        S.init_bubble(**cfg["bubble"])
        ms, st = timed_steps(S, nsteps)
        runs.append(dict(ms=ms, iters_per_solve=st.total_iters / max(st.total_solves, 1),
                         max_rel_res=st.max_rel_res, fallbacks=st.total_fallbacks))
        log(f"[bench] {cfg['name']} {form}: full run of {nsteps} steps #{r + 1}: {ms:.1f} ms, "
            f"{runs[-1]['iters_per_solve']:.2f} iterations a solve, max rel_res {st.max_rel_res:.3e}")
    S.close()
    med = statistics.median(r["ms"] for r in runs)
    return dict(steps=nsteps, reps=reps, cell_steps_per_s=nc * nsteps / (med * 1e-3),
                ms_per_step=med / nsteps, runs_ms=[round(r["ms"], 2) for r in runs],
                iters_per_solve=runs[0]["iters_per_solve"],
                max_rel_res=max(r["max_rel_res"] for r in runs),
                fallbacks=sum(r["fallbacks"] for r in runs))


def roofline_entry(rr):
    """the roofline object of a kernel candidate (see run_window)"""
    t = rr["avg_ms"] * 1e-3
    if rr["bound"] == "hbm":
        achieved = rr["bytes_alg"] / t / 1e9
        fused = rr["bytes_fused"] / t / 1e9
        return dict(bound="hbm", kernel=rr["kernel"], achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    avg_launch_us=round(rr["avg_ms"] * 1e3, 2),
                    bytes_per_cell=rr["per_cell"][0], bytes_per_launch=rr["bytes_alg"],
                    fused_bytes_per_cell=rr["per_cell"][1], achieved_fused=round(fused, 1),
                    frac_fused=round(fused / HBM_PEAK_GBS, 4),
                    traffic=read_traffic(rr["kernel"]))
    peak = MFMA_BF16_PEAK_TFLOPS if rr["bound"] == "mfma" else VALU_DOT2_PEAK_TFLOPS
    achieved = rr["flop"] / t / 1e12
    return dict(bound=rr["bound"], kernel=rr["kernel"], achieved=round(achieved, 1), peak=peak,
                unit="TFLOP/s", frac=round(achieved / peak, 4), avg_launch_us=round(rr["avg_ms"] * 1e3, 2),
                flop_per_launch=rr["flop"], traffic=None)


def cpu_baseline(cfg, all_core_steps=3):
    """The oracle as it stands on the host's cores: one step from the initial
    state single-threaded, then the -fopenmp build of the same source (every
    reduction serial, so the same bits, checked here) for a few steps on all
    cores."""
    import numpy as np
    from oracle import geao
    one = geao.Oracle(cfg["mesh"], cfg["params"])
    s1 = one.init_bubble(**cfg["bubble"])
    t = time.time()
    one.step(s1, 1)
    dt1 = time.time() - t
    many = geao.Oracle(cfg["mesh"], cfg["params"], omp=True)
    threads = many.L.geao_threads()
    s2 = many.init_bubble(**cfg["bubble"])
    t = time.time()
    many.step(s2, 1)
    dts = [time.time() - t]
    same = all(np.array_equal(getattr(s1, f), getattr(s2, f)) for f in ("rho", "u", "T", "pp", "p"))
    for _ in range(all_core_steps - 1):
        t = time.time()
        many.step(s2, 1)
        dts.append(time.time() - t)
    nc = one.nc
    return dict(value=nc * len(dts) / sum(dts), unit="cell-steps/s", cores=threads, kind="oracle",
                sample=f"steps 1-{len(dts)} of {cfg['name']} from the initial state, FP64 Jacobi-PCG "
                       f"at tol {cfg['params']['tol']:g}: the oracle's -fopenmp build on {threads} "
                       f"threads ({sum(dts):.1f} s; step 1 bitwise equal to the single-threaded "
                       f"build: {same})",
                one_core=dict(value=nc / dt1, cores=1,
                              sample=f"step 1 single-threaded (gcc -O2), {dt1:.1f} s"),
                same_bits_as_one_core=same)


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


def learned_available(cfg):
    from paper_2303_10499_amd import learned
    ndim = 2 if cfg["mesh"]["ny"] == 1 else 3
    m = cfg["mesh"]
    ok = all(n % 4 == 0 for n in (m["nx"], m["nz"])) and (ndim == 2 or m["ny"] % 4 == 0)
    return ok and os.path.exists(learned.weights_file(ndim))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="bubble3d_256x256x128")
    ap.add_argument("--also", default="nonsmooth2d_2048_eval",
                    help="second evaluation mesh reported beside the first ('' for none)")
    ap.add_argument("--forms", default="pcg64,mixed,learned,learned_always,learned_fcg")
    ap.add_argument("--kernel-steps", type=int, default=3)
    ap.add_argument("--full-reps", type=int, default=3, help="full runs per form on the first mesh")
    ap.add_argument("--full-reps-also", type=int, default=1, help="full runs per form on the second mesh")
    ap.add_argument("--full-forms-also", default="pcg64,mixed,learned,learned_always")
    ap.add_argument("--no-full", action="store_true", help="skip the full evaluation runs")
    ap.add_argument("--no-transport", action="store_true",
                    help="skip the implicit-transport variant (Steps 1-2 by BiCGStab)")
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

    def workload(name):
        cfg = configs.get(name)
        cfg["params"]["tol"] = 1e-8
        cfg["params"]["inner_tol"] = 1e-4
        cfg["params"]["max_iter"] = 200000
        return cfg

    def run_workload(cfg, full_reps, full_forms):
        res = {}
        for f in forms:
            if FORMS[f][0] == "learned" and not learned_available(cfg):
                log(f"[bench] {f} skipped: no trained weights for this workload")
                continue
            res[f] = run_window(cfg, f, args.steps, args.warmup, args.kernel_steps)
        full = None
        if not args.no_full:
            full = {"workload": cfg["name"], "steps": cfg["steps"], "forms": {}}
            for f in full_forms:
                if f in res:
                    full["forms"][f] = run_full(cfg, f, cfg["steps"], full_reps)
            if "pcg64" in full["forms"]:
                base = full["forms"]["pcg64"]["cell_steps_per_s"]
                full["speedup_vs_pcg64"] = {k: round(v["cell_steps_per_s"] / base, 3)
                                            for k, v in full["forms"].items()}
            full["forms"] = {k: clean(v) for k, v in full["forms"].items()}
        return res, full

    def speedups(res):
        if "pcg64" not in res:
            return None
        base = res["pcg64"]["cell_steps_per_s"]
        return {k: round(v["cell_steps_per_s"] / base, 3) for k, v in res.items()}

    def public(res):
        return {k: clean({kk: vv for kk, vv in v.items() if not kk.startswith("_")}) for k, v in res.items()}

    cfg = workload(args.workload)
    results, full = run_workload(cfg, args.full_reps, forms)
    also = None
    if args.also:
        cfg2 = workload(args.also)
        res2, full2 = run_workload(cfg2, args.full_reps_also,
                                   [f for f in args.full_forms_also.split(",") if f])
        also = {"workload": cfg2["name"],
                "cells": cfg2["mesh"]["nx"] * cfg2["mesh"]["ny"] * cfg2["mesh"]["nz"],
                "forms": public(res2), "speedup_vs_pcg64": speedups(res2),
                "roofline": {k: roofline_entry(v["_roofline"]) for k, v in res2.items()},
                "full_run": full2,
                "implicit_transport": None if args.no_transport else
                run_transport(cfg2, args.steps, args.warmup)}
    primary = "learned" if "learned" in results else ("mixed" if "mixed" in results else forms[0])
    R = results[primary]
    nc = cfg["mesh"]["nx"] * cfg["mesh"]["ny"] * cfg["mesh"]["nz"]
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = clean(cpu_baseline(cfg))
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
        "forms": public(results),
        "speedup_vs_pcg64": speedups(results),
        "full_run": full,
        "roofline": roofline_entry(R["_roofline"]),
        "roofline_by_form": {k: roofline_entry(v["_roofline"]) for k, v in results.items()},
        "implicit_transport": None if args.no_transport else run_transport(cfg, args.steps, args.warmup),
        "cpu_baseline": cpu,
        "also": also,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
