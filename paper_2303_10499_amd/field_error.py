"""Per-field error of the pressure-solve forms over whole runs.

Each form (FP64 Jacobi-PCG, FP32/FP64 refinement, the learned form with its
gate, the learned form on every solve) runs the workload at the solve
tolerance of the metric (relative residual 1e-8); a reference run takes FP64
Jacobi-PCG to a tight tolerance (1e-12).  All runs advance in lockstep from
the same device-built initial state, and at checkpoints every field of every
form is compared with the reference: max|x - x_ref| / max|x_ref| for rho, u,
T, p', p.  The FP64 form's own error at 1e-8 is the error that tolerance
allows; a mixed or learned form is as accurate as FP64 when its error is of
that size.  (The reference is the GPU's FP64 path, which the parity tests hold
to the CPU oracle at 1e-10 per field.)

    python -m paper_2303_10499_amd.field_error --workload nonsmooth2d_2048 --steps 500
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

FIELDS = ("rho", "u", "T", "pp", "p")
# form name: (library solver, learned_always)
FORMS = {"pcg64": ("pcg64", 0), "mixed": ("mixed", 0), "learned": ("learned", 0),
         "learned_always": ("learned", 1)}


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def run(workload: str, steps: int, checkpoints: int = 5, tol: float = 1e-8, ref_tol: float = 1e-12,
        forms=("pcg64", "mixed", "learned", "learned_always"), inner_tol: float = 1e-4,
        log=None) -> dict:
    from . import configs, gea
    if log is None:
        def log(msg):
            print(msg, file=sys.stderr, flush=True)
    base = configs.get(workload)
    solvers = {}
    for name in ("reference",) + tuple(forms):
        solver, always = ("pcg64", 0) if name == "reference" else FORMS[name]
        par = dict(base["params"], tol=ref_tol if name == "reference" else tol,
                   inner_tol=inner_tol, learned_always=always,
                   max_iter=max(int(base["params"].get("max_iter", 20000)), 200000))
        S = gea.Solver(base["mesh"], par, solver=solver)
        if solver == "learned":
            S.load_weights()
        S.init_bubble(**base["bubble"])
        solvers[name] = S
    marks = sorted({max(1, round(steps * (q + 1) / checkpoints)) for q in range(checkpoints)})
    out = {"workload": workload, "steps": steps, "tol": tol, "ref_tol": ref_tol,
           "cells": solvers["reference"].nc, "checkpoints": {}}
    done = 0
    stats = {n: dict(iters=0, solves=0, max_rel_res=0.0, fallbacks=0) for n in solvers}
    t0 = time.time()
    for m in marks:
        for n, S in solvers.items():
            st = S.step(m - done)
            stats[n]["iters"] += st.total_iters
            stats[n]["solves"] += st.total_solves
            stats[n]["fallbacks"] += st.total_fallbacks
            stats[n]["max_rel_res"] = max(stats[n]["max_rel_res"], st.max_rel_res)
        done = m
        ref = solvers["reference"].state()
        errs = {}
        for n in forms:
            g = solvers[n].state()
            errs[n] = {f: rel(g[f], ref[f]) for f in FIELDS}
        out["checkpoints"][str(m)] = errs
        log(f"[field_error] {workload} step {m} ({time.time() - t0:.1f} s): " +
            "; ".join(f"{n} " + " ".join(f"{f} {e:.2e}" for f, e in errs[n].items())
                      for n in forms))
    out["solves"] = {n: dict(iters_per_solve=s["iters"] / max(s["solves"], 1),
                             max_rel_res=s["max_rel_res"], fallbacks=s["fallbacks"])
                     for n, s in stats.items()}
    for S in solvers.values():
        S.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="nonsmooth2d_2048")
    ap.add_argument("--steps", type=int, default=None, help="default: the workload's run length")
    ap.add_argument("--checkpoints", type=int, default=5)
    ap.add_argument("--forms", default="pcg64,mixed,learned,learned_always")
    args = ap.parse_args(argv)
    from . import configs
    steps = args.steps or configs.get(args.workload)["steps"]
    res = run(args.workload, steps, args.checkpoints, forms=tuple(args.forms.split(",")))
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
