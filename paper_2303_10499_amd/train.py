"""Train the learned initial guess / preconditioner of the pressure solve.

Training pairs come from the solver itself (gea_make_pair): for a rising
bubble drawn at random (theta_c ~ U(0.25, 3) K, r_c ~ U(150, 2500) m clipped
to [2 dx, 0.4 min(Lx, Lz)], numpy PCG64 seeded: 0 for training, 1 for
held-out evaluation), a few time steps are taken, then the next step's
first-corrector pressure system is assembled and solved tightly; the pair is
(r0/s, c/diag) -> delta/s with r0 = b - A p', delta = x - p' and s the
field's max |r0| (the scaling the solver applies to the network's input).
Crops of 128^2 (2D) or 32^3 (3D) cells are cut from each full-mesh pair on
the GPU.  With --crop-scale local each crop is rescaled by its own max |r0|
and crops below 5 % of the field's maximum are dropped; with global the crops
keep the field's scaling (as the network sees them in use) and only crops of
pure round-off (below 1e-6 of the maximum) are dropped.  Targets are divided
by their RMS over the training set (the flexible-CG line search makes the
network's output scale irrelevant to the solve).  Training runs the library's
bfloat16 forward and backward kernels with Adam (FP32 master weights).  The
held-out error is reported on crops and on whole fields.

Data (--data sources, the default): 20000 pairs dumped from whole runs of
the 2D workloads bubble2d_64x32, bubble2d_1280x640 and nonsmooth2d_2048 (one
pair a step, each from a fresh random bubble every 100 steps; 10000, 8500
and 1500 pairs) for the 2D network, and 20000 pairs from runs on a small 3D
mesh with the evaluation mesh's cells and time step (bubble3d_64x64x32_train)
for the 3D network; one 32^2 or 32^3 crop a pair.  --data workload cuts
the crops from runs on the evaluation workload itself instead.  Held-out
pairs come from the same sources with seed 1, and whole fields of the
evaluation workload measure the error the solver sees.

Usage: python -m paper_2303_10499_amd.train --ndim 2 [--data sources|workload] [--out w2d.npy]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2303_10499_amd import configs, gea, learned  # noqa: E402

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def weights_path(ndim: int) -> str:
    return os.path.join(WEIGHTS_DIR, f"net{ndim}d.npy")


def log(msg):
    print(msg, flush=True)


def he_init(ndim: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for (co, nt, ci), nb in learned.layer_shapes(ndim):
        std = np.sqrt(2.0 / (nt * ci))
        parts.append(rng.normal(0.0, std, size=co * nt * ci))
        parts.append(np.zeros(nb))
    return np.concatenate(parts).astype(np.float32)


def draw_bubble(rng, cfg):
    m = cfg["mesh"]
    dx = m["lx"] / m["nx"]
    lo, hi = 2 * dx, 0.4 * min(m["lx"], m["lz"])
    rc = float(np.clip(rng.uniform(150.0, 2500.0), lo, hi))
    amp = float(rng.uniform(0.25, 3.0))
    kind = int(rng.integers(1, 3))
    xc = float(rng.uniform(0.3, 0.7) * m["lx"])
    yc = float(rng.uniform(0.3, 0.7) * m["ly"])
    zc = float(np.clip(rng.uniform(0.15, 0.5) * m["lz"], rc, m["lz"] - rc))
    return dict(kind=kind, xc=xc, yc=yc, zc=zc, rc=rc, amp=amp)


def make_pairs(workload: str, runs: int, crops_per_run: int, seed: int, device="cuda:0",
               crop_scale: str = "local", fields: list | None = None):
    """crops (X: [n, cells, 2], T: [n, cells]) as torch tensors on the GPU;
    with fields given, the whole-field pairs (x, t) are appended to it"""
    import torch
    cfg = configs.get(workload)
    m = cfg["mesh"]
    ndim = 2 if m["ny"] == 1 else 3
    cs = 128 if ndim == 2 else 32
    cfg["params"].update(tol=1e-8, inner_tol=1e-4, max_iter=200000)
    S = gea.Solver(m, cfg["params"], solver="mixed", device=device)
    L = learned._lib()
    rng = np.random.default_rng(seed)
    nc = S.nc
    r = torch.empty(nc, dtype=torch.float32, device=device)
    a = torch.empty_like(r)
    d = torch.empty_like(r)
    Xs, Ts = [], []
    shape = (m["nz"], m["nx"]) if ndim == 2 else (m["nz"], m["ny"], m["nx"])
    t0 = time.time()
    for run in range(runs):
        b = draw_bubble(rng, cfg)
        S.init_bubble(**b)
        S.step(int(rng.integers(1, 5)))
        sc = C.c_double(0.0)
        rc = L.gea_make_pair(S.ctx, 1e-12, C.c_void_p(r.data_ptr()), C.c_void_p(a.data_ptr()),
                             C.c_void_p(d.data_ptr()), C.byref(sc), gea.DEVICE)
        if rc != gea.OK:
            raise gea.GeaError(rc, "gea_make_pair")
        R, A, D = (v.view(shape) for v in (r, a, d))
        if fields is not None:
            fields.append((torch.stack([r, a], dim=-1).clone(), d.clone()))
        tries = 0
        kept = 0
        floor = 0.05 if crop_scale == "local" else 1e-6
        while kept < crops_per_run and tries < 20 * crops_per_run:
            tries += 1
            o = [int(rng.integers(0, n - cs + 1)) for n in shape]
            sl = tuple(slice(oi, oi + cs) for oi in o)
            rr, aa, dd = R[sl], A[sl], D[sl]
            s = float(rr.abs().max())   # the full field has max |r0/s| = 1
            if s < floor:
                continue
            kept += 1
            if crop_scale == "global":
                s = 1.0
            Xs.append(torch.stack([rr / s, aa], dim=-1).reshape(-1, 2).clone())
            Ts.append((dd / s).reshape(-1).clone())
        if run % 10 == 0:
            log(f"[pairs] {workload} seed {seed}: run {run + 1}/{runs}, {len(Xs)} crops, "
                f"{time.time() - t0:.1f} s")
    S.close()
    return torch.stack(Xs), torch.stack(Ts), ndim, cs


# pair sources of the default training set: (workload, pairs a seed-0 set of
# 20000 holds; a run gives one pair a step)
SOURCES = {2: [("bubble2d_64x32", 10000), ("bubble2d_1280x640", 8500), ("nonsmooth2d_2048", 1500)],
           3: [("bubble3d_64x64x32_train", 20000)]}
EVAL_WORKLOAD = {2: "nonsmooth2d_2048", 3: "bubble3d_256x256x128"}


def make_source_pairs(ndim: int, total: int, seed: int, device="cuda:0", cs: int = 32,
                      steps_per_run: int = 100):
    """one cs^ndim crop (rescaled by its own max |r0|, at least 5 % of the
    field's maximum) from each of `total` pairs dumped step by step from
    runs of the source workloads (shares as in SOURCES)"""
    import torch
    L = learned._lib()
    rng = np.random.default_rng(seed)
    ref = sum(n for _, n in SOURCES[ndim])
    Xs, Ts = [], []
    t0 = time.time()
    for wl, share in SOURCES[ndim]:
        want = max(1, round(total * share / ref))
        cfg = configs.get(wl)
        m = cfg["mesh"]
        cfg["params"].update(tol=1e-8, inner_tol=1e-4, max_iter=200000)
        S = gea.Solver(m, cfg["params"], solver="mixed", device=device)
        nc = S.nc
        r = torch.empty(nc, dtype=torch.float32, device=device)
        a = torch.empty_like(r)
        d = torch.empty_like(r)
        shape = (m["nz"], m["nx"]) if ndim == 2 else (m["nz"], m["ny"], m["nx"])
        R, A, D = (v.view(shape) for v in (r, a, d))
        got = 0
        n_step = steps_per_run
        t_log = time.time()
        while got < want:
            if n_step >= steps_per_run:
                S.init_bubble(**draw_bubble(rng, cfg))
                n_step = 0
            rc, st = S.step_status(1)
            n_step += 1
            if rc != gea.OK:       # a bubble the mesh cannot carry: draw another
                n_step = steps_per_run
                continue
            sc = C.c_double(0.0)
            rc = L.gea_make_pair(S.ctx, 1e-12, C.c_void_p(r.data_ptr()), C.c_void_p(a.data_ptr()),
                                 C.c_void_p(d.data_ptr()), C.byref(sc), gea.DEVICE)
            if rc != gea.OK:
                raise gea.GeaError(rc, "gea_make_pair")
            for _ in range(20):
                o = [int(rng.integers(0, n - cs + 1)) for n in shape]
                sl = tuple(slice(oi, oi + cs) for oi in o)
                s = float(R[sl].abs().max())
                if s >= 0.05:
                    Xs.append(torch.stack([R[sl] / s, A[sl]], dim=-1).reshape(-1, 2).clone())
                    Ts.append((D[sl] / s).reshape(-1).clone())
                    got += 1
                    break
            if time.time() - t_log > 10.0 or got == want:
                t_log = time.time()
                log(f"[pairs] {wl} seed {seed}: {got}/{want} pairs ({time.time() - t0:.1f} s)")
        S.close()
    return torch.stack(Xs), torch.stack(Ts), cs


def eval_fields(ndim: int, runs: int, seed: int, device="cuda:0"):
    """whole-field pairs (x, t) of the evaluation workload (held out)"""
    fields = []
    make_pairs(EVAL_WORKLOAD[ndim], runs, 1, seed=seed, device=device, fields=fields)
    return fields


def rel_error(net, X, T) -> float:
    """||y - t|| / ||t|| over held-out crops"""
    num = den = 0.0
    for i in range(X.shape[0]):
        y = net.forward(X[i])
        num += float(((y - T[i]) ** 2).sum())
        den += float((T[i] ** 2).sum())
    return (num / den) ** 0.5


def train(X, T, ndim, cs, steps: int, batch: int, lr: float, seed: int = 0, Xv=None, Tv=None):
    import torch
    shape = (cs, 1, cs) if ndim == 2 else (cs, cs, cs)
    net = learned.Net(ndim, *shape, train=True)
    net.set_params(he_init(ndim, seed))
    rng = np.random.default_rng(seed + 100)
    n = X.shape[0]
    losses = []
    t0 = time.time()
    for step in range(1, steps + 1):
        # cosine decay of the learning rate
        lr_s = lr * 0.5 * (1 + np.cos(np.pi * (step - 1) / steps))
        acc = 0.0
        for k in range(batch):
            i = int(rng.integers(0, n))
            net.forward(X[i])
            acc += net.backward(T[i], accumulate=k > 0)
        net.adam(lr_s, step, grad_scale=1.0 / batch)
        losses.append(acc / batch)
        if step % 200 == 0 or step == 1:
            msg = f"[train] step {step}/{steps} loss {np.mean(losses[-200:]):.4e} ({time.time() - t0:.1f} s)"
            if Xv is not None:
                msg += f" held-out {evaluate(net, Xv, Tv):.4e}"
            log(msg)
    torch.cuda.synchronize()
    return net, losses


def field_error(ndim, shape, params, fields) -> float:
    """mean over whole fields of min_c ||c net(x) - t|| / ||t|| (the output
    scale is free: the solver takes the optimal step along it)"""
    import torch
    nz, ny, nx = (shape[0], 1, shape[1]) if ndim == 2 else shape
    net = learned.Net(ndim, nx, ny, nz, train=False)
    net.set_params(params)
    errs = []
    for x, t in fields:
        y = net.forward(x.contiguous()).double()
        t = t.double()
        c = float((y * t).sum() / (y * y).sum().clamp_min(1e-300))
        errs.append(float((c * y - t).norm() / t.norm()))
    net.close()
    torch.cuda.synchronize()
    return float(np.mean(errs))


def evaluate(net, X, T) -> float:
    """mean loss and the relative error of the correction, over held-out crops"""
    tot = 0.0
    for i in range(X.shape[0]):
        y = net.forward(X[i])
        tot += float(((y - T[i]) ** 2).sum() / (2 * y.numel()))
    return tot / X.shape[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ndim", type=int, default=2)
    ap.add_argument("--data", choices=("sources", "workload"), default="sources")
    ap.add_argument("--pairs", type=int, default=20000, help="--data sources: training pairs")
    ap.add_argument("--heldout-pairs", type=int, default=400)
    ap.add_argument("--workload", default=None, help="--data workload: default the evaluation mesh")
    ap.add_argument("--runs", type=int, default=40)
    ap.add_argument("--crops", type=int, default=50)
    ap.add_argument("--eval-runs", type=int, default=4)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--crop-scale", choices=("local", "global"), default="local")
    args = ap.parse_args()
    ndim = args.ndim
    if args.data == "sources":
        X, T, cs = make_source_pairs(ndim, args.pairs, seed=0)
        Xv, Tv, _ = make_source_pairs(ndim, args.heldout_pairs, seed=1)
        fields = eval_fields(ndim, args.eval_runs, seed=1)
        workload = "+".join(w for w, _ in SOURCES[ndim])
    else:
        workload = args.workload or EVAL_WORKLOAD[ndim]
        X, T, ndim, cs = make_pairs(workload, args.runs, args.crops, seed=0,
                                    crop_scale=args.crop_scale)
        fields = []
        Xv, Tv, _, _ = make_pairs(workload, args.eval_runs, 16, seed=1,
                                  crop_scale=args.crop_scale, fields=fields)
    sigma = float(T.pow(2).mean().sqrt())
    T /= sigma
    Tv /= sigma
    log(f"[pairs] {X.shape[0]} training crops, {Xv.shape[0]} held-out crops of {cs}^{ndim}, "
        f"target RMS {sigma:.4e}")
    net, losses = train(X, T, ndim, cs, args.steps, args.batch, args.lr, Xv=Xv, Tv=Tv)
    ev = evaluate(net, Xv, Tv)
    rel = rel_error(net, Xv, Tv)
    base = float(sum(float((Tv[i] ** 2).sum() / (2 * Tv[i].numel())) for i in range(Tv.shape[0])) / Tv.shape[0])
    out = args.out or weights_path(ndim)
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    params = net.get_params()
    np.save(out, params)
    m = configs.get(EVAL_WORKLOAD[ndim] if args.data == "sources" else workload)["mesh"]
    shape = (m["nz"], m["nx"]) if ndim == 2 else (m["nz"], m["ny"], m["nx"])
    ferr = field_error(ndim, shape, params, fields)
    summary = dict(data=args.data, workload=workload, ndim=ndim, crop=cs, crop_scale=args.crop_scale,
                   heldout_field_rel_error=ferr, train_crops=int(X.shape[0]),
                   heldout_crops=int(Xv.shape[0]), steps=args.steps, batch=args.batch,
                   first_loss=float(np.mean(losses[:20])), last_loss=float(np.mean(losses[-200:])),
                   heldout_loss=ev, heldout_zero_predictor_loss=base, heldout_rel_error=rel,
                   target_rms=sigma, out=out)
    log("[train] " + json.dumps(summary))


if __name__ == "__main__":
    main()
