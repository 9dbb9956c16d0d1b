"""Workload definitions: meshes, physical constants, time steps and bubbles.

Plain numbers only (no arithmetic of the method).  The rising-bubble family is
the one of Sec. 4 (smooth bubble, eq. dcEqn1; non-smooth bubble, eq. dcEqn2),
at the sizes the benchmarks and parity tests use.  Both the GPU library and
the CPU oracle receive these numbers unchanged.

Bubble kinds: 0 none, 1 cosine theta' = amp/2 (1 + cos(pi r/rc)) for r <= rc,
2 uniform theta' = amp for r <= rc.
"""
from __future__ import annotations

import copy

AIR = dict(R=287.0, cp=1004.0, cv=717.0, g=9.81, p0=1.0e5, theta0=300.0, Pr=1.0)


def _cfg(name, nx, ny, nz, lx, ly, lz, dt, mu, steps, bubble, solver, tol, **extra):
    params = dict(AIR, mu=mu, dt=dt, n_corr=2, n_energy_sweeps=2, tol=tol,
                  max_iter=extra.pop("max_iter", 20000))
    return dict(name=name, mesh=dict(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz),
                params=params, bubble=bubble, steps=steps, solver=solver, **extra)


# 2D meshes are one cell thick in y; that cell is as deep as it is wide.
CONFIGS = {
    # smooth bubble, 64x32 over 20 km x 10 km, plain FP64 (parity workload)
    "bubble2d_64x32": _cfg(
        "bubble2d_64x32", 64, 1, 32, 20000.0, 312.5, 10000.0, dt=1.0, mu=0.15, steps=20,
        bubble=dict(kind=1, xc=10000.0, yc=0.0, zc=2000.0, rc=2000.0, amp=2.0),
        solver="pcg64", tol=1e-13),
    # the same bubble at 15.625 m
    "bubble2d_1280x640": _cfg(
        "bubble2d_1280x640", 1280, 1, 640, 20000.0, 15.625, 10000.0, dt=0.1, mu=0.15,
        steps=2000, bubble=dict(kind=1, xc=10000.0, yc=0.0, zc=2000.0, rc=2000.0, amp=2.0),
        solver="pcg64", tol=1e-10),
    # non-smooth bubble of Sec. 4 on a 2048^2 mesh over 1 km x 1 km
    "nonsmooth2d_2048": _cfg(
        "nonsmooth2d_2048", 2048, 1, 2048, 1000.0, 1000.0 / 2048, 1000.0, dt=0.1, mu=0.3,
        steps=500, bubble=dict(kind=2, xc=500.0, yc=0.0, zc=260.0, rc=250.0, amp=0.5),
        solver="mixed", tol=1e-8, max_iter=200000),
    # 3D smooth bubble, 384x384x192 over 20 km x 20 km x 10 km
    "bubble3d_384x384x192": _cfg(
        "bubble3d_384x384x192", 384, 384, 192, 20000.0, 20000.0, 10000.0, dt=0.5, mu=0.15,
        steps=200, bubble=dict(kind=1, xc=10000.0, yc=10000.0, zc=2000.0, rc=2000.0, amp=2.0),
        solver="mixed", tol=1e-8),
    # evaluation meshes of the learned preconditioner
    "bubble3d_256x256x128": _cfg(
        "bubble3d_256x256x128", 256, 256, 128, 20000.0, 20000.0, 10000.0, dt=0.5, mu=0.15,
        steps=200, bubble=dict(kind=1, xc=10000.0, yc=10000.0, zc=2000.0, rc=2000.0, amp=2.0),
        solver="learned", tol=1e-8),
}
# small 3D runs for the 3D network's training pairs: the evaluation mesh's
# 78 m cells and time step on a 5 km x 5 km x 2.5 km box
CONFIGS["bubble3d_64x64x32_train"] = _cfg(
    "bubble3d_64x64x32_train", 64, 64, 32, 5000.0, 5000.0, 2500.0, dt=0.5, mu=0.15, steps=100,
    bubble=dict(kind=1, xc=2500.0, yc=2500.0, zc=800.0, rc=500.0, amp=2.0),
    solver="mixed", tol=1e-8)
# The paper's own validation runs (Sec. 4): the 1000 m x 1000 m box, c_v = 715.5 and
# c_p = R + c_v, dt 0.1 s, to 600 s; the smooth bubble (eq. dcEqn1: 0.5 K peak, r_c 250 m,
# centre (500, 350) m, mu 0.15) on 5 m cells and the non-smooth one (eq. dcEqn2: 0.5 K,
# centre (500, 260) m, mu 0.3) on 5 m and 10 m cells.
AIR_PAPER = dict(AIR, cv=715.5, cp=287.0 + 715.5)


def _paper(name, n, mu, bubble):
    c = _cfg(name, n, 1, n, 1000.0, 1000.0 / n, 1000.0, dt=0.1, mu=mu, steps=6000, bubble=bubble,
             solver="pcg64", tol=1e-10, max_iter=100000)
    c["params"].update(cv=AIR_PAPER["cv"], cp=AIR_PAPER["cp"])
    return c


CONFIGS["paper_smooth_5m"] = _paper(
    "paper_smooth_5m", 200, 0.15, dict(kind=1, xc=500.0, yc=0.0, zc=350.0, rc=250.0, amp=0.5))
CONFIGS["paper_nonsmooth_5m"] = _paper(
    "paper_nonsmooth_5m", 200, 0.3, dict(kind=2, xc=500.0, yc=0.0, zc=260.0, rc=250.0, amp=0.5))
CONFIGS["paper_nonsmooth_10m"] = _paper(
    "paper_nonsmooth_10m", 100, 0.3, dict(kind=2, xc=500.0, yc=0.0, zc=260.0, rc=250.0, amp=0.5))
CONFIGS["nonsmooth2d_2048_eval"] = dict(copy.deepcopy(CONFIGS["nonsmooth2d_2048"]),
                                        name="nonsmooth2d_2048_eval", solver="learned")


def get(name: str, **overrides) -> dict:
    """A deep copy of a workload; keyword overrides go into ``params``."""
    cfg = copy.deepcopy(CONFIGS[name])
    for k, v in overrides.items():
        if k in cfg["mesh"]:
            cfg["mesh"][k] = v
        else:
            cfg["params"][k] = v
    return cfg


def scaled(name: str, nx: int, nz: int, ny: int | None = None) -> dict:
    """A workload with the same physical domain on a different mesh."""
    cfg = get(name)
    m = cfg["mesh"]
    m["nx"], m["nz"] = nx, nz
    if m["ny"] == 1:
        m["ly"] = m["lx"] / nx
    elif ny is not None:
        m["ny"] = ny
    return cfg
