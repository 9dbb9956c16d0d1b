"""Python binding of the C-ABI library ``libgea.so`` (declared in include/gea.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch supplies device memory (the workspace and any device
arrays passed in or out) and the HIP stream.  The library must have been
built (``paper_2303_10499_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GEA_LIB_PATH overrides the library file (e.g. a build with other tuning)
LIB_PATH = os.environ.get("GEA_LIB_PATH") or os.path.join(_HERE, "libgea.so")

OK, ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_NOCONV, ERR_NAN, ERR_STATE = 0, -1, -2, -3, -4, -5, -6
HOST, DEVICE = 0, 1
PCG_JACOBI_FP64, IR_FP32_FP64, LEARNED_MIXED = 0, 1, 2
SOLVERS = {"pcg64": PCG_JACOBI_FP64, "mixed": IR_FP32_FP64, "learned": LEARNED_MIXED}

FIELD_RHO, FIELD_U, FIELD_T, FIELD_PPRIME, FIELD_P, FIELD_C, FIELD_D, FIELD_B, FIELD_PHI = (
    1 << 0, 1 << 1, 1 << 2, 1 << 3, 1 << 4, 1 << 5, 1 << 6, 1 << 7, 1 << 8)
FIELD_HISTORY = 1 << 9


class GeaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gea status {status}: {msg}")
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double)]


class Params(C.Structure):
    _fields_ = [("R", C.c_double), ("cp", C.c_double), ("cv", C.c_double), ("g", C.c_double),
                ("p0", C.c_double), ("theta0", C.c_double), ("mu", C.c_double),
                ("Pr", C.c_double), ("dt", C.c_double), ("n_corr", C.c_int32),
                ("n_energy_sweeps", C.c_int32), ("solver", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("check_every", C.c_int32), ("inner_tol", C.c_double),
                ("learned_steps", C.c_int32), ("inner_target", C.c_double),
                ("learned_always", C.c_int32), ("energy_form", C.c_int32),
                ("transport", C.c_int32)]


class Bubble(C.Structure):
    _fields_ = [("kind", C.c_int32), ("xc", C.c_double), ("yc", C.c_double),
                ("zc", C.c_double), ("rc", C.c_double), ("amp", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("fallbacks", C.c_int32),
                ("status", C.c_int32), ("rel_res0", C.c_double), ("rel_res", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepStats(C.Structure):
    _fields_ = [("steps_done", C.c_int32), ("n_solves", C.c_int32), ("solve", SolveStats * 8),
                ("total_iters", C.c_int64), ("total_solves", C.c_int64),
                ("eos_mismatch", C.c_double), ("mass", C.c_double),
                ("max_rel_res", C.c_double), ("total_fallbacks", C.c_int64),
                ("energy_iters", C.c_int64), ("transport_iters", C.c_int64)]


class Extrema(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("u_min", "u_max", "v_min", "v_max", "w_min", "w_max",
                                           "theta_min", "theta_max")]


_lib = None


def lib():
    """Load libgea.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2303_10499_amd.build")
        L = C.CDLL(LIB_PATH)
        P, vp, dp = C.POINTER, C.c_void_p, C.c_void_p
        L.gea_workspace_bytes.argtypes = [P(Mesh), P(Params), P(C.c_size_t)]
        L.gea_init_mesh.argtypes = [P(Mesh), P(Params), vp, vp, C.c_size_t, P(vp)]
        L.gea_set_solver.argtypes = [vp, C.c_int32, C.c_double, C.c_int32, C.c_double]
        L.gea_init_bubble.argtypes = [vp, P(Bubble)]
        L.gea_set_state.argtypes = [vp, dp, dp, dp, dp, dp, dp, C.c_int]
        L.gea_set_face_flux.argtypes = [vp, dp, C.c_int]
        L.gea_set_history.argtypes = [vp, dp, dp, C.c_int]
        L.gea_step.argtypes = [vp, C.c_int32, P(StepStats)]
        L.gea_pressure_solve.argtypes = [vp, dp, dp, C.c_int, P(SolveStats)]
        L.gea_apply_pressure_operator.argtypes = [vp, dp, dp, C.c_int]
        L.gea_get_fields.argtypes = [vp, C.c_uint32, dp, C.c_int]
        L.gea_kernel_timing.argtypes = [vp, C.c_int32, C.c_int32]
        L.gea_kernel_times.argtypes = [vp, P(C.c_double), P(C.c_int64)]
        L.gea_time_solver_kernels.argtypes = [vp, C.c_int32, P(C.c_double)]
        L.gea_time_network.argtypes = [vp, C.c_int32, P(C.c_double), P(C.c_double)]
        L.gea_state_extrema.argtypes = [vp, P(Extrema)]
        L.gea_pressure_solve_static.argtypes = [P(Mesh), dp, dp, dp, dp, C.c_double, C.c_int32,
                                                vp, P(SolveStats)]
        L.gea_destroy.argtypes = [vp]
        L.gea_destroy.restype = None
        L.gea_last_error.argtypes = [vp]
        L.gea_last_error.restype = C.c_char_p
        for name in ("gea_workspace_bytes", "gea_init_mesh", "gea_set_solver", "gea_init_bubble",
                     "gea_set_state", "gea_step", "gea_pressure_solve",
                     "gea_apply_pressure_operator", "gea_get_fields", "gea_kernel_timing",
                     "gea_kernel_times", "gea_time_solver_kernels", "gea_time_network",
                     "gea_pressure_solve_static", "gea_state_extrema", "gea_set_face_flux",
                     "gea_set_history"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def make_mesh(m: dict) -> Mesh:
    return Mesh(int(m["nx"]), int(m["ny"]), int(m["nz"]), float(m["lx"]), float(m["ly"]),
                float(m["lz"]))


def make_params(p: dict, solver="pcg64") -> Params:
    s = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    return Params(*(float(p[k]) for k in ("R", "cp", "cv", "g", "p0", "theta0", "mu", "Pr", "dt")),
                  int(p.get("n_corr", 2)), int(p.get("n_energy_sweeps", 2)), s,
                  float(p.get("tol", 1e-10)), int(p.get("max_iter", 20000)),
                  int(p.get("check_every", 8)), float(p.get("inner_tol", 1e-4)),
                  int(p.get("learned_steps", 1)), float(p.get("inner_target", 0.0)),
                  int(p.get("learned_always", 0)), int(p.get("energy_form", 0)),
                  int(p.get("transport", 0)))


def _ptr(a):
    """(address, kind) of a contiguous FP64 torch tensor or numpy array."""
    if isinstance(a, np.ndarray):
        assert a.dtype == np.float64 and a.flags.c_contiguous
        return a.ctypes.data, HOST
    import torch
    assert isinstance(a, torch.Tensor) and a.dtype == torch.float64 and a.is_contiguous()
    return a.data_ptr(), (DEVICE if a.is_cuda else HOST)


class Solver:
    """One context of the library on one mesh (see include/gea.h)."""

    def __init__(self, mesh: dict, params: dict, solver="pcg64", device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.L = lib()
        self.mesh = make_mesh(mesh)
        self.params = make_params(params, solver)
        self.ndim = 2 if self.mesh.ny == 1 else 3
        self.nc = self.mesh.nx * self.mesh.ny * self.mesh.nz
        nbytes = C.c_size_t(0)
        self._check(self.L.gea_workspace_bytes(C.byref(self.mesh), C.byref(self.params),
                                               C.byref(nbytes)), None)
        self.workspace_bytes = nbytes.value
        # torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        self._check(self.L.gea_init_mesh(C.byref(self.mesh), C.byref(self.params),
                                         C.c_void_p(self.stream.cuda_stream),
                                         C.c_void_p(self.workspace.data_ptr()),
                                         self.workspace_bytes, C.byref(ctx)), None)
        self.ctx = ctx

    def _check(self, rc, ctx):
        if rc != OK:
            msg = self.L.gea_last_error(ctx).decode()
            raise GeaError(rc, msg)

    def close(self):
        if getattr(self, "ctx", None):
            self.L.gea_destroy(self.ctx)
            self.ctx = None

    __del__ = close

    # ---- API ---------------------------------------------------------------
    def set_solver(self, solver, tol, max_iter=None, inner_tol=None):
        s = SOLVERS[solver] if isinstance(solver, str) else int(solver)
        mi = int(max_iter if max_iter is not None else self.params.max_iter)
        it = float(inner_tol if inner_tol is not None else self.params.inner_tol)
        self._check(self.L.gea_set_solver(self.ctx, s, float(tol), mi, it), self.ctx)
        self.params.solver, self.params.tol, self.params.max_iter, self.params.inner_tol = s, tol, mi, it

    def init_bubble(self, kind, xc=0.0, yc=0.0, zc=0.0, rc=1.0, amp=0.0):
        b = Bubble(int(kind), float(xc), float(yc), float(zc), float(rc), float(amp))
        self._check(self.L.gea_init_bubble(self.ctx, C.byref(b)), self.ctx)

    def set_state(self, rho, u, T, pp, p, Tbg):
        arrs = [rho, u, T, pp, p, Tbg]
        ptrs = [_ptr(a) for a in arrs]
        kinds = {k for _, k in ptrs}
        assert len(kinds) == 1, "all arrays must live on the same side"
        self._check(self.L.gea_set_state(self.ctx, *[C.c_void_p(q) for q, _ in ptrs], kinds.pop()),
                    self.ctx)

    def set_history(self, p_old, K_old):
        """the enthalpy form's lagged terms p^{n-1}, K^{n-1} of the current state"""
        (q1, k1), (q2, k2) = _ptr(p_old), _ptr(K_old)
        assert k1 == k2, "both arrays must live on the same side"
        self._check(self.L.gea_set_history(self.ctx, C.c_void_p(q1), C.c_void_p(q2), k1), self.ctx)

    def history(self):
        """(p^{n-1}, K^{n-1}) of the current state (host arrays)"""
        f = self.get_fields(FIELD_HISTORY)
        return f[0], f[1]

    def set_face_flux(self, phi):
        """replace the state's face mass flux ((ndim, nc) values, GEA_FIELD_PHI layout)"""
        q, kind = _ptr(phi)
        self._check(self.L.gea_set_face_flux(self.ctx, C.c_void_p(q), kind), self.ctx)

    def step(self, nsteps=1) -> StepStats:
        st = StepStats()
        self._check(self.L.gea_step(self.ctx, int(nsteps), C.byref(st)), self.ctx)
        return st

    def step_status(self, nsteps=1):
        """(status, stats) without raising."""
        st = StepStats()
        return self.L.gea_step(self.ctx, int(nsteps), C.byref(st)), st

    def pressure_solve(self, x, b=None):
        """Solve the next step's first-corrector pressure system; x: initial
        guess in, solution out (torch tensor or numpy array)."""
        st = SolveStats()
        xp, kind = _ptr(x)
        bp = C.c_void_p(_ptr(b)[0]) if b is not None else None
        rc = self.L.gea_pressure_solve(self.ctx, bp, C.c_void_p(xp), kind, C.byref(st))
        self._check(rc, self.ctx)
        return st

    def apply_A(self, x, y):
        xp, kind = _ptr(x)
        yp, _ = _ptr(y)
        self._check(self.L.gea_apply_pressure_operator(self.ctx, C.c_void_p(xp), C.c_void_p(yp),
                                                       kind), self.ctx)

    def extrema(self):
        """extrema of u, v, w and theta' of the current state (a dict)"""
        e = Extrema()
        self._check(self.L.gea_state_extrema(self.ctx, C.byref(e)), self.ctx)
        return {n: getattr(e, n) for n, _ in Extrema._fields_}

    def get_fields(self, mask, host=True):
        n = 0
        for bit in range(10):
            if mask & (1 << bit):
                n += self.ndim if (1 << bit) in (FIELD_U, FIELD_PHI) else \
                    2 if (1 << bit) == FIELD_HISTORY else 1
        if host:
            out = np.empty((n, self.nc), dtype=np.float64)
        else:
            out = self.torch.empty((n, self.nc), dtype=self.torch.float64, device=self.device)
        p, kind = _ptr(out)
        self._check(self.L.gea_get_fields(self.ctx, int(mask), C.c_void_p(p), kind), self.ctx)
        return out

    def load_weights(self, params=None):
        """give the learned form its network weights (packed FP32; default:
        the trained weights shipped with the package for this dimension)"""
        from . import learned
        if params is None:
            params = np.load(learned.weights_file(self.ndim), allow_pickle=False)
        params = np.ascontiguousarray(params, dtype=np.float32)
        L = learned._lib()
        self._check(L.gea_load_weights(self.ctx, C.c_void_p(params.ctypes.data), HOST), self.ctx)

    def kernel_timing(self, on: bool, reset: bool = True):
        self._check(self.L.gea_kernel_timing(self.ctx, int(on), int(reset)), self.ctx)

    def kernel_times(self):
        """(ms[8], launches[8]) summed per kernel class since the last reset"""
        ms = (C.c_double * 8)()
        n = (C.c_int64 * 8)()
        self._check(self.L.gea_kernel_times(self.ctx, ms, n), self.ctx)
        return list(ms), list(n)

    def time_solver_kernels(self, reps=50):
        """average ms per launch: FP64 spmv, FP64 update, FP32 spmv, FP32 update"""
        ms = (C.c_double * 4)()
        self._check(self.L.gea_time_solver_kernels(self.ctx, int(reps), ms), self.ctx)
        return list(ms)

    def time_network(self, reps=20):
        """average ms per launch and GFLOP per launch of the six forward convolutions"""
        ms = (C.c_double * 6)()
        gf = (C.c_double * 6)()
        self._check(self.L.gea_time_network(self.ctx, int(reps), ms, gf), self.ctx)
        return list(ms), list(gf)

    def state(self):
        """dict of host arrays: rho, u (ndim, nc), T, pp, p, phi (ndim, nc)"""
        f = self.get_fields(FIELD_RHO | FIELD_U | FIELD_T | FIELD_PPRIME | FIELD_P | FIELD_PHI)
        d = self.ndim
        return dict(rho=f[0], u=f[1:1 + d], T=f[1 + d], pp=f[2 + d], p=f[3 + d],
                    phi=f[4 + d:4 + 2 * d])


def pressure_solve_static(mesh: dict, c, D, b, x, tol, max_iter=20000, stream=None):
    """gea_pressure_solve_static: FP64 Jacobi-PCG of the system (c, D, b) from
    the initial guess in x (solution written to x); c, D, b, x contiguous FP64
    CUDA tensors of ncell values.  Allocates no device memory."""
    import torch
    for a in (c, D, b, x):
        assert isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()
    m = make_mesh(mesh)
    st = SolveStats()
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    L = lib()
    rc = L.gea_pressure_solve_static(C.byref(m), C.c_void_p(c.data_ptr()), C.c_void_p(D.data_ptr()),
                                     C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(tol),
                                     int(max_iter), C.c_void_p(stream.cuda_stream), C.byref(st))
    if rc != OK:
        raise GeaError(rc, L.gea_last_error(None).decode())
    return st
