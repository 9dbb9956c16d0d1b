"""ctypes binding of the plain FP64 CPU oracle (``geao.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It imports
nothing from the GPU package; inputs are plain numbers and numpy arrays.

Every array is FP64, structure-of-arrays, index ``i + nx*(j + ny*k)``; the
velocity holds ``ndim`` blocks of ``ncell`` values ((u, w) in 2D, (u, v, w) in
3D).  See ``geao.h`` for the passage of the paper each routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "geao.c")
_LIB = os.path.join(_HERE, "libgeao.so")
_LIB_OMP = os.path.join(_HERE, "libgeao_omp.so")


def build(force: bool = True, omp: bool = False) -> str:
    """Compile ``libgeao.so`` with plain gcc -O2 (no fast-math, one thread);
    with omp, ``libgeao_omp.so`` from the same source with -fopenmp (its
    per-cell loops shared among threads, every reduction serial: the same
    results bit for bit, used only to time the oracle on all host cores)."""
    out = _LIB_OMP if omp else _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared"]
            + (["-fopenmp"] if omp else []) + ["-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, out)
    return out


class Mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double)]


class Params(C.Structure):
    _fields_ = [("R", C.c_double), ("cp", C.c_double), ("cv", C.c_double),
                ("g", C.c_double), ("p0", C.c_double), ("theta0", C.c_double),
                ("mu", C.c_double), ("Pr", C.c_double), ("dt", C.c_double),
                ("n_corr", C.c_int32), ("n_energy_sweeps", C.c_int32),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("energy_form", C.c_int32),
                ("transport", C.c_int32)]


class Bubble(C.Structure):
    _fields_ = [("kind", C.c_int32), ("xc", C.c_double), ("yc", C.c_double),
                ("zc", C.c_double), ("rc", C.c_double), ("amp", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32),
                ("rel_res0", C.c_double), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("n_solves", C.c_int32), ("solve", SolveStats * 16),
                ("eos_mismatch", C.c_double)]


OK, ERR_ARG, ERR_NOCONV, ERR_NAN = 0, -1, -4, -5

_libs = {}


def lib(omp: bool = False):
    if omp not in _libs:
        path = build(force=False, omp=omp)
        L = C.CDLL(path)
        P = C.POINTER
        d = P(C.c_double)
        L.geao_ndim.argtypes = [P(Mesh)]
        L.geao_init_bubble.argtypes = [P(Mesh), P(Params), P(Bubble), d, d, d, d, d, d]
        for name in ("geao_face_interp4", "geao_face_sngrad"):
            getattr(L, name).argtypes = [P(Mesh), d, C.c_int, d]
        L.geao_reconstruct.argtypes = [P(Mesh), d, d]
        L.geao_divergence.argtypes = [P(Mesh), d, d]
        L.geao_viscous.argtypes = [P(Mesh), d, C.c_int, C.c_double, d]
        L.geao_convective.argtypes = [P(Mesh), d, d, d]
        L.geao_potential.argtypes = [P(Mesh), P(Params), d]
        L.geao_mass_predictor.argtypes = [P(Mesh), P(Params), d, d, d, d]
        L.geao_momentum_predictor.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d]
        L.geao_energy.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d, d]
        L.geao_energy_enthalpy.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d, d, d, d]
        L.geao_momentum_operator.argtypes = [P(Mesh), P(Params), d, d, C.c_int, d, d]
        L.geao_energy_operator.argtypes = [P(Mesh), P(Params), d, d, d, d]
        L.geao_transport_diag.argtypes = [P(Mesh), P(Params), d, d, d, C.c_int, d]
        L.geao_bicgstab_momentum.argtypes = [P(Mesh), P(Params), d, d, C.c_int, d, d, C.c_double,
                                             C.c_int, P(SolveStats)]
        L.geao_momentum_predictor_implicit.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d]
        L.geao_energy_implicit.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d, d, d, d, d]
        L.geao_eos_coeffs.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d]
        L.geao_H.argtypes = [P(Mesh), P(Params), d, d, d, d, d]
        L.geao_predicted_flux_rhs.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d]
        L.geao_apply_A.argtypes = [P(Mesh), d, d, d, d]
        L.geao_pcg.argtypes = [P(Mesh), d, d, d, d, C.c_double, C.c_int, P(SolveStats)]
        L.geao_correct.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d, d]
        L.geao_finalize.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d, d]
        L.geao_pressure_system.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d, d, d, d, d, d]
        L.geao_step.argtypes = [P(Mesh), P(Params), d, d, d, d, d, d, d, d, d, P(StepStats)]
        L.geao_face_mass_flux.argtypes = [P(Mesh), d, d, d]
        L.geao_density_predictor.argtypes = [P(Mesh), P(Params), d, d, d]
        L.geao_theta_prime.argtypes = [P(Mesh), P(Params), d, d, d]
        L.geao_threads.argtypes = []
        L.geao_threads.restype = C.c_int
        _libs[omp] = L
    return _libs[omp]


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class State:
    rho: np.ndarray
    u: np.ndarray      # (ndim, ncell)
    T: np.ndarray
    pp: np.ndarray     # p'
    p: np.ndarray
    Tbg: np.ndarray    # (nz,)
    phi: np.ndarray = None  # (ndim, ncell) face mass flux; None: I4(rho u) S when first needed
    p_old: np.ndarray = None  # p^{n-1}; None: p^n (a state without history)
    K_old: np.ndarray = None  # K^{n-1}; None: K^n

    def copy(self) -> "State":
        return State(*(None if a is None else np.array(a, copy=True) for a in
                       (self.rho, self.u, self.T, self.pp, self.p, self.Tbg, self.phi,
                        self.p_old, self.K_old)))


class Oracle:
    """The oracle bound to one mesh and one parameter set (plain numbers)."""

    def __init__(self, mesh: dict, params: dict, omp: bool = False):
        self.mesh = Mesh(int(mesh["nx"]), int(mesh["ny"]), int(mesh["nz"]),
                         float(mesh["lx"]), float(mesh["ly"]), float(mesh["lz"]))
        self.params = Params(*(float(params[k]) for k in ("R", "cp", "cv", "g", "p0",
                                                          "theta0", "mu", "Pr", "dt")),
                             int(params.get("n_corr", 2)), int(params.get("n_energy_sweeps", 2)),
                             float(params.get("tol", 1e-13)), int(params.get("max_iter", 100000)),
                             int(params.get("energy_form", 0)), int(params.get("transport", 0)))
        self.L = lib(omp)
        self.ndim = 2 if self.mesh.ny == 1 else 3
        self.nc = self.mesh.nx * self.mesh.ny * self.mesh.nz

    # ---- helpers -----------------------------------------------------------
    def zeros(self, *lead) -> np.ndarray:
        return np.zeros(lead + (self.nc,), dtype=np.float64)

    def cell_centres(self):
        m = self.mesh
        dx, dy, dz = m.lx / m.nx, m.ly / m.ny, m.lz / m.nz
        k, j, i = np.meshgrid(np.arange(m.nz), np.arange(m.ny), np.arange(m.nx), indexing="ij")
        return ((i + 0.5) * dx).ravel(), ((j + 0.5) * dy).ravel(), ((k + 0.5) * dz).ravel()

    # ---- state -------------------------------------------------------------
    def init_bubble(self, kind: int, xc=0.0, yc=0.0, zc=0.0, rc=1.0, amp=0.0) -> State:
        s = State(self.zeros(), self.zeros(self.ndim), self.zeros(), self.zeros(), self.zeros(),
                  np.zeros(self.mesh.nz))
        b = Bubble(int(kind), float(xc), float(yc), float(zc), float(rc), float(amp))
        rc_ = self.L.geao_init_bubble(C.byref(self.mesh), C.byref(self.params), C.byref(b),
                                      _p(s.rho), _p(s.u), _p(s.T), _p(s.pp), _p(s.p), _p(s.Tbg))
        if rc_ != OK:
            raise ValueError(f"geao_init_bubble failed: {rc_}")
        s.phi = self.face_mass_flux(s.rho, s.u)
        return s

    def face_mass_flux(self, rho, u):
        phi = self.zeros(self.ndim)
        self.L.geao_face_mass_flux(C.byref(self.mesh), _p(np.ascontiguousarray(rho)),
                                   _p(np.ascontiguousarray(u)), _p(phi))
        return phi

    def _flux(self, s: State):
        if s.phi is None:
            s.phi = self.face_mass_flux(s.rho, s.u)
        return s.phi

    def _history(self, s: State):
        """p^{n-1}, K^{n-1} of the state; a state without history takes its own
        p^n and K^n = |u^n|^2/2 (so the lagged terms vanish on its first step)"""
        if s.p_old is None:
            s.p_old = np.array(s.p, copy=True)
        if s.K_old is None:
            s.K_old = 0.5 * np.sum(s.u * s.u, axis=0)
        return s.p_old, s.K_old

    def step(self, s: State, nsteps: int = 1) -> list:
        stats = []
        for _ in range(nsteps):
            st = StepStats()
            phi = self._flux(s)
            p_old, K_old = self._history(s)
            rc = self.L.geao_step(C.byref(self.mesh), C.byref(self.params), _p(s.rho), _p(s.u),
                                  _p(s.T), _p(s.pp), _p(s.p), _p(phi), _p(p_old), _p(K_old),
                                  _p(s.Tbg), C.byref(st))
            stats.append(st)
            if rc != OK:
                raise RuntimeError(f"geao_step failed with status {rc}")
        return stats

    def pressure_system(self, s: State):
        c, D, b = self.zeros(), self.zeros(), self.zeros()
        p_old, K_old = self._history(s)
        rc = self.L.geao_pressure_system(C.byref(self.mesh), C.byref(self.params), _p(s.rho),
                                         _p(s.u), _p(s.T), _p(s.pp), _p(s.p), _p(self._flux(s)),
                                         _p(p_old), _p(K_old), _p(s.Tbg), _p(c), _p(D), _p(b))
        if rc != OK:
            raise ValueError(f"geao_pressure_system failed: {rc}")
        return c, D, b

    def apply_A(self, c, D, x):
        y = self.zeros()
        self.L.geao_apply_A(C.byref(self.mesh), _p(np.ascontiguousarray(c)),
                            _p(np.ascontiguousarray(D)), _p(np.ascontiguousarray(x)), _p(y))
        return y

    def pcg(self, c, D, b, x0, tol, max_iter=100000):
        x = np.array(x0, dtype=np.float64, copy=True)
        st = SolveStats()
        rc = self.L.geao_pcg(C.byref(self.mesh), _p(np.ascontiguousarray(c)),
                             _p(np.ascontiguousarray(D)), _p(np.ascontiguousarray(b)), _p(x),
                             float(tol), int(max_iter), C.byref(st))
        return x, st, rc

    def theta_prime(self, s: State):
        out = self.zeros()
        self.L.geao_theta_prime(C.byref(self.mesh), C.byref(self.params), _p(s.T), _p(s.p), _p(out))
        return out

    # ---- operators ---------------------------------------------------------
    def face_interp4(self, s, d):
        out = self.zeros()
        self.L.geao_face_interp4(C.byref(self.mesh), _p(np.ascontiguousarray(s, dtype=np.float64)), d, _p(out))
        return out

    def face_sngrad(self, s, d):
        out = self.zeros()
        self.L.geao_face_sngrad(C.byref(self.mesh), _p(np.ascontiguousarray(s, dtype=np.float64)), d, _p(out))
        return out

    def reconstruct(self, faces):
        out = self.zeros(self.ndim)
        self.L.geao_reconstruct(C.byref(self.mesh), _p(np.ascontiguousarray(faces, dtype=np.float64)), _p(out))
        return out

    def divergence(self, faces):
        out = self.zeros()
        self.L.geao_divergence(C.byref(self.mesh), _p(np.ascontiguousarray(faces, dtype=np.float64)), _p(out))
        return out

    def viscous(self, uc, comp, mu):
        out = self.zeros()
        self.L.geao_viscous(C.byref(self.mesh), _p(np.ascontiguousarray(uc, dtype=np.float64)), comp, float(mu), _p(out))
        return out

    def convective(self, phi, s):
        out = self.zeros()
        self.L.geao_convective(C.byref(self.mesh), _p(np.ascontiguousarray(phi, dtype=np.float64)),
                               _p(np.ascontiguousarray(s, dtype=np.float64)), _p(out))
        return out

    def potential(self):
        out = self.zeros()
        self.L.geao_potential(C.byref(self.mesh), C.byref(self.params), _p(out))
        return out

    # ---- sub-steps ---------------------------------------------------------
    def mass_predictor(self, rho, u):
        phi, rs = self.zeros(self.ndim), self.zeros()
        self.L.geao_mass_predictor(C.byref(self.mesh), C.byref(self.params), _p(rho), _p(u), _p(phi), _p(rs))
        return phi, rs

    def density_predictor(self, rho, phi):
        rs = self.zeros()
        self.L.geao_density_predictor(C.byref(self.mesh), C.byref(self.params),
                                      _p(np.ascontiguousarray(rho)), _p(np.ascontiguousarray(phi)), _p(rs))
        return rs

    def momentum_predictor(self, rho, u, pp, rho_star, phi):
        us = self.zeros(self.ndim)
        self.L.geao_momentum_predictor(C.byref(self.mesh), C.byref(self.params), _p(rho), _p(u), _p(pp),
                                       _p(rho_star), _p(phi), _p(us))
        return us

    def energy(self, rho, u, T, u_star, rho_star, phi, Tbg):
        Tn = self.zeros()
        self.L.geao_energy(C.byref(self.mesh), C.byref(self.params), _p(rho), _p(u), _p(T), _p(u_star),
                           _p(rho_star), _p(phi), _p(Tbg), _p(Tn))
        return Tn

    def energy_enthalpy(self, rho, T, p, p_old, K_old, u_star, rho_star, phi, Tbg):
        Tn = self.zeros()
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in
             (rho, T, p, p_old, K_old, u_star, rho_star, phi, Tbg)]
        self.L.geao_energy_enthalpy(C.byref(self.mesh), C.byref(self.params), *[_p(x) for x in a],
                                    _p(Tn))
        return Tn

    # ---- implicit transport ------------------------------------------------
    def momentum_operator(self, rho_star, phi, comp, x):
        y = self.zeros()
        self.L.geao_momentum_operator(C.byref(self.mesh), C.byref(self.params),
                                      _p(np.ascontiguousarray(rho_star, dtype=np.float64)),
                                      _p(np.ascontiguousarray(phi, dtype=np.float64)), int(comp),
                                      _p(np.ascontiguousarray(x, dtype=np.float64)), _p(y))
        return y

    def energy_operator(self, cT, phi, x):
        y = self.zeros()
        self.L.geao_energy_operator(C.byref(self.mesh), C.byref(self.params),
                                    _p(np.ascontiguousarray(cT, dtype=np.float64)),
                                    _p(np.ascontiguousarray(phi, dtype=np.float64)),
                                    _p(np.ascontiguousarray(x, dtype=np.float64)), _p(y))
        return y

    def transport_diag(self, phi, comp, rho_star=None, cT=None):
        out = self.zeros()
        z = self.zeros()
        self.L.geao_transport_diag(C.byref(self.mesh), C.byref(self.params),
                                   _p(np.ascontiguousarray(z if rho_star is None else rho_star, dtype=np.float64)),
                                   _p(np.ascontiguousarray(z if cT is None else cT, dtype=np.float64)),
                                   _p(np.ascontiguousarray(phi, dtype=np.float64)), int(comp), _p(out))
        return out

    def bicgstab_momentum(self, rho_star, phi, comp, b, x0, tol, max_iter=1000):
        x = np.array(x0, dtype=np.float64, copy=True)
        st = SolveStats()
        rc = self.L.geao_bicgstab_momentum(C.byref(self.mesh), C.byref(self.params),
                                           _p(np.ascontiguousarray(rho_star, dtype=np.float64)),
                                           _p(np.ascontiguousarray(phi, dtype=np.float64)), int(comp),
                                           _p(np.ascontiguousarray(b, dtype=np.float64)), _p(x),
                                           float(tol), int(max_iter), C.byref(st))
        return x, st, rc

    def momentum_predictor_implicit(self, rho, u, pp, rho_star, phi, u_guess):
        us = np.array(u_guess, dtype=np.float64, copy=True)
        rc = self.L.geao_momentum_predictor_implicit(
            C.byref(self.mesh), C.byref(self.params), *[_p(np.ascontiguousarray(a, dtype=np.float64))
                                                        for a in (rho, u, pp, rho_star, phi)], _p(us))
        if rc != OK:
            raise RuntimeError(f"geao_momentum_predictor_implicit failed: {rc}")
        return us

    def energy_implicit(self, rho, u, T, p, p_old, K_old, u_star, rho_star, phi, Tbg):
        Tn = self.zeros()
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in
             (rho, u, T, p, p_old, K_old, u_star, rho_star, phi, Tbg)]
        rc = self.L.geao_energy_implicit(C.byref(self.mesh), C.byref(self.params), *[_p(x) for x in a],
                                         _p(Tn))
        if rc != OK:
            raise RuntimeError(f"geao_energy_implicit failed: {rc}")
        return Tn

    def eos_coeffs(self, p, T_new, rho_star):
        r23, psi, c, D = self.zeros(), self.zeros(), self.zeros(), self.zeros()
        self.L.geao_eos_coeffs(C.byref(self.mesh), C.byref(self.params), _p(p), _p(T_new), _p(rho_star),
                               _p(r23), _p(psi), _p(c), _p(D))
        return r23, psi, c, D

    def H(self, rho, u, u_prev, phi):
        H = self.zeros(self.ndim)
        self.L.geao_H(C.byref(self.mesh), C.byref(self.params), _p(rho), _p(u), _p(u_prev), _p(phi), _p(H))
        return H

    def predicted_flux_rhs(self, rho, rho23, psi, D, H):
        pt, b = self.zeros(self.ndim), self.zeros()
        self.L.geao_predicted_flux_rhs(C.byref(self.mesh), C.byref(self.params), _p(rho), _p(rho23), _p(psi),
                                       _p(D), _p(H), _p(pt), _p(b))
        return pt, b

    def correct(self, pp, rho23, H, D, rho_star, phi_tilde):
        phi, u = self.zeros(self.ndim), self.zeros(self.ndim)
        self.L.geao_correct(C.byref(self.mesh), C.byref(self.params), _p(pp), _p(rho23), _p(H), _p(D),
                            _p(rho_star), _p(phi_tilde), _p(phi), _p(u))
        return phi, u

    def finalize(self, rho_old, phi, pp, rho23, psi):
        rn, pn = self.zeros(), self.zeros()
        mm = C.c_double(0.0)
        self.L.geao_finalize(C.byref(self.mesh), C.byref(self.params), _p(rho_old), _p(phi), _p(pp),
                             _p(rho23), _p(psi), _p(rn), _p(pn), C.byref(mm))
        return rn, pn, mm.value
