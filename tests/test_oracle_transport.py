"""Pins of the oracle's implicit transport (reading R19: Steps 1 and 2 with
the convective and diffusive terms at the new level, as eqs. step2_sd and
step3_sd write them, solved by BiCGStab).

The operators are pinned on uniform fields (closed forms) and as the sum of
the separately pinned convective and viscous terms; their diagonals against
the assembled matrix; BiCGStab against a dense direct solve; the implicit
predictors against the explicit predictor where the transport vanishes and
against the fixed point of the explicit Picard iteration where it does not;
and the whole step by its invariants (rest, mass, symmetry) and as the
composition of the pinned sub-steps.
"""
import numpy as np
import pytest

from paper_2303_10499_amd import configs

MESH2 = dict(nx=7, ny=1, nz=6, lx=700.0, ly=100.0, lz=600.0)
MESH3 = dict(nx=5, ny=4, nz=6, lx=500.0, ly=400.0, lz=600.0)


def make(oracle_lib, mesh=MESH2, **over):
    par = dict(configs.AIR, mu=0.15, dt=0.7, n_corr=2, n_energy_sweeps=2, tol=1e-14,
               max_iter=5000, transport=1)
    par.update(over)
    return oracle_lib.Oracle(mesh, par), par


def flux(O, rng, scale=30.0):
    """a random face flux, zero on the upper walls"""
    m = O.mesh
    n = [m.nx, m.ny, m.nz] if O.ndim == 3 else [m.nx, m.nz]
    st = [1, m.nx, m.nx * m.ny] if O.ndim == 3 else [1, m.nx]
    phi = scale * rng.standard_normal((O.ndim, O.nc))
    for d in range(O.ndim):
        phi[d][(np.arange(O.nc) // st[d]) % n[d] == n[d] - 1] = 0.0
    return phi


def dense(apply, nc):
    """the matrix of a linear map by its action on the unit vectors"""
    M = np.zeros((nc, nc))
    for j in range(nc):
        e = np.zeros(nc)
        e[j] = 1.0
        M[:, j] = apply(e)
    return M


def volume(O):
    m = O.mesh
    return m.lx / m.nx * m.ly / m.ny * m.lz / m.nz


@pytest.mark.parametrize("mesh", [MESH2, MESH3])
def test_momentum_operator_is_time_plus_convection_minus_viscosity(oracle_lib, mesh):
    O, par = make(oracle_lib, mesh)
    rng = np.random.default_rng(0)
    rs = 1.0 + 0.1 * rng.random(O.nc)
    phi = flux(O, rng)
    x = rng.standard_normal(O.nc)
    V = volume(O)
    for comp in range(O.ndim):
        want = rs * V / par["dt"] * x + O.convective(phi, x) - O.viscous(x, comp, par["mu"])
        np.testing.assert_allclose(O.momentum_operator(rs, phi, comp, x), want, rtol=1e-13,
                                   atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("mesh", [MESH2, MESH3])
def test_operators_on_a_uniform_field(oracle_lib, mesh):
    """I4 of a constant is the constant, snGrad zero: A 1 = rho* V/dt +
    sum_out phi (+ the wall-normal component's wall friction 2 mu S/h on
    each wall face); the energy operator gives cT + c_p sum_out phi"""
    O, par = make(oracle_lib, mesh)
    rng = np.random.default_rng(1)
    rs = 1.0 + 0.1 * rng.random(O.nc)
    phi = flux(O, rng)
    one = np.ones(O.nc)
    V = volume(O)
    div = O.divergence(phi) * V
    m = O.mesh
    n = [m.nx, m.ny, m.nz] if O.ndim == 3 else [m.nx, m.nz]
    st = [1, m.nx, m.nx * m.ny] if O.ndim == 3 else [1, m.nx]
    h = [m.lx / m.nx, m.ly / m.ny, m.lz / m.nz] if O.ndim == 3 else [m.lx / m.nx, m.lz / m.nz]
    P = np.arange(O.nc)
    for comp in range(O.ndim):
        q = (P // st[comp]) % n[comp]
        walls = (q == 0).astype(float) + (q == n[comp] - 1).astype(float)
        S = V / h[comp]
        want = rs * V / par["dt"] + div + walls * 2.0 * par["mu"] * S / h[comp]
        np.testing.assert_allclose(O.momentum_operator(rs, phi, comp, one), want, rtol=1e-13)
    cT = rs * par["cp"] * V / par["dt"]
    np.testing.assert_allclose(O.energy_operator(cT, phi, one), cT + par["cp"] * div, rtol=1e-13)


@pytest.mark.parametrize("mesh", [MESH2, MESH3])
def test_transport_diagonals_match_the_assembled_matrices(oracle_lib, mesh):
    O, par = make(oracle_lib, mesh)
    rng = np.random.default_rng(2)
    rs = 1.0 + 0.1 * rng.random(O.nc)
    phi = flux(O, rng)
    for comp in range(O.ndim):
        M = dense(lambda e: O.momentum_operator(rs, phi, comp, e), O.nc)
        np.testing.assert_allclose(O.transport_diag(phi, comp, rho_star=rs), np.diag(M), rtol=1e-13)
    cT = 1e3 * (1.0 + rng.random(O.nc))
    M = dense(lambda e: O.energy_operator(cT, phi, e), O.nc)
    np.testing.assert_allclose(O.transport_diag(phi, -1, cT=cT), np.diag(M), rtol=1e-13)
    # the convective part makes the operators non-symmetric
    assert np.max(np.abs(M - M.T)) > 1e-3 * np.max(np.abs(M))


@pytest.mark.parametrize("mesh", [MESH2, MESH3])
def test_bicgstab_matches_a_dense_solve(oracle_lib, mesh):
    O, par = make(oracle_lib, mesh, mu=3.0)
    rng = np.random.default_rng(3)
    rs = 1.0 + 0.1 * rng.random(O.nc)
    phi = flux(O, rng, scale=200.0)       # strong transport: far from symmetric
    for comp in range(O.ndim):
        M = dense(lambda e: O.momentum_operator(rs, phi, comp, e), O.nc)
        b = rng.standard_normal(O.nc)
        x, st, rc = O.bicgstab_momentum(rs, phi, comp, b, np.zeros(O.nc), 1e-13)
        assert rc == 0 and st.converged and st.iters > 1
        assert np.linalg.norm(b - M @ x) <= 2e-13 * np.linalg.norm(b)
        np.testing.assert_allclose(x, np.linalg.solve(M, b), rtol=0, atol=1e-11 * np.abs(x).max())
    # zero right-hand side: x = 0 at once; an iteration cap of 1 does not converge
    x, st, rc = O.bicgstab_momentum(rs, phi, 0, np.zeros(O.nc), rng.standard_normal(O.nc), 1e-13)
    assert rc == 0 and st.iters == 0 and not np.any(x)
    x, st, rc = O.bicgstab_momentum(rs, phi, 0, rng.standard_normal(O.nc), np.zeros(O.nc), 1e-13,
                                    max_iter=1)
    assert rc != 0 and not st.converged


def test_implicit_predictor_is_the_explicit_one_without_transport(oracle_lib):
    """phi = 0 and mu = 0 leave only the time term: rho* u* = rho u - dt R(F)
    on both sides"""
    O, par = make(oracle_lib, MESH3, mu=0.0)
    rng = np.random.default_rng(4)
    rho = 1.0 + 0.05 * rng.random(O.nc)
    u = rng.standard_normal((3, O.nc))
    pp = 1e5 + 50.0 * rng.standard_normal(O.nc)
    rs = rho * (1.0 + 0.01 * rng.standard_normal(O.nc))
    phi = np.zeros((3, O.nc))
    us_e = O.momentum_predictor(rho, u, pp, rs, phi)
    us_i = O.momentum_predictor_implicit(rho, u, pp, rs, phi, u)
    np.testing.assert_allclose(us_i, us_e, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("mesh", [MESH2, MESH3])
def test_implicit_predictor_is_the_fixed_point_of_the_explicit_iteration(oracle_lib, mesh):
    """the implicit predictor solves rho* u V/dt + C(u) - Visc(u) = b, b the
    explicit predictor's right-hand side (V/dt rho* u*_e + C(u^n) - Visc(u^n)
    from the pinned explicit predictor); iterating u <- (b - C(u) + Visc(u))
    dt/(rho* V) with the pinned convective and viscous terms converges to it"""
    O, par = make(oracle_lib, mesh, mu=2.0)
    rng = np.random.default_rng(5)
    rho = 1.0 + 0.05 * rng.random(O.nc)
    u = 3.0 * rng.standard_normal((O.ndim, O.nc))
    pp = 1e5 + 50.0 * rng.standard_normal(O.nc)
    phi = flux(O, rng, scale=400.0)
    rs = O.density_predictor(rho, phi)
    V, dt, mu = volume(O), par["dt"], par["mu"]
    us_e = O.momentum_predictor(rho, u, pp, rs, phi)
    us_i = O.momentum_predictor_implicit(rho, u, pp, rs, phi, us_e)
    for c in range(O.ndim):
        b = rs * V / dt * us_e[c] + O.convective(phi, u[c]) - O.viscous(u[c], c, mu)
        x = u[c].copy()
        for _ in range(200):
            x = (b - O.convective(phi, x) + O.viscous(x, c, mu)) * dt / (rs * V)
        np.testing.assert_allclose(us_i[c], x, rtol=0, atol=1e-10 * np.abs(x).max())
        assert np.max(np.abs(us_i[c] - us_e[c])) > 1e-6 * np.abs(x).max()   # transport matters


@pytest.mark.parametrize("form", [0, 1])
def test_implicit_energy_is_the_limit_of_the_picard_sweeps(oracle_lib, form):
    """the implicit energy solve is the fixed point of the explicit sweeps
    (each sweep transports the previous sweep's T): with many sweeps the
    explicit form converges to it"""
    cfg = configs.get("bubble2d_64x32", tol=1e-13, energy_form=form)
    cfg["mesh"].update(nx=16, nz=12, ly=1250.0)
    cfg["params"]["dt"] = 4.0
    Oe = oracle_lib.Oracle(cfg["mesh"], dict(cfg["params"], transport=0, n_energy_sweeps=60))
    Oi = oracle_lib.Oracle(cfg["mesh"], dict(cfg["params"], transport=1))
    s = Oe.init_bubble(**dict(cfg["bubble"], xc=9000.0))
    Oe.step(s, 3)                                   # a moving state
    phi = s.phi
    rs = Oe.density_predictor(s.rho, phi)
    us = Oe.momentum_predictor(s.rho, s.u, s.pp, rs, phi)
    p_old, K_old = Oe._history(s)
    if form == 1:
        Te = Oe.energy_enthalpy(s.rho, s.T, s.p, p_old, K_old, us, rs, phi, s.Tbg)
    else:
        Te = Oe.energy(s.rho, s.u, s.T, us, rs, phi, s.Tbg)
    Ti = Oi.energy_implicit(s.rho, s.u, s.T, s.p, p_old, K_old, us, rs, phi, s.Tbg)
    dT = np.abs(Ti - s.T).max()
    assert dT > 1e-6
    np.testing.assert_allclose(Ti, Te, rtol=0, atol=1e-9 * dT + 1e-11)


def test_implicit_enthalpy_keeps_uniform_h(oracle_lib):
    """a uniform h stays uniform under a face flux consistent with Step 1's
    density change, now with the transport implicit"""
    O, par = make(oracle_lib, MESH3, mu=0.4, energy_form=1)
    rng = np.random.default_rng(6)
    rho = 1.1 + 0.05 * rng.standard_normal(O.nc)
    phi = flux(O, rng, scale=40.0)
    rs = O.density_predictor(rho, phi)
    T0 = 287.5
    T = np.full(O.nc, T0)
    p = 9e4 + 100.0 * rng.standard_normal(O.nc)
    zero3 = np.zeros((3, O.nc))
    Tn = O.energy_implicit(rho, zero3, T, p, p, np.zeros(O.nc), zero3, rs, phi,
                           np.full(O.mesh.nz, T0))
    np.testing.assert_allclose(Tn, T0, rtol=1e-13)


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("mesh3d", [False, True])
def test_implicit_transport_rest_state_stays_at_rest(oracle_lib, form, mesh3d):
    if mesh3d:
        cfg = configs.scaled("bubble3d_256x256x128", 8, 6, ny=7)
    else:
        cfg = configs.get("bubble2d_64x32")
    cfg["params"].update(tol=1e-14, energy_form=form, transport=1)
    O = oracle_lib.Oracle(cfg["mesh"], cfg["params"])
    s = O.init_bubble(0)
    s0 = s.copy()
    O.step(s, 10)
    assert np.max(np.abs(s.u)) <= 1e-10
    for f in ("rho", "T", "pp", "p"):
        a, b = getattr(s, f), getattr(s0, f)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b)), f


def test_implicit_transport_bubble_mass_symmetry_and_sign(oracle_lib):
    cfg = configs.scaled("bubble2d_64x32", 32, 16)
    cfg["params"].update(tol=1e-14, transport=1, dt=4.0)
    O = oracle_lib.Oracle(cfg["mesh"], cfg["params"])
    b = cfg["bubble"]
    s = O.init_bubble(**b)
    m0 = s.rho.sum()
    st = O.step(s, 8)
    x, y, z = O.cell_centres()
    r = np.hypot(x - b["xc"], z - b["zc"])
    assert s.u[-1][np.argmin(r)] > 0
    assert abs(s.rho.sum() - m0) <= 1e-13 * m0
    for x_ in st:
        assert all(x_.solve[q].converged for q in range(x_.n_solves))
    shape = (O.mesh.nz, O.mesh.nx)
    u = s.u[0].reshape(shape)
    assert np.max(np.abs(u + u[:, ::-1])) <= 1e-11 * np.max(np.abs(u))
    for f in (s.rho, s.T, s.pp, s.u[-1]):
        f = f.reshape(shape)
        assert np.max(np.abs(f - f[:, ::-1])) <= 1e-11 * np.max(np.abs(f))


@pytest.mark.parametrize("form", [0, 1])
def test_implicit_step_is_the_composition_of_the_pinned_substeps(oracle_lib, form):
    cfg = configs.get("bubble2d_64x32", tol=1e-13, energy_form=form, transport=1)
    cfg["mesh"].update(nx=16, nz=12, ly=1250.0)
    O = oracle_lib.Oracle(cfg["mesh"], cfg["params"])
    s = O.init_bubble(**dict(cfg["bubble"], xc=9000.0))
    O.step(s, 2)
    want = s.copy()
    O.step(want, 1)
    phi = s.phi
    rs = O.density_predictor(s.rho, phi)
    us = O.momentum_predictor(s.rho, s.u, s.pp, rs, phi)
    us = O.momentum_predictor_implicit(s.rho, s.u, s.pp, rs, phi, us)
    Tn = O.energy_implicit(s.rho, s.u, s.T, s.p, s.p_old, s.K_old, us, rs, phi, s.Tbg)
    r23, psi, c, D = O.eos_coeffs(s.p, Tn, rs)
    uk, ppk = us, s.pp.copy()
    for k in range(cfg["params"]["n_corr"]):
        H = O.H(s.rho, s.u, uk, phi)
        pt, b = O.predicted_flux_rhs(s.rho, r23, psi, D, H)
        ppk, st, rc = O.pcg(c, D, b, ppk, cfg["params"]["tol"])
        assert rc == 0
        phik, uk = O.correct(ppk, r23, H, D, rs, pt)
    rn, pn, mm = O.finalize(s.rho, phik, ppk, r23, psi)
    for got, ref in ((rn, want.rho), (uk, want.u), (Tn, want.T), (ppk, want.pp), (pn, want.p),
                     (phik, want.phi)):
        np.testing.assert_array_equal(got, ref)
