"""Pins of the oracle's discrete operators against closed forms.

Sec. 3 (last paragraph) fixes second-order gradient and Laplacian and a
fourth-order divergence.  These tests check each operator on polynomials for
which the discrete form is exact, and the wall treatment of Sec. 4
(impenetrable, free-slip) on the cells next to the walls.
"""
import numpy as np
import pytest

MESH2 = dict(nx=12, ny=1, nz=10, lx=1200.0, ly=100.0, lz=1000.0)
MESH3 = dict(nx=8, ny=6, nz=7, lx=800.0, ly=900.0, lz=350.0)
PAR = dict(R=287.0, cp=1004.0, cv=717.0, g=9.81, p0=1e5, theta0=300.0, mu=0.15, Pr=1.0,
           dt=1.0)


@pytest.fixture(params=["2d", "3d"])
def O(request, oracle_lib):
    mesh = MESH2 if request.param == "2d" else MESH3
    return oracle_lib.Oracle(mesh, PAR)


def axes(O):
    """cell-centre coordinate, index and spacing along each direction"""
    x, y, z = O.cell_centres()
    m = O.mesh
    nx, ny, nz = m.nx, m.ny, m.nz
    P = np.arange(O.nc)
    i, j, k = P % nx, (P // nx) % ny, P // (nx * ny)
    h = (m.lx / nx, m.ly / ny, m.lz / nz)
    if O.ndim == 2:
        return [(x, i, nx, h[0]), (z, k, nz, h[2])]
    return [(x, i, nx, h[0]), (y, j, ny, h[1]), (z, k, nz, h[2])]


def test_interp4_exact_on_cubics_and_linear_next_to_walls(O):
    rng = np.random.default_rng(1)
    for d, (X, idx, n, h) in enumerate(axes(O)):
        a = rng.normal(size=4)
        f = lambda t: a[0] + a[1] * t / 100 + a[2] * (t / 100) ** 2 + a[3] * (t / 100) ** 3
        out = O.face_interp4(f(X), d)
        xf = X + 0.5 * h
        inner = (idx >= 1) & (idx <= n - 3)
        np.testing.assert_allclose(out[inner], f(xf[inner]), rtol=1e-12, atol=1e-12)
        # next to a wall: the mean of the two cells
        edge = (idx == 0) | (idx == n - 2)
        Pe = np.nonzero(edge)[0]
        st = [1, O.mesh.nx, O.mesh.nx * O.mesh.ny][[0, 2][d] if O.ndim == 2 else d]
        s = f(X)
        np.testing.assert_allclose(out[Pe], 0.5 * (s[Pe] + s[Pe + st]), rtol=1e-14)
        # exact for linear fields there too
        lin = 3.0 + 0.25 * X
        np.testing.assert_allclose(O.face_interp4(lin, d)[edge], (3.0 + 0.25 * xf)[edge], rtol=1e-13)
        # the wall face carries nothing
        assert np.all(out[idx == n - 1] == 0.0)


def test_sngrad_exact_on_quadratics(O):
    for d, (X, idx, n, h) in enumerate(axes(O)):
        f = 2.0 - 0.3 * X + 1e-3 * X ** 2
        out = O.face_sngrad(f, d)
        xf = X + 0.5 * h
        inner = idx <= n - 2
        np.testing.assert_allclose(out[inner], (-0.3 + 2e-3 * xf)[inner], rtol=1e-10, atol=1e-12)
        assert np.all(out[idx == n - 1] == 0.0)


def test_reconstruct_exact_on_linear_faces_and_halves_at_walls(O):
    ax = axes(O)
    faces = np.zeros((O.ndim, O.nc))
    for d, (X, idx, n, h) in enumerate(ax):
        xf = X + 0.5 * h
        faces[d] = np.where(idx <= n - 2, 5.0 + 0.01 * (d + 1) * xf, 0.0)
    out = O.reconstruct(faces)
    for d, (X, idx, n, h) in enumerate(ax):
        inner = (idx >= 1) & (idx <= n - 2)
        np.testing.assert_allclose(out[d][inner], (5.0 + 0.01 * (d + 1) * X)[inner], rtol=1e-13)
        # a wall face counts as zero: half of the one interior face
        lo = idx == 0
        np.testing.assert_allclose(out[d][lo], 0.5 * (5.0 + 0.01 * (d + 1) * (X + 0.5 * h))[lo], rtol=1e-13)
        hi = idx == n - 1
        np.testing.assert_allclose(out[d][hi], 0.5 * (5.0 + 0.01 * (d + 1) * (X - 0.5 * h))[hi], rtol=1e-13)


def test_divergence_exact_on_quadratic_fluxes(O):
    ax = axes(O)
    m = O.mesh
    V = (m.lx / m.nx) * (m.ly / m.ny) * (m.lz / m.nz)
    faces = np.zeros((O.ndim, O.nc))
    want = np.zeros(O.nc)
    S = []
    for d, (X, idx, n, h) in enumerate(ax):
        S.append(V / h)
    for d, (X, idx, n, h) in enumerate(ax):
        f = lambda t: 1.0 + 0.02 * t - 3e-5 * t * t
        fp = lambda t: 0.02 - 6e-5 * t
        xf = X + 0.5 * h
        faces[d] = np.where(idx <= n - 2, f(xf) * S[d], 0.0)
        inner = (idx >= 1) & (idx <= n - 2)
        want += np.where(inner, fp(X), 0.0)
    out = O.divergence(faces)
    inner_all = np.ones(O.nc, bool)
    for d, (X, idx, n, h) in enumerate(ax):
        inner_all &= (idx >= 1) & (idx <= n - 2)
    np.testing.assert_allclose(out[inner_all], want[inner_all], rtol=1e-9, atol=1e-13)
    # telescoping: the sum over all cells of V * div is exactly the boundary flux (= 0 here)
    assert abs(np.sum(out * V)) < 1e-9 * np.abs(faces).sum()


def test_viscous_is_laplacian_inside_and_wall_dirichlet_for_normal_component(O):
    m = O.mesh
    V = (m.lx / m.nx) * (m.ly / m.ny) * (m.lz / m.nz)
    mu = 0.7
    ax = axes(O)
    coef = [1e-3, -2e-3, 5e-4][:O.ndim]
    u = 4.0 + sum(cf * X ** 2 for cf, (X, *_r) in zip(coef, ax))
    lap = 2.0 * sum(coef)
    inner = np.ones(O.nc, bool)
    for X, idx, n, h in ax:
        inner &= (idx >= 1) & (idx <= n - 2)
    for comp in range(O.ndim):
        out = O.viscous(u, comp, mu)
        np.testing.assert_allclose(out[inner], mu * V * lap, rtol=1e-9)
    # wall cells: the component normal to a wall sees u = 0 at the wall (distance h/2);
    # a tangential component sees no shear.  A uniform field isolates the wall terms.
    one = np.ones(O.nc)
    for comp, (X, idx, n, h) in enumerate(ax):
        out = O.viscous(one, comp, mu)
        S = V / h
        nwalls = (idx == 0).astype(float) + (idx == n - 1).astype(float)
        np.testing.assert_allclose(out, -2.0 * mu * S / h * nwalls, rtol=1e-13, atol=1e-14)


def test_convective_exact_for_uniform_flux(O):
    # constant face flux phi through every interior face of direction d and a
    # linear field s: sum_out phi I4(s) = phi (s(x+h/2) - s(x-h/2)) inside
    for d, (X, idx, n, h) in enumerate(axes(O)):
        phi = np.zeros((O.ndim, O.nc))
        phi[d] = np.where(idx <= n - 2, 2.5, 0.0)
        s = 1.0 + 0.1 * X
        out = O.convective(phi, s)
        inner = (idx >= 1) & (idx <= n - 2)
        np.testing.assert_allclose(out[inner], 2.5 * 0.1 * h, rtol=1e-12)
        # the wall cell only has its interior face: outflow at the low wall cell
        lo = idx == 0
        np.testing.assert_allclose(out[lo], (2.5 * (1.0 + 0.1 * (X + 0.5 * h)))[lo], rtol=1e-13)


def test_potential_is_g_times_height(O):
    x, y, z = O.cell_centres()
    np.testing.assert_allclose(O.potential(), 9.81 * z, rtol=1e-15)
