"""Pins of the oracle's immersed-boundary part against closed forms and
invariants (no GPU).  Each test targets a mistake a plausible slip in the
oracle would make: a wrong kernel branch, a wrong staggering offset, a
dropped wall rule, a transposed spread, a wrong marker volume or a wrong sign
in the force/torque sums."""
import math

import numpy as np
import pytest

RNG = np.random.default_rng(12345)


def params(orc, nx=16, ny=12, nz=16, h=0.1, nl=314, **kw):
    return orc.make_params(nx=nx, ny=ny, nz=nz, h=h, nl=nl, **kw)


def node_coords(p, comp):
    """Physical coordinates of the stored nodes of one staggered component."""
    o = [0.5, 0.5, 0.5]
    o[comp] = 0.0
    nyc = p.ny + 1 if comp == 1 else p.ny
    k, j, i = np.meshgrid(np.arange(p.nz), np.arange(nyc), np.arange(p.nx), indexing="ij")
    return (i + o[0]) * p.h, (j + o[1]) * p.h, (k + o[2]) * p.h


# ---------------------------------------------------------------- kernel ---
def test_phi_special_values(orc):
    assert orc.phi(0.0) == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert orc.phi(0.5) == pytest.approx(0.5, abs=1e-15)
    assert orc.phi(-0.5) == pytest.approx(0.5, abs=1e-15)
    assert orc.phi(1.0) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert orc.phi(1.5) == pytest.approx(0.0, abs=1e-15)
    assert orc.phi(-1.5) == pytest.approx(0.0, abs=1e-15)
    assert orc.phi(1.6) == 0.0 and orc.phi(-7.0) == 0.0


def test_phi_moment_conditions(orc):
    """Three-point kernel: partition of unity, zero first moment and
    sum of squares 1/2 for every shift (closed-form identities)."""
    for r in RNG.uniform(-3, 3, 4000):
        j = np.arange(math.floor(r) - 3, math.floor(r) + 4)
        w = np.array([orc.phi(r - jj) for jj in j])
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs(((r - j) * w).sum()) < 1e-14
        assert abs((w * w).sum() - 0.5) < 1e-14


def test_phi_is_continuous_and_even(orc):
    for r in (0.5, 1.5):
        for eps in (1e-9, 1e-12):
            assert abs(orc.phi(r - eps) - orc.phi(r + eps)) < 1e-6
    for r in RNG.uniform(0, 2, 100):
        assert orc.phi(r) == orc.phi(-r)


# -------------------------------------------------------------- template ---
@pytest.mark.parametrize("nl,R,h", [(314, 0.5, 0.1), (804, 0.5, 1 / 16), (315, 0.5, 0.1), (7, 1.0, 0.3)])
def test_template_geometry(orc, nl, R, h):
    t, dV = orc.template(nl, R, h)
    assert t.shape == (nl, 3)
    assert np.allclose(np.linalg.norm(t, axis=1), 1.0, atol=1e-14)
    assert abs(t[:, 1].sum()) < 1e-12                    # symmetric pole coordinate
    # marker volume: a shell of thickness h around the sphere, shared equally
    shell = 4.0 / 3.0 * math.pi * ((R + h / 2) ** 3 - (R - h / 2) ** 3)
    assert dV * nl == pytest.approx(shell, rel=1e-13)
    # points spread over the sphere: centroid near the centre
    assert np.linalg.norm(t.mean(axis=0)) < 2.0 / math.sqrt(nl)


def test_template_values_at_paper_resolution(orc):
    t, dV = orc.template(314, 0.5, 0.1)
    assert dV / 0.1 ** 3 == pytest.approx(1.00384, abs=5e-6)
    t, dV = orc.template(804, 0.5, 1.0 / 16)
    assert dV * 16 ** 3 == pytest.approx(1.00161, abs=5e-6)


# ---------------------------------------------------------- interpolation ---
def test_linear_fields_interpolate_exactly(orc):
    """PoU + first moment => any affine field is reproduced exactly at markers
    at least 1.5 h from the walls, for each staggered component with its own
    node offsets (a wrong offset gives an error of B . offset)."""
    p = params(orc, nx=24, ny=20, nz=24, nl=64)
    a = RNG.normal(size=3)
    B = RNG.normal(size=(3, 3))
    grids = []
    for c in range(3):
        X, Y, Z = node_coords(p, c)
        grids.append(np.ascontiguousarray(a[c] + B[c, 0] * X + B[c, 1] * Y + B[c, 2] * Z))
    n = 6
    x = np.stack([RNG.uniform(0.7, 1.7, n), RNG.uniform(0.72, 1.28, n), RNG.uniform(0.7, 1.7, n)], 1)
    U, Ud = orc.interpolate(p, grids, x, np.zeros((n, 3)), np.zeros((n, 3)))
    t, _ = orc.template(p.nl, p.R, p.h)
    X = x[:, None, :] + p.R * t[None]
    expect = a[None, None, :] + np.einsum("ca,pla->plc", B, X)
    assert np.abs(U - expect).max() < 1e-12


def test_desired_velocity_is_rigid_motion(orc):
    p = params(orc, nl=50)
    x = np.array([[0.8, 0.6, 0.8]])
    up = np.array([[0.1, -0.2, 0.3]])
    om = np.array([[1.0, 2.0, -0.5]])
    g = [np.zeros(s) for s in orc.grid_shapes(p)]
    _, Ud = orc.interpolate(p, g, x, up, om)
    t, _ = orc.template(p.nl, p.R, p.h)
    assert np.allclose(Ud[0], up[0] + np.cross(om[0], p.R * t), atol=1e-15)


def test_interpolation_wraps_periodic_seams(orc):
    """A field periodic in x and z: a sphere straddling the seam sees the same
    values as the same sphere shifted by one period."""
    p = params(orc, nx=20, ny=14, nz=20, nl=100)
    grids = []
    for c in range(3):
        X, Y, Z = node_coords(p, c)
        Lx, Lz = p.nx * p.h, p.nz * p.h
        grids.append(np.ascontiguousarray(np.sin(2 * np.pi * X / Lx) * np.cos(2 * np.pi * Z / Lz) + Y))
    x1 = np.array([[0.05, 0.7, 1.98]])
    x2 = x1 + [[2.0, 0.0, -2.0]]  # one period in x and in z
    z = np.zeros((1, 3))
    U1, _ = orc.interpolate(p, grids, x1, z, z)
    U2, _ = orc.interpolate(p, grids, x2 - [[0, 0, 0]], z, z)
    assert np.abs(U1 - U2).max() < 1e-12


# ------------------------------------------------------------- spreading ---
def test_spread_conserves_force_and_moment(orc):
    p = params(orc, nx=24, ny=20, nz=24, nl=120)
    n = 3
    x = np.stack([RNG.uniform(0.8, 1.6, n), RNG.uniform(0.8, 1.2, n), RNG.uniform(0.8, 1.6, n)], 1)
    F = RNG.normal(size=(n, p.nl, 3))
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    orc.spread(p, x, F, f)
    t, dV = orc.template(p.nl, p.R, p.h)
    Xm = x[:, None, :] + p.R * t[None]
    h3 = p.h ** 3
    total = np.array([f[c].sum() * h3 for c in range(3)])
    assert np.allclose(total, dV * F.sum(axis=(0, 1)), rtol=1e-12, atol=1e-12)
    # first moment (angular momentum) of the spread force equals that of the markers
    coords = [node_coords(p, c) for c in range(3)]
    mom_grid = np.zeros(3)
    for c in range(3):
        pos = coords[c]
        e = np.zeros(3)
        e[c] = 1.0
        for a in range(3):
            # (x_n x f_n)_a = eps_abc x_b f_c
            for b in range(3):
                eps = np.linalg.det(np.array([np.eye(3)[a], np.eye(3)[b], e]))
                if eps != 0:
                    mom_grid[a] += eps * (pos[b] * f[c]).sum() * h3
    mom_mark = dV * np.cross(Xm, F).sum(axis=(0, 1))
    assert np.allclose(mom_grid, mom_mark, rtol=1e-11, atol=1e-11)


def test_spread_is_adjoint_of_interpolation(orc):
    """<I[u], F> dV = <u, S[F]> h^3 for random u and F, with spheres touching
    the walls and straddling the periodic seams (wall-dropped nodes included)."""
    p = params(orc, nx=20, ny=14, nz=18, nl=200)
    x = np.array([[0.03, 0.45, 0.9], [1.0, 0.52, 1.79], [1.5, 0.9, 0.01], [1.96, 1.0, 1.0]])
    u = [RNG.normal(size=s) for s in orc.grid_shapes(p)]
    F = RNG.normal(size=(len(x), p.nl, 3))
    U, _ = orc.interpolate(p, u, x, np.zeros_like(x), np.zeros_like(x))
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    orc.spread(p, x, F, f)
    _, dV = orc.template(p.nl, p.R, p.h)
    lhs = (U * F).sum() * dV
    rhs = sum((u[c] * f[c]).sum() for c in range(3)) * p.h ** 3
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_wall_rule_drops_wall_faces(orc):
    """Wall-normal faces on the walls never receive spread force."""
    p = params(orc, nx=16, ny=10, nz=16, nl=200)
    x = np.array([[0.8, 0.5, 0.8], [0.8, 0.5, 0.8]])
    x[1, 1] = p.ny * p.h - 0.5
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    orc.spread(p, x, RNG.normal(size=(2, p.nl, 3)), f)
    assert np.all(f[1][:, 0, :] == 0.0) and np.all(f[1][:, p.ny, :] == 0.0)
    assert np.abs(f[1][:, 1, :]).max() > 0.0


def test_window_matches_full_grid_for_interior_particles(orc):
    """The windowed form (used for large-domain checks) gives the full-grid
    result for particles whose dependency cone lies inside the window."""
    full = params(orc, nx=40, ny=12, nz=36, nl=100, n_iter=2)
    u = [RNG.normal(size=s) for s in orc.grid_shapes(full)]
    x = np.array([[2.0, 0.6, 1.8], [2.4, 0.55, 2.1], [0.2, 0.6, 0.3]])
    up = RNG.normal(size=x.shape)
    om = RNG.normal(size=x.shape)
    f = [np.zeros(s) for s in orc.grid_shapes(full)]
    ref = orc.ib_forcing(full, u, f, x, up, om)
    win = params(orc, nx=40, ny=12, nz=36, nl=100, n_iter=2, wi0=10, wnx=24, wk0=8, wnz=20)
    sub = [np.ascontiguousarray(np.roll(np.roll(a, -10, axis=2), -8, axis=0)[:20, :, :24]) for a in u]
    fw = [np.zeros(s) for s in orc.grid_shapes(win)]
    got = orc.ib_forcing(win, sub, fw, x[:2], up[:2], om[:2])
    assert np.abs(got["Fh"] - ref["Fh"][:2]).max() < 1e-12 * np.abs(ref["Fh"]).max()
    assert np.abs(got["Th"] - ref["Th"][:2]).max() < 1e-12 * np.abs(ref["Th"]).max()


# ------------------------------------------------------------------- MDF ---
def test_single_marker_residual_ratio(orc):
    """One marker: each iteration multiplies the slip by 1 - dV/(8 h^3)
    (sum of squared weights is 1/2 per axis), at any position."""
    h = 0.1
    p = params(orc, nx=20, ny=20, nz=20, h=h, nl=1, R=0.01, n_iter=5)
    _, dV = orc.template(1, p.R, h)
    ratio = 1.0 - dV / (8 * h ** 3)
    for _ in range(4):
        x = np.array([[RNG.uniform(0.6, 1.4), RNG.uniform(0.6, 1.4), RNG.uniform(0.6, 1.4)]])
        u = [RNG.normal(size=s) for s in orc.grid_shapes(p)]
        f = [np.zeros(s) for s in orc.grid_shapes(p)]
        out = orc.ib_forcing(p, u, f, x, RNG.normal(size=(1, 3)), np.zeros((1, 3)))
        s = out["slip"]
        assert s[0] == pytest.approx(1.0, abs=1e-14)
        assert np.allclose(s[1:] / s[:-1], ratio, rtol=1e-10)


def test_rigid_motion_needs_no_force(orc):
    """Uniform flow with u_p = U, and rigid rotation with omega_p = Omega:
    the markers already move with the fluid, so the forcing is zero."""
    p = params(orc, nx=24, ny=20, nz=24, nl=150, n_iter=3)
    x = np.array([[1.2, 1.0, 1.1]])
    U = np.array([0.3, -0.2, 0.5])
    Om = np.array([0.7, -1.1, 0.4])
    grids = []
    for c in range(3):
        X, Y, Z = node_coords(p, c)
        rel = np.stack([X - x[0, 0], Y - x[0, 1], Z - x[0, 2]], -1)
        grids.append(np.ascontiguousarray(U[c] + np.cross(Om, rel)[..., c]))
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    out = orc.ib_forcing(p, grids, f, x, U[None], Om[None], want_marker_force=True)
    assert np.abs(out["Fmark"]).max() < 1e-9
    assert np.abs(out["Fh"]).max() < 1e-10 and np.abs(out["Th"]).max() < 1e-10


def test_first_iteration_force_of_sphere_in_still_fluid(orc):
    """Still fluid, sphere moving with U: after one iteration every marker
    force is U/(alpha dt), so F_h = -rho_f dV N_L U/(alpha dt) (antiparallel
    to U) and T_h = 0 by the template's symmetry up to its centroid."""
    p = params(orc, nx=24, ny=20, nz=24, nl=314, n_iter=1, rho_f=1.3, alpha=0.5)
    x = np.array([[1.2, 1.0, 1.1]])
    U = np.array([[0.3, -0.2, 0.5]])
    g = [np.zeros(s) for s in orc.grid_shapes(p)]
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    out = orc.ib_forcing(p, g, f, x, U, np.zeros((1, 3)))
    t, dV = orc.template(p.nl, p.R, p.h)
    adt = p.alpha * p.dt_f
    assert np.allclose(out["Fh"][0], -p.rho_f * dV * p.nl * U[0] / adt, rtol=1e-12)
    expect_T = -p.rho_f * dV * np.cross(p.R * t.sum(0), U[0] / adt)
    assert np.allclose(out["Th"][0], expect_T, atol=1e-9 * np.abs(out["Fh"]).max())


def test_step_feeds_its_forcing_to_the_particle_motion(orc):
    """The whole step for one free sphere (no contacts), in closed form: the
    forcing of a sphere moving with U through still fluid (one iteration,
    F_h = -rho_f dV N_L U/(alpha dt)), then n_sub symplectic Euler substeps
    of eqs. 7-8 with F_h, T_h and the buoyant weight held fixed:
    u = U + n dt a, x = x0 + n dt U + dt^2 a n(n+1)/2, omega = n dt T_h/I,
    a = (F_h + (rho_p - rho_f) V g)/m_p, dt = dt_f/n.  A dropped buoyancy,
    a flipped F_h or an unused T_h fails it."""
    p = params(orc, nx=24, ny=20, nz=24, nl=314, n_iter=1, rho_f=1.3, rho_p=2.1, alpha=0.5,
               n_sub=7)
    x0 = np.array([[1.2, 1.0, 1.1]])
    U = np.array([[0.3, -0.2, 0.5]])
    x, u, om = x0.copy(), U.copy(), np.zeros((1, 3))
    g = [np.zeros(s) for s in orc.grid_shapes(p)]
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    rc, out = orc.step(p, g, f, x, u, om, orc.History(1))
    assert rc == 0
    t, dV = orc.template(p.nl, p.R, p.h)
    Fh, Th = out["Fh"][0], out["Th"][0]
    assert np.allclose(Fh, -p.rho_f * dV * p.nl * U[0] / (p.alpha * p.dt_f), rtol=1e-12)
    V = 4.0 / 3.0 * math.pi * p.R ** 3
    m = p.rho_p * V
    I = 0.4 * m * p.R ** 2
    a = (Fh + (p.rho_p - p.rho_f) * V * np.array(p.g[:])) / m
    n, dt = p.n_sub, p.dt_f / p.n_sub
    assert np.allclose(u[0], U[0] + n * dt * a, rtol=0, atol=1e-12 * np.abs(u).max())
    assert np.allclose(x[0], x0[0] + n * dt * U[0] + dt * dt * a * n * (n + 1) / 2, rtol=0,
                       atol=1e-13)
    assert np.allclose(om[0], n * dt * Th / I, rtol=1e-12, atol=1e-300)
    assert np.abs(om[0]).max() > 0       # the template's centroid offset gives a torque


def test_step_with_a_contact_balances_momentum(orc):
    """Two touching spheres (normal and tangential contact forces) through a
    whole step: the contact forces cancel in pairs, so over the step the
    pair's momentum changes by exactly (sum F_h + 2 (rho_p - rho_f) V g) dt_f,
    with F_h the step's own forcing result."""
    p = params(orc, nx=32, ny=24, nz=24, nl=314, n_iter=2, rho_f=1.0, rho_p=2.5, n_sub=9)
    x = np.array([[1.0, 1.2, 1.2], [1.99, 1.2, 1.2]])
    u = np.array([[0.2, 0.05, 0.0], [-0.1, 0.0, 0.03]])
    om = np.array([[0.0, 0.0, 0.4], [0.1, 0.0, 0.0]])
    u0 = u.copy()
    g = [np.zeros(s) for s in orc.grid_shapes(p)]
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    H = orc.History(2)
    rc, out = orc.step(p, g, f, x, u, om, H)
    assert rc == 0 and H.cnt.tolist() == [1, 1]          # the pair stayed in contact
    V = 4.0 / 3.0 * math.pi * p.R ** 3
    m = p.rho_p * V
    dP = m * (u - u0).sum(axis=0)
    expect = (out["Fh"].sum(axis=0) + 2 * (p.rho_p - p.rho_f) * V * np.array(p.g[:])) * p.dt_f
    assert np.abs(dP - expect).max() < 1e-12 * np.abs(m * u0).max()
    # the contact did act: the spheres' relative velocity differs from what
    # the hydrodynamic forces alone give
    free = u0 + (out["Fh"] / m + (1 - p.rho_f / p.rho_p) * np.array(p.g[:])) * p.dt_f
    assert np.abs((u - free)[0] - (u - free)[1]).max() > 1e-3


def test_force_field_sums_to_minus_particle_force(orc):
    """Momentum balance: the force given to the fluid equals minus the force
    on the particles, rho_f sum_n f_n h^3 = -sum_p F_h (interior spheres)."""
    p = params(orc, nx=30, ny=20, nz=30, nl=200, n_iter=3)
    x = np.array([[1.0, 1.0, 1.0], [1.9, 1.05, 1.4]])
    u = [RNG.normal(size=s) * 0.1 for s in orc.grid_shapes(p)]
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    out = orc.ib_forcing(p, u, f, x, RNG.normal(size=(2, 3)), RNG.normal(size=(2, 3)))
    mom = np.array([f[c].sum() for c in range(3)]) * p.h ** 3 * p.rho_f
    assert np.allclose(mom, -out["Fh"].sum(0), rtol=1e-11)


def test_ustar_is_uhat_plus_alpha_dt_f(orc):
    """Eq. 4: the intermediate velocity is u-hat plus alpha dt_f times the force."""
    p = params(orc, nx=20, ny=14, nz=20, nl=100, n_iter=2, alpha=0.5)
    u = [RNG.normal(size=s) for s in orc.grid_shapes(p)]
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    x = np.array([[1.0, 0.7, 1.0]])
    out = orc.ib_forcing(p, u, f, x, RNG.normal(size=(1, 3)), np.zeros((1, 3)), want_ustar=True)
    adt = p.alpha * p.dt_f
    for c in range(3):
        assert np.abs(out["ustar"][c] - (u[c] + adt * f[c])).max() < 1e-12


def test_tolerance_mode_stops_on_slip(orc):
    p = params(orc, nx=20, ny=20, nz=20, nl=100, tol_mode=1, tol=0.05, max_iter=30)
    u = [np.zeros(s) for s in orc.grid_shapes(p)]
    f = [np.zeros(s) for s in orc.grid_shapes(p)]
    out = orc.ib_forcing(p, u, f, np.array([[1.0, 1.0, 1.0]]), np.array([[0.1, 0.0, 0.0]]),
                         np.zeros((1, 3)))
    s = out["slip"]
    assert s[-1] < 0.05 and np.all(s[:-1] >= 0.05)
    assert len(s) == out["iters"] + 1
    assert np.all(np.diff(s) < 0)


def test_initial_marker_force_is_spread_first(orc):
    """Starting from a marker force F0 equals starting from F0's spread field:
    u** = u-hat + alpha dt S[F0] (the field form of a warm start)."""
    p = params(orc, nx=20, ny=14, nz=20, nl=80, n_iter=2)
    u = [RNG.normal(size=s) for s in orc.grid_shapes(p)]
    x = np.array([[1.0, 0.7, 1.0]])
    up = RNG.normal(size=(1, 3))
    F0 = RNG.normal(size=(1, p.nl, 3))
    f1 = [np.zeros(s) for s in orc.grid_shapes(p)]
    a = orc.ib_forcing(p, u, f1, x, up, np.zeros((1, 3)), F0=F0)
    f2 = [np.zeros(s) for s in orc.grid_shapes(p)]
    orc.spread(p, x, F0, f2)
    f2c = [c.copy() for c in f2]
    b = orc.ib_forcing(p, u, f2c, x, up, np.zeros((1, 3)))
    _, dV = orc.template(p.nl, p.R, p.h)
    extra = -p.rho_f * dV * F0.sum(axis=(0, 1))
    assert np.allclose(a["Fh"][0], b["Fh"][0] + extra, rtol=1e-10, atol=1e-10)
    for c in range(3):
        assert np.abs(f1[c] - f2c[c]).max() < 1e-10 * max(1.0, np.abs(f1[c]).max())
