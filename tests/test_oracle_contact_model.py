"""Pins of the oracle's collision-time calibrated contact coefficients
(contact_model = 1, a reading of sec. 2.1 and 4.1 for the linear
spring-dashpot), no GPU.  The paper's sand parameters: e_n = 0.97,
e_t = 0.39, mu_c = 0.15, T_c = 10 dt_f.  Closed forms of a damped
oscillator fix what the calibration must give, whatever the mass:
- a head-on sphere-sphere collision and a sphere-wall collision last T_c and
  return e_n times the approach speed (to the substep's O(dt) error, which
  shrinks as the substep does);
- a contact that sticks throughout returns its tangential contact-point
  velocity with restitution e_t;
- a contact that slides throughout changes the tangential velocity by
  mu J+ / m (J+ the compressive normal impulse) and the spin by 5/2 of it."""
import math

import numpy as np
import pytest

DTF = 8.27944e-4
TC = 10 * DTF


def params(orc, n_sub, **kw):
    kw.setdefault("g", (0.0, 0.0, 0.0))
    kw.setdefault("mu", 0.15)
    return orc.make_params(nx=80, ny=100, nz=80, h=0.1, nl=10, dt_f=DTF / 20, n_sub=n_sub,
                           contact_model=1, t_c=TC, e_n=0.97, e_t=0.39, **kw)


def run_until_apart(orc, p, x, u, om, cap=200000):
    H = orc.History(len(x))
    Z = np.zeros_like(x)
    steps, touched = 0, False
    while steps < cap:
        orc.dem(p, x, u, om, Z, Z, H)
        steps += 1
        if H.cnt.sum() > 0:
            touched = True
        elif touched:
            break
    return steps


@pytest.mark.parametrize("n_sub,tol", [(1, 0.004), (4, 0.001)])
def test_pair_collision_lasts_tc_with_restitution_en(orc, n_sub, tol):
    p = params(orc, n_sub)
    dtp = p.dt_f / n_sub
    x = np.array([[3.0, 5.0, 4.0], [3.0 + 2 * p.R - 1e-9, 5.0, 4.0]])
    u = np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
    om = np.zeros((2, 3))
    steps = run_until_apart(orc, p, x, u, om)
    e = (u[1, 0] - u[0, 0]) / 1.0
    assert e == pytest.approx(0.97, abs=tol)
    # contact substeps (the last call, with no contact left, excluded)
    assert (steps - 1) * dtp * n_sub == pytest.approx(TC, rel=0.01)
    assert np.allclose(u[0] + u[1], 0.0, atol=1e-12)


@pytest.mark.parametrize("n_sub,tol", [(1, 0.004), (4, 0.001)])
def test_wall_collision_lasts_tc_with_restitution_en(orc, n_sub, tol):
    p = params(orc, n_sub)
    dtp = p.dt_f / n_sub
    x = np.array([[3.0, p.R - 1e-9, 4.0]])
    u = np.array([[0.0, -1.0, 0.0]])
    om = np.zeros((1, 3))
    steps = run_until_apart(orc, p, x, u, om)
    assert u[0, 1] == pytest.approx(0.97, abs=tol)
    assert (steps - 1) * dtp * n_sub == pytest.approx(TC, rel=0.01)


def sticking_limit(m, v_n, v_t):
    """Continuous-time tangential restitution of a sphere-wall contact that
    sticks (no friction limit while the normal force pushes): the normal and
    tangential oscillators with the calibrated coefficients, integrated by
    classical Runge-Kutta on a fine step until the normal force vanishes;
    after that the friction limit mu max(0, f_n) is zero, the tangential
    force too, and the contact-point velocity keeps its value."""
    le, lt = math.log(0.97), math.log(0.39)
    mt = 2.0 / 7.0 * m
    d, k = -2 * m * le / TC, m * (math.pi ** 2 + le * le) / TC ** 2
    dt_, kt = -2 * mt * lt / TC, mt * (math.pi ** 2 + lt * lt) / TC ** 2

    def f(y):
        xi, w, de, s = y
        return np.array([w, -(k * xi + d * w) / m, s, -(kt * de + dt_ * s) / mt])

    y = np.array([0.0, v_n, 0.0, v_t])
    h = TC / 20000
    while True:
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if k * y[0] + d * y[1] <= 0.0:
            return -y[3] / v_t


@pytest.mark.parametrize("n_sub,tol", [(4, 2e-3), (64, 2e-4)])
def test_sticking_contact_restitution_et(orc, n_sub, tol):
    """Without the friction limit the contact-point velocity would return
    with restitution e_t exactly; the limit mu max(0, f_n) releases it in the
    short tensile tail of the normal force, which the continuous-time
    reference includes (it lies within 1.5 % of e_t)."""
    p = params(orc, n_sub, mu=1e12)
    m = p.rho_p * 4.0 / 3.0 * math.pi * p.R ** 3
    ref = sticking_limit(m, 1.0, 0.3)
    assert ref == pytest.approx(0.39, rel=0.015)
    x = np.array([[3.0, p.R - 1e-12, 4.0]])
    u = np.array([[0.3, -1.0, 0.0]])
    om = np.zeros((1, 3))
    run_until_apart(orc, p, x, u, om)
    vcp = u[0, 0] + p.R * om[0, 2]      # x-part of u + R omega x n, n = -y
    assert -vcp / 0.3 == pytest.approx(ref, abs=tol)


def test_sliding_contact_impulse(orc):
    p = params(orc, 1)
    m = p.rho_p * 4.0 / 3.0 * math.pi * p.R ** 3
    x = np.array([[3.0, p.R - 1e-9, 4.0]])
    u = np.array([[5.0, -1.0, 0.0]])
    om = np.zeros((1, 3))
    run_until_apart(orc, p, x, u, om)
    # compressive normal impulse of the same discrete normal motion, by an
    # independent recurrence with the closed-form calibrated coefficients
    le = math.log(0.97)
    d = -2 * m * le / TC
    k = m * (math.pi ** 2 + le * le) / TC ** 2
    xi, v, J, dt = 1e-9, 1.0, 0.0, p.dt_f
    while True:
        fn = k * xi + d * v
        J += dt * max(0.0, fn)
        v -= dt * fn / m
        xi += dt * v
        if xi <= 0:
            break
    assert 5.0 - u[0, 0] == pytest.approx(0.15 * J / m, rel=1e-6)
    assert p.R * abs(om[0, 2]) == pytest.approx(2.5 * 0.15 * J / m, rel=1e-6)


def test_fixed_model_unchanged(orc):
    """contact_model = 0 keeps the fixed linear law (e = 0.9 restitution)."""
    p = orc.make_params(nx=80, ny=100, nz=80, h=0.1, nl=10, n_sub=80, g=(0, 0, 0))
    x = np.array([[3.0, 5.0, 4.0], [3.0 + 2 * p.R - 1e-9, 5.0, 4.0]])
    u = np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
    om = np.zeros((2, 3))
    H = orc.History(2)
    Z = np.zeros((2, 3))
    for _ in range(40):
        orc.dem(p, x, u, om, Z, Z, H)
    assert (u[1, 0] - u[0, 0]) == pytest.approx(0.9, abs=0.005)
